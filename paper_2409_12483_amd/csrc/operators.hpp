// Host-side construction of the 1-D operator tables of the ADER schemes.
//
// Sec. 1.1 (LST-DG predictor): Gauss-Legendre nodes/weights (eq. gl_rule),
// k~ = Lambda^-1 Xi and kappa~ = Upsilon^-1 Lambda from the mass, stiffness
// and Upsilon matrices (eq. m_and_kappa_matrices).  Sec. 1.2: D~_kl = w_l
// D^phi_kl, psi_k = phi_k(0), psi~_k = phi_k(1).  Sec. 1.4: subcell
// projection P_jk = N_s * integral of phi_k over subcell j, N_s = 2N+1, and
// the reconstruction R = (P^T P)^-1 P^T (so that R P = 1).
// WENO tables (reading of eq. weno_reconstr, see weno_tables below).
#pragma once

#include <cstdint>

namespace aderdg {

constexpr int kMaxN = 9;
constexpr int kMaxn = kMaxN + 1;
constexpr int kMaxNs = 2 * kMaxN + 1;

struct OpTables {
  int N = 0, n = 1, Ns = 1;
  double xi[kMaxn] = {};
  double w[kMaxn] = {};
  double ktil[kMaxn][kMaxn] = {};    // k~[l][j] = phi_j'(xi_l): space contraction
  double kappa[kMaxn][kMaxn] = {};   // kappa~[a][b]: time contraction
  double Dtil[kMaxn][kMaxn] = {};    // D~[k][l] = w_l phi_k'(xi_l)
  double psi0[kMaxn] = {};           // phi_k(0)
  double psi1[kMaxn] = {};           // phi_k(1)
  double P[kMaxNs][kMaxn] = {};      // subcell averages
  double R[kMaxn][kMaxNs] = {};      // subcell reconstruction: least-squares inverse of P
};

// WENO reconstruction of degree Nw from Nw+1 cell averages per stencil: for
// even Nw three stencils, left {i-Nw..i}, central {i-Nw/2..i+Nw/2}, right
// {i..i+Nw}; for Nw = 1 the two one-sided stencils {i-1, i} and {i, i+1}.
struct WenoTables {
  int Nw = 0, n = 1, width = 1, nstencils = 3;
  int offset[4] = {};                          // first stencil cell relative to i
  double R[4][kMaxn][kMaxn] = {};              // nodal value k = sum_i R[s][k][i] v_{offset+i}
  double S[4][kMaxn][kMaxn] = {};              // sigma_s = v^T S[s] v (oscillation indicator)
};

bool build_op_tables(int N, OpTables& out);
bool build_weno_tables(int Nw, WenoTables& out);

}  // namespace aderdg
