// Host construction of the operator tables (see operators.hpp for the citations).
//
// Gauss-Legendre nodes by Newton's method on the Legendre three-term
// recurrence, weights 2 / ((1 - x^2) P_n'(x)^2); Lagrange derivatives by
// barycentric weights; kappa~ by Gaussian elimination with partial pivoting.
#include "operators.hpp"

#include <cmath>

namespace aderdg {

namespace {

// Legendre P_n(x) and P_n'(x) on [-1, 1].
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre(int n, double* xi, double* w) {
  // roots in descending x for i = 0.. ; map xi = (1 - x) / 2 gives ascending xi
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, x, p, dp);
      double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double p, dp;
    legendre(n, x, p, dp);
    double wt = 2.0 / ((1.0 - x * x) * dp * dp);
    xi[i] = 0.5 * (1.0 - x);
    xi[n - 1 - i] = 0.5 * (1.0 + x);
    w[i] = w[n - 1 - i] = 0.5 * wt;
  }
  if (n % 2 == 1) xi[n / 2] = 0.5;
}

double lagrange(const double* nodes, int n, int k, double x) {
  double v = 1.0;
  for (int m = 0; m < n; ++m)
    if (m != k) v *= (x - nodes[m]) / (nodes[k] - nodes[m]);
  return v;
}

// Solve A X = B for X (n x n), A overwritten.  Partial pivoting.
bool solve(int n, double A[kMaxn][kMaxn], double B[kMaxn][kMaxn], double X[kMaxn][kMaxn]) {
  double a[kMaxn][2 * kMaxn];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) { a[i][j] = A[i][j]; a[i][n + j] = B[i][j]; }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
    if (a[piv][c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) { double t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r][c] / a[c][c];
      for (int j = c; j < 2 * n; ++j) a[r][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) X[i][j] = a[i][n + j] / a[i][i];
  return true;
}

// Solve A X = B for X (n x m, m <= kMaxNs), A overwritten.  Partial pivoting.
bool solve_wide(int n, int m, double A[kMaxn][kMaxn], double B[kMaxn][kMaxNs], double X[kMaxn][kMaxNs]) {
  double a[kMaxn][kMaxn + kMaxNs];
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) a[i][j] = A[i][j];
    for (int j = 0; j < m; ++j) a[i][n + j] = B[i][j];
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
    if (a[piv][c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < n + m; ++j) { double t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r][c] / a[c][c];
      for (int j = c; j < n + m; ++j) a[r][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) X[i][j] = a[i][n + j] / a[i][i];
  return true;
}

}  // namespace

bool build_op_tables(int N, OpTables& o) {
  if (N < 0 || N > kMaxN) return false;
  o = OpTables();
  const int n = N + 1;
  o.N = N;
  o.n = n;
  o.Ns = 2 * N + 1;
  gauss_legendre(n, o.xi, o.w);

  // barycentric weights b_k = 1 / prod_{m != k} (xi_k - xi_m)
  double b[kMaxn];
  for (int k = 0; k < n; ++k) {
    double p = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != k) p *= o.xi[k] - o.xi[m];
    b[k] = 1.0 / p;
  }
  // dphi[l][k] = phi_k'(xi_l)
  double dphi[kMaxn][kMaxn];
  for (int l = 0; l < n; ++l) {
    double diag = 0.0;
    for (int k = 0; k < n; ++k) {
      if (k == l) continue;
      dphi[l][k] = (b[k] / b[l]) / (o.xi[l] - o.xi[k]);
      diag += 1.0 / (o.xi[l] - o.xi[k]);
    }
    dphi[l][l] = diag;
  }
  for (int l = 0; l < n; ++l)
    for (int j = 0; j < n; ++j) o.ktil[l][j] = dphi[l][j];
  // D~[k][l] = w_l phi_k'(xi_l)
  for (int k = 0; k < n; ++k)
    for (int l = 0; l < n; ++l) o.Dtil[k][l] = o.w[l] * dphi[l][k];
  // boundary values by the barycentric formula (0 and 1 are never nodes)
  for (int side = 0; side < 2; ++side) {
    double x = side ? 1.0 : 0.0, den = 0.0;
    for (int m = 0; m < n; ++m) den += b[m] / (x - o.xi[m]);
    for (int k = 0; k < n; ++k) (side ? o.psi1 : o.psi0)[k] = (b[k] / (x - o.xi[k])) / den;
  }
  // Xi_kl = int phi_k phi_l' = w_k phi_l'(xi_k) (GL exact for degree 2N-1);
  // Upsilon_kl = phi_k(1) phi_l(1) - Xi_lk ; kappa~ = Upsilon^-1 Lambda, Lambda = diag(w)
  double U[kMaxn][kMaxn], L[kMaxn][kMaxn] = {};
  for (int k = 0; k < n; ++k)
    for (int l = 0; l < n; ++l) U[k][l] = o.psi1[k] * o.psi1[l] - o.w[l] * dphi[l][k];
  for (int k = 0; k < n; ++k) L[k][k] = o.w[k];
  if (!solve(n, U, L, o.kappa)) return false;
  // P_jk = N_s int_{j/Ns}^{(j+1)/Ns} phi_k = sum_q w_q phi_k(j/Ns + xi_q/Ns)  (exact: degree N)
  for (int j = 0; j < o.Ns; ++j)
    for (int k = 0; k < n; ++k) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += o.w[q] * lagrange(o.xi, n, k, (j + o.xi[q]) / o.Ns);
      o.P[j][k] = s;
    }
  // R = (P^T P)^-1 P^T: the normal equations of the least-squares fit of a
  // degree-N polynomial to N_s subcell averages (R P = 1, P R != 1 for N_s > n)
  double A[kMaxn][kMaxn], Pt[kMaxn][kMaxNs];
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int q = 0; q < o.Ns; ++q) s += o.P[q][i] * o.P[q][j];
      A[i][j] = s;
    }
    for (int q = 0; q < o.Ns; ++q) Pt[i][q] = o.P[q][i];
  }
  return solve_wide(n, o.Ns, A, Pt, o.R);
}

bool build_weno_tables(int Nw, WenoTables& t) {
  if (Nw < 1 || Nw > 8) return false;
  t = WenoTables();
  const int n = Nw + 1;       // nodes of the reconstruction = stencil width
  t.Nw = Nw;
  t.n = n;
  t.width = n;
  if (Nw == 1) {              // the two one-sided stencils {i-1, i}, {i, i+1}
    t.nstencils = 2;
    t.offset[0] = -1;
    t.offset[1] = 0;
  } else if (Nw % 2) {        // odd degree: one-sided, the two nearest-centred, one-sided
    t.nstencils = 4;
    t.offset[0] = -Nw;
    t.offset[1] = -(Nw + 1) / 2;
    t.offset[2] = -(Nw - 1) / 2;
    t.offset[3] = 0;
  } else {
    t.nstencils = 3;
    t.offset[0] = -Nw;
    t.offset[1] = -Nw / 2;
    t.offset[2] = 0;
  }
  OpTables ops;
  if (!build_op_tables(Nw, ops)) return false;
  // monomials (xi - 1/2)^m; integral of (xi - 1/2)^p over [o, o+1]
  auto cell_int = [](int o, int p) {
    return (std::pow(o + 0.5, p + 1) - std::pow(o - 0.5, p + 1)) / (p + 1);
  };
  // Gram matrix of all derivatives of order 1..Nw over [0,1]
  double G[kMaxn][kMaxn] = {};
  for (int a = 1; a <= Nw; ++a)
    for (int m = a; m < n; ++m)
      for (int mm = a; mm < n; ++mm) {
        double fm = 1.0, fmm = 1.0;
        for (int i = 0; i < a; ++i) { fm *= (m - i); fmm *= (mm - i); }
        G[m][mm] += fm * fmm * cell_int(0, (m - a) + (mm - a));
      }
  for (int s = 0; s < t.nstencils; ++s) {
    double A[kMaxn][kMaxn], I[kMaxn][kMaxn] = {}, Ainv[kMaxn][kMaxn];
    for (int i = 0; i < n; ++i) {
      for (int m = 0; m < n; ++m) A[i][m] = cell_int(t.offset[s] + i, m);
      I[i][i] = 1.0;
    }
    if (!solve(n, A, I, Ainv)) return false;   // coefficients c = Ainv v
    for (int k = 0; k < n; ++k)
      for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int m = 0; m < n; ++m) r += std::pow(ops.xi[k] - 0.5, m) * Ainv[m][i];
        t.R[s][k][i] = r;
      }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double v = 0.0;
        for (int m = 0; m < n; ++m)
          for (int mm = 0; mm < n; ++mm) v += Ainv[m][i] * G[m][mm] * Ainv[mm][j];
        t.S[s][i][j] = v;
      }
  }
  return true;
}

}  // namespace aderdg
