// LST-DG predictor on one wavefront (Sec. 1.1).
//
// The nested Picard iteration of eq. (lst_dg_predictor_nested_picards) in
// the factored form L^xi = kappa~ (x) k~, L^sigma = kappa~ (x) I,
// L^0 u = broadcast of u over the time nodes (eq. ind_prop):
//
//   q^(l+1,m+1)[a][l] = u[l] + sum_b kappa~[a][b] ( s - b - k~ f^(l) )[b][l]
//
// Work mapping (MI355X, wave64): each cell is served by n = N+1 consecutive
// lanes; lane a of a cell owns time row a of the AoS tile q[a][0..N][0..M-1]
// in registers.  The space contraction k~ (Algorithm 2, k_ksi_kernel) and the
// point-wise flux / source / non-conservative terms (Algorithms 2-3) are
// in-lane, with the operator coefficients as wave-uniform operands.
// The time contraction kappa~ (Algorithm 1, kappa_kernel) needs a column of
// the tile: the residual is transposed through the cell's LDS block, lane a
// then owns space column a, applies kappa~ in-lane, and transposes the new
// iterate back.  No exchange ever leaves the wavefront, so a wave-level
// fence replaces workgroup barriers.
//
// The operator coefficients k~ and kappa~ are wave-uniform scalar operands
// from the constant tables: held in scalar registers across a sweep when
// both fit the scalar budget, otherwise read where they are used.
//
// Stopping test (the paper leaves the norm open): per cell,
// max|q_new - q_old| <= tol * max(1, max|q_new|), each cell stopping on its
// own: once converged, a cell's lanes skip their LDS writes, so the tile
// they read back each sweep is their frozen result.  A cell's result thus
// depends on its own data only (not on which cells share its wavefront),
// which keeps the face fluxes of recomputed halo cells bitwise identical
// and the scheme exactly conservative.  With no source and no
// non-conservative term the inner loop is one pass.  With `stagnation`
// (FP32 predictor) a loop also stops once its increment stops decreasing,
// so that float round-off cannot spin it to the iteration limit.
#pragma once

#include "device_common.hpp"

namespace aderdg {

extern __constant__ DevOps c_ops[kDevMaxn];
extern __constant__ DevOpsF c_opsf[kDevMaxn];

// Operator rows in the constant address space.  opaque() hides the pointer
// from loop-invariant code motion, so each sweep re-reads its coefficients
// with scalar loads (scalar cache hits) right where they are used instead of
// holding both operators in scalar registers across the loop.
template <class T> using cptr = const __attribute__((address_space(4))) T*;
template <class T> __device__ __forceinline__ cptr<T> opaque(cptr<T> p) {
  asm volatile("" : "+s"(p));
  return p;
}
template <int N, class TP> struct OpSrc;
template <int N> struct OpSrc<N, double> {
  __device__ static cptr<double> K() { return (cptr<double>)&c_ops[N].ktil[0][0]; }
  __device__ static cptr<double> Kap() { return (cptr<double>)&c_ops[N].kappa[0][0]; }
};
template <int N> struct OpSrc<N, float> {
  __device__ static cptr<float> K() { return (cptr<float>)&c_opsf[N].ktil[0][0]; }
  __device__ static cptr<float> Kap() { return (cptr<float>)&c_opsf[N].kappa[0][0]; }
};

// MFMA contraction (FP32 predictor): v_mfma_f32_4x4x1f32 treats the wave as
// 16 blocks of 4 lanes and forms, per block, the outer product of a 4-row
// column held by the block's lanes (A: lane 4k+i gives row i) with a 4-column
// row (B: lane 4k+j gives column j), accumulated into the 4x4 block (lane
// 4k+j holds column j, rows 0..3).  With the operator rows as A (row
// rb*4 + lane%4, the same in every block) and each lane's own value as B,
// every lane gets rows rb*4..rb*4+3 of operator x (its own column): the
// contraction along the index the lane already owns, with no data movement.
// Issued on the matrix pipe, it runs beside the VALU's point-wise work.
typedef float mf_v4 __attribute__((ext_vector_type(4)));

template <int n, int M, int NRB>
__device__ __forceinline__ void mfma_apply(const float (&A)[NRB][n], const float (&B)[n][M],
                                           const float* c0, float (&out)[n][M]) {
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      const float init = c0 ? c0[r] : 0.0f;
      mf_v4 acc = {init, init, init, init};
#pragma unroll
      for (int j = 0; j < n; ++j) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(A[rb][j], B[j][r], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (rb * 4 + v < n) out[rb * 4 + v][r] = acc[v];
    }
}

// Newton inner iterations (Sec. 1.1: for stiff source terms the inner
// process of eq. lst_dg_predictor_nested_picards can use Newton's method).
// For a model whose source is linear, the Jacobian of the inner system
// G(q) = q - P(q) (P: the Picard map with the flux terms frozen) is the same
// for every space node: I - dt (kappa~ (x) A) on the variables the source
// couples (A = dS/dq there), the identity elsewhere.  Its inverse, of size
// L = n * kSrcVars, is formed once per workgroup and step in LDS by the first
// wavefront (Gauss-Jordan with partial pivoting) and read as wave-uniform
// operands.  `aug` holds L rows of 2L doubles; the inverse is its right half.
template <int N, class PDE>
struct NewtonDims {
  static constexpr int n = N + 1;
  static constexpr int L = n * PDE::kSrcVars;
  static constexpr int W = 2 * L;                // row stride of the augmented matrix
  static constexpr int kSize = L > 0 ? L * W : 1;
};

template <int N, class PDE>
__device__ void newton_prepare(double* aug, double dt, const PdeParams& pp) {
  using D = NewtonDims<N, PDE>;
  constexpr int n = D::n, KS = PDE::kSrcVars, L = D::L, W = D::W;
  static_assert(L > 0 && W <= 64, "one wavefront spans the augmented rows");
  if (threadIdx.x >= 64) return;
  const int j = threadIdx.x;          // column of the augmented matrix
  if (j < W) {
    for (int i = 0; i < L; ++i) {
      double v;
      if (j < L) {
        const int a = i / KS, k = i % KS, b = j / KS, k2 = j % KS;
        v = (i == j ? 1.0 : 0.0) - dt * c_ops[N].kappa[a][b] * PDE::src_jac(k, k2, pp);
      } else {
        v = (j - L == i) ? 1.0 : 0.0;
      }
      aug[i * W + j] = v;
    }
  }
  wave_sync();
  for (int c = 0; c < L; ++c) {
    // pivot: the largest |aug[r][c]| over r >= c (lane r), ties to the lowest row
    double mag = -1.0;
    int row = c;
    if (j >= c && j < L) {
      mag = fabs(aug[j * W + c]);
      row = j;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double om = __shfl_xor(mag, off, 64);
      const int orow = __shfl_xor(row, off, 64);
      if (om > mag || (om == mag && orow < row)) {
        mag = om;
        row = orow;
      }
    }
    if (row != c && j < W) {
      const double t = aug[c * W + j];
      aug[c * W + j] = aug[row * W + j];
      aug[row * W + j] = t;
    }
    wave_sync();
    const double inv = 1.0 / aug[c * W + c];
    wave_sync();
    if (j < W) aug[c * W + j] *= inv;
    wave_sync();
    for (int r = 0; r < L; ++r) {
      if (r == c) continue;
      const double f = aug[r * W + c];
      wave_sync();
      if (j < W) aug[r * W + j] -= f * aug[c * W + j];
      wave_sync();
    }
  }
}

template <int N, class PDE, class TP, bool MF = false, bool NEWTON = false>
struct Predictor {
  static_assert(!MF || sizeof(TP) == 4, "the MFMA contractions are FP32");
  static_assert(!NEWTON || (PDE::kSource && !PDE::kNcp && PDE::kSrcVars > 0),
                "Newton inner iterations serve models with a linear source only");
  static constexpr int n = N + 1;
  static constexpr int M = PDE::M;
  static constexpr int NRB = (n + 3) / 4;   // 4-row blocks of an operator (MFMA path)
  // Per-lane operator rows for the MFMA path: row rb*4 + lane%4 of k~ and of
  // -(dt/dx) kappa~ (zero past n).
  struct MfOps {
    TP k[MF ? NRB : 1][MF ? n : 1];
    TP kap[MF ? NRB : 1][MF ? n : 1];
  };
  __device__ static void mf_init(MfOps& mo, TP dtdx) {
    if constexpr (MF) {
      const int q4 = threadIdx.x & 3;
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        const int row = rb * 4 + q4;
#pragma unroll
        for (int j = 0; j < n; ++j) {
          mo.k[rb][j] = row < n ? c_opsf[N].ktil[row < n ? row : 0][j] : TP(0);
          mo.kap[rb][j] = row < n ? -dtdx * c_opsf[N].kappa[row < n ? row : 0][j] : TP(0);
        }
      }
    }
  }
  static constexpr int RS = LdsLayout<n, M, sizeof(TP)>::RS;   // row stride of the exchange block
  static constexpr bool kInner = PDE::kSource || PDE::kNcp;
  // k~ is held in scalar registers across a sweep only while it fits beside
  // kappa~'s fetch (72 dwords); larger operators are read where they are used
  static constexpr bool kPreloadK = n * n * sizeof(TP) <= 288;

  // Row residual of time node a in flux units: k~ F - dx S + B(q) k~ q, evaluated
  // on the inner iterate qi; the time contraction subtracts (dt/dx) kappa~ of it
  // from the initial data (s = dt S and b = (dt/dx) B k~ q, so this is
  // (dx/dt) (k~ f - s + b)).
  __device__ static void residual_row(const TP (&qi)[n][M], const TP (&KF)[n][M], TP* row,
                                      int a, TP dt, TP dtdx, double xl, double dx, double t0,
                                      const PdeParams& pp) {
    const TP ta = TP(t0 + (double)dt * c_ops[N].xi[a]);
    const cptr<TP> Kc = opaque(OpSrc<N, TP>::K());
#pragma unroll
    for (int l = 0; l < n; ++l) {
      TP R[M];
#pragma unroll
      for (int r = 0; r < M; ++r) R[r] = KF[l][r];
      if constexpr (PDE::kSource) {
        TP s[M];
        PDE::source(qi[l], TP(xl + dx * c_ops[N].xi[l]), ta, s, pp);
#pragma unroll
        for (int r = 0; r < M; ++r) R[r] -= TP(dx) * s[r];
      }
      if constexpr (PDE::kNcp) {
        TP dq[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          TP acc = TP(0);
#pragma unroll
          for (int j = 0; j < n; ++j) acc += Kc[l * kDevMaxn + j] * qi[j][r];
          dq[r] = acc;
        }
        TP b[M];
        PDE::ncp(qi[l], dq, b, pp);
#pragma unroll
        for (int r = 0; r < M; ++r) R[r] += b[r];
      }
#pragma unroll
      for (int r = 0; r < M; ++r) row[l * M + r] = R[r];
    }
  }

  // Per-cell max of the lanes' norms: an integer max on the cell's two LDS
  // words (order-preserving bit patterns of the non-negative norms; a NaN
  // wins), read back by every lane of the cell, then cleared by all of them
  // for the next reduction.  The cell's lanes share a wavefront, whose LDS
  // accesses complete in program order; idle lanes own a separate pair, so
  // no lane needs a branch here.
  using Bits = decltype(ord_bits(TP(0)));
  __device__ static void cell_reduce(TP* red, TP& e, TP& qm) {
    Bits* w = reinterpret_cast<Bits*>(red);
    atomicMax(&w[0], ord_bits(e));
    atomicMax(&w[1], ord_bits(qm));
    wave_sync();
    const TP E = from_bits(w[0]), Q = from_bits(w[1]);
    wave_sync();
    w[0] = 0;
    w[1] = 0;
    e = E;
    qm = Q;
  }

  // One kappa~ application: row residual -> (transpose) -> column update -> (transpose) -> row.
  // xb: the cell's LDS block (rows of RS elements).  On return `q` holds row a of
  // q_init - (dt/dx) kappa~ (residual), and e, qm this lane's part of the
  // convergence norms of the update.  Every lane overwrites only block
  // elements it has itself read before, so the only cross-lane ordering
  // needed is write-then-read, provided by wave_sync().
  // A converged cell (write == false on all its lanes) writes nothing: its
  // block still holds the tile read back at its last update, so `out`
  // returns that tile unchanged and the cell stays frozen bit for bit.
  __device__ static void load_k(TP (&kt)[n][n]) {
    if constexpr (!kPreloadK) return;
    const cptr<TP> K = opaque(OpSrc<N, TP>::K());
#pragma unroll
    for (int l = 0; l < n; ++l)
#pragma unroll
      for (int j = 0; j < n; ++j) kt[l][j] = K[l * kDevMaxn + j];
  }

  // RELOAD_K: also fetch k~ for the next sweep once kappa~ is dead, ahead of
  // the read-back fence, so that its scalar-load latency overlaps the LDS
  // round trip (k~ and kappa~ never need scalar registers at the same time).
  template <bool RELOAD_K>
  __device__ static void time_contraction(const TP* rowres, const TP (&ucol)[M], TP* xb, int a,
                                          bool write, TP dtdx, TP (&q)[n][M], TP (&kt)[n][n],
                                          const MfOps& mo, TP& e, TP& qm) {
    if (write) {
#pragma unroll
      for (int l = 0; l < n; ++l)
#pragma unroll
        for (int r = 0; r < M; ++r) xb[a * RS + l * M + r] = rowres[l * M + r];
    }
    if constexpr (MF) {
      wave_sync();
      TP col[n][M], qn[n][M];
#pragma unroll
      for (int b = 0; b < n; ++b)
#pragma unroll
        for (int r = 0; r < M; ++r) col[b][r] = xb[b * RS + a * M + r];
      mfma_apply<n, M, NRB>(mo.kap, col, ucol, qn);
      if (write) {
#pragma unroll
        for (int a2 = 0; a2 < n; ++a2)
#pragma unroll
          for (int r = 0; r < M; ++r) xb[a2 * RS + a * M + r] = qn[a2][r];
      }
      wave_sync();
#pragma unroll
      for (int l = 0; l < n; ++l)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          const TP v = xb[a * RS + l * M + r];
          const TP d = v - q[l][r];
          if (l == 0 && r == 0) {
            e = dabs(d);
            qm = dabs(v);
          } else {
            e = max_abs(e, d);
            qm = max_abs(qm, v);
          }
          q[l][r] = v;
        }
      return;
    }
    // kappa~ is fetched before the fence (when it fits the scalar budget):
    // its latency then overlaps the transpose
    TP kap[n][n];
    const cptr<TP> Kp = opaque(OpSrc<N, TP>::Kap());
    if constexpr (kPreloadK) {
#pragma unroll
      for (int a2 = 0; a2 < n; ++a2)
#pragma unroll
        for (int b = 0; b < n; ++b) kap[a2][b] = Kp[a2 * kDevMaxn + b];
    }
    auto kp = [&](int a2, int b) -> TP { return kPreloadK ? kap[a2][b] : Kp[a2 * kDevMaxn + b]; };
    wave_sync();
    TP col[n][M];
#pragma unroll
    for (int b = 0; b < n; ++b)
#pragma unroll
      for (int r = 0; r < M; ++r) col[b][r] = xb[b * RS + a * M + r];
#pragma unroll
    for (int a2 = 0; a2 < n; ++a2)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        TP acc = kp(a2, 0) * col[0][r];
#pragma unroll
        for (int b = 1; b < n; ++b) acc += kp(a2, b) * col[b][r];
        if (write) xb[a2 * RS + a * M + r] = ucol[r] - dtdx * acc;
      }
    if constexpr (RELOAD_K) load_k(kt);
    wave_sync();
    // read back in place, with the lane's share of the convergence norms:
    // e = max |q_new - q|, qm = max |q_new| over the row
#pragma unroll
    for (int l = 0; l < n; ++l)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const TP v = xb[a * RS + l * M + r];
        const TP d = v - q[l][r];
        if (l == 0 && r == 0) {
          e = dabs(d);
          qm = dabs(v);
        } else {
          e = max_abs(e, d);
          qm = max_abs(qm, v);
        }
        q[l][r] = v;
      }
  }

  // Inner iterations by Newton's method, in the column role: lane a holds the
  // space node a of its cell for every time level (KF and the iterate are
  // transposed once through the cell's LDS block), evaluates the point-wise
  // source and the Picard map P on its column, and applies the inverse
  // Jacobian to the source variables: q <- q + J^-1 (P(q) - q) there, P(q)
  // elsewhere.  On exit q holds row a of the converged inner iterate and
  // e, qm the lane's share of the outer norms (against the row on entry).
  __device__ static void newton_inner(const TP (&KF)[n][M], TP (&q)[n][M], const TP (&ucol)[M],
                                      TP* xb, TP* red, int a, bool write, TP dt, TP dtdx, double xl,
                                      double dx, double t0, const PdeParams& pp, TP tol,
                                      int max_iter, bool stagnation, const double* jinv,
                                      int& sweeps, bool& failed, TP& e, TP& qm) {
    using D = NewtonDims<N, PDE>;
    constexpr int KS = PDE::kSrcVars, L = D::L, W = D::W;
    TP kfc[n][M], qc[n][M];
    if (write) {
#pragma unroll
      for (int l = 0; l < n; ++l)
#pragma unroll
        for (int r = 0; r < M; ++r) xb[a * RS + l * M + r] = KF[l][r];
    }
    wave_sync();
#pragma unroll
    for (int b = 0; b < n; ++b)
#pragma unroll
      for (int r = 0; r < M; ++r) kfc[b][r] = xb[b * RS + a * M + r];
    wave_sync();
    if (write) {
#pragma unroll
      for (int l = 0; l < n; ++l)
#pragma unroll
        for (int r = 0; r < M; ++r) xb[a * RS + l * M + r] = q[l][r];
    }
    wave_sync();
#pragma unroll
    for (int b = 0; b < n; ++b)
#pragma unroll
      for (int r = 0; r < M; ++r) qc[b][r] = xb[b * RS + a * M + r];
    const TP xa = TP(xl + dx * c_ops[N].xi[a < n ? a : 0]);
    const cptr<TP> Kp = opaque(OpSrc<N, TP>::Kap());
    bool idone = !write;
    TP ieps_prev = TP(3.0e38);
    for (int m = 0; m < max_iter; ++m) {
      if (!__any(!idone)) break;
      // Picard map on the column
      TP R[n][M];
#pragma unroll
      for (int b = 0; b < n; ++b) {
        TP sv[M];
        PDE::source(qc[b], xa, TP(t0 + (double)dt * c_ops[N].xi[b]), sv, pp);
#pragma unroll
        for (int r = 0; r < M; ++r) R[b][r] = kfc[b][r] - TP(dx) * sv[r];
      }
      TP qp[n][M];
#pragma unroll
      for (int a2 = 0; a2 < n; ++a2)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          TP acc = Kp[a2 * kDevMaxn] * R[0][r];
#pragma unroll
          for (int b = 1; b < n; ++b) acc += Kp[a2 * kDevMaxn + b] * R[b][r];
          qp[a2][r] = ucol[r] - dtdx * acc;
        }
      // Newton correction on the source variables
      TP dlt[L];
#pragma unroll
      for (int b = 0; b < n; ++b)
#pragma unroll
        for (int k = 0; k < KS; ++k) dlt[b * KS + k] = qp[b][PDE::src_var(k)] - qc[b][PDE::src_var(k)];
#pragma unroll
      for (int i = 0; i < L; ++i) {
        TP acc = TP(0);
#pragma unroll
        for (int j2 = 0; j2 < L; ++j2) acc += TP(jinv[i * W + L + j2]) * dlt[j2];
        const int a2 = i / KS, v = PDE::src_var(i % KS);
        qp[a2][v] = qc[a2][v] + acc;
      }
      TP ie = TP(0), iqm = TP(0);
#pragma unroll
      for (int b = 0; b < n; ++b)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          ie = max_abs(ie, qp[b][r] - qc[b][r]);
          iqm = max_abs(iqm, qp[b][r]);
          if (!idone) qc[b][r] = qp[b][r];
        }
      if (!idone) sweeps += 1 << 16;
      cell_reduce(red, ie, iqm);
      if (!idone) {
        const bool conv = ie <= tol * dmax(TP(1), iqm);
        const bool stag = stagnation && m >= 1 && ie >= ieps_prev;
        ieps_prev = ie;
        if (conv || stag) idone = true;
      }
    }
    if (!idone) failed = true;
    // back to rows, with the outer norms
    wave_sync();
    if (write) {
#pragma unroll
      for (int b = 0; b < n; ++b)
#pragma unroll
        for (int r = 0; r < M; ++r) xb[b * RS + a * M + r] = qc[b][r];
    }
    wave_sync();
#pragma unroll
    for (int l = 0; l < n; ++l)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const TP v = xb[a * RS + l * M + r];
        const TP d = v - q[l][r];
        if (l == 0 && r == 0) {
          e = dabs(d);
          qm = dabs(v);
        } else {
          e = max_abs(e, d);
          qm = max_abs(qm, v);
        }
        q[l][r] = v;
      }
  }

  // q: row a of the initial guess on entry (broadcast of the initial data),
  // the converged row on exit.  ucol: initial data at space node a.
  __device__ static void run(TP (&q)[n][M], const TP (&ucol)[M], int a, TP* xb, TP* red,
                             TP dt, TP dtdx, double xl, double dx, double t0, const PdeParams& pp,
                             TP tol, int max_iter, bool stagnation, bool active, int& sweeps,
                             int& contractions, bool& failed, const double* jinv = nullptr) {
    bool done = !active;
    // outer sweeps; with an inner loop, its iterations (the kappa~ applications
    // this cell needed) ride in the high 16 bits of the same register
    sweeps = 0;
    failed = false;
    TP eps_prev = TP(3.0e38);
    TP row[n * M];
    TP kt[n][n];
    MfOps mo;
    mf_init(mo, dtdx);
    if constexpr (!MF) load_k(kt);
    reinterpret_cast<Bits*>(red)[0] = 0;   // the cell's reduction words start cleared
    reinterpret_cast<Bits*>(red)[1] = 0;
    // one outer sweep
    auto sweep = [&]() __attribute__((always_inline)) {
      if constexpr (kInner && !MF) load_k(kt);
      // Algorithm 2: fluxes at every node of the row, then k~ along space.
      TP KF[n][M];
      if constexpr (MF) {
        TP f[n][M];
#pragma unroll
        for (int j = 0; j < n; ++j) PDE::flux(q[j], f[j], pp);
        mfma_apply<n, M, NRB>(mo.k, f, nullptr, KF);
      } else {
      const cptr<TP> Kc = opaque(OpSrc<N, TP>::K());
      auto kc = [&](int l, int j) -> TP { return kPreloadK ? kt[l][j] : Kc[l * kDevMaxn + j]; };
#pragma unroll
      for (int j = 0; j < n; ++j) {
        TP f[M];
        PDE::flux(q[j], f, pp);
#pragma unroll
        for (int r = 0; r < M; ++r) {
#pragma unroll
          for (int l = 0; l < n; ++l)
            KF[l][r] = j == 0 ? kc(l, 0) * f[r] : KF[l][r] + kc(l, j) * f[r];
        }
      }
      }
      TP e, qm;
      if constexpr (!kInner) {
        residual_row(q, KF, row, a, dt, dtdx, xl, dx, t0, pp);
        time_contraction<true>(row, ucol, xb, a, active && !done, dtdx, q, kt, mo, e, qm);
      } else if constexpr (NEWTON) {
        newton_inner(KF, q, ucol, xb, red, a, active && !done, dt, dtdx, xl, dx, t0, pp, tol, max_iter,
                     stagnation, jinv, sweeps, failed, e, qm);
      } else {
        // inner loop over source / non-conservative terms (Algorithm 1, inner repeat)
        TP qi[n][M];
#pragma unroll
        for (int l = 0; l < n; ++l)
#pragma unroll
          for (int r = 0; r < M; ++r) qi[l][r] = q[l][r];
        bool idone = done;
        TP ieps_prev = TP(3.0e38);
        int m = 0;
        for (; m < max_iter; ++m) {
          if (!__any(!idone)) break;
          residual_row(qi, KF, row, a, dt, dtdx, xl, dx, t0, pp);
          TP ie, iqm;
          if (!idone) sweeps += 1 << 16;
          time_contraction<false>(row, ucol, xb, a, active && !idone, dtdx, qi, kt, mo, ie, iqm);
          cell_reduce(red, ie, iqm);
          if (!idone) {
            const bool conv = ie <= tol * dmax(TP(1), iqm);
            const bool stag = stagnation && m >= 1 && ie >= ieps_prev;
            ieps_prev = ie;
            if (conv || stag) idone = true;
          }
        }
        if (!idone) failed = true;
        // outer update and its norms
#pragma unroll
        for (int l = 0; l < n; ++l)
#pragma unroll
          for (int r = 0; r < M; ++r) {
            const TP d = qi[l][r] - q[l][r];
            if (l == 0 && r == 0) {
              e = dabs(d);
              qm = dabs(qi[l][r]);
            } else {
              e = max_abs(e, d);
              qm = max_abs(qm, qi[l][r]);
            }
            q[l][r] = qi[l][r];
          }
      }
      // outer convergence
      cell_reduce(red, e, qm);
      if (!done) {
        ++sweeps;
        const bool conv = e <= tol * dmax(TP(1), qm);
        const bool stag = stagnation && (sweeps & 0xffff) >= 2 && e >= eps_prev;
        eps_prev = e;
        if (conv || stag) done = true;
      }
    };
    if constexpr (!kInner) {
      // two sweeps per trip: the in-place update of q then alternates between
      // two register sets instead of being copied back at the loop edge
      for (int it = 0; it < max_iter; it += 2) {
        if (!__any(!done)) break;
        sweep();
        if (it + 1 >= max_iter || !__any(!done)) break;
        sweep();
      }
    } else {
      for (int it = 0; it < max_iter; ++it) {
        if (!__any(!done)) break;
        sweep();
      }
    }
    if (!done) failed = true;
    contractions = kInner ? (sweeps >> 16) : sweeps;
    sweeps &= 0xffff;
  }
};

}  // namespace aderdg
