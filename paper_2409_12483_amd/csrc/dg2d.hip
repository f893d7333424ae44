// 2-D ADER-DG step for the Euler gas on a uniform periodic Cartesian mesh
// (gfx950, wave64): the LST-DG predictor of Sec. 1.1 with the Kronecker
// factors L^xi = kappa~ (x) k~ (x) I and L^eta = kappa~ (x) I (x) k~ (d = 2),
// and the corrector of Sec. 1.2, eq. ader_dg_method_full, with the time step
// of Sec. 1.5 (d = 2, signal speeds on the (2N+1)^2 subcell averages of
// Sec. 1.4).
//
// Predictor kernel.  A workgroup owns CPB cells; each cell is served by
// n^2 threads (n = N+1), and every thread plays three roles on the cell's
// space-time tile q[a][i][j][r] (time node a, x node i, y node j, variable r):
//   T role, thread (i, j):  updates the time line q[.][i][j];
//   X role, thread (a, j):  contracts k~ along the x line q[a][.][j];
//   Y role, thread (a, i):  contracts k~ along the y line q[a][i][.].
// The tile q lives in LDS (Q).  One Picard sweep: X threads evaluate the x
// fluxes on their lines and write k~ fx into R; Y threads evaluate the y
// fluxes on their lines and add k~ fy into R; T threads read their lines of
// R, apply kappa~ in registers, write q_new over their own time lines of Q
// and test convergence (cell maxima by LDS integer max on order-preserving
// bit patterns).  Each
// contraction runs from registers over a line the thread owns, so an LDS
// word read feeds n multiply-adds.  A converged cell freezes while the
// others of the workgroup go on; the loop ends when no cell is active.
// The epilogue writes the face traces of every cell (x faces from the X
// role, y faces from the Y role; summed in FP64, stored in the predictor
// precision) and u + volume terms in FP64.
//
// Corrector kernel.  Rusanov fluxes through the four faces of every cell
// from its own and its neighbours' traces (each face is evaluated by both
// adjacent cells, identically), the surface update of u in place, the
// admissibility test, and the signal-speed maxima of the new state on the
// subcell averages for the next step's dt.
#include "launch2d.hpp"
#include "weno_device.hpp"

namespace aderdg {

__constant__ DevOps c2_ops[kDevMaxn];
__constant__ DevOpsF c2_opsf[kDevMaxn];
__constant__ DevWeno c2_weno[3];   // WENO of degree 1 (two one-sided stencils), 2 (three) and 3 (four)

// ------------------------------------------------------------- model ----
// Sec. 2, eq. system_of_equations with two space dimensions:
// U = (rho, rho u, rho v, E), p = (gamma - 1) (E - (rho u u + rho v v) / 2).
struct Euler2 {
  static constexpr int M = 4;
  template <class T> __device__ static void flux_x(const T* q, T* f, T gm1) {
    const T ri = recip(q[0]);
    const T u = q[1] * ri, v = q[2] * ri;
    const T p = gm1 * (q[3] - T(0.5) * (q[1] * u + q[2] * v));
    f[0] = q[1];
    f[1] = q[1] * u + p;
    f[2] = q[1] * v;
    f[3] = u * (q[3] + p);
  }
  template <class T> __device__ static void flux_y(const T* q, T* f, T gm1) {
    const T ri = recip(q[0]);
    const T u = q[1] * ri, v = q[2] * ri;
    const T p = gm1 * (q[3] - T(0.5) * (q[1] * u + q[2] * v));
    f[0] = q[2];
    f[1] = q[2] * u;
    f[2] = q[2] * v + p;
    f[3] = v * (q[3] + p);
  }
  // |u| + c and |v| + c
  __device__ static void speeds(const double* q, double gamma, double& sx, double& sy) {
    const double ri = recip(q[0]);
    const double u = q[1] * ri, v = q[2] * ri;
    const double p = (gamma - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * v));
    const double c = sqrt(gamma * p * ri);
    sx = fabs(u) + c;
    sy = fabs(v) + c;
  }
  __device__ static bool admissible(const double* q, double gamma) {
    const double ri = recip(q[0]);
    const double p = (gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) * ri);
    return isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]) && q[0] > 0.0 &&
           p > 0.0;
  }
};

// Rusanov flux along x (dir 0) or y (dir 1), unscaled.
template <int DIR>
__device__ __forceinline__ void rusanov2(const double* qm, const double* qp, double* G, double gamma) {
  double fm[4], fp[4], sxm, sym, sxp, syp;
  if (DIR == 0) {
    Euler2::flux_x(qm, fm, gamma - 1.0);
    Euler2::flux_x(qp, fp, gamma - 1.0);
  } else {
    Euler2::flux_y(qm, fm, gamma - 1.0);
    Euler2::flux_y(qp, fp, gamma - 1.0);
  }
  Euler2::speeds(qm, gamma, sxm, sym);
  Euler2::speeds(qp, gamma, sxp, syp);
  // a state without a sound speed (p < 0) makes the flux NaN, as in the oracle
  // (fmax alone would drop the NaN and hide the non-physical trace)
  const double a = DIR == 0 ? sxm : sym, b = DIR == 0 ? sxp : syp;
  const double s = (isnan(a) || isnan(b)) ? a + b : fmax(a, b);
#pragma unroll
  for (int r = 0; r < 4; ++r) G[r] = 0.5 * (fm[r] + fp[r]) - 0.5 * s * (qp[r] - qm[r]);
}

// Operator coefficients in the constant address space.  launder() hides the
// pointer from loop-invariant code motion: each sweep re-reads the column
// or row it needs with scalar loads (scalar-cache hits) where it is used,
// instead of holding both n x n operators in scalar registers across the
// sweep loop, which would spill them into vector-register lanes.
template <class T> using cptr = const __attribute__((address_space(4))) T*;
template <class T> __device__ __forceinline__ cptr<T> launder(cptr<T> p) {
  asm volatile("" : "+s"(p));
  return p;
}
template <int N, class TP> __device__ __forceinline__ cptr<TP> ktil_base() {
  if constexpr (sizeof(TP) == 8) return (cptr<TP>)&c2_ops[N].ktil[0][0];
  else return (cptr<TP>)&c2_opsf[N].ktil[0][0];
}
template <int N, class TP> __device__ __forceinline__ cptr<TP> kappa_base() {
  if constexpr (sizeof(TP) == 8) return (cptr<TP>)&c2_ops[N].kappa[0][0];
  else return (cptr<TP>)&c2_opsf[N].kappa[0][0];
}

// ------------------------------------------------------- time stepping ----
// Step size of the current step (uniform over the workgroup) and, by
// workgroup 0 of the predictor launch, the clock update: next time, last dt,
// reset of the signal-speed buffer the step after next will fill, and carry
// of the current maxima when the problem has already reached t_end.
template <int N>
__device__ __forceinline__ double step_dt2d(const Args2D& A, double& t, double* bcast, bool owner) {
  if (A.mode == k2dPredict) {
    t = A.t;
    return A.dt;
  }
  Clock2D& clk = *A.clk;
  const int s = A.step;
  t = clk.t[s & 1];
  double dt;
  if (A.fixed_dt > 0.0) {
    dt = A.fixed_dt;
  } else {
    if (threadIdx.x < 64) {
      const int l = threadIdx.x & 31;
      double v = __longlong_as_double(
          (long long)(threadIdx.x < 32 ? clk.lamx[s % 3][l].v : clk.lamy[s % 3][l].v));
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
      if (l == 0) bcast[threadIdx.x >> 5] = v;
    }
    __syncthreads();
    // Sec. 1.5 with d = 2; the finite-volume scheme has no 1/(2N+1) factor
    dt = A.cfl / (2.0 * (A.scheme ? 1 : 2 * N + 1)) * fmin(A.dx / bcast[0], A.dy / bcast[1]);
  }
  const double rem = A.t_end[0] - t;
  if (dt > rem) dt = rem;
  if (!(dt > 0.0)) dt = 0.0;
  if (owner) {
    if (threadIdx.x == 0) {
      clk.t[(s + 1) & 1] = t + dt;
      if (dt > 0.0) clk.dt_last = dt;
    }
    if (threadIdx.x < kSlots) {
      clk.lamx[(s + 2) % 3][threadIdx.x].v = 0ull;
      clk.lamy[(s + 2) % 3][threadIdx.x].v = 0ull;
      if (dt == 0.0) {
        clk.lamx[(s + 1) % 3][threadIdx.x].v = clk.lamx[s % 3][threadIdx.x].v;
        clk.lamy[(s + 1) % 3][threadIdx.x].v = clk.lamy[s % 3][threadIdx.x].v;
      }
    }
  }
  return dt;
}

// ----------------------------------------------------------- predictor ----
// Cells per workgroup: as many n^2-thread cells as fill four waves, fewer
// where the two LDS tiles of a cell would not leave room for a second
// resident workgroup (the barriers of one workgroup are then overlapped by
// another's work).
// LDS tile layout.  The unit is 16 bytes: an FP32 node (its M = 4 values)
// or half an FP64 node; FP64 tiles keep the two halves of every node in two
// planes, so that every node access is one 16-byte LDS access per plane.
// Node (a, i, j) of a cell sits at unit a*SA + i*n + j.  Each role may map
// its lanes to its lines in either index order; the strides SA, the cell
// stride and the orders below were chosen per n (with the cells per
// workgroup) so that 8- and 16-lane groups of the three access patterns of
// a sweep (X: lanes over (a, j); Y: lanes over (a, i); T: lanes over (i, j))
// fall on distinct 16-byte bank groups as far as a linear layout allows;
// at n = 3 and n = 5 the tiles are unpadded instead, since the padding cost
// resident workgroups (3 -> 6 and 3 -> 4 per CU) worth more than the
// conflicts it removed (measured: -11 % per step at both in FP64).
// Cells per workgroup: whole wavefronts with few idle lanes and room for a
// second resident workgroup up to N = 5; one cell (one or two wavefronts)
// from N = 6 on, where many small workgroups per CU hide latency better than
// a few wide ones (measured: N = 6 -18 %, N = 7 -7 % per step).
struct Layout2 {
  int cpb;            // cells per workgroup
  int SA, CELL;       // time-slice and cell strides in units
  int oT, oX, oY;     // 1: the role's first line index runs fastest over lanes
};
constexpr Layout2 kLayout2[11] = {
    {0, 0, 0, 0, 0, 0},        {0, 0, 0, 0, 0, 0},       {64, 5, 12, 0, 0, 0},
    {14, 9, 27, 0, 1, 1},      {8, 19, 76, 0, 0, 1},     {5, 25, 125, 0, 0, 0},
    {5, 41, 252, 0, 0, 1},     {1, 49, 353, 0, 0, 1},    {1, 65, 520, 0, 0, 1},
    {3, 81, 729, 1, 0, 0},     {1, 105, 1050, 0, 0, 1}};

#ifndef ADERDG2D_CPB_OVERRIDE
#define ADERDG2D_CPB_OVERRIDE 0
#endif

template <int N, class TP>
struct Pred2Geo {
  static constexpr int n = N + 1, L = n * n, M = 4;
  static constexpr Layout2 lay = kLayout2[N + 1];
  static constexpr int V = 16 / (int)sizeof(TP);       // elements per unit
  static constexpr int P = M / V;                      // planes (2 in FP64, 1 in FP32)
  static constexpr int CPB = ADERDG2D_CPB_OVERRIDE > 0 ? ADERDG2D_CPB_OVERRIDE : lay.cpb;
  static constexpr int CELLE = lay.CELL * V;            // elements of one cell in one plane
  static constexpr int PLANE = CPB * CELLE;            // elements between the planes
  static constexpr int BUF = P * PLANE;                // elements of one tile buffer
  static constexpr bool kVbAlias = BUF * (int)sizeof(TP) >= CPB * 2 * L * M * 8;
  static constexpr int NT = ((CPB * L + 63) / 64) * 64;
  static_assert(2 * BUF * (int)sizeof(TP) + (kVbAlias ? 0 : CPB * 2 * L * M * 8) <= 159 * 1024,
                "tiles must fit in LDS");
  __device__ static constexpr int at(int a, int i, int j) { return (a * lay.SA + i * n + j) * V; }
};

// The four values of a node: one 16-byte LDS access per plane.
template <int PLANE>
__device__ __forceinline__ void ld4(const double* p, double* v) {
  const double2 x = *reinterpret_cast<const double2*>(p);
  const double2 y = *reinterpret_cast<const double2*>(p + PLANE);
  v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}
template <int PLANE>
__device__ __forceinline__ void ld4(const float* p, float* v) {
  const float4 x = *reinterpret_cast<const float4*>(p);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
template <int PLANE>
__device__ __forceinline__ void st4(double* p, const double* v) {
  *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  *reinterpret_cast<double2*>(p + PLANE) = make_double2(v[2], v[3]);
}
template <int PLANE>
__device__ __forceinline__ void st4(float* p, const float* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}

template <int N, class TP>
__global__ void __launch_bounds__((Pred2Geo<N, TP>::NT))
pred2d_kernel(Args2D A) {
  using G = Pred2Geo<N, TP>;
  constexpr int n = G::n, L = G::L, M = G::M, CPB = G::CPB, PL = G::PLANE;
  using Bits = decltype(ord_bits(TP(0)));

  __shared__ __align__(16) TP Qs[G::BUF];
  __shared__ __align__(16) TP Rs[G::BUF];
  __shared__ double Vsep[G::kVbAlias ? 1 : CPB * 2 * L * M];
  __shared__ Bits red[2][CPB][2];
  __shared__ double bcast[2];
  __shared__ unsigned int swsum;

  const int tid = threadIdx.x;
  const int cl = tid / L, line = tid - cl * L;
  const int hi = line / n, lo = line - hi * n;
  // line indices of the three roles (lane order per the layout table)
  const int ti = G::lay.oT ? lo : hi, tj = G::lay.oT ? hi : lo;      // T: node (i, j)
  const int xa = G::lay.oX ? lo : hi, xj = G::lay.oX ? hi : lo;      // X: line (a, j)
  const int ya = G::lay.oY ? lo : hi, yi = G::lay.oY ? hi : lo;      // Y: line (a, i)
  const int node = ti * n + tj;
  const int64_t ncells = A.cx * A.cy;
  const int64_t cell = (int64_t)blockIdx.x * CPB + cl;
  const bool mine = cl < CPB && cell < ncells;

  double t;
  const double dt = step_dt2d<N>(A, t, bcast, blockIdx.x == 0);
  if (!(dt > 0.0)) return;                                  // uniform: nothing to do this step
  const double dtdx = dt / A.dx, dtdy = dt / A.dy;
  const TP cxs = TP(dtdx), cys = TP(dtdy), gm1 = TP(A.gamma - 1.0);

  if (tid < 4 * CPB) (&red[0][0][0])[tid] = 0;
  if (tid == 0) swsum = 0u;

  // The tile lives in LDS only.  T role: node (ti, tj); the initial guess is
  // u on every time level.
  TP* const Qc = Qs + (mine ? cl : 0) * G::CELLE;
  TP* const Rc = Rs + (mine ? cl : 0) * G::CELLE;
  double u0[M];
#pragma unroll
  for (int r = 0; r < M; ++r) u0[r] = mine ? A.u[(cell * L + node) * M + r] : 1.0;
  // the T role also keeps its time line in registers (the old values for the
  // convergence test without re-reading them from the tile)
  TP qt[n][M];
#pragma unroll
  for (int a = 0; a < n; ++a)
#pragma unroll
    for (int r = 0; r < M; ++r) qt[a][r] = TP(u0[r]);
  if (mine) {
#pragma unroll
    for (int a = 0; a < n; ++a) st4<PL>(Qc + G::at(a, ti, tj), qt[a]);
  }
  const TP tol = TP(A.tol);
  bool active = mine, failed = false;
  int sweeps = 0;

  for (int it = 0;; ++it) {
    // the tile of every active cell (initial guess or the last T role's
    // update) is visible past this barrier
    if (!__syncthreads_or(active)) break;
    if (active) {
      // X role, line (a, j) = (xa, xj): R[a][i][j] = sum_i' k~[i][i'] (dt/dx) Fx(q[a][i'][j])
      TP acc[n][M];
#pragma unroll
      for (int i = 0; i < n; ++i)
#pragma unroll
        for (int r = 0; r < M; ++r) acc[i][r] = TP(0);
#pragma unroll
      for (int ip = 0; ip < n; ++ip) {
        TP qq[M], f[M];
        ld4<PL>(Qc + G::at(xa, ip, xj), qq);
        Euler2::flux_x(qq, f, gm1);
#pragma unroll
        for (int r = 0; r < M; ++r) f[r] *= cxs;
        const cptr<TP> K = launder(ktil_base<N, TP>() + ip);        // column ip of k~
#pragma unroll
        for (int i = 0; i < n; ++i)
#pragma unroll
          for (int r = 0; r < M; ++r) acc[i][r] = fma(K[i * kDevMaxn], f[r], acc[i][r]);
      }
#pragma unroll
      for (int i = 0; i < n; ++i) st4<PL>(Rc + G::at(xa, i, xj), acc[i]);
    }
    __syncthreads();
    if (active) {
      // Y role, line (a, i) = (ya, yi): R[a][i][j] += sum_j' k~[j][j'] (dt/dy) Fy(q[a][i][j'])
      TP acc[n][M];
#pragma unroll
      for (int j = 0; j < n; ++j)
#pragma unroll
        for (int r = 0; r < M; ++r) acc[j][r] = TP(0);
#pragma unroll
      for (int jp = 0; jp < n; ++jp) {
        TP qq[M], f[M];
        ld4<PL>(Qc + G::at(ya, yi, jp), qq);
        Euler2::flux_y(qq, f, gm1);
#pragma unroll
        for (int r = 0; r < M; ++r) f[r] *= cys;
        const cptr<TP> K = launder(ktil_base<N, TP>() + jp);        // column jp of k~
#pragma unroll
        for (int j = 0; j < n; ++j)
#pragma unroll
          for (int r = 0; r < M; ++r) acc[j][r] = fma(K[j * kDevMaxn], f[r], acc[j][r]);
      }
#pragma unroll
      for (int j = 0; j < n; ++j) {
        TP v[M];
        ld4<PL>(Rc + G::at(ya, yi, j), v);
#pragma unroll
        for (int r = 0; r < M; ++r) v[r] += acc[j][r];
        st4<PL>(Rc + G::at(ya, yi, j), v);
      }
    }
    __syncthreads();
    TP e_ = TP(0), qm_ = TP(0);
    if (active) {
      // T role: q_new[a] = u - sum_b kappa~[a][b] R[b][i][j], kept in registers
      // and written over the thread's own time line of the tile (no other
      // thread reads it now)
      TP rr[n][M];
#pragma unroll
      for (int b = 0; b < n; ++b) ld4<PL>(Rc + G::at(b, ti, tj), rr[b]);
      TP e = TP(0), qm = TP(0);
#pragma unroll
      for (int a = 0; a < n; ++a) {
        const cptr<TP> Kp = launder(kappa_base<N, TP>() + a * kDevMaxn);   // row a of kappa~
#pragma unroll
        for (int r = 0; r < M; ++r) {
          TP acc = TP(0);
#pragma unroll
          for (int b = 0; b < n; ++b) acc = fma(Kp[b], rr[b][r], acc);
          const TP qn = TP(u0[r]) - acc;
          e = max_abs(e, qn - qt[a][r]);
          qm = max_abs(qm, qn);
          qt[a][r] = qn;
        }
        st4<PL>(Qc + G::at(a, ti, tj), qt[a]);
      }
      e_ = e;
      qm_ = qm;
      ++sweeps;
    }
    {
      // maxima along the thread's row of n lanes (same cell; rows start at
      // multiples of n), within the wavefront, then one LDS
      // atomic per row segment.  Every lane takes part in the shuffles
      // (inactive lanes contribute zeros).
      const int lane = tid & 63;
#pragma unroll
      for (int off = 1; off < n; off <<= 1) {
        const TP e2 = __shfl_down(e_, off, 64), q2 = __shfl_down(qm_, off, 64);
        if (lo + off < n && lane + off < 64) {
          e_ = dmax(e_, e2);
          qm_ = dmax(qm_, q2);
        }
      }
      if (active && (lo == 0 || lane == 0)) {
        atomicMax(&red[it & 1][cl][0], ord_bits(e_));
        atomicMax(&red[it & 1][cl][1], ord_bits(qm_));
      }
    }
    // the other parity's maxima were read before this sweep's first barrier
    if (tid < 2 * CPB) (&red[(it + 1) & 1][0][0])[tid] = 0;
    __syncthreads();
    if (active) {
      const TP E = from_bits(red[it & 1][cl][0]), Qm = from_bits(red[it & 1][cl][1]);
      if (E <= tol * dmax(TP(1), Qm)) {
        active = false;
      } else if (sweeps >= A.max_iter) {
        active = false;
        failed = true;
      }
    }
  }

  // ---- epilogue (the loop's last barrier made every final tile visible)
  if (mine) {
    // x faces from the X role's line (a, j), y faces from the Y role's line (a, i)
    double tw[M], te[M], ts[M], tn[M];
#pragma unroll
    for (int r = 0; r < M; ++r) tw[r] = te[r] = ts[r] = tn[r] = 0.0;
#pragma unroll
    for (int p = 0; p < n; ++p) {
      const double p0 = c2_ops[N].psi0[p], p1 = c2_ops[N].psi1[p];
      TP vx[M], vy[M];
      ld4<PL>(Qc + G::at(xa, p, xj), vx);
      ld4<PL>(Qc + G::at(ya, yi, p), vy);
#pragma unroll
      for (int r = 0; r < M; ++r) {
        tw[r] = fma(p0, (double)vx[r], tw[r]);
        te[r] = fma(p1, (double)vx[r], te[r]);
        ts[r] = fma(p0, (double)vy[r], ts[r]);
        tn[r] = fma(p1, (double)vy[r], tn[r]);
      }
    }
    TP* trc = reinterpret_cast<TP*>(A.tr) + cell * (4 * L * M);
    const int lx = xa * n + xj, ly = ya * n + yi;
#pragma unroll
    for (int r = 0; r < M; ++r) {
      trc[(0 * L + lx) * M + r] = TP(tw[r]);
      trc[(1 * L + lx) * M + r] = TP(te[r]);
      trc[(2 * L + ly) * M + r] = TP(ts[r]);
      trc[(3 * L + ly) * M + r] = TP(tn[r]);
    }
    if (A.mode == k2dPredict) {
      TP* qo = reinterpret_cast<TP*>(A.q_out) + cell * (n * L * M);
#pragma unroll
      for (int a = 0; a < n; ++a) {
        TP v[M];
        ld4<PL>(Qc + G::at(a, ti, tj), v);
#pragma unroll
        for (int r = 0; r < M; ++r) qo[(a * L + node) * M + r] = v[r];
      }
      if (A.iters && line == 0) A.iters[cell] = sweeps;
    }
  }
  // volume terms (DG only: the finite-volume update needs only the traces;
  // the scheme is the same for every thread, so the barrier inside is too)
  if (A.scheme == 0) {
    // volume terms: time-integrated fluxes of the (promoted) predictor at every node
    double* const Vb = G::kVbAlias ? reinterpret_cast<double*>(Rs) : Vsep;
    double* const Vc = Vb + (mine ? cl : 0) * (2 * L * M);
    if (mine) {
      double fxb[M], fyb[M];
#pragma unroll
      for (int r = 0; r < M; ++r) fxb[r] = fyb[r] = 0.0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        double qd[M], f[M];
        TP v[M];
        ld4<PL>(Qc + G::at(a, ti, tj), v);
#pragma unroll
        for (int r = 0; r < M; ++r) qd[r] = (double)v[r];
        const double wa = c2_ops[N].w[a];
        Euler2::flux_x(qd, f, A.gamma - 1.0);
#pragma unroll
        for (int r = 0; r < M; ++r) fxb[r] = fma(wa, dtdx * f[r], fxb[r]);
        Euler2::flux_y(qd, f, A.gamma - 1.0);
#pragma unroll
        for (int r = 0; r < M; ++r) fyb[r] = fma(wa, dtdy * f[r], fyb[r]);
      }
      // in FP64, Vb aliases R, last read before the loop's final barriers
#pragma unroll
      for (int r = 0; r < M; ++r) {
        Vc[node * M + r] = fxb[r];
        Vc[(L + node) * M + r] = fyb[r];
      }
    }
    __syncthreads();
    if (mine) {
      double vol[M];
#pragma unroll
      for (int r = 0; r < M; ++r) vol[r] = 0.0;
#pragma unroll
      for (int l = 0; l < n; ++l) {
        const double dx_ = c2_ops[N].Dw[ti][l], dy_ = c2_ops[N].Dw[tj][l];
#pragma unroll
        for (int r = 0; r < M; ++r) vol[r] = fma(dx_, Vc[(l * n + tj) * M + r], vol[r]);
#pragma unroll
        for (int r = 0; r < M; ++r) vol[r] = fma(dy_, Vc[(L + ti * n + l) * M + r], vol[r]);
      }
      double* pc = A.part + (cell * L + node) * M;
#pragma unroll
      for (int r = 0; r < M; ++r) pc[r] = u0[r] + vol[r];
    }
  }

  // sweeps and status
  if (mine && line == 0) atomicAdd(&swsum, (unsigned int)sweeps);
  const bool any_fail = __any(failed);
  __syncthreads();
  if (A.mode == k2dStep) {
    const int slot = (int)(blockIdx.x % kSlots);
    if (tid == 0 && swsum) atomicAdd(&A.clk->sweeps[slot].v, (unsigned long long)swsum);
    if ((tid & 63) == 0 && any_fail) atomicMin(&A.clk->stat[(slot + (tid >> 6)) % kSlots].v, -4);
  }
}

// ----------------------------------------------------------- corrector ----
template <int N>
struct Corr2Geo {
  static constexpr int n = N + 1, L = n * n, M = 4, Ns = 2 * N + 1;
  static constexpr int CPB = 256 / L;
  static constexpr int NT = 256;
};

// Signal-speed maxima over the (2N+1)^2 subcell averages (P (x) P) u of the
// workgroup's cells; U holds u of each cell in LDS, V1 the x-projected
// averages.  Returns this thread's maxima (to be reduced by the caller).
template <int N>
__device__ __forceinline__ void subcell_speeds(const double* U, double* V1, int ncl, double gamma,
                                               double& lx, double& ly) {
  using G = Corr2Geo<N>;
  constexpr int n = G::n, L = G::L, M = G::M, Ns = G::Ns;
  for (int w = threadIdx.x; w < ncl * Ns * n; w += G::NT) {
    const int cl = w / (Ns * n), rem = w - cl * (Ns * n), s = rem / n, j = rem - s * n;
    double v[M];
#pragma unroll
    for (int r = 0; r < M; ++r) v[r] = 0.0;
#pragma unroll
    for (int i = 0; i < n; ++i) {
      const double P = c2_ops[N].P[s][i];
#pragma unroll
      for (int r = 0; r < M; ++r) v[r] = fma(P, U[(cl * L + i * n + j) * M + r], v[r]);
    }
#pragma unroll
    for (int r = 0; r < M; ++r) V1[((cl * Ns + s) * n + j) * M + r] = v[r];
  }
  __syncthreads();
  lx = 0.0;
  ly = 0.0;
  for (int w = threadIdx.x; w < ncl * Ns * Ns; w += G::NT) {
    const int cl = w / (Ns * Ns), rem = w - cl * (Ns * Ns), s = rem / Ns, tt = rem - s * Ns;
    double v[M];
#pragma unroll
    for (int r = 0; r < M; ++r) v[r] = 0.0;
#pragma unroll
    for (int j = 0; j < n; ++j) {
      const double P = c2_ops[N].P[tt][j];
#pragma unroll
      for (int r = 0; r < M; ++r) v[r] = fma(P, V1[((cl * Ns + s) * n + j) * M + r], v[r]);
    }
    double sx, sy;
    Euler2::speeds(v, gamma, sx, sy);
    lx = fmax(lx, sx);
    ly = fmax(ly, sy);
  }
}

// Workgroup maxima of (lx, ly) into slot (block % kSlots) of lambda buffer buf.
__device__ __forceinline__ void publish_lambda(Clock2D& clk, int buf, double lx, double ly,
                                               double* part) {
  lx = wave_max(lx);
  ly = wave_max(ly);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[2 * wv] = lx;
    part[2 * wv + 1] = ly;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double X = 0.0, Y = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      X = fmax(X, part[2 * w]);
      Y = fmax(Y, part[2 * w + 1]);
    }
    const int slot = (int)(blockIdx.x % kSlots);
    atomic_max_nonneg(&clk.lamx[buf][slot].v, X);
    atomic_max_nonneg(&clk.lamy[buf][slot].v, Y);
  }
}

template <int N, class TP>
__global__ void __launch_bounds__(256)
corr2d_kernel(Args2D A) {
  using G = Corr2Geo<N>;
  constexpr int n = G::n, L = G::L, M = G::M, Ns = G::Ns, CPB = G::CPB;
  __shared__ double Gf[CPB * 4 * n * M];
  __shared__ double U[CPB * L * M];
  __shared__ double V1[CPB * Ns * n * M];
  __shared__ double bcast[2];
  __shared__ double part[8];

  double t;
  const double dt = step_dt2d<N>(A, t, bcast, false);
  if (!(dt > 0.0)) return;
  const double dtdx = dt / A.dx, dtdy = dt / A.dy;
  const int64_t ncells = A.cx * A.cy;
  const int64_t cell0 = (int64_t)blockIdx.x * CPB;
  const int ncl = (int)((ncells - cell0) < CPB ? (ncells - cell0) : CPB);

  // face fluxes, time-integrated: face 0 west, 1 east, 2 south, 3 north
  for (int w = threadIdx.x; w < ncl * 4 * n; w += G::NT) {
    const int cl = w / (4 * n), rem = w - cl * (4 * n), f = rem / n, k = rem - f * n;
    const int64_t c = cell0 + cl;
    const int64_t ix = c / A.cy, iy = c - ix * A.cy;
    int64_t cm, cp;         // the cell on the minus side and on the plus side of the face
    int fm, fp;             // the trace taken from each: east/west or north/south
    if (f == 0) { cm = (ix == 0 ? A.cx - 1 : ix - 1) * A.cy + iy; cp = c; }
    else if (f == 1) { cm = c; cp = (ix + 1 == A.cx ? 0 : ix + 1) * A.cy + iy; }
    else if (f == 2) { cm = ix * A.cy + (iy == 0 ? A.cy - 1 : iy - 1); cp = c; }
    else { cm = c; cp = ix * A.cy + (iy + 1 == A.cy ? 0 : iy + 1); }
    fm = f < 2 ? 1 : 3;
    fp = f < 2 ? 0 : 2;
    const double sc = f < 2 ? dtdx : dtdy;
    double acc[M];
#pragma unroll
    for (int r = 0; r < M; ++r) acc[r] = 0.0;
    for (int a = 0; a < n; ++a) {
      double qm[M], qp[M], Gr[M];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        qm[r] = (double)reinterpret_cast<const TP*>(A.tr)[((cm * 4 + fm) * L + a * n + k) * M + r];
        qp[r] = (double)reinterpret_cast<const TP*>(A.tr)[((cp * 4 + fp) * L + a * n + k) * M + r];
      }
      if (f < 2) rusanov2<0>(qm, qp, Gr, A.gamma);
      else rusanov2<1>(qm, qp, Gr, A.gamma);
      const double wa = c2_ops[N].w[a];
#pragma unroll
      for (int r = 0; r < M; ++r) acc[r] = fma(wa, sc * Gr[r], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < M; ++r) Gf[((cl * 4 + f) * n + k) * M + r] = acc[r];
    if (A.gface && (f == 1 || f == 3)) {
#pragma unroll
      for (int r = 0; r < M; ++r) A.gface[((c * 2 + (f >> 1)) * n + k) * M + r] = acc[r];
    }
  }
  __syncthreads();

  // surface update of every node, in place
  bool bad = false;
  for (int w = threadIdx.x; w < ncl * L; w += G::NT) {
    const int cl = w / L, line = w - cl * L, i = line / n, j = line - i * n;
    const int64_t c = cell0 + cl;
    const double* pc = A.part + (c * L + line) * M;
    const double wix = c2_ops[N].winv[i], wiy = c2_ops[N].winv[j];
    const double p0i = c2_ops[N].psi0[i], p1i = c2_ops[N].psi1[i];
    const double p0j = c2_ops[N].psi0[j], p1j = c2_ops[N].psi1[j];
    const double* Gc = Gf + cl * 4 * n * M;
    double un[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const double sx = (p1i * Gc[(1 * n + j) * M + r] - p0i * Gc[(0 * n + j) * M + r]) * wix;
      const double sy = (p1j * Gc[(3 * n + i) * M + r] - p0j * Gc[(2 * n + i) * M + r]) * wiy;
      un[r] = pc[r] - sx - sy;
      A.u[(c * L + line) * M + r] = un[r];
      U[(cl * L + line) * M + r] = un[r];
    }
    bad |= !Euler2::admissible(un, A.gamma);
  }
  if (A.candidate) return;                  // the limited step takes over (uniform branch)
  if (__any(bad) && (threadIdx.x & 63) == 0)
    atomicMin(&A.clk->stat[(blockIdx.x + (threadIdx.x >> 6)) % kSlots].v, -5);
  __syncthreads();

  double lx, ly;
  subcell_speeds<N>(U, V1, ncl, A.gamma, lx, ly);
  publish_lambda(*A.clk, (A.step + 1) % 3, lx, ly, part);
}

// Signal-speed maxima of the initial state into lambda buffer 0.
template <int N>
__global__ void __launch_bounds__(256)
lambda2d_kernel(Args2D A) {
  using G = Corr2Geo<N>;
  constexpr int L = G::L, M = G::M, Ns = G::Ns, n = G::n, CPB = G::CPB;
  __shared__ double U[CPB * L * M];
  __shared__ double V1[CPB * Ns * n * M];
  __shared__ double part[8];
  const int64_t ncells = A.cx * A.cy;
  const int64_t cell0 = (int64_t)blockIdx.x * CPB;
  const int ncl = (int)((ncells - cell0) < CPB ? (ncells - cell0) : CPB);
  for (int w = threadIdx.x; w < ncl * L * M; w += G::NT) U[w] = A.u[cell0 * L * M + w];
  __syncthreads();
  double lx, ly;
  subcell_speeds<N>(U, V1, ncl, A.gamma, lx, ly);
  publish_lambda(*A.clk, 0, lx, ly, part);
}

__global__ void clock2d_begin_kernel(Clock2D* clk, const double* t_user) {
  const int i = threadIdx.x;
  if (i == 0) {
    clk->t[0] = t_user[0];
    clk->t[1] = t_user[0];
    clk->dt_last = 0.0;
  }
  if (i < kSlots) {
    for (int b = 0; b < 3; ++b) {
      clk->lamx[b][i].v = 0ull;
      clk->lamy[b][i].v = 0ull;
    }
    clk->stat[i].v = 0;
  }
}

__global__ void clock2d_end_kernel(const Clock2D* clk, double* t_user, double* dt_user,
                                   int32_t* status_user, int parity) {
  if (threadIdx.x != 0) return;
  t_user[0] = clk->t[parity];
  dt_user[0] = clk->dt_last;
  int st = 0;
  for (int i = 0; i < kSlots; ++i) st = min(st, clk->stat[i].v);
  status_user[0] = st;
}

// -------------------------------------------------------------- dispatch ----
// ------------------------------------------------- ADER-WENO (scheme 1) ----
// Dimension-by-dimension WENO reconstruction: the 1-D reconstruction along x
// of every row of cell averages gives, at the x nodes, the averages over y of
// the solution; the same reconstruction along y of those gives the nodal
// values.  The oscillation indicators are evaluated on differences from the
// centre value (the quadratic forms vanish on constants).
// One workgroup per tile of kWenoTile x kWenoTile cells: the averages of the
// tile and its halo of NW cells are staged in LDS; the x reconstruction is
// formed once for every (tile column, halo row, variable) and kept in LDS at
// the n x nodes; the y reconstruction of every (cell, x node, variable)
// follows from it.
constexpr int kWenoTile = 8;

template <int NW>
__global__ void __launch_bounds__(kFv2dThreads) weno2d_kernel(Args2D A, double* w) {
  constexpr int n = NW + 1, M = 4, S = 2 * NW + 1, T = kWenoTile, H = T + 2 * NW;
  __shared__ double va[H * H * M];          // [x][y][r], tile + halo
  __shared__ double wx[T * H * n * M];      // [tile column][halo row][x node][r]
  const DevWeno& WT = c2_weno[NW - 1];
  const int64_t tiles_y = (A.cy + T - 1) / T;
  const int64_t tx = blockIdx.x / tiles_y, ty = blockIdx.x - tx * tiles_y;
  const int64_t ix0 = tx * T, iy0 = ty * T;
  for (int e = threadIdx.x; e < H * H * M; e += kFv2dThreads) {
    const int hx = e / (H * M), rem = e - hx * (H * M), hy = rem / M, r = rem - hy * M;
    int64_t jx = ix0 - NW + hx, jy = iy0 - NW + hy;
    jx = (jx % A.cx + A.cx) % A.cx;
    jy = (jy % A.cy + A.cy) % A.cy;
    va[e] = A.u[(jx * A.cy + jy) * M + r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < T * H * M; e += kFv2dThreads) {
    const int cx_ = e / (H * M), rem = e - cx_ * (H * M), hy = rem / M, r = rem - hy * M;
    double row[S], o[n];
#pragma unroll
    for (int d = 0; d < S; ++d) row[d] = va[((cx_ + d) * H + hy) * M + r];
    weno1d<NW>(row, WT, o, -1);
#pragma unroll
    for (int k = 0; k < n; ++k) wx[((cx_ * H + hy) * n + k) * M + r] = o[k];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < T * T * n * M; e += kFv2dThreads) {
    const int cx_ = e / (T * n * M), rem = e - cx_ * (T * n * M);
    const int cy_ = rem / (n * M), rem2 = rem - cy_ * (n * M), k = rem2 / M, r = rem2 - k * M;
    const int64_t ix = ix0 + cx_, iy = iy0 + cy_;
    if (ix >= A.cx || iy >= A.cy) continue;
    double col[S], o[n];
#pragma unroll
    for (int d = 0; d < S; ++d) col[d] = wx[((cx_ * H + cy_ + d) * n + k) * M + r];
    weno1d<NW>(col, WT, o, -1);
    const int64_t cell = ix * A.cy + iy;
#pragma unroll
    for (int l = 0; l < n; ++l) w[((cell * n + k) * n + l) * M + r] = o[l];
  }
}

// Finite-volume update of the averages (in place):
// v -= sum_k w_k (Gx(east, k) - Gx(west, k) + Gy(north, k) - Gy(south, k)),
// G the time-integrated Rusanov flux of the face traces.  One workgroup per
// tile of kFvTile x kFvTile cells: for each direction, one thread per (face,
// face node) of the tile evaluates each face once into LDS (the tile's
// boundary faces are evaluated by both neighbouring tiles, identically); one
// thread per cell takes the difference of its two faces, updates v and forms
// the signal speed of the new averages (the next step's dt).
constexpr int kFvTile = 8;

template <int N>
__global__ void __launch_bounds__(kFv2dThreads) fv2d_corr_kernel(Args2D A) {
  constexpr int n = N + 1, L = n * n, M = 4, T = kFvTile, kFaces = (T + 1) * T;
  static_assert(T * T <= kFv2dThreads, "one thread per cell of the tile");
  __shared__ double Gf[kFaces * n * M];
  __shared__ double bcast[2];
  __shared__ double part[2 * (kFv2dThreads / 64)];
  double t;
  const double dt = step_dt2d<N>(A, t, bcast, false);
  if (!(dt > 0.0)) return;
  const int64_t c[2] = {A.cx, A.cy};
  const int64_t ty = (A.cy + T - 1) / T;
  const int64_t o[2] = {((int64_t)blockIdx.x / ty) * T, ((int64_t)blockIdx.x % ty) * T};
  const int ext[2] = {(int)((c[0] - o[0]) < T ? (c[0] - o[0]) : T), (int)((c[1] - o[1]) < T ? (c[1] - o[1]) : T)};
  const int tid = threadIdx.x;
  const int lc[2] = {tid / T, tid % T};
  const bool own = tid < T * T && lc[0] < ext[0] && lc[1] < ext[1];
  double dv[M];
#pragma unroll
  for (int r = 0; r < M; ++r) dv[r] = 0.0;

#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const int e = 1 - d;
    const int nf = (ext[d] + 1) * ext[e];
    const double sc = dt / (d == 0 ? A.dx : A.dy);
    for (int w = tid; w < nf * n; w += kFv2dThreads) {
      const int face = w / n, k = w - face * n;
      const int fd = face / ext[e], r1 = face - fd * ext[e];
      // face fd lies between local cells fd - 1 (minus side) and fd (plus side)
      int64_t pc[2], mc[2];
      pc[d] = o[d] + fd;
      if (pc[d] == c[d]) pc[d] = 0;
      mc[d] = o[d] + fd - 1;
      if (mc[d] < 0) mc[d] = c[d] - 1;
      pc[e] = mc[e] = o[e] + r1;
      const int64_t cm = mc[0] * A.cy + mc[1], cp = pc[0] * A.cy + pc[1];
      const int fm = 2 * d + 1, fp = 2 * d;        // minus cell's plus face, plus cell's minus face
      double acc[M];
#pragma unroll
      for (int r = 0; r < M; ++r) acc[r] = 0.0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        double qm[M], qp[M], Gr[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          qm[r] = reinterpret_cast<const double*>(A.tr)[((cm * 4 + fm) * L + a * n + k) * M + r];
          qp[r] = reinterpret_cast<const double*>(A.tr)[((cp * 4 + fp) * L + a * n + k) * M + r];
        }
        if (d == 0) rusanov2<0>(qm, qp, Gr, A.gamma);
        else rusanov2<1>(qm, qp, Gr, A.gamma);
        const double wa = c2_ops[N].w[a];
#pragma unroll
        for (int r = 0; r < M; ++r) acc[r] = fma(wa, sc * Gr[r], acc[r]);
      }
      const double wk = c2_ops[N].w[k];
#pragma unroll
      for (int r = 0; r < M; ++r) Gf[(face * n + k) * M + r] = wk * acc[r];
    }
    __syncthreads();
    if (own) {
      const int lo = lc[d] * ext[e] + lc[e], hi = (lc[d] + 1) * ext[e] + lc[e];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) sum += Gf[(hi * n + k) * M + r] - Gf[(lo * n + k) * M + r];
        dv[r] += sum;
      }
    }
    __syncthreads();
  }

  double lx = 0.0, ly = 0.0;
  bool bad = false;
  if (own) {
    const int64_t cell = (o[0] + lc[0]) * A.cy + (o[1] + lc[1]);
    double vn[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      vn[r] = A.u[cell * M + r] - dv[r];
      A.u[cell * M + r] = vn[r];
    }
    bad = !Euler2::admissible(vn, A.gamma);
    Euler2::speeds(vn, A.gamma, lx, ly);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0)
    atomicMin(&A.clk->stat[(blockIdx.x + (threadIdx.x >> 6)) % kSlots].v, -5);
  publish_lambda(*A.clk, (A.step + 1) % 3, lx, ly, part);
}

// Signal speeds of the initial averages into lambda buffer 0.
__global__ void __launch_bounds__(kFv2dThreads) fv2d_lambda_kernel(Args2D A) {
  __shared__ double part[2 * (kFv2dThreads / 64)];
  const int64_t c = (int64_t)blockIdx.x * kFv2dThreads + threadIdx.x;
  double lx = 0.0, ly = 0.0;
  if (c < A.cx * A.cy) Euler2::speeds(A.u + c * 4, A.gamma, lx, ly);
  publish_lambda(*A.clk, 0, lx, ly, part);
}

template <class TP>
static hipError_t launch_pred2d_p(int N, const Args2D& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks);
  switch (N) {
#define ADERDG2_CASE(NN)                                                                      \
  case NN:                                                                                    \
    hipLaunchKernelGGL((pred2d_kernel<NN, TP>), grid, dim3(Pred2Geo<NN, TP>::NT), 0, st, A); \
    break;
    ADERDG2_CASE(1) ADERDG2_CASE(2) ADERDG2_CASE(3) ADERDG2_CASE(4) ADERDG2_CASE(5)
    ADERDG2_CASE(6) ADERDG2_CASE(7) ADERDG2_CASE(8) ADERDG2_CASE(9)
#undef ADERDG2_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class TP> static int cpb_p(int N) {
  switch (N) {
    case 1: return Pred2Geo<1, TP>::CPB; case 2: return Pred2Geo<2, TP>::CPB;
    case 3: return Pred2Geo<3, TP>::CPB; case 4: return Pred2Geo<4, TP>::CPB;
    case 5: return Pred2Geo<5, TP>::CPB; case 6: return Pred2Geo<6, TP>::CPB;
    case 7: return Pred2Geo<7, TP>::CPB; case 8: return Pred2Geo<8, TP>::CPB;
    case 9: return Pred2Geo<9, TP>::CPB;
    default: return 0;
  }
}

int cells_per_block_2d(int N, int prec) { return prec ? cpb_p<float>(N) : cpb_p<double>(N); }
int threads_per_block_2d(int N, int prec) {
  const int L = (N + 1) * (N + 1), c = cells_per_block_2d(N, prec);
  return ((c * L + 63) / 64) * 64;
}
int cells_per_block_corr2d(int N) { return 256 / ((N + 1) * (N + 1)); }

hipError_t launch_pred2d(int N, int prec, const Args2D& A, int64_t blocks, hipStream_t st) {
  return prec ? launch_pred2d_p<float>(N, A, blocks, st) : launch_pred2d_p<double>(N, A, blocks, st);
}

template <class TP>
static hipError_t launch_corr2d_p(int N, const Args2D& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks), block(256);
  switch (N) {
#define ADERDG2_CASE(NN) case NN: hipLaunchKernelGGL((corr2d_kernel<NN, TP>), grid, block, 0, st, A); break;
    ADERDG2_CASE(1) ADERDG2_CASE(2) ADERDG2_CASE(3) ADERDG2_CASE(4) ADERDG2_CASE(5)
    ADERDG2_CASE(6) ADERDG2_CASE(7) ADERDG2_CASE(8) ADERDG2_CASE(9)
#undef ADERDG2_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_corr2d(int N, int prec, const Args2D& A, int64_t blocks, hipStream_t st) {
  return prec ? launch_corr2d_p<float>(N, A, blocks, st) : launch_corr2d_p<double>(N, A, blocks, st);
}

hipError_t launch_lambda2d(int N, const Args2D& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks), block(256);
  switch (N) {
#define ADERDG2_CASE(NN) case NN: hipLaunchKernelGGL((lambda2d_kernel<NN>), grid, block, 0, st, A); break;
    ADERDG2_CASE(1) ADERDG2_CASE(2) ADERDG2_CASE(3) ADERDG2_CASE(4) ADERDG2_CASE(5)
    ADERDG2_CASE(6) ADERDG2_CASE(7) ADERDG2_CASE(8) ADERDG2_CASE(9)
#undef ADERDG2_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_clock2d_begin(Clock2D* clk, const double* t_user, hipStream_t st) {
  hipLaunchKernelGGL(clock2d_begin_kernel, dim3(1), dim3(64), 0, st, clk, t_user);
  return hipGetLastError();
}

hipError_t launch_clock2d_end(const Clock2D* clk, double* t_user, double* dt_user,
                              int32_t* status_user, int parity, hipStream_t st) {
  hipLaunchKernelGGL(clock2d_end_kernel, dim3(1), dim3(64), 0, st, clk, t_user, dt_user,
                     status_user, parity);
  return hipGetLastError();
}

hipError_t launch_weno2d(int NW, const Args2D& A, double* w, hipStream_t st) {
  const int64_t tiles = ((A.cx + kWenoTile - 1) / kWenoTile) * ((A.cy + kWenoTile - 1) / kWenoTile);
  dim3 grid((unsigned)tiles), block(kFv2dThreads);
  if (NW == 1) hipLaunchKernelGGL((weno2d_kernel<1>), grid, block, 0, st, A, w);
  else if (NW == 2) hipLaunchKernelGGL((weno2d_kernel<2>), grid, block, 0, st, A, w);
  else if (NW == 3) hipLaunchKernelGGL((weno2d_kernel<3>), grid, block, 0, st, A, w);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fv2d_corr(int NW, const Args2D& A, hipStream_t st) {
  const int64_t tiles = ((A.cx + kFvTile - 1) / kFvTile) * ((A.cy + kFvTile - 1) / kFvTile);
  dim3 grid((unsigned)tiles), block(kFv2dThreads);
  if (NW == 1) hipLaunchKernelGGL((fv2d_corr_kernel<1>), grid, block, 0, st, A);
  else if (NW == 2) hipLaunchKernelGGL((fv2d_corr_kernel<2>), grid, block, 0, st, A);
  else if (NW == 3) hipLaunchKernelGGL((fv2d_corr_kernel<3>), grid, block, 0, st, A);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fv2d_lambda(const Args2D& A, hipStream_t st) {
  dim3 grid((unsigned)((A.cx * A.cy + kFv2dThreads - 1) / kFv2dThreads)), block(kFv2dThreads);
  hipLaunchKernelGGL(fv2d_lambda_kernel, grid, block, 0, st, A);
  return hipGetLastError();
}

hipError_t upload_tables_2d(const DevOps* ops, const DevOpsF* opsf, const DevWeno* weno) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c2_ops), ops, sizeof(DevOps) * kDevMaxn);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c2_opsf), opsf, sizeof(DevOpsF) * kDevMaxn);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c2_weno), weno, sizeof(DevWeno) * 3);
}

}  // namespace aderdg

// Kernels of the limited 2-D step (they share this file's operator and WENO tables).
#include "limiter2d.hpp"
