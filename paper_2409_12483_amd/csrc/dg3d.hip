// 3-D ADER-DG step for the Euler gas on a uniform periodic Cartesian mesh
// (gfx950, wave64): the LST-DG predictor of Sec. 1.1 with the Kronecker
// factors kappa~ (x) k~ along x, y and z, and the corrector of Sec. 1.2,
// eq. ader_dg_method_full, with the time step of Sec. 1.5 (d = 3, signal
// speeds on the (2N+1)^3 subcell averages of Sec. 1.4).
//
// The design is that of the 2-D step with a fourth role.  Each cell is
// served by n^3 threads; its space-time tile q[a][i][j][k][r] lives in LDS
// (Q), with a second tile R for the contracted fluxes.  A thread's line index
// (h2, h1, h0) reads as
//   X role: the x line (a, j, k)      Y role: the y line (a, i, k)
//   Z role: the z line (a, i, j)      T role: the time line of node (i, j, k)
// One Picard sweep: X writes k~ fx into R, Y and Z add k~ fy and k~ fz, T
// applies kappa~ from registers, writes q_new over its own time line of Q and
// tests convergence.  Every contraction runs from registers over a line the
// thread owns.  Two tiles of n^4 M values must fit in LDS: N <= 5 in FP64,
// N <= 6 in the FP32-predictor mode; above, pred3d_slab_kernel streams the
// time slices instead (see there).  The epilogue writes the six face traces
// (in the predictor precision) and u + volume terms (FP64); the corrector kernel evaluates the Rusanov
// fluxes through the six faces, updates u in place and reduces the subcell
// signal speeds for the next step.
#include "launch3d.hpp"
#include "weno_device.hpp"

namespace aderdg {

__constant__ DevOps c3_ops[kDevMaxn];
__constant__ DevOpsF c3_opsf[kDevMaxn];
__constant__ DevWeno c3_weno[3];   // WENO of degree 1 (two one-sided stencils), 2 (three) and 3 (four)

// Sec. 2, eq. system_of_equations in three dimensions:
// U = (rho, rho u, rho v, rho w, E), p = (gamma - 1) (E - rho |v|^2 / 2).
struct Euler3 {
  static constexpr int M = 5;
  template <int D, class T> __device__ static void flux(const T* q, T* f, T gm1) {
    const T ri = recip(q[0]);
    const T u = q[1] * ri, v = q[2] * ri, w = q[3] * ri;
    const T p = gm1 * (q[4] - T(0.5) * (q[1] * u + q[2] * v + q[3] * w));
    const T m = q[1 + D];
    const T vd = D == 0 ? u : (D == 1 ? v : w);
    f[0] = m;
    f[1] = m * u;
    f[2] = m * v;
    f[3] = m * w;
    f[1 + D] += p;
    f[4] = vd * (q[4] + p);
  }
  template <int D> __device__ static double speed(const double* q, double gamma) {
    const double ri = recip(q[0]);
    const double u = q[1] * ri, v = q[2] * ri, w = q[3] * ri;
    const double p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] * u + q[2] * v + q[3] * w));
    return fabs(D == 0 ? u : (D == 1 ? v : w)) + sqrt(gamma * p * ri);
  }
  __device__ static void speeds(const double* q, double gamma, double* s) {
    const double ri = recip(q[0]);
    const double u = q[1] * ri, v = q[2] * ri, w = q[3] * ri;
    const double p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] * u + q[2] * v + q[3] * w));
    const double c = sqrt(gamma * p * ri);
    s[0] = fabs(u) + c;
    s[1] = fabs(v) + c;
    s[2] = fabs(w) + c;
  }
  __device__ static bool admissible(const double* q, double gamma) {
    const double ri = recip(q[0]);
    const double p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * ri);
    return isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]) && isfinite(q[4]) &&
           q[0] > 0.0 && p > 0.0;
  }
};

template <int D>
__device__ __forceinline__ void rusanov3(const double* qm, const double* qp, double* G, double gamma) {
  double fm[5], fp[5];
  Euler3::flux<D>(qm, fm, gamma - 1.0);
  Euler3::flux<D>(qp, fp, gamma - 1.0);
  const double s = fmax(Euler3::speed<D>(qm, gamma), Euler3::speed<D>(qp, gamma));
#pragma unroll
  for (int r = 0; r < 5; ++r) G[r] = 0.5 * (fm[r] + fp[r]) - 0.5 * s * (qp[r] - qm[r]);
}

// Operator coefficients re-read where used (see the 2-D kernels): the
// laundered pointer keeps them out of loop-invariant code motion.
template <class T> using cptr3 = const __attribute__((address_space(4))) T*;
template <class T> __device__ __forceinline__ cptr3<T> launder3(cptr3<T> p) {
  asm volatile("" : "+s"(p));
  return p;
}
template <int N, class TP> __device__ __forceinline__ cptr3<TP> ktil3() {
  if constexpr (sizeof(TP) == 8) return (cptr3<TP>)&c3_ops[N].ktil[0][0];
  else return (cptr3<TP>)&c3_opsf[N].ktil[0][0];
}
template <int N, class TP> __device__ __forceinline__ cptr3<TP> kappa3() {
  if constexpr (sizeof(TP) == 8) return (cptr3<TP>)&c3_ops[N].kappa[0][0];
  else return (cptr3<TP>)&c3_opsf[N].kappa[0][0];
}

// Step size of the current step and, by workgroup 0 of the predictor, the
// clock update (as in the 2-D step).
template <int N>
__device__ __forceinline__ double step_dt3d(const Args3D& A, double* bcast, bool owner) {
  if (A.mode == k3dPredict) return A.dt;
  Clock3D& clk = *A.clk;
  const int s = A.step;
  const double t = clk.t[s & 1];
  double dt;
  if (A.fixed_dt > 0.0) {
    dt = A.fixed_dt;
  } else {
    if (threadIdx.x < 64) {             // wave 0 (every workgroup has one)
      const int l = threadIdx.x & 31;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double v = __longlong_as_double((long long)clk.lam[d][s % 3][l].v);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        if (threadIdx.x == 0) bcast[d] = v;
      }
    }
    __syncthreads();
    // Sec. 1.5 with d = 3; the finite-volume scheme has no 1/(2N+1) factor
    dt = A.cfl / (3.0 * (A.scheme ? 1 : 2 * N + 1)) *
         fmin(fmin(A.h[0] / bcast[0], A.h[1] / bcast[1]), A.h[2] / bcast[2]);
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
      for (int d = 0; d < 3; ++d) {
        clk.lam[d][(s + 2) % 3][threadIdx.x].v = 0ull;
        if (dt == 0.0) clk.lam[d][(s + 1) % 3][threadIdx.x].v = clk.lam[d][s % 3][threadIdx.x].v;
      }
    }
  }
  return dt;
}

// ----------------------------------------------------------- predictor ----
// Tile strides: a node's M = 5 values are contiguous; the j-line, i-line and
// time-slice strides carry small pads (per n, in elements) chosen by a
// bank-model search so that the four access patterns of a sweep (lanes over
// (a, j, k), (a, i, k), (a, i, j) and (i, j, k)) spread over the LDS banks.
constexpr int kPad3[11][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 3, 4}, {0, 0, 0},
                              {0, 0, 0}, {0, 0, 2}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};

template <int N, class TP>
struct Pred3Geo {
  static constexpr int n = N + 1, L = n * n * n, M = 5;
  static constexpr int SJ = n * M + kPad3[N + 1][0];
  static constexpr int SI = n * SJ + kPad3[N + 1][1];
  static constexpr int SA = n * SI + kPad3[N + 1][2];
  static constexpr int TILE = n * SA;                    // elements of one tile
  // whole wavefronts with few idle lanes; in FP64 at N = 1, 2 fewer cells, so
  // that more workgroups (and more cells in all) fit in the LDS of a CU
  static constexpr int CPB = L >= 64 ? 1 : sizeof(TP) == 8 && N <= 2 ? (N == 1 ? 16 : 4) : 256 / L;
  static constexpr int NT = ((CPB * L + 63) / 64) * 64;
  static constexpr int VB = CPB * 3 * L * M;             // doubles of the volume buffer
  static constexpr bool kVbAlias = CPB * TILE * (int)sizeof(TP) >= VB * 8;
  // too large for R alone but not for Q and R together (both dead once the
  // fluxes of the volume terms are in registers): overlay both, one barrier more
  static constexpr bool kVbOverQR = !kVbAlias && 2 * CPB * TILE * (int)sizeof(TP) >= VB * 8;
  static constexpr int kBytes = 2 * CPB * TILE * (int)sizeof(TP) + (kVbAlias || kVbOverQR ? 0 : VB * 8);
  // tiles too large for LDS (FP64 from N = 6, FP32 from N = 7): served by
  // the slice-streaming kernel below instead
  static constexpr bool kGlobal = kBytes > 159 * 1024;
  __device__ static constexpr int at(int a, int i, int j, int k) { return a * SA + i * SI + j * SJ + k * M; }
};



// Epilogue of the predictor kernels, for the cell's node (h2, h1, h0) =
// line: the six face traces from the lines through the node (in the
// predictor precision), q and the sweep count in predictor-only mode, the
// volume terms of the corrector from the time-integrated fluxes (through the
// buffer Vc of 3 L M doubles per cell, which may overlay tiles that are dead
// once the loop is over: sync_before_vb adds a barrier before it is
// written), u + volume terms into A.part (DG), and the counters.
template <int N, class TP, class G>
__device__ __forceinline__ void pred3d_epilogue(const Args3D& A, const TP* Qc, double* Vc, const double (&u0)[5],
                                                double dt, bool mine, int64_t cell, int line, int h2, int h1,
                                                int h0, int sweeps, bool failed, unsigned int* swsum_p,
                                                bool sync_before_vb) {
  constexpr int n = G::n, L = G::L, M = G::M;
  unsigned int& swsum = *swsum_p;
  const int tid = threadIdx.x;
  // ---- epilogue: traces from the X, Y, Z roles' lines (line index = (a, s, t))
  if (mine) {
    double tm[3][M], tp[3][M];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int r = 0; r < M; ++r) tm[d][r] = tp[d][r] = 0.0;
#pragma unroll
    for (int p = 0; p < n; ++p) {
      const double p0 = c3_ops[N].psi0[p], p1 = c3_ops[N].psi1[p];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const double vx = (double)Qc[G::at(h2, p, h1, h0) + r];
        const double vy = (double)Qc[G::at(h2, h1, p, h0) + r];
        const double vz = (double)Qc[G::at(h2, h1, h0, p) + r];
        tm[0][r] = fma(p0, vx, tm[0][r]);
        tp[0][r] = fma(p1, vx, tp[0][r]);
        tm[1][r] = fma(p0, vy, tm[1][r]);
        tp[1][r] = fma(p1, vy, tp[1][r]);
        tm[2][r] = fma(p0, vz, tm[2][r]);
        tp[2][r] = fma(p1, vz, tp[2][r]);
      }
    }
    TP* trc = reinterpret_cast<TP*>(A.tr) + cell * (6 * L * M);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        trc[((2 * d) * L + line) * M + r] = TP(tm[d][r]);
        trc[((2 * d + 1) * L + line) * M + r] = TP(tp[d][r]);
      }
    if (A.mode == k3dPredict) {
      TP* qo = reinterpret_cast<TP*>(A.q_out) + cell * (n * L * M);
#pragma unroll
      for (int a = 0; a < n; ++a)
#pragma unroll
        for (int r = 0; r < M; ++r) qo[(a * L + line) * M + r] = Qc[G::at(a, h2, h1, h0) + r];
      if (A.iters && line == 0) A.iters[cell] = sweeps;
    }
  }
  // volume terms (DG only: the finite-volume update needs only the traces;
  // the scheme is the same for every thread, so the barriers inside are too)
  if (A.scheme == 0) {
    // volume terms from the time-integrated fluxes of the (promoted) predictor
    double fb[3][M];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int r = 0; r < M; ++r) fb[d][r] = 0.0;
    if (mine) {
#pragma unroll
      for (int a = 0; a < n; ++a) {
        double qd[M], f[M];
#pragma unroll
        for (int r = 0; r < M; ++r) qd[r] = (double)Qc[G::at(a, h2, h1, h0) + r];
        const double wa = c3_ops[N].w[a];
        Euler3::flux<0>(qd, f, A.gamma - 1.0);
#pragma unroll
        for (int r = 0; r < M; ++r) fb[0][r] = fma(wa, (dt / A.h[0]) * f[r], fb[0][r]);
        Euler3::flux<1>(qd, f, A.gamma - 1.0);
#pragma unroll
        for (int r = 0; r < M; ++r) fb[1][r] = fma(wa, (dt / A.h[1]) * f[r], fb[1][r]);
        Euler3::flux<2>(qd, f, A.gamma - 1.0);
#pragma unroll
        for (int r = 0; r < M; ++r) fb[2][r] = fma(wa, (dt / A.h[2]) * f[r], fb[2][r]);
      }
    }
    // Vb overlays R (last read before the loop's final barriers), or Q and R:
    // then every read of Q above must be done before the first store
    if (sync_before_vb) __syncthreads();
    if (mine) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int r = 0; r < M; ++r) Vc[(d * L + line) * M + r] = fb[d][r];
    }
    __syncthreads();
    if (mine) {
      double vol[M];
#pragma unroll
      for (int r = 0; r < M; ++r) vol[r] = 0.0;
#pragma unroll
      for (int l = 0; l < n; ++l) {
        const double dx_ = c3_ops[N].Dw[h2][l], dy_ = c3_ops[N].Dw[h1][l], dz_ = c3_ops[N].Dw[h0][l];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          vol[r] = fma(dx_, Vc[(0 * L + (l * n + h1) * n + h0) * M + r], vol[r]);
          vol[r] = fma(dy_, Vc[(1 * L + (h2 * n + l) * n + h0) * M + r], vol[r]);
          vol[r] = fma(dz_, Vc[(2 * L + (h2 * n + h1) * n + l) * M + r], vol[r]);
        }
      }
      double* pc = A.part + (cell * L + line) * M;
#pragma unroll
      for (int r = 0; r < M; ++r) pc[r] = u0[r] + vol[r];
    }
  }

  if (mine && line == 0) atomicAdd(&swsum, (unsigned int)sweeps);
  const bool any_fail = __any(failed);
  __syncthreads();
  if (A.mode == k3dStep) {
    const int slot = (int)(blockIdx.x % kSlots);
    if (tid == 0 && swsum) atomicAdd(&A.clk->sweeps[slot].v, (unsigned long long)swsum);
    if ((tid & 63) == 0 && any_fail) atomicMin(&A.clk->stat[(slot + (tid >> 6)) % kSlots].v, -4);
  }
}

template <int N, class TP>
__global__ void __launch_bounds__((Pred3Geo<N, TP>::NT))
pred3d_kernel(Args3D A) {
  using G = Pred3Geo<N, TP>;
  constexpr int n = G::n, L = G::L, M = G::M, CPB = G::CPB;
  using Bits = decltype(ord_bits(TP(0)));

  static_assert(!G::kGlobal, "tiles beyond LDS are served by pred3d_slab_kernel");
  constexpr bool kQR = G::kVbOverQR;
  __shared__ __align__(16) TP QR[kQR ? 2 * CPB * G::TILE : 1];
  __shared__ TP Qsep[kQR ? 1 : CPB * G::TILE];
  __shared__ TP Rsep[kQR ? 1 : CPB * G::TILE];
  __shared__ double Vsep[G::kVbAlias || kQR ? 1 : G::VB];
  TP* const Qs = kQR ? QR : Qsep;
  TP* const Rs = kQR ? QR + CPB * G::TILE : Rsep;
  __shared__ Bits red[2][CPB][2];
  __shared__ double bcast[3];
  __shared__ unsigned int swsum;

  const int tid = threadIdx.x;
  const int cl = tid / L, line = tid - cl * L;
  const int h2 = line / (n * n), h1 = (line / n) % n, h0 = line % n;
  const int64_t ncells = A.c[0] * A.c[1] * A.c[2];
  const int64_t cell = (int64_t)blockIdx.x * CPB + cl;
  const bool mine = cl < CPB && cell < ncells;

  const double dt = step_dt3d<N>(A, bcast, blockIdx.x == 0);
  if (!(dt > 0.0)) return;
  const TP c0 = TP(dt / A.h[0]), c1 = TP(dt / A.h[1]), c2 = TP(dt / A.h[2]), gm1 = TP(A.gamma - 1.0);

  if (tid < 4 * CPB) (&red[0][0][0])[tid] = 0;
  if (tid == 0) swsum = 0u;

  TP* const Qc = Qs + (mine ? cl : 0) * G::TILE;
  TP* const Rc = Rs + (mine ? cl : 0) * G::TILE;
  // T role: node (i, j, k) = (h2, h1, h0)
  double u0[M];
#pragma unroll
  for (int r = 0; r < M; ++r) u0[r] = mine ? A.u[(cell * L + line) * M + r] : 1.0;
  if (mine) {
#pragma unroll
    for (int a = 0; a < n; ++a)
#pragma unroll
      for (int r = 0; r < M; ++r) Qc[G::at(a, h2, h1, h0) + r] = TP(u0[r]);
  }
  const TP tol = TP(A.tol);
  bool active = mine, failed = false;
  int sweeps = 0;

  for (int it = 0;; ++it) {
    if (!__syncthreads_or(active)) break;
    if (active) {
      // X role, line (a, j, k): R = k~ (dt/dx) Fx along i
      TP acc[n][M];
#pragma unroll
      for (int i = 0; i < n; ++i)
#pragma unroll
        for (int r = 0; r < M; ++r) acc[i][r] = TP(0);
#pragma unroll
      for (int ip = 0; ip < n; ++ip) {
        TP qq[M], f[M];
#pragma unroll
        for (int r = 0; r < M; ++r) qq[r] = Qc[G::at(h2, ip, h1, h0) + r];
        Euler3::flux<0>(qq, f, gm1);
        const cptr3<TP> K = launder3(ktil3<N, TP>() + ip);
#pragma unroll
        for (int i = 0; i < n; ++i)
#pragma unroll
          for (int r = 0; r < M; ++r) acc[i][r] = fma(K[i * kDevMaxn], c0 * f[r], acc[i][r]);
      }
#pragma unroll
      for (int i = 0; i < n; ++i)
#pragma unroll
        for (int r = 0; r < M; ++r) Rc[G::at(h2, i, h1, h0) + r] = acc[i][r];
    }
    __syncthreads();
    if (active) {
      // Y role, line (a, i, k): R += k~ (dt/dy) Fy along j
      TP acc[n][M];
#pragma unroll
      for (int j = 0; j < n; ++j)
#pragma unroll
        for (int r = 0; r < M; ++r) acc[j][r] = TP(0);
#pragma unroll
      for (int jp = 0; jp < n; ++jp) {
        TP qq[M], f[M];
#pragma unroll
        for (int r = 0; r < M; ++r) qq[r] = Qc[G::at(h2, h1, jp, h0) + r];
        Euler3::flux<1>(qq, f, gm1);
        const cptr3<TP> K = launder3(ktil3<N, TP>() + jp);
#pragma unroll
        for (int j = 0; j < n; ++j)
#pragma unroll
          for (int r = 0; r < M; ++r) acc[j][r] = fma(K[j * kDevMaxn], c1 * f[r], acc[j][r]);
      }
#pragma unroll
      for (int j = 0; j < n; ++j)
#pragma unroll
        for (int r = 0; r < M; ++r) Rc[G::at(h2, h1, j, h0) + r] += acc[j][r];
    }
    __syncthreads();
    if (active) {
      // Z role, line (a, i, j): R += k~ (dt/dz) Fz along k
      TP acc[n][M];
#pragma unroll
      for (int k = 0; k < n; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) acc[k][r] = TP(0);
#pragma unroll
      for (int kp = 0; kp < n; ++kp) {
        TP qq[M], f[M];
#pragma unroll
        for (int r = 0; r < M; ++r) qq[r] = Qc[G::at(h2, h1, h0, kp) + r];
        Euler3::flux<2>(qq, f, gm1);
        const cptr3<TP> K = launder3(ktil3<N, TP>() + kp);
#pragma unroll
        for (int k = 0; k < n; ++k)
#pragma unroll
          for (int r = 0; r < M; ++r) acc[k][r] = fma(K[k * kDevMaxn], c2 * f[r], acc[k][r]);
      }
#pragma unroll
      for (int k = 0; k < n; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) Rc[G::at(h2, h1, h0, k) + r] += acc[k][r];
    }
    __syncthreads();
    TP e_ = TP(0), qm_ = TP(0);
    if (active) {
      // T role: q_new[a] = u - sum_b kappa~[a][b] R[b][i][j][k] over the own time line
      {
        TP rr[n][M];
#pragma unroll
        for (int b = 0; b < n; ++b)
#pragma unroll
          for (int r = 0; r < M; ++r) rr[b][r] = Rc[G::at(b, h2, h1, h0) + r];
#pragma unroll
        for (int a = 0; a < n; ++a) {
          const cptr3<TP> Kp = launder3(kappa3<N, TP>() + a * kDevMaxn);
#pragma unroll
          for (int r = 0; r < M; ++r) {
            TP acc = TP(0);
#pragma unroll
            for (int b = 0; b < n; ++b) acc = fma(Kp[b], rr[b][r], acc);
            const TP qn = TP(u0[r]) - acc;
            TP* p = &Qc[G::at(a, h2, h1, h0) + r];
            e_ = max_abs(e_, qn - *p);
            qm_ = max_abs(qm_, qn);
            *p = qn;
          }
        }
      }
      ++sweeps;
    }
    {
      // cell maxima: one cell per workgroup -> whole-wavefront reduction;
      // otherwise along rows of n lanes (rows start at multiples of n).  All
      // lanes take part in the shuffles; inactive lanes contribute zeros.
      const int lane = tid & 63;
      bool head;
      if (CPB == 1) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          e_ = dmax(e_, __shfl_xor(e_, off, 64));
          qm_ = dmax(qm_, __shfl_xor(qm_, off, 64));
        }
        head = lane == 0;
      } else {
#pragma unroll
        for (int off = 1; off < n; off <<= 1) {
          const TP e2 = __shfl_down(e_, off, 64), q2 = __shfl_down(qm_, off, 64);
          if (h0 + off < n && lane + off < 64) {
            e_ = dmax(e_, e2);
            qm_ = dmax(qm_, q2);
          }
        }
        head = h0 == 0 || lane == 0;
      }
      if (active && head) {
        atomicMax(&red[it & 1][cl][0], ord_bits(e_));
        atomicMax(&red[it & 1][cl][1], ord_bits(qm_));
      }
    }
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

  // volume-term buffer: overlays R (dead after the loop), or Q and R
  double* const Vb = G::kVbAlias ? reinterpret_cast<double*>(Rs) : kQR ? reinterpret_cast<double*>(QR) : Vsep;
  pred3d_epilogue<N, TP, G>(A, Qc, Vb + (mine ? cl : 0) * (3 * L * M), u0, dt, mine, cell, line, h2, h1, h0,
                            sweeps, failed, &swsum, kQR);
}

// ------------------------------------------ predictor, large tiles ----
// Degrees whose two tiles do not fit in LDS (FP64 N >= 6, FP32 N >= 7): the
// sweep streams the time slices of Q.  A cell is served by n^3 threads, one
// per node (i, j, k), each owning the node's time line of Q.  For each time
// slice b: every thread evaluates the three fluxes of its node into LDS; after
// a barrier every thread forms R[b] at its node from the k~ contractions
// along x, y and z of those fluxes (the sums of the line-owner kernel, in its
// order), and adds kappa~[a][b] R[b] to its registers for every time node a.
// After the last slice each thread writes its own time line of Q: Q is only
// ever touched by its owner inside the loop, so it stays in LDS where it fits
// (FP64 N = 6, FP32 N = 7) and otherwise lives in a per-cell device buffer,
// read and written once per sweep.  LDS holds one slice of fluxes (3 n^3 5
// values), which is the volume-term buffer of the epilogue afterwards.
template <int N, class TP>
struct Slab3Geo {
  using G = Pred3Geo<N, TP>;
  static constexpr int L = G::L, M = G::M;
  static constexpr int NT = ((L + 63) / 64) * 64;
  static constexpr bool kQlds = G::TILE * (int)sizeof(TP) + 3 * L * M * 8 <= 159 * 1024;
  static constexpr int kGStride = ((G::TILE * (int)sizeof(TP) + 255) / 256) * 256 / (int)sizeof(TP);
};

// Degrees served by the slice-streaming kernel: those whose tiles exceed LDS,
// and (one cell per workgroup) those from ADERDG_SLAB_FROM on.
#ifndef ADERDG_SLAB_FROM
#define ADERDG_SLAB_FROM 10
#endif
template <int N, class TP>
struct UseSlab3 {
  static constexpr bool value = Pred3Geo<N, TP>::kGlobal || (N >= ADERDG_SLAB_FROM && Pred3Geo<N, TP>::CPB == 1);
};

template <int N, class TP>
__global__ void __launch_bounds__((Slab3Geo<N, TP>::NT))
pred3d_slab_kernel(Args3D A) {
  using G = Pred3Geo<N, TP>;
  using S = Slab3Geo<N, TP>;
  constexpr int n = G::n, L = G::L, M = G::M;
  using Bits = decltype(ord_bits(TP(0)));
  __shared__ __align__(16) TP Qlds[S::kQlds ? G::TILE : 1];
  __shared__ __align__(16) double FV[3 * L * M];
  __shared__ Bits red[2][2];
  __shared__ double bcast[3];
  __shared__ unsigned int swsum;

  const int tid = threadIdx.x;
  const int line = tid;
  const int h2 = line / (n * n), h1 = (line / n) % n, h0 = line % n;
  const int64_t ncells = A.c[0] * A.c[1] * A.c[2];
  const int64_t cell = blockIdx.x;
  const bool mine = line < L && cell < ncells;

  const double dt = step_dt3d<N>(A, bcast, blockIdx.x == 0);
  if (!(dt > 0.0)) return;
  const TP c0 = TP(dt / A.h[0]), c1 = TP(dt / A.h[1]), c2 = TP(dt / A.h[2]), gm1 = TP(A.gamma - 1.0);
  if (tid < 4) (&red[0][0])[tid] = 0;
  if (tid == 0) swsum = 0u;

  TP* const Qc = S::kQlds ? Qlds : reinterpret_cast<TP*>(A.qs) + (int64_t)blockIdx.x * S::kGStride;
  TP* const Fx = reinterpret_cast<TP*>(FV);
  TP* const Fy = Fx + L * M;
  TP* const Fz = Fy + L * M;
  double u0[M];
#pragma unroll
  for (int r = 0; r < M; ++r) u0[r] = mine ? A.u[(cell * L + line) * M + r] : 1.0;
  if (mine) {
#pragma unroll
    for (int a = 0; a < n; ++a)
#pragma unroll
      for (int r = 0; r < M; ++r) Qc[G::at(a, h2, h1, h0) + r] = TP(u0[r]);
  }
  const TP tol = TP(A.tol);
  bool active = mine, failed = false;
  int sweeps = 0;

  for (int it = 0;; ++it) {
    if (!__syncthreads_or(active)) break;
    TP acc[n][M];
#pragma unroll
    for (int a = 0; a < n; ++a)
#pragma unroll
      for (int r = 0; r < M; ++r) acc[a][r] = TP(0);
    for (int b = 0; b < n; ++b) {
      if (active) {
        TP qq[M], f[M];
#pragma unroll
        for (int r = 0; r < M; ++r) qq[r] = Qc[G::at(b, h2, h1, h0) + r];
        Euler3::flux<0>(qq, f, gm1);
#pragma unroll
        for (int r = 0; r < M; ++r) Fx[line * M + r] = f[r];
        Euler3::flux<1>(qq, f, gm1);
#pragma unroll
        for (int r = 0; r < M; ++r) Fy[line * M + r] = f[r];
        Euler3::flux<2>(qq, f, gm1);
#pragma unroll
        for (int r = 0; r < M; ++r) Fz[line * M + r] = f[r];
      }
      __syncthreads();
      if (active) {
        TP R[M], t[M];
#pragma unroll
        for (int r = 0; r < M; ++r) R[r] = TP(0);
#pragma unroll
        for (int p = 0; p < n; ++p) {        // along x: node (p, j, k)
          const TP k = launder3(ktil3<N, TP>() + p)[h2 * kDevMaxn];
#pragma unroll
          for (int r = 0; r < M; ++r) R[r] = fma(k, c0 * Fx[((p * n + h1) * n + h0) * M + r], R[r]);
        }
#pragma unroll
        for (int r = 0; r < M; ++r) t[r] = TP(0);
#pragma unroll
        for (int p = 0; p < n; ++p) {        // along y: node (i, p, k)
          const TP k = launder3(ktil3<N, TP>() + p)[h1 * kDevMaxn];
#pragma unroll
          for (int r = 0; r < M; ++r) t[r] = fma(k, c1 * Fy[((h2 * n + p) * n + h0) * M + r], t[r]);
        }
#pragma unroll
        for (int r = 0; r < M; ++r) R[r] += t[r];
#pragma unroll
        for (int r = 0; r < M; ++r) t[r] = TP(0);
#pragma unroll
        for (int p = 0; p < n; ++p) {        // along z: node (i, j, p)
          const TP k = launder3(ktil3<N, TP>() + p)[h0 * kDevMaxn];
#pragma unroll
          for (int r = 0; r < M; ++r) t[r] = fma(k, c2 * Fz[((h2 * n + h1) * n + p) * M + r], t[r]);
        }
#pragma unroll
        for (int r = 0; r < M; ++r) R[r] += t[r];
        // kappa~ along time: acc[a] += kappa~[a][b] R[b]
#pragma unroll
        for (int a = 0; a < n; ++a) {
          const TP kb = launder3(kappa3<N, TP>() + a * kDevMaxn)[b];
#pragma unroll
          for (int r = 0; r < M; ++r) acc[a][r] = fma(kb, R[r], acc[a][r]);
        }
      }
      __syncthreads();                       // the next slice overwrites the fluxes
    }
    TP e_ = TP(0), qm_ = TP(0);
    if (active) {
#pragma unroll
      for (int a = 0; a < n; ++a)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          const TP qn = TP(u0[r]) - acc[a][r];
          TP* p = &Qc[G::at(a, h2, h1, h0) + r];
          e_ = max_abs(e_, qn - *p);
          qm_ = max_abs(qm_, qn);
          *p = qn;
        }
      ++sweeps;
    }
    // cell maxima: one cell per workgroup -> whole-wavefront reductions;
    // every lane takes part, inactive lanes contribute zeros
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      e_ = dmax(e_, __shfl_xor(e_, off, 64));
      qm_ = dmax(qm_, __shfl_xor(qm_, off, 64));
    }
    if (active && (tid & 63) == 0) {
      atomicMax(&red[it & 1][0], ord_bits(e_));
      atomicMax(&red[it & 1][1], ord_bits(qm_));
    }
    if (tid < 2) red[(it + 1) & 1][tid] = 0;
    __syncthreads();
    if (active) {
      const TP E = from_bits(red[it & 1][0]), Qm = from_bits(red[it & 1][1]);
      if (E <= tol * dmax(TP(1), Qm)) {
        active = false;
      } else if (sweeps >= A.max_iter) {
        active = false;
        failed = true;
      }
    }
  }
  pred3d_epilogue<N, TP, G>(A, Qc, FV, u0, dt, mine, cell, line, h2, h1, h0, sweeps, failed, &swsum, false);
}

// ----------------------------------------------------------- corrector ----
template <int N>
struct Corr3Geo {
  static constexpr int n = N + 1, L = n * n * n, M = 5, Ns = 2 * N + 1;
  static constexpr int CPB = L >= 256 ? 1 : 256 / L;
  static constexpr int NT = 256;
};

// Signal-speed maxima per direction over the (2N+1)^3 subcell averages
// (P (x) P (x) P) u of the workgroup's cells (u in LDS U): the x projection
// V1 goes through LDS; then one thread per (cell, s, t) forms the y-projected
// line sum_j P[t][j] V1[s][j][.] in registers and runs along z.  Keeping the
// second projection out of LDS leaves room for more resident workgroups.
template <int N>
__device__ __forceinline__ void subcell_speeds3(const double* U, double* V1, int ncl, double gamma,
                                                double* lam) {
  using G = Corr3Geo<N>;
  constexpr int n = G::n, L = G::L, M = G::M, Ns = G::Ns;
  for (int w = threadIdx.x; w < ncl * Ns * n * n; w += G::NT) {
    const int cl = w / (Ns * n * n), rem = w - cl * (Ns * n * n), s = rem / (n * n), jk = rem - s * (n * n);
    double v[M];
#pragma unroll
    for (int r = 0; r < M; ++r) v[r] = 0.0;
#pragma unroll
    for (int i = 0; i < n; ++i) {
      const double P = c3_ops[N].P[s][i];
#pragma unroll
      for (int r = 0; r < M; ++r) v[r] = fma(P, U[(cl * L + i * n * n + jk) * M + r], v[r]);
    }
#pragma unroll
    for (int r = 0; r < M; ++r) V1[((cl * Ns + s) * n * n + jk) * M + r] = v[r];
  }
  __syncthreads();
  lam[0] = lam[1] = lam[2] = 0.0;
  for (int w = threadIdx.x; w < ncl * Ns * Ns; w += G::NT) {
    const int cl = w / (Ns * Ns), rem = w - cl * (Ns * Ns), s = rem / Ns, t = rem - s * Ns;
    double v2[n][M];
#pragma unroll
    for (int k = 0; k < n; ++k)
#pragma unroll
      for (int r = 0; r < M; ++r) v2[k][r] = 0.0;
#pragma unroll
    for (int j = 0; j < n; ++j) {
      const double P = c3_ops[N].P[t][j];
#pragma unroll
      for (int k = 0; k < n; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) v2[k][r] = fma(P, V1[((cl * Ns + s) * n * n + j * n + k) * M + r], v2[k][r]);
    }
    for (int z = 0; z < Ns; ++z) {
      double v[M], sp[3];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        v[r] = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) v[r] = fma(c3_ops[N].P[z][k], v2[k][r], v[r]);
      }
      Euler3::speeds(v, gamma, sp);
#pragma unroll
      for (int d = 0; d < 3; ++d) lam[d] = fmax(lam[d], sp[d]);
    }
  }
}

__device__ __forceinline__ void publish_lambda3(Clock3D& clk, int buf, double* lam, double* part) {
#pragma unroll
  for (int d = 0; d < 3; ++d) lam[d] = wave_max(lam[d]);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int d = 0; d < 3; ++d) part[3 * wv + d] = lam[d];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int slot = (int)(blockIdx.x % kSlots);
    for (int d = 0; d < 3; ++d) {
      double X = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) X = fmax(X, part[3 * w + d]);
      atomic_max_nonneg(&clk.lam[d][buf][slot].v, X);
    }
  }
}

template <int N, class TP>
__global__ void __launch_bounds__(256)
corr3d_kernel(Args3D A) {
  using G = Corr3Geo<N>;
  constexpr int n = G::n, L = G::L, M = G::M, Ns = G::Ns, CPB = G::CPB, F = n * n;
  // the face fluxes Gf are dead once the nodes are updated (a barrier later),
  // so the x projection V1 of the subcell averages reuses their LDS
  __shared__ double GV[CPB * (6 > Ns ? 6 : Ns) * F * M];
  __shared__ double U[CPB * L * M];
  __shared__ double bcast[3];
  __shared__ double part[12];
  double* const Gf = GV;
  double* const V1 = GV;

  const double dt = step_dt3d<N>(A, bcast, false);
  if (!(dt > 0.0)) return;
  const int64_t ncells = A.c[0] * A.c[1] * A.c[2];
  const int64_t cell0 = (int64_t)blockIdx.x * CPB;
  const int ncl = (int)((ncells - cell0) < CPB ? (ncells - cell0) : CPB);

  // fluxes through the faces, time-integrated: face 2d = minus side, 2d+1 = plus side of direction d
  for (int w = threadIdx.x; w < ncl * 6 * F; w += G::NT) {
    const int cl = w / (6 * F), rem = w - cl * (6 * F), f = rem / F, st = rem - f * F;
    const int d = f >> 1;
    const int64_t c = cell0 + cl;
    int64_t idx[3] = {c / (A.c[1] * A.c[2]), (c / A.c[2]) % A.c[1], c % A.c[2]};
    int64_t nb[3] = {idx[0], idx[1], idx[2]};
    if (f & 1) nb[d] = (nb[d] + 1 == A.c[d]) ? 0 : nb[d] + 1;
    else nb[d] = (nb[d] == 0) ? A.c[d] - 1 : nb[d] - 1;
    const int64_t other = (nb[0] * A.c[1] + nb[1]) * A.c[2] + nb[2];
    const int64_t cm = (f & 1) ? c : other, cp = (f & 1) ? other : c;
    const double sc = dt / A.h[d];
    double acc[M];
#pragma unroll
    for (int r = 0; r < M; ++r) acc[r] = 0.0;
    for (int a = 0; a < n; ++a) {
      double qm[M], qp[M], Gr[M];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        qm[r] = (double)reinterpret_cast<const TP*>(A.tr)[((cm * 6 + 2 * d + 1) * L + a * F + st) * M + r];
        qp[r] = (double)reinterpret_cast<const TP*>(A.tr)[((cp * 6 + 2 * d) * L + a * F + st) * M + r];
      }
      if (d == 0) rusanov3<0>(qm, qp, Gr, A.gamma);
      else if (d == 1) rusanov3<1>(qm, qp, Gr, A.gamma);
      else rusanov3<2>(qm, qp, Gr, A.gamma);
      const double wa = c3_ops[N].w[a];
#pragma unroll
      for (int r = 0; r < M; ++r) acc[r] = fma(wa, sc * Gr[r], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < M; ++r) Gf[((cl * 6 + f) * F + st) * M + r] = acc[r];
  }
  __syncthreads();

  bool bad = false;
  for (int w = threadIdx.x; w < ncl * L; w += G::NT) {
    const int cl = w / L, line = w - cl * L;
    const int i = line / F, j = (line / n) % n, k = line % n;
    const int64_t c = cell0 + cl;
    const double* pc = A.part + (c * L + line) * M;
    const double* Gc = Gf + cl * 6 * F * M;
    const double* ps0 = c3_ops[N].psi0;
    const double* ps1 = c3_ops[N].psi1;
    const double* wi = c3_ops[N].winv;
    double un[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const double sx = (ps1[i] * Gc[(1 * F + j * n + k) * M + r] - ps0[i] * Gc[(0 * F + j * n + k) * M + r]) * wi[i];
      const double sy = (ps1[j] * Gc[(3 * F + i * n + k) * M + r] - ps0[j] * Gc[(2 * F + i * n + k) * M + r]) * wi[j];
      const double sz = (ps1[k] * Gc[(5 * F + i * n + j) * M + r] - ps0[k] * Gc[(4 * F + i * n + j) * M + r]) * wi[k];
      un[r] = pc[r] - sx - sy - sz;
      A.u[(c * L + line) * M + r] = un[r];
      U[(cl * L + line) * M + r] = un[r];
    }
    bad |= !Euler3::admissible(un, A.gamma);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0)
    atomicMin(&A.clk->stat[(blockIdx.x + (threadIdx.x >> 6)) % kSlots].v, -5);
  __syncthreads();
  double lam[3];
  subcell_speeds3<N>(U, V1, ncl, A.gamma, lam);
  publish_lambda3(*A.clk, (A.step + 1) % 3, lam, part);
}

template <int N>
__global__ void __launch_bounds__(256)
lambda3d_kernel(Args3D A) {
  using G = Corr3Geo<N>;
  constexpr int n = G::n, L = G::L, M = G::M, Ns = G::Ns, CPB = G::CPB, F = n * n;
  __shared__ double U[CPB * L * M];
  __shared__ double V1[CPB * Ns * F * M];
  __shared__ double part[12];
  const int64_t ncells = A.c[0] * A.c[1] * A.c[2];
  const int64_t cell0 = (int64_t)blockIdx.x * CPB;
  const int ncl = (int)((ncells - cell0) < CPB ? (ncells - cell0) : CPB);
  for (int w = threadIdx.x; w < ncl * L * M; w += G::NT) U[w] = A.u[cell0 * L * M + w];
  __syncthreads();
  double lam[3];
  subcell_speeds3<N>(U, V1, ncl, A.gamma, lam);
  publish_lambda3(*A.clk, 0, lam, part);
}

// ------------------------------------------------- ADER-WENO (scheme 1) ----
// Dimension-by-dimension WENO: along x for every line of cells, then along y
// at every x node, then along z at every (x, y) node pair.  One workgroup per
// tile of 4 x 4 x 2 cells (2 x 4 x 2 at degree 3, whose y results of n^2
// values per cell and halo layer would otherwise leave room for one workgroup
// per CU; the x extent does not change the sweeps per cell): the averages of
// the tile and its halo of NW cells are staged in LDS; the x sweep runs once
// per (tile x, halo y, halo z, variable), the y sweep once per (tile x,
// tile y, halo z, x node, variable), the z sweep per (cell, x node, y node,
// variable).  The y results reuse the staging buffer (dead after the x sweep).
template <int NW>
struct W3Tile {
  static constexpr int x = NW >= 3 ? 2 : 4, y = 4, z = 2;
};

template <int NW>
__global__ void __launch_bounds__(kFv3dThreads) weno3d_kernel(Args3D A, double* w) {
  constexpr int n = NW + 1, M = 5, S = 2 * NW + 1;
  constexpr int kW3x = W3Tile<NW>::x, kW3y = W3Tile<NW>::y, kW3z = W3Tile<NW>::z;
  constexpr int Hx = kW3x + 2 * NW, Hy = kW3y + 2 * NW, Hz = kW3z + 2 * NW;
  constexpr int VA = Hx * Hy * Hz * M, WY = kW3x * kW3y * Hz * n * n * M;
  __shared__ double buf[VA > WY ? VA : WY];            // staged averages, then the y sweep
  __shared__ double wx[kW3x * Hy * Hz * n * M];
  double* const va = buf;
  double* const wy = buf;
  const DevWeno& WT = c3_weno[NW - 1];
  const int64_t tz = (A.c[2] + kW3z - 1) / kW3z, ty = (A.c[1] + kW3y - 1) / kW3y;
  const int64_t bx = blockIdx.x / (ty * tz), by = (blockIdx.x / tz) % ty, bz = blockIdx.x % tz;
  const int64_t x0 = bx * kW3x, y0 = by * kW3y, z0 = bz * kW3z;
  for (int e = threadIdx.x; e < VA; e += kFv3dThreads) {
    const int hx = e / (Hy * Hz * M), hy = (e / (Hz * M)) % Hy, hz = (e / M) % Hz, r = e % M;
    int64_t jx = x0 - NW + hx, jy = y0 - NW + hy, jz = z0 - NW + hz;
    jx = (jx % A.c[0] + A.c[0]) % A.c[0];
    jy = (jy % A.c[1] + A.c[1]) % A.c[1];
    jz = (jz % A.c[2] + A.c[2]) % A.c[2];
    va[e] = A.u[((jx * A.c[1] + jy) * A.c[2] + jz) * M + r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kW3x * Hy * Hz * M; e += kFv3dThreads) {
    const int cx = e / (Hy * Hz * M), hy = (e / (Hz * M)) % Hy, hz = (e / M) % Hz, r = e % M;
    double row[S], o[n];
#pragma unroll
    for (int d = 0; d < S; ++d) row[d] = va[(((cx + d) * Hy + hy) * Hz + hz) * M + r];
    weno1d<NW>(row, WT, o, -1);
#pragma unroll
    for (int k = 0; k < n; ++k) wx[(((cx * Hy + hy) * Hz + hz) * n + k) * M + r] = o[k];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kW3x * kW3y * Hz * n * M; e += kFv3dThreads) {
    const int cx = e / (kW3y * Hz * n * M), cy = (e / (Hz * n * M)) % kW3y, hz = (e / (n * M)) % Hz;
    const int kx = (e / M) % n, r = e % M;
    double col[S], o[n];
#pragma unroll
    for (int d = 0; d < S; ++d) col[d] = wx[(((cx * Hy + cy + d) * Hz + hz) * n + kx) * M + r];
    weno1d<NW>(col, WT, o, -1);
#pragma unroll
    for (int k = 0; k < n; ++k) wy[((((cx * kW3y + cy) * Hz + hz) * n + kx) * n + k) * M + r] = o[k];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kW3x * kW3y * kW3z * n * n * M; e += kFv3dThreads) {
    const int cx = e / (kW3y * kW3z * n * n * M), cy = (e / (kW3z * n * n * M)) % kW3y;
    const int cz = (e / (n * n * M)) % kW3z, kx = (e / (n * M)) % n, ky = (e / M) % n, r = e % M;
    const int64_t ix = x0 + cx, iy = y0 + cy, iz = z0 + cz;
    if (ix >= A.c[0] || iy >= A.c[1] || iz >= A.c[2]) continue;
    double col[S], o[n];
#pragma unroll
    for (int d = 0; d < S; ++d) col[d] = wy[((((cx * kW3y + cy) * Hz + cz + d) * n + kx) * n + ky) * M + r];
    weno1d<NW>(col, WT, o, -1);
    const int64_t cell = (ix * A.c[1] + iy) * A.c[2] + iz;
#pragma unroll
    for (int k = 0; k < n; ++k) w[(cell * n * n * n + (kx * n + ky) * n + k) * M + r] = o[k];
  }
}

// Finite-volume update of the averages (in place): v -= sum over the three
// directions of the differences of the time- and face-integrated Rusanov
// fluxes through a cell's two faces (weighted by the face nodes' weights);
// then the signal speeds of the new averages for the next step's dt.  One
// workgroup per tile of 4^3 cells: for each direction, one thread per
// (face, face node) of the tile evaluates each face once (the tile's boundary
// faces are evaluated by both neighbouring tiles, identically) into LDS, and
// one thread per cell takes the difference of its two faces.
constexpr int kF3 = 4;

template <int N>
__global__ void __launch_bounds__(kFv3dThreads) fv3d_corr_kernel(Args3D A) {
  constexpr int n = N + 1, L = n * n * n, M = 5, F = n * n;
  constexpr int kFaces = (kF3 + 1) * kF3 * kF3;
  __shared__ double Gf[kFaces * F * M];
  __shared__ double bcast[3];
  __shared__ double part[3 * (kFv3dThreads / 64)];
  const double dt = step_dt3d<N>(A, bcast, false);
  if (!(dt > 0.0)) return;
  const int64_t ty = (A.c[1] + kF3 - 1) / kF3, tz = (A.c[2] + kF3 - 1) / kF3;
  const int64_t b = blockIdx.x;
  const int64_t o[3] = {(b / (ty * tz)) * kF3, ((b / tz) % ty) * kF3, (b % tz) * kF3};
  int ext[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) ext[d] = (int)((A.c[d] - o[d]) < kF3 ? (A.c[d] - o[d]) : kF3);
  const int tid = threadIdx.x;
  const int lc[3] = {tid / (kF3 * kF3), (tid / kF3) % kF3, tid % kF3};
  const bool own = tid < kF3 * kF3 * kF3 && lc[0] < ext[0] && lc[1] < ext[1] && lc[2] < ext[2];
  double dv[M];
#pragma unroll
  for (int r = 0; r < M; ++r) dv[r] = 0.0;

#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
    const int nf = (ext[d] + 1) * ext[e1] * ext[e2];
    const double sc = dt / A.h[d];
    for (int w = tid; w < nf * F; w += kFv3dThreads) {
      const int face = w / F, st = w - face * F;
      const int fd = face / (ext[e1] * ext[e2]), r1 = (face / ext[e2]) % ext[e1], r2 = face % ext[e2];
      // face fd lies between local cells fd - 1 (minus side) and fd (plus side)
      int64_t pc[3], mc[3];
      pc[d] = o[d] + fd;
      if (pc[d] == A.c[d]) pc[d] = 0;
      mc[d] = o[d] + fd - 1;
      if (mc[d] < 0) mc[d] = A.c[d] - 1;
      pc[e1] = mc[e1] = o[e1] + r1;
      pc[e2] = mc[e2] = o[e2] + r2;
      const int64_t cm = (mc[0] * A.c[1] + mc[1]) * A.c[2] + mc[2];
      const int64_t cp = (pc[0] * A.c[1] + pc[1]) * A.c[2] + pc[2];
      double acc[M];
#pragma unroll
      for (int r = 0; r < M; ++r) acc[r] = 0.0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        double qm[M], qp[M], Gr[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          qm[r] = reinterpret_cast<const double*>(A.tr)[((cm * 6 + 2 * d + 1) * L + a * F + st) * M + r];
          qp[r] = reinterpret_cast<const double*>(A.tr)[((cp * 6 + 2 * d) * L + a * F + st) * M + r];
        }
        if (d == 0) rusanov3<0>(qm, qp, Gr, A.gamma);
        else if (d == 1) rusanov3<1>(qm, qp, Gr, A.gamma);
        else rusanov3<2>(qm, qp, Gr, A.gamma);
        const double wa = c3_ops[N].w[a];
#pragma unroll
        for (int r = 0; r < M; ++r) acc[r] = fma(wa, sc * Gr[r], acc[r]);
      }
      const double wst = c3_ops[N].w[st / n] * c3_ops[N].w[st % n];
#pragma unroll
      for (int r = 0; r < M; ++r) Gf[(face * F + st) * M + r] = wst * acc[r];
    }
    __syncthreads();
    if (own) {
      const int lo = (lc[d] * ext[e1] + lc[e1]) * ext[e2] + lc[e2];
      const int hi = ((lc[d] + 1) * ext[e1] + lc[e1]) * ext[e2] + lc[e2];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double s = 0.0;
        for (int st = 0; st < F; ++st) s += Gf[(hi * F + st) * M + r] - Gf[(lo * F + st) * M + r];
        dv[r] += s;
      }
    }
    __syncthreads();
  }

  double lam[3] = {0.0, 0.0, 0.0};
  bool bad = false;
  if (own) {
    const int64_t c = ((o[0] + lc[0]) * A.c[1] + (o[1] + lc[1])) * A.c[2] + (o[2] + lc[2]);
    double vn[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      vn[r] = A.u[c * M + r] - dv[r];
      A.u[c * M + r] = vn[r];
    }
    bad = !Euler3::admissible(vn, A.gamma);
    Euler3::speeds(vn, A.gamma, lam);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0)
    atomicMin(&A.clk->stat[(blockIdx.x + (threadIdx.x >> 6)) % kSlots].v, -5);
  publish_lambda3(*A.clk, (A.step + 1) % 3, lam, part);
}

// Signal speeds of the initial averages into lambda buffer 0.
__global__ void __launch_bounds__(kFv3dThreads) fv3d_lambda_kernel(Args3D A) {
  __shared__ double part[3 * (kFv3dThreads / 64)];
  const int64_t c = (int64_t)blockIdx.x * kFv3dThreads + threadIdx.x;
  double lam[3] = {0.0, 0.0, 0.0};
  if (c < A.c[0] * A.c[1] * A.c[2]) Euler3::speeds(A.u + c * 5, A.gamma, lam);
  publish_lambda3(*A.clk, 0, lam, part);
}

__global__ void clock3d_begin_kernel(Clock3D* clk, const double* t_user) {
  const int i = threadIdx.x;
  if (i == 0) {
    clk->t[0] = t_user[0];
    clk->t[1] = t_user[0];
    clk->dt_last = 0.0;
  }
  if (i < kSlots) {
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < 3; ++b) clk->lam[d][b][i].v = 0ull;
    clk->stat[i].v = 0;
  }
}

__global__ void clock3d_end_kernel(const Clock3D* clk, double* t_user, double* dt_user,
                                   int32_t* status_user, int parity) {
  if (threadIdx.x != 0) return;
  t_user[0] = clk->t[parity];
  dt_user[0] = clk->dt_last;
  int st = 0;
  for (int i = 0; i < kSlots; ++i) st = min(st, clk->stat[i].v);
  status_user[0] = st;
}

// -------------------------------------------------------------- dispatch ----
template <int N, class TP>
static hipError_t pred3d_one(const Args3D& A, int64_t blocks, hipStream_t st) {
  if constexpr (UseSlab3<N, TP>::value) {
    if (!Slab3Geo<N, TP>::kQlds && A.qs == nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL((pred3d_slab_kernel<N, TP>), dim3((unsigned)blocks), dim3(Slab3Geo<N, TP>::NT), 0, st, A);
  } else {
    hipLaunchKernelGGL((pred3d_kernel<N, TP>), dim3((unsigned)blocks), dim3(Pred3Geo<N, TP>::NT), 0, st, A);
  }
  return hipGetLastError();
}

#define ADERDG3_DEGREES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9)

template <class TP>
static hipError_t launch_pred3d_p(int N, const Args3D& A, int64_t blocks, hipStream_t st) {
  switch (N) {
#define ADERDG3_CASE(NN) case NN: return pred3d_one<NN, TP>(A, blocks, st);
    ADERDG3_DEGREES(ADERDG3_CASE)
#undef ADERDG3_CASE
    default: return hipErrorInvalidValue;
  }
}

template <class TP> static int cpb3_p(int N) {
  switch (N) {
#define ADERDG3_CASE(NN) case NN: return Pred3Geo<NN, TP>::CPB;
    ADERDG3_DEGREES(ADERDG3_CASE)
#undef ADERDG3_CASE
    default: return 0;
  }
}

// Bytes of the device buffer a cell's predictor tile needs (0: it is in LDS).
template <int N, class TP>
constexpr int64_t pred3d_global_bytes() {
  if constexpr (UseSlab3<N, TP>::value && !Slab3Geo<N, TP>::kQlds)
    return (int64_t)Slab3Geo<N, TP>::kGStride * (int64_t)sizeof(TP);
  else
    return 0;
}

template <class TP> static int64_t gbytes3_p(int N) {
  switch (N) {
#define ADERDG3_CASE(NN) case NN: return pred3d_global_bytes<NN, TP>();
    ADERDG3_DEGREES(ADERDG3_CASE)
#undef ADERDG3_CASE
    default: return 0;
  }
}

bool supported_3d(int N, int prec) { return N >= 1 && N <= 9 && (prec == 0 || prec == 1); }
int cells_per_block_3d(int N, int prec) { return prec ? cpb3_p<float>(N) : cpb3_p<double>(N); }
int64_t pred3d_tile_bytes_per_cell(int N, int prec) { return prec ? gbytes3_p<float>(N) : gbytes3_p<double>(N); }
int cells_per_block_corr3d(int N) {
  const int L = (N + 1) * (N + 1) * (N + 1);
  return L >= 256 ? 1 : 256 / L;
}

hipError_t launch_pred3d(int N, int prec, const Args3D& A, int64_t blocks, hipStream_t st) {
  return prec ? launch_pred3d_p<float>(N, A, blocks, st) : launch_pred3d_p<double>(N, A, blocks, st);
}

template <class TP>
static hipError_t launch_corr3d_p(int N, const Args3D& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks), block(256);
  switch (N) {
#define ADERDG3_CASE(NN) case NN: hipLaunchKernelGGL((corr3d_kernel<NN, TP>), grid, block, 0, st, A); break;
    ADERDG3_DEGREES(ADERDG3_CASE)
#undef ADERDG3_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_corr3d(int N, int prec, const Args3D& A, int64_t blocks, hipStream_t st) {
  return prec ? launch_corr3d_p<float>(N, A, blocks, st) : launch_corr3d_p<double>(N, A, blocks, st);
}

hipError_t launch_lambda3d(int N, const Args3D& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks), block(256);
  switch (N) {
#define ADERDG3_CASE(NN) case NN: hipLaunchKernelGGL((lambda3d_kernel<NN>), grid, block, 0, st, A); break;
    ADERDG3_DEGREES(ADERDG3_CASE)
#undef ADERDG3_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_clock3d_begin(Clock3D* clk, const double* t_user, hipStream_t st) {
  hipLaunchKernelGGL(clock3d_begin_kernel, dim3(1), dim3(64), 0, st, clk, t_user);
  return hipGetLastError();
}

hipError_t launch_clock3d_end(const Clock3D* clk, double* t_user, double* dt_user,
                              int32_t* status_user, int parity, hipStream_t st) {
  hipLaunchKernelGGL(clock3d_end_kernel, dim3(1), dim3(64), 0, st, clk, t_user, dt_user,
                     status_user, parity);
  return hipGetLastError();
}

template <int NW>
static int64_t weno3d_tiles(const Args3D& A) {
  using T = W3Tile<NW>;
  return ((A.c[0] + T::x - 1) / T::x) * ((A.c[1] + T::y - 1) / T::y) * ((A.c[2] + T::z - 1) / T::z);
}

hipError_t launch_weno3d(int NW, const Args3D& A, double* w, hipStream_t st) {
  const int64_t tiles = NW == 1 ? weno3d_tiles<1>(A) : NW == 2 ? weno3d_tiles<2>(A) : weno3d_tiles<3>(A);
  dim3 grid((unsigned)tiles), block(kFv3dThreads);
  if (NW == 1) hipLaunchKernelGGL((weno3d_kernel<1>), grid, block, 0, st, A, w);
  else if (NW == 2) hipLaunchKernelGGL((weno3d_kernel<2>), grid, block, 0, st, A, w);
  else if (NW == 3) hipLaunchKernelGGL((weno3d_kernel<3>), grid, block, 0, st, A, w);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fv3d_corr(int NW, const Args3D& A, hipStream_t st) {
  const int64_t tiles = ((A.c[0] + kF3 - 1) / kF3) * ((A.c[1] + kF3 - 1) / kF3) * ((A.c[2] + kF3 - 1) / kF3);
  dim3 grid((unsigned)tiles), block(kFv3dThreads);
  if (NW == 1) hipLaunchKernelGGL((fv3d_corr_kernel<1>), grid, block, 0, st, A);
  else if (NW == 2) hipLaunchKernelGGL((fv3d_corr_kernel<2>), grid, block, 0, st, A);
  else if (NW == 3) hipLaunchKernelGGL((fv3d_corr_kernel<3>), grid, block, 0, st, A);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fv3d_lambda(const Args3D& A, hipStream_t st) {
  const int64_t cells = A.c[0] * A.c[1] * A.c[2];
  dim3 grid((unsigned)((cells + kFv3dThreads - 1) / kFv3dThreads)), block(kFv3dThreads);
  hipLaunchKernelGGL(fv3d_lambda_kernel, grid, block, 0, st, A);
  return hipGetLastError();
}

hipError_t upload_tables_3d(const DevOps* ops, const DevOpsF* opsf, const DevWeno* weno) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c3_ops), ops, sizeof(DevOps) * kDevMaxn);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c3_opsf), opsf, sizeof(DevOpsF) * kDevMaxn);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c3_weno), weno, sizeof(DevWeno) * 3);
}

}  // namespace aderdg
