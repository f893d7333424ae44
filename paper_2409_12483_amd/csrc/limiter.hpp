// Kernels of the 1-D ADER-DG step with a posteriori subcell ADER-WENO2
// limiting (Sec. 1.4, Sec. 1.6) for the Euler gas.  Included once, by
// kernels.hip, so that they share its operator and WENO tables.
//
// One step is six launches on the problem's stream:
//   lim_clock     dt from the CFL rule (Sec. 1.5) over the subcell averages
//   lim_pred      LST-DG predictor of every cell and of the two ghost cells;
//                 per cell: the candidate's volume terms and the face traces
//                 of every time node
//   lim_cand      time-integrated Rusanov flux of every face, candidate
//                 u* = u + volume - surface (in place), PAD and NAD on its
//                 subcell averages, the list of troubled cells (one lane per
//                 (cell, node))
//   lim_subgrid   ADER-WENO step (WENO degree 1 or 2) on the subgrid of every
//                 troubled cell, from the stored subcell averages (one
//                 wavefront per cell)
//   lim_subgrid0  first-order redo of those subgrid steps, only when one of
//                 them left the admissible set
//   lim_finish    u = R v in troubled cells (scaled toward the mean when
//                 needed), the subgrid flux at their faces in the unlimited
//                 neighbours, new subcell averages and their per-cell
//                 extrema, the next step's signal speed
#pragma once

#include "device_common.hpp"
#include "dg_step.hpp"
#include "launch.hpp"
#include "launch_lim.hpp"
#include "predictor.hpp"

namespace aderdg {

__constant__ DevLimR c_limR[kDevMaxn];
__constant__ DevWeno c_weno1;           // WENO of degree 1 (two one-sided stencils)

constexpr int kLimM = 3;   // Euler: (rho, rho u, E)
constexpr double kLimDelta0 = 1.0e-4, kLimEps0 = 1.0e-3;   // NAD tolerances (Sec. 1.6)

// Index of subcell (or cell) j of a grid of S under the boundary condition:
// periodic wrap, or the mirror image across the domain ends (free outflow).
// *mirrored tells whether the image is reflected.
__device__ __forceinline__ int64_t lim_map(int64_t j, int64_t S, int bc, bool* mirrored) {
  if (bc == kLimPeriodic) {
    j %= S;
    if (j < 0) j += S;
    *mirrored = false;
    return j;
  }
  int64_t m = j % (2 * S);
  if (m < 0) m += 2 * S;
  *mirrored = m >= S;
  return m < S ? m : 2 * S - 1 - m;
}

__device__ __forceinline__ void lim_status(LimClock* clk, int64_t key, bool bad, bool failed) {
  const bool any_bad = __any(bad), any_fail = __any(failed);
  if ((threadIdx.x & 63) == 0 && (any_bad || any_fail)) {
    const int slot = (int)((key * 17 + (threadIdx.x >> 6)) % kSlots);
    atomicMin(&clk->stat[slot].v, any_bad ? -5 : -4);
  }
}

// Max of the wave's values into one of the clock's signal-speed slots.
__device__ __forceinline__ void lim_publish_lambda(LimClock* clk, int buf, double lam) {
  lam = wave_max(lam);
  if ((threadIdx.x & 63) == 0)
    atomic_max_nonneg(&clk->lam[buf][(blockIdx.x * 4 + (threadIdx.x >> 6)) % kSlots].v, lam);
}

// Rusanov flux whose signal speed is NaN when either state's is (a trace with
// negative pressure has no sound speed): such a flux makes the candidate, or
// the subgrid result, inadmissible, so the cell is limited, or the subgrid
// step falls back to first order.  (fmax would drop the NaN and keep the
// other state's speed.)
__device__ __forceinline__ void lim_rusanov(const double* qm, const double* qp, double* G, const PdeParams& p) {
  double fm[kLimM], fp[kLimM];
  Euler::flux(qm, fm, p);
  Euler::flux(qp, fp, p);
  const double sm = Euler::speed(qm, p), sp = Euler::speed(qp, p);
  const double s = (sm != sm || sp != sp) ? __builtin_nan("") : (sm > sp ? sm : sp);
#pragma unroll
  for (int r = 0; r < kLimM; ++r) G[r] = 0.5 * (fm[r] + fp[r]) - 0.5 * s * (qp[r] - qm[r]);
}

// max over the 2N+1 subcell averages of a cell's nodal state of |u| + c
template <int N>
__device__ __forceinline__ double lim_cell_speed(const double (&uc)[N + 1][kLimM], const PdeParams& pp) {
  double lam = 0.0;
#pragma unroll
  for (int s = 0; s < 2 * N + 1; ++s) {
    double v[kLimM];
#pragma unroll
    for (int r = 0; r < kLimM; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k <= N; ++k) acc += c_ops[N].P[s][k] * uc[k][r];
      v[r] = acc;
    }
    lam = dmax(lam, Euler::speed(v, pp));
  }
  return lam;
}

// Per-cell extrema of the subcell averages v (per variable), for the NAD
// window of the next step.
template <int Ns>
__device__ __forceinline__ void lim_store_extrema(const LimArgs& A, int64_t i, const double (&vs)[Ns][kLimM]) {
#pragma unroll
  for (int r = 0; r < kLimM; ++r) {
    double mn = vs[0][r], mx = vs[0][r];
#pragma unroll
    for (int s = 1; s < Ns; ++s) {
      mn = fmin(mn, vs[s][r]);
      mx = fmax(mx, vs[s][r]);
    }
    A.vext[(i * 2) * kLimM + r] = mn;
    A.vext[(i * 2 + 1) * kLimM + r] = mx;
  }
}

// ------------------------------------------------------------ clock ----
__global__ void lim_begin_kernel(LimClock* clk, const double* t_user) {
  const int i = threadIdx.x;
  if (i == 0) {
    clk->t = t_user[0];
    clk->t_next = t_user[0];
    clk->dt = 0.0;
    clk->dt_last = 0.0;
  }
  if (i < kSlots) {
    clk->lam[0][i].v = 0ull;
    clk->lam[1][i].v = 0ull;
    clk->stat[i].v = 0;
  }
}

__global__ void lim_end_kernel(const LimClock* clk, double* t_user, double* dt_user, int32_t* status_user) {
  if (threadIdx.x == 0) {
    t_user[0] = clk->t_next;
    dt_user[0] = clk->dt_last;
    int st = 0;
    for (int i = 0; i < kSlots; ++i) st = min(st, clk->stat[i].v);
    status_user[0] = st;
  }
}

// dt of step A.step from the signal speed of its start state (one wavefront)
__global__ void lim_clock_kernel(LimArgs A) {
  LimClock* clk = A.clk;
  const int lane = threadIdx.x;
  const int buf = A.step & 1;
  double lam = lane < kSlots ? from_bits(clk->lam[buf][lane].v) : 0.0;
  lam = wave_max(lam);
  if (lane < kSlots) {
    clk->lam[buf ^ 1][lane].v = 0ull;
    clk->ntr[lane].v = 0;
  }
  if (lane == 0) {
    const double t = clk->t_next;
    double dt = A.cfl_d * A.dx / ((2.0 * A.N + 1.0) * lam);
    const double rem = A.t_end[0] - t;
    if (dt > rem) dt = rem;
    if (!(dt > 0.0)) dt = 0.0;
    clk->t = t;
    clk->t_next = t + dt;
    clk->dt = dt;
    clk->fallback = 0;
    if (dt > 0.0) {
      clk->dt_last = dt;
      clk->total_steps += 1;
    }
  }
}

// ------------------------------------------------------ projection ----
template <int N>
__global__ void __launch_bounds__(256) lim_project_kernel(const double* u, double* v, int64_t C) {
  constexpr int n = N + 1, Ns = 2 * N + 1;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= C) return;
  double uc[n][kLimM];
#pragma unroll
  for (int k = 0; k < n; ++k)
#pragma unroll
    for (int r = 0; r < kLimM; ++r) uc[k][r] = u[(i * n + k) * kLimM + r];
#pragma unroll
  for (int s = 0; s < Ns; ++s)
#pragma unroll
    for (int r = 0; r < kLimM; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < n; ++k) acc += c_ops[N].P[s][k] * uc[k][r];
      v[(i * Ns + s) * kLimM + r] = acc;
    }
}

// signal speed of the state and the subcell extrema at the start of a call
// (one thread per cell)
template <int N>
__global__ void __launch_bounds__(256) lim_lambda_kernel(LimArgs A, int buf) {
  constexpr int n = N + 1;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double lam = 0.0;
  if (i < A.C) {
    double uc[n][kLimM];
#pragma unroll
    for (int k = 0; k < n; ++k)
#pragma unroll
      for (int r = 0; r < kLimM; ++r) uc[k][r] = A.u[(i * n + k) * kLimM + r];
    lam = lim_cell_speed<N>(uc, A.pp);
    constexpr int Ns = 2 * N + 1;
    double vs[Ns][kLimM];
#pragma unroll
    for (int s = 0; s < Ns; ++s)
#pragma unroll
      for (int r = 0; r < kLimM; ++r) vs[s][r] = A.v[(i * Ns + s) * kLimM + r];
    lim_store_extrema<Ns>(A, i, vs);
  }
  lim_publish_lambda(A.clk, buf, lam);
}

// -------------------------------------------------------- predictor ----
// LST-DG predictor of the padded cells p = 0..C+1 (cell p-1; p = 0 and C+1
// are the ghosts), lanes as in the fused step: one lane per (cell, time row).
template <int N, int WAVES>
__global__ void __launch_bounds__(WAVES * 64)
__attribute__((amdgpu_waves_per_eu(DgOccupancy<N, Euler>::value)))
lim_pred_kernel(LimArgs A) {
  using G = Geo<N, kLimM, WAVES, false>;
  constexpr int n = G::n, M = kLimM, CPW = G::CPW, PC = G::PC, RSD = G::RSD;
  using Pred = Predictor<N, Euler, double, false, false>;
  __shared__ double xb_all[WAVES * G::XB];
  __shared__ double red_all[WAVES * G::RED];

  const double dt = A.clk->dt;
  if (!(dt > 0.0)) return;
  const double t0 = A.clk->t;
  const int64_t C = A.C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot0 = lane / n;
  const bool active = slot0 < CPW;
  const int slot = active ? slot0 : 0;
  const int a = active ? lane % n : lane - CPW * n;
  const int64_t p = (int64_t)blockIdx.x * PC + wave * CPW + slot;   // padded cell
  const bool out = active && p < C + 2;
  bool mir = false;
  const int64_t gc = lim_map(p - 1, C, A.bc, &mir);
  const double* ucell = A.u + gc * (n * M);
  double* xb = xb_all + wave * G::XB + slot * G::CBD;
  double* xbp = pred_block<G, double>(xb_all, wave, slot);
  double* red = red_all + wave * G::RED + (active ? slot : CPW) * 2;
  const PdeParams pp = A.pp;
  const double dx = A.dx, dtdx = dt / dx;
  const double xl = A.x0 + dx * (double)(p - 1);

  double q[n][M], ucol[M];
#pragma unroll
  for (int l = 0; l < n; ++l)
#pragma unroll
    for (int r = 0; r < M; ++r) q[l][r] = ucell[(mir ? n - 1 - l : l) * M + r];
  const int an = a < n ? a : 0;
#pragma unroll
  for (int r = 0; r < M; ++r) ucol[r] = ucell[(mir ? n - 1 - an : an) * M + r];
  int sweeps = 0, contractions = 0;
  bool failed = false;
  Pred::run(q, ucol, a, xbp, red, dt, dtdx, xl, dx, t0, pp, A.tol, A.max_iter, false, active, sweeps,
            contractions, failed);

  // row a's share of the volume term at node k: w_a (dt/dx) (D~ F)_k / w_k
  const double wdx = c_ops[N].w[an] * dtdx;
  double fd[n][M];
#pragma unroll
  for (int l = 0; l < n; ++l) Euler::flux(q[l], fd[l], pp);
  wave_sync();
#pragma unroll
  for (int k = 0; k < n; ++k) {
#pragma unroll
    for (int r = 0; r < M; ++r) {
      double acc = c_ops[N].Dw[k][0] * fd[0][r];
#pragma unroll
      for (int l = 1; l < n; ++l) acc += c_ops[N].Dw[k][l] * fd[l][r];
      if (active) xb[a * RSD + k * M + r] = wdx * acc;
    }
  }
  double sl[M], sr[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    sl[r] = 0.0;
    sr[r] = 0.0;
#pragma unroll
    for (int j = 0; j < n; ++j) {
      sl[r] += c_ops[N].psi0[j] * q[j][r];
      sr[r] += c_ops[N].psi1[j] * q[j][r];
    }
  }
  wave_sync();
  if (out) {
#pragma unroll
    for (int r = 0; r < M; ++r) {
      A.trL[(p * n + a) * M + r] = sl[r];
      A.trR[(p * n + a) * M + r] = sr[r];
    }
    if (p >= 1 && p <= C) {
      // column role: lane a = space node k, the volume term summed over time rows
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < n; ++b) acc += xb[b * RSD + a * M + r];
        A.vol[((p - 1) * n + a) * M + r] = acc;
      }
    }
  }
  const unsigned long long sw = wave_sum((out && a == 0 && p >= 1 && p <= C) ? (unsigned long long)(sweeps & 0xffff) : 0ull);
  if (lane == 0 && sw) atomicAdd(&A.clk->sweeps[(blockIdx.x * WAVES + wave) % kSlots].v, sw);
  lim_status(A.clk, blockIdx.x, false, failed && out);
}

// ------------------------------------------- faces, candidate, detectors ----
// Lanes as in the predictor: lane a of a cell is time node a for the face
// fluxes and space node a for the candidate.  Each cell computes the
// time-integrated Rusanov flux of both its faces (a face's two cells do the
// same arithmetic on the same traces, so they agree bit for bit), then
// u* = u + volume - surface at node a (in place), PAD at the node; the
// candidate's subcell averages s = a and s = a + n go through NAD against the
// per-cell subcell extrema of V_i and PAD; a troubled cell joins the list.
constexpr int kLimCandWaves = 4;

template <int N>
__global__ void __launch_bounds__(kLimCandWaves * 64) lim_cand_kernel(LimArgs A) {
  constexpr int n = N + 1, M = kLimM, Ns = 2 * N + 1, CPW = 64 / n;
  constexpr int CB = CPW * n * M;                       // doubles of one wave's cell blocks
  __shared__ double sx[kLimCandWaves * CB];             // per cell: [n][M] face-flux parts, then u*
  __shared__ int sbad[kLimCandWaves * CPW];
  const int64_t C = A.C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot0 = lane / n;
  const bool active = slot0 < CPW;
  const int slot = active ? slot0 : 0;
  const int a = active ? lane % n : 0;
  const int64_t i = ((int64_t)blockIdx.x * kLimCandWaves + wave) * CPW + slot;
  const bool live = active && i < C;
  const double dt = A.clk->dt;
  if (!(dt > 0.0)) {
    if (live && a == 0) A.troubled[i] = 0;
    return;
  }
  const double dtdx = dt / A.dx;
  const PdeParams pp = A.pp;
  double* blk = sx + wave * CB + slot * (n * M);
  // face fluxes: lane a takes time node a of both faces
  double GL[M], GR[M];
  {
    const int64_t ic = live ? i : 0;
    double qm[M], qp[M], hl[M], hr[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      qm[r] = A.trR[(ic * n + a) * M + r];              // padded cell i: cell i-1
      qp[r] = A.trL[((ic + 1) * n + a) * M + r];        // padded cell i+1: cell i
    }
    lim_rusanov(qm, qp, hl, pp);
#pragma unroll
    for (int r = 0; r < M; ++r) {
      qm[r] = A.trR[((ic + 1) * n + a) * M + r];
      qp[r] = A.trL[((ic + 2) * n + a) * M + r];
    }
    lim_rusanov(qm, qp, hr, pp);
    const double wa = c_ops[N].w[a] * dtdx;
    // the two faces' weighted parts through the cell's block, summed over a in order
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      wave_sync();
      if (active) {
#pragma unroll
        for (int r = 0; r < M; ++r) blk[a * M + r] = wa * (side ? hr[r] : hl[r]);
      }
      wave_sync();
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < n; ++b) acc += blk[b * M + r];
        (side ? GR : GL)[r] = acc;
      }
    }
  }
  if (live && a == 0) {
#pragma unroll
    for (int r = 0; r < M; ++r) {
      A.G[(i + 1) * M + r] = GR[r];
      if (i == 0) A.G[r] = GL[r];
    }
  }
  // candidate at node a
  double uk[M];
  bool bad = false;
  {
    const int64_t ic = live ? i : 0;
    const double winv = c_ops[N].winv[a], p0 = c_ops[N].psi0[a], p1 = c_ops[N].psi1[a];
#pragma unroll
    for (int r = 0; r < M; ++r)
      uk[r] = A.u[(ic * n + a) * M + r] + A.vol[(ic * n + a) * M + r] - winv * (p1 * GR[r] - p0 * GL[r]);
    if (live) {
#pragma unroll
      for (int r = 0; r < M; ++r) A.u[(i * n + a) * M + r] = uk[r];
      bad = !Euler::admissible(uk, pp);
    }
  }
  wave_sync();
  if (active) {
#pragma unroll
    for (int r = 0; r < M; ++r) blk[a * M + r] = uk[r];
    if (a == 0) sbad[wave * CPW + slot] = 0;
  }
  wave_sync();
  if (live) {
    // V_i: the cell and its face neighbours (one neighbour at a free-outflow end)
    int64_t il = i - 1, ir = i + 1;
    if (A.bc == kLimPeriodic) {
      if (il < 0) il += C;
      if (ir >= C) ir -= C;
    } else {
      if (il < 0) il = 0;
      if (ir >= C) ir = C - 1;
    }
    double lo[M], hi[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const double mn = fmin(fmin(A.vext[(il * 2) * M + r], A.vext[(i * 2) * M + r]), A.vext[(ir * 2) * M + r]);
      const double mx = fmax(fmax(A.vext[(il * 2 + 1) * M + r], A.vext[(i * 2 + 1) * M + r]),
                             A.vext[(ir * 2 + 1) * M + r]);
      const double delta = fmax(kLimDelta0, kLimEps0 * (mx - mn));
      lo[r] = mn - delta;
      hi[r] = mx + delta;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int s = a + h * n;
      if (s < Ns) {
        double vs[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < n; ++k) acc += c_ops[N].P[s][k] * blk[k * M + r];
          vs[r] = acc;
          bad |= !(acc >= lo[r] && acc <= hi[r]);
        }
        bad |= !Euler::admissible(vs, pp);
      }
    }
    if (bad) sbad[wave * CPW + slot] = 1;
  }
  wave_sync();
  // append to sub-list blockIdx % kSlots: one atomic per wavefront, so that
  // thousands of troubled cells do not serialise on one counter
  const bool tb = live && a == 0 && sbad[wave * CPW + slot] != 0;
  if (live && a == 0) A.troubled[i] = tb ? 1 : 0;
  const unsigned long long mask = __ballot(tb);
  if (mask) {
    const int k = (int)(blockIdx.x % kSlots);
    int base = 0;
    if (lane == 0) base = atomicAdd(&A.clk->ntr[k].v, __popcll(mask));
    base = __shfl(base, 0, 64);
    if (tb) A.list[k * A.list_cap + base + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)i;
  }
}

// Entry b of the step's troubled list (sub-lists in slot order); counts[k]
// holds sub-list k's length in every lane of the calling wavefront's registers.
__device__ __forceinline__ int64_t lim_list_entry(const LimArgs& A, int cnt_lane, int b) {
  int k = 0;
  for (; k < kSlots; ++k) {
    const int c = __shfl(cnt_lane, k, 64);
    if (b < c) break;
    b -= c;
  }
  return A.list[k * A.list_cap + b];
}

// Sub-list lengths (lane k holds sub-list k's) and their total.
__device__ __forceinline__ int lim_list_counts(const LimArgs& A, int* total) {
  const int lane = threadIdx.x & 63;
  const int c = lane < kSlots ? A.clk->ntr[lane].v : 0;
  int t = c;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  *total = t;
  return c;
}

// ------------------------------------------------- subgrid ADER-WENO ----
// One wavefront per troubled cell: its N_s subcells plus one on each side
// are reconstructed (WENO of degree NW from the stored subcell averages, the
// boundary condition applied on the subgrid; NW = 1 is the paper's
// ADER-WENO2, NW = 2 ADER-WENO3), predicted (LST-DG of degree NW) and
// updated; the fluxes through the cell's two faces are kept.
template <int N, int NW>
__global__ void __launch_bounds__(64) lim_subgrid_kernel(LimArgs A) {
  constexpr int M = kLimM, Ns = 2 * N + 1;
  constexpr int NS = NW == 1 ? 2 : 3;              // stencils
  const DevWeno& WT = NW == 1 ? c_weno1 : c_weno[0];
  using G = Geo<NW, M, 1, true>;
  constexpr int n = G::n, CPW = G::CPW, PC = G::PC;
  constexpr int NV = PC + 2 * NW;
  static_assert(Ns + 2 <= PC, "a cell's subgrid and its two halo subcells fit one wavefront");
  using Pred = Predictor<NW, Euler, double, false, false>;
  __shared__ double vb[NV * M];
  __shared__ double xb_all[G::XB];
  __shared__ double red_all[G::RED];
  auto trL = [&](int cell) { return xb_all + cell * G::CBD; };
  auto trR = [&](int cell) { return trL(cell) + G::RSD; };

  const double dt = A.clk->dt;
  if (!(dt > 0.0)) return;
  int ntr;
  const int cnt = lim_list_counts(A, &ntr);
  const int64_t S = A.C * Ns;
  const double dxs = A.dx / Ns, dtdx = dt / dxs;
  const double t0 = A.clk->t;
  const PdeParams pp = A.pp;
  const int lane = threadIdx.x;
  const int slot0 = lane / n;
  const bool active = slot0 < CPW;
  const int pc = active ? slot0 : 0;
  const int a = active ? lane % n : lane - CPW * n;
  const int an = a < n ? a : 0;
  double* xb = xb_all + pc * G::CBD;
  double* xbp = pred_block<G, double>(xb_all, 0, pc);
  double* red = red_all + (active ? pc : CPW) * 2;

  for (int b = blockIdx.x; b < ntr; b += gridDim.x) {
    const int64_t i = lim_list_entry(A, cnt, b);
    const int64_t j0 = i * Ns;                     // first subcell of the cell
    __syncthreads();
    for (int e = lane; e < NV * M; e += 64) {
      const int cc = e / M, r = e % M;
      bool mir;
      const int64_t j = lim_map(j0 - 1 - NW + cc, S, A.bc, &mir);
      vb[e] = A.v[j * M + r];
    }
    __syncthreads();
    // WENO reconstruction at node a (the indicator on differences from the
    // subcell's own average, as in the finite-volume step)
    double what[M];
    {
      const int base = pc + NW;
      double wsum[M], acc[M];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int off = NW == 1 ? s - 1 : (s == 0 ? -NW : (s == 1 ? -NW / 2 : 0));
        const double lam = (NW != 1 && s == 1) ? 1.0e5 : 1.0;
#pragma unroll
        for (int r = 0; r < M; ++r) {
          double v[n], d[n];
          const double vc = vb[base * M + r];
#pragma unroll
          for (int q = 0; q < n; ++q) {
            v[q] = vb[(base + off + q) * M + r];
            d[q] = v[q] - vc;
          }
          double sig = 0.0, val = 0.0;
#pragma unroll
          for (int q = 0; q < n; ++q) {
            double si = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) si += WT.S[s][q][k] * d[k];
            sig += d[q] * si;
            val += WT.R[s][an][q] * v[q];
          }
          const double e = sig + 1.0e-14;
          const double e2 = e * e, e4 = e2 * e2, e8 = e4 * e4;
          const double om = lam / e8;
          wsum[r] = s == 0 ? om : wsum[r] + om;
          acc[r] = s == 0 ? om * val : acc[r] + om * val;
        }
      }
#pragma unroll
      for (int r = 0; r < M; ++r) what[r] = acc[r] / wsum[r];
    }
    wave_sync();
    if (active) {
#pragma unroll
      for (int r = 0; r < M; ++r) xb[a * M + r] = what[r];
    }
    wave_sync();
    double q[n][M];
#pragma unroll
    for (int l = 0; l < n; ++l)
#pragma unroll
      for (int r = 0; r < M; ++r) q[l][r] = xb[l * M + r];
    int sweeps = 0, contractions = 0;
    bool failed = false;
    const double xl = A.x0 + dxs * (double)(j0 - 1 + pc);
    Pred::run(q, what, a, xbp, red, dt, dtdx, xl, dxs, t0, pp, A.tol, A.max_iter, false, active,
              sweeps, contractions, failed);
    // face traces of time node a, then the weighted Rusanov flux at the face on each subcell's right
    wave_sync();
    if (active) {
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double sl = 0.0, sr = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) {
          sl += c_ops[NW].psi0[k] * q[k][r];
          sr += c_ops[NW].psi1[k] * q[k][r];
        }
        trL(pc)[a * M + r] = sl;
        trR(pc)[a * M + r] = sr;
      }
    }
    __syncthreads();
    const double wa = c_ops[NW].w[an];
    if (active && pc < PC - 1) {
      double qm[M], qp[M], g[M];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        qm[r] = trR(pc)[a * M + r];
        qp[r] = trL(pc + 1)[a * M + r];
      }
      lim_rusanov(qm, qp, g, pp);
#pragma unroll
      for (int r = 0; r < M; ++r) trR(pc)[a * M + r] = wa * dtdx * g[r];
    }
    __syncthreads();
    bool bad = false;
    if (active && a == 0 && pc >= 1 && pc <= Ns) {
      double vnew[M];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double GR = 0.0, GL = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) {
          GR += trR(pc)[k * M + r];
          GL += trR(pc - 1)[k * M + r];
        }
        vnew[r] = vb[(pc + NW) * M + r] - (GR - GL);
        A.vfv[(j0 + pc - 1) * M + r] = vnew[r];
        if (pc == 1) A.gs[(i * 2 + 0) * M + r] = GL;
        if (pc == Ns) A.gs[(i * 2 + 1) * M + r] = GR;
      }
      bad = !Euler::admissible(vnew, pp);
    }
    if (__any(bad) && lane == 0) atomicOr(&A.clk->fallback, 1);
    lim_status(A.clk, b, false, failed && active && pc <= Ns + 1);
  }
}

// First-order (Rusanov finite-volume) redo of every troubled cell's subgrid
// step, when one of the ADER-WENO2 subgrid steps left the admissible set.
template <int N>
__global__ void __launch_bounds__(64) lim_subgrid0_kernel(LimArgs A) {
  constexpr int M = kLimM, Ns = 2 * N + 1;
  __shared__ double F[(Ns + 1) * M];
  const double dt = A.clk->dt;
  if (!(dt > 0.0) || !A.clk->fallback) return;
  int ntr;
  const int cnt = lim_list_counts(A, &ntr);
  const int64_t S = A.C * Ns;
  const double dtdx = dt / (A.dx / Ns);
  const int s = threadIdx.x;
  for (int b = blockIdx.x; b < ntr; b += gridDim.x) {
    const int64_t i = lim_list_entry(A, cnt, b);
    const int64_t j0 = i * Ns;
    __syncthreads();
    if (s <= Ns) {
      bool mir;
      const int64_t jl = lim_map(j0 + s - 1, S, A.bc, &mir), jr = lim_map(j0 + s, S, A.bc, &mir);
      double qm[M], qp[M], g[M];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        qm[r] = A.v[jl * M + r];
        qp[r] = A.v[jr * M + r];
      }
      lim_rusanov(qm, qp, g, A.pp);
#pragma unroll
      for (int r = 0; r < M; ++r) F[s * M + r] = dtdx * g[r];
    }
    __syncthreads();
    if (s < Ns) {
#pragma unroll
      for (int r = 0; r < M; ++r)
        A.vfv[(j0 + s) * M + r] = A.v[(j0 + s) * M + r] - (F[(s + 1) * M + r] - F[s * M + r]);
    }
    if (s < M) {
      A.gs[(i * 2 + 0) * M + s] = F[s];
      A.gs[(i * 2 + 1) * M + s] = F[Ns * M + s];
    }
  }
}

// ------------------------------------------------------------ finish ----
template <int N>
__global__ void __launch_bounds__(256) lim_finish_kernel(LimArgs A) {
  constexpr int n = N + 1, M = kLimM, Ns = 2 * N + 1;
  const int64_t C = A.C;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  LimClock* clk = A.clk;
  const double dt = clk->dt;
  const PdeParams pp = A.pp;
  if (blockIdx.x == 0 && threadIdx.x == 0 && dt > 0.0) {
    int ntr = 0;
    for (int k = 0; k < kSlots; ++k) ntr += clk->ntr[k].v;
    clk->total_troubled += (unsigned long long)ntr;
    if (clk->fallback) clk->total_fallback += 1;
  }
  double uc[n][M];
  double lam = 0.0;
  bool bad = false;
  if (i < C) {
    if (dt > 0.0 && A.troubled[i]) {
      double vs[Ns][M], m[M];
#pragma unroll
      for (int r = 0; r < M; ++r) m[r] = 0.0;
#pragma unroll
      for (int s = 0; s < Ns; ++s)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          vs[s][r] = A.vfv[(i * Ns + s) * M + r];
          m[r] += vs[s][r];
        }
#pragma unroll
      for (int r = 0; r < M; ++r) m[r] /= (double)Ns;
      double rv[n][M];
#pragma unroll
      for (int k = 0; k < n; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int s = 0; s < Ns; ++s) acc += c_limR[N].R[k][s] * vs[s][r];
          rv[k][r] = acc;
        }
      // largest theta in {1, 1/2, ..., 2^-11} with u and P u admissible, else the mean
      double theta = 1.0;
      bool ok = false;
      for (int it = 0; it < 12 && !ok; ++it) {
#pragma unroll
        for (int k = 0; k < n; ++k)
#pragma unroll
          for (int r = 0; r < M; ++r) uc[k][r] = m[r] + theta * (rv[k][r] - m[r]);
        ok = true;
#pragma unroll
        for (int k = 0; k < n; ++k) ok &= Euler::admissible(uc[k], pp);
#pragma unroll
        for (int s = 0; s < Ns; ++s) {
          double w[M];
#pragma unroll
          for (int r = 0; r < M; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) acc += c_ops[N].P[s][k] * uc[k][r];
            w[r] = acc;
          }
          ok &= Euler::admissible(w, pp);
        }
        theta *= 0.5;
      }
      if (!ok) {
#pragma unroll
        for (int k = 0; k < n; ++k)
#pragma unroll
          for (int r = 0; r < M; ++r) uc[k][r] = m[r];
      }
#pragma unroll
      for (int k = 0; k < n; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) A.u[(i * n + k) * M + r] = uc[k][r];
#pragma unroll
      for (int s = 0; s < Ns; ++s)
#pragma unroll
        for (int r = 0; r < M; ++r) A.v[(i * Ns + s) * M + r] = vs[s][r];
      lim_store_extrema<Ns>(A, i, vs);
    } else {
#pragma unroll
      for (int k = 0; k < n; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) uc[k][r] = A.u[(i * n + k) * M + r];
      if (dt > 0.0) {
        // one flux per face: the subgrid flux where a troubled neighbour touches it
        const bool per = A.bc == kLimPeriodic;
        const int64_t il = i > 0 ? i - 1 : (per ? C - 1 : -1);
        const int64_t ir = i < C - 1 ? i + 1 : (per ? 0 : -1);
        bool changed = false;
        if (il >= 0 && A.troubled[il]) {
#pragma unroll
          for (int r = 0; r < M; ++r) {
            const double dG = A.gs[(il * 2 + 1) * M + r] / (double)Ns - A.G[i * M + r];
#pragma unroll
            for (int k = 0; k < n; ++k) uc[k][r] += c_ops[N].psi0[k] * c_ops[N].winv[k] * dG;
          }
          changed = true;
        }
        if (ir >= 0 && A.troubled[ir]) {
#pragma unroll
          for (int r = 0; r < M; ++r) {
            const double dG = A.gs[(ir * 2 + 0) * M + r] / (double)Ns - A.G[(i + 1) * M + r];
#pragma unroll
            for (int k = 0; k < n; ++k) uc[k][r] -= c_ops[N].psi1[k] * c_ops[N].winv[k] * dG;
          }
          changed = true;
        }
        if (changed) {
#pragma unroll
          for (int k = 0; k < n; ++k)
#pragma unroll
            for (int r = 0; r < M; ++r) A.u[(i * n + k) * M + r] = uc[k][r];
        }
        double vs[Ns][M];
#pragma unroll
        for (int s = 0; s < Ns; ++s)
#pragma unroll
          for (int r = 0; r < M; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) acc += c_ops[N].P[s][k] * uc[k][r];
            vs[s][r] = acc;
            A.v[(i * Ns + s) * M + r] = acc;
          }
        lim_store_extrema<Ns>(A, i, vs);
      }
    }
#pragma unroll
    for (int k = 0; k < n; ++k) bad |= !Euler::admissible(uc[k], pp);
    lam = lim_cell_speed<N>(uc, pp);
  }
  lim_publish_lambda(clk, (A.step + 1) & 1, lam);
  lim_status(clk, blockIdx.x, bad, false);
}

// ---------------------------------------------------------- launches ----
template <int N>
static hipError_t launch_lim_step_n(const LimArgs& A, hipStream_t st) {
  constexpr int kWaves = 4;
  const int64_t C = A.C;
  const int64_t pc = (int64_t)kWaves * (64 / (N + 1));
  const unsigned cb = (unsigned)((C + 255) / 256);
  const int64_t kc = (int64_t)kLimCandWaves * (64 / (N + 1));
  const unsigned kb = (unsigned)((C + kc - 1) / kc);
  LimArgs B = A;
  B.list_cap = ((int64_t)kb + kSlots - 1) / kSlots * kc;   // cells of the workgroups of one sub-list
  const unsigned pb = (unsigned)((C + 2 + pc - 1) / pc);
  const unsigned sb = (unsigned)(C < kLimSubgridBlocks ? C : kLimSubgridBlocks);
  hipLaunchKernelGGL(lim_clock_kernel, dim3(1), dim3(64), 0, st, B);
  hipLaunchKernelGGL((lim_pred_kernel<N, kWaves>), dim3(pb), dim3(kWaves * 64), 0, st, B);
  hipLaunchKernelGGL((lim_cand_kernel<N>), dim3(kb), dim3(kLimCandWaves * 64), 0, st, B);
  if (A.weno == 1)
    hipLaunchKernelGGL((lim_subgrid_kernel<N, 1>), dim3(sb), dim3(64), 0, st, B);
  else
    hipLaunchKernelGGL((lim_subgrid_kernel<N, 2>), dim3(sb), dim3(64), 0, st, B);
  hipLaunchKernelGGL((lim_subgrid0_kernel<N>), dim3(sb), dim3(64), 0, st, B);
  hipLaunchKernelGGL((lim_finish_kernel<N>), dim3(cb), dim3(256), 0, st, B);
  return hipGetLastError();
}

hipError_t launch_lim_step(const LimArgs& A, hipStream_t st) {
  switch (A.N) {
#define ADERDG_CASE(NN) case NN: return launch_lim_step_n<NN>(A, st);
    ADERDG_CASE(1) ADERDG_CASE(2) ADERDG_CASE(3) ADERDG_CASE(4) ADERDG_CASE(5)
    ADERDG_CASE(6) ADERDG_CASE(7) ADERDG_CASE(8) ADERDG_CASE(9)
#undef ADERDG_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lim_lambda(const LimArgs& A, int buf, hipStream_t st) {
  const unsigned cb = (unsigned)((A.C + 255) / 256);
  switch (A.N) {
#define ADERDG_CASE(NN) case NN: hipLaunchKernelGGL((lim_lambda_kernel<NN>), dim3(cb), dim3(256), 0, st, A, buf); break;
    ADERDG_CASE(1) ADERDG_CASE(2) ADERDG_CASE(3) ADERDG_CASE(4) ADERDG_CASE(5)
    ADERDG_CASE(6) ADERDG_CASE(7) ADERDG_CASE(8) ADERDG_CASE(9)
#undef ADERDG_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lim_project(int N, const double* u, double* v, int64_t C, hipStream_t st) {
  const unsigned cb = (unsigned)((C + 255) / 256);
  switch (N) {
#define ADERDG_CASE(NN) case NN: hipLaunchKernelGGL((lim_project_kernel<NN>), dim3(cb), dim3(256), 0, st, u, v, C); break;
    ADERDG_CASE(1) ADERDG_CASE(2) ADERDG_CASE(3) ADERDG_CASE(4) ADERDG_CASE(5)
    ADERDG_CASE(6) ADERDG_CASE(7) ADERDG_CASE(8) ADERDG_CASE(9)
#undef ADERDG_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lim_begin(LimClock* clk, const double* t_user, hipStream_t st) {
  hipLaunchKernelGGL(lim_begin_kernel, dim3(1), dim3(64), 0, st, clk, t_user);
  return hipGetLastError();
}

hipError_t launch_lim_end(const LimClock* clk, double* t_user, double* dt_user, int32_t* status_user,
                          hipStream_t st) {
  hipLaunchKernelGGL(lim_end_kernel, dim3(1), dim3(64), 0, st, clk, t_user, dt_user, status_user);
  return hipGetLastError();
}

hipError_t upload_lim_tables(const DevLimR* r, const DevWeno* weno1) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_limR), r, sizeof(DevLimR) * kDevMaxn);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_weno1), weno1, sizeof(DevWeno));
}

}  // namespace aderdg
