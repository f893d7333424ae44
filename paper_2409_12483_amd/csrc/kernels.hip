// HIP kernels of the 1-D ADER-DG / ADER-WENO-FV hot path for gfx950.
//
// One translation unit holds every kernel so that the constant-memory
// operator tables need no relocatable device code.  Kernels:
//   dg_kernel<MODE>   predictor only / corrector only / fused step
//                     (Secs. 1.1-1.2, Algorithms 1-7)
//   fv_kernel         ADER-WENO finite-volume step (Sec. 1.3, Algorithms 8-11)
//   lambda_kernel     max signal speed for the CFL rule (Secs. 1.4-1.5)
//   clock kernels     per-problem device time / dt / status bookkeeping
//
// Fused step, per workgroup of WAVES wavefronts: a tile of consecutive
// cells plus one halo cell on each side, whose predictor is recomputed
// redundantly so that the neighbour traces never leave the chip.  Each
// cell is served by n = N+1 lanes (lane a = time row a of the predictor
// tile, see predictor.hpp).  After the predictor:
//   volume terms   in-lane (row a), summed over time rows through LDS;
//   face traces    in-lane (psi, psi~ contractions), staged in LDS;
//   Riemann flux   per (face, time node) by the left cell's lane a;
//   surface update per (cell, space node) in column layout, AoS store;
//   epilogue       signal speed on the 2N+1 subcell averages of u^{n+1} and
//                  the work counters, reduced over the workgroup into one
//                  64-bit atomic per quantity on a clock slot (exact).
#include "device_common.hpp"
#include "launch.hpp"
#include "predictor.hpp"
#include "dg_step.hpp"

namespace aderdg {

__constant__ DevOps c_ops[kDevMaxn];
__constant__ DevOpsF c_opsf[kDevMaxn];
__constant__ DevWeno c_weno[2];  // WENO degree 2 and 4

// ------------------------------------------------------------------ FV ----
// ADER-WENO-FV step: WENO reconstruction (degree NW) -> predictor -> FV update.
template <int NW, class PDE, class TP, int WAVES>
__global__ void __launch_bounds__(WAVES * 64)
fv_kernel(StepArgs A) {
  using G = Geo<NW, PDE::M, WAVES, true>;
  constexpr int n = G::n, M = PDE::M, CPW = G::CPW, PC = G::PC;
  constexpr int NV = PC + 2 * NW;   // cell averages staged: predictor cells + WENO reach
  using Pred = Predictor<NW, PDE, TP, sizeof(TP) == 4 && kFp32Mfma>;
  constexpr int wi = NW / 2 - 1;    // c_weno index

  __shared__ double vb[NV * M];
  __shared__ double xb_all[WAVES * G::XB];
  __shared__ TP red_all[WAVES * G::RED];
  __shared__ double jmp[PDE::kNcp ? PC * n * M : 1];
  __shared__ double lam_wave[WAVES];
  __shared__ unsigned long long sw_wave[WAVES];
  __shared__ double bcast;

  // After the predictor, every cell's exchange block holds its left traces
  // [a][r], right traces [a][r] (later the weighted face flux) and weighted
  // volume source terms [a][r].
  auto trL = [&](int cell) { return xb_all + (cell / CPW) * G::XB + (cell % CPW) * G::CBD; };
  auto trR = [&](int cell) { return trL(cell) + G::RSD; };
  auto volb = [&](int cell) { return trL(cell) + 2 * G::RSD; };

  const int pidx = find_problem(A.probs, A.nprob, blockIdx.x);
  const ProbDev& P = A.probs[pidx];
  StepCtx c;
  c.tile = (int64_t)blockIdx.x - P.tile_begin;
  const int64_t C = P.ncells;
  const int64_t first = c.tile * G::TILE;
  if (first >= C) return;
  const int64_t count = (C - first < G::TILE) ? C - first : G::TILE;
  // stage cell averages of cells first-1-NW .. first-1+PC+NW-1 (periodic);
  // issued before the clock read so that the two latencies overlap
  {
    const double* v_src = P.state[A.step & 1];
    for (int i = threadIdx.x; i < NV * M; i += blockDim.x) {
      const int cc = i / M, r = i % M;
      int64_t g = first - 1 - NW + cc;
      if (g < 0) g += C;
      if (g >= C) g -= C;
      if (g < 0 || g >= C) {                            // meshes smaller than the stencil reach
        g %= C;
        if (g < 0) g += C;
      }
      vb[i] = v_src[g * M + r];
    }
  }
  if (!step_setup<false, NW>(A, P, c, &bcast)) {
    copy_tile(c.u_in, c.u_out, first, count, M);
    return;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot0 = lane / n;
  const bool active = slot0 < CPW;
  const int slot = active ? slot0 : 0;
  const int a = active ? lane % n : lane - CPW * n;
  const int pc = wave * CPW + slot;
  int64_t gc = first + pc - 1;
  if (gc < 0) gc += C;
  if (gc >= C) {
    gc -= C;
    if (gc >= C) gc %= C;                                // meshes smaller than a tile
  }
  const bool out_cell = active && pc >= 1 && pc <= PC - 2 && (first + pc - 1) < C;
  double* xb = xb_all + wave * G::XB + slot * G::CBD;
  TP* xbp = pred_block<G, TP>(xb_all, wave, slot);
  TP* red = red_all + wave * G::RED + (active ? slot : CPW) * 2;   // idle lanes: a pair of their own
  const PdeParams pp = P.pp;
  const int max_iter = P.max_iter;
  const double dx = P.dx, dt = c.dt, dtdx = dt / dx;
  const double xl = P.x0 + dx * (double)gc;

  // ---- WENO reconstruction at node a (reading of eq. weno_reconstr) ----
  // Stencils outermost: the oscillation-indicator form of one stencil (wave-
  // uniform, scalar registers) is live for all M variables, then released.
  // The indicator is a quadratic form that vanishes on constants, so it is
  // evaluated on the averages minus the cell's own: on nearly constant data
  // the form of the raw averages would cancel to round-off of |v|^2, which
  // the weights' (sigma + eps)^-8 would amplify.
  double what[M];
  {
    const int base = (active ? pc : 0) + NW;   // vb index of this cell
    double wsum[M], acc[M];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int off = s == 0 ? -NW : (s == 1 ? -NW / 2 : 0);
      const cptr<double> S = opaque((cptr<double>)&c_weno[wi].S[s][0][0]);
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double v[n], d[n];
        const double vc = vb[base * M + r];
#pragma unroll
        for (int i = 0; i < n; ++i) {
          v[i] = vb[(base + off + i) * M + r];
          d[i] = v[i] - vc;
        }
        double sig = 0.0, val = 0.0;
#pragma unroll
        for (int i = 0; i < n; ++i) {
          double si = 0.0;
#pragma unroll
          for (int j = 0; j < n; ++j) si += S[i * kWenoMaxn + j] * d[j];
          sig += d[i] * si;
          val += c_weno[wi].R[s][a < n ? a : 0][i] * v[i];
        }
        const double e = sig + 1.0e-14;
        const double e2 = e * e, e4 = e2 * e2, e8 = e4 * e4;
        const double om = (s == 1 ? 1.0e5 : 1.0) / e8;
        wsum[r] = s == 0 ? om : wsum[r] + om;
        acc[r] = s == 0 ? om * val : acc[r] + om * val;
      }
    }
#pragma unroll
    for (int r = 0; r < M; ++r) what[r] = acc[r] / wsum[r];
  }
  // broadcast the reconstruction to every row of the cell
  wave_sync();
  if (active) {
#pragma unroll
    for (int r = 0; r < M; ++r) xb[a * M + r] = what[r];
  }
  wave_sync();
  TP q[n][M], ucol[M];
#pragma unroll
  for (int l = 0; l < n; ++l)
#pragma unroll
    for (int r = 0; r < M; ++r) q[l][r] = TP(xb[l * M + r]);
#pragma unroll
  for (int r = 0; r < M; ++r) ucol[r] = TP(what[r]);
  int sweeps = 0, contractions = 0;
  bool failed = false;
  Pred::run(q, ucol, a, xbp, red, TP(dt), TP(dtdx), xl, dx, c.t, pp, TP(P.tol), max_iter,
            sizeof(TP) == 4, active, sweeps, contractions, failed);

  // ---- FV corrector ----
  const double wa = c_ops[NW].w[a < n ? a : 0];
  const double ta = c.t + dt * c_ops[NW].xi[a < n ? a : 0];
  double qd[n][M];
#pragma unroll
  for (int l = 0; l < n; ++l)
#pragma unroll
    for (int r = 0; r < M; ++r) qd[l][r] = (double)q[l][r];
  if (active) {
    double V[M];
#pragma unroll
    for (int r = 0; r < M; ++r) V[r] = 0.0;
    if constexpr (PDE::kSource || PDE::kNcp) {
#pragma unroll
      for (int k = 0; k < n; ++k) {
        double sb[M];
#pragma unroll
        for (int r = 0; r < M; ++r) sb[r] = 0.0;
        if constexpr (PDE::kSource) {
          double s[M];
          PDE::source(qd[k], xl + dx * c_ops[NW].xi[k], ta, s, pp);
#pragma unroll
          for (int r = 0; r < M; ++r) sb[r] += dt * s[r];
        }
        if constexpr (PDE::kNcp) {
          double dq[M], b[M];
#pragma unroll
          for (int r = 0; r < M; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < n; ++j) acc += c_ops[NW].ktil[k][j] * qd[j][r];
            dq[r] = acc;
          }
          PDE::ncp(qd[k], dq, b, pp);
#pragma unroll
          for (int r = 0; r < M; ++r) sb[r] -= dtdx * b[r];
        }
#pragma unroll
        for (int r = 0; r < M; ++r) V[r] += c_ops[NW].w[k] * sb[r];
      }
    }
    // block elements (0..2, a) of this lane's own column: last read by this lane
#pragma unroll
    for (int r = 0; r < M; ++r) {
      volb(pc)[a * M + r] = wa * V[r];
      double sl = 0.0, sr = 0.0;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        sl += c_ops[NW].psi0[j] * qd[j][r];
        sr += c_ops[NW].psi1[j] * qd[j][r];
      }
      trL(pc)[a * M + r] = sl;
      trR(pc)[a * M + r] = sr;
    }
  }
  __syncthreads();
  if (active && pc < PC - 1) {
    double qm[M], qp[M], Gf[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      qm[r] = trR(pc)[a * M + r];
      qp[r] = trL(pc + 1)[a * M + r];
    }
    rusanov<PDE>(qm, qp, Gf, pp);
    if constexpr (PDE::kNcp) {
      double J[M];
      PDE::jump(qm, qp, J, pp);
#pragma unroll
      for (int r = 0; r < M; ++r) jmp[(pc * n + a) * M + r] = 0.5 * wa * dtdx * J[r];
    }
#pragma unroll
    for (int r = 0; r < M; ++r) trR(pc)[a * M + r] = wa * dtdx * Gf[r];
  }
  __syncthreads();
  double lam = 0.0;
  bool bad = false;
  if (out_cell && a == 0) {
    double vnew[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      double GR = 0.0, GL = 0.0, VV = 0.0, JR = 0.0, JL = 0.0;
#pragma unroll
      for (int b = 0; b < n; ++b) {
        GR += trR(pc)[b * M + r];
        GL += trR(pc - 1)[b * M + r];
        VV += volb(pc)[b * M + r];
        if constexpr (PDE::kNcp) {
          JR += jmp[(pc * n + b) * M + r];
          JL += jmp[((pc - 1) * n + b) * M + r];
        }
      }
      vnew[r] = vb[(pc + NW) * M + r] - (GR - GL) - (JR + JL) + VV;
      c.u_out[gc * M + r] = vnew[r];
    }
    bad = !PDE::admissible(vnew, pp);
    lam = PDE::speed(vnew, pp);
  }
  report_status(A.clocks[c.pid], c.tile, bad, failed && out_cell);
  const unsigned long long sw = (out_cell && a == 0) ? (unsigned long long)sweeps : 0ull;
  const unsigned long long cw = (out_cell && a == 0) ? (unsigned long long)contractions : 0ull;
  publish<WAVES>(A.clocks[c.pid], (A.step + 1) % 3, c.tile, wave, lane, sw, cw, lam, sw_wave,
                 lam_wave);
}

// ------------------------------------------------- conserved totals ----
// dx * sum_i sum_k w_k u_i[k][r] per variable r (DG; FV: dx * sum_i v_i[r]),
// the quantity the corrector's telescoping face terms keep constant
// (Sec. 1.2).  Two passes with a fixed association order, so the result is
// bitwise reproducible: every workgroup sums a fixed range of kTotCellsPerBlock
// cells (thread i takes cells i, i + 256, ...; then a fixed LDS tree), the
// second pass sums the per-workgroup partials the same way.
constexpr int kTotThreads = 256;

__device__ __forceinline__ void tree_sum(double (&acc)[kTotMaxVars], int M, double* lds) {
  for (int r = 0; r < M; ++r) lds[r * kTotThreads + threadIdx.x] = acc[r];
  __syncthreads();
  for (int off = kTotThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int r = 0; r < M; ++r)
        lds[r * kTotThreads + threadIdx.x] += lds[r * kTotThreads + threadIdx.x + off];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kTotThreads)
totals_partial_kernel(const double* __restrict__ u, int64_t ncells, int N, int nodes, int M,
                      double* __restrict__ partials) {
  __shared__ double lds[kTotMaxVars * kTotThreads];
  double acc[kTotMaxVars] = {};
  const int64_t c0 = (int64_t)blockIdx.x * kTotCellsPerBlock;
  for (int j = threadIdx.x; j < kTotCellsPerBlock; j += kTotThreads) {
    const int64_t c = c0 + j;
    if (c >= ncells) break;
    const double* uc = u + c * nodes * M;
    for (int k = 0; k < nodes; ++k) {
      const double w = nodes > 1 ? c_ops[N].w[k] : 1.0;
      for (int r = 0; r < M; ++r) acc[r] = fma(w, uc[k * M + r], acc[r]);
    }
  }
  tree_sum(acc, M, lds);
  if (threadIdx.x == 0)
    for (int r = 0; r < M; ++r) partials[(int64_t)blockIdx.x * M + r] = lds[r * kTotThreads];
}

__global__ void __launch_bounds__(kTotThreads)
totals_final_kernel(const double* __restrict__ partials, int64_t nparts, int M, double dx,
                    double* __restrict__ out) {
  __shared__ double lds[kTotMaxVars * kTotThreads];
  double acc[kTotMaxVars] = {};
  for (int64_t b = threadIdx.x; b < nparts; b += kTotThreads)
    for (int r = 0; r < M; ++r) acc[r] += partials[b * M + r];
  tree_sum(acc, M, lds);
  if ((int)threadIdx.x < M) out[threadIdx.x] = dx * lds[threadIdx.x * kTotThreads];
}

hipError_t launch_totals(const double* u, int64_t ncells, int N, int nodes, int M, double dx,
                         double* partials, double* out, hipStream_t st) {
  if (M < 1 || M > kTotMaxVars || N < 0 || N >= kDevMaxn) return hipErrorInvalidValue;
  const int64_t nb = totals_partials(ncells);
  hipLaunchKernelGGL(totals_partial_kernel, dim3((unsigned)nb), dim3(kTotThreads), 0, st, u, ncells,
                     N, nodes, M, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(kTotThreads), 0, st, partials, nb, M, dx, out);
  return hipGetLastError();
}

// ------------------------------------------------ stream-ordered setup ----
// Problem tables and state pointers travel as kernel arguments, so a handle
// is set up and re-pointed in stream order: no host copy, no host sync, and
// nothing the caller's graph capture could not record.
__global__ void write_probs_kernel(ProbChunk c, ProbDev* dst) {
  const int i = threadIdx.x;
  if (i < c.n) dst[c.first + i] = c.d[i];
}

__global__ void write_state_ptrs_kernel(PtrChunk c, ProbDev* dst, ProbDev* dst2) {
  const int i = threadIdx.x;
  if (i < c.n) {
    dst[c.first + i].state[0] = c.p[i];
    if (dst2) dst2[c.first + i].state[0] = c.p[i];
  }
}

__global__ void zero_words_kernel(unsigned long long* p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

hipError_t launch_write_probs(const ProbDev* src, int count, ProbDev* dst, hipStream_t st) {
  for (int first = 0; first < count; first += kProbChunk) {
    ProbChunk c{};
    c.first = first;
    c.n = count - first < kProbChunk ? count - first : kProbChunk;
    for (int i = 0; i < c.n; ++i) c.d[i] = src[first + i];
    hipLaunchKernelGGL(write_probs_kernel, dim3(1), dim3(kProbChunk), 0, st, c, dst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_write_state_ptrs(double* const* ptrs, int count, ProbDev* dst, ProbDev* dst2,
                                   hipStream_t st) {
  for (int first = 0; first < count; first += kPtrChunk) {
    PtrChunk c{};
    c.first = first;
    c.n = count - first < kPtrChunk ? count - first : kPtrChunk;
    for (int i = 0; i < c.n; ++i) c.p[i] = ptrs[first + i];
    hipLaunchKernelGGL(write_state_ptrs_kernel, dim3(1), dim3(kPtrChunk), 0, st, c, dst, dst2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const int64_t words = (int64_t)(bytes / 8);
  int64_t blocks = (words + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<unsigned long long*>(p), words);
  return hipGetLastError();
}

__global__ void clock_begin_kernel(ProbClock* clocks, const double* t_user, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  ProbClock& c = clocks[p];
  c.t[0] = t_user[p];
  c.t[1] = t_user[p];
  for (int b = 0; b < 3; ++b)
    for (int i = 0; i < kSlots; ++i) c.lam[b][i].v = 0ull;
  for (int i = 0; i < kSlots; ++i) c.stat[i].v = 0;
  c.dt_last = 0.0;
  c.status = 0;
}

__global__ void clock_end_kernel(const ProbClock* clocks, double* t_user, double* dt_user,
                                 int32_t* status_user, int nprob, int parity) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  t_user[p] = clocks[p].t[parity];
  dt_user[p] = clocks[p].dt_last;
  int st = 0;
  for (int i = 0; i < kSlots; ++i) st = min(st, clocks[p].stat[i].v);
  status_user[p] = st;
}

__global__ void status_reset_kernel(ProbClock* clocks, int p) {
  if (blockIdx.x == 0 && threadIdx.x < kSlots) clocks[p].stat[threadIdx.x].v = 0;
}

__global__ void copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// -------------------------------------------------------------- dispatch ----
template <int N, class PDE, class TP, int WAVES, bool NEWTON>
static hipError_t launch_dg_t(int mode, const StepArgs& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks), block(WAVES * 64);
  switch (mode) {
    case kPredict: hipLaunchKernelGGL((dg_kernel<N, PDE, TP, WAVES, kPredict, NEWTON>), grid, block, 0, st, A); break;
    case kCorrect: hipLaunchKernelGGL((dg_kernel<N, PDE, TP, WAVES, kCorrect>), grid, block, 0, st, A); break;
    default: hipLaunchKernelGGL((dg_kernel<N, PDE, TP, WAVES, kStep, NEWTON>), grid, block, 0, st, A); break;
  }
  return hipGetLastError();
}

template <class PDE, class TP, bool NEWTON>
static hipError_t launch_dg_n(int N, int mode, const StepArgs& A, int64_t blocks, hipStream_t st) {
  switch (N) {
#define ADERDG_CASE(NN) case NN: return launch_dg_t<NN, PDE, TP, kDgWaves, NEWTON>(mode, A, blocks, st);
    ADERDG_CASE(1) ADERDG_CASE(2) ADERDG_CASE(3) ADERDG_CASE(4) ADERDG_CASE(5)
    ADERDG_CASE(6) ADERDG_CASE(7) ADERDG_CASE(8) ADERDG_CASE(9)
#undef ADERDG_CASE
    default: return hipErrorInvalidValue;
  }
}

// The fused step with kDgWavesAlt wavefronts per workgroup (the tile of a
// workgroup shrinks with it; every cell's arithmetic is the same).
template <class PDE, class TP>
static hipError_t launch_dg_alt(int N, const StepArgs& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks), block(kDgWavesAlt * 64);
  switch (N) {
#define ADERDG_CASE(NN)                                                                                  \
  case NN:                                                                                               \
    hipLaunchKernelGGL((dg_kernel<NN, PDE, TP, kDgWavesAlt, kStep, false>), grid, block, 0, st, A); \
    break;
    ADERDG_CASE(1) ADERDG_CASE(2) ADERDG_CASE(3) ADERDG_CASE(4) ADERDG_CASE(5)
    ADERDG_CASE(6) ADERDG_CASE(7) ADERDG_CASE(8) ADERDG_CASE(9)
#undef ADERDG_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class PDE, bool NEWTON = false>
static hipError_t launch_dg_p(int N, int prec, int mode, const StepArgs& A, int64_t blocks,
                              hipStream_t st, int waves) {
  if (waves == kDgWavesAlt) {
    if (NEWTON || mode != kStep) return hipErrorInvalidValue;
    return prec == 1 ? launch_dg_alt<PDE, float>(N, A, blocks, st) : launch_dg_alt<PDE, double>(N, A, blocks, st);
  }
  if (waves != kDgWaves) return hipErrorInvalidValue;
  return prec == 1 ? launch_dg_n<PDE, float, NEWTON>(N, mode, A, blocks, st)
                   : launch_dg_n<PDE, double, NEWTON>(N, mode, A, blocks, st);
}

hipError_t launch_dg(int pde, int N, int prec, int mode, const StepArgs& A, int64_t blocks,
                     hipStream_t st, bool newton, int waves) {
  if (newton) {
    // Newton inner iterations are compiled for the model with a linear source
    if (pde != 2) return hipErrorInvalidValue;
    return launch_dg_p<EulerReact, true>(N, prec, mode, A, blocks, st, waves);
  }
  switch (pde) {
    case 0: return launch_dg_p<Advection>(N, prec, mode, A, blocks, st, waves);
    case 1: return launch_dg_p<Euler>(N, prec, mode, A, blocks, st, waves);
    case 2: return launch_dg_p<EulerReact>(N, prec, mode, A, blocks, st, waves);
    case 3: return launch_dg_p<ShallowWater>(N, prec, mode, A, blocks, st, waves);
    default: return hipErrorInvalidValue;
  }
}

template <class PDE, class TP>
static hipError_t launch_fv_n(int NW, const StepArgs& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks), block(kFvWaves * 64);
  if (NW == 2) hipLaunchKernelGGL((fv_kernel<2, PDE, TP, kFvWaves>), grid, block, 0, st, A);
  else if (NW == 4) hipLaunchKernelGGL((fv_kernel<4, PDE, TP, kFvWaves>), grid, block, 0, st, A);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fv(int pde, int NW, int prec, const StepArgs& A, int64_t blocks, hipStream_t st) {
  switch (pde) {
    case 0: return prec ? launch_fv_n<Advection, float>(NW, A, blocks, st) : launch_fv_n<Advection, double>(NW, A, blocks, st);
    case 1: return prec ? launch_fv_n<Euler, float>(NW, A, blocks, st) : launch_fv_n<Euler, double>(NW, A, blocks, st);
    case 2: return prec ? launch_fv_n<EulerReact, float>(NW, A, blocks, st) : launch_fv_n<EulerReact, double>(NW, A, blocks, st);
    case 3: return prec ? launch_fv_n<ShallowWater, float>(NW, A, blocks, st) : launch_fv_n<ShallowWater, double>(NW, A, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

template <class PDE, bool DG>
static hipError_t launch_lambda_p(int N, const StepArgs& A, int64_t blocks, hipStream_t st) {
  dim3 grid((unsigned)blocks), block(256);
  switch (N) {
#define ADERDG_CASE(NN) case NN: hipLaunchKernelGGL((lambda_kernel<NN, PDE, DG>), grid, block, 0, st, A); break;
    ADERDG_CASE(1) ADERDG_CASE(2) ADERDG_CASE(3) ADERDG_CASE(4) ADERDG_CASE(5)
    ADERDG_CASE(6) ADERDG_CASE(7) ADERDG_CASE(8) ADERDG_CASE(9)
#undef ADERDG_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lambda(int pde, int N, bool dg, const StepArgs& A, int64_t blocks, hipStream_t st) {
  switch (pde) {
    case 0: return dg ? launch_lambda_p<Advection, true>(N, A, blocks, st) : launch_lambda_p<Advection, false>(N, A, blocks, st);
    case 1: return dg ? launch_lambda_p<Euler, true>(N, A, blocks, st) : launch_lambda_p<Euler, false>(N, A, blocks, st);
    case 2: return dg ? launch_lambda_p<EulerReact, true>(N, A, blocks, st) : launch_lambda_p<EulerReact, false>(N, A, blocks, st);
    case 3: return dg ? launch_lambda_p<ShallowWater, true>(N, A, blocks, st) : launch_lambda_p<ShallowWater, false>(N, A, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_clock_begin(ProbClock* clocks, const double* t_user, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(clock_begin_kernel, dim3((nprob + 63) / 64), dim3(64), 0, st, clocks, t_user, nprob);
  return hipGetLastError();
}

hipError_t launch_clock_end(const ProbClock* clocks, double* t_user, double* dt_user,
                            int32_t* status_user, int nprob, int parity, hipStream_t st) {
  hipLaunchKernelGGL(clock_end_kernel, dim3((nprob + 63) / 64), dim3(64), 0, st, clocks, t_user,
                     dt_user, status_user, nprob, parity);
  return hipGetLastError();
}

hipError_t launch_status_reset(ProbClock* clocks, int p, hipStream_t st) {
  hipLaunchKernelGGL(status_reset_kernel, dim3(1), dim3(64), 0, st, clocks, p);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t count, hipStream_t st) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

int64_t dg_tile_cells(int N, bool halo, int waves) {
  const int cpw = 64 / (N + 1);
  return (int64_t)waves * cpw - (halo ? 2 : 0);
}

int64_t fv_tile_cells(int NW) { return (int64_t)kFvWaves * (64 / (NW + 1)) - 2; }

hipError_t upload_tables(const DevOps* ops, const DevOpsF* opsf, const DevWeno* weno) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_ops), ops, sizeof(DevOps) * kDevMaxn);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_opsf), opsf, sizeof(DevOpsF) * kDevMaxn);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_weno), weno, sizeof(DevWeno) * 2);
}

}  // namespace aderdg

// Kernels of the limited 1-D step (they share this file's operator and WENO tables).
#include "limiter.hpp"
