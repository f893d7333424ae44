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

namespace aderdg {

__constant__ DevOps c_ops[kDevMaxn];
__constant__ DevOpsF c_opsf[kDevMaxn];
__constant__ DevWeno c_weno[2];  // WENO degree 2 and 4

enum Mode { kPredict = 0, kCorrect = 1, kStep = 2 };

#ifndef ADERDG_FP32_MFMA
#define ADERDG_FP32_MFMA 0
#endif
constexpr bool kFp32Mfma = ADERDG_FP32_MFMA;

// Geometry of a workgroup for degree N and M variables.  Each cell owns an
// LDS exchange block: rows of RSD doubles, CBD doubles per block (padded
// against bank conflicts); in FP32-predictor mode the predictor addresses
// the same block as floats with its own padded strides.
template <int N, int M, int WAVES, bool HALO>
struct Geo {
  static constexpr int n = N + 1;
  static constexpr int CPW = 64 / n;                 // cells per wavefront
  static constexpr int PC = WAVES * CPW;             // predictor cells per workgroup
  static constexpr int TILE = HALO ? PC - 2 : PC;    // cells written per workgroup
  static constexpr int RSD = LdsLayout<n, M, 8>::RS;
  static constexpr int CBD = LdsLayout<n, M, 8>::CB;
  static constexpr int CBF = LdsLayout<n, M, 4>::CB;
  static_assert(CBF <= 2 * CBD, "float block must fit the double block");
  static constexpr int XB = CPW * CBD;               // doubles of LDS exchange per wave
  static constexpr int RED = (CPW + 1) * 2;          // per wave: 2 reduction words per cell + idle lanes' pair
};

// Predictor view (element type TP) of a cell's exchange block.
template <class G, class TP>
__device__ __forceinline__ TP* pred_block(double* xb_all, int wave, int slot) {
  constexpr int CB = sizeof(TP) == 8 ? G::CBD : G::CBF;
  return reinterpret_cast<TP*>(xb_all + wave * G::XB) + slot * CB;
}


// Problem-level step parameters for a workgroup.
struct StepCtx {
  int pid;
  double t, dt;
  const double* u_in;
  double* u_out;
  int64_t tile;
};

// Max of a problem's signal-speed slots, read by wave 0 and broadcast through LDS.
__device__ __forceinline__ double read_lambda(const ProbClock& clk, int buf, double* bcast) {
  if (threadIdx.x < 64) {
    double v = 0.0;
    if (threadIdx.x < kSlots) v = __longlong_as_double((long long)clk.lam[buf][threadIdx.x].v);
    v = wave_max(v);
    if (threadIdx.x == 0) *bcast = v;
  }
  __syncthreads();
  return *bcast;
}

// Resolve the problem, time and step size of this workgroup (step mode).
template <bool DG, int N>
__device__ __forceinline__ bool step_setup(const StepArgs& A, const ProbDev& P, StepCtx& c,
                                           double* bcast) {
  ProbClock& clk = A.clocks[P.pid];
  const int s = A.step;
  c.pid = P.pid;
  c.t = clk.t[s & 1];
  double dt;
  if (P.fixed_dt > 0.0) {
    dt = P.fixed_dt;
  } else {
    const double lam = read_lambda(clk, s % 3, bcast);
    dt = DG ? P.cfl * P.dx / ((2.0 * N + 1.0) * lam) : P.cfl * P.dx / lam;
  }
  const double rem = A.t_end[P.pid] - c.t;
  if (dt > rem) dt = rem;
  if (!(dt > 0.0)) dt = 0.0;
  c.dt = dt;
  c.u_in = P.state[s & 1];
  c.u_out = P.state[(s + 1) & 1];
  if (c.tile == 0) {
    if (threadIdx.x == 0) {
      clk.t[(s + 1) & 1] = c.t + dt;
      if (dt > 0.0) clk.dt_last = dt;
    }
    if (threadIdx.x < kSlots) {
      clk.lam[(s + 2) % 3][threadIdx.x].v = 0ull;
      if (dt == 0.0)   // state unchanged: carry lambda
        clk.lam[(s + 1) % 3][threadIdx.x].v = clk.lam[s % 3][threadIdx.x].v;
    }
  }
  return dt > 0.0;
}

// Workgroup-level epilogue: sum of sweeps and max of signal speed over the
// waves (per-wave partials in LDS), one atomic each into slot (tile % kSlots).
template <int WAVES>
__device__ __forceinline__ void publish(ProbClock& clk, int buf, int64_t tile, int wave, int lane,
                                        unsigned long long sw, unsigned long long cw, double lam,
                                        unsigned long long* sw_wave, double* lam_wave) {
  // the two counters travel as one 64-bit sum (each stays far below 2^32 per wave)
  const unsigned long long both = wave_sum(sw | (cw << 32));
  lam = wave_max(lam);
  if (lane == 0) {
    sw_wave[wave] = both;
    lam_wave[wave] = lam;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long S = 0, K = 0;
    double L = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      S += sw_wave[w] & 0xffffffffull;
      K += sw_wave[w] >> 32;
      L = dmax(L, lam_wave[w]);
    }
    const int slot = (int)(tile % kSlots);
    if (S) atomicAdd(&clk.sweeps[slot].v, S);
    if (K) atomicAdd(&clk.contractions[slot].v, K);
    atomic_max_nonneg(&clk.lam[buf][slot].v, L);
  }
}

// Most severe status of the wavefront (non-physical state over Picard
// non-convergence), at most one atomic per wave, into one of kSlots status
// slots so that a failing problem does not serialise its workgroups on one
// address.  Call from all lanes.
__device__ __forceinline__ void report_status(ProbClock& clk, int64_t tile, bool bad, bool failed) {
  const bool any_bad = __any(bad), any_fail = __any(failed);
  if ((threadIdx.x & 63) == 0 && (any_bad || any_fail)) {
    const int slot = (int)((tile * 17 + (threadIdx.x >> 6)) % kSlots);
    atomicMin(&clk.stat[slot].v, any_bad ? -5 : -4);
  }
}

// Copy a tile unchanged (problem already at t_end).
__device__ __forceinline__ void copy_tile(const double* in, double* out, int64_t first,
                                          int64_t count, int per_cell) {
  const int64_t total = count * per_cell, base = first * per_cell;
  for (int64_t i = threadIdx.x; i < total; i += blockDim.x) out[base + i] = in[base + i];
}

// ------------------------------------------------------------------ DG ----
// Requested waves per SIMD: 4 for conservation laws up to N = 5, whose
// working sets fit 128 VGPRs without spilling; other variants (larger N, or
// an inner loop for source / non-conservative terms) take what their
// registers allow rather than spill.
template <int N, class PDE>
struct DgOccupancy {
  static constexpr int value = (PDE::kSource || PDE::kNcp || N > 5) ? 1 : 4;
};

template <int N, class PDE, class TP, int WAVES, int MODE, bool NEWTON = false>
__global__ void __launch_bounds__(WAVES * 64)
__attribute__((amdgpu_waves_per_eu(DgOccupancy<N, PDE>::value)))
dg_kernel(StepArgs A) {
  constexpr bool HALO = MODE != kPredict;
  using G = Geo<N, PDE::M, WAVES, HALO>;
  constexpr int n = G::n, M = PDE::M, CPW = G::CPW, PC = G::PC;
  using Pred = Predictor<N, PDE, TP, sizeof(TP) == 4 && kFp32Mfma, NEWTON>;
  // inverse Jacobian of the Newton inner iterations (augmented rows)
  __shared__ double jinv[NEWTON ? NewtonDims<N, PDE>::kSize : 1];

  __shared__ double xb_all[WAVES * G::XB];
  __shared__ TP red_all[WAVES * G::RED];
  __shared__ double jmp[PDE::kNcp ? PC * n * M : 1];
  __shared__ double lam_wave[WAVES];
  __shared__ unsigned long long sw_wave[WAVES];
  __shared__ double bcast;
  // After the predictor, the first 2nM doubles of every cell's exchange block
  // hold its face traces: left [a][r], then right [a][r] (the right ones are
  // overwritten by the weighted face flux of the face on the cell's right).
  auto trL = [&](int cell) { return xb_all + (cell / CPW) * G::XB + (cell % CPW) * G::CBD; };
  auto trR = [&](int cell) { return trL(cell) + G::RSD; };
  constexpr int RSD = G::RSD;

  const int pidx = MODE == kStep ? find_problem(A.probs, A.nprob, blockIdx.x) : A.k;
  const ProbDev& P = A.probs[pidx];
  StepCtx c;
  c.tile = (int64_t)blockIdx.x - (MODE == kStep ? P.tile_begin : 0);
  const int64_t C = P.ncells;
  const int64_t first = c.tile * G::TILE;
  if (first >= C) return;
  const int64_t count = (C - first < G::TILE) ? C - first : G::TILE;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot0 = lane / n;
  const bool active = slot0 < CPW;
  const int slot = active ? slot0 : 0;                  // idle lanes read (never write) slot 0
  const int a = active ? lane % n : lane - CPW * n;
  const int pc = wave * CPW + slot;                      // predictor cell in the workgroup
  int64_t gc = first + pc - (HALO ? 1 : 0);              // global cell (periodic wrap)
  if (gc < 0) gc += C;
  if (gc >= C) {
    gc -= C;
    if (gc >= C) gc %= C;                                // meshes smaller than a tile
  }
  const bool out_cell = active && (HALO ? (pc >= 1 && pc <= PC - 2) : true) &&
                        (first + pc - (HALO ? 1 : 0)) < C;

  if constexpr (MODE == kStep) {
    if (!step_setup<true, N>(A, P, c, &bcast)) {
      copy_tile(c.u_in, c.u_out, first, count, n * M);
      return;
    }
  } else {
    c.pid = P.pid;
    c.t = A.t;
    c.dt = A.dt;
    c.u_in = A.u_in;
    c.u_out = A.u_out;
  }
  const double* ucell = c.u_in + gc * (n * M);   // the cell's state [n][M]

  double* xb = xb_all + wave * G::XB + slot * G::CBD;
  TP* xbp = pred_block<G, TP>(xb_all, wave, slot);
  TP* red = red_all + wave * G::RED + (active ? slot : CPW) * 2;   // idle lanes: a pair of their own

  // problem parameters in registers (the wave fences below would otherwise
  // force them to be re-read from memory)
  const PdeParams pp = P.pp;
  const int max_iter = P.max_iter, cfl_mode = P.cfl_mode;
  const double dx = P.dx, dt = c.dt, dtdx = dt / dx;
  const double xl = P.x0 + dx * (double)gc;

  // ---- predictor (or load of a given predictor) ----
  TP q[n][M];
  int sweeps = 0, contractions = 0;
  bool failed = false;
  if constexpr (MODE == kCorrect) {
    const TP* qin = reinterpret_cast<const TP*>(A.q) + gc * (n * n * M) + a * (n * M);
#pragma unroll
    for (int l = 0; l < n; ++l)
#pragma unroll
      for (int r = 0; r < M; ++r) q[l][r] = qin[l * M + r];
  } else {
    TP ucol[M];
#pragma unroll
    for (int l = 0; l < n; ++l)
#pragma unroll
      for (int r = 0; r < M; ++r) q[l][r] = TP(ucell[l * M + r]);
#pragma unroll
    for (int r = 0; r < M; ++r) ucol[r] = TP(ucell[a * M + r]);
    const TP tol = TP(P.tol);
    if constexpr (NEWTON) {
      newton_prepare<N, PDE>(jinv, dt, pp);
      __syncthreads();
    }
    Pred::run(q, ucol, a, xbp, red, TP(dt), TP(dtdx), xl, dx, c.t, pp, tol, max_iter,
              sizeof(TP) == 4, active, sweeps, contractions, failed, jinv);
  }

  if constexpr (MODE == kPredict) {
    if (out_cell) {
      TP* qo = reinterpret_cast<TP*>(A.q) + gc * (n * n * M) + a * (n * M);
#pragma unroll
      for (int l = 0; l < n; ++l)
#pragma unroll
        for (int r = 0; r < M; ++r) qo[l * M + r] = q[l][r];
      if (A.iters && a == 0) A.iters[gc] = sweeps;
    }
    report_status(A.clocks[c.pid], c.tile, false, failed && out_cell);
    return;
  } else {
    // ---- corrector: volume terms of time row a ----
    const double wa = c_ops[N].w[a];
    const double ta = c.t + dt * c_ops[N].xi[a];
    double qd[n][M];
#pragma unroll
    for (int l = 0; l < n; ++l)
#pragma unroll
      for (int r = 0; r < M; ++r) qd[l][r] = (double)q[l][r];
    double fd[n][M];
#pragma unroll
    for (int l = 0; l < n; ++l) PDE::flux(qd[l], fd[l], pp);
    wave_sync();
    // row a's share of the volume term at node k: w_a (dt/dx) (D~ F)_k / w_k
    // (+ w_a dt S - w_a (dt/dx) B(q) k~q)
    const double wdx = wa * dtdx;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      double V[M];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double acc = c_ops[N].Dw[k][0] * fd[0][r];
#pragma unroll
        for (int l = 1; l < n; ++l) acc += c_ops[N].Dw[k][l] * fd[l][r];
        V[r] = wdx * acc;
      }
      if constexpr (PDE::kSource) {
        double s[M];
        PDE::source(qd[k], xl + dx * c_ops[N].xi[k], ta, s, pp);
#pragma unroll
        for (int r = 0; r < M; ++r) V[r] += (wa * dt) * s[r];
      }
      if constexpr (PDE::kNcp) {
        double dq[M], b[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < n; ++j) acc += c_ops[N].ktil[k][j] * qd[j][r];
          dq[r] = acc;
        }
        PDE::ncp(qd[k], dq, b, pp);
#pragma unroll
        for (int r = 0; r < M; ++r) V[r] -= wdx * b[r];
      }
      if (active) {
#pragma unroll
        for (int r = 0; r < M; ++r) xb[a * RSD + k * M + r] = V[r];
      }
    }
    // face traces of time row a
    double sl[M], sr[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      sl[r] = 0.0;
      sr[r] = 0.0;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        sl[r] += c_ops[N].psi0[j] * qd[j][r];
        sr[r] += c_ops[N].psi1[j] * qd[j][r];
      }
    }
    wave_sync();
    // column role: lane a = space node k, volume increment summed over time rows
    double vol[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < n; ++b) acc += xb[b * RSD + a * M + r];
      vol[r] = acc;
    }
    // traces into the block elements (0, a) and (1, a), which this lane just read
    if (active) {
#pragma unroll
      for (int r = 0; r < M; ++r) {
        trL(pc)[a * M + r] = sl[r];
        trR(pc)[a * M + r] = sr[r];
      }
    }
    __syncthreads();
    // Riemann solver at face pc+1/2 and time node a (left cell's lane), weighted by w_a dt/dx
    if (active && pc < PC - 1) {
      double qm[M], qp[M], G[M];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        qm[r] = trR(pc)[a * M + r];
        qp[r] = trL(pc + 1)[a * M + r];
      }
      rusanov<PDE>(qm, qp, G, pp);
      if constexpr (PDE::kNcp) {
        double J[M];
        PDE::jump(qm, qp, J, pp);
#pragma unroll
        for (int r = 0; r < M; ++r) jmp[(pc * n + a) * M + r] = 0.5 * wa * dtdx * J[r];
      }
#pragma unroll
      for (int r = 0; r < M; ++r) trR(pc)[a * M + r] = wa * dtdx * G[r];
    }
    __syncthreads();
    // surface terms and store (column role, lane a = node k)
    double unew[M];
    bool bad = false;
    if (out_cell) {
      const int k = a;
      const double winv = c_ops[N].winv[k], p0 = c_ops[N].psi0[k], p1 = c_ops[N].psi1[k];
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double GR = 0.0, GL = 0.0;
#pragma unroll
        for (int b = 0; b < n; ++b) {
          GR += trR(pc)[b * M + r];
          GL += trR(pc - 1)[b * M + r];
        }
        double v = ucell[k * M + r] + vol[r] - winv * (p1 * GR - p0 * GL);
        if constexpr (PDE::kNcp) {
          double JR = 0.0, JL = 0.0;
#pragma unroll
          for (int b = 0; b < n; ++b) {
            JR += jmp[(pc * n + b) * M + r];
            JL += jmp[((pc - 1) * n + b) * M + r];
          }
          v -= winv * (p1 * JR + p0 * JL);
        }
        unew[r] = v;
        c.u_out[gc * (n * M) + k * M + r] = v;
      }
      bad = !PDE::admissible(unew, pp);
    }
    // ---- epilogue: status, sweep count, signal speed of u^{n+1} ----
    if constexpr (MODE == kStep) {
      report_status(A.clocks[c.pid], c.tile, bad, failed && out_cell);
      const unsigned long long sw = (out_cell && a == 0) ? (unsigned long long)sweeps : 0ull;
      const unsigned long long cw = (out_cell && a == 0) ? (unsigned long long)contractions : 0ull;
      double lam = 0.0;
      if (cfl_mode == 1) {
        if (out_cell) lam = PDE::speed(unew, pp);
      } else {
        wave_sync();
        if (out_cell) {
#pragma unroll
          for (int r = 0; r < M; ++r) xb[a * M + r] = unew[r];
        }
        wave_sync();
        if (out_cell) {
          constexpr int Ns = 2 * N + 1;
#pragma unroll
          for (int s0 = 0; s0 < Ns; s0 += n) {
            const int s = s0 + a;
            if (s < Ns) {
              double v[M];
#pragma unroll
              for (int r = 0; r < M; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < n; ++k) acc += c_ops[N].P[s][k] * xb[k * M + r];
                v[r] = acc;
              }
              lam = dmax(lam, PDE::speed(v, pp));
            }
          }
        }
      }
      publish<WAVES>(A.clocks[c.pid], (A.step + 1) % 3, c.tile, wave, lane, sw, cw, lam, sw_wave,
                     lam_wave);
    } else {
      report_status(A.clocks[c.pid], c.tile, bad, false);
    }
  }
}

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

// ------------------------------------------------------- lambda / clock ----
// Max signal speed of the current state of every problem of a group (one
// thread per cell): DG on the 2N+1 subcell averages (or nodal values), FV on
// the cell averages.
template <int N, class PDE, bool DG>
__global__ void __launch_bounds__(256)
lambda_kernel(StepArgs A) {
  constexpr int n = N + 1, M = PDE::M;
  const int pidx = find_problem(A.probs, A.nprob, blockIdx.x);
  const ProbDev& P = A.probs[pidx];
  const int64_t cell = ((int64_t)blockIdx.x - P.tile_begin) * 256 + threadIdx.x;
  double lam = 0.0;
  if (cell < P.ncells) {
    const double* u = P.state[0];
    if (!DG) {
      double v[M];
#pragma unroll
      for (int r = 0; r < M; ++r) v[r] = u[cell * M + r];
      lam = PDE::speed(v, P.pp);
    } else if (P.cfl_mode == 1) {
#pragma unroll
      for (int k = 0; k < n; ++k) {
        double v[M];
#pragma unroll
        for (int r = 0; r < M; ++r) v[r] = u[cell * n * M + k * M + r];
        lam = dmax(lam, PDE::speed(v, P.pp));
      }
    } else {
      double uc[n][M];
#pragma unroll
      for (int k = 0; k < n; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) uc[k][r] = u[cell * n * M + k * M + r];
#pragma unroll
      for (int s = 0; s < 2 * N + 1; ++s) {
        double v[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < n; ++k) acc += c_ops[N].P[s][k] * uc[k][r];
          v[r] = acc;
        }
        lam = dmax(lam, PDE::speed(v, P.pp));
      }
    }
  }
  __shared__ double part[4];
  lam = wave_max(lam);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = lam;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = dmax(dmax(part[0], part[1]), dmax(part[2], part[3]));
    const int64_t blk = (int64_t)blockIdx.x - P.tile_begin;
    atomic_max_nonneg(&A.clocks[P.pid].lam[0][blk % kSlots].v, m);
  }
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

template <class PDE, bool NEWTON = false>
static hipError_t launch_dg_p(int N, int prec, int mode, const StepArgs& A, int64_t blocks,
                              hipStream_t st) {
  return prec == 1 ? launch_dg_n<PDE, float, NEWTON>(N, mode, A, blocks, st)
                   : launch_dg_n<PDE, double, NEWTON>(N, mode, A, blocks, st);
}

hipError_t launch_dg(int pde, int N, int prec, int mode, const StepArgs& A, int64_t blocks,
                     hipStream_t st, bool newton) {
  if (newton) {
    // Newton inner iterations are compiled for the model with a linear source
    if (pde != 2) return hipErrorInvalidValue;
    return launch_dg_p<EulerReact, true>(N, prec, mode, A, blocks, st);
  }
  switch (pde) {
    case 0: return launch_dg_p<Advection>(N, prec, mode, A, blocks, st);
    case 1: return launch_dg_p<Euler>(N, prec, mode, A, blocks, st);
    case 2: return launch_dg_p<EulerReact>(N, prec, mode, A, blocks, st);
    case 3: return launch_dg_p<ShallowWater>(N, prec, mode, A, blocks, st);
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

int64_t dg_tile_cells(int N, bool halo) {
  const int cpw = 64 / (N + 1);
  return (int64_t)kDgWaves * cpw - (halo ? 2 : 0);
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
