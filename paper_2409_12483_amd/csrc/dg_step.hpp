// Device templates of the fused 1-D ADER-DG step, shared by the library's
// own build (kernels.hip instantiates them for the compiled-in models) and by
// the runtime compilation of user-defined models (rtc.cpp compiles this text
// together with the user's model with hipRTC).  Nothing here is host code.
#pragma once

#include "device_common.hpp"
#include "predictor.hpp"

namespace aderdg {

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

}  // namespace aderdg
