// Device-side building blocks shared by the DG and FV kernels (gfx950).
//
//  * operator tables in constant memory, indexed with compile-time indices
//    so that every coefficient is a wave-uniform scalar load;
//  * point-wise PDE traits (flux, source, non-conservative product, signal
//    speed), evaluated in registers straight from the AoS state (Sec. 1.1:
//    fluxes, sources and non-conservative matrices are computed per node on
//    q_{p,r} without transposition);
//  * the interface solver (Rusanov + straight-path jump);
//  * wave-level LDS synchronisation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aderdg {

constexpr int kDevMaxn = 10;
constexpr int kDevMaxNs = 19;
constexpr int kWenoMaxn = 5;

struct DevOps {
  double xi[kDevMaxn];
  double w[kDevMaxn];
  double winv[kDevMaxn];
  double ktil[kDevMaxn][kDevMaxn];
  double kappa[kDevMaxn][kDevMaxn];
  double Dw[kDevMaxn][kDevMaxn];     // D~[k][l] / w_k (DG volume term at node k)
  double psi0[kDevMaxn];
  double psi1[kDevMaxn];
  double P[kDevMaxNs][kDevMaxn];
};

struct DevOpsF {
  float ktil[kDevMaxn][kDevMaxn];
  float kappa[kDevMaxn][kDevMaxn];
};

struct DevWeno {
  double R[4][kWenoMaxn][kWenoMaxn];   // up to four stencils (odd degrees >= 3)
  double S[4][kWenoMaxn][kWenoMaxn];
};

struct PdeParams {
  double gamma, g, omega, a;
};

// ---------------------------------------------------------------- sync ----
// Orders LDS traffic among the lanes of one wavefront (no s_barrier needed:
// every exchange in the predictor stays inside one wave).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double dabs(double x) { return fabs(x); }
__device__ __forceinline__ float dabs(float x) { return fabsf(x); }
__device__ __forceinline__ double dmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float dmax(float a, float b) { return fmaxf(a, b); }

// max(a, |b|) and max(|a|, |b|) as single VALU instructions.  fmax() on a
// value read from memory costs an extra instruction that quiets signalling
// NaNs; the operands here are arithmetic results or values this kernel
// wrote itself, so that step is skipped.  A NaN operand still yields the
// other operand, as fmax does.
__device__ __forceinline__ double max_abs(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, |%2|" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float max_abs(float a, float b) {
  float r;
  asm("v_max_f32_e64 %0, %1, |%2|" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double max_abs2(double a, double b) {
  double r;
  asm("v_max_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float max_abs2(float a, float b) {
  float r;
  asm("v_max_f32_e64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// 1/x by the hardware reciprocal refined with two Newton steps (relative
// error within a couple of ulps of the rounded quotient; x finite, non-zero).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// ------------------------------------------------------------ PDE traits ----
// Each model: M, kSource, kNcp, flux(q,f), speed(q), admissible(q); models
// with sources add source(q,x,t,s); with non-conservative products
// ncp(q,dq,b) = B(q).dq and jump(qm,qp,j) = B~ (qp - qm); diss(r) is the
// Rusanov dissipation mask.

struct Advection {
  static constexpr int M = 1;
  static constexpr bool kSource = false, kNcp = false;
  static constexpr int kSrcVars = 0;
  template <class T> __device__ static void flux(const T* q, T* f, const PdeParams& p) {
    f[0] = T(p.a) * q[0];
  }
  template <class T> __device__ static T speed(const T*, const PdeParams& p) { return dabs(T(p.a)); }
  __device__ static bool admissible(const double* q, const PdeParams&) { return isfinite(q[0]); }
  __device__ static constexpr double diss(int) { return 1.0; }
};

struct Euler {  // Sec. 2, eq. system_of_equations in 1-D: (rho, rho u, E)
  static constexpr int M = 3;
  static constexpr bool kSource = false, kNcp = false;
  static constexpr int kSrcVars = 0;
  template <class T> __device__ static void flux(const T* q, T* f, const PdeParams& p) {
    const T u = q[1] * recip(q[0]);
    const T pr = T(p.gamma - 1.0) * (q[2] - T(0.5) * q[1] * u);
    f[0] = q[1];
    f[1] = q[1] * u + pr;
    f[2] = u * (q[2] + pr);
  }
  template <class T> __device__ static T speed(const T* q, const PdeParams& p) {
    const T ri = recip(q[0]);
    const T u = q[1] * ri;
    const T pr = T(p.gamma - 1.0) * (q[2] - T(0.5) * q[1] * u);
    return dabs(u) + sqrt(T(p.gamma) * pr * ri);
  }
  __device__ static bool admissible(const double* q, const PdeParams& p) {
    const double u = q[1] * recip(q[0]);
    const double pr = (p.gamma - 1.0) * (q[2] - 0.5 * q[1] * u);
    return isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && q[0] > 0.0 && pr > 0.0;
  }
  __device__ static constexpr double diss(int) { return 1.0; }
};

struct EulerReact {  // Sec. 2.1, eq. pdes_2_comps in 1-D: (rho, rho u, E, rho c1, rho c2)
  static constexpr int M = 5;
  static constexpr bool kSource = true, kNcp = false;
  template <class T> __device__ static void flux(const T* q, T* f, const PdeParams& p) {
    const T u = q[1] * recip(q[0]);
    const T pr = T(p.gamma - 1.0) * (q[2] - T(0.5) * q[1] * u);
    f[0] = q[1];
    f[1] = q[1] * u + pr;
    f[2] = u * (q[2] + pr);
    f[3] = q[3] * u;
    f[4] = q[4] * u;
  }
  template <class T> __device__ static void source(const T* q, T, T, T* s, const PdeParams& p) {
    s[0] = s[1] = s[2] = T(0);
    s[3] = q[4];
    s[4] = -T(p.omega * p.omega) * q[3];
  }
  // The source is linear: its Jacobian is constant and non-zero only among
  // the variables src_var(0..kSrcVars-1) = (rho c1, rho c2).
  static constexpr int kSrcVars = 2;
  __device__ static constexpr int src_var(int k) { return 3 + k; }
  __device__ static double src_jac(int k, int k2, const PdeParams& p) {
    return k == 0 ? (k2 == 1 ? 1.0 : 0.0) : (k2 == 0 ? -p.omega * p.omega : 0.0);
  }
  template <class T> __device__ static T speed(const T* q, const PdeParams& p) {
    return Euler::speed(q, p);
  }
  __device__ static bool admissible(const double* q, const PdeParams& p) {
    return Euler::admissible(q, p) && isfinite(q[3]) && isfinite(q[4]);
  }
  __device__ static constexpr double diss(int) { return 1.0; }
};

struct ShallowWater {  // (h, hu, b); B(Q) dQ/dx = (0, g h db/dx, 0)
  static constexpr int M = 3;
  static constexpr bool kSource = false, kNcp = true;
  static constexpr int kSrcVars = 0;
  template <class T> __device__ static void flux(const T* q, T* f, const PdeParams& p) {
    const T u = q[1] * recip(q[0]);
    f[0] = q[1];
    f[1] = q[1] * u + T(0.5 * p.g) * q[0] * q[0];
    f[2] = T(0);
  }
  template <class T> __device__ static void ncp(const T* q, const T* dq, T* b, const PdeParams& p) {
    b[0] = T(0);
    b[1] = T(p.g) * q[0] * dq[2];
    b[2] = T(0);
  }
  template <class T> __device__ static void jump(const T* qm, const T* qp, T* j, const PdeParams& p) {
    j[0] = T(0);
    j[1] = T(p.g) * T(0.5) * (qm[0] + qp[0]) * (qp[2] - qm[2]);
    j[2] = T(0);
  }
  template <class T> __device__ static T speed(const T* q, const PdeParams& p) {
    return dabs(q[1] * recip(q[0])) + sqrt(T(p.g) * q[0]);
  }
  __device__ static bool admissible(const double* q, const PdeParams&) {
    return isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && q[0] > 0.0;
  }
  __device__ static constexpr double diss(int r) { return r == 2 ? 0.0 : 1.0; }
};

// Rusanov flux (unscaled): (F(qm)+F(qp))/2 - s/2 D (qp-qm), s = max signal speed.
template <class PDE>
__device__ __forceinline__ void rusanov(const double* qm, const double* qp, double* G,
                                        const PdeParams& p) {
  double fm[PDE::M], fp[PDE::M];
  PDE::flux(qm, fm, p);
  PDE::flux(qp, fp, p);
  const double s = dmax(PDE::speed(qm, p), PDE::speed(qp, p));
#pragma unroll
  for (int r = 0; r < PDE::M; ++r)
    G[r] = 0.5 * (fm[r] + fp[r]) - 0.5 * s * PDE::diss(r) * (qp[r] - qm[r]);
}

// ------------------------------------------------------- LDS layout ----
// Layout of a cell's LDS exchange block [n rows][n cols][M vars] of element
// type T: row stride RS and block stride CB (in elements) padded so that the
// lanes of a wavefront (cell c, row/column a) hit distinct LDS banks in both
// the row phase (lane a touches row a) and the column phase (lane a touches
// column a).  Bank model: 32 four-byte banks, 64-bit accesses served 16
// lanes at a time (32 lanes for 32-bit accesses); the padding minimising
// the worst bank multiplicity per lane group is found at compile time.
template <int n, int M, int ES>
struct LdsLayout {
  static constexpr int conflicts(int RS, int CB) {
    const int banks = 128 / ES;
    const int G = ES == 8 ? 16 : 32;
    const int cpw = 64 / n;
    int total = 0;
    for (int phase = 0; phase < 2; ++phase) {
      for (int g0 = 0; g0 < cpw * n; g0 += G) {
        int cnt[32] = {};
        int worst = 0;
        for (int L = g0; L < g0 + G && L < cpw * n; ++L) {
          const int c = L / n, a = L % n;
          const int off = c * CB + (phase == 0 ? a * RS : a * M);
          const int b = off % banks;
          cnt[b] += 1;
          if (cnt[b] > worst) worst = cnt[b];
        }
        total += worst;
      }
    }
    return total;
  }
  static constexpr int search(bool want_rs) {
    int best = 1 << 30, best_rs = n * M, best_cb = n * n * M;
    for (int pr = 0; pr < 4; ++pr)
      for (int pc = 0; pc < 32; ++pc) {
        const int RS = n * M + pr, CB = n * RS + pc;
        const int c = conflicts(RS, CB) * 64 + pr + pc;
        if (c < best) { best = c; best_rs = RS; best_cb = CB; }
      }
    return want_rs ? best_rs : best_cb;
  }
  static constexpr int RS = search(true);
  static constexpr int CB = search(false);
};

// ------------------------------------------------------------- problems ----
// One problem of a launch group (library-owned device array).
struct ProbDev {
  double* state[2];       // [0] caller's buffer, [1] library scratch (ping-pong)
  int64_t ncells;
  int64_t tile_begin;     // first workgroup of this problem in the group's grid
  int64_t tiles;
  double x0, dx;
  double cfl, fixed_dt, tol;
  int32_t max_iter;
  int32_t cfl_mode;
  int32_t pid;            // index into the handle's per-problem arrays
  int32_t pad;
  PdeParams pp;
};

// Per-problem device clock (library-owned).  The signal-speed maxima and the
// sweep counter are spread over kSlots counters on separate 128-byte lines:
// thousands of workgroups updating one address would serialise at the
// memory-side atomic unit.  Readers combine the slots.
constexpr int kSlots = 32;
struct alignas(128) Slot {
  unsigned long long v;
  unsigned long long pad[15];
};
struct alignas(128) StatusSlot {
  int32_t v;
  int32_t pad[31];
};
struct ProbClock {
  double t[2];                    // t^n of even / odd steps
  double dt_last;
  int32_t status;                 // unused by the step kernels (see stat)
  int32_t pad;
  unsigned long long pad2[12];
  Slot lam[3][kSlots];            // max signal speed (bit pattern of a non-negative double)
  Slot sweeps[kSlots];            // outer Picard sweeps summed over cells
  Slot contractions[kSlots];      // kappa~ applications (outer sweeps + inner iterations) summed over cells
  StatusSlot stat[kSlots];        // most severe status code seen (min)
};

// Kernel arguments (passed by value).
struct StepArgs {
  const ProbDev* probs;   // problems of the launch group (device)
  int32_t nprob;
  int32_t k;              // standalone modes: index into probs
  ProbClock* clocks;      // per-problem clocks of the handle (device)
  const double* t_end;    // caller's t_end array (device), indexed by ProbDev::pid
  int32_t step;           // step index within the current call (ping-pong / clock parity)
  int32_t pad;
  // standalone predictor / corrector
  const double* u_in;
  double* u_out;
  void* q;
  int32_t* iters;
  double t, dt;
};

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

// Order-preserving bit patterns of non-negative floating-point values, so
// that integer max on LDS words (ds_max) reduces them exactly; a NaN (all
// exponent bits set) compares above every finite value.
__device__ __forceinline__ unsigned long long ord_bits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ unsigned int ord_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ double from_bits(unsigned long long b) {
  return __longlong_as_double((long long)b);
}
__device__ __forceinline__ float from_bits(unsigned int b) { return __uint_as_float(b); }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = dmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroup -> problem of the launch group (binary search on tile_begin).
__device__ __forceinline__ int find_problem(const ProbDev* probs, int nprob, int64_t block) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_begin <= block) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace aderdg
