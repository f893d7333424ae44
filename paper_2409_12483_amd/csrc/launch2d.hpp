// Host-visible launch interface of dg2d.hip (used by abi.cpp): 2-D ADER-DG
// for the Euler gas on a uniform periodic Cartesian mesh.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace aderdg {

// Device clock of a 2-D problem (library-owned): time of even / odd steps,
// last step size, rotating signal-speed maxima per direction (bit patterns of
// non-negative doubles spread over kSlots lines), Picard sweeps and status.
struct alignas(128) Clock2D {
  double t[2];
  double dt_last;
  int32_t pad0[2];
  unsigned long long pad1[12];
  Slot lamx[3][kSlots];
  Slot lamy[3][kSlots];
  Slot sweeps[kSlots];
  StatusSlot stat[kSlots];
};

enum { k2dStep = 0, k2dPredict = 1 };

// Kernel arguments (passed by value).
struct Args2D {
  int64_t cx, cy;          // cells along x and y; cell index = ix * cy + iy
  double dx, dy;
  double cfl, fixed_dt, tol;
  double gamma;
  int32_t max_iter;
  int32_t mode;            // k2dStep or k2dPredict
  int32_t step;            // step index within the call (clock parity / lambda buffer)
  int32_t scheme;          // 0: ADER-DG; 1: ADER-WENO finite volumes (state = cell averages)
  double t, dt;            // predictor mode: given time and step
  Clock2D* clk;
  const double* t_end;     // device, one value
  double* u;               // state [cells][n][n][4] (the corrector updates it in place)
  double* part;            // scratch [cells][n][n][4]: u + volume terms
  void* tr;                // scratch [cells][4 faces][n time][n face nodes][4]: face traces, in the
                           // predictor precision (FP64, or FP32 in the FP32-predictor mode)
  void* q_out;             // predictor mode: q [cells][n][n][n][4] in the predictor precision
  int32_t* iters;          // predictor mode: sweeps per cell (may be null)
  double* gface;           // candidate mode: the corrector's time-integrated fluxes through the east
                           // and north face of every cell [cells][2][n][4] (null: not stored)
  int32_t candidate;       // 1: the corrector neither publishes signal speeds nor reports a
                           // non-physical state (the limited step decides on both)
  int32_t pad_c;
};

int cells_per_block_2d(int N, int prec);
int threads_per_block_2d(int N, int prec);
hipError_t launch_pred2d(int N, int prec, const Args2D& A, int64_t blocks, hipStream_t st);
hipError_t launch_corr2d(int N, int prec, const Args2D& A, int64_t blocks, hipStream_t st);
hipError_t launch_lambda2d(int N, const Args2D& A, int64_t blocks, hipStream_t st);
int cells_per_block_corr2d(int N);
hipError_t launch_clock2d_begin(Clock2D* clk, const double* t_user, hipStream_t st);
hipError_t launch_clock2d_end(const Clock2D* clk, double* t_user, double* dt_user,
                              int32_t* status_user, int parity, hipStream_t st);
hipError_t upload_tables_2d(const DevOps* ops, const DevOpsF* opsf,
                            const DevWeno* weno);   // WENO of degree 1, 2, 3
// ADER-WENO finite volumes (scheme 1; NW = reconstruction degree = predictor degree, 1..3):
// nodal WENO values w [cells][n][n][4] of the averages v (A.u), the update of
// the averages in place from the predictor's traces, the signal speed of the
// start state (kFv2dThreads per workgroup).
constexpr int kFv2dThreads = 256;
hipError_t launch_weno2d(int NW, const Args2D& A, double* w, hipStream_t st);
hipError_t launch_fv2d_corr(int NW, const Args2D& A, hipStream_t st);
hipError_t launch_fv2d_lambda(const Args2D& A, hipStream_t st);

// ---- limited 2-D step (a posteriori subcell ADER-WENO2 limiting; the kernels
// live in limiter2d.hpp, compiled as part of dg2d.hip) ----
enum { kLim2Periodic = 0, kLim2Transmissive = 1 };
struct Lim2Args {
  Args2D dg;               // the DG step on the padded mesh (cx + 2) x (cy + 2): clock, step, dt
  int64_t cx, cy;          // interior cells
  int32_t N, bc;
  double* up;              // padded state [(cx+2)(cy+2)][n][n][4] (ghost ring around the interior)
  double* u;               // caller's state [cx][cy][n][n][4] (copied in and out once per call)
  double* v;               // caller's subcell averages [cx][cy][Ns][Ns][4] (v^n in, v^{n+1} out)
  int32_t* troubled;       // caller's mask [cx][cy]
  double* vfv;             // [cx][cy][Ns][Ns][4] subgrid results of troubled cells
  double* sflux;           // [cx][cy][4 faces W,E,S,N][Ns][4] subgrid fluxes through a troubled cell's faces
  unsigned long long* cnt; // [0] troubled cells summed over steps, [1] first-order redo steps, [2] redo flag
  double* uout;            // [cx][cy][n][n][4] corrected state of the current pass
  double* vout;            // [cx][cy][Ns][Ns][4] its subcell averages
  int32_t pass, npass;     // detection / correction pass of the step (troubled = pass of detection)
};
hipError_t upload_lim2d_tables(const void* limR);     // DevLimR[kDevMaxn]
hipError_t launch_lim2d_copy(const Lim2Args& L, int to_padded, hipStream_t st);
hipError_t launch_lim2d_ghosts(const Lim2Args& L, hipStream_t st);
hipError_t launch_lim2d_project(const Lim2Args& L, hipStream_t st);
// the limiter kernels of one step after the candidate (detect, subgrid, first-order redo, finish)
hipError_t launch_lim2d_after_candidate(const Lim2Args& L, hipStream_t st);

}  // namespace aderdg
