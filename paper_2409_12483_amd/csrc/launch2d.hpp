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

}  // namespace aderdg
