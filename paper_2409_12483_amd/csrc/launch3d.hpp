// Host-visible launch interface of dg3d.hip (used by abi.cpp): 3-D ADER-DG
// for the Euler gas on a uniform periodic Cartesian mesh.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace aderdg {

// Device clock of a 3-D problem (library-owned): time of even / odd steps,
// last step size, rotating signal-speed maxima per direction, sweeps, status.
struct alignas(128) Clock3D {
  double t[2];
  double dt_last;
  int32_t pad0[2];
  unsigned long long pad1[12];
  Slot lam[3][3][kSlots];          // [direction][rotating buffer][slot]
  Slot sweeps[kSlots];
  StatusSlot stat[kSlots];
};

enum { k3dStep = 0, k3dPredict = 1 };

struct Args3D {
  int64_t c[3];            // cells per direction; cell index = (ix * cy + iy) * cz + iz
  double h[3];             // cell sizes
  double cfl, fixed_dt, tol, gamma;
  int32_t max_iter, mode, step;
  int32_t scheme;          // 0: ADER-DG; 1: ADER-WENO finite volumes (state = cell averages)
  double t, dt;            // predictor mode: given time and step
  Clock3D* clk;
  const double* t_end;     // device, one value
  double* u;               // state [cells][n][n][n][5], updated in place by the corrector
  double* part;            // scratch [cells][n][n][n][5]: u + volume terms
  void* tr;                // scratch [cells][6 faces][n time][n][n][5], predictor precision
  void* q_out;             // predictor mode: q [cells][n][n][n][n][5] in the predictor precision
  int32_t* iters;          // predictor mode: sweeps per cell (may be null)
  void* qs;                // predictor tiles Q and R per cell where they exceed LDS
                           // (pred3d_tile_bytes_per_cell > 0), else null
};

bool supported_3d(int N, int prec);
int cells_per_block_3d(int N, int prec);
// bytes of device memory per cell for the predictor's tiles when they do not
// fit in LDS (FP64 N >= 6, FP32 N >= 7); 0 otherwise
int64_t pred3d_tile_bytes_per_cell(int N, int prec);
int cells_per_block_corr3d(int N);
hipError_t launch_pred3d(int N, int prec, const Args3D& A, int64_t blocks, hipStream_t st);
hipError_t launch_corr3d(int N, int prec, const Args3D& A, int64_t blocks, hipStream_t st);
hipError_t launch_lambda3d(int N, const Args3D& A, int64_t blocks, hipStream_t st);
hipError_t launch_clock3d_begin(Clock3D* clk, const double* t_user, hipStream_t st);
hipError_t launch_clock3d_end(const Clock3D* clk, double* t_user, double* dt_user,
                              int32_t* status_user, int parity, hipStream_t st);
hipError_t upload_tables_3d(const DevOps* ops, const DevOpsF* opsf,
                            const DevWeno* weno);   // WENO of degree 1, 2, 3
// ADER-WENO finite volumes (scheme 1; NW = reconstruction degree = predictor
// degree, 1..3): nodal WENO values w [cells][n][n][n][5] of the averages
// (A.u), the update of the averages in place from the predictor's traces, the
// signal speeds of the start state.
constexpr int kFv3dThreads = 256;
hipError_t launch_weno3d(int NW, const Args3D& A, double* w, hipStream_t st);
hipError_t launch_fv3d_corr(int NW, const Args3D& A, hipStream_t st);
hipError_t launch_fv3d_lambda(const Args3D& A, hipStream_t st);

}  // namespace aderdg
