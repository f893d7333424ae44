// Host-visible launch interface of kernels.hip (used by abi.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace aderdg {

constexpr int kDgWaves = 4;   // wavefronts per DG workgroup
constexpr int kFvWaves = 4;   // wavefronts per FV workgroup

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

hipError_t launch_dg(int pde, int N, int prec, int mode, const StepArgs& A, int64_t blocks,
                     hipStream_t st);
hipError_t launch_fv(int pde, int NW, int prec, const StepArgs& A, int64_t blocks, hipStream_t st);
hipError_t launch_lambda(int pde, int N, bool dg, const StepArgs& A, int64_t blocks, hipStream_t st);
hipError_t launch_clock_begin(ProbClock* clocks, const double* t_user, int nprob, hipStream_t st);
hipError_t launch_clock_end(const ProbClock* clocks, double* t_user, double* dt_user,
                            int32_t* status_user, int nprob, int parity, hipStream_t st);
hipError_t launch_status_reset(ProbClock* clocks, int p, hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, int64_t count, hipStream_t st);
hipError_t upload_tables(const DevOps* ops, const DevOpsF* opsf, const DevWeno* weno);
int64_t dg_tile_cells(int N, bool halo);
int64_t fv_tile_cells(int NW);

}  // namespace aderdg
