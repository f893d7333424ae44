// Host-visible launch interface of kernels.hip (used by abi.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace aderdg {

constexpr int kDgWaves = 4;   // wavefronts per DG workgroup (default)
constexpr int kDgWavesAlt = 2;   // the other compiled size of the fused step (Picard, built-in models)
constexpr int kFvWaves = 4;   // wavefronts per FV workgroup

// waves: wavefronts per workgroup of the fused step; kDgWavesAlt is compiled
// for mode 2 (step) with Picard inner iterations, every other launch uses
// kDgWaves (hipErrorInvalidValue otherwise)
hipError_t launch_dg(int pde, int N, int prec, int mode, const StepArgs& A, int64_t blocks,
                     hipStream_t st, bool newton = false, int waves = kDgWaves);
hipError_t launch_fv(int pde, int NW, int prec, const StepArgs& A, int64_t blocks, hipStream_t st);
hipError_t launch_lambda(int pde, int N, bool dg, const StepArgs& A, int64_t blocks, hipStream_t st);
hipError_t launch_clock_begin(ProbClock* clocks, const double* t_user, int nprob, hipStream_t st);
hipError_t launch_clock_end(const ProbClock* clocks, double* t_user, double* dt_user,
                            int32_t* status_user, int nprob, int parity, hipStream_t st);
hipError_t launch_status_reset(ProbClock* clocks, int p, hipStream_t st);
// Stream-ordered table set-up (kernel arguments carry the data).
constexpr int kProbChunk = 8;
constexpr int kPtrChunk = 32;
struct ProbChunk {
  ProbDev d[kProbChunk];
  int32_t n, first;
};
struct PtrChunk {
  double* p[kPtrChunk];
  int32_t n, first;
};
hipError_t launch_write_probs(const ProbDev* src, int count, ProbDev* dst, hipStream_t st);
hipError_t launch_write_state_ptrs(double* const* ptrs, int count, ProbDev* dst, ProbDev* dst2,
                                   hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, int64_t count, hipStream_t st);
hipError_t upload_tables(const DevOps* ops, const DevOpsF* opsf, const DevWeno* weno);
// Conserved totals (two deterministic passes; partials: totals_partials(ncells) * M doubles).
constexpr int kTotMaxVars = 5;
constexpr int kTotCellsPerBlock = 4096;
inline int64_t totals_partials(int64_t ncells) {
  const int64_t nb = (ncells + kTotCellsPerBlock - 1) / kTotCellsPerBlock;
  return nb > 0 ? nb : 1;
}
hipError_t launch_totals(const double* u, int64_t ncells, int N, int nodes, int M, double dx,
                         double* partials, double* out, hipStream_t st);
int64_t dg_tile_cells(int N, bool halo, int waves = kDgWaves);
int64_t fv_tile_cells(int NW);

// Static scratch of the allocation-free step entry point (noalloc.hip):
// descriptors, one problem clock, then the ping-pong state.
constexpr size_t kNoallocBytes = size_t(64) << 20;                 // 64 MiB per device
constexpr size_t kNoallocStepDesc = 0;                             // ProbDev of the step kernel
constexpr size_t kNoallocLamDesc = 256;                            // ProbDev of the lambda kernel
constexpr size_t kNoallocClock = 1024;                             // ProbClock
constexpr size_t kNoallocState = size_t(64) << 10;                 // state copy, 8-byte elements
constexpr size_t kNoallocMaxElems = (kNoallocBytes - kNoallocState) / sizeof(double);
static_assert(sizeof(ProbDev) <= 256, "descriptor slot");
static_assert(kNoallocClock + sizeof(ProbClock) <= kNoallocState, "clock slot");
hipError_t noalloc_scratch(int device, void** out);
hipError_t launch_noalloc_setup(const ProbDev& step, const ProbDev& lam, void* base, hipStream_t st);

}  // namespace aderdg
