// Host interface of the runtime compilation of user-defined models (rtc.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "device_common.hpp"

namespace aderdg {

constexpr int kRtcWaves = 4;   // wavefronts per workgroup of the runtime-compiled step

// The loaded module of one (model source, N, precision): the step kernel in
// its three modes (predict, correct, fused step) and the signal-speed kernel.
struct RtcModule {
  hipModule_t mod;
  hipFunction_t dg[3];
  hipFunction_t lambda;
};

// Compile only (no device needed): 0 on success; the compiler log in *log.
int rtc_compile_check(const std::string& model, int nvars, int N, int prec, std::string* log);
// Compile (once per model, N, precision and device) and load; tables from the host copies.
int rtc_module(const std::string& model, int nvars, int N, int prec, int device, const DevOps* ops,
               const DevOpsF* opsf, const RtcModule** out, std::string* log);
hipError_t rtc_launch(hipFunction_t fn, const StepArgs& A, int64_t blocks, int threads, hipStream_t st);

}  // namespace aderdg
