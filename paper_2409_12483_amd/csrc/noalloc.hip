// Library-resident scratch for the allocation-free step entry point
// (aderdg_step_noalloc in include/aderdg.h).
//
// The fused step needs device memory beyond the caller's buffers: the
// ping-pong partner of the state (a step reads neighbour cells of u^n while
// other workgroups write u^{n+1}), the per-problem clock with its rotating
// signal-speed slots, and the problem descriptors the kernels read.  The
// handle-based entry points allocate these in aderdg_init; this file holds
// them in one static device array instead, so that a caller that may not
// allocate (code under stream capture, tight serving loops) can still step.
//
// The array's name is only a host-side stand-in for the device symbol: host
// code never passes it to a kernel or a copy.  The device address is looked
// up once per device with hipGetSymbolAddress (with that device current)
// and kept per device; every later use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_common.hpp"
#include "launch.hpp"

namespace aderdg {

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

// Writes the two problem descriptors (step kernel, lambda kernel) into the
// scratch area.  Descriptors travel as kernel arguments, so nothing is copied
// from host memory and the call sequence stays capturable.
__global__ void noalloc_setup_kernel(ProbDev step, ProbDev lam, unsigned char* base) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *reinterpret_cast<ProbDev*>(base + kNoallocStepDesc) = step;
    *reinterpret_cast<ProbDev*>(base + kNoallocLamDesc) = lam;
  }
}

}  // namespace

// Device address of the scratch array on `device` (looked up on first use,
// with the device current).  Returns hipSuccess or the lookup's error.
hipError_t noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) {
      e = hipSetDevice(device);
      if (e != hipSuccess) return e;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

hipError_t launch_noalloc_setup(const ProbDev& step, const ProbDev& lam, void* base, hipStream_t st) {
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(64), 0, st, step, lam,
                     static_cast<unsigned char*>(base));
  return hipGetLastError();
}

}  // namespace aderdg
