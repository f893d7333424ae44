// Host-visible launch interface of the limited 1-D step (limiter.hpp, compiled
// as part of kernels.hip; used by abi.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace aderdg {

// Subcell reconstruction R [n][N_s] per degree (constant memory of kernels.hip).
struct DevLimR {
  double R[kDevMaxn][kDevMaxNs];
};
// R per degree and the WENO tables of degree 1 (the ADER-WENO2 subgrid scheme)
hipError_t upload_lim_tables(const DevLimR* r, const DevWeno* weno1);

enum { kLimPeriodic = 0, kLimTransmissive = 1 };

// Device clock of a limited problem (library-owned).
struct alignas(128) LimClock {
  double t;                         // start of the current step
  double t_next;                    // its end
  double dt;                        // current step (0: the problem is at t_end)
  double dt_last;                   // last step > 0 of the call
  int32_t fallback;                 // the step's subgrid step fell back to first order
  int32_t pad0;
  unsigned long long total_troubled, total_fallback, total_steps;
  unsigned long long pad[9];
  Slot lam[2][kSlots];              // max signal speed of the state (bit patterns), by step parity
  Slot sweeps[kSlots];              // outer Picard sweeps of the candidate's predictor, summed over cells
  StatusSlot stat[kSlots];          // most severe status (min)
  StatusSlot ntr[kSlots];           // troubled cells of the current step, per sub-list
};

// Kernel arguments (passed by value).
struct LimArgs {
  int64_t C;
  int32_t N, bc;
  double x0, dx, cfl_d, tol;        // cfl_d = CFL / d
  int32_t max_iter, step;
  int32_t weno, pad1;               // WENO degree of the subgrid scheme (1 or 2)
  PdeParams pp;
  double* u;                        // [C][n][3] caller's state
  double* v;                        // [C][Ns][3] caller's subcell averages
  int32_t* troubled;                // [C] caller's mask
  const double* t_end;              // caller's t_end [1]
  LimClock* clk;
  double* vol;                      // [C][n][3] candidate volume terms
  double* trL;                      // [C+2][n time][3] left face traces of the padded cells
  double* trR;                      // [C+2][n time][3] right face traces
  double* G;                        // [C+1][3] time-integrated DG face fluxes (dt/dx units)
  double* vext;                     // [C][2][3] per-cell min / max of the subcell averages v
  int32_t* list;                    // troubled cells of the step: kSlots sub-lists of list_cap entries
  int64_t list_cap;
  double* vfv;                      // [C][Ns][3] subgrid results (troubled cells)
  double* gs;                       // [C][2][3] subgrid fluxes at a troubled cell's faces (dt/dxs units)
};

constexpr int kLimSubgridBlocks = 16384;  // workgroups (one wavefront each) of the subgrid kernels
hipError_t launch_lim_begin(LimClock* clk, const double* t_user, hipStream_t st);
hipError_t launch_lim_end(const LimClock* clk, double* t_user, double* dt_user, int32_t* status_user,
                          hipStream_t st);
hipError_t launch_lim_project(int N, const double* u, double* v, int64_t C, hipStream_t st);
hipError_t launch_lim_lambda(const LimArgs& A, int buf, hipStream_t st);
// the six kernels of one limited step
hipError_t launch_lim_step(const LimArgs& A, hipStream_t st);

}  // namespace aderdg
