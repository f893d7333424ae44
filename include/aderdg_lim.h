/*
 * aderdg_lim.h -- C ABI of the 1-D ADER-DG step with a posteriori subcell
 * ADER-WENO finite-volume limiting, for the Euler gas (MI355X, gfx950).
 *
 * Method: I.S. Popov, "The effective use of BLAS interface for implementation
 * of finite-element ADER-DG and finite-volume ADER-WENO methods",
 * arXiv 2409.12483: the ADER-DG step (Sec. 1.1, 1.2) gives a candidate; the
 * candidate is checked in the subcell representation v = P u of N_s = 2N+1
 * subcells (Sec. 1.4) by the physical and numerical admissibility detectors
 * (Sec. 1.6); every troubled cell is recomputed by the ADER-WENO2
 * finite-volume scheme (Sec. 1.3; WENO of degree 1 in the paper's
 * ADER-WENO(N+1) naming) on its subgrid and returns to the DG
 * representation by u = R v, R the least-squares inverse of P (Sec. 1.4).
 * The PDE is Sec. 2, eq. system_of_equations in 1-D: U = (rho, rho u, E).
 *
 * Readings where the paper is silent (the test oracle takes the same ones):
 *   - a limited cell keeps its subcell averages v between steps; the
 *     detectors and the next subgrid step start from them (never from P R v);
 *   - faces between a limited and an unlimited cell carry one flux, the
 *     subgrid scheme's: the unlimited cell's update takes it in place of its
 *     DG flux;
 *   - if the ADER-WENO subgrid step leaves the admissible set in any troubled
 *     cell, the subgrid step of that time step is redone at first order
 *     (Rusanov finite volumes), for every troubled cell;
 *   - a limited cell's u = m + theta (R v - m), m the mean of v, theta the
 *     largest of 1, 1/2, ..., 2^-12 (else 0) for which u and P u are
 *     admissible; the mean is kept.
 *   - NAD: V_i = the cell and its two face neighbours (at a free-outflow end,
 *     the one neighbour), delta = max(1e-4, 1e-3 (max - min)) per variable.
 *
 * Conventions (as in aderdg.h): int32 status, 0 = ADERDG_OK, negative =
 * error (codes of aderdg.h); on ADERDG_E_INVAL nothing was enqueued and
 * aderdg_last_error() explains.  "device" pointers are HIP device
 * allocations owned by the caller, contiguous and 8-byte aligned.  Work is
 * enqueued on the handle's stream without host synchronisation (except in
 * init, free and the counter read).  One host thread per handle at a time.
 *
 * Layouts (array-of-structures, variable index fastest):
 *   u         [ncells][N+1 (node)][3]        fp64 nodal DG state
 *   v         [ncells][2N+1 (subcell)][3]    fp64 subcell averages
 *   troubled  [ncells]                       int32, 1 = limited in the last step
 * Cell i spans [x0 + i dx, x0 + (i+1) dx]; nodes are the Gauss-Legendre
 * points of [0, 1]; subcell j of a cell spans [j/(2N+1), (j+1)/(2N+1)].
 */
#ifndef ADERDG_LIM_H
#define ADERDG_LIM_H

#include <stdint.h>

#include "aderdg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary conditions of a limited problem. */
enum aderdg_lim_bc {
  ADERDG_LIM_PERIODIC = 0,
  /* free outflow (Sec. 2.2): a ghost cell is the mirror image of the boundary
   * cell (nodal values in reversed order, no sign change); subgrid ghosts
   * mirror the boundary subcells the same way */
  ADERDG_LIM_TRANSMISSIVE = 1
};

typedef struct {
  int32_t N;               /* DG degree, 1..9 */
  int32_t bc;              /* enum aderdg_lim_bc */
  int64_t ncells;          /* >= 3 */
  double x0, x1;           /* domain, x1 > x0 */
  double gamma;            /* ratio of specific heats, > 1 */
  double cfl;              /* 0 < cfl <= 1 */
  int32_t dims;            /* d of the CFL rule of Sec. 1.5, 1..3: a 1-D problem
                              standing for a flow on a d-dimensional mesh (the
                              Riemann tests of Sec. 2.2 run on a 2-D mesh) */
  int32_t picard_max_iter; /* <= 0: 64 */
  double picard_tol;       /* <= 0: 1e-14 */
  int32_t weno_degree;     /* WENO degree of the subgrid scheme: 1 (0 = default) is the
                              paper's ADER-WENO2 (its ADER-WENO(N+1) naming), 2 is
                              ADER-WENO3 */
  int32_t reserved;        /* must be 0 */
} aderdg_lim_config;

typedef struct aderdg_lim_handle aderdg_lim_handle;

/*
 * aderdg_lim_init -- create a limited problem.  cfg is copied.  hip_stream: a
 * hipStream_t (NULL = default stream).  Allocates library-owned device
 * memory of (5 N + 9) * 3 doubles and one int32 per cell (candidate volume terms,
 * face traces and fluxes, subcell extrema, subgrid results, the troubled-cell
 * list) and a clock.
 * Errors: E_INVAL (*out untouched), E_NOMEM, E_DEVICE.
 */
int aderdg_lim_init(const aderdg_lim_config* cfg, void* hip_stream, aderdg_lim_handle** out);

/*
 * aderdg_lim_project -- v = P u for every cell (Sec. 1.4, eq. p_operator):
 * the subcell averages that start a run.  u, v: device (layouts above).
 */
int aderdg_lim_project(aderdg_lim_handle* h, const double* u, double* v);

/*
 * aderdg_lim_step -- advance by nsteps limited steps.  Each step: dt from the
 * CFL rule of Sec. 1.5, dt = CFL / d / (2N+1) dx / max(|u| + c) over the
 * subcell averages P u of every cell, clamped to t_end; the ADER-DG candidate
 * (nested Picard predictor, Rusanov fluxes; ghost cells as the boundary
 * condition says); PAD (rho > 0, p > 0 of the candidate's subcell averages
 * and nodes) and NAD (eq. nad_ineq on the subcell averages) per cell; the
 * ADER-WENO subgrid step (WENO and LST-DG predictor of degree weno_degree,
 * CFL-compatible since N_s = 2N+1) for the troubled cells; u = R v in them and the flux
 * exchange at their faces.
 *   u         device state, updated in place.
 *   v         device subcell averages, in/out: aderdg_lim_project(u) before
 *             the first step, then as the previous call left them.
 *   troubled  device int32 [ncells], out: the last step's troubled cells.
 *   t         device fp64 [1], in/out.   t_end  device fp64 [1], in.
 *   dt        device fp64 [1], out: last step taken (0 if none).
 *   status    device int32 [1], out: 0, or the most severe of
 *             ADERDG_E_NOCONV (a Picard iteration did not converge) /
 *             ADERDG_E_NONPHYS (the new state is not admissible) met during
 *             the call.
 * Six kernel launches per step plus three per call; no host synchronisation.
 */
int aderdg_lim_step(aderdg_lim_handle* h, double* u, double* v, int32_t* troubled, double* t,
                    const double* t_end, double* dt, int32_t* status, int32_t nsteps);

/* aderdg_lim_counters -- host output, synchronous read: out[0] = troubled
 * cell-steps since init, out[1] = steps whose subgrid step fell back to first
 * order, out[2] = steps taken (dt > 0), out[3] = outer Picard sweeps of the
 * candidate predictor summed over cells and steps (ghost cells excluded). */
int aderdg_lim_counters(aderdg_lim_handle* h, int64_t* out4);

/* aderdg_lim_free -- release the handle (synchronises its stream).  NULL accepted. */
int aderdg_lim_free(aderdg_lim_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* ADERDG_LIM_H */
