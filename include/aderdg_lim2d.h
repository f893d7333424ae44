/*
 * aderdg_lim2d.h -- C ABI of the 2-D ADER-DG step with a posteriori subcell
 * ADER-WENO finite-volume limiting, for the Euler gas (MI355X, gfx950).
 *
 * Method: I.S. Popov, "The effective use of BLAS interface for implementation
 * of finite-element ADER-DG and finite-volume ADER-WENO methods",
 * arXiv 2409.12483, with d = 2: the 2-D ADER-DG step (Sec. 1.1, 1.2; the one
 * of aderdg2d.h) gives a candidate; the candidate is checked in the subcell
 * representation v = (P (x) P) u of N_s x N_s subcells, N_s = 2N+1 (Sec. 1.4,
 * the projection applied per direction) by the physical and numerical
 * admissibility detectors (Sec. 1.6); every troubled cell is recomputed by
 * the 2-D ADER-WENO2 finite-volume scheme (Sec. 1.3; WENO of degree 1, x
 * then y) on its subgrid with the DG step's dt and returns to the DG
 * representation by u = (R (x) R) v, R the least-squares inverse of P.
 * The PDE is Sec. 2, eq. system_of_equations in 2-D: U = (rho, rho u, rho v, E).
 * Time step: Sec. 1.5 with d = 2, dt = CFL / (2 (2N+1)) min(dx / max(|u|+c),
 * dy / max(|v|+c)) over the subcell averages of the state.
 *
 * Readings where the paper is silent (the test oracle takes the same ones):
 * those of aderdg_lim.h per direction, and
 *   - NAD: V_i = the cell and its eight vertex neighbours (the Voronoi
 *     neighbours of a Cartesian cell), delta = max(1e-4, 1e-3 (max - min))
 *     per variable;
 *   - at a face between a limited and an unlimited cell, the unlimited
 *     cell's flux at face node k is replaced by
 *     sum_s F_s (integral of phi_k over sub-face s) / (N_s w_k), F_s the
 *     subgrid fluxes of the face's N_s sub-faces: every face carries one
 *     flux, and the totals telescope;
 *   - detection / correction cascade: an unlimited cell whose state after
 *     that exchange fails PAD joins the limited cells and the correction is
 *     redone, three passes at most.
 *
 * Conventions (as in aderdg.h): int32 status, 0 = ADERDG_OK, negative =
 * error (codes of aderdg.h); on ADERDG_E_INVAL nothing was enqueued and
 * aderdg_last_error() explains.  "device" pointers are HIP device
 * allocations owned by the caller, contiguous and 8-byte aligned.  Work is
 * enqueued on the handle's stream without host synchronisation (except in
 * init, free and the counter read).  One host thread per handle at a time.
 *
 * Layouts (array-of-structures, variable index fastest; cell (ix, iy) at
 * ix * cells_y + iy):
 *   u         [cells_x][cells_y][N+1 (x node)][N+1 (y node)][4]      fp64
 *   v         [cells_x][cells_y][2N+1 (x subcell)][2N+1 (y subcell)][4]  fp64
 *   troubled  [cells_x][cells_y]                  int32, nonzero = limited in the last step:
 *             1 = found by the detectors, 2 or 3 = added by the detection /
 *             correction cascade (an unlimited cell whose state after the flux
 *             exchange failed PAD; the pass that added it)
 */
#ifndef ADERDG_LIM2D_H
#define ADERDG_LIM2D_H

#include <stdint.h>

#include "aderdg.h"
#include "aderdg_lim.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aderdg2d_lim_config {
  int32_t N;               /* DG degree, 1..9 */
  int32_t bc;              /* ADERDG_LIM_PERIODIC or ADERDG_LIM_TRANSMISSIVE (free outflow,
                            * Sec. 2.2: ghost cells mirror the boundary cells) */
  int64_t cells_x, cells_y;/* >= 3 each */
  double x0, x1, y0, y1;   /* domain */
  double cfl;              /* Courant number in (0, 1] */
  double gamma;            /* > 1 */
  double picard_tol;       /* <= 0: 1e-14 (the candidate's and the subgrid's predictors) */
  int32_t picard_max_iter; /* <= 0: 64 */
  int32_t reserved;        /* must be 0 */
} aderdg2d_lim_config;

typedef struct aderdg2d_lim_handle aderdg2d_lim_handle;

/* Allocates the padded state, the candidate's and the subgrid's scratch and
 * the clock.  E_INVAL for a bad configuration, E_NOMEM on allocation failure. */
int aderdg2d_lim_init(const aderdg2d_lim_config* cfg, void* hip_stream, aderdg2d_lim_handle** out);

/* v = (P (x) P) u (Sec. 1.4): the subcell averages a first limited step
 * starts from.  u, v: device, layouts above. */
int aderdg2d_lim_project(aderdg2d_lim_handle* h, const double* u, double* v);

/* nsteps limited steps of u (in/out), v (in/out: the subcell averages of the
 * step's start, then of its end: P u for unlimited cells, the subgrid result
 * for limited ones) and troubled (out, the last step's).  t (in/out), t_end (in), dt (out),
 * status (out): device arrays of one value, as in aderdg2d_step; status is
 * ADERDG_E_NONPHYS if a subcell average of a final state leaves the admissible
 * set (the limiter keeps those admissible; a polynomial may dip below zero at
 * a node between them, and its next candidate then fails the detectors and
 * is recomputed from them) and ADERDG_E_NOCONV if a candidate's predictor did
 * not converge. */
int aderdg2d_lim_step(aderdg2d_lim_handle* h, double* u, double* v, int32_t* troubled, double* t,
                      const double* t_end, double* dt, int32_t* status, int32_t nsteps);

/* Host copy of the counters since init: out4[0] troubled cells summed over
 * steps, [1] steps whose subgrid step was redone at first order, [2] unused
 * (0), [3] outer Picard sweeps of the candidates' predictors, summed over the
 * padded mesh.  Synchronises the handle's stream. */
int aderdg2d_lim_counters(aderdg2d_lim_handle* h, int64_t* out4);

/* Synchronises the handle's stream and releases it (NULL: no-op). */
int aderdg2d_lim_free(aderdg2d_lim_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* ADERDG_LIM2D_H */
