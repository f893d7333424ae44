/*
 * aderdg2d.h -- C ABI of the 2-D ADER-DG step for the Euler gas on a uniform
 * periodic Cartesian mesh (MI355X, gfx950).
 *
 * Method: I.S. Popov, "The effective use of BLAS interface for implementation
 * of finite-element ADER-DG and finite-volume ADER-WENO methods",
 * arXiv 2409.12483, with two space dimensions (the zeta direction of its
 * 3-D formulas dropped).  The PDE is Sec. 2, eq. system_of_equations:
 * U = (rho, rho u, rho v, E), ideal gas p = (gamma - 1)(E - rho (u^2+v^2)/2).
 *
 * Conventions (as in aderdg.h): int32 status, 0 = ADERDG_OK, negative =
 * error (codes of aderdg.h); on ADERDG_E_INVAL nothing was enqueued and
 * aderdg_last_error() explains.  "device" pointers are HIP device
 * allocations owned by the caller, contiguous and 8-byte aligned.  Work is
 * enqueued on the handle's stream without host synchronisation (except in
 * init, free and the counter read).  One host thread per handle at a time.
 *
 * Layouts (array-of-structures, variable index fastest; the index order of
 * the Kronecker factors of Sec. 1.1, time before xi before eta):
 *   u  [cells_x][cells_y][N+1 (x node)][N+1 (y node)][4]          fp64
 *   q  [cells_x][cells_y][N+1 (time)][N+1 (x)][N+1 (y)][4]        fp64, or
 *                                         fp32 in ADERDG_FP32_PREDICTOR mode
 *   v  [cells_x][cells_y][4]                                       fp64 cell averages
 *                                         (the state of the ADER-WENO scheme)
 * Cell (ix, iy) spans [x0 + ix dx, x0 + (ix+1) dx] x [y0 + iy dy, ...];
 * nodes are the Gauss-Legendre points of [0, 1] in each direction.
 */
#ifndef ADERDG2D_H
#define ADERDG2D_H

#include <stdint.h>

#include "aderdg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t N;               /* polynomial degree, 1..9 */
  int32_t precision;       /* enum aderdg_prec */
  int64_t cells_x;         /* >= 1 */
  int64_t cells_y;         /* >= 1; cells_x * cells_y <= 2^31 - 1 */
  double x0, x1, y0, y1;   /* domain, x1 > x0, y1 > y0 */
  double gamma;            /* ratio of specific heats, > 1 */
  double cfl;              /* 0 < cfl <= 1 (Sec. 1.5) */
  double fixed_dt;         /* > 0: use this dt instead of the CFL rule; 0: CFL rule */
  double picard_tol;       /* <= 0: 1e-14 (FP64) or 1e-6 (FP32 predictor) */
  int32_t picard_max_iter; /* <= 0: 64 */
  int32_t scheme;          /* ADERDG_SCHEME_DG (0), or ADERDG_SCHEME_FV: ADER-WENO finite
                              volumes (Sec. 1.3 with d = 2), N = the WENO degree (1: the
                              paper's ADER-WENO2, 2: ADER-WENO3, 3: ADER-WENO4), FP64 only */
} aderdg2d_config;

typedef struct aderdg2d_handle aderdg2d_handle;

/*
 * aderdg2d_init -- create a 2-D problem.  cfg is copied.  hip_stream: a
 * hipStream_t (NULL = default stream).  Allocates library-owned device
 * memory: per cell u + volume terms ((N+1)^2 4 doubles) and the four face
 * traces (4 (N+1)^2 4 values in the predictor precision), and a clock.
 * Errors: E_INVAL (*out untouched), E_NOMEM, E_DEVICE.
 */
int aderdg2d_init(const aderdg2d_config* cfg, void* hip_stream, aderdg2d_handle** out);

/*
 * aderdg2d_predict -- (DG scheme) LST-DG predictor of every cell (Sec. 1.1, the nested
 * Picard iteration with the factors kappa~ (x) k~ (x) I and
 * kappa~ (x) I (x) k~; Algorithm 1 with the k_ksi and k_eta kernels of
 * Table 2).  u: device state (layout above); t, dt > 0: start and length of
 * the step.  q_out: device predictor (layout above, predictor precision).
 * iters_out: optional device int32 [cells] receiving each cell's sweeps.
 * Each cell stops when max|dq| <= tol * max(1, max|q|).
 */
int aderdg2d_predict(aderdg2d_handle* h, const double* u, double t, double dt, void* q_out,
                     int32_t* iters_out);

/*
 * aderdg2d_step -- advance the problem by nsteps steps: predictor, then the
 * corrector of Sec. 1.2, eq. ader_dg_method_full (volume terms, Rusanov
 * fluxes through the four faces), with dt from Sec. 1.5 for d = 2:
 * dt = CFL / (2 (2N+1)) min(dx / max(|u|+c), dy / max(|v|+c)), the maxima
 * over the (2N+1)^2 subcell averages of every cell (Sec. 1.4), or fixed_dt;
 * the last step is clamped to t_end.
 *   u       device state, updated in place.
 *   t       device fp64 [1], in/out.   t_end  device fp64 [1], in.
 *   dt      device fp64 [1], out: last step taken (0 if none).
 *   status  device int32 [1], out: 0, or the most severe of ADERDG_E_NOCONV /
 *           ADERDG_E_NONPHYS met during the call.
 * Two kernel launches per step; no host synchronisation.
 * With scheme ADERDG_SCHEME_FV the state is v (cell averages) and a step is
 * the ADER-WENO scheme of Sec. 1.3 with d = 2: WENO reconstruction of degree N
 * of the averages, dimension by dimension (along x for every row of cells,
 * giving the averages over y at the x nodes, then along y at every x node;
 * degree 1: stencils {i-1, i}, {i, i+1}; degree 2: {i-2..i}, {i-1..i+1},
 * {i..i+2}; degree 3: {i-3..i}, {i-2..i+1}, {i-1..i+2}, {i..i+3}; weights
 * lambda_s / (sigma_s + 1e-14)^8, lambda = 1e5 for the central stencils,
 * else 1), the predictor above from those nodal values, and
 * v -= sum over the four faces of the time- and face-integrated Rusanov
 * fluxes; dt = CFL / 2 min(dx / max(|u|+c), dy / max(|v|+c)) over the
 * averages.  Three launches per step.
 */
int aderdg2d_step(aderdg2d_handle* h, double* u, double* t, const double* t_end, double* dt,
                  int32_t* status, int32_t nsteps);

/* aderdg2d_sweep_count -- Picard sweeps summed over cells and steps since
 * init (host output, synchronous read). */
int aderdg2d_sweep_count(aderdg2d_handle* h, int64_t* sweeps_out);

/* aderdg2d_free -- release the handle (synchronises its stream).  NULL accepted. */
int aderdg2d_free(aderdg2d_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* ADERDG2D_H */
