/*
 * aderdg3d.h -- C ABI of the 3-D ADER-DG step for the Euler gas on a uniform
 * periodic Cartesian mesh (MI355X, gfx950).
 *
 * Method: I.S. Popov, arXiv 2409.12483, in the three space dimensions its
 * formulas are written for.  The PDE is Sec. 2, eq. system_of_equations:
 * U = (rho, rho u, rho v, rho w, E), ideal gas.
 *
 * Conventions and error codes: those of aderdg.h.  Layouts (AoS, variables
 * fastest; time before xi before eta before zeta, the index order of the
 * Kronecker factors of Sec. 1.1):
 *   u  [cells_x][cells_y][cells_z][N+1 (x)][N+1 (y)][N+1 (z)][5]           fp64
 *   q  [cells_x][cells_y][cells_z][N+1 (time)][N+1][N+1][N+1][5]           fp64,
 *                                    or fp32 in ADERDG_FP32_PREDICTOR mode
 * Cell (ix, iy, iz) has index (ix * cells_y + iy) * cells_z + iz.
 * Degrees N = 1..9.  The predictor keeps two space-time tiles of
 * (N+1)^4 * 5 values of a cell in the 160 KB of LDS of a compute unit up to
 * N = 5 in FP64 and N = 6 with the FP32 predictor; above, the two tiles live
 * in a library-owned device buffer of 2 (N+1)^4 * 5 values (predictor
 * precision, rounded up to 256 bytes) per cell, e.g. 0.8 MB per cell at
 * N = 9 in FP64.
 */
#ifndef ADERDG3D_H
#define ADERDG3D_H

#include <stdint.h>

#include "aderdg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t N;               /* 1..9 (DG); 1..3 (ADER-WENO) */
  int32_t precision;       /* enum aderdg_prec */
  int64_t cells_x, cells_y, cells_z;   /* >= 1, product <= 2^31 - 1 */
  double x0, x1, y0, y1, z0, z1;       /* domain, upper > lower */
  double gamma;            /* > 1 */
  double cfl;              /* 0 < cfl <= 1 (Sec. 1.5) */
  double fixed_dt;         /* > 0: this dt instead of the CFL rule */
  double picard_tol;       /* <= 0: 1e-14 (FP64) or 1e-6 (FP32 predictor) */
  int32_t picard_max_iter; /* <= 0: 64 */
  int32_t scheme;          /* ADERDG_SCHEME_DG (0), or ADERDG_SCHEME_FV: ADER-WENO finite
                              volumes (Sec. 1.3 with d = 3), N = the WENO degree (1: the
                              paper's ADER-WENO2, 2: ADER-WENO3, 3: ADER-WENO4), FP64 only;
                              the state is
                              then the cell averages v [cells_x][cells_y][cells_z][5] */
} aderdg3d_config;

typedef struct aderdg3d_handle aderdg3d_handle;

/*
 * aderdg3d_init -- create a 3-D problem (cfg copied; hip_stream NULL = default
 * stream).  Allocates per cell u + volume terms ((N+1)^3 5 doubles; ADER-WENO:
 * the nodal WENO values, as many), the six face traces (6 (N+1)^3 5 values in
 * the predictor precision) and, where the predictor's tiles exceed LDS, those
 * tiles (above), and a device clock.  E_INVAL (*out untouched), E_NOMEM, E_DEVICE.
 */
int aderdg3d_init(const aderdg3d_config* cfg, void* hip_stream, aderdg3d_handle** out);

/*
 * aderdg3d_predict -- LST-DG predictor of every cell (Sec. 1.1, Algorithm 1
 * with the k_ksi, k_eta, k_zeta kernels of Table 2).  u: device state; t and
 * dt > 0: the step.  q_out: device predictor (layout above).  iters_out:
 * optional device int32 [cells], each cell's sweeps.  Stopping test per cell:
 * max|dq| <= tol * max(1, max|q|).
 */
int aderdg3d_predict(aderdg3d_handle* h, const double* u, double t, double dt, void* q_out,
                     int32_t* iters_out);

/*
 * aderdg3d_step -- nsteps steps of the predictor and the corrector of Sec. 1.2,
 * eq. ader_dg_method_full (Rusanov fluxes through the six faces), with
 * dt = CFL / (3 (2N+1)) min over directions of h / max(|u_d| + c), the maxima
 * over the (2N+1)^3 subcell averages of every cell (Sec. 1.4-1.5), or
 * fixed_dt; the last step is clamped to t_end.  u in place; t, t_end, dt,
 * status: device scalars as in aderdg2d_step.  No host synchronisation.
 */
int aderdg3d_step(aderdg3d_handle* h, double* u, double* t, const double* t_end, double* dt,
                  int32_t* status, int32_t nsteps);

/* aderdg3d_sweep_count -- Picard sweeps summed over cells and steps since
 * init (host output, synchronous). */
int aderdg3d_sweep_count(aderdg3d_handle* h, int64_t* sweeps_out);

/* aderdg3d_free -- release the handle (synchronises its stream).  NULL accepted. */
int aderdg3d_free(aderdg3d_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* ADERDG3D_H */
