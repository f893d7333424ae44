"""Two-dimensional ADER-WENO finite volumes on a uniform periodic Cartesian
mesh (Euler gas).

Sec. 1.3 with d = 2: the cell averages v (eq. fv_repr) are reconstructed to
nodal values w of a degree-N polynomial per cell (eq. weno_reconstr), w is
the initial data of the LST-DG predictor (Sec. 1.1, the remark after the
predictor's weak form), and the averages are updated with the time- and
face-integrated interface fluxes (eq. ader_weno_fv_method_full):

    v_new = v - sum_a sum_k w_a w_k ( Gx(east; a, k) - Gx(west; a, k) )
              - sum_a sum_k w_a w_k ( Gy(north; a, k) - Gy(south; a, k) ),

G the Rusanov flux of the face traces scaled by dt/dx (dt/dy), a the time
node and k the node along the face.

Reading (the paper states for its WENO timing runs that the reconstruction
is done dimension by dimension, and gives no formula): the 1-D WENO
reconstruction of the oracle's `weno` module along x for every row of cells
gives, at the x nodes, the averages over y of the solution; the same 1-D
reconstruction along y applied to those, node by node, gives the nodal
values.  Time step: Sec. 1.5 with d = 2 and the finite-volume signal speed of
the cell averages, dt = CFL / 2 * min(dx / max(|u|+c), dy / max(|v|+c)).
Test infrastructure only.
"""

import numpy as np

from . import weno
from .dg2d import predict2d, rusanov_x, rusanov_y


def reconstruct2d(v, ops):
    """Nodal WENO values w[Cx, Cy, n (x node), n (y node), M] from the cell
    averages v[Cx, Cy, M] (periodic), dimension by dimension."""
    Cx, Cy, M = v.shape
    n = ops.n
    wx = np.stack([weno.reconstruct(v[:, iy, :], ops) for iy in range(Cy)], axis=1)   # [Cx, Cy, n, M]
    w = np.empty((Cx, Cy, n, n, M))
    for ix in range(Cx):
        for k in range(n):
            w[ix, :, k, :, :] = weno.reconstruct(wx[ix, :, k, :], ops)                # [Cy, n, M]
    return w


def fv2d_dt(pde, v, dx, dy, cfl):
    """Sec. 1.5 with d = 2 for the finite-volume scheme (signal speeds of the averages)."""
    return cfl / 2.0 * min(dx / float(pde.speed_x(v).max()), dy / float(pde.speed_y(v).max()))


def fv2d_step(ops, pde, v, dt, dx, dy, tol=1e-14, max_iter=64, fluxes=False):
    """One ADER-WENO step of the averages; returns (v_new, sweeps, failed), and
    with fluxes=True also the integrated fluxes through the east and the north
    face of every cell [Cx, Cy, M] (v_new = v - the differences of these)."""
    w_hat = reconstruct2d(v, ops)
    q, sweeps, failed = predict2d(ops, pde, w_hat, dt, dx, dy, tol, max_iter)
    w = ops.w
    west = np.einsum("p,xyapjr->xyajr", ops.psi0, q)
    east = np.einsum("p,xyapjr->xyajr", ops.psi1, q)
    south = np.einsum("p,xyaipr->xyair", ops.psi0, q)
    north = np.einsum("p,xyaipr->xyair", ops.psi1, q)
    Gx = (dt / dx) * rusanov_x(pde, east, np.roll(west, -1, axis=0))      # east face of every cell
    Gy = (dt / dy) * rusanov_y(pde, north, np.roll(south, -1, axis=1))    # north face
    Fx = np.einsum("a,k,xyakr->xyr", w, w, Gx)
    Fy = np.einsum("a,k,xyakr->xyr", w, w, Gy)
    v_new = v - (Fx - np.roll(Fx, 1, axis=0)) - (Fy - np.roll(Fy, 1, axis=1))
    if fluxes:
        return v_new, sweeps, failed, Fx, Fy
    return v_new, sweeps, failed


def fv2d_run(ops, pde, v, extent=(0.0, 1.0, 0.0, 1.0), cfl=0.4, t_end=np.inf, nsteps=None, t0=0.0,
             fixed_dt=None, tol=1e-14, max_iter=64):
    """Advance until t_end or for nsteps steps.  Returns (v, t, info)."""
    v = np.array(v, dtype=np.float64, copy=True)
    Cx, Cy = v.shape[:2]
    x0, x1, y0, y1 = extent
    dx, dy = (x1 - x0) / Cx, (y1 - y0) / Cy
    t, steps, dts, any_failed = float(t0), 0, [], False
    while (nsteps is None or steps < nsteps) and t < t_end:
        dt = fixed_dt if fixed_dt else fv2d_dt(pde, v, dx, dy, cfl)
        dt = min(dt, t_end - t)
        if dt <= 0:
            break
        v, sweeps, failed = fv2d_step(ops, pde, v, dt, dx, dy, tol, max_iter)
        any_failed |= bool(failed.any())
        t += dt
        dts.append(dt)
        steps += 1
    return v, t, {"steps": steps, "dts": dts, "failed": any_failed}
