"""Three-dimensional ADER-WENO finite volumes on a uniform periodic Cartesian
mesh (Euler gas).

Sec. 1.3 with d = 3, in the same way as the 2-D oracle (`fv2d`): the cell
averages are reconstructed dimension by dimension (the 1-D WENO of the
oracle's `weno` module along x for every line of cells, then along y at every
x node, then along z at every (x, y) node pair) to nodal values of a degree-N
polynomial, which start the 3-D LST-DG predictor; the averages are updated
with the time- and face-integrated Rusanov fluxes,

    v_new = v - sum_d ( F_d(+ face) - F_d(- face) ),
    F_d = sum_a sum_s sum_t w_a w_s w_t (dt/h_d) G_d(a, s, t),

(s, t) the nodes of the face.  Time step: Sec. 1.5 with d = 3 and the signal
speeds of the averages, dt = CFL / 3 * min_d h_d / max(|u_d| + c).
Test infrastructure only.
"""

import numpy as np

from . import weno
from .dg3d import predict3d, rusanov


def _along(v, ops, axis):
    """1-D WENO of v along `axis` (periodic), every other index treated as a
    separate variable; the new node index is appended before the last axis."""
    moved = np.moveaxis(v, axis, 0)
    C = moved.shape[0]
    rest = moved.shape[1:]
    w = weno.reconstruct(moved.reshape(C, -1), ops)                  # [C, n, prod(rest)]
    w = w.reshape((C, ops.n) + rest)                                  # [C, n, *rest]
    w = np.moveaxis(w, 1, -1)                                         # node last
    w = np.moveaxis(w, 0, axis)                                       # C back in place
    return np.moveaxis(w, -1, -2)                                     # node before the variables


def reconstruct3d(v, ops):
    """Nodal WENO values w[Cx, Cy, Cz, n (x), n (y), n (z), M] from the averages
    v[Cx, Cy, Cz, M], dimension by dimension."""
    wx = _along(v, ops, 0)                        # [Cx, Cy, Cz, nx, M]
    wy = _along(wx, ops, 1)                       # [Cx, Cy, Cz, nx, ny, M]
    return _along(wy, ops, 2)                     # [Cx, Cy, Cz, nx, ny, nz, M]


def fv3d_dt(pde, v, h, cfl):
    return cfl / 3.0 * min(h[d] / float(pde.speed(v, d).max()) for d in range(3))


def fv3d_step(ops, pde, v, dt, h, tol=1e-14, max_iter=64, fluxes=False):
    """One ADER-WENO step of the averages; returns (v_new, sweeps, failed), and
    with fluxes=True also the integrated fluxes through the + face of every
    cell along x, y and z ([Cx, Cy, Cz, M] each)."""
    w_hat = reconstruct3d(v, ops)
    q, sweeps, failed = predict3d(ops, pde, w_hat, dt, h, tol, max_iter)
    w = ops.w
    v_new = np.array(v, dtype=np.float64, copy=True)
    Fs = []
    for d in range(3):
        sub = ["p,xyzapjkr->xyzajkr", "p,xyzaipkr->xyzaikr", "p,xyzaijpr->xyzaijr"][d]
        lo = np.einsum(sub, ops.psi0, q)
        hi = np.einsum(sub, ops.psi1, q)
        G = (dt / h[d]) * rusanov(pde, hi, np.roll(lo, -1, axis=d), d)          # + face of every cell
        F = np.einsum("a,s,t,xyzastr->xyzr", w, w, w, G)
        v_new = v_new - (F - np.roll(F, 1, axis=d))
        Fs.append(F)
    if fluxes:
        return v_new, sweeps, failed, Fs
    return v_new, sweeps, failed


def fv3d_run(ops, pde, v, extent=(1.0, 1.0, 1.0), cfl=0.4, t_end=np.inf, nsteps=None, t0=0.0,
             fixed_dt=None, tol=1e-14, max_iter=64):
    v = np.array(v, dtype=np.float64, copy=True)
    h = tuple(extent[d] / v.shape[d] for d in range(3))
    t, steps, dts, any_failed = float(t0), 0, [], False
    while (nsteps is None or steps < nsteps) and t < t_end:
        dt = fixed_dt if fixed_dt else fv3d_dt(pde, v, h, cfl)
        dt = min(dt, t_end - t)
        if dt <= 0:
            break
        v, sweeps, failed = fv3d_step(ops, pde, v, dt, h, tol, max_iter)
        any_failed |= bool(failed.any())
        t += dt
        dts.append(dt)
        steps += 1
    return v, t, {"steps": steps, "dts": dts, "failed": any_failed}
