"""One-step ADER-WENO finite-volume scheme (1-D, periodic).

Sec. 1.3, eq. (ader_weno_fv_method_full) with Algorithms 8-11
(get_fv_solution, update_volume_terms, set_interfaces_terms_ksi), in 1-D:

  v^{n+1} = v^n - sum_a w_a [ G(qR_i(a), qL_{i+1}(a)) - G(qR_{i-1}(a), qL_i(a)) ]
                - sum_a sum_j w_a w_j [ B(q_aj) sum_r D^phi_rj q_ar - s(q_aj) ]

where q is the LST-DG predictor started from the WENO reconstruction
(Sec. 1.1: "select the initial condition q(0, xi) = w(xi)").  G is the
Rusanov flux plus half of the path-conservative jump given to each adjacent
cell (same reading as the DG corrector; parity unpinned).
CFL (Sec. 1.5): the finite-volume form has no 2N+1 factor: dt = CFL dx / |lambda_max|
with lambda over the cell averages.
Test infrastructure only.
"""

import numpy as np

from .dg import interface_terms, volume_source_terms
from .predictor import predict
from .weno import reconstruct


def fv_dt(pde, v, dx, cfl):
    return cfl * dx / float(pde.max_speed(v).max())


def _fv_update(ops, pde, v, t, dt, dx, x_left, tol, max_iter):
    w_hat = reconstruct(v, ops)
    q, sweeps, failed = predict(ops, pde, w_hat, dt, dx, x_left, t, tol, max_iter)
    Gbar, Jbar = interface_terms(ops, pde, q, dt, dx)
    sb = volume_source_terms(ops, pde, q, dt, dx, x_left, t)      # [C, n, M]
    vol = np.einsum("k,ckr->cr", ops.w, sb)                       # w over space nodes
    v_new = v - (Gbar - np.roll(Gbar, 1, axis=0)) - (Jbar + np.roll(Jbar, 1, axis=0)) + vol
    return v_new, sweeps, failed, Gbar


def fv_step(ops, pde, v, t, dt, dx, x_left, tol=1e-14, max_iter=64):
    v_new, sweeps, failed, _ = _fv_update(ops, pde, v, t, dt, dx, x_left, tol, max_iter)
    return v_new, sweeps, failed


def fv_step_terms(ops, pde, v, t, dt, dx, x_left, tol=1e-14, max_iter=64):
    """fv_step's new averages and its time-integrated flux through the right
    face of every cell (for the subcell limiter's face bookkeeping)."""
    v_new, _, _, Gbar = _fv_update(ops, pde, v, t, dt, dx, x_left, tol, max_iter)
    return v_new, Gbar


def fv_run(ops, pde, v, x0, x1, cfl=0.4, t_end=np.inf, nsteps=None, t0=0.0,
           fixed_dt=None, tol=1e-14, max_iter=64):
    v = np.array(v, dtype=np.float64, copy=True)
    C = v.shape[0]
    dx = (x1 - x0) / C
    x_left = x0 + dx * np.arange(C)
    t = float(t0)
    steps = 0
    sweep_hist = {}
    dts = []
    any_failed = False
    while (nsteps is None or steps < nsteps) and t < t_end:
        dt = fixed_dt if fixed_dt else fv_dt(pde, v, dx, cfl)
        dt = min(dt, t_end - t)
        if dt <= 0:
            break
        v, sweeps, failed = fv_step(ops, pde, v, t, dt, dx, x_left, tol, max_iter)
        any_failed |= bool(failed.any())
        for s, c in zip(*np.unique(sweeps, return_counts=True)):
            sweep_hist[int(s)] = sweep_hist.get(int(s), 0) + int(c)
        t += dt
        dts.append(dt)
        steps += 1
    return v, t, {"steps": steps, "dts": dts, "sweep_hist": sweep_hist, "failed": any_failed}
