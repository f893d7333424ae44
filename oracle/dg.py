"""One-step ADER-DG corrector, CFL time step and the time loop (1-D, periodic).

Corrector: Sec. 1.2, eq. (ader_dg_method_full) with Algorithms 4-7
(get_dg_solution, update_volume_terms, update_interface_terms,
set_interfaces_terms_ksi), in 1-D:

  w_k (u_k^{n+1} - u_k^n) =  sum_a w_a sum_l w_l D^phi_kl f(q_al)                  (volume, flux)
                           - sum_a w_a ( psi~_k G(qR_i(a), qL_{i+1}(a))
                                        - psi_k  G(qR_{i-1}(a), qL_i(a)) )          (surface)
                           - sum_a w_a w_k ( B(q_ak) sum_r D^phi_rk q_ar - s(q_ak) ) (volume, NC + source)

The interface solver G is Rusanov plus, for non-conservative systems, half
of the path-conservative jump B~ (q+ - q-) given to each adjacent cell
(readings: the paper names "a Riemann solver taking into account
non-conservative terms" without a formula; parity unpinned).  f, s and the
jump are rescaled by dt/dx and dt (Sec. 1, definitions after eq. pde_ref).

CFL: Sec. 1.5, d = 1:  dt = CFL / (2N+1) * dx / |lambda_max|, with lambda_max
taken over the finite-volume subcell averages v = P u of every cell
(Sec. 1.4 states that the subcell representation is used to bound the
signal speed), |lambda| = |u| + c.  The last step is clamped to t_end.
Test infrastructure only.
"""

import numpy as np

from .pde import rusanov
from .predictor import predict, traces


def cfl_lambda(ops, pde, u, mode="subcell"):
    """max |lambda| over all cells; 'subcell' uses v = P u (N_s = 2N+1 subcells)."""
    if mode == "subcell":
        v = np.einsum("sk,ckr->csr", ops.P, u)
        return float(pde.max_speed(v).max())
    if mode == "nodal":
        return float(pde.max_speed(u).max())
    raise ValueError(mode)


def cfl_dt(ops, pde, u, dx, cfl, mode="subcell"):
    lam = cfl_lambda(ops, pde, u, mode)
    return cfl * dx / ((2 * ops.N + 1) * lam)


def interface_terms(ops, pde, q, dt, dx):
    """Time-integrated interface flux and jump at every right face i+1/2.

    Returns (Gbar [C, M], Jbar [C, M]); face i+1/2 sits between cell i (its
    right trace) and cell i+1 (its left trace), periodic.
    """
    dtdx = dt / dx
    qL, qR = traces(ops, q)
    qm = qR
    qp = np.roll(qL, -1, axis=0)
    G = dtdx * rusanov(pde, qm, qp)                       # [C, n, M] per time node
    Gbar = np.einsum("a,car->cr", ops.w, G)               # w over time (interface::w_conv_kernel)
    if pde.has_ncp:
        J = dtdx * 0.5 * pde.ncp_jump(qm, qp)
        Jbar = np.einsum("a,car->cr", ops.w, J)
    else:
        Jbar = np.zeros_like(Gbar)
    return Gbar, Jbar


def volume_source_terms(ops, pde, q, dt, dx, x_left, t0):
    """sum_a w_a (s - b)[a, k] at every space node k: [C, n, M]."""
    C = q.shape[0]
    sb = np.zeros_like(q)
    if pde.has_source:
        xs = np.asarray(x_left)[:, None] + dx * ops.xi[None, :]
        ts = t0 + dt * ops.xi
        sb = sb + dt * pde.source(q, xs[:, None, :], ts[None, :, None])
    if pde.has_ncp:
        dq = np.einsum("lj,cajr->calr", ops.ktil, q)       # sum_r D^phi_rl q_ar
        sb = sb - (dt / dx) * pde.ncp(q, dq)
    return np.einsum("a,cakr->ckr", ops.w, sb) if C else sb[:, 0]


def dg_correct(ops, pde, u, q, dt, dx, x_left, t0):
    """u^{n+1} from u^n and the predictor q (eq. ader_dg_method_full)."""
    w = ops.w
    f = (dt / dx) * pde.flux(q)
    fbar = np.einsum("a,calr->clr", w, f)                  # volume::w_conv_kernel
    vol = np.einsum("kl,clr->ckr", ops.Dtil, fbar) / w[None, :, None]   # d_tilde_f_ksi_kernel
    Gbar, Jbar = interface_terms(ops, pde, q, dt, dx)
    G_right, G_left = Gbar, np.roll(Gbar, 1, axis=0)
    J_right, J_left = Jbar, np.roll(Jbar, 1, axis=0)
    surf = (ops.psi1[None, :, None] * G_right[:, None, :]
            - ops.psi0[None, :, None] * G_left[:, None, :]) / w[None, :, None]
    jump = (ops.psi1[None, :, None] * J_right[:, None, :]
            + ops.psi0[None, :, None] * J_left[:, None, :]) / w[None, :, None]
    sb = volume_source_terms(ops, pde, q, dt, dx, x_left, t0)
    return u + vol - surf - jump + sb


def dg_step(ops, pde, u, t, dt, dx, x_left, tol=1e-14, max_iter=64, inner="picard"):
    """One full ADER-DG step: predictor then corrector."""
    q, sweeps, failed = predict(ops, pde, u, dt, dx, x_left, t, tol, max_iter, inner)
    return dg_correct(ops, pde, u, q, dt, dx, x_left, t), sweeps, failed


def conserved_totals(ops, u, dx):
    """dx * sum_i sum_k w_k u_i[k, r] per variable (exact integral of the DG polynomial)."""
    return dx * np.einsum("k,ckr->r", ops.w, u)


def dg_run(ops, pde, u, x0, x1, cfl=0.4, t_end=np.inf, nsteps=None, t0=0.0,
           fixed_dt=None, cfl_mode="subcell", tol=1e-14, max_iter=64, inner="picard"):
    """Advance until t_end or for nsteps steps.  Returns (u, t, info)."""
    u = np.array(u, dtype=np.float64, copy=True)
    C = u.shape[0]
    dx = (x1 - x0) / C
    x_left = x0 + dx * np.arange(C)
    t = float(t0)
    steps = 0
    sweep_hist = {}
    dts = []
    any_failed = False
    while (nsteps is None or steps < nsteps) and t < t_end:
        dt = fixed_dt if fixed_dt else cfl_dt(ops, pde, u, dx, cfl, cfl_mode)
        dt = min(dt, t_end - t)
        if dt <= 0:
            break
        u, sweeps, failed = dg_step(ops, pde, u, t, dt, dx, x_left, tol, max_iter, inner)
        any_failed |= bool(failed.any())
        for s, c in zip(*np.unique(sweeps, return_counts=True)):
            sweep_hist[int(s)] = sweep_hist.get(int(s), 0) + int(c)
        t = t + dt
        dts.append(dt)
        steps += 1
    return u, t, {"steps": steps, "dts": dts, "sweep_hist": sweep_hist, "failed": any_failed}
