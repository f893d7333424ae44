"""LST-DG predictor: the nested Picard iteration of Sec. 1.1.

Implements eq. (lst_dg_predictor_nested_picards) in the factored form
derived in Sec. 1.1 "Using the BLAS interface":

    L^sigma = kappa~ (x) I,   L^xi = kappa~ (x) k~,   L^0 u = broadcast of u over time nodes
                                                       (property eq. ind_prop)
so that for one cell, with f = (dt/dx) F, s = dt S, b = (dt/dx) B(q) . (k~ q):

    q^(l+1,m+1)[a,l] = u[l] + sum_b kappa~[a,b] ( s^(l+1,m) - b^(l+1,m) - (k~ f^(l))[b] )[l]

The loop structure is that of Algorithm 1 (get_cell_local_solution) with its
supporting procedures Algorithm 2 (flux terms: k~ applied along the space
index) and Algorithm 3 (non-conservative terms: dq = (D^phi)^T q along the
space index, then B(q_p) dq_p point-wise): an outer loop over flux
iterations and an inner loop over source / non-conservative iterations.

Readings where the paper is silent (Sec. 1.1 leaves the norm, the
tolerance form and loop protection open):
  * per-cell stopping test  max|q_new - q_old| <= eps0 * max(1, max|q_new|);
  * each cell stops on its own test (cells are independent problems);
  * when S = 0 and B = 0 the inner loop is one pass, since its result does
    not depend on the inner iterate;
  * at most max_iter passes of either loop; cells that hit it are flagged.
Test infrastructure only.
"""

import numpy as np


def _cellmax(a):
    return np.abs(a).reshape(a.shape[0], -1).max(axis=1)


def _newton_update(ops, pde, qi, qp, x, ts, dt):
    """One Newton step for the inner system G(q) = q - P(q) = 0, P the Picard
    map with the flux terms frozen (source terms only, which act point-wise,
    so the system splits into one per space node): the Jacobian is
    I - dt (kappa~ (x) I_M) blockdiag_b(dS/dq(q[b, l])), of size nM per node.
    qi: current inner iterate, qp = P(qi); returns the next iterate."""
    C, n, _, M = qi.shape
    Js = pde.source_jacobian(qi, x, ts[None, :, None])                  # [C, b, l, M, M]
    Jm = np.einsum("ab,cblrs->clarbs", ops.kappa, Js)                    # [C, l, a, r, b, s]
    Jm = np.eye(n * M)[None, None] - dt * Jm.reshape(C, n, n * M, n * M)
    G = np.transpose(qi - qp, (0, 2, 1, 3)).reshape(C, n, n * M)        # [C, l, (a, r)]
    delta = np.linalg.solve(Jm, -G[..., None])[..., 0]
    return qi + np.transpose(delta.reshape(C, n, n, M), (0, 2, 1, 3))


def predict(ops, pde, u, dt, dx, x_left, t0, tol=1e-14, max_iter=64, inner="picard"):
    """Space-time predictor for every cell.

    u       : [C, n, M] DG nodal coefficients at t0
    dt, dx  : time step and cell width (uniform mesh)
    x_left  : [C] left edge of each cell (source-term coordinates)
    inner   : "picard" (the nested Picard iteration of eq.
              lst_dg_predictor_nested_picards) or "newton": the inner
              iterations on the source terms by Newton's method, which Sec. 1.1
              recommends for stiff sources (models with a source and no
              non-conservative term)
    returns (q [C, n, n, M] indexed [cell, time node, space node, var],
             outer sweep counts [C], not-converged flags [C])
    """
    if inner not in ("picard", "newton"):
        raise ValueError(inner)
    newton = inner == "newton"
    if newton and (pde.has_ncp or not pde.has_source):
        raise ValueError("Newton inner iterations need a model with a source and no "
                         "non-conservative term")
    u = np.asarray(u, dtype=np.float64)
    C, n, M = u.shape
    assert n == ops.n and M == pde.M
    dtdx = dt / dx
    xs = np.asarray(x_left, dtype=np.float64)[:, None] + dx * ops.xi[None, :]   # [C, n]
    ts = t0 + dt * ops.xi                                                        # [n]
    iterative_inner = pde.has_source or pde.has_ncp

    # q_init[p0] <- u for every time level (Algorithm 1, property eq. ind_prop)
    q_init = np.broadcast_to(u[:, None, :, :], (C, n, n, M)).copy()
    q_prev = q_init.copy()          # init_iter: simple broadcast
    sweeps = np.zeros(C, dtype=np.int64)
    failed = np.zeros(C, dtype=bool)
    active = np.arange(C)

    for _ in range(max_iter):
        if active.size == 0:
            break
        qp = q_prev[active]
        # Algorithm 2: rescaled fluxes at every node, then k~ along the space index
        f = dtdx * pde.flux(qp)
        kf = np.einsum("lj,cajr->calr", ops.ktil, f)
        # inner loop over source / non-conservative terms
        q_int = qp.copy()
        inner_active = np.arange(active.size)
        for _ in range(max_iter):
            qi = q_int[inner_active]
            rhs = -kf[inner_active]
            if pde.has_source:
                x = xs[active[inner_active]][:, None, :]
                rhs = rhs + dt * pde.source(qi, x, ts[None, :, None])
            if pde.has_ncp:
                # Algorithm 3: dq = (D^phi)^T q along the space index (= k~ q), then B(q) dq
                dq = np.einsum("lj,cajr->calr", ops.ktil, qi)
                rhs = rhs - dtdx * pde.ncp(qi, dq)
            # kappa~ along the time index, added onto q_init (Algorithm 1, kappa_kernel)
            qn = q_init[active[inner_active]] + np.einsum("ab,cblr->calr", ops.kappa, rhs)
            if newton:
                qn = _newton_update(ops, pde, qi, qn, xs[active[inner_active]][:, None, :], ts, dt)
            eps_in = _cellmax(qn - qi)
            q_int[inner_active] = qn
            if not iterative_inner:
                inner_active = inner_active[:0]
                break
            done = eps_in <= tol * np.maximum(1.0, _cellmax(qn))
            inner_active = inner_active[~done]
            if inner_active.size == 0:
                break
        if inner_active.size:
            failed[active[inner_active]] = True
        eps_out = _cellmax(q_int - qp)
        q_prev[active] = q_int
        sweeps[active] += 1
        done = eps_out <= tol * np.maximum(1.0, _cellmax(q_int))
        active = active[~done]
    if active.size:
        failed[active] = True
    return q_prev, sweeps, failed


def traces(ops, q):
    """Face values of the predictor at xi = 0 and xi = 1 for every time node.

    qL[c, a] = sum_j psi_j q[c, a, j]   (left face, psi_j = phi_j(0))
    qR[c, a] = sum_j psi~_j q[c, a, j]  (right face, psi~_j = phi_j(1))
    Sec. 1.2, eq. (ader_dg_method_full) and Algorithm 7 (psi_ksi_conv_kernel).
    """
    qL = np.einsum("j,cajr->car", ops.psi0, q)
    qR = np.einsum("j,cajr->car", ops.psi1, q)
    return qL, qR


def evaluate(ops, q, tau, xi):
    """Value of the space-time polynomial q(tau, xi) of every cell: [C, M]."""
    from .basis import lagrange_eval
    pt = lagrange_eval(ops.xi, tau)[0]
    px = lagrange_eval(ops.xi, xi)[0]
    return np.einsum("a,j,cajr->cr", pt, px, q)
