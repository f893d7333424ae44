"""Two-dimensional ADER-DG on a uniform periodic Cartesian mesh (Euler gas).

The paper's formulas are written for d = 3; here they are taken with d = 2
(the zeta direction dropped):

  * predictor, Sec. 1.1 "Using the BLAS interface": the Kronecker factors
    L^sigma = kappa~ (x) I (x) I, L^xi = kappa~ (x) k~ (x) I and
    L^eta = kappa~ (x) I (x) k~, so one Picard sweep of a cell is

      q_new[a,i,j] = u[i,j] + sum_b kappa~[a,b] ( - (k~ fx)[b,i,j] - (k~ fy)[b,i,j] ),
      (k~ fx)[b,i,j] = sum_i' k~[i,i'] (dt/dx) Fx(q[b,i',j]),
      (k~ fy)[b,i,j] = sum_j' k~[j,j'] (dt/dy) Fy(q[b,i,j']);

    the loop structure is Algorithm 1 with the k_ksi / k_eta kernels of
    Table 2 (no source and no non-conservative term, so one inner pass);
  * corrector, Sec. 1.2, eq. (ader_dg_method_full) divided by w_i w_j:

      u_new[i,j] = u[i,j]
        + sum_a w_a ( sum_l (w_l D^phi_il / w_i) fx[a,l,j] + sum_l (w_l D^phi_jl / w_j) fy[a,i,l] )
        - (1/w_i) sum_a w_a ( psi~_i Gx(east face; a, j) - psi_i Gx(west face; a, j) )
        - (1/w_j) sum_a w_a ( psi~_j Gy(north face; a, i) - psi_j Gy(south face; a, i) ),

    with fx = (dt/dx) Fx, fy = (dt/dy) Fy, face traces sum_p psi~_p q[., p, .]
    and sum_p psi_p q[., p, .] (Algorithm 7 per direction) and G the Rusanov
    flux along the face normal scaled like f;
  * time step, Sec. 1.5 with d = 2:
      dt = CFL / (d (2N+1)) * min( dx / max|u|+c, dy / max|v|+c ),
    the maxima taken over the (2N+1)^2 subcell averages (P (x) P) u of every
    cell (Sec. 1.4, the projection applied per direction).

The readings of the 1-D oracle carry over: per-cell stopping test
max|q_new - q_old| <= eps0 * max(1, max|q_new|), each cell stopping on its own,
at most max_iter sweeps; Rusanov interface flux (the paper leaves the Riemann
solver open).  Array layout: cells [Cx, Cy] with x slowest, nodes [x node]
[y node], variables fastest; q[cx, cy, a, i, j, r] with the time node first
(the index order of the Kronecker factors above).
Test infrastructure only.
"""

import numpy as np

from .basis import gauss_legendre_01, lagrange_eval


class Euler2D:
    """2-D Euler equations of an ideal gas (Sec. 2, eq. system_of_equations,
    two space dimensions): U = (rho, rho u, rho v, E)."""

    M = 4

    def __init__(self, gamma=1.4):
        self.gamma = float(gamma)

    def primitives(self, Q):
        rho, mx, my, E = Q[..., 0], Q[..., 1], Q[..., 2], Q[..., 3]
        u = mx / rho
        v = my / rho
        p = (self.gamma - 1.0) * (E - 0.5 * (mx * u + my * v))
        return rho, u, v, p

    def flux_x(self, Q):
        rho, u, v, p = self.primitives(Q)
        mx, E = Q[..., 1], Q[..., 3]
        return np.stack([mx, mx * u + p, mx * v, u * (E + p)], axis=-1)

    def flux_y(self, Q):
        rho, u, v, p = self.primitives(Q)
        my, E = Q[..., 2], Q[..., 3]
        return np.stack([my, my * u, my * v + p, v * (E + p)], axis=-1)

    def sound_speed(self, Q):
        rho, u, v, p = self.primitives(Q)
        return np.sqrt(self.gamma * p / rho)

    def speed_x(self, Q):
        return np.abs(self.primitives(Q)[1]) + self.sound_speed(Q)

    def speed_y(self, Q):
        return np.abs(self.primitives(Q)[2]) + self.sound_speed(Q)

    def admissible(self, Q):
        rho, u, v, p = self.primitives(Q)
        return np.isfinite(Q).all(axis=-1) & (rho > 0) & (p > 0)


def rusanov_x(pde, qm, qp):
    """Rusanov flux across a face of normal +x (qm west of it, qp east); parity unpinned."""
    s = np.maximum(pde.speed_x(qm), pde.speed_x(qp))
    return 0.5 * (pde.flux_x(qm) + pde.flux_x(qp)) - 0.5 * s[..., None] * (qp - qm)


def rusanov_y(pde, qm, qp):
    """Rusanov flux across a face of normal +y (qm south of it, qp north); parity unpinned."""
    s = np.maximum(pde.speed_y(qm), pde.speed_y(qp))
    return 0.5 * (pde.flux_y(qm) + pde.flux_y(qp)) - 0.5 * s[..., None] * (qp - qm)


def _cellmax(a):
    return np.abs(a).reshape(a.shape[0], -1).max(axis=1)


def predict2d(ops, pde, u, dt, dx, dy, tol=1e-14, max_iter=64):
    """Space-time predictor of every cell (Sec. 1.1, Algorithm 1, d = 2).

    u : [Cx, Cy, n, n, M] nodal state at the start of the step.
    returns (q [Cx, Cy, n(time), n(x), n(y), M], sweeps [Cx, Cy], failed [Cx, Cy]).
    """
    u = np.asarray(u, dtype=np.float64)
    Cx, Cy, n, _, M = u.shape
    assert n == ops.n and M == pde.M
    uc = u.reshape(Cx * Cy, n, n, M)
    C = uc.shape[0]
    q_init = np.broadcast_to(uc[:, None], (C, n, n, n, M)).copy()   # every time level <- u
    q_prev = q_init.copy()
    sweeps = np.zeros(C, dtype=np.int64)
    failed = np.zeros(C, dtype=bool)
    active = np.arange(C)
    for _ in range(max_iter):
        if active.size == 0:
            break
        qp = q_prev[active]
        fx = (dt / dx) * pde.flux_x(qp)
        fy = (dt / dy) * pde.flux_y(qp)
        kfx = np.einsum("ik,cakjr->caijr", ops.ktil, fx)        # k_ksi_kernel
        kfy = np.einsum("jk,caikr->caijr", ops.ktil, fy)        # k_eta_kernel
        qn = q_init[active] + np.einsum("ab,cbijr->caijr", ops.kappa, -(kfx + kfy))   # kappa_kernel
        eps = _cellmax(qn - qp)
        q_prev[active] = qn
        sweeps[active] += 1
        done = eps <= tol * np.maximum(1.0, _cellmax(qn))
        active = active[~done]
    if active.size:
        failed[active] = True
    return (q_prev.reshape(Cx, Cy, n, n, n, M), sweeps.reshape(Cx, Cy), failed.reshape(Cx, Cy))


def face_fluxes2d(ops, pde, q, dt, dx, dy):
    """Time-integrated Rusanov fluxes through the east face [Cx, Cy, n (y node), M]
    and the north face [Cx, Cy, n (x node), M] of every cell (periodic
    neighbours), scaled by dt/dx and dt/dy: sum_a w_a G(trace; a, node)."""
    w = ops.w
    # face traces (Algorithm 7 per direction): [Cx, Cy, a, j or i, M]
    west = np.einsum("p,xyapjr->xyajr", ops.psi0, q)
    east = np.einsum("p,xyapjr->xyajr", ops.psi1, q)
    south = np.einsum("p,xyaipr->xyair", ops.psi0, q)
    north = np.einsum("p,xyaipr->xyair", ops.psi1, q)
    # flux through the east face of every cell: this cell's east trace, the next cell's west trace
    Gx = (dt / dx) * rusanov_x(pde, east, np.roll(west, -1, axis=0))
    Gy = (dt / dy) * rusanov_y(pde, north, np.roll(south, -1, axis=1))
    return np.einsum("a,xyajr->xyjr", w, Gx), np.einsum("a,xyair->xyir", w, Gy)


def correct2d(ops, pde, u, q, dt, dx, dy):
    """u^{n+1} from u^n and the predictor (eq. ader_dg_method_full, d = 2)."""
    w = ops.w
    fx = (dt / dx) * pde.flux_x(q)
    fy = (dt / dy) * pde.flux_y(q)
    fxbar = np.einsum("a,xyaijr->xyijr", w, fx)                              # time quadrature
    fybar = np.einsum("a,xyaijr->xyijr", w, fy)
    vol = (np.einsum("il,xyljr->xyijr", ops.Dtil, fxbar) / w[None, None, :, None, None]
           + np.einsum("jl,xyilr->xyijr", ops.Dtil, fybar) / w[None, None, None, :, None])
    Gxbar, Gybar = face_fluxes2d(ops, pde, q, dt, dx, dy)
    Gx_e, Gx_w = Gxbar, np.roll(Gxbar, 1, axis=0)
    Gy_n, Gy_s = Gybar, np.roll(Gybar, 1, axis=1)
    surf_x = (ops.psi1[None, None, :, None, None] * Gx_e[:, :, None, :, :]
              - ops.psi0[None, None, :, None, None] * Gx_w[:, :, None, :, :]) / w[None, None, :, None, None]
    surf_y = (ops.psi1[None, None, None, :, None] * Gy_n[:, :, :, None, :]
              - ops.psi0[None, None, None, :, None] * Gy_s[:, :, :, None, :]) / w[None, None, None, :, None]
    return u + vol - surf_x - surf_y


def subcell_averages(ops, u):
    """(P (x) P) u: the (2N+1)^2 subcell averages of every cell (Sec. 1.4)."""
    return np.einsum("si,tj,xyijr->xystr", ops.P, ops.P, u, optimize=True)


def cfl_dt2d(ops, pde, u, dx, dy, cfl):
    """Sec. 1.5 with d = 2 and the signal speeds taken on the subcell averages."""
    v = subcell_averages(ops, u)
    lx = float(pde.speed_x(v).max())
    ly = float(pde.speed_y(v).max())
    return cfl / (2.0 * (2 * ops.N + 1)) * min(dx / lx, dy / ly)


def dg2d_step(ops, pde, u, dt, dx, dy, tol=1e-14, max_iter=64):
    q, sweeps, failed = predict2d(ops, pde, u, dt, dx, dy, tol, max_iter)
    return correct2d(ops, pde, u, q, dt, dx, dy), sweeps, failed


def dg2d_run(ops, pde, u, extent=(0.0, 1.0, 0.0, 1.0), cfl=0.4, t_end=np.inf, nsteps=None, t0=0.0,
             fixed_dt=None, tol=1e-14, max_iter=64):
    """Advance until t_end or for nsteps steps.  Returns (u, t, info)."""
    u = np.array(u, dtype=np.float64, copy=True)
    Cx, Cy = u.shape[:2]
    x0, x1, y0, y1 = extent
    dx, dy = (x1 - x0) / Cx, (y1 - y0) / Cy
    t = float(t0)
    steps = 0
    sweep_hist = {}
    dts = []
    any_failed = False
    while (nsteps is None or steps < nsteps) and t < t_end:
        dt = fixed_dt if fixed_dt else cfl_dt2d(ops, pde, u, dx, dy, cfl)
        dt = min(dt, t_end - t)
        if dt <= 0:
            break
        u, sweeps, failed = dg2d_step(ops, pde, u, dt, dx, dy, tol, max_iter)
        any_failed |= bool(failed.any())
        for s, c in zip(*np.unique(sweeps, return_counts=True)):
            sweep_hist[int(s)] = sweep_hist.get(int(s), 0) + int(c)
        t = t + dt
        dts.append(dt)
        steps += 1
    return u, t, {"steps": steps, "dts": dts, "sweep_hist": sweep_hist, "failed": any_failed}


def conserved_totals2d(ops, u, dx, dy):
    """dx dy sum over cells of sum_ij w_i w_j u[i, j, r] (exact integral of the DG polynomial)."""
    return dx * dy * np.einsum("i,j,xyijr->r", ops.w, ops.w, u)


def dg2d_errors(ops, u, exact, extent=(0.0, 1.0, 0.0, 1.0), var=0, npts=25):
    """L1 and L2 errors of component `var` (Sec. 2.1, eq. epsilons): integrals of
    the DG polynomial cell by cell with an npts-point Gauss-Legendre rule per
    direction.  exact(x, y) takes broadcastable coordinate arrays."""
    Cx, Cy = u.shape[:2]
    x0, x1, y0, y1 = extent
    dx, dy = (x1 - x0) / Cx, (y1 - y0) / Cy
    xq, wq = gauss_legendre_01(npts)
    phi = lagrange_eval(ops.xi, xq)                                   # [Q, n]
    uh = np.einsum("pi,qj,xyij->xypq", phi, phi, u[..., var], optimize=True)
    X = x0 + dx * (np.arange(Cx)[:, None, None, None] + xq[None, None, :, None])
    Y = y0 + dy * (np.arange(Cy)[None, :, None, None] + xq[None, None, None, :])
    err = np.abs(uh - exact(X, Y))
    W = dx * dy * wq[:, None] * wq[None, :]
    l1 = float(np.einsum("pq,xypq->", W, err))
    l2 = float(np.sqrt(np.einsum("pq,xypq->", W, err ** 2)))
    return l1, l2, float(err.max())
