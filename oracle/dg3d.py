"""Three-dimensional ADER-DG on a uniform periodic Cartesian mesh (Euler gas).

The paper's formulas as written (d = 3):

  * predictor, Sec. 1.1 "Using the BLAS interface": the Kronecker factors
    L^xi = kappa~ (x) k~ (x) I (x) I, L^eta = kappa~ (x) I (x) k~ (x) I and
    L^zeta = kappa~ (x) I (x) I (x) k~, so one Picard sweep of a cell is

      q_new[a,i,j,k] = u[i,j,k] + sum_b kappa~[a,b] ( - (k~ fx) - (k~ fy) - (k~ fz) )[b,i,j,k],

    with fx = (dt/dx) Fx(q) contracted by k~ along i, fy along j, fz along k
    (Algorithm 1 with the k_ksi, k_eta, k_zeta kernels of Table 2; no source
    and no non-conservative term, so one inner pass);
  * corrector, Sec. 1.2, eq. (ader_dg_method_full) divided by w_i w_j w_k:
    volume terms sum_a w_a sum_l (w_l D^phi_il / w_i) fx[a,l,j,k] and the like
    along j and k; surface terms (1/w_i) sum_a w_a (psi~_i G(+x face) -
    psi_i G(-x face)) and the like, from the face traces of Algorithm 7 in
    each direction, G the Rusanov flux along the face normal scaled like f;
  * time step, Sec. 1.5 with d = 3: dt = CFL / (3 (2N+1)) * min over the
    directions of h / max(|u_d| + c), the maxima over the (2N+1)^3 subcell
    averages (P (x) P (x) P) u of every cell (Sec. 1.4).

Readings as in the 2-D oracle (oracle.dg2d).  Array layout: cells
[Cx, Cy, Cz] (x slowest), nodes [x][y][z], variables fastest;
q[cx, cy, cz, a, i, j, k, r] with the time node first.
Test infrastructure only.
"""

import numpy as np

from .basis import gauss_legendre_01, lagrange_eval


class Euler3D:
    """3-D Euler equations of an ideal gas (Sec. 2, eq. system_of_equations):
    U = (rho, rho u, rho v, rho w, E)."""

    M = 5

    def __init__(self, gamma=1.4):
        self.gamma = float(gamma)

    def primitives(self, Q):
        rho = Q[..., 0]
        vel = [Q[..., 1] / rho, Q[..., 2] / rho, Q[..., 3] / rho]
        p = (self.gamma - 1.0) * (Q[..., 4] - 0.5 * (Q[..., 1] * vel[0] + Q[..., 2] * vel[1]
                                                     + Q[..., 3] * vel[2]))
        return rho, vel, p

    def flux(self, Q, d):
        """Flux along direction d (0: x, 1: y, 2: z)."""
        rho, vel, p = self.primitives(Q)
        m = Q[..., 1 + d]
        f = [m, m * vel[0], m * vel[1], m * vel[2], vel[d] * (Q[..., 4] + p)]
        f[1 + d] = f[1 + d] + p
        return np.stack(f, axis=-1)

    def speed(self, Q, d):
        rho, vel, p = self.primitives(Q)
        return np.abs(vel[d]) + np.sqrt(self.gamma * p / rho)

    def admissible(self, Q):
        """rho > 0 and p > 0 (and finite): the physical admissibility of Sec. 1.6."""
        rho, vel, p = self.primitives(Q)
        return np.isfinite(Q).all(axis=-1) & (rho > 0) & (p > 0)


def rusanov(pde, qm, qp, d):
    """Rusanov flux across a face of normal +e_d (qm on the minus side); parity unpinned."""
    s = np.maximum(pde.speed(qm, d), pde.speed(qp, d))
    return 0.5 * (pde.flux(qm, d) + pde.flux(qp, d)) - 0.5 * s[..., None] * (qp - qm)


def _cellmax(a):
    return np.abs(a).reshape(a.shape[0], -1).max(axis=1)


# einsum subscripts of the contraction along space direction d of a
# [cell, time, x, y, z, var] array by an n x n operator
_ALONG = ["il,calmnr->caimnr", "jm,calmnr->caljnr", "kn,calmnr->calmkr"]


def predict3d(ops, pde, u, dt, h, tol=1e-14, max_iter=64):
    """Space-time predictor of every cell (Sec. 1.1, Algorithm 1, d = 3).

    u : [Cx, Cy, Cz, n, n, n, M]; h = (dx, dy, dz).
    returns (q [Cx, Cy, Cz, n(time), n, n, n, M], sweeps [Cx, Cy, Cz], failed).
    """
    u = np.asarray(u, dtype=np.float64)
    shape = u.shape[:3]
    n, M = u.shape[3], u.shape[-1]
    assert n == ops.n and M == pde.M
    uc = u.reshape((-1, n, n, n, M))
    C = uc.shape[0]
    q_init = np.broadcast_to(uc[:, None], (C, n, n, n, n, M)).copy()
    q_prev = q_init.copy()
    sweeps = np.zeros(C, dtype=np.int64)
    failed = np.zeros(C, dtype=bool)
    active = np.arange(C)
    for _ in range(max_iter):
        if active.size == 0:
            break
        qp = q_prev[active]
        kf = 0.0
        for d in range(3):
            kf = kf + np.einsum(_ALONG[d], ops.ktil, (dt / h[d]) * pde.flux(qp, d))   # k_ksi/eta/zeta
        qn = q_init[active] + np.einsum("ab,cbijkr->caijkr", ops.kappa, -kf)          # kappa_kernel
        eps = _cellmax(qn - qp)
        q_prev[active] = qn
        sweeps[active] += 1
        done = eps <= tol * np.maximum(1.0, _cellmax(qn))
        active = active[~done]
    if active.size:
        failed[active] = True
    return (q_prev.reshape(shape + (n, n, n, n, M)), sweeps.reshape(shape), failed.reshape(shape))


def face_fluxes3d(ops, pde, q, dt, h):
    """Time-integrated Rusanov fluxes through the + face of every cell along
    each direction d, scaled by dt/h_d: [Cx, Cy, Cz, n, n, M] per d, the two
    face-node indices in the order of the remaining axes (periodic
    neighbours); q [Cx, Cy, Cz, n (time), n, n, n, M]."""
    w = ops.w
    out = []
    for d in range(3):
        # traces on the minus (psi) and plus (psi~) faces along d: [Cx, Cy, Cz, a, ., ., M]
        sub = ["p,xyzapjkr->xyzajkr", "p,xyzaipkr->xyzaikr", "p,xyzaijpr->xyzaijr"][d]
        lo = np.einsum(sub, ops.psi0, q)
        hi = np.einsum(sub, ops.psi1, q)
        G = (dt / h[d]) * rusanov(pde, hi, np.roll(lo, -1, axis=d), d)   # through the + face of each cell
        out.append(np.einsum("a,xyzastr->xyzstr", w, G))
    return out


def correct3d(ops, pde, u, q, dt, h):
    """u^{n+1} from u^n and the predictor (eq. ader_dg_method_full, d = 3)."""
    w = ops.w
    n = ops.n
    Cx, Cy, Cz = u.shape[:3]
    M = u.shape[-1]
    flat = q.reshape((-1, n, n, n, n, M))
    out = np.array(u, dtype=np.float64, copy=True).reshape((-1, n, n, n, M))
    wshape = [(n, 1, 1, 1), (1, n, 1, 1), (1, 1, n, 1)]
    for d in range(3):
        f = (dt / h[d]) * pde.flux(flat, d)
        fbar = np.einsum("a,caijkr->cijkr", w, f)                                   # time quadrature
        sub = ["il,cljkr->cijkr", "jl,cilkr->cijkr", "kl,cijlr->cijkr"][d]
        out = out + np.einsum(sub, ops.Dtil, fbar) / w.reshape(wshape[d])
    faces = face_fluxes3d(ops, pde, q.reshape((Cx, Cy, Cz, n, n, n, n, M)), dt, h)
    for d in range(3):
        Gbar = faces[d]                                                    # [Cx, Cy, Cz, ., ., M]
        Gm = np.roll(Gbar, 1, axis=d)                                      # through the - face
        Gp = Gbar.reshape((-1,) + Gbar.shape[3:])
        Gm = Gm.reshape((-1,) + Gm.shape[3:])
        # insert the face-normal node index at position d of (i, j, k)
        p1 = ops.psi1 / w
        p0 = ops.psi0 / w
        if d == 0:
            surf = p1[None, :, None, None, None] * Gp[:, None] - p0[None, :, None, None, None] * Gm[:, None]
        elif d == 1:
            surf = p1[None, None, :, None, None] * Gp[:, :, None] - p0[None, None, :, None, None] * Gm[:, :, None]
        else:
            surf = p1[None, None, None, :, None] * Gp[:, :, :, None] - p0[None, None, None, :, None] * Gm[:, :, :, None]
        out = out - surf
    return out.reshape(u.shape)


def subcell_averages(ops, u):
    """(P (x) P (x) P) u: the (2N+1)^3 subcell averages of every cell (Sec. 1.4)."""
    return np.einsum("si,tj,vk,xyzijkr->xyzstvr", ops.P, ops.P, ops.P, u, optimize=True)


def cfl_dt3d(ops, pde, u, h, cfl):
    """Sec. 1.5 with d = 3 and the signal speeds taken on the subcell averages."""
    v = subcell_averages(ops, u)
    return cfl / (3.0 * (2 * ops.N + 1)) * min(h[d] / float(pde.speed(v, d).max()) for d in range(3))


def dg3d_run(ops, pde, u, extent=(1.0, 1.0, 1.0), cfl=0.4, t_end=np.inf, nsteps=None, t0=0.0,
             fixed_dt=None, tol=1e-14, max_iter=64):
    """Advance until t_end or for nsteps steps (domain [0, Lx] x [0, Ly] x [0, Lz])."""
    u = np.array(u, dtype=np.float64, copy=True)
    h = tuple(extent[d] / u.shape[d] for d in range(3))
    t = float(t0)
    steps = 0
    sweep_hist = {}
    dts = []
    any_failed = False
    while (nsteps is None or steps < nsteps) and t < t_end:
        dt = fixed_dt if fixed_dt else cfl_dt3d(ops, pde, u, h, cfl)
        dt = min(dt, t_end - t)
        if dt <= 0:
            break
        q, sweeps, failed = predict3d(ops, pde, u, dt, h, tol, max_iter)
        u = correct3d(ops, pde, u, q, dt, h)
        any_failed |= bool(failed.any())
        for s, c in zip(*np.unique(sweeps, return_counts=True)):
            sweep_hist[int(s)] = sweep_hist.get(int(s), 0) + int(c)
        t = t + dt
        dts.append(dt)
        steps += 1
    return u, t, {"steps": steps, "dts": dts, "sweep_hist": sweep_hist, "failed": any_failed}


def conserved_totals3d(ops, u, h):
    """Exact integral of the DG polynomial of every variable over the domain."""
    return h[0] * h[1] * h[2] * np.einsum("i,j,k,xyzijkr->r", ops.w, ops.w, ops.w, u, optimize=True)


def dg3d_errors(ops, u, exact, extent=(1.0, 1.0, 1.0), var=0, npts=10):
    """L1 and L2 errors of component `var` (Sec. 2.1, eq. epsilons) with an
    npts-point Gauss-Legendre rule per direction in every cell."""
    Cx, Cy, Cz = u.shape[:3]
    h = [extent[d] / u.shape[d] for d in range(3)]
    xq, wq = gauss_legendre_01(npts)
    phi = lagrange_eval(ops.xi, xq)
    uh = np.einsum("pi,qj,sk,xyzijk->xyzpqs", phi, phi, phi, u[..., var], optimize=True)
    X = h[0] * (np.arange(Cx)[:, None, None, None, None, None] + xq[None, None, None, :, None, None])
    Y = h[1] * (np.arange(Cy)[None, :, None, None, None, None] + xq[None, None, None, None, :, None])
    Z = h[2] * (np.arange(Cz)[None, None, :, None, None, None] + xq[None, None, None, None, None, :])
    err = np.abs(uh - exact(X, Y, Z))
    W = h[0] * h[1] * h[2] * np.einsum("p,q,s->pqs", wq, wq, wq)
    return (float(np.einsum("pqs,xyzpqs->", W, err)), float(np.sqrt(np.einsum("pqs,xyzpqs->", W, err ** 2))),
            float(err.max()))
