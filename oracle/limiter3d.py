"""A posteriori subcell finite-volume limiting of the 3-D ADER-DG step (Euler gas).

Sec. 1.4 and Sec. 1.6 with d = 3: the construction of the 2-D limiter of this
oracle (module `limiter2d`, with its readings) taken per direction:

  * candidate u* from the 3-D ADER-DG step (module `dg3d`) on a mesh padded
    with one ghost cell per side (periodic images, or mirror images for free
    outflow: nodes or subcells reversed along the face normal);
  * PAD on the candidate's nodes and (P (x) P (x) P) subcell averages; NAD over
    the cell and its 26 vertex neighbours, delta as in 1-D;
  * troubled cells recomputed by the 3-D ADER-WENO scheme (module `fv3d`,
    reconstruction of degree nw) on the padded mesh's whole subgrid from v^n
    with the DG step's dt (first order when that leaves the admissible set in
    a troubled cell); u = (R (x) R (x) R) v, scaled toward the mean until
    admissible;
  * one flux per face node: an unlimited neighbour's flux at face node (k, l)
    is replaced by sum_{s,t} F_st (integral of phi_k phi_l over sub-face
    (s, t)) / (N_s^2 w_k w_l) in face units, i.e. sum_{s,t} F_st p[s,k] p[t,l]
    / N_s with p = P / (N_s w) (F_st the subgrid fluxes in subcell units);
  * the detection / correction cascade, three passes at most.
Test infrastructure only.
"""

import numpy as np

from . import basis
from .dg3d import cfl_dt3d, correct3d, face_fluxes3d, predict3d, subcell_averages
from .fv3d import fv3d_step
from .limiter import DELTA0, EPS0, subcell_R

PASSES = 3


def pad3d(a, bc):
    """One ghost cell on every side of per-cell data a[Cx, Cy, Cz, k, l, m, ...]
    whose axes 3, 4, 5 run along x, y, z inside the cell."""
    for d in range(3):
        if bc == "periodic":
            lo, hi = np.take(a, [-1], axis=d), np.take(a, [0], axis=d)
        else:
            lo = np.flip(np.take(a, [0], axis=d), axis=3 + d)
            hi = np.flip(np.take(a, [-1], axis=d), axis=3 + d)
        a = np.concatenate([lo, a, hi], axis=d)
    return a


def to_subgrid3(v):
    Cx, Cy, Cz, Ns, _, _, M = v.shape
    return v.transpose(0, 3, 1, 4, 2, 5, 6).reshape(Cx * Ns, Cy * Ns, Cz * Ns, M)


def from_subgrid3(s, Ns):
    X, Y, Z, M = s.shape
    return s.reshape(X // Ns, Ns, Y // Ns, Ns, Z // Ns, Ns, M).transpose(0, 2, 4, 1, 3, 5, 6)


def troubled_cells3d(ops, pde, v_old, u_cand, bc):
    """PAD and NAD (Sec. 1.6) on the subcell averages over the 3 x 3 x 3 cells."""
    C = u_cand.shape[:3]
    v_new = subcell_averages(ops, u_cand)
    vp = pad3d(v_old, bc)
    mn = np.full(C + (v_old.shape[-1],), np.inf)
    mx = np.full_like(mn, -np.inf)
    for ox in range(3):
        for oy in range(3):
            for oz in range(3):
                blk = vp[ox:ox + C[0], oy:oy + C[1], oz:oz + C[2]]
                mn = np.minimum(mn, blk.min(axis=(3, 4, 5)))
                mx = np.maximum(mx, blk.max(axis=(3, 4, 5)))
    delta = np.maximum(DELTA0, EPS0 * (mx - mn))
    lo, hi = (mn - delta)[:, :, :, None, None, None, :], (mx + delta)[:, :, :, None, None, None, :]
    nad = ((v_new >= lo) & (v_new <= hi)).all(axis=(3, 4, 5, 6))
    pad_ok = pde.admissible(v_new).all(axis=(3, 4, 5)) & pde.admissible(u_cand).all(axis=(3, 4, 5))
    return ~(nad & pad_ok)


def admissible_reconstruction3d(ops, pde, R, v):
    """u = (R (x) R (x) R) v [Ns, Ns, Ns, M] -> [n, n, n, M], scaled toward the
    mean (theta in {1, 1/2, ..., 2^-11}, else 0) until every subcell average
    and node is admissible."""
    u = np.einsum("is,jt,kq,stqr->ijkr", R, R, R, v)
    m = np.broadcast_to(v.mean(axis=(0, 1, 2)), u.shape)
    theta = 1.0
    for _ in range(12):
        cand = m + theta * (u - m)
        sub = np.einsum("si,tj,qk,ijkr->stqr", ops.P, ops.P, ops.P, cand)
        if pde.admissible(sub).all() and pde.admissible(cand).all():
            return cand
        theta *= 0.5
    return np.array(m)


def _correct(ops, pde, u_cand, bad, v_fv, Fsub, G, bc):
    C = u_cand.shape[:3]
    Ns = ops.Ns
    periodic = bc == "periodic"
    R = subcell_R(ops)
    u_new = u_cand.copy()
    for c in zip(*np.nonzero(bad)):
        u_new[c] = admissible_reconstruction3d(ops, pde, R, v_fv[c])
    p = ops.P / (Ns * ops.w[None, :])                       # [Ns, n]
    s0, s1 = ops.psi0 / ops.w, ops.psi1 / ops.w
    for d in range(3):
        a, b = [e for e in range(3) if e != d]
        shape = [1, 1, 1]
        shape[d] = -1
        for c in np.ndindex(*C):
            if not periodic and c[d] == C[d] - 1:
                continue
            c2 = list(c)
            c2[d] = (c[d] + 1) % C[d]
            c2 = tuple(c2)
            lb, rb = bad[c], bad[c2]
            if lb == rb:
                continue
            idx = [0, 0, 0]
            idx[d] = slice((c[d] + 2) * Ns - 1, (c[d] + 2) * Ns)
            idx[a] = slice((c[a] + 1) * Ns, (c[a] + 2) * Ns)
            idx[b] = slice((c[b] + 1) * Ns, (c[b] + 2) * Ns)
            Fs = Fsub[d][tuple(idx)]
            Fs = Fs.reshape(Ns, Ns, -1)                      # [s (axis a), t (axis b), M]
            Gp = np.einsum("sk,tl,str->klr", p, p, Fs) / Ns
            dG = Gp - G[d][c[0] + 1, c[1] + 1, c[2] + 1]     # [n (axis a), n (axis b), M]
            dGx = np.expand_dims(dG, axis=d)                 # node axis d inserted
            if not lb:
                u_new[c] -= s1.reshape(shape)[..., None] * dGx
            if not rb:
                u_new[c2] += s0.reshape(shape)[..., None] * dGx
    v_new = subcell_averages(ops, u_new)
    v_new[bad] = v_fv[bad]
    return u_new, v_new


def limited_step3d(ops, pde, u, dt, h, bc="periodic", nw=1, v=None, tol=1e-14, max_iter=64):
    """One 3-D ADER-DG step with a posteriori subcell ADER-WENO limiting.
    u [Cx, Cy, Cz, n, n, n, M]; v [Cx, Cy, Cz, Ns, Ns, Ns, M] or None (P u).
    Returns (u_new, troubled mask [Cx, Cy, Cz], v_new)."""
    Ns = ops.Ns
    if v is None:
        v = subcell_averages(ops, u)
    up = pad3d(u, bc)
    q, _, _ = predict3d(ops, pde, up, dt, h, tol, max_iter)
    u_cand = correct3d(ops, pde, up, q, dt, h)[1:-1, 1:-1, 1:-1]
    G = face_fluxes3d(ops, pde, q, dt, h)
    bad = troubled_cells3d(ops, pde, v, u_cand, bc)
    if not bad.any():
        return u_cand, bad, subcell_averages(ops, u_cand)
    sub = to_subgrid3(pad3d(v, bc))
    hs = tuple(x / Ns for x in h)
    with np.errstate(all="ignore"):
        s_ho, _, _, F_ho = fv3d_step(basis.build_operators(nw), pde, sub, dt, hs, tol, max_iter, fluxes=True)
    first_order = None
    for pss in range(PASSES):
        v_fv, Fsub = from_subgrid3(s_ho, Ns)[1:-1, 1:-1, 1:-1], F_ho
        if first_order is None and not pde.admissible(v_fv[bad]).all():
            with np.errstate(all="ignore"):
                first_order = fv3d_step(basis.build_operators(0), pde, sub, dt, hs, tol, max_iter, fluxes=True)
        if first_order is not None:
            v_fv, Fsub = from_subgrid3(first_order[0], Ns)[1:-1, 1:-1, 1:-1], first_order[3]
        u_new, v_new = _correct(ops, pde, u_cand, bad, v_fv, Fsub, G, bc)
        fails = ~bad & ~(pde.admissible(u_new).all(axis=(3, 4, 5)) & pde.admissible(v_new).all(axis=(3, 4, 5)))
        if pss == PASSES - 1 or not fails.any():
            return u_new, bad, v_new
        bad = bad | fails


def limited_run3d(ops, pde, u, extent=(2.0, 2.0, 2.0), cfl=0.4, nsteps=1, bc="periodic", nw=1, fixed_dt=None):
    """nsteps limited 3-D steps, dt by the DG rule of Sec. 1.5 with d = 3."""
    u = np.array(u, dtype=np.float64, copy=True)
    h = tuple(extent[d] / u.shape[d] for d in range(3))
    t, troubled, v = 0.0, [], None
    for _ in range(nsteps):
        dt = fixed_dt if fixed_dt else cfl_dt3d(ops, pde, u, h, cfl)
        u, bad, v = limited_step3d(ops, pde, u, dt, h, bc, nw, v)
        troubled.append(int(bad.sum()))
        t += dt
    return u, t, {"troubled": troubled, "v": v}
