"""A posteriori subcell finite-volume limiting of the 2-D ADER-DG step (Euler gas).

Sec. 1.4 (representation transformations) and Sec. 1.6 (admissibility
criteria) with d = 2; the construction of the one-dimensional limiter of this
oracle (module `limiter`), taken per direction:

  * the 2-D ADER-DG step (module `dg2d`) gives a candidate u*;
  * the candidate is checked in the subcell representation v = (P (x) P) u,
    N_s = 2N+1 subcells per direction (Sec. 1.4, the projection applied per
    direction):
      PAD: every subcell average and every node of u* physically admissible
           (rho > 0, internal energy > 0);
      NAD: eq. nad_ineq per component, min over V_i of v^n - delta <= v* <=
           max over V_i of v^n + delta, delta = max(delta_0, eps_0 (max - min)),
           delta_0 = 1e-4, eps_0 = 1e-3.  Reading: V_i is the cell and the
           eight cells that share a vertex with it (the Voronoi neighbours of
           a cell of a Cartesian mesh);
  * a troubled cell is recomputed by the 2-D ADER-WENO scheme (module `fv2d`,
    reconstruction of degree nw) on its subgrid, from v^n, with the DG step's
    dt, and returns to the DG representation by u = (R (x) R) v, R the
    pseudo-inverse of P (the pseudo-inverse of a Kronecker product is the
    Kronecker product of the pseudo-inverses), scaled toward its mean when
    that polynomial would leave the admissible set (as in one dimension);
  * conservation at a face between a troubled and an admissible cell (the
    one-dimensional reading, per face node): the admissible cell's surface
    term takes, in place of its DG flux at face node k, the subgrid fluxes
    F_s of the N_s sub-faces of that face projected onto the nodal basis
    along the face,
        G_k = sum_s F_s (integral of phi_k over sub-face s) / (N_s w_k),
    whose nodal quadrature sum_k w_k G_k is the face's total subgrid flux
    (sum_k phi_k = 1), so that every face carries one flux and the totals
    telescope.  For fluxes that do not vary along the face this is the
    one-dimensional exchange.

The subgrid scheme runs on the whole mesh's subgrid (cells left unlimited
take no part in the result); when it leaves the admissible set in a troubled
cell, it is redone at first order (reconstruction and predictor of degree 0),
as in one dimension.  The exchange changes unlimited cells after their
detection, so the detection and correction cascade (the a posteriori loop
repeated while a corrected state fails the checks, reading): an unlimited
cell whose corrected state fails PAD joins the troubled cells and the
correction is redone, three passes at most.

Boundaries: periodic, or transmissive (free outflow, Sec. 2.2): one ghost cell
on every side, the mirror image of the boundary cell (nodes, or subcells, in
reversed order along the face normal, no sign change; corners mirrored in
both directions).  The scheme is evaluated on the padded mesh taken as
periodic; ghost results are discarded.  With periodic boundaries the ghosts
are the periodic images, and the results are those of the periodic mesh.
Test infrastructure only.
"""

import numpy as np

from . import basis
from .dg2d import correct2d, face_fluxes2d, predict2d, subcell_averages, cfl_dt2d
from .fv2d import fv2d_step
from .limiter import DELTA0, EPS0, subcell_R


def pad2d(a, bc):
    """One ghost cell on every side of per-cell data a[Cx, Cy, k, l, ...] whose
    axes 2 and 3 run along x and y inside the cell (DG nodes or subcells)."""
    if bc == "periodic":
        a = np.concatenate([a[-1:], a, a[:1]], axis=0)
        return np.concatenate([a[:, -1:], a, a[:, :1]], axis=1)
    a = np.concatenate([a[:1, :, ::-1], a, a[-1:, :, ::-1]], axis=0)
    return np.concatenate([a[:, :1, :, ::-1], a, a[:, -1:, :, ::-1]], axis=1)


def to_subgrid(v):
    """[Cx, Cy, Ns, Ns, M] subcell averages -> the subgrid [Cx Ns, Cy Ns, M]."""
    Cx, Cy, Ns, _, M = v.shape
    return v.transpose(0, 2, 1, 3, 4).reshape(Cx * Ns, Cy * Ns, M)


def from_subgrid(s, Ns):
    X, Y, M = s.shape
    return s.reshape(X // Ns, Ns, Y // Ns, Ns, M).transpose(0, 2, 1, 3, 4)


def face_projection(ops):
    """proj[s, k] = (integral over sub-face s of phi_k) / (N_s w_k), from the
    subcell-average operator P[s, k] = N_s * that integral (Sec. 1.4)."""
    return ops.P / (ops.Ns * ops.Ns * ops.w[None, :])


def troubled_cells2d(ops, pde, v_old, u_cand, bc):
    """PAD and NAD (Sec. 1.6) on the subcell averages: True where the
    candidate u_cand [Cx, Cy, n, n, M] is not admissible; v_old
    [Cx, Cy, Ns, Ns, M] are the subcell averages of the step's start."""
    Cx, Cy = u_cand.shape[:2]
    v_new = subcell_averages(ops, u_cand)
    vp = pad2d(v_old, bc)                         # mirrored ghosts: the same extrema as the cell
    mn = np.full((Cx, Cy, v_old.shape[-1]), np.inf)
    mx = np.full_like(mn, -np.inf)
    for ox in range(3):
        for oy in range(3):
            blk = vp[ox:ox + Cx, oy:oy + Cy]
            mn = np.minimum(mn, blk.min(axis=(2, 3)))
            mx = np.maximum(mx, blk.max(axis=(2, 3)))
    delta = np.maximum(DELTA0, EPS0 * (mx - mn))
    lo, hi = (mn - delta)[:, :, None, None, :], (mx + delta)[:, :, None, None, :]
    nad = ((v_new >= lo) & (v_new <= hi)).all(axis=(2, 3, 4))
    pad_ok = pde.admissible(v_new).all(axis=(2, 3)) & pde.admissible(u_cand).all(axis=(2, 3))
    return ~(nad & pad_ok)


def admissible_reconstruction2d(ops, pde, R, v):
    """u = (R (x) R) v for one cell [Ns, Ns, M] -> [n, n, M], scaled toward
    the cell mean (u = m + theta (R v - m), the largest theta in {1, 1/2, ...,
    2^-11, 0}) until every subcell average and node is admissible."""
    u = np.einsum("is,jt,str->ijr", R, R, v)
    m = np.broadcast_to(v.mean(axis=(0, 1)), u.shape)
    theta = 1.0
    for _ in range(12):
        cand = m + theta * (u - m)
        sub = np.einsum("si,tj,ijr->str", ops.P, ops.P, cand)
        if pde.admissible(sub).all() and pde.admissible(cand).all():
            return cand
        theta *= 0.5
    return np.array(m)


PASSES = 3


def limited_step2d(ops, pde, u, dt, dx, dy, bc="periodic", nw=1, v=None, tol=1e-14, max_iter=64):
    """One 2-D ADER-DG step with a posteriori subcell ADER-WENO limiting.

    u [Cx, Cy, n, n, M]; v [Cx, Cy, Ns, Ns, M] the subcell averages at the
    step's start (P u for a cell the previous step left unlimited, its
    finite-volume averages for a cell it limited; None: (P (x) P) u).
    Returns (u_new, troubled mask [Cx, Cy], v_new).

    Detection and correction cascade (reading: the a posteriori limiting
    loop is repeated while a corrected state fails the checks): an unlimited
    cell whose state after the flux exchange fails PAD (nodes or subcell
    averages) joins the troubled cells and the correction is redone, at most
    PASSES times in all."""
    Cx, Cy, n, _, M = u.shape
    Ns = ops.Ns
    if v is None:
        v = subcell_averages(ops, u)
    up = pad2d(u, bc)
    q, _, _ = predict2d(ops, pde, up, dt, dx, dy, tol, max_iter)
    u_cand = correct2d(ops, pde, up, q, dt, dx, dy)[1:-1, 1:-1]
    Gx, Gy = face_fluxes2d(ops, pde, q, dt, dx, dy)        # east / north faces of the padded cells
    bad = troubled_cells2d(ops, pde, v, u_cand, bc)
    if not bad.any():
        return u_cand, bad, subcell_averages(ops, u_cand)
    sub = to_subgrid(pad2d(v, bc))
    with np.errstate(all="ignore"):
        s_ho, _, _, Fx_ho, Fy_ho = fv2d_step(basis.build_operators(nw), pde, sub, dt, dx / Ns, dy / Ns,
                                             tol, max_iter, fluxes=True)
    first_order = None
    for p in range(PASSES):
        v_fv, Fx, Fy = from_subgrid(s_ho, Ns)[1:-1, 1:-1], Fx_ho, Fy_ho
        if first_order is None and not pde.admissible(v_fv[bad]).all():
            # first order on the whole subgrid (degree-0 reconstruction and predictor)
            first_order = fv2d_step(basis.build_operators(0), pde, sub, dt, dx / Ns, dy / Ns,
                                    tol, max_iter, fluxes=True)
        if first_order is not None:
            v_fv, Fx, Fy = from_subgrid(first_order[0], Ns)[1:-1, 1:-1], first_order[3], first_order[4]
        u_new, v_new = _correct(ops, pde, u_cand, bad, v_fv, Fx, Fy, Gx, Gy, bc)
        fails = ~bad & ~(pde.admissible(u_new).all(axis=(2, 3)) & pde.admissible(v_new).all(axis=(2, 3)))
        if p == PASSES - 1 or not fails.any():
            return u_new, bad, v_new
        bad = bad | fails


def _correct(ops, pde, u_cand, bad, v_fv, Fx, Fy, Gx, Gy, bc):
    """The corrected state of one pass: (R (x) R) v_fv in the troubled cells,
    the candidate with the exchanged face fluxes elsewhere; and its subcell
    averages (the finite-volume ones in the troubled cells)."""
    Cx, Cy = u_cand.shape[:2]
    Ns = ops.Ns
    periodic = bc == "periodic"
    R = subcell_R(ops)
    u_new = u_cand.copy()
    for ix, iy in zip(*np.nonzero(bad)):
        u_new[ix, iy] = admissible_reconstruction2d(ops, pde, R, v_fv[ix, iy])
    proj = face_projection(ops)
    s0, s1 = (ops.psi0 / ops.w), (ops.psi1 / ops.w)
    # x faces: between interior cells ix and ix+1 (padded p = ix+1 and p+1);
    # with transmissive boundaries the two boundary faces have no second cell
    for ix in range(Cx if periodic else Cx - 1):
        jx = (ix + 1) % Cx
        X = (ix + 2) * Ns - 1                                  # the last subcell column of padded cell ix+1
        for iy in range(Cy):
            lb, rb = bad[ix, iy], bad[jx, iy]
            if lb == rb:
                continue
            Fs = Fx[X, (iy + 1) * Ns:(iy + 2) * Ns]             # [Ns, M], subcell units
            dG = proj.T @ Fs - Gx[ix + 1, iy + 1]                # [n (y node), M]
            if not lb:
                u_new[ix, iy] -= s1[:, None, None] * dG[None, :, :]
            if not rb:
                u_new[jx, iy] += s0[:, None, None] * dG[None, :, :]
    # y faces: between interior cells iy and iy+1
    for iy in range(Cy if periodic else Cy - 1):
        jy = (iy + 1) % Cy
        Y = (iy + 2) * Ns - 1
        for ix in range(Cx):
            lb, rb = bad[ix, iy], bad[ix, jy]
            if lb == rb:
                continue
            Fs = Fy[(ix + 1) * Ns:(ix + 2) * Ns, Y]
            dG = proj.T @ Fs - Gy[ix + 1, iy + 1]                # [n (x node), M]
            if not lb:
                u_new[ix, iy] -= s1[None, :, None] * dG[:, None, :]
            if not rb:
                u_new[ix, jy] += s0[None, :, None] * dG[:, None, :]
    v_new = subcell_averages(ops, u_new)
    v_new[bad] = v_fv[bad]
    return u_new, v_new


def limited_run2d(ops, pde, u, extent=(0.0, 1.0, 0.0, 1.0), cfl=0.4, t_end=np.inf, nsteps=None,
                  bc="periodic", nw=1, fixed_dt=None):
    """Limited 2-D steps to t_end (or nsteps), dt by the DG rule of Sec. 1.5
    with d = 2 (module `dg2d`).  Returns (u, t, info)."""
    u = np.array(u, dtype=np.float64, copy=True)
    Cx, Cy = u.shape[:2]
    x0, x1, y0, y1 = extent
    dx, dy = (x1 - x0) / Cx, (y1 - y0) / Cy
    t, steps, troubled, v = 0.0, 0, [], None
    while (nsteps is None or steps < nsteps) and t < t_end:
        dt = fixed_dt if fixed_dt else cfl_dt2d(ops, pde, u, dx, dy, cfl)
        dt = min(dt, t_end - t)
        if dt <= 0:
            break
        u, bad, v = limited_step2d(ops, pde, u, dt, dx, dy, bc, nw, v)
        troubled.append(int(bad.sum()))
        t += dt
        steps += 1
    return u, t, {"steps": steps, "troubled": troubled, "v": v}
