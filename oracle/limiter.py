"""A posteriori subcell finite-volume limiting of the ADER-DG step (1-D).

Sec. 1.4 (representation transformations) and Sec. 1.6 (admissibility
criteria), in one space dimension:

  * the ADER-DG step gives a candidate u* (Sec. 1.6);
  * the candidate is checked in the subcell representation v = P u with
    N_s = 2N+1 subcells (Sec. 1.4, eq. p_operator and the formula of P):
      PAD: the physical admissibility of every subcell average (Euler: rho > 0,
           internal energy > 0);
      NAD: eq. nad_ineq, per component: min over V_i of v^n - delta <= v* <=
           max over V_i of v^n + delta, V_i = the cell and its two neighbours,
           delta = max(delta_0, eps_0 (max - min)), delta_0 = 1e-4,
           eps_0 = 1e-3 (Sec. 1.6);
  * a troubled cell is recomputed by the finite-volume ADER-WENO scheme
    (Sec. 1.3, WENO of degree nw) on its subgrid of N_s subcells, from
    v^n = P u^n, with the DG step's dt (with N_s = 2N+1 it is the finite-volume CFL step of the
    subgrid, Sec. 1.5), and returns to the DG representation by u = R v,
    R the pseudo-inverse of P (Sec. 1.4: R P = 1);
  * conservation at the faces between a troubled and an admissible cell: the
    admissible cell's update takes the subgrid flux through that face in place
    of its DG flux (reading: the paper does not say how the two fluxes meet;
    with this exchange every face carries one flux and the totals telescope).

Boundaries: periodic, or transmissive (free outflow, Sec. 2.2): a ghost cell
is the mirror image of the boundary cell (nodal values in reversed order, no
sign change), so the Riemann problem at the boundary face has equal states.
The scheme is evaluated on a padded periodic mesh whose ghost cells are
refreshed every step; ghost results are discarded.

Limiter readings: the paper names ADER-WENO2 as the limiter of its Riemann
tests, and its ADER-WENO(N+1) naming (the WENO timing tables of Sec. 3) makes
that the reconstruction of degree 1 (nw = 1, the default); nw = 2 gives
ADER-WENO3.  When the subgrid step leaves the admissible
set in a troubled cell, the subgrid step is redone at first order (degree 0);
a limited cell's polynomial R v is scaled toward its mean when its subcell
averages would leave the admissible set (admissible_reconstruction).  The
paper's limiter sections do not discuss either safeguard.  Test
infrastructure only.
"""

import numpy as np

from . import basis
from .dg import cfl_lambda, dg_correct, interface_terms
from .fv import fv_step_terms
from .predictor import predict

DELTA0 = 1.0e-4
EPS0 = 1.0e-3


def subcell_R(ops):
    """Pseudo-inverse of P (n x N_s): R = (P^T P)^-1 P^T, so that R P = 1."""
    return np.linalg.solve(ops.P.T @ ops.P, ops.P.T)


def mirror_pad_cells(u, g):
    """Pad [C, n, M] DG data with g transmissive ghost cells per side."""
    left = [u[k][::-1] for k in range(g - 1, -1, -1)]
    right = [u[-1 - k][::-1] for k in range(g)]
    return np.concatenate([np.array(left), u, np.array(right)], axis=0)


def mirror_pad_averages(v, g):
    """Pad [C, M] finite-volume averages with g mirrored ghost averages per side."""
    return np.concatenate([v[g - 1::-1], v, v[:-g - 1:-1]], axis=0)


def pad(u, g, bc, dg=True):
    if bc == "periodic":
        return np.concatenate([u[-g:], u, u[:g]], axis=0)
    return mirror_pad_cells(u, g) if dg else mirror_pad_averages(u, g)


def admissible_reconstruction(ops, pde, R, v):
    """u = R v for one cell (Sec. 1.4), scaled toward the cell mean when needed:
    P R v is not v when N_s > N+1 (Sec. 1.4), and its subcell averages, which
    the next step's detectors and subgrid start from, may leave the admissible
    set although v is in it.  Reading: u = m + theta (R v - m), m the mean of v,
    with the largest theta in {1, 1/2, 1/4, ..., 0} for which every subcell
    average and node of u is admissible; theta = 0 (the mean) always is, for an
    admissible v and a convex admissible set.  The mean is kept exactly."""
    u = R @ v
    m = np.broadcast_to(v.mean(axis=0), u.shape)
    theta = 1.0
    for _ in range(12):
        cand = m + theta * (u - m)
        if pde.admissible(ops.P @ cand).all() and pde.admissible(cand).all():
            return cand
        theta *= 0.5
    return np.array(m)


def dg_candidate(ops, pde, u, t, dt, dx, x0, bc, tol=1e-14, max_iter=64):
    """The unlimited ADER-DG step with the boundary condition, and the
    time-integrated face fluxes Gbar [C+1, M] (face i-1/2 of cell i, then the
    right face of the last cell) it used."""
    C = u.shape[0]
    up = pad(u, 1, bc)
    x_left = x0 + dx * (np.arange(C + 2) - 1)
    q, _, failed = predict(ops, pde, up, dt, dx, x_left, t, tol, max_iter)
    un = dg_correct(ops, pde, up, q, dt, dx, x_left, t)[1:-1]
    Gbar, _ = interface_terms(ops, pde, q, dt, dx)           # right face of every padded cell
    return un, Gbar[0:C + 1], failed[1:-1]


def fv_subgrid(ops_fv, pde, v, t, dt, dxs, x0, bc, tol=1e-14, max_iter=64):
    """One ADER-WENO-FV step on the subgrid averages v [S, M] with the boundary
    condition; returns (v_new [S, M], face fluxes [S+1, M] in subcell units)."""
    S = v.shape[0]
    g = ops_fv.N + 2
    vp = pad(v, g, bc, dg=False)
    x_left = x0 + dxs * (np.arange(S + 2 * g) - g)
    v_new, Gbar = fv_step_terms(ops_fv, pde, vp, t, dt, dxs, x_left, tol, max_iter)
    return v_new[g:g + S], Gbar[g - 1:g + S]


def troubled_cells(ops, pde, v_old, u_cand, bc):
    """PAD and NAD (Sec. 1.6) on the subcell averages: True where the candidate
    u_cand [C, n, M] is not admissible; v_old [C, N_s, M] are the subcell
    averages of the step's start."""
    v_new = np.einsum("sk,ckr->csr", ops.P, u_cand)
    vp = pad(v_old, 1, bc) if bc == "periodic" else np.concatenate([v_old[:1], v_old, v_old[-1:]], axis=0)
    win = np.concatenate([vp[:-2], vp[1:-1], vp[2:]], axis=1)        # [C, 3 Ns, M]: V_i
    mn, mx = win.min(axis=1), win.max(axis=1)
    delta = np.maximum(DELTA0, EPS0 * (mx - mn))
    nad = ((v_new >= (mn - delta)[:, None, :]) & (v_new <= (mx + delta)[:, None, :])).all(axis=(1, 2))
    pad_ok = pde.admissible(v_new).all(axis=1) & pde.admissible(u_cand).all(axis=1)
    return ~(nad & pad_ok)


def subcell_averages(ops, u):
    """v = P u for every cell: [C, n, M] -> [C, N_s, M] (Sec. 1.4, eq. p_operator)."""
    return np.einsum("sk,ckr->csr", ops.P, u)


def limited_step(ops, pde, u, t, dt, dx, x0, bc="periodic", nw=1, v=None, tol=1e-14, max_iter=64):
    """One ADER-DG step with a posteriori subcell ADER-WENO limiting.

    v [C, N_s, M] are the subcell averages at the step's start: P u for a cell
    the previous step left unlimited, the finite-volume averages it computed
    for a cell it limited (reading, after the subcell method the paper builds
    on: a limited cell keeps its subcell data, so that P R v, which is not v,
    never feeds the detectors or the subgrid scheme).  None means P u.
    Returns (u_new, troubled mask [C], v_new [C, N_s, M])."""
    C, n, M = u.shape
    Ns = ops.Ns
    if v is None:
        v = subcell_averages(ops, u)
    u_cand, G_dg, _ = dg_candidate(ops, pde, u, t, dt, dx, x0, bc, tol, max_iter)
    bad = troubled_cells(ops, pde, v, u_cand, bc)
    if not bad.any():
        return u_cand, bad, subcell_averages(ops, u_cand)
    v = v.reshape(C * Ns, M)
    with np.errstate(all="ignore"):
        v_fv, g_fv = fv_subgrid(basis.build_operators(nw), pde, v, t, dt, dx / Ns, x0, bc, tol, max_iter)
    sub_bad = np.repeat(bad, Ns)
    if not pde.admissible(v_fv[sub_bad]).all():
        # the subgrid scheme left the admissible set in a troubled cell: the
        # whole subgrid step falls back to first order (reconstruction and
        # predictor of degree 0: the Rusanov finite-volume scheme, positive at
        # the subgrid Courant number CFL <= 1/2), so every face keeps one flux
        v_fv, g_fv = fv_subgrid(basis.build_operators(0), pde, v, t, dt, dx / Ns, x0, bc, tol, max_iter)
    R = subcell_R(ops)
    u_new = u_cand.copy()
    for i in np.nonzero(bad)[0]:
        u_new[i] = admissible_reconstruction(ops, pde, R, v_fv[i * Ns:(i + 1) * Ns])
    # one flux per face: the subgrid flux wherever a troubled cell touches the face
    G_fv = g_fv[::Ns] / Ns                                            # cell faces, cell-mean units
    w, psi0, psi1 = ops.w, ops.psi0, ops.psi1
    periodic = bc == "periodic"
    for f in range(C if periodic else C + 1):                         # face f: between cells f-1 and f
        lc = (f - 1) % C if periodic else (f - 1 if f >= 1 else None)
        rc = f if f < C else None
        left_bad = lc is not None and bad[lc]
        right_bad = rc is not None and bad[rc]
        if not (left_bad or right_bad):
            continue
        dG = G_fv[f] - G_dg[f]
        if lc is not None and not left_bad:                           # its right face
            u_new[lc] -= (psi1 / w)[:, None] * dG[None, :]
        if rc is not None and not right_bad:                          # its left face
            u_new[rc] += (psi0 / w)[:, None] * dG[None, :]
    v_new = subcell_averages(ops, u_new)
    v_new[bad] = v_fv.reshape(C, Ns, M)[bad]
    return u_new, bad, v_new


def limited_run(ops, pde, u, x0, x1, cfl=0.4, t_end=np.inf, nsteps=None, bc="periodic", nw=1, dims=1):
    """Limited ADER-DG steps to t_end (or nsteps).  The step is the CFL
    condition of Sec. 1.5, dt = CFL / d / (2N+1) * h / |lambda_max|; dims
    gives d: the Riemann tests of Sec. 2.2 run on a two-dimensional mesh,
    so their step carries d = 2 although the flow is one-dimensional."""
    u = np.array(u, dtype=np.float64, copy=True)
    C = u.shape[0]
    dx = (x1 - x0) / C
    t, steps, troubled, v = 0.0, 0, [], None
    while (nsteps is None or steps < nsteps) and t < t_end:
        dt = min(cfl / dims * dx / ((2 * ops.N + 1) * cfl_lambda(ops, pde, u)), t_end - t)
        if dt <= 0:
            break
        u, bad, v = limited_step(ops, pde, u, t, dt, dx, x0, bc, nw, v)
        troubled.append(int(bad.sum()))
        t += dt
        steps += 1
    return u, t, {"steps": steps, "troubled": troubled, "v": v}
