"""Pins of the oracle's 2-D a posteriori subcell limiter (Sec. 1.4 and 1.6 with
d = 2, module oracle/limiter2d.py).

* The face projection of the subgrid fluxes equals the integrals of the nodal
  basis over the sub-faces, by brute-force quadrature (independent of P).
* Data that vary along x only (a Table 9 Riemann problem with free outflow,
  constant along y): the 2-D limited step equals the pinned 1-D limited step
  on (rho, rho u, E) row by row, with the same troubled cells, over two steps
  (the subcell data of limited cells carried between the steps); rho v stays
  zero.  The same along y after exchanging the axes.  This covers the
  candidate, the detectors, the subgrid scheme, R and the flux exchange at
  faces normal to x (resp. y).
* The cylindrical explosion of Sec. 2.2 with periodic boundaries, where the
  troubled cells line a circle: the totals of all four variables are kept to
  rounding (the exchange gives every face one flux, along both directions and
  with fluxes that vary along the face), the troubled cells keep the symmetry
  x <-> y of the data at every step, and the states stay admissible.  The
  state itself keeps that symmetry to rounding after the first step only:
  the dimension-by-dimension reconstruction (x, then y) does not commute
  with the exchange of the axes once its nonlinear weights differ along the
  two directions (3.5e-5 between the two orders on the data of the third
  step, N = 2 on 10^2 cells).
* A uniform state is kept and no cell is troubled.
* The detection / correction cascade adds a cell whose corrected state fails
  PAD (control flow only: its physics is parity unpinned, since no small
  configuration triggers it; the GPU's 41^2 explosion at N = 8 does).
"""

import numpy as np
import pytest

from oracle import basis, dg2d, limiter, limiter2d
from oracle import pde as OP
from paper_2409_12483_amd import workloads as W

E1, E2 = OP.Euler(), dg2d.Euler2D()


@pytest.mark.parametrize("N", [1, 2, 5])
def test_face_projection_is_the_subface_integral(N):
    ops = basis.build_operators(N)
    Ns = ops.Ns
    proj = limiter2d.face_projection(ops)
    m = 4000                                                     # midpoints per sub-face
    for s in range(Ns):
        y = (s + (np.arange(m) + 0.5) / m) / Ns
        integral = basis.lagrange_eval(ops.xi, y).mean(axis=0) / Ns        # [n]
        assert np.abs(proj[s] - integral / (Ns * ops.w)).max() <= 1e-7
    # the nodal quadrature of the projected fluxes is the sum of the sub-face fluxes
    F = np.random.default_rng(N).uniform(-1, 1, (Ns, 4))
    assert np.abs(ops.w @ (proj.T @ F) - F.sum(axis=0) / Ns ** 2).max() <= 1e-14


def _rows(u1, Cy):
    """1-D state [C, n, 3] -> 2-D [C, Cy, n, n, 4] constant along y."""
    C, n, _ = u1.shape
    u2 = np.zeros((C, Cy, n, n, 4))
    u2[..., 0] = u1[:, None, :, None, 0]
    u2[..., 1] = u1[:, None, :, None, 1]
    u2[..., 3] = u1[:, None, :, None, 2]
    return u2


def _swap(u):
    """Exchange the x and y axes (cells, nodes) and the two momenta."""
    return np.ascontiguousarray(np.swapaxes(np.swapaxes(u, 0, 1), 2, 3)[..., [0, 2, 1, 3]])


@pytest.mark.parametrize("N,test", [(2, 1), (3, 3)])
def test_reduces_to_the_1d_limiter(N, test):
    ops = basis.build_operators(N)
    C, Cy = 24, 3
    dx, dy = 1.0 / C, 0.7 / Cy
    u1 = W.riemann_nodal(C, N, test)
    u2 = _rows(u1, Cy)
    dt = 0.4 / 2 / (2 * N + 1) * dx / 3.0
    v1 = v2 = None
    any_bad = False
    for _ in range(2):
        u1, bad1, v1 = limiter.limited_step(ops, E1, u1, 0.0, dt, dx, 0.0, "transmissive", 1, v1)
        u2, bad2, v2 = limiter2d.limited_step2d(ops, E2, u2, dt, dx, dy, "transmissive", 1, v2)
        any_bad |= bool(bad1.any())
        assert (bad2 == bad1[:, None]).all()
        scale = np.abs(u1).max()
        assert np.abs(u2[..., [0, 1, 3]] - u1[:, None, :, None, :]).max() <= 1e-12 * scale
        assert np.abs(u2[..., 2]).max() <= 1e-14 * scale
    assert any_bad
    # the same flow along y
    u1 = W.riemann_nodal(C, N, test)
    uy = _swap(_rows(u1, Cy))
    ux, _, _ = limiter2d.limited_step2d(ops, E2, _rows(u1, Cy), dt, dx, dy, "transmissive")
    gy, bady, _ = limiter2d.limited_step2d(ops, E2, uy, dt, dy, dx, "transmissive")
    assert bady.any()
    assert np.abs(_swap(gy) - ux).max() <= 1e-12 * np.abs(ux).max()


def _explosion(C, N):
    return W.euler2d_explosion_nodal(C, C, N)


@pytest.mark.parametrize("N,C", [(2, 10), (3, 8)])
def test_explosion_conservation_symmetry_admissibility(N, C):
    ops = basis.build_operators(N)
    u0 = _explosion(C, N)
    h = 2.0 / C
    u, v = u0, None
    for k in range(4):
        dt = dg2d.cfl_dt2d(ops, E2, u, h, h, 0.4)
        u, bad, v = limiter2d.limited_step2d(ops, E2, u, dt, h, h, "periodic", 1, v)
        assert bad.any() and (bad == bad.T).all()
        if k == 0:
            assert np.abs(_swap(u) - u).max() <= 1e-13 * np.abs(u).max()
        assert E2.admissible(u).all()
        assert E2.admissible(dg2d.subcell_averages(ops, u)).all()
    tot0 = dg2d.conserved_totals2d(ops, u0, h, h)
    tot = dg2d.conserved_totals2d(ops, u, h, h)
    assert np.abs(tot - tot0).max() <= 1e-12 * np.abs(tot0).max()


def test_explosion_with_free_outflow_runs_admissibly():
    N, C = 2, 10
    ops = basis.build_operators(N)
    u, t, info = limiter2d.limited_run2d(ops, E2, _explosion(C, N), extent=(-1, 1, -1, 1), nsteps=6,
                                         bc="transmissive")
    assert info["steps"] == 6 and min(info["troubled"]) > 0
    assert E2.admissible(u).all()


def test_uniform_state_is_kept():
    N = 3
    ops = basis.build_operators(N)
    u0 = np.tile([1.2, 0.3, -0.2, 2.9], (6, 5, N + 1, N + 1, 1))
    for bc in ("periodic", "transmissive"):
        u, bad, _ = limiter2d.limited_step2d(ops, E2, u0, 0.01, 0.2, 0.2, bc)
        assert not bad.any()
        assert np.abs(u - u0).max() <= 1e-13


def _nad_case(rho_centre):
    """5^2 cells, N = 1: every subcell at the base state except the cell
    diagonal to the centre, at rho = 2; the centre's candidate at rho_centre."""
    N = 1
    ops = basis.build_operators(N)
    base = np.array([1.0, 0.0, 0.0, 2.5])
    v_old = np.tile(base, (5, 5, ops.Ns, ops.Ns, 1))
    v_old[1, 1, ..., 0] = 2.0
    cand = np.tile(base, (5, 5, N + 1, N + 1, 1))
    cand[1, 1, ..., 0] = 2.0
    cand[2, 2, ..., 0] = rho_centre
    return limiter2d.troubled_cells2d(ops, E2, v_old, cand, "periodic")


def test_nad_takes_the_vertex_neighbours():
    """V_i holds the cells that share a vertex with cell i: a candidate between
    the bounds that only a diagonal neighbour sets is admissible."""
    assert not _nad_case(1.5).any()
    bad = _nad_case(2.5)
    assert bad[2, 2] and bad.sum() == 1


def test_reconstruction_is_scaled_into_the_admissible_set():
    """Subcell averages with a near-vacuum corner (N = 5: (R (x) R) v
    undershoots to a density of -0.23 at a node); the returned polynomial is
    admissible at every node and subcell and keeps the cell mean."""
    N = 5
    ops = basis.build_operators(N)
    Ns = ops.Ns
    v = np.tile([1.0, 0.0, 0.0, 2.5], (Ns, Ns, 1))
    v[0, 0] = [1e-3, 0.0, 0.0, 2.5e-3]
    R = limiter.subcell_R(ops)
    plain = np.einsum("is,jt,str->ijr", R, R, v)
    assert not E2.admissible(plain).all()
    u = limiter2d.admissible_reconstruction2d(ops, E2, R, v)
    sub = np.einsum("si,tj,ijr->str", ops.P, ops.P, u)
    assert E2.admissible(u).all() and E2.admissible(sub).all()
    assert np.abs(np.einsum("i,j,ijr->r", ops.w, ops.w, u) - v.mean(axis=(0, 1))).max() <= 1e-14


def test_cascade_adds_cells_that_fail_after_the_exchange(monkeypatch):
    """The detection / correction cascade: an unlimited cell whose corrected
    state fails PAD joins the troubled cells and the correction is redone
    with it (control flow, with a corrected state made to fail once: no small
    configuration of the explosion triggers the cascade within 40 steps)."""
    N, C = 2, 10
    ops = basis.build_operators(N)
    u0 = _explosion(C, N)
    h = 2.0 / C
    dt = dg2d.cfl_dt2d(ops, E2, u0, h, h, 0.4)
    _, bad0, _ = limiter2d.limited_step2d(ops, E2, u0, dt, h, h, "periodic")
    target = (0, 0)
    assert not bad0[target]
    real, calls = limiter2d._correct, []

    def failing_once(ops_, pde, u_cand, bad, *rest):
        calls.append(bad.copy())
        u_new, v_new = real(ops_, pde, u_cand, bad, *rest)
        if len(calls) == 1:
            v_new = v_new.copy()
            v_new[target][0, 0, 0] = -1.0                 # a negative density after the exchange
        return u_new, v_new

    monkeypatch.setattr(limiter2d, "_correct", failing_once)
    _, bad1, _ = limiter2d.limited_step2d(ops, E2, u0, dt, h, h, "periodic")
    assert len(calls) == 2 and bad1[target] and (bad1 == (bad0 | (np.arange(C)[:, None] == 0)
                                                          & (np.arange(C)[None, :] == 0))).all()
    assert not calls[0][target] and calls[1][target]


# ------------------------------------------------------ planted mistakes ----
def _pins():
    ok = []
    try:
        test_face_projection_is_the_subface_integral(2)
        ok.append("projection")
    except AssertionError:
        pass
    for name, fn in (("reduce", lambda: test_reduces_to_the_1d_limiter(2, 1)),
                     ("explosion", lambda: test_explosion_conservation_symmetry_admissibility(2, 10)),
                     ("nad", test_nad_takes_the_vertex_neighbours), ("uniform", test_uniform_state_is_kept),
                     ("scaling", test_reconstruction_is_scaled_into_the_admissible_set)):
        try:
            with np.errstate(all="ignore"):
                fn()
            ok.append(name)
        except (AssertionError, FloatingPointError, ValueError, IndexError):
            pass
    return ok


def _no_weight_projection(ops):
    return ops.P / (ops.Ns * ops.Ns)


def _ns_projection(ops):
    return ops.P / (ops.Ns * ops.w[None, :])


def _five_point_nad(ops, pde, v_old, u_cand, bc):
    Cx, Cy = u_cand.shape[:2]
    v_new = dg2d.subcell_averages(ops, u_cand)
    vp = limiter2d.pad2d(v_old, bc)
    mn = np.full((Cx, Cy, v_old.shape[-1]), np.inf)
    mx = np.full_like(mn, -np.inf)
    for ox, oy in ((1, 1), (0, 1), (2, 1), (1, 0), (1, 2)):
        blk = vp[ox:ox + Cx, oy:oy + Cy]
        mn, mx = np.minimum(mn, blk.min(axis=(2, 3))), np.maximum(mx, blk.max(axis=(2, 3)))
    delta = np.maximum(limiter2d.DELTA0, limiter2d.EPS0 * (mx - mn))
    nad = ((v_new >= (mn - delta)[:, :, None, None]) & (v_new <= (mx + delta)[:, :, None, None])).all(axis=(2, 3, 4))
    return ~(nad & pde.admissible(v_new).all(axis=(2, 3)) & pde.admissible(u_cand).all(axis=(2, 3)))


def _plain_reconstruction(ops, pde, R, v):
    return np.einsum("is,jt,str->ijr", R, R, v)


def _transposed_R(ops):
    return ops.P.T / ops.Ns


def _periodic_ghosts(a, bc):
    a = np.concatenate([a[-1:], a, a[:1]], axis=0)
    return np.concatenate([a[:, -1:], a, a[:, :1]], axis=1)


MUTATIONS = {
    "projection without 1/w_k": ("face_projection", _no_weight_projection),
    "projection scaled by 1/N_s": ("face_projection", _ns_projection),
    "V_i without the diagonal cells": ("troubled_cells2d", _five_point_nad),
    "reconstruction without the admissibility scaling": ("admissible_reconstruction2d", _plain_reconstruction),
    "R = P^T / N_s": ("subcell_R", _transposed_R),
    "periodic ghosts for free outflow": ("pad2d", _periodic_ghosts),
}


def test_unmutated_oracle_passes_every_pin():
    assert _pins() == ["projection", "reduce", "explosion", "nad", "uniform", "scaling"]


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_breaks_a_pin(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(limiter2d, attr, fn)
    assert len(_pins()) < 6, name
