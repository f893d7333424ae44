"""Pins of the oracle's 3-D a posteriori subcell limiter (Sec. 1.4 and 1.6 with
d = 3, module oracle/limiter3d.py).

* Data constant along one axis (the cylindrical explosion of Sec. 2.2 in the
  plane of the other two, the momentum along the constant axis zero): the
  3-D limited step equals the pinned 2-D limited step slice by slice, with
  the same troubled cells, over two steps (the subcell data of limited cells
  carried between them), for each of the three constant axes, with periodic
  and with free-outflow boundaries.  The exchanged flux at a face node (k, l)
  sums the sub-face fluxes against the projections of both face directions;
  along the constant one they sum to one, so the reduction covers the 3-D
  candidate, the 27-cell NAD, the 3-D subgrid scheme, R (x) R (x) R and the
  exchange at faces normal to each axis.
* A fully 3-D spherical explosion with periodic boundaries: the totals of all
  five variables are kept to rounding (every face carries one flux, also
  where the subgrid fluxes vary in both face directions) and the states stay
  admissible.
* NAD (Sec. 1.6) takes V_i = the cell and its 26 vertex neighbours: a
  candidate above its own cell's bounds is admissible when any one of them,
  alone, holds a larger subcell average, and troubled otherwise.
* A uniform state is kept and no cell is troubled.
* Planted mistakes (face nodes transposed, subgrid fluxes of another
  direction, a flipped exchange sign, periodic ghosts for free outflow, NAD
  over the face neighbours only) each break one of these pins.
"""

import copy

import numpy as np
import pytest

from oracle import basis, dg2d, dg3d, limiter2d, limiter3d
from paper_2409_12483_amd import workloads as W

E2, E3 = dg2d.Euler2D(), dg3d.Euler3D()


def _lift(u2, c, Cc):
    """2-D state [Ca, Cb, na, nb, 4] over the axes a < b other than c ->
    3-D [Cx, Cy, Cz, n, n, n, 5] constant along axis c."""
    a, b = [e for e in range(3) if e != c]
    n = u2.shape[2]
    q = np.zeros(u2.shape[:4] + (5,))
    q[..., 0], q[..., 1 + a], q[..., 1 + b], q[..., 4] = u2[..., 0], u2[..., 1], u2[..., 2], u2[..., 3]
    q = np.expand_dims(q, axis=c)                     # cell axis c
    q = np.expand_dims(q, axis=3 + c)                 # node axis c
    reps = [1] * 7
    reps[c], reps[3 + c] = Cc, n
    return np.tile(q, reps)


def _drop(u3, c):
    """Slice k = 0 along axis c of a 3-D state -> the 2-D one over (a, b)."""
    a, b = [e for e in range(3) if e != c]
    q = np.take(np.take(u3, 0, axis=3 + c), 0, axis=c)
    return q[..., [0, 1 + a, 1 + b, 4]]


@pytest.mark.parametrize("c,bc", [(2, "periodic"), (1, "transmissive"), (0, "periodic"), (2, "transmissive")])
def test_constant_axis_reduces_to_2d(c, bc):
    N, C2, Cc = 2, 6, 3
    ops = basis.build_operators(N)
    u2 = W.euler2d_explosion_nodal(C2, C2, N, r0=0.45)
    u3 = _lift(u2, c, Cc)
    h2, hc = 2.0 / C2, 0.7
    h3 = [h2, h2, h2]
    h3[c] = hc
    dt = 0.25 * dg2d.cfl_dt2d(ops, E2, u2, h2, h2, 0.4)
    v2 = v3 = None
    for step in range(2):
        u2, bad2, v2 = limiter2d.limited_step2d(ops, E2, u2, dt, h2, h2, bc, v=v2)
        u3, bad3, v3 = limiter3d.limited_step3d(ops, E3, u3, dt, tuple(h3), bc, v=v3)
        assert bad2.any()
        assert (np.take(bad3, 0, axis=c) == bad2).all()
        for k in range(Cc):
            assert (np.take(bad3, k, axis=c) == bad2).all()
        # constant along c, zero momentum along c
        for k in range(1, Cc):
            assert np.abs(np.take(u3, k, axis=c) - np.take(u3, 0, axis=c)).max() <= 1e-13
        assert np.abs(u3[..., 1 + c]).max() <= 1e-13
        assert np.abs(_drop(u3, c) - u2).max() <= 1e-11 * max(1.0, np.abs(u2).max()), step


def _sphere(C, N, r0=0.5):
    xs = W.cell_points(C, N + 1, -1.0, 1.0)
    X = xs[:, None, None, :, None, None]
    Y = xs[None, :, None, None, :, None]
    Z = xs[None, None, :, None, None, :]
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    rho = np.where(r <= r0, 1.0, 0.125)
    p = np.where(r <= r0, 1.0, 0.1)
    u = np.zeros(rho.shape + (5,))
    u[..., 0], u[..., 4] = rho, p / 0.4
    inner = r <= r0
    cut = inner.any(axis=(3, 4, 5)) & ~inner.all(axis=(3, 4, 5))
    _, w = W.gl_points_01(N + 1)
    mean = np.einsum("i,j,k,xyzijkr->xyzr", w, w, w, u)
    u[cut] = mean[cut][:, None, None, None, :]
    return u


def test_spherical_explosion_conserves_and_stays_admissible():
    N, C = 1, 6
    ops = basis.build_operators(N)
    u = _sphere(C, N)
    h = (2.0 / C,) * 3
    tot0 = dg3d.conserved_totals3d(ops, u, h)
    u1, t, info = limiter3d.limited_run3d(ops, E3, u, extent=(2.0, 2.0, 2.0), nsteps=3, bc="periodic")
    assert min(info["troubled"]) > 0
    tot1 = dg3d.conserved_totals3d(ops, u1, h)
    assert np.abs(tot1 - tot0).max() <= 1e-13 * np.abs(tot0).max()
    assert E3.admissible(info["v"]).all()


def test_uniform_state_is_kept():
    N, C = 2, 4
    ops = basis.build_operators(N)
    u = np.zeros((C, C, C, N + 1, N + 1, N + 1, 5))
    u[..., 0], u[..., 1], u[..., 2], u[..., 3], u[..., 4] = 1.0, 0.3, -0.2, 0.1, 3.0
    u1, bad, v = limiter3d.limited_step3d(ops, E3, u, 0.01, (0.5, 0.5, 0.5), "transmissive")
    assert not bad.any()
    assert np.abs(u1 - u).max() <= 1e-13


def _nad_holds(offset):
    """A candidate in cell (2, 2, 2) of a uniform 5^3 mesh above the cell's own
    bounds: admissible when the neighbour at `offset` alone holds a subcell
    above it, troubled when nothing does."""
    N = 1
    ops = basis.build_operators(N)
    Ns, C = ops.Ns, 5
    v = np.zeros((C, C, C, Ns, Ns, Ns, 5))
    v[..., 0], v[..., 4] = 1.0, 2.5
    u = np.zeros((C, C, C, N + 1, N + 1, N + 1, 5))
    u[..., 0], u[..., 4] = 1.0, 2.5
    u[2, 2, 2, ..., 0] = 1.5
    nb = tuple(2 + o for o in offset)
    v[nb][0, 0, 0, 0] = 2.0
    ok = not limiter3d.troubled_cells3d(ops, E3, v, u, "periodic")[2, 2, 2]
    v[nb][0, 0, 0, 0] = 1.0
    bad = limiter3d.troubled_cells3d(ops, E3, v, u, "periodic")
    return ok and bool(bad[2, 2, 2]) and int(bad.sum()) == 1


OFFSETS = [o for o in np.ndindex(3, 3, 3) if o != (1, 1, 1)]


@pytest.mark.parametrize("offset", [tuple(int(x) - 1 for x in o) for o in OFFSETS])
def test_nad_takes_the_26_vertex_neighbours(offset):
    assert _nad_holds(offset)


# ---- planted mistakes (CPU only): each must break one of the quick pins ----

def _reduction_holds(c, bc):
    """Two limited steps of the lifted explosion, its density and energy
    scaled by a ramp along the first in-plane axis (no mirror symmetry, so
    the ghost cells matter), against the 2-D oracle."""
    N, C2, Cc = 2, 6, 3
    ops = basis.build_operators(N)
    u2 = W.euler2d_explosion_nodal(C2, C2, N, r0=0.45)
    u2 = u2 * (1.0 + 0.3 * np.arange(C2) / C2)[:, None, None, None, None]
    u3 = _lift(u2, c, Cc)
    h3 = [2.0 / C2] * 3
    h3[c] = 0.7
    dt = 0.25 * dg2d.cfl_dt2d(ops, E2, u2, 2.0 / C2, 2.0 / C2, 0.4)
    v2 = v3 = None
    ok = True
    for _ in range(2):
        u2, b2, v2 = limiter2d.limited_step2d(ops, E2, u2, dt, 2.0 / C2, 2.0 / C2, bc, v=v2)
        with np.errstate(all="ignore"):
            u3, b3, v3 = limiter3d.limited_step3d(ops, E3, u3, dt, tuple(h3), bc, v=v3)
        ok = ok and bool((np.take(b3, 0, axis=c) == b2).all()) and bool(np.abs(_drop(u3, c) - u2).max() <= 1e-11)
    return ok


def _conserves():
    ops = basis.build_operators(1)
    u = _sphere(6, 1)
    h = (2.0 / 6,) * 3
    tot0 = dg3d.conserved_totals3d(ops, u, h)
    with np.errstate(all="ignore"):
        u1, _, _ = limiter3d.limited_run3d(ops, E3, u, nsteps=2, bc="periodic")
    return bool(np.abs(dg3d.conserved_totals3d(ops, u1, h) - tot0).max() <= 1e-13 * np.abs(tot0).max())


def _all_pins_hold():
    """The quick pins, cheapest first; False at the first that breaks."""
    return all(f() for f in (lambda: _nad_holds((1, 1, 1)), lambda: _nad_holds((-1, 0, 1)),
                             lambda: _reduction_holds(2, "transmissive"),
                             lambda: _reduction_holds(0, "periodic"), _conserves))


def _swap_face_axes(mp):
    orig = limiter3d.face_fluxes3d
    mp.setattr(limiter3d, "face_fluxes3d", lambda *a: [np.swapaxes(G, 3, 4) for G in orig(*a)])


def _fluxes_of_wrong_direction(mp):
    orig = limiter3d.fv3d_step

    def step(*a, **k):
        out = orig(*a, **k)
        return out[:3] + (out[3][::-1],) if k.get("fluxes") else out
    mp.setattr(limiter3d, "fv3d_step", step)


def _exchange_sign(mp):
    orig = limiter3d._correct

    def correct(ops, *a):
        o = copy.copy(ops)
        o.psi0 = -ops.psi0
        return orig(o, *a)
    mp.setattr(limiter3d, "_correct", correct)


def _periodic_ghosts_only(mp):
    orig = limiter3d.pad3d
    mp.setattr(limiter3d, "pad3d", lambda a, bc: orig(a, "periodic"))


def _face_neighbours_only(mp):
    def detect(ops, pde, v_old, u_cand, bc):
        C = u_cand.shape[:3]
        v_new = dg3d.subcell_averages(ops, u_cand)
        vp = limiter3d.pad3d(v_old, bc)
        mn = v_old.min(axis=(3, 4, 5))
        mx = v_old.max(axis=(3, 4, 5))
        for o in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]:
            blk = vp[o[0]:o[0] + C[0], o[1]:o[1] + C[1], o[2]:o[2] + C[2]]
            mn, mx = np.minimum(mn, blk.min(axis=(3, 4, 5))), np.maximum(mx, blk.max(axis=(3, 4, 5)))
        delta = np.maximum(limiter3d.DELTA0, limiter3d.EPS0 * (mx - mn))
        lo, hi = (mn - delta)[:, :, :, None, None, None], (mx + delta)[:, :, :, None, None, None]
        nad = ((v_new >= lo) & (v_new <= hi)).all(axis=(3, 4, 5, 6))
        ok = pde.admissible(v_new).all(axis=(3, 4, 5)) & pde.admissible(u_cand).all(axis=(3, 4, 5))
        return ~(nad & ok)
    mp.setattr(limiter3d, "troubled_cells3d", detect)


MUTATIONS = {"face node axes swapped": _swap_face_axes,
             "subgrid fluxes of the wrong direction": _fluxes_of_wrong_direction,
             "exchange sign flipped on one side": _exchange_sign,
             "periodic ghosts for free outflow": _periodic_ghosts_only,
             "NAD over the face neighbours only": _face_neighbours_only}


def test_unmutated_limiter3d_passes_the_quick_pins():
    assert _all_pins_hold()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_limiter3d_mistake_breaks_a_pin(name, monkeypatch):
    MUTATIONS[name](monkeypatch)
    assert not _all_pins_hold(), name
