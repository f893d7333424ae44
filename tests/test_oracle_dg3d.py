"""Pins of the 3-D ADER-DG oracle (oracle.dg3d):

* data constant along one axis (that velocity component 0) reduce the 3-D
  scheme to the 2-D one on the other two axes (oracle.dg2d, pinned on its own
  by 1-D reductions and Table 5), for each of the three axes, on a domain of
  unequal sides: every operator, trace, flux and scaling of each direction is
  checked, with the per-cell sweep counts;
* the CFL step of such data is the 2-D step times 2/3 (Sec. 1.5, factor 1/d);
* a uniform state is preserved; totals are conserved to rounding;
* a cyclic permutation of the axes permutes the result;
* the sine wave converges at order about N + 1 over a short time;
* opt-in (ADERDG_SLOW_TESTS=1, about 4 minutes): the N = 2 errors on 10^3
  cells of Table 6 (tests/golden/table6_sine_wave_3d.txt) within 30 %.
"""

import os

import numpy as np
import pytest

from oracle import basis, dg2d, dg3d, norms
from paper_2409_12483_amd import workloads as W

E3, E2 = dg3d.Euler3D(), dg2d.Euler2D()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table6_sine_wave_3d.txt")
# 2-D variable -> 3-D variable, for the two retained axes (first, second)
_VARS = {0: (2, 3), 1: (1, 3), 2: (1, 2)}


def _embed(u2, axis, size):
    """2-D state on the axes other than `axis` -> 3-D state constant along `axis`."""
    cx, cy, n = u2.shape[0], u2.shape[1], u2.shape[2]
    a, b = _VARS[axis]
    shape3 = [cx, cy]
    shape3.insert(axis, size)
    out = np.zeros(tuple(shape3) + (n, n, n, 5))
    src = np.expand_dims(u2, axis)                  # [.., 1 at axis, .., n, n, M]
    src = np.expand_dims(src, 3 + axis)             # node axis inserted too
    out[..., 0] = src[..., 0]
    out[..., a] = src[..., 1]
    out[..., b] = src[..., 2]
    out[..., 4] = src[..., 3]
    return out, (a, b)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("N", [1, 2])
def test_data_constant_along_an_axis_reduce_to_2d(N, axis):
    ops = basis.build_operators(N)
    lengths = [0.9, 0.7, 0.5]
    keep = [d for d in range(3) if d != axis]
    u2 = W.euler2d_sine_wave(4, 3, N, noise=1e-2, seed=10 * N + axis, velocity=(0.7, -0.4),
                             x1=lengths[keep[0]], y1=lengths[keep[1]])
    u3, (a, b) = _embed(u2, axis, 2)
    dt = 1e-3
    r2, _, i2 = dg2d.dg2d_run(ops, E2, u2, extent=(0, lengths[keep[0]], 0, lengths[keep[1]]),
                              fixed_dt=dt, nsteps=3)
    r3, _, i3 = dg3d.dg3d_run(ops, E3, u3, extent=tuple(lengths), fixed_dt=dt, nsteps=3)
    ref, _ = _embed(r2, axis, 2)
    scale = np.abs(r2).max()
    assert np.abs(r3 - ref).max() <= 1e-13 * scale
    assert sum(i3["sweep_hist"].values()) == 2 * sum(i2["sweep_hist"].values())
    assert set(i3["sweep_hist"]) == set(i2["sweep_hist"])


def test_cfl_has_the_dimension_factor():
    N = 3
    ops = basis.build_operators(N)
    u2 = W.euler2d_sine_wave(5, 5, N, amp=0.3)
    u3, _ = _embed(u2, 2, 5)
    dt2 = dg2d.cfl_dt2d(ops, E2, u2, 0.2, 0.2, 0.4)
    dt3 = dg3d.cfl_dt3d(ops, E3, u3, (0.2, 0.2, 0.2), 0.4)
    assert abs(dt3 - dt2 * 2.0 / 3.0) <= 1e-15 * dt2


def test_uniform_state_and_conservation():
    N = 2
    ops = basis.build_operators(N)
    u = W.euler3d_sine_wave(3, 2, 2, N, amp=0.0, velocity=(0.3, -0.5, 0.8))
    r, _, _ = dg3d.dg3d_run(ops, E3, u, nsteps=2)
    assert np.abs(r - u).max() <= 1e-14 * np.abs(u).max()
    u = W.euler3d_sine_wave(3, 4, 2, N, noise=1e-2, seed=2, velocity=(0.3, -0.6, 0.9))
    r, _, _ = dg3d.dg3d_run(ops, E3, u, nsteps=3)
    h = (1 / 3, 1 / 4, 1 / 2)
    before, after = dg3d.conserved_totals3d(ops, u, h), dg3d.conserved_totals3d(ops, r, h)
    assert np.abs(after - before).max() <= 1e-14 * np.abs(before).max()
    assert np.abs(r - u).max() > 1e-4


def test_cyclic_permutation_of_the_axes():
    N = 2
    ops = basis.build_operators(N)
    u = W.euler3d_sine_wave(4, 3, 2, N, noise=1e-2, seed=5, k=(1, 2, 1), velocity=(0.5, -0.3, 0.2))
    r, _, _ = dg3d.dg3d_run(ops, E3, u, nsteps=2)
    # (x, y, z) -> (y, z, x): cells, nodes and momentum components move together
    perm = lambda a: np.transpose(a, (1, 2, 0, 4, 5, 3, 6))[..., [0, 2, 3, 1, 4]]
    rp, _, _ = dg3d.dg3d_run(ops, E3, perm(u), nsteps=2)
    assert np.abs(rp - perm(r)).max() <= 1e-14 * np.abs(r).max()


def test_convergence_order_over_a_short_time():
    N = 1
    ops = basis.build_operators(N)
    errs = []
    for C in (4, 8):
        u = W.euler3d_sine_wave(C, C, C, N, amp=0.2)
        r, t, _ = dg3d.dg3d_run(ops, E3, u, t_end=0.05)
        errs.append(dg3d.dg3d_errors(ops, r, lambda x, y, z: W.euler3d_sine_wave_exact(
            x, y, z, 0.05, amp=0.2))[1])
    p = norms.order(errs[0], errs[1], 1 / 4, 1 / 8)
    assert 1.7 <= p <= 3.2, p


@pytest.mark.skipif(not os.environ.get("ADERDG_SLOW_TESTS"), reason="about 4 minutes; set ADERDG_SLOW_TESTS=1")
def test_table6_errors_at_degree_2():
    rows = {(int(v[0]), int(v[1])): (float(v[2]), float(v[3]))
            for v in (l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#"))}
    N, C = 2, 10
    l1, l2 = rows[(N, C)]
    ops = basis.build_operators(N)
    r, t, info = dg3d.dg3d_run(ops, E3, W.euler3d_sine_wave(C, C, C, N), t_end=1.0)
    assert t == 1.0 and not info["failed"]
    e = dg3d.dg3d_errors(ops, r, lambda x, y, z: W.euler3d_sine_wave_exact(x, y, z, 0.0))
    assert abs(e[0] / l1 - 1.0) <= 0.3 and abs(e[1] / l2 - 1.0) <= 0.3, e
