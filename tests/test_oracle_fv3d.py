"""Pins of the oracle's 3-D ADER-WENO finite-volume step (Sec. 1.3 with d = 3).

* Data constant along one axis (and no momentum along it): the 3-D step equals
  the 2-D oracle's step on the other two axes (pinned on its own, down to the
  1-D scheme).  (A general permutation of the axes is not a symmetry: the
  sweeps of the reconstruction run x, y, z and their nonlinear weights do not
  commute.)
* A uniform state is kept; the totals of all five variables are conserved.
* The 3-D sine wave of Sec. 2.1 at WENO degree 2: the error falls at order
  about 3.
"""

import numpy as np
import pytest

from oracle import basis, dg2d, dg3d, fv2d, fv3d, norms
from paper_2409_12483_amd import workloads as W

E3 = dg3d.Euler3D()


def _state(cx, cy, cz, seed):
    v = W.euler3d_sine_averages(cx, cy, cz, velocity=(0.7, -0.4, 0.5))
    rng = np.random.default_rng(seed)
    v[..., 0] += 0.03 * rng.uniform(-1, 1, v.shape[:3])
    v[..., 4] += 0.05 * rng.uniform(-1, 1, v.shape[:3])
    return v


@pytest.mark.parametrize("N,const_axis", [(1, 2), (2, 2), (2, 0), (2, 1), (3, 1)])
def test_reduces_to_the_2d_scheme(N, const_axis):
    """Data constant along one axis, with no momentum along it: the other two
    axes, in their order, carry the 2-D step (the dimension-by-dimension
    sweeps keep that order, so the reconstruction is the 2-D one)."""
    ops = basis.build_operators(N)
    v2 = W.euler2d_sine_averages(9, 7, velocity=(0.7, -0.4))
    v2[..., 0] += 0.03 * np.random.default_rng(N).uniform(-1, 1, (9, 7))
    dt, h2 = 0.004, (1 / 9, 1 / 7)
    ref, _, _ = fv2d.fv2d_step(ops, dg2d.Euler2D(), v2, dt, h2[0], h2[1])
    axes = [a for a in range(3) if a != const_axis]               # the 2-D x and y axes
    shape = [0, 0, 0]
    shape[axes[0]], shape[axes[1]], shape[const_axis] = 9, 7, 4
    v3 = np.zeros(tuple(shape) + (5,))
    mom = [1 + axes[0], 1 + axes[1]]
    idx = [slice(None)] * 3
    idx[const_axis] = None
    v3[..., 0] = v2[..., 0][tuple(idx)]
    v3[..., mom[0]] = v2[..., 1][tuple(idx)]
    v3[..., mom[1]] = v2[..., 2][tuple(idx)]
    v3[..., 4] = v2[..., 3][tuple(idx)]
    h = [0.0, 0.0, 0.0]
    h[axes[0]], h[axes[1]], h[const_axis] = h2[0], h2[1], 0.25
    got, _, failed = fv3d.fv3d_step(ops, E3, v3, dt, tuple(h))
    assert not failed.any()
    g = np.moveaxis(got, const_axis, 2)                           # [x2, y2, const, 5]
    assert np.abs(g[..., [0, mom[0], mom[1], 4]] - ref[:, :, None, :]).max() <= 1e-13
    assert np.abs(g[..., 1 + const_axis]).max() <= 1e-15


@pytest.mark.parametrize("N", [1, 2, 3])
def test_uniform_state_and_conservation(N):
    ops = basis.build_operators(N)
    u = np.tile([1.3, 0.4, -0.2, 0.1, 3.1], (4, 5, 3, 1))
    v1, _, info = fv3d.fv3d_run(ops, E3, u, cfl=0.4, nsteps=5)
    assert np.abs(v1 - u).max() <= 1e-13 and not info["failed"]
    v0 = _state(5, 4, 6, 1)
    vn, _, _ = fv3d.fv3d_run(ops, E3, v0, cfl=0.4, nsteps=5)
    assert np.abs(vn.sum(axis=(0, 1, 2)) - v0.sum(axis=(0, 1, 2))).max() <= 1e-12


def test_sine_wave_order_degree_2():
    ops = basis.build_operators(2)
    errs = []
    for C in (8, 16):
        v, t, _ = fv3d.fv3d_run(ops, E3, W.euler3d_sine_averages(C, C, C), cfl=0.4, t_end=0.05)
        errs.append(np.abs(v[..., 0] - W.euler3d_sine_averages(C, C, C, t=t)[..., 0]).mean())
    p = norms.order(errs[0], errs[1], 1 / 8, 1 / 16)
    assert p >= 2.3, (errs, p)
