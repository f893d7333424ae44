"""Pins of the oracle's 2-D ADER-WENO finite-volume step (Sec. 1.3 with d = 2).

* The dimension-by-dimension reconstruction is exact for tensor products of
  polynomials of the reconstruction degree (cells whose stencils do not wrap).
* Data that vary along x only: the 2-D step equals the 1-D oracle's
  ADER-WENO step (pinned on its own) on (rho, rho u, E), with rho v staying
  zero; the same along y after exchanging the axes.
* A uniform state is kept; the totals of all four variables are conserved.
* The 2-D sine wave of Sec. 2.1: the error falls at the order of the
  reconstruction degree + 1 (degree 1: the paper's ADER-WENO2; degree 2:
  ADER-WENO3; degree 3: ADER-WENO4, measured 5.3 on 8 -> 16 cells).
"""

import numpy as np
import pytest

from oracle import basis, dg2d, fv, fv2d, norms
from oracle import pde as P
from paper_2409_12483_amd import workloads as W


def _poly_avgs(c, C):
    Pi = np.polyint(c)
    e = np.linspace(0, 1, C + 1)
    return (np.polyval(Pi, e[1:]) - np.polyval(Pi, e[:-1])) * C


@pytest.mark.parametrize("N", [1, 2, 3])
def test_reconstruction_exact_for_tensor_polynomials(N):
    ops = basis.build_operators(N)
    rng = np.random.default_rng(N)
    cxp, cyp = rng.uniform(-1, 1, N + 1), rng.uniform(-1, 1, N + 1)
    Cx, Cy = 12, 10
    v = (_poly_avgs(cxp, Cx)[:, None] * _poly_avgs(cyp, Cy)[None, :])[..., None]
    w = fv2d.reconstruct2d(v, ops)
    xs, ys = W.cell_points(Cx, N + 1), W.cell_points(Cy, N + 1)
    exact = np.polyval(cxp, xs)[:, None, :, None] * np.polyval(cyp, ys)[None, :, None, :]
    sx, sy = slice(N, Cx - N), slice(N, Cy - N)
    assert np.abs(w[sx, sy, :, :, 0] - exact[sx, sy]).max() <= 1e-12


def _x_only(C, Cy, seed):
    rng = np.random.default_rng(seed)
    x = (np.arange(C) + 0.5) / C
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x) + 0.05 * rng.uniform(-1, 1, C)
    u = 0.4 + 0.2 * np.cos(2 * np.pi * x)
    p = 1.0 + 0.1 * np.sin(4 * np.pi * x)
    v1 = np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u], axis=-1)               # [C, 3]
    v2 = np.zeros((C, Cy, 4))
    v2[..., 0], v2[..., 1], v2[..., 3] = rho[:, None], (rho * u)[:, None], v1[:, None, 2]
    return v1, v2


@pytest.mark.parametrize("N", [1, 2, 3])
def test_reduces_to_the_1d_scheme_along_each_axis(N):
    ops = basis.build_operators(N)
    C, Cy, dt = 24, 5, 0.004
    v1, v2 = _x_only(C, Cy, N)
    ref, _, _ = fv.fv_step(ops, P.Euler(), v1, 0.0, dt, 1.0 / C, np.arange(C) / C)
    got, _, failed = fv2d.fv2d_step(ops, dg2d.Euler2D(), v2, dt, 1.0 / C, 1.0 / Cy)
    assert not failed.any()
    assert np.abs(got[..., [0, 1, 3]] - ref[:, None, :]).max() <= 1e-13
    assert np.abs(got[..., 2]).max() <= 1e-15
    # the same flow along y: exchange the axes and the momenta
    v2y = np.swapaxes(v2, 0, 1)[..., [0, 2, 1, 3]].copy()
    goty, _, _ = fv2d.fv2d_step(ops, dg2d.Euler2D(), v2y, dt, 1.0 / Cy, 1.0 / C)
    assert np.abs(np.swapaxes(goty, 0, 1)[..., [0, 2, 1, 3]] - got).max() <= 1e-13


@pytest.mark.parametrize("N", [1, 2, 3])
def test_uniform_state_and_conservation(N):
    ops = basis.build_operators(N)
    e = dg2d.Euler2D()
    u = np.tile([1.3, 0.4, -0.2, 3.1], (6, 7, 1))
    v1, _, info = fv2d.fv2d_run(ops, e, u, cfl=0.4, nsteps=10)
    assert np.abs(v1 - u).max() <= 1e-13 and not info["failed"]
    v0 = W.euler2d_sine_averages(9, 7)
    v0[..., 0] += 0.05 * np.random.default_rng(1).uniform(-1, 1, (9, 7))
    vn, _, _ = fv2d.fv2d_run(ops, e, v0, cfl=0.4, nsteps=10)
    assert np.abs(vn.sum(axis=(0, 1)) - v0.sum(axis=(0, 1))).max() <= 1e-12


@pytest.mark.parametrize("N,meshes,p_min", [(1, (32, 64), 1.7), (2, (16, 32), 2.6), (3, (8, 16), 3.5)])
def test_sine_wave_order(N, meshes, p_min):
    """Degree 1 is pre-asymptotic on 16 cells (its nonlinear weights pick the
    flatter one-sided slope near the extrema): 16 -> 32 gives order 1.06,
    32 -> 64 gives 1.79."""
    ops = basis.build_operators(N)
    e = dg2d.Euler2D()
    t_end = 0.1
    errs = []
    for C in meshes:
        v, t, _ = fv2d.fv2d_run(ops, e, W.euler2d_sine_averages(C, C), cfl=0.4, t_end=t_end)
        errs.append(np.abs(v[..., 0] - W.euler2d_sine_averages(C, C, t=t)[..., 0]).mean())
    p = norms.order(errs[0], errs[1], 1 / meshes[0], 1 / meshes[1])
    assert p >= p_min, (errs, p)
