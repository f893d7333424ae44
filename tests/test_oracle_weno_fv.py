"""Pins of the oracle's WENO reconstruction and ADER-WENO-FV step (Sec. 1.3).

The WENO stencils and constants are a reading (the paper gives none); the
pins below are what the mathematics fixes for any such reconstruction:
polynomial exactness, convex weights, mirror symmetry and order N+1.
"""

import numpy as np
import pytest

from oracle import basis, fv, norms, weno
from oracle import pde as P
from paper_2409_12483_amd import workloads as W


def _poly_cell_averages(coeffs, C):
    # exact averages of a polynomial on [0,1] split into C cells
    P_int = np.polyint(coeffs)
    e = np.linspace(0, 1, C + 1)
    return (np.polyval(P_int, e[1:]) - np.polyval(P_int, e[:-1])) * C


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_weno_exact_for_polynomials(N):
    ops = basis.build_operators(N)
    C = 24
    rng = np.random.default_rng(N)
    coeffs = rng.uniform(-1, 1, N + 1)
    v = _poly_cell_averages(coeffs, C)[:, None]
    w_hat = weno.reconstruct(v, ops)
    xs = W.cell_points(C, N + 1)
    interior = slice(N, C - N)          # stencils that do not wrap around
    assert np.allclose(w_hat[interior, :, 0], np.polyval(coeffs, xs[interior]), atol=1e-12)


def test_weno_weights_are_convex_and_favour_smooth_stencil():
    ops = basis.build_operators(4)
    C = 40
    x = (np.arange(C) + 0.5) / C
    v = np.where(x < 0.5, 1.0, 0.1)[:, None] + 0.01 * np.sin(2 * np.pi * x)[:, None]
    coeff = weno.stencil_polynomials(v, 4)
    om = weno.weights(weno.oscillation_indicators(coeff, 4))
    assert np.allclose(om.sum(0), 1.0, atol=1e-14) and (om >= 0).all()
    # the cell just left of the jump takes its left (smooth) stencil
    i = int(np.searchsorted(x, 0.5)) - 1
    assert om[0, i, 0] > 0.99
    # and the reconstruction stays close to the data range (non-oscillatory)
    w_hat = weno.reconstruct(v, ops)
    assert w_hat.max() < 1.02 and w_hat.min() > 0.08


@pytest.mark.parametrize("N", [1, 3, 4])
def test_weno_mirror_symmetry(N):
    ops = basis.build_operators(N)
    C = 30
    rng = np.random.default_rng(3)
    v = rng.uniform(0.5, 1.5, (C, 2))
    a = weno.reconstruct(v, ops)
    b = weno.reconstruct(v[::-1].copy(), ops)
    assert np.allclose(a, b[::-1, ::-1], atol=1e-12)


@pytest.mark.parametrize("N,p_min", [(3, 3.5), (4, 4.5)])
def test_weno_order_on_smooth_data(N, p_min):
    ops = basis.build_operators(N)
    errs = []
    Cs = [20, 40, 80]
    for C in Cs:
        v = W.smooth_averages(C, lambda x: np.sin(2 * np.pi * x))[:, None]
        w_hat = weno.reconstruct(v, ops)
        errs.append(np.abs(w_hat[:, :, 0] - np.sin(2 * np.pi * W.cell_points(C, N + 1))).max())
    p = norms.order(errs[-2], errs[-1], 1 / Cs[-2], 1 / Cs[-1])
    assert p >= p_min, (errs, p)


def test_weno_degree_three_stencils_and_weights():
    """Degree 3 (ADER-WENO4): four stencils of four cells, {i-3..i},
    {i-2..i+1}, {i-1..i+2}, {i..i+3}; on smooth data the two central ones
    carry almost all the weight (linear weights 1e5 against 1), at a jump
    the stencils that stay on one side do."""
    assert weno.stencil_offsets(3) == [[-3, -2, -1, 0], [-2, -1, 0, 1], [-1, 0, 1, 2], [0, 1, 2, 3]]
    C = 40
    x = (np.arange(C) + 0.5) / C
    v = W.smooth_averages(C, lambda y: np.sin(2 * np.pi * y))[:, None]
    om = weno.weights(weno.oscillation_indicators(weno.stencil_polynomials(v, 3), 3), 3)
    assert np.allclose(om.sum(0), 1.0, atol=1e-14) and (om >= 0).all()
    assert (om[1] + om[2]).min() > 0.99
    vj = np.where(x < 0.5, 1.0, 0.1)[:, None] + 0.01 * np.sin(2 * np.pi * x)[:, None]
    omj = weno.weights(weno.oscillation_indicators(weno.stencil_polynomials(vj, 3), 3), 3)
    i = int(np.searchsorted(x, 0.5)) - 1        # last cell left of the jump: only {i-3..i} avoids it
    assert omj[0, i, 0] > 0.99


def test_weno_degree_one_closed_forms():
    """Degree 1 (ADER-WENO2): the stencil polynomials are the two one-sided
    slopes, sigma_s = slope_s^2, the weights are (sigma + eps)^-8 normalised,
    and the reconstruction keeps the cell average; at a kink it takes the
    flatter side."""
    ops = basis.build_operators(1)
    rng = np.random.default_rng(7)
    C = 12
    v = rng.uniform(0.5, 1.5, (C, 1))
    coeff = weno.stencil_polynomials(v, 1)
    sl = v - np.roll(v, 1, axis=0)              # {i-1, i}
    sr = np.roll(v, -1, axis=0) - v             # {i, i+1}
    assert np.allclose(coeff[0, :, 1], sl, atol=1e-14) and np.allclose(coeff[1, :, 1], sr, atol=1e-14)
    assert np.allclose(coeff[:, :, 0], v[None], atol=1e-14)        # value at the cell centre
    sig = weno.oscillation_indicators(coeff, 1)
    assert np.allclose(sig[0], sl ** 2, rtol=1e-13) and np.allclose(sig[1], sr ** 2, rtol=1e-13)
    om = weno.weights(sig, 1)
    a, b = (sl ** 2 + 1e-14) ** -8, (sr ** 2 + 1e-14) ** -8
    assert np.allclose(om[0], a / (a + b), rtol=1e-12)
    w_hat = weno.reconstruct(v, ops)
    assert np.allclose(np.einsum("k,ckr->cr", ops.w, w_hat), v, atol=1e-14)
    kink = np.array([0.0, 1.0, 2.0, 2.0, 2.0, 1.0, 0.0, 0.0])[:, None]
    wk = weno.reconstruct(kink, ops)
    assert np.allclose(wk[2], 2.0, atol=1e-10)                     # flat right side chosen at the kink


def test_fv_constant_state_preserved():
    ops = basis.build_operators(4)
    e = P.Euler()
    v = np.tile([1.2, 0.3, 2.9], (16, 1))
    v1, _, info = fv.fv_run(ops, e, v, 0.0, 1.0, cfl=0.4, nsteps=50)
    assert np.abs(v1 - v).max() <= 1e-13
    assert not info["failed"]


def test_fv_conservation_and_static_bathymetry():
    ops = basis.build_operators(4)
    swe = P.ShallowWater()
    v = W.swe_bump_averages(64)
    v1, _, info = fv.fv_run(ops, swe, v, 0.0, 1.0, cfl=0.4, nsteps=30)
    assert abs(v1[:, 0].sum() - v[:, 0].sum()) <= 1e-13 * v[:, 0].sum()
    assert np.array_equal(v1[:, 2], v[:, 2])
    assert np.abs(v1[:, 0] - v[:, 0]).max() > 1e-4
    assert not info["failed"]


def test_fv_order_density_wave():
    """ADER-WENO5-FV (WENO degree 4 + LST-DG predictor N = 4): order ~5 on the density wave."""
    ops = basis.build_operators(4)
    e = P.Euler()
    errs = []
    Cs = [16, 32, 64]
    t_end = 0.1
    for C in Cs:
        rho = W.smooth_averages(C, lambda x: 1 + 0.2 * np.sin(2 * np.pi * x))
        v = np.stack([rho, rho, 2.5 + 0.5 * rho], axis=1)
        v1, t, _ = fv.fv_run(ops, e, v, 0.0, 1.0, cfl=0.4, t_end=t_end)
        exact = W.smooth_averages(C, lambda x: 1 + 0.2 * np.sin(2 * np.pi * (x - t_end)))
        errs.append(norms.fv_errors(v1, exact)[1])
    p = norms.order(errs[-2], errs[-1], 1 / Cs[-2], 1 / Cs[-1])
    assert p >= 4.5, (errs, p)
