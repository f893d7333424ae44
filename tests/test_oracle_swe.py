"""Pins of the oracle's shallow-water non-conservative terms (CPU).

The bathymetry enters the shallow-water model only through the
non-conservative product B(Q) dQ/dx = (0, g h db/dx, 0) (Sec. 1, eq. pde_src)
and, at cell faces, through the path-conservative jump of the interface
solver (reading of Sec. 1.2, parity unpinned as a choice).  Neither touches
the rows that conservation and the static bathymetry pin, so these tests pin
them with what the mathematics fixes for the lake at rest (h + b = const,
u = 0):

* DG, b continuous and piecewise linear (kinks at the cell edges), N >= 2:
  inside a cell g h^2 / 2 is a polynomial of degree 2 <= N, so the nodal
  derivative is exact and d/dx(g h^2/2) + g h db/dx = g h (h + b)_x = 0 at
  every node; the predictor keeps q = u (one sweep), the faces see equal
  states on both sides (zero jump, zero dissipation), hence hu stays at
  round-off for any number of steps.
* DG, b constant in every cell (jumps at the edges), one step: inside a cell
  nothing varies, and at a face between h- and h+ the Rusanov momentum flux
  is g (h-^2 + h+^2) / 4 while half the straight-path jump is
  g (h- + h+)(b+ - b-) / 4 = g (h-^2 - h+^2) / 4.  A cell i thus loses
  g h_i^2 / 2 through its right face (flux + jump) and gains g h_i^2 / 2
  through its left face (flux - jump): hu^{n+1} = 0 exactly.  A wrong sign,
  factor or state average of the jump leaves a momentum of order g dh dt/dx.
* ADER-WENO-FV on the Gaussian bump: the cell averages satisfy h + b = 1
  exactly but h and b are reconstructed with separate nonlinear weights, so
  hu grows only at the truncation error of the fifth-order scheme: the max
  of |hu| at a fixed time falls at order ~5 under refinement.
* Sec. 1.5: the finite-volume step of a uniform state is CFL dx / (|u| + c).
"""

import numpy as np
import pytest

from oracle import basis, dg, fv, norms
from oracle import pde as P
from paper_2409_12483_amd import workloads as W


@pytest.mark.parametrize("N", [2, 3, 5])
def test_dg_lake_at_rest_piecewise_linear_bathymetry(N):
    swe = P.ShallowWater()
    u = W.swe_lake_at_rest_nodal(16, N, kind="linear")
    u1, _, info = dg.dg_run(basis.build_operators(N), swe, u, 0.0, 1.0, cfl=0.4, nsteps=50)
    assert np.abs(u1[..., 1]).max() <= 1e-13
    assert np.abs(u1[..., 0] + u1[..., 2] - 1.0).max() <= 1e-13
    assert np.array_equal(u1[..., 2], u[..., 2])
    assert info["sweep_hist"] == {1: 16 * 50}          # the predictor keeps q = u


@pytest.mark.parametrize("N", [1, 2, 4])
def test_dg_step_bathymetry_first_step_keeps_momentum_zero(N):
    swe = P.ShallowWater()
    u = W.swe_lake_at_rest_nodal(16, N, kind="step")
    u1, _, _ = dg.dg_run(basis.build_operators(N), swe, u, 0.0, 1.0, cfl=0.4, nsteps=1)
    assert np.abs(u1[..., 1]).max() <= 1e-14
    # the Rusanov dissipation does move water between cells of different depth
    assert np.abs(u1[..., 0] - u[..., 0]).max() > 1e-3


def _fv_lake_errors(cells, t_end=0.02):
    swe = P.ShallowWater()
    ops = basis.build_operators(4)
    errs = []
    for C in cells:
        v = W.swe_lake_at_rest_averages(C)
        v1, t, info = fv.fv_run(ops, swe, v, 0.0, 1.0, cfl=0.4, t_end=t_end)
        assert abs(t - t_end) <= 1e-15 and not info["failed"]
        errs.append(float(np.abs(v1[:, 1]).max()))
    return errs


def test_fv_lake_at_rest_converges_at_fifth_order():
    cells = [64, 128, 256]
    errs = _fv_lake_errors(cells)
    p = norms.order(errs[-2], errs[-1], 1 / cells[-2], 1 / cells[-1])
    assert p >= 4.5, (errs, p)
    assert errs[-1] <= 1e-7, errs


@pytest.mark.parametrize("pde,state,speed", [
    (P.ShallowWater(9.81), [1.3, 0.39, 0.2], 0.3 + np.sqrt(9.81 * 1.3)),
    (P.Euler(1.4), [1.2, 0.3, 2.9], 0.25 + np.sqrt(1.4 * 0.4 * (2.9 - 0.5 * 0.3 * 0.25) / 1.2)),
])
def test_fv_time_step_closed_form(pde, state, speed):
    C, cfl = 40, 0.4
    v = np.tile(state, (C, 1))
    _, t, info = fv.fv_run(basis.build_operators(4), pde, v, 0.0, 2.0, cfl=cfl, nsteps=1)
    expect = cfl * (2.0 / C) / speed
    assert abs(info["dts"][0] - expect) <= 1e-15 * expect
    assert t == info["dts"][0]
