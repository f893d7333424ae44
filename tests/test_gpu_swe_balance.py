"""GPU: the shallow-water non-conservative terms on the lake at rest.

The oracle's pins of these terms (tests/test_oracle_swe.py) carried over to
the HIP path through the C ABI: DG over a continuous piecewise-linear
bathymetry stays at rest to round-off; the first DG step over a step
bathymetry keeps the momentum at zero (the path-conservative jump balances
the Rusanov momentum flux face by face); ADER-WENO-FV on the Gaussian bump
keeps hu at the scheme's truncation error.  Each run is also compared with
the oracle on the same input.
"""

import numpy as np
import pytest

from oracle import basis, dg, fv
from oracle import pde as OP
from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import rel_l2, run_steps

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("N,C", [(2, 45), (3, 77), (5, 40)])
def test_gpu_dg_lake_at_rest_linear_bathymetry(N, C):
    _say("dg lake linear", N, C)
    u0 = W.swe_lake_at_rest_nodal(C, N, kind="linear", seed=N)
    ref, _, _ = dg.dg_run(basis.build_operators(N), OP.ShallowWater(), u0, 0.0, 1.0, cfl=0.4, nsteps=50)
    (u,), _, _, st, sweeps = run_steps([abi.pde_desc(abi.PDE_SWE)], [abi.config(N, C)], [u0], 50)
    assert st[0] == 0
    assert np.abs(u[..., 1]).max() <= 1e-13
    assert np.abs(u[..., 0] + u[..., 2] - 1.0).max() <= 1e-13
    assert np.array_equal(u[..., 2], u0[..., 2])
    assert sweeps[0] == C * 50
    assert np.abs(u - ref).max() <= 1e-13


@pytest.mark.parametrize("N,C", [(1, 60), (2, 39), (4, 25)])
def test_gpu_dg_step_bathymetry_first_step(N, C):
    _say("dg lake step", N, C)
    u0 = W.swe_lake_at_rest_nodal(C, N, kind="step", seed=N)
    ref, _, _ = dg.dg_run(basis.build_operators(N), OP.ShallowWater(), u0, 0.0, 1.0, cfl=0.4, nsteps=1)
    (u,), _, _, st, _ = run_steps([abi.pde_desc(abi.PDE_SWE)], [abi.config(N, C)], [u0], 1)
    assert st[0] == 0
    assert np.abs(u[..., 1]).max() <= 1e-14
    assert rel_l2(u - u0, ref - u0) <= 1e-12


@pytest.mark.parametrize("prec,tol", [(abi.FP64, 1e-12), (abi.FP32_PREDICTOR, 1e-5)])
def test_gpu_fv_lake_at_rest_bump(prec, tol):
    _say("fv lake bump", prec)
    C = 128
    v0 = W.swe_lake_at_rest_averages(C)
    ref, t_ref, info = fv.fv_run(basis.build_operators(4), OP.ShallowWater(), v0, 0.0, 1.0,
                                 cfl=0.4, t_end=0.02)
    (v,), t, _, st, _ = run_steps([abi.pde_desc(abi.PDE_SWE)],
                                  [abi.config(4, C, precision=prec, scheme=abi.SCHEME_FV)], [v0],
                                  info["steps"] + 3, t_end=np.array([0.02]), fv_scheme=True)
    assert st[0] == 0 and abs(t[0] - t_ref) <= 1e-15
    assert np.array_equal(v[:, 2], v0[:, 2])
    assert rel_l2(v, ref) <= tol
    # momentum at the level of the oracle's truncation error (1.1e-6 at 128 cells)
    assert np.abs(v[:, 1]).max() <= 3e-6
    if prec == abi.FP64:
        assert np.abs(v[:, 1] - ref[:, 1]).max() <= 1e-13
