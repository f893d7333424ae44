"""Edge cases of the HIP path against the FP64 oracle (through the C ABI).

* meshes smaller than a workgroup tile and than the WENO stencil reach
  (periodic neighbours wrap several times): DG on 1-3 cells, FV on 2N+1 cells;
* nsteps = 0 leaves state, time and step untouched;
* the largest degree (N = 9) in the FP32-predictor mode;
* FP64 and FP32-predictor problems mixed in one handle.
"""

import numpy as np
import pytest

from oracle import basis, dg, fv
from oracle import pde as OP
from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import BIG, rel_l2, run_steps

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("N,C", [(3, 1), (2, 2), (5, 3)])
def test_dg_meshes_smaller_than_a_tile(N, C):
    _say("tiny dg mesh", N, C)
    ops = basis.build_operators(N)
    u0 = W.euler_density_wave(C, N, amp=0.1)
    ref, t_ref, _ = dg.dg_run(ops, OP.Euler(), u0, 0.0, 1.0, cfl=0.4, nsteps=5)
    (u,), t, dt, st, _ = run_steps([abi.pde_desc(abi.PDE_EULER)], [abi.config(N, C)], [u0], 5)
    assert st[0] == 0
    assert rel_l2(u, ref) <= 1e-12
    assert abs(t[0] - t_ref) <= 1e-14 * t_ref


@pytest.mark.parametrize("NW", [2, 4])
def test_fv_mesh_of_the_minimum_size(NW):
    C = 2 * NW + 1
    _say("tiny fv mesh", NW, C)
    ops = basis.build_operators(NW)
    v0 = W.swe_bump_averages(C)
    ref, t_ref, _ = fv.fv_run(ops, OP.ShallowWater(), v0, 0.0, 1.0, cfl=0.4, nsteps=4)
    (v,), t, dt, st, _ = run_steps([abi.pde_desc(abi.PDE_SWE)],
                                   [abi.config(NW, C, scheme=abi.SCHEME_FV)], [v0], 4, fv_scheme=True)
    assert st[0] == 0
    assert rel_l2(v, ref) <= 1e-12
    assert np.array_equal(v[:, 2], v0[:, 2])


def test_zero_steps_change_nothing():
    _say("zero steps")
    u0 = W.euler_density_wave(50, 4)
    (u,), t, dt, st, sw = run_steps([abi.pde_desc(abi.PDE_EULER)], [abi.config(4, 50)], [u0], 0,
                                    t0=np.array([0.25]))
    assert np.array_equal(u, u0) and t[0] == 0.25 and dt[0] == 0.0 and st[0] == 0 and sw[0] == 0


def test_fp32_predictor_at_the_largest_degree():
    _say("fp32 N=9")
    N, C = 9, 40
    ops = basis.build_operators(N)
    u0 = W.euler_density_wave(C, N)
    ref, _, _ = dg.dg_run(ops, OP.Euler(), u0, 0.0, 1.0, cfl=0.3, nsteps=3)
    (u,), _, _, st, _ = run_steps([abi.pde_desc(abi.PDE_EULER)],
                                  [abi.config(N, C, cfl=0.3, precision=abi.FP32_PREDICTOR)], [u0], 3)
    assert st[0] == 0
    assert rel_l2(u, ref) <= 1e-5


def test_precisions_mixed_in_one_handle():
    _say("mixed precision batch")
    descs = [abi.pde_desc(abi.PDE_EULER)] * 2
    cfgs = [abi.config(4, 60), abi.config(4, 60, precision=abi.FP32_PREDICTOR)]
    u0 = W.euler_density_wave(60, 4, noise=1e-3, seed=2)
    out, t, dt, st, _ = run_steps(descs, cfgs, [u0, u0], 3)
    ops = basis.build_operators(4)
    ref, _, _ = dg.dg_run(ops, OP.Euler(), u0, 0.0, 1.0, cfl=0.4, nsteps=3)
    assert (st == 0).all()
    assert rel_l2(out[0], ref) <= 1e-12
    assert 0.0 < rel_l2(out[1], ref) <= 1e-5       # the FP32 predictor is a different path
    (alone,), *_ = run_steps([descs[1]], [cfgs[1]], [u0], 3)
    assert np.array_equal(out[1], alone)
