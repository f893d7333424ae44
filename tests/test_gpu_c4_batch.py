"""GPU: the 256-problem batch (uneven Euler problems, N = 1..7) problem by problem.

All 256 specs of the batched workload (seeded wave numbers, phases, degrees),
with the cell counts scaled down 100-fold so that the oracle can run every
problem: the whole batch is advanced in one handle (one launch per degree
group and step), and every problem is compared with the oracle run alone:
1e-12 (FP64) and 1e-5 (FP32 predictor) relative L2.
"""

import numpy as np
import pytest

from oracle import basis, dg
from oracle import pde as OP
from paper_2409_12483_amd import abi
from paper_2409_12483_amd import batch as B
from paper_2409_12483_amd import workloads as W

from gpu_util import rel_l2, run_steps

pytestmark = pytest.mark.gpu

STEPS = 3


def _specs():
    specs = W.batched_euler_problems(nprob=256, seed=0)
    for s in specs:
        s["ncells"] = max(3, int(round(s["ncells"] / 100)))
    return specs


@pytest.fixture(scope="module")
def oracle_states():
    out = []
    e = OP.Euler()
    for s in _specs():
        u0 = B.initial_state(s)
        ref, _, _ = dg.dg_run(basis.build_operators(s["N"]), e, u0, 0.0, 1.0, cfl=0.4, nsteps=STEPS)
        out.append((u0, ref))
    return out


@pytest.mark.parametrize("prec,tol", [(abi.FP64, 1e-12), (abi.FP32_PREDICTOR, 1e-5)])
def test_c4_shaped_batch_every_problem_matches_oracle(oracle_states, prec, tol):
    print("[case] C4 batch", prec, flush=True)
    specs = _specs()
    descs = [abi.pde_desc(abi.PDE_EULER) for _ in specs]
    cfgs = [abi.config(s["N"], s["ncells"], precision=prec) for s in specs]
    us, t, dt, st, _ = run_steps(descs, cfgs, [u0 for u0, _ in oracle_states], STEPS)
    assert (st == 0).all()
    errs = [rel_l2(u, ref) for u, (_, ref) in zip(us, oracle_states)]
    print("  worst problem", int(np.argmax(errs)), max(errs), flush=True)
    assert max(errs) <= tol
    assert sorted({s["N"] for s in specs}) == list(range(1, 8))
