"""The two compiled workgroup sizes of the fused 1-D DG step and the
autotuner that chooses between them, through the C ABI.

* 2 and 4 wavefronts per workgroup give bitwise the same states, times, step
  sizes, statuses and sweep counts (every cell's arithmetic is the same; only
  the tiling of the mesh differs): four models, both precisions, ragged and
  small meshes, a batch of problems of unequal sizes.
* aderdg_autotune leaves the problems as they were: steps before and after
  it equal the same number of steps without it, bit for bit, sweep counters
  included; it reports 2 or 4 per problem, the same on a second call (cached),
  and 4 for groups that have one size only (Newton inner iterations).
* aderdg_set_waves refuses other sizes.
"""

import numpy as np
import pytest

from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import BIG, tensor, torch_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _initial(pde, N, C, seed):
    if pde == abi.PDE_EULER:
        return W.euler_density_wave(C, N, noise=1e-3, seed=seed)
    if pde == abi.PDE_SWE:
        return W.swe_bump_nodal(C, N)
    if pde == abi.PDE_ADVECTION:
        return W.advection_nodal(C, N, lambda x: np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x))
    u = W.euler_density_wave(C, N, noise=1e-3, seed=seed)            # the two extra variables constant
    return np.concatenate([u, np.full((C, N + 1, 1), 0.8), np.full((C, N + 1, 1), -0.2)], axis=-1)


class Run:
    def __init__(self, descs, cfgs, states):
        torch, dev = torch_dev()
        self.torch = torch
        n = len(descs)
        self.h = abi.aderdg_init(descs, cfgs)
        self.u = [tensor(s) for s in states]
        self.t = tensor(np.zeros(n))
        self.te = tensor(np.full(n, BIG))
        self.dt = tensor(np.zeros(n))
        self.st = torch.zeros(n, dtype=torch.int32, device=dev)
        self.n = n

    def steps(self, k):
        abi.aderdg_step(self.h, self.u, self.t, self.te, self.dt, self.st, k)

    def result(self):
        self.torch.cuda.synchronize()
        return ([u.cpu().numpy() for u in self.u], self.t.cpu().numpy(), self.dt.cpu().numpy(),
                self.st.cpu().numpy(), [abi.aderdg_sweep_count(self.h, k) for k in range(self.n)])

    def close(self):
        abi.aderdg_free(self.h)


def _same(a, b):
    ua, ta, dta, sta, swa = a
    ub, tb, dtb, stb, swb = b
    for x, y in zip(ua, ub):
        assert np.array_equal(x, y)
    assert np.array_equal(ta, tb) and np.array_equal(dta, dtb) and np.array_equal(sta, stb)
    assert swa == swb


CASES = [
    ([(abi.PDE_EULER, 5, 1000)], abi.FP64),
    ([(abi.PDE_EULER, 2, 101)], abi.FP64),
    ([(abi.PDE_EULER, 5, 1000)], abi.FP32_PREDICTOR),
    ([(abi.PDE_SWE, 3, 257)], abi.FP64),
    ([(abi.PDE_ADVECTION, 9, 77)], abi.FP64),
    ([(abi.PDE_EULER_REACT, 4, 130)], abi.FP64),
    ([(abi.PDE_EULER, 4, 300), (abi.PDE_EULER, 4, 17), (abi.PDE_EULER, 4, 1201)], abi.FP64),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_two_workgroup_sizes_are_bitwise_equal(case):
    probs, prec = CASES[case]
    _say("waves 2 vs 4", probs, prec)
    descs = [abi.pde_desc(p) for p, _, _ in probs]
    cfgs = [abi.config(N, C, precision=prec) for _, N, C in probs]
    states = [_initial(p, N, C, seed=i) for i, (p, N, C) in enumerate(probs)]
    out = []
    for waves in (4, 2):
        r = Run(descs, cfgs, states)
        try:
            abi.aderdg_set_waves(r.h, waves)
            r.steps(7)
            out.append(r.result())
        finally:
            r.close()
    assert out[0][3].max() == 0
    _same(out[0], out[1])


def test_autotune_leaves_the_problems_unchanged():
    _say("autotune transparency")
    probs = [(abi.PDE_EULER, 5, 2000), (abi.PDE_EULER, 2, 300), (abi.PDE_SWE, 3, 500)]
    descs = [abi.pde_desc(p) for p, _, _ in probs]
    cfgs = [abi.config(N, C) for _, N, C in probs]
    states = [_initial(p, N, C, seed=i) for i, (p, N, C) in enumerate(probs)]
    ref = Run(descs, cfgs, states)
    tuned = Run(descs, cfgs, states)
    try:
        ref.steps(7)
        a = ref.result()
        tuned.steps(3)
        waves = abi.aderdg_autotune(tuned.h, tuned.u, 5)
        assert all(w in (2, 4) for w in waves) and len(waves) == 3
        tuned.steps(4)
        b = tuned.result()
        _same(a, b)
        again = abi.aderdg_autotune(tuned.h, tuned.u, 5)         # cached: same choice
        assert again == waves
    finally:
        ref.close()
        tuned.close()


def test_groups_with_one_size_are_left_at_four():
    _say("autotune: Newton group untouched")
    N, C = 3, 64
    descs = [abi.pde_desc(abi.PDE_EULER_REACT), abi.pde_desc(abi.PDE_EULER)]
    cfgs = [abi.config(N, C, inner=abi.INNER_NEWTON), abi.config(N, 2 * C)]
    states = [W.euler_react_uniform(C, N), _initial(abi.PDE_EULER, N, 2 * C, 1)]
    r = Run(descs, cfgs, states)
    try:
        waves = abi.aderdg_autotune(r.h, r.u, 3)
        assert waves[0] == 4 and waves[1] in (2, 4)
        r.steps(2)
        assert r.result()[3].max() == 0
    finally:
        r.close()


def test_set_waves_refuses_other_sizes():
    r = Run([abi.pde_desc(abi.PDE_EULER)], [abi.config(2, 50)], [_initial(abi.PDE_EULER, 2, 50, 0)])
    try:
        for w in (0, 1, 3, 8):
            with pytest.raises(abi.AderdgError):
                abi.aderdg_set_waves(r.h, w)
    finally:
        r.close()
