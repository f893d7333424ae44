"""2-D and 3-D steps captured in a HIP graph replay like eager calls.

aderdg2d_step / aderdg3d_step enqueue kernels only (no host synchronisation,
no memset), so a call can be captured once and replayed.  Each replay is
checked bitwise against the same call made eagerly on a second handle, with
the program's own eager work and synchronisations between the replays.
"""

import numpy as np
import pytest

from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import torch_dev

pytestmark = pytest.mark.gpu


def _state(torch, dev, u0):
    return (torch.tensor(u0, device=dev), torch.zeros(1, dtype=torch.float64, device=dev),
            torch.full((1,), 1e300, dtype=torch.float64, device=dev),
            torch.zeros(1, dtype=torch.float64, device=dev), torch.zeros(1, dtype=torch.int32, device=dev))


@pytest.mark.parametrize("dim", [2, 3])
def test_graph_replays_equal_eager_steps(dim):
    print("[case] graph replay", dim, flush=True)
    torch, dev = torch_dev()
    if dim == 2:
        u0 = W.euler2d_sine_wave(40, 24, 4, noise=1e-3, seed=1)
        init = lambda s: abi.aderdg2d_init(abi.config2d(4, 40, 24, precision=abi.FP32_PREDICTOR), stream=s)
        step, free = abi.aderdg2d_step, abi.aderdg2d_free
    else:
        u0 = W.euler3d_sine_wave(8, 6, 5, 3, noise=1e-3, seed=1)
        init = lambda s: abi.aderdg3d_init(abi.config3d(3, (8, 6, 5)), stream=s)
        step, free = abi.aderdg3d_step, abi.aderdg3d_free
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g = _state(torch, dev, u0)
        hg = init(side.cuda_stream)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            step(hg, *g, 3)
    e = _state(torch, dev, u0)
    he = init(torch.cuda.current_stream().cuda_stream)
    try:
        for rep in range(3):
            graph.replay()
            side.synchronize()
            step(he, *e, 3)
            torch.cuda.synchronize()
            assert torch.equal(g[0], e[0]), rep
            assert torch.equal(g[1], e[1]) and torch.equal(g[3], e[3]) and int(g[4]) == 0
            junk = torch.ones(1 << 20, device=dev).sum()      # unrelated eager work
            assert float(junk) == float(1 << 20)
    finally:
        free(hg)
        free(he)


def test_limited_2d_step_in_a_graph_replays_like_eager_steps():
    """aderdg2d_lim_step enqueues kernels only as well: three replays of a
    captured call of 4 limited steps (the explosion, troubled cells on every
    step) against eager calls on a second handle, state, subcell averages,
    troubled mask, time and status bitwise."""
    print("[case] graph replay, limited 2-D step", flush=True)
    torch, dev = torch_dev()
    N, C = 2, 10
    u0 = W.euler2d_explosion_nodal(C, C, N)

    def make(stream):
        h = abi.aderdg2d_lim_init(abi.lim2d_config(N, C, C), stream=stream)
        u, t, te, dt, st = _state(torch, dev, u0)
        v = torch.zeros((C, C, 2 * N + 1, 2 * N + 1, 4), dtype=torch.float64, device=dev)
        tr = torch.zeros((C, C), dtype=torch.int32, device=dev)
        abi.aderdg2d_lim_project(h, u, v)
        return h, (u, v, tr, t, te, dt, st)

    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        hg, g = make(side.cuda_stream)
        side.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            abi.aderdg2d_lim_step(hg, *g, 4)
    he, e = make(torch.cuda.current_stream().cuda_stream)
    try:
        for rep in range(3):
            graph.replay()
            side.synchronize()
            abi.aderdg2d_lim_step(he, *e, 4)
            torch.cuda.synchronize()
            for a, b in zip(g, e):
                assert torch.equal(a, b), rep
            assert int(g[6]) == 0 and int(g[2].sum()) > 0
            junk = torch.ones(1 << 20, device=dev).sum()      # unrelated eager work
            assert float(junk) == float(1 << 20)
    finally:
        abi.aderdg2d_lim_free(hg)
        abi.aderdg2d_lim_free(he)
