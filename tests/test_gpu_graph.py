"""A captured HIP graph of an aderdg_step call replays exactly the eager call.

The call sequence (clock kernel, signal-speed kernel, step kernels, clock
kernel) holds no memset node, so it can be captured once the state pointers
are bound.  Every replay is compared bitwise with an eager handle advanced by
the same number of steps, with unrelated eager work and synchronisations
between the replays.
"""

import numpy as np
import pytest

from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import BIG, tensor, torch_dev

pytestmark = pytest.mark.gpu


def _handle(N, C, stream, fv=False):
    torch, dev = torch_dev()
    desc = abi.pde_desc(abi.PDE_SWE if fv else abi.PDE_EULER)
    cfg = abi.config(N, C, scheme=abi.SCHEME_FV if fv else abi.SCHEME_DG)
    h = abi.aderdg_init([desc], [cfg], stream=stream)
    u0 = W.swe_bump_averages(C) if fv else W.euler_density_wave(C, N, noise=1e-3, seed=3)
    bufs = (tensor(u0), tensor(np.zeros(1)), tensor(np.full(1, BIG)), tensor(np.zeros(1)),
            torch.zeros(1, dtype=torch.int32, device=dev))
    return h, bufs


@pytest.mark.parametrize("fv,N,C,k", [(False, 2, 100, 6), (False, 5, 1000, 3), (True, 4, 500, 4)])
def test_graph_replays_match_eager(fv, N, C, k):
    print("[case] graph", "fv" if fv else "dg", N, C, k, flush=True)
    torch, dev = torch_dev()
    step = abi.aderweno_step if fv else abi.aderdg_step
    s = torch.cuda.Stream()
    hg, (ug, tg, teg, dtg, stg) = _handle(N, C, s.cuda_stream, fv)
    he, (ue, te_, tee, dte, ste) = _handle(N, C, None, fv)
    try:
        with torch.cuda.stream(s):
            step(hg, [ug], tg, teg, dtg, stg, k)          # binds the pointers
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step(hg, [ug], tg, teg, dtg, stg, k)          # recorded, not run
        step(he, [ue], te_, tee, dte, ste, k)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue) and torch.equal(tg, te_)
        for rep in range(4):
            with torch.cuda.stream(s):
                g.replay()
            s.synchronize()
            junk = torch.randn(4096, device=dev).sum()     # eager work between replays
            step(he, [ue], te_, tee, dte, ste, k)
            torch.cuda.synchronize()
            assert junk.isfinite()
            assert int(stg.item()) == 0 and int(ste.item()) == 0
            assert torch.equal(tg, te_) and torch.equal(dtg, dte), rep
            assert torch.equal(ug, ue), rep
        del g
    finally:
        abi.aderdg_free(hg)
        abi.aderdg_free(he)
