"""A 1-D mesh whose state holds more than 2^31 elements, through the C ABI.

N = 5 Euler on 1.2e8 periodic cells: 2.16e9 doubles (17.3 GB) per state
buffer, so element offsets pass 2^31 and byte offsets pass 2^34.  One fused
step with a fixed step size (no global signal-speed maximum is needed on the
host side); the cells on both sides of element 2^31 and of byte offset 2^32,
the first and last cells (periodic wrap) and random cells are compared with
the oracle's step of the same input, each from its 3-cell window (eq.
ader_dg_method_full couples a cell to its two neighbours only).
"""

import numpy as np
import pytest

from oracle import basis
from oracle import pde as OP
from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import BIG, oracle_dg_window, rel_l2, torch_dev

pytestmark = pytest.mark.gpu


def test_state_beyond_2_31_elements_sampled():
    torch, dev = torch_dev()
    N, C, M = 5, 120_000_000, 3
    n = N + 1
    assert C * n * M > 2 ** 31
    dx = 1.0 / C
    dt = 0.4 * dx / (11 * 2.5)                     # below the CFL limit of this state
    print("[case] large mesh", N, C, flush=True)
    u = torch.empty((C, n, M), dtype=torch.float64, device=dev)
    chunk = 10_000_000
    for j, c0 in enumerate(range(0, C, chunk)):
        c1 = min(C, c0 + chunk)
        part = W.euler_density_wave(c1 - c0, N, k=1000, noise=1e-3, seed=j, x0=c0 * dx, x1=c1 * dx)
        u[c0:c1].copy_(torch.from_numpy(part))
    rng = np.random.default_rng(3)
    b31 = 2 ** 31 // (n * M)                       # cell holding element 2^31
    b32 = 2 ** 29 // (n * M)                       # cell holding byte offset 2^32
    idx = np.unique(np.concatenate([[0, 1, b32 - 1, b32, b32 + 1, b31 - 1, b31, b31 + 1, C - 2, C - 1],
                                    rng.integers(0, C, 300)]))
    win = (idx[:, None] + np.arange(-1, 2)[None, :]) % C
    u_win = u[torch.from_numpy(win.reshape(-1)).to(dev)].cpu().numpy()      # the exact inputs
    h = abi.aderdg_init([abi.pde_desc(abi.PDE_EULER)], [abi.config(N, C, fixed_dt=dt)])
    try:
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        te = torch.full((1,), BIG, dtype=torch.float64, device=dev)
        dto = torch.zeros(1, dtype=torch.float64, device=dev)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        abi.aderdg_step(h, [u], t, te, dto, st, 1)
        torch.cuda.synchronize()
        assert int(st[0]) == 0 and float(t[0]) == dt and float(dto[0]) == dt
    finally:
        abi.aderdg_free(h)
    got = u[torch.from_numpy(idx).to(dev)].cpu().numpy()
    del u
    ops = basis.build_operators(N)
    centre = 3 * np.arange(len(idx)) + 1
    ref = oracle_dg_window(ops, OP.Euler(), u_win, dt, dx, 0.0, centre)
    u0 = u_win[centre]
    assert rel_l2(got - u0, ref - u0) <= 1e-10
    assert rel_l2(got, ref) <= 1e-12
