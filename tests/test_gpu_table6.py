"""The paper's 3-D accuracy table (Sec. 2.1, Table 6) reproduced on the GPU
through the C ABI: the sine wave of the Euler gas to t_final = 1 on the
paper's meshes for N = 2..9 (tests/golden/table6_sine_wave_3d.txt).

* The density errors eps_L1 and eps_L2 (eq. epsilons, evaluated by the
  oracle's quadrature on the GPU result) lie within [0.5, 3.5] of the paper's
  (the Riemann solvers differ: Rusanov here, unstated there), and every
  convergence order between consecutive meshes lies within 0.5 of the
  paper's, wherever both errors are above 1e-12 and the coarser mesh has at
  least 4 cells per side.
* The N = 1 rows are left out (their printed orders, 3.89 / 2.95 / 2.21, are
  pre-asymptotic; the oracle's N = 1 error on 10^3 cells is 4.5x below the
  printed one).  N = 6, 7 use their first three meshes (the 20^3 runs take
  about a minute); N = 8, 9 run at CFL 0.3 (at 0.4 the step leaves the
  admissible set at N = 9 with the Rusanov flux, as in 2-D).
"""

import os

import numpy as np
import pytest

from oracle import basis, dg3d
from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import torch_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table6_sine_wave_3d.txt")


def _golden():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                rows.setdefault(int(v[0]), []).append((int(v[1]), float(v[2]), float(v[3])))
    return rows


def _say(*a):
    print("[case]", *a, flush=True)


def sine_errors(N, C, cfl):
    torch, dev = torch_dev()
    h = abi.aderdg3d_init(abi.config3d(N, (C, C, C), cfl=cfl))
    try:
        u = torch.tensor(W.euler3d_sine_wave(C, C, C, N), device=dev)
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        te = torch.ones(1, dtype=torch.float64, device=dev)
        dt = torch.zeros_like(t)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        for _ in range(200):                       # chunks of steps until t_final
            abi.aderdg3d_step(h, u, t, te, dt, st, 256)
            torch.cuda.synchronize()
            if float(t[0]) >= 1.0 or int(st[0]) != 0:
                break
        assert int(st[0]) == 0 and float(t[0]) == 1.0
        ops = basis.build_operators(N)
        l1, l2, _ = dg3d.dg3d_errors(ops, u.cpu().numpy(),
                                     lambda x, y, z: W.euler3d_sine_wave_exact(x, y, z, 0.0))
        return l1, l2
    finally:
        abi.aderdg3d_free(h)


@pytest.mark.parametrize("N", range(2, 10))
def test_table6_row_on_the_gpu(N):
    rows = _golden()[N]
    if N in (6, 7):
        rows = rows[:3]
    cfl = 0.3 if N >= 8 else 0.4
    _say("table 6", N, [r[0] for r in rows], cfl)
    ours = [sine_errors(N, C, cfl) for C, _, _ in rows]
    for (C, p1, p2), (e1, e2) in zip(rows, ours):
        _say("  ", C, e1, p1, e2, p2)
        assert 0.5 <= e1 / p1 <= 3.5 and 0.5 <= e2 / p2 <= 3.5, (N, C, e1, p1, e2, p2)
    for k in range(1, len(rows)):
        (c0, pa1, pa2), (c1, pb1, pb2) = rows[k - 1], rows[k]
        (ea1, ea2), (eb1, eb2) = ours[k - 1], ours[k]
        for ea, eb, pa, pb in ((ea1, eb1, pa1, pb1), (ea2, eb2, pa2, pb2)):
            if min(ea, eb, pa, pb) < 1e-12 or c0 < 4:
                continue
            ours_p = np.log(ea / eb) / np.log(c1 / c0)
            paper_p = np.log(pa / pb) / np.log(c1 / c0)
            assert abs(ours_p - paper_p) <= 0.5, (N, c0, c1, ours_p, paper_p)
