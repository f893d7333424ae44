"""GPU: convergence order N+1 of the fused ADER-DG step in both precision modes.

The 1-D density wave (rho = 1 + 0.2 sin(2 pi x), u = 1, p = 1; Sec. 2.1's
sine-wave problem restated in 1-D) run to t = 1 on three meshes per degree;
the error is the L2 norm of the density against the exact translate,
integrated cell by cell with the 25-point Gauss-Legendre rule of
Sec. 2.1 (eq. epsilons).  The FP64 path and the FP32-predictor path must
each show a fitted order of at least N + 1 - 0.3 between the two finest
meshes, and the FP32-predictor state must stay within 1e-5 (relative L2)
of the FP64 oracle's.  The meshes are those where the pinned oracle reaches
that order.

The FP32-predictor mode has its own error floor: float round-off in the
predictor leaves the state about 5e-8..1e-7 (relative L2) away from the FP64
result after a run to t = 1.  At N = 2 and 3 the discretisation error on the
order meshes stays far above it; at N = 4 and 5 the meshes where the scheme
is in its asymptotic range already have errors near 1e-7, so there the
FP32-predictor order is measured on coarser meshes (errors >= 3e-6, at least
40x the floor), where the scheme is still pre-asymptotic: it must match the
FP64 path's order on the same meshes within 0.1, and reach N + 1 - 0.6.
"""

import numpy as np
import pytest

from oracle import basis, dg, norms
from oracle import pde as OP
from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import rel_l2, run_steps

pytestmark = pytest.mark.gpu

MESHES = {2: (16, 24, 32), 3: (8, 12, 16), 4: (6, 9, 12), 5: (4, 5, 6)}
# (wave number, meshes) above the FP32-predictor floor at N = 4, 5
COARSE = {4: (1, (4, 5, 6)), 5: (3, (6, 8, 10))}
T_END = 1.0


def _errors(N, prec, meshes, k=1):
    ops = basis.build_operators(N)
    errs, devs = [], []
    for C in meshes:
        u0 = W.euler_density_wave(C, N, k=k)
        ref, t_ref, info = dg.dg_run(ops, OP.Euler(), u0, 0.0, 1.0, cfl=0.4, t_end=T_END)
        (u,), t, _, st, _ = run_steps([abi.pde_desc(abi.PDE_EULER)],
                                      [abi.config(N, C, precision=prec)], [u0],
                                      info["steps"] + 2, t_end=np.array([T_END]))
        assert st[0] == 0 and abs(t[0] - T_END) <= 1e-14
        errs.append(norms.dg_errors(ops, u, lambda x: W.euler_density_wave_exact(x, T_END, k=k),
                                    0.0, 1.0)[1])
        devs.append(rel_l2(u, ref))
    return errs, devs


def _order(errs, meshes):
    return norms.order(errs[-2], errs[-1], 1.0 / meshes[-2], 1.0 / meshes[-1])


@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("prec", [abi.FP64, abi.FP32_PREDICTOR])
def test_gpu_convergence_order(N, prec):
    print("[case] order", N, prec, flush=True)
    if prec == abi.FP32_PREDICTOR and N in COARSE:
        k, m = COARSE[N]
        e32, d32 = _errors(N, prec, m, k)
        e64, d64 = _errors(N, abi.FP64, m, k)
        p32, p64 = _order(e32, m), _order(e64, m)
        print("  coarse meshes", m, "k", k, "errors", e32, e64, "orders", p32, p64, "dev", d32, flush=True)
        assert min(e32) >= 3e-6
        assert abs(p32 - p64) <= 0.1 and p32 >= N + 1 - 0.6, (p32, p64)
        assert max(d32) <= 1e-5 and max(d64) <= 1e-12
        return
    m = MESHES[N]
    errs, devs = _errors(N, prec, m)
    p = _order(errs, m)
    print("  errors", errs, "order", p, "deviation from the FP64 oracle", devs, flush=True)
    assert p >= N + 1 - 0.3, (errs, p)
    assert max(devs) <= (1e-12 if prec == abi.FP64 else 1e-5), devs
