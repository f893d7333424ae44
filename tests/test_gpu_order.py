"""GPU: convergence order N+1 of the fused ADER-DG step in both precision modes.

The 1-D density wave (rho = 1 + 0.2 sin(2 pi x), u = 1, p = 1; Sec. 2.1's
sine-wave problem restated in 1-D) run to t = 1 on three meshes per degree;
the error is the L2 norm of the density against the exact translate,
integrated cell by cell with the 25-point Gauss-Legendre rule of
Sec. 2.1 (eq. epsilons).  The FP64 path and the FP32-predictor path must
each show a fitted order of at least N + 1 - 0.3 between the two finest
meshes, and the FP32-predictor state must stay within 1e-5 (relative L2)
of the FP64 oracle's.  The meshes are those where the pinned oracle reaches
that order; the error on them stays well above the FP32-predictor mode's
own deviation from the FP64 result, so that deviation cannot mask or fake
the order.
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
T_END = 1.0


def _errors(N, prec):
    ops = basis.build_operators(N)
    errs, devs = [], []
    for C in MESHES[N]:
        u0 = W.euler_density_wave(C, N)
        ref, t_ref, info = dg.dg_run(ops, OP.Euler(), u0, 0.0, 1.0, cfl=0.4, t_end=T_END)
        (u,), t, _, st, _ = run_steps([abi.pde_desc(abi.PDE_EULER)],
                                      [abi.config(N, C, precision=prec)], [u0],
                                      info["steps"] + 2, t_end=np.array([T_END]))
        assert st[0] == 0 and abs(t[0] - T_END) <= 1e-14
        errs.append(norms.dg_errors(ops, u, lambda x: W.euler_density_wave_exact(x, T_END),
                                    0.0, 1.0)[1])
        devs.append(rel_l2(u, ref))
    return errs, devs


@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("prec", [abi.FP64, abi.FP32_PREDICTOR])
def test_gpu_convergence_order(N, prec):
    print("[case] order", N, prec, flush=True)
    errs, devs = _errors(N, prec)
    m = MESHES[N]
    p = norms.order(errs[-2], errs[-1], 1.0 / m[-2], 1.0 / m[-1])
    print("  errors", errs, "order", p, "deviation from the FP64 oracle", devs, flush=True)
    assert p >= N + 1 - 0.3, (errs, p)
    assert max(devs) <= (1e-12 if prec == abi.FP64 else 1e-5), devs
