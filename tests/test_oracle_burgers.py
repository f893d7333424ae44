"""Pins of the oracle's Burgers model (the test model of runtime-compiled user
models; not one of the paper's models).

Before its first shock the solution of q_t + (q^2/2)_x = 0 is constant along
characteristics: q(x, t) = q0(x - q t), an implicit closed form solved here by
Newton's method per point.  ADER-DG-P_N must converge to it at order N+1 (the
paper's order claim, Sec. 2.1), conserve the integral of q, and its predictor
must match the brute-force dense solve of the space-time system.
"""

import numpy as np
import pytest

from oracle import basis, brute, dg, norms, predictor
from oracle import pde as P
from paper_2409_12483_amd import workloads as W

A0, A1 = 1.0, 0.3


def q0(x):
    return A0 + A1 * np.sin(2 * np.pi * x)


def exact(x, t):
    """Solve q = q0(x - q t) by Newton's method (t below the shock time 1/(2 pi A1))."""
    q = q0(x)
    for _ in range(60):
        g = q - q0(x - q * t)
        dg_ = 1.0 + t * A1 * 2 * np.pi * np.cos(2 * np.pi * (x - q * t))
        q = q - g / dg_
    return q


def test_exact_solution_satisfies_the_characteristic_relation():
    x = np.linspace(0, 1, 101)
    t = 0.2
    q = exact(x, t)
    assert np.abs(q - q0(x - q * t)).max() <= 1e-14


def _error(N, C, t_end=0.2):
    ops = basis.build_operators(N)
    u = W.advection_nodal(C, N, q0)
    u1, t, _ = dg.dg_run(ops, P.Burgers(), u, 0.0, 1.0, cfl=0.4, t_end=t_end)
    return norms.dg_errors(ops, u1, lambda x: exact(x, t_end), 0.0, 1.0)[1], u, u1, ops


@pytest.mark.parametrize("N,meshes", [(2, (32, 64)), (3, (32, 64))])
def test_burgers_order_before_the_shock(N, meshes):
    e = [_error(N, C)[0] for C in meshes]
    p = norms.order(e[0], e[1], 1.0 / meshes[0], 1.0 / meshes[1])
    assert p >= N + 1 - 0.3, (e, p)


def test_burgers_conserves_the_integral():
    _, u, u1, ops = _error(3, 40)
    assert abs(dg.conserved_totals(ops, u1, 1 / 40)[0] - dg.conserved_totals(ops, u, 1 / 40)[0]) <= 1e-14


def test_burgers_predictor_matches_brute_force():
    N, C = 3, 3
    ops = basis.build_operators(N)
    u = W.advection_nodal(C, N, q0)
    dx, dt = 1.0 / C, 0.05
    q, _, _ = predictor.predict(ops, P.Burgers(), u, dt, dx, dx * np.arange(C), 0.0)
    mats = brute.assemble(ops)
    for c in range(C):
        qb = brute.solve_cell(ops, P.Burgers(), u[c], dt, dx, dx * c, 0.0, mats)
        assert np.abs(q[c] - qb).max() <= 1e-12
