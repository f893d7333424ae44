"""Pins of the oracle's ADER-DG corrector, CFL and time loop (Sec. 1.2, 1.5, 2.1)."""

import numpy as np
import pytest

from oracle import basis, dg, norms
from oracle import pde as P
from paper_2409_12483_amd import workloads as W


@pytest.mark.parametrize("N", [1, 2, 5])
def test_constant_state_preserved(N):
    ops = basis.build_operators(N)
    e = P.Euler()
    u = W.euler_density_wave(6, N, amp=0.0, velocity=0.8, pressure=1.3)
    u1, t, info = dg.dg_run(ops, e, u, 0.0, 1.0, cfl=0.4, nsteps=200)
    assert np.abs(u1 - u).max() <= 2e-14 * np.abs(u).max()


def test_constant_state_preserved_swe_flat_bottom():
    ops = basis.build_operators(3)
    swe = P.ShallowWater()
    u = np.zeros((5, 4, 3))
    u[..., 0] = 1.3
    u[..., 1] = 0.4
    u[..., 2] = 0.05
    u1, _, _ = dg.dg_run(ops, swe, u, 0.0, 1.0, cfl=0.4, nsteps=100)
    assert np.abs(u1 - u).max() <= 1e-13    # rounding random walk over 100 steps


@pytest.mark.parametrize("N", [2, 4])
def test_exact_conservation_euler(N):
    ops = basis.build_operators(N)
    e = P.Euler()
    u = W.euler_density_wave(40, N, amp=0.2, noise=1e-3, seed=0)
    dx = 1.0 / 40
    m0 = dg.conserved_totals(ops, u, dx)
    u1, _, _ = dg.dg_run(ops, e, u, 0.0, 1.0, cfl=0.4, nsteps=150)
    m1 = dg.conserved_totals(ops, u1, dx)
    assert np.allclose(m1, m0, rtol=1e-13, atol=0)
    assert np.abs(u1 - u).max() > 1e-3          # the solution did move


def test_exact_conservation_swe_and_static_bathymetry():
    ops = basis.build_operators(3)
    swe = P.ShallowWater()
    u = W.swe_bump_nodal(50, 3)
    dx = 1.0 / 50
    m0 = dg.conserved_totals(ops, u, dx)
    u1, _, info = dg.dg_run(ops, swe, u, 0.0, 1.0, cfl=0.4, nsteps=80)
    m1 = dg.conserved_totals(ops, u1, dx)
    assert abs(m1[0] - m0[0]) <= 1e-13 * abs(m0[0])
    assert np.array_equal(u1[..., 2], u[..., 2])              # b bitwise invariant
    assert not info["failed"]


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_cfl_closed_form_uniform_state(N):
    ops = basis.build_operators(N)
    e = P.Euler(gamma=1.4)
    rho, vel, p = 1.7, -0.6, 2.2
    u = W.euler_density_wave(3, N, amp=0.0, velocity=vel, pressure=p)
    u[..., 0] = rho
    u[..., 1] = rho * vel
    u[..., 2] = p / 0.4 + 0.5 * rho * vel ** 2
    dt = dg.cfl_dt(ops, e, u, 0.1, 0.4)
    exact = 0.4 * 0.1 / ((2 * N + 1) * (abs(vel) + np.sqrt(1.4 * p / rho)))
    assert abs(dt - exact) <= 1e-15 * exact


def _density_wave_error(N, C, t_end):
    ops = basis.build_operators(N)
    e = P.Euler()
    u = W.euler_density_wave(C, N)
    u1, t, _ = dg.dg_run(ops, e, u, 0.0, 1.0, cfl=0.4, t_end=t_end)
    assert abs(t - t_end) < 1e-14
    return norms.dg_errors(ops, u1, lambda x: W.euler_density_wave_exact(x, t_end), 0.0, 1.0)[1]


@pytest.mark.parametrize("N,meshes", [(1, (8, 16, 32)), (2, (8, 16, 32)), (3, (8, 16, 32)),
                                      (4, (6, 12, 24)), (5, (4, 6, 8)), (6, (8, 10, 12))])
def test_convergence_order_density_wave(N, meshes):
    """Order N+1 of ADER-DG-P_N on the 1-D density wave (the 1-D analogue of
    Table 5's sine-wave advection; exact solution rho(x - t))."""
    errs = [_density_wave_error(N, C, 0.25) for C in meshes]
    p = norms.order(errs[-2], errs[-1], 1.0 / meshes[-2], 1.0 / meshes[-1])
    assert p >= N + 1 - 0.3, (errs, p)


def test_time_loop_clamps_to_end_time():
    ops = basis.build_operators(2)
    e = P.Euler()
    u = W.euler_density_wave(10, 2)
    _, t, info = dg.dg_run(ops, e, u, 0.0, 1.0, cfl=0.4, t_end=0.0123)
    assert t == 0.0123
    assert info["dts"][-1] <= info["dts"][0]
