"""Pins of the oracle's LST-DG predictor (Sec. 1.1)."""

import numpy as np
import pytest

from oracle import basis, brute, predictor
from oracle import pde as P
from paper_2409_12483_amd import workloads as W


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_kronecker_forms_match_first_principles_assembly(N):
    """L^xi, L^sigma, L^0, D^xi from the defining space-time integrals equal
    kappa~ (x) k~, kappa~ (x) I, 1 (x) I and I (x) (D^phi)^T (Sec. 1.1, Kronecker forms)."""
    ops = basis.build_operators(N)
    m = brute.assemble(ops)
    n = ops.n
    Kinv = np.linalg.inv(m["Ktau"])
    assert np.allclose(Kinv @ m["Kxi"], np.kron(ops.kappa, ops.ktil), atol=1e-11)
    assert np.allclose(Kinv @ m["M"], np.kron(ops.kappa, np.eye(n)), atol=1e-12)
    assert np.allclose(Kinv @ m["F0"], np.kron(np.ones((n, 1)), np.eye(n)), atol=1e-11)
    assert np.allclose(m["Dxi"], np.kron(np.eye(n), ops.Dphi.T), atol=1e-11)


@pytest.mark.parametrize("N", [0, 1, 4, 9])
def test_constant_state_is_a_fixed_point(N):
    ops = basis.build_operators(N)
    e = P.Euler()
    u = W.euler_density_wave(3, N, amp=0.0, velocity=0.7, pressure=2.0)
    q, sweeps, failed = predictor.predict(ops, e, u, 0.01, 0.1, 0.1 * np.arange(3), 0.0)
    assert not failed.any()
    assert np.all(sweeps == 1)
    # k~ annihilates constants up to rounding of its row sums
    assert np.allclose(q, u[:, None, :, :], atol=1e-13, rtol=0)


def _poly_density(ops, coeffs):
    return np.polyval(coeffs, ops.xi)


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_linear_flux_gives_exact_translation(N):
    """Euler with u = 1, p = 1 transports density linearly: for rho a degree-N
    polynomial in the cell, q(tau, xi) = rho(xi - c tau), c = dt/dx (closed form);
    nilpotency of L^xi makes the Picard loop exact after N+1 sweeps."""
    ops = basis.build_operators(N)
    e = P.Euler()
    rng = np.random.default_rng(N)
    coeffs = rng.uniform(-0.3, 0.3, N + 1)
    coeffs[-1] = 1.0
    rho = _poly_density(ops, coeffs)[None, :]
    u = np.stack([rho, rho, 2.5 + 0.5 * rho], axis=-1)           # u = 1, p = 1, gamma = 1.4
    dt, dx = 0.004, 0.05
    q, sweeps, failed = predictor.predict(ops, e, u, dt, dx, np.array([0.0]), 0.0)
    c = dt / dx
    exact = np.polyval(coeffs, ops.xi[None, :] - c * ops.xi[:, None])   # [a, j]
    assert not failed.any()
    assert sweeps[0] <= N + 2
    assert np.allclose(q[0, :, :, 0], exact, atol=1e-13)
    assert np.allclose(q[0, :, :, 1], exact, atol=1e-13)
    assert np.allclose(q[0, :, :, 2], 2.5 + 0.5 * exact, atol=1e-13)


@pytest.mark.parametrize("N", [2, 6])
def test_scalar_advection_exact_translation(N):
    ops = basis.build_operators(N)
    adv = P.Advection(a=-1.7)
    coeffs = np.linspace(1, 0.2, N + 1)
    u = _poly_density(ops, coeffs)[None, :, None]
    dt, dx = 0.01, 0.1
    q, sweeps, _ = predictor.predict(ops, adv, u, dt, dx, np.array([0.0]), 0.0)
    exact = np.polyval(coeffs, ops.xi[None, :] + 1.7 * dt / dx * ops.xi[:, None])
    assert np.allclose(q[0, :, :, 0], exact, atol=1e-13)


def _random_euler(N, C, seed):
    rng = np.random.default_rng(seed)
    xs = W.cell_points(C, N + 1)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * xs + rng.uniform(0, 6)) + 0.05 * rng.uniform(-1, 1, xs.shape)
    vel = 0.5 + 0.4 * np.cos(2 * np.pi * xs)
    p = 1.0 + 0.2 * np.sin(4 * np.pi * xs)
    return np.stack([rho, rho * vel, p / 0.4 + 0.5 * rho * vel ** 2], axis=-1)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_picard_matches_brute_force_newton_euler(N):
    ops = basis.build_operators(N)
    e = P.Euler()
    C = 3
    u = _random_euler(N, C, seed=N)
    dx = 1.0 / C
    from oracle.dg import cfl_dt
    dt = cfl_dt(ops, e, u, dx, 0.9)
    q, sweeps, failed = predictor.predict(ops, e, u, dt, dx, dx * np.arange(C), 0.3)
    mats = brute.assemble(ops)
    for c in range(C):
        qb = brute.solve_cell(ops, e, u[c], dt, dx, dx * c, 0.3, mats)
        assert np.abs(q[c] - qb).max() <= 1e-12 * np.abs(qb).max()
    assert not failed.any()


@pytest.mark.parametrize("N", [1, 3])
def test_picard_matches_brute_force_newton_swe(N):
    ops = basis.build_operators(N)
    swe = P.ShallowWater()
    C = 4
    u = W.swe_bump_nodal(C, N)
    u[..., 1] = 0.3 * u[..., 0]                                  # some flow
    u[..., 2] *= 3.0                                             # steeper bathymetry
    dx = 1.0 / C
    lam = float(swe.max_speed(u).max())
    dt = 0.9 * dx / ((2 * N + 1) * lam)
    q, sweeps, failed = predictor.predict(ops, swe, u, dt, dx, dx * np.arange(C), 0.0)
    mats = brute.assemble(ops)
    for c in range(C):
        qb = brute.solve_cell(ops, swe, u[c], dt, dx, dx * c, 0.0, mats)
        assert np.abs(q[c] - qb).max() <= 1e-12 * np.abs(qb).max()
    # bathymetry is static: its coefficients never change
    assert np.array_equal(q[..., 2], np.broadcast_to(u[:, None, :, 2], q[..., 2].shape))


def test_picard_matches_brute_force_newton_source():
    N = 2
    ops = basis.build_operators(N)
    pr = P.EulerReact(omega=3.0)
    u = np.concatenate([_random_euler(N, 2, seed=7),
                        np.full((2, N + 1, 1), 0.8), np.full((2, N + 1, 1), -0.2)], axis=-1)
    dx = 0.5
    dt = 0.05
    q, _, failed = predictor.predict(ops, pr, u, dt, dx, dx * np.arange(2), 0.0)
    mats = brute.assemble(ops)
    qb = brute.solve_cell(ops, pr, u[1], dt, dx, dx, 0.0, mats)
    assert np.abs(q[1] - qb).max() <= 1e-12 * np.abs(qb).max()
    assert not failed.any()


def test_iteration_guard_flags_nonconvergence():
    ops = basis.build_operators(3)
    e = P.Euler()
    u = _random_euler(3, 2, seed=3)
    q, sweeps, failed = predictor.predict(ops, e, u, 0.05, 0.5, np.array([0, 0.5]), 0.0, max_iter=1)
    assert failed.all() and np.all(sweeps == 1)
