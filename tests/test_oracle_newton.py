"""Pins of the oracle's Newton inner iterations (Sec. 1.1: for stiff source
terms the inner iterative process of eq. lst_dg_predictor_nested_picards may
use Newton's method instead of Picard's).

* The model's source Jacobian equals central finite differences of its source.
* The ODE problem of Sec. 2.1 (a uniform two-species state: the harmonic
  oscillator) at time steps so large that the inner Picard iteration diverges
  (omega dt beyond the contraction bound of kappa~): with Newton, every step
  equals the (N, N+1) Pade approximant of exp(dt A) (closed form, oracle.pade).
* Where Picard converges, both inner solvers give the same step.
* On tiny non-uniform meshes (flux and source terms both active) the predictor
  with Newton inner iterations matches the brute-force dense Newton solve of
  the assembled space-time system (oracle.brute), which shares none of its code.
"""

import numpy as np
import pytest

from oracle import basis, brute, dg, pade, predictor
from oracle import pde as P
from paper_2409_12483_amd import workloads as W

WIDE = 1000.0     # a spatially uniform ODE test: a wide cell keeps the flux loop stable


def test_source_jacobian_matches_finite_differences():
    pr = P.EulerReact(omega=1.7)
    rng = np.random.default_rng(0)
    Q = rng.uniform(0.5, 2.0, (7, 5))
    J = pr.source_jacobian(Q, None, None)
    h = 1e-6
    for s in range(5):
        e = np.zeros(5)
        e[s] = h
        fd = (pr.source(Q + e, None, None) - pr.source(Q - e, None, None)) / (2 * h)
        assert np.allclose(J[..., :, s], fd, atol=1e-9)


def _ode_run(N, nsteps, inner, max_iter=64):
    ops = basis.build_operators(N)
    pr = P.EulerReact(omega=1.0)
    u = W.euler_react_uniform(1, N)
    dt = 2 * np.pi / nsteps
    t, failed_any = 0.0, False
    for _ in range(nsteps):
        q, _, failed = predictor.predict(ops, pr, u, dt, WIDE, np.array([0.0]), t, max_iter=max_iter,
                                         inner=inner)
        failed_any |= bool(failed.any())
        u = dg.dg_correct(ops, pr, u, q, dt, WIDE, np.array([0.0]), t)
        t += dt
    return u, failed_any


@pytest.mark.parametrize("N,nsteps", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (4, 1)])
def test_newton_steps_equal_pade_where_picard_diverges(N, nsteps):
    with np.errstate(all="ignore"):
        _, picard_failed = _ode_run(N, nsteps, "picard")
    assert picard_failed                       # the case is stiff for the Picard inner loop
    u, failed = _ode_run(N, nsteps, "newton")
    assert not failed
    closed = pade.oscillator_trajectory(N, nsteps)[-1]
    assert np.abs(u[0, :, 3:] - closed).max() <= 1e-13


@pytest.mark.parametrize("N", [1, 3, 5])
def test_newton_and_picard_agree_where_both_converge(N):
    a, fa = _ode_run(N, 12, "picard")
    b, fb = _ode_run(N, 12, "newton")
    assert not fa and not fb
    assert np.abs(a - b).max() <= 1e-13


@pytest.mark.parametrize("N", [1, 2, 3])
def test_newton_predictor_matches_brute_force(N):
    ops = basis.build_operators(N)
    pr = P.EulerReact(omega=3.0)
    C = 3
    xs = W.cell_points(C, N + 1)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * xs)
    vel = 0.6 + 0.2 * np.cos(2 * np.pi * xs)
    base = np.stack([rho, rho * vel, 2.5 + 0.5 * rho * vel ** 2], axis=-1)
    u = np.concatenate([base, (0.7 * rho)[..., None], (0.2 * rho)[..., None]], axis=-1)
    dx, dt = 1.0 / C, 0.02
    q, _, failed = predictor.predict(ops, pr, u, dt, dx, dx * np.arange(C), 0.1, inner="newton")
    assert not failed.any()
    mats = brute.assemble(ops)
    for c in range(C):
        qb = brute.solve_cell(ops, pr, u[c], dt, dx, dx * c, 0.1, mats)
        assert np.abs(q[c] - qb).max() <= 1e-12 * max(1.0, np.abs(qb).max())


def test_newton_rejects_models_it_does_not_serve():
    ops = basis.build_operators(2)
    with pytest.raises(ValueError):
        predictor.predict(ops, P.ShallowWater(), W.swe_bump_nodal(4, 2), 0.01, 0.25,
                          0.25 * np.arange(4), 0.0, inner="newton")
