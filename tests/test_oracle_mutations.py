"""Planted mistakes: each plausible slip in the oracle must break at least one pin.

The mistakes are planted in copies of the oracle's operator tables or by
replacing one oracle function for the duration of a test (CPU only).  The
pins are quick versions of the ones in the other oracle tests:
brute-force Newton agreement, constant-state preservation, the Pade closed
form of the ODE test, and the density-wave error level.
"""

import copy

import numpy as np
import pytest

from oracle import basis, brute, dg, pade, predictor
from oracle import pde as P
from paper_2409_12483_amd import workloads as W

N = 2


def _pin_brute(ops):
    e = P.Euler()
    xs = W.cell_points(2, N + 1)
    rho = 1 + 0.3 * np.sin(2 * np.pi * xs)
    vel = 0.5 + 0.3 * np.cos(2 * np.pi * xs)
    u = np.stack([rho, rho * vel, 2.5 + 0.5 * rho * vel ** 2], -1)
    q, _, _ = predictor.predict(ops, e, u, 0.02, 0.5, np.array([0, 0.5]), 0.0)
    qb = brute.solve_cell(basis.build_operators(N), e, u[0], 0.02, 0.5, 0.0, 0.0)
    return np.abs(q[0] - qb).max() <= 1e-12


def _pin_constant(ops):
    e = P.Euler()
    u = W.euler_density_wave(5, N, amp=0.0, velocity=0.6)
    x_left = 0.2 * np.arange(5)
    u1 = u
    for s in range(10):
        u1, _, _ = dg.dg_step(ops, e, u1, 0.0, 0.005, 0.2, x_left)
    return np.abs(u1 - u).max() <= 1e-13


def _pin_pade(ops):
    pr = P.EulerReact()
    u = W.euler_react_uniform(1, N)
    dt = 2 * np.pi / 10
    u1, _, _ = dg.dg_step(ops, pr, u, 0.0, dt, 1000.0, np.array([0.0]), max_iter=200)
    closed = pade.oscillator_trajectory(N, 10)[1]
    return np.abs(u1[0, 0, 3:] - closed).max() <= 1e-12


def _density_error(ops):
    e = P.Euler()
    C = 16
    u = W.euler_density_wave(C, N)
    x_left = np.arange(C) / C
    t = 0.0
    for _ in range(40):
        dt = dg.cfl_dt(ops, e, u, 1.0 / C, 0.4)
        u, _, _ = dg.dg_step(ops, e, u, t, dt, 1.0 / C, x_left)
        t += dt
    xs = W.cell_points(C, N + 1)
    return np.abs(u[..., 0] - W.euler_density_wave_exact(xs, t)).max()


REFERENCE_ERROR = None


def _pin_accuracy(ops):
    global REFERENCE_ERROR
    if REFERENCE_ERROR is None:
        REFERENCE_ERROR = _density_error(basis.build_operators(N))
    err = _density_error(ops)
    return np.isfinite(err) and err <= 2.0 * REFERENCE_ERROR


PINS = [_pin_brute, _pin_constant, _pin_pade, _pin_accuracy]


def _all_pins_pass(ops):
    with np.errstate(all="ignore"):
        return all(pin(ops) for pin in PINS)


def test_unmutated_oracle_passes_every_pin():
    assert _all_pins_pass(basis.build_operators(N))


def _mutated(field, fn):
    ops = copy.deepcopy(basis.build_operators(N))
    setattr(ops, field, fn(getattr(ops, field)))
    return ops


@pytest.mark.parametrize("name,make", [
    ("k~ transposed", lambda: _mutated("ktil", lambda a: a.T.copy())),
    ("kappa~ transposed", lambda: _mutated("kappa", lambda a: a.T.copy())),
    ("D~ transposed", lambda: _mutated("Dtil", lambda a: a.T.copy())),
    ("uniform time weights", lambda: _mutated("w", lambda a: np.full_like(a, 1.0 / len(a)))),
    ("k~ sign flipped", lambda: _mutated("ktil", lambda a: -a)),
    ("psi0/psi1 swapped", lambda: (lambda o: (setattr(o, "psi0", o.psi1.copy()),
                                             setattr(o, "psi1", basis.build_operators(N).psi0.copy()), o)[-1])(
        copy.deepcopy(basis.build_operators(N)))),
])
def test_planted_operator_mistake_is_caught(name, make):
    assert not _all_pins_pass(make()), name


def test_planted_sign_error_in_surface_term_is_caught(monkeypatch):
    orig = dg.interface_terms

    def wrong(ops, pde, q, dt, dx):
        G, J = orig(ops, pde, q, dt, dx)
        return -G, J
    monkeypatch.setattr(dg, "interface_terms", wrong)
    assert not _all_pins_pass(basis.build_operators(N))


def test_planted_antidissipative_riemann_solver_is_caught(monkeypatch):
    def wrong(pde, qm, qp):
        s = np.maximum(pde.max_speed(qm), pde.max_speed(qp))
        return 0.5 * (pde.flux(qm) + pde.flux(qp)) + 0.5 * s[..., None] * (qp - qm)
    monkeypatch.setattr(dg, "rusanov", wrong)
    assert not _all_pins_pass(basis.build_operators(N))


def test_planted_missing_source_in_corrector_is_caught(monkeypatch):
    monkeypatch.setattr(dg, "volume_source_terms",
                        lambda ops, pde, q, dt, dx, x_left, t0: np.zeros((q.shape[0], ops.n, q.shape[-1])))
    assert not _all_pins_pass(basis.build_operators(N))
