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

from oracle import basis, brute, dg, fv, limiter, pade, predictor
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


# ------------------------------------------------------------ shallow water ----
# Quick versions of the pins in test_oracle_swe.py: the DG lake at rest over a
# piecewise-linear bathymetry, the first step over a step bathymetry (momentum
# stays zero), the FV lake at rest at fifth order, and the FV time step of a
# uniform state.  The shallow-water mistakes below must each break one of them.

def _swe_pin_dg_linear_lake():
    swe = P.ShallowWater()
    u = W.swe_lake_at_rest_nodal(8, 2, kind="linear")
    u1, _, _ = dg.dg_run(basis.build_operators(2), swe, u, 0.0, 1.0, cfl=0.4, nsteps=10)
    return np.abs(u1[..., 1]).max() <= 1e-13


def _swe_pin_dg_step_lake():
    swe = P.ShallowWater()
    u = W.swe_lake_at_rest_nodal(8, 1, kind="step")
    u1, _, _ = dg.dg_run(basis.build_operators(1), swe, u, 0.0, 1.0, cfl=0.4, nsteps=1)
    return np.abs(u1[..., 1]).max() <= 1e-14


def _swe_pin_fv_lake_order():
    swe = P.ShallowWater()
    ops = basis.build_operators(4)
    errs = []
    for C in (64, 128):
        v = W.swe_lake_at_rest_averages(C)
        v1, _, _ = fv.fv_run(ops, swe, v, 0.0, 1.0, cfl=0.4, t_end=0.02)
        errs.append(np.abs(v1[:, 1]).max())
    return np.isfinite(errs).all() and np.log2(errs[0] / errs[1]) >= 4.5 and errs[1] <= 3e-6


def _swe_pin_fv_dt():
    swe = P.ShallowWater()
    v = np.tile([1.3, 0.39, 0.2], (20, 1))
    _, _, info = fv.fv_run(basis.build_operators(4), swe, v, 0.0, 1.0, cfl=0.4, nsteps=1)
    expect = 0.4 * 0.05 / (0.3 + np.sqrt(9.81 * 1.3))
    return abs(info["dts"][0] - expect) <= 1e-15 * expect


SWE_PINS = [_swe_pin_dg_linear_lake, _swe_pin_dg_step_lake, _swe_pin_fv_lake_order, _swe_pin_fv_dt]


def _all_swe_pins_pass():
    with np.errstate(all="ignore"):
        return all(pin() for pin in SWE_PINS)


def test_unmutated_oracle_passes_every_shallow_water_pin():
    assert _all_swe_pins_pass()


def test_planted_sign_error_in_volume_non_conservative_term_is_caught(monkeypatch):
    # the corrector's volume term with + (dt/dx) B(q) dq instead of - (shared by DG and FV)
    def wrong(ops, pde, q, dt, dx, x_left, t0):
        sb = np.zeros_like(q)
        if pde.has_ncp:
            dq = np.einsum("lj,cajr->calr", ops.ktil, q)
            sb = sb + (dt / dx) * pde.ncp(q, dq)
        return np.einsum("a,cakr->ckr", ops.w, sb)
    monkeypatch.setattr(dg, "volume_source_terms", wrong)
    monkeypatch.setattr(fv, "volume_source_terms", wrong)
    assert not _all_swe_pins_pass()


def test_planted_doubled_non_conservative_product_is_caught(monkeypatch):
    orig = P.ShallowWater.ncp
    monkeypatch.setattr(P.ShallowWater, "ncp", lambda self, Q, dQ: 2.0 * orig(self, Q, dQ))
    assert not _all_swe_pins_pass()


@pytest.mark.parametrize("factor", [-1.0, 0.0, 2.0])
def test_planted_wrong_path_conservative_jump_is_caught(monkeypatch, factor):
    orig = P.ShallowWater.ncp_jump
    monkeypatch.setattr(P.ShallowWater, "ncp_jump", lambda self, a, b: factor * orig(self, a, b))
    assert not _all_swe_pins_pass()


def test_planted_halved_finite_volume_time_step_is_caught(monkeypatch):
    orig = fv.fv_dt
    monkeypatch.setattr(fv, "fv_dt", lambda pde, v, dx, cfl: 0.5 * orig(pde, v, dx, cfl))
    assert not _all_swe_pins_pass()


# ------------------------------------------------------- Newton inner loop ----
def _newton_pade_pin():
    ops = basis.build_operators(2)
    pr = P.EulerReact(omega=1.0)
    u = W.euler_react_uniform(1, 2)
    dt = 2 * np.pi
    q, _, failed = predictor.predict(ops, pr, u, dt, 1000.0, np.array([0.0]), 0.0, inner="newton")
    u1 = dg.dg_correct(ops, pr, u, q, dt, 1000.0, np.array([0.0]), 0.0)
    closed = pade.oscillator_trajectory(2, 1)[-1]
    return (not failed.any()) and np.abs(u1[0, :, 3:] - closed).max() <= 1e-13


def test_unmutated_newton_passes_its_pin():
    assert _newton_pade_pin()


@pytest.mark.parametrize("mutate", [lambda J: -J, lambda J: np.swapaxes(J, -1, -2), lambda J: 0.5 * J])
def test_planted_wrong_source_jacobian_is_caught(monkeypatch, mutate):
    orig = P.EulerReact.source_jacobian
    monkeypatch.setattr(P.EulerReact, "source_jacobian", lambda self, Q, x, t: mutate(orig(self, Q, x, t)))
    with np.errstate(all="ignore"):
        assert not _newton_pade_pin()


# the subcell limiter: R P = 1, exact conservation through limited steps on a
# periodic mesh, and no limiting of smooth flow


def _lim_pin_left_inverse():
    ops = basis.build_operators(N)
    return np.abs(limiter.subcell_R(ops) @ ops.P - np.eye(N + 1)).max() <= 1e-11


def _lim_pin_conservation():
    ops = basis.build_operators(N)
    u0 = W.riemann_nodal(10, N, 1)
    with np.errstate(all="ignore"):
        u, _, info = limiter.limited_run(ops, P.Euler(), u0, 0.0, 1.0, cfl=0.4, nsteps=16, dims=2)
    tot = lambda a: np.einsum("k,ckm->m", ops.w, a)
    return min(info["troubled"]) > 0 and np.abs(tot(u) - tot(u0)).max() <= 1e-13


def _lim_pin_smooth():
    ops = basis.build_operators(N)
    _, _, info = limiter.limited_run(ops, P.Euler(), W.euler_density_wave(16, N), 0.0, 1.0, cfl=0.4, nsteps=6)
    return sum(info["troubled"]) == 0


def _all_limiter_pins_pass():
    return _lim_pin_left_inverse() and _lim_pin_conservation() and _lim_pin_smooth()


def test_unmutated_limiter_passes_its_pins():
    assert _all_limiter_pins_pass()


def test_planted_transposed_reconstruction_is_caught(monkeypatch):
    monkeypatch.setattr(limiter, "subcell_R", lambda ops: ops.P.T * (N + 1) / (2 * N + 1))
    assert not _all_limiter_pins_pass()


def test_planted_face_shift_in_subgrid_fluxes_is_caught(monkeypatch):
    orig = limiter.fv_subgrid

    def shifted(*a, **k):
        v, g = orig(*a, **k)
        return v, np.roll(g, 1, axis=0)
    monkeypatch.setattr(limiter, "fv_subgrid", shifted)
    assert not _all_limiter_pins_pass()


def test_planted_missing_nad_tolerance_is_caught(monkeypatch):
    monkeypatch.setattr(limiter, "DELTA0", 0.0)
    monkeypatch.setattr(limiter, "EPS0", 0.0)
    assert not _all_limiter_pins_pass()
