"""Planted mistakes in the 2-D and 3-D oracles (DG and ADER-WENO): each must
break at least one pin.

Each mistake is planted for the duration of one test, by a copy of the
operator tables or by replacing one oracle function or model method (CPU
only).  The pins are quick versions of those in test_oracle_dg2d.py and
test_oracle_dg3d.py: reduction of one-dimensional data to the pinned lower
dimension along each axis on a domain of unequal sides, uniform-state
preservation, conservation, and the 1/d factor of the time step.
"""

import copy

import numpy as np
import pytest

from oracle import basis, dg, dg2d, dg3d
from oracle import pde as P
from paper_2409_12483_amd import workloads as W

N = 2


def _pins_2d(ops):
    """Names of the 2-D pins that hold for the (possibly mutated) oracle."""
    e2 = dg2d.Euler2D()
    ok = []
    L = 0.7
    u1 = W.euler_density_wave(6, N, amp=0.2, noise=1e-3, seed=1, x1=L)
    dt = 1e-3
    r1, _, _ = dg.dg_run(basis.build_operators(N), P.Euler(), u1, 0.0, L, fixed_dt=dt, nsteps=2)
    for axis in (0, 1):
        u2 = np.zeros((6, 2, N + 1, N + 1, 4)) if axis == 0 else np.zeros((2, 6, N + 1, N + 1, 4))
        mom = 1 if axis == 0 else 2
        src = u1[:, None, :, None, :] if axis == 0 else u1[None, :, None, :, :]
        u2[..., 0], u2[..., mom], u2[..., 3] = src[..., 0], src[..., 1], src[..., 2]
        ext = (0.0, L, 0.0, 0.4) if axis == 0 else (0.0, 0.4, 0.0, L)
        r2, _, _ = dg2d.dg2d_run(ops, e2, u2, extent=ext, fixed_dt=dt, nsteps=2)
        ref = r1[:, None, :, None, :] if axis == 0 else r1[None, :, None, :, :]
        if np.abs(r2[..., [0, mom, 3]] - ref).max() <= 1e-12:
            ok.append(f"reduce{axis}")
    u = W.euler2d_sine_wave(3, 3, N, amp=0.0, velocity=(0.6, -0.4))
    r, _, _ = dg2d.dg2d_run(ops, e2, u, nsteps=2)
    if np.abs(r - u).max() <= 1e-13:
        ok.append("uniform")
    u = W.euler2d_sine_wave(4, 3, N, noise=1e-2, seed=2, velocity=(0.6, -0.4), y1=0.8)
    r, _, _ = dg2d.dg2d_run(ops, e2, u, nsteps=2, extent=(0, 1, 0, 0.8))
    b = dg2d.conserved_totals2d(basis.build_operators(N), u, 1 / 4, 0.8 / 3)
    a = dg2d.conserved_totals2d(basis.build_operators(N), r, 1 / 4, 0.8 / 3)
    if np.abs(a - b).max() <= 1e-13:
        ok.append("conserve")
    uc = W.euler_density_wave(5, N, amp=0.3)
    dt1 = dg.cfl_dt(basis.build_operators(N), P.Euler(), uc, 0.2, 0.4)
    u2 = np.zeros((5, 5, N + 1, N + 1, 4))
    u2[..., 0], u2[..., 1], u2[..., 3] = (uc[:, None, :, None, k] for k in range(3))
    if abs(dg2d.cfl_dt2d(ops, e2, u2, 0.2, 0.2, 0.4) - dt1 / 2) <= 1e-15 * dt1:
        ok.append("cfl")
    return ok


ALL_2D = {"reduce0", "reduce1", "uniform", "conserve", "cfl"}


def test_unmutated_2d_oracle_passes_every_pin():
    assert set(_pins_2d(basis.build_operators(N))) == ALL_2D


MUTATIONS_2D = {
    "transposed k~": lambda m, o: setattr(o, "ktil", o.ktil.T.copy()),
    "transposed kappa~": lambda m, o: setattr(o, "kappa", o.kappa.T.copy()),
    "transposed D~": lambda m, o: setattr(o, "Dtil", o.Dtil.T.copy()),
    "swapped face values psi / psi~": lambda m, o: (setattr(o, "psi0", o.psi1.copy()),
                                                    setattr(o, "psi1", basis.build_operators(N).psi0.copy())),
    "y flux with the x scaling": lambda m, o: m.setattr(
        dg2d, "predict2d", (lambda f: lambda ops, pde, u, dt, dx, dy, *a: f(ops, pde, u, dt, dx, dx, *a))(dg2d.predict2d)),
    "corrector y terms with the x scaling": lambda m, o: m.setattr(
        dg2d, "correct2d", (lambda f: lambda ops, pde, u, q, dt, dx, dy: f(ops, pde, u, q, dt, dx, dx))(dg2d.correct2d)),
    "y Riemann flux with the x flux": lambda m, o: m.setattr(dg2d, "rusanov_y", dg2d.rusanov_x),
    "y flux with swapped momenta": lambda m, o: m.setattr(
        dg2d.Euler2D, "flux_y", lambda self, Q: dg2d.Euler2D.flux_x(self, Q[..., [0, 2, 1, 3]])),
    "time step without the 1/d factor": lambda m, o: m.setattr(
        dg2d, "cfl_dt2d", (lambda f: lambda *a: 2.0 * f(*a))(dg2d.cfl_dt2d)),
    "y surface term with the wrong sign": lambda m, o: m.setattr(
        dg2d, "rusanov_y", (lambda f: lambda pde, qm, qp: -f(pde, qm, qp))(dg2d.rusanov_y)),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS_2D))
def test_planted_2d_mistake_breaks_a_pin(name, monkeypatch):
    ops = copy.deepcopy(basis.build_operators(N))
    MUTATIONS_2D[name](monkeypatch, ops)
    held = set(_pins_2d(ops))
    assert held != ALL_2D, f"{name}: every pin still holds"


def _pins_3d(ops):
    """Names of the 3-D pins that hold: reduction to the (pinned) 2-D oracle along each axis."""
    e3, e2 = dg3d.Euler3D(), dg2d.Euler2D()
    ok = []
    lengths = [0.9, 0.7, 0.5]
    vars_of = {0: (2, 3), 1: (1, 3), 2: (1, 2)}
    ops2 = basis.build_operators(N)
    for axis in range(3):
        keep = [d for d in range(3) if d != axis]
        u2 = W.euler2d_sine_wave(3, 2, N, noise=1e-2, seed=axis, velocity=(0.7, -0.4),
                                 x1=lengths[keep[0]], y1=lengths[keep[1]])
        r2, _, _ = dg2d.dg2d_run(ops2, e2, u2, extent=(0, lengths[keep[0]], 0, lengths[keep[1]]),
                                 fixed_dt=1e-3, nsteps=2)
        a, b = vars_of[axis]

        def embed(x):
            src = np.expand_dims(np.expand_dims(x, axis), 3 + axis)
            shape = [3, 2]
            shape.insert(axis, 2)
            out = np.zeros(tuple(shape) + (N + 1,) * 3 + (5,))
            out[..., 0], out[..., a], out[..., b], out[..., 4] = src[..., 0], src[..., 1], src[..., 2], src[..., 3]
            return out
        r3, _, _ = dg3d.dg3d_run(ops, e3, embed(u2), extent=tuple(lengths), fixed_dt=1e-3, nsteps=2)
        if np.abs(r3 - embed(r2)).max() <= 1e-12:
            ok.append(f"reduce{axis}")
    u = W.euler3d_sine_wave(2, 2, 2, N, noise=1e-2, seed=3, velocity=(0.3, -0.5, 0.8))
    r, _, _ = dg3d.dg3d_run(ops, e3, u, nsteps=2)
    h = (0.5, 0.5, 0.5)
    if np.abs(dg3d.conserved_totals3d(ops2, r, h) - dg3d.conserved_totals3d(ops2, u, h)).max() <= 1e-13:
        ok.append("conserve")
    return ok


ALL_3D = {"reduce0", "reduce1", "reduce2", "conserve"}


def test_unmutated_3d_oracle_passes_every_pin():
    assert set(_pins_3d(basis.build_operators(N))) == ALL_3D


MUTATIONS_3D = {
    "transposed k~": lambda m, o: setattr(o, "ktil", o.ktil.T.copy()),
    "transposed D~": lambda m, o: setattr(o, "Dtil", o.Dtil.T.copy()),
    "swapped face values psi / psi~": lambda m, o: (setattr(o, "psi0", o.psi1.copy()),
                                                    setattr(o, "psi1", basis.build_operators(N).psi0.copy())),
    "z flux with the y scaling": lambda m, o: m.setattr(
        dg3d, "predict3d", (lambda f: lambda ops, pde, u, dt, h, *a: f(ops, pde, u, dt, (h[0], h[1], h[1]), *a))(dg3d.predict3d)),
    "z Riemann flux along y": lambda m, o: m.setattr(
        dg3d, "rusanov", (lambda f: lambda pde, qm, qp, d: f(pde, qm, qp, 1 if d == 2 else d))(dg3d.rusanov)),
    "flux pressure on the wrong momentum": lambda m, o: m.setattr(
        dg3d.Euler3D, "flux", (lambda f: lambda self, Q, d: f(self, Q, d)[..., [0, 1, 3, 2, 4]] if d == 2 else f(self, Q, d))(dg3d.Euler3D.flux)),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS_3D))
def test_planted_3d_mistake_breaks_a_pin(name, monkeypatch):
    ops = copy.deepcopy(basis.build_operators(N))
    MUTATIONS_3D[name](monkeypatch, ops)
    held = set(_pins_3d(ops))
    assert held != ALL_3D, f"{name}: every pin still holds"


# 2-D ADER-WENO finite volumes: the tensor-polynomial exactness of the
# reconstruction, the reduction to the 1-D scheme, and conservation


def _pins_fv2d():
    from oracle import fv, fv2d
    from oracle import pde as P1
    N = 2
    ops = basis.build_operators(N)
    ok = True
    # reconstruction of x*y (degree 1 per direction, exact for degree 2)
    Cx, Cy = 8, 8
    e = np.linspace(0, 1, Cx + 1)
    ax = (e[1:] ** 2 - e[:-1] ** 2) / 2 * Cx
    v = (ax[:, None] * ax[None, :])[..., None]
    w = fv2d.reconstruct2d(v, ops)
    xs = W.cell_points(Cx, N + 1)
    exact = xs[:, None, :, None] * xs[None, :, None, :]
    ok &= np.abs(w[2:-2, 2:-2, :, :, 0] - exact[2:-2, 2:-2]).max() <= 1e-12
    # x-only flow against the 1-D scheme
    C, dt = 16, 0.004
    x = (np.arange(C) + 0.5) / C
    rho = 1 + 0.3 * np.sin(2 * np.pi * x)
    v1 = np.stack([rho, 0.5 * rho, 1 / 0.4 + 0.125 * rho], -1)
    v2 = np.zeros((C, 3, 4))
    v2[..., 0], v2[..., 1], v2[..., 3] = rho[:, None], 0.5 * rho[:, None], v1[:, None, 2]
    ref, _, _ = fv.fv_step(ops, P1.Euler(), v1, 0.0, dt, 1 / C, np.arange(C) / C)
    got, _, _ = fv2d.fv2d_step(ops, dg2d.Euler2D(), v2, dt, 1 / C, 1 / 3)
    ok &= np.abs(got[..., [0, 1, 3]] - ref[:, None, :]).max() <= 1e-13
    # conservation on a 2-D wave
    v0 = W.euler2d_sine_averages(6, 5)
    vn, _, _ = fv2d.fv2d_step(ops, dg2d.Euler2D(), v0, 0.002, 1 / 6, 1 / 5)
    ok &= np.abs(vn.sum(axis=(0, 1)) - v0.sum(axis=(0, 1))).max() <= 1e-12
    return bool(ok)


def test_unmutated_fv2d_oracle_passes_its_pins():
    assert _pins_fv2d()


def test_planted_fv2d_mistakes_break_a_pin(monkeypatch):
    from oracle import fv2d
    orig = fv2d.reconstruct2d

    def x_only(v, ops):            # the y sweep forgotten: x reconstruction broadcast along y
        from oracle import weno
        wx = np.stack([weno.reconstruct(v[:, iy, :], ops) for iy in range(v.shape[1])], axis=1)
        return np.repeat(wx[:, :, :, None, :], ops.n, axis=3)
    monkeypatch.setattr(fv2d, "reconstruct2d", x_only)
    assert not _pins_fv2d()
    monkeypatch.setattr(fv2d, "reconstruct2d", orig)
    orig_rx = fv2d.rusanov_x
    monkeypatch.setattr(fv2d, "rusanov_x", lambda pde, qm, qp: orig_rx(pde, qp, qm))   # face states swapped
    assert not _pins_fv2d()


# 3-D ADER-WENO finite volumes: the reconstruction's exactness for a
# trilinear product, the reduction to the pinned 2-D scheme along z, the
# closed-form time step on a uniform state, and conservation


def _pins_fv3d():
    from oracle import fv2d, fv3d
    N = 2
    ops = basis.build_operators(N)
    e3 = dg3d.Euler3D()
    ok = True
    # reconstruction of x*y*z (degree 1 per direction, exact for degree 2)
    C = 7
    e = np.linspace(0, 1, C + 1)
    ax = (e[1:] ** 2 - e[:-1] ** 2) / 2 * C
    v = (ax[:, None, None] * ax[None, :, None] * ax[None, None, :])[..., None]
    w = fv3d.reconstruct3d(v, ops)
    xs = W.cell_points(C, N + 1)
    exact = xs[:, None, None, :, None, None] * xs[None, :, None, None, :, None] * xs[None, None, :, None, None, :]
    s = slice(2, C - 2)
    ok &= np.abs(w[s, s, s, :, :, :, 0] - exact[s, s, s]).max() <= 1e-12
    # flow in the x-y plane, constant along z, against the 2-D scheme
    v2 = W.euler2d_sine_averages(6, 5, velocity=(0.7, -0.4))
    dt = 0.003
    ref, _, _ = fv2d.fv2d_step(ops, dg2d.Euler2D(), v2, dt, 1 / 6, 1 / 5)
    v3 = np.zeros((6, 5, 3, 5))
    v3[..., 0], v3[..., 1], v3[..., 2], v3[..., 4] = (v2[..., k][:, :, None] for k in range(4))
    got, _, _ = fv3d.fv3d_step(ops, e3, v3, dt, (1 / 6, 1 / 5, 1 / 3))
    ok &= np.abs(got[..., [0, 1, 2, 4]] - ref[:, :, None, :]).max() <= 1e-13
    # Sec. 1.5 with d = 3 on a uniform state: CFL / 3 * min_d h_d / (|u_d| + c)
    q = np.array([1.2, 0.6, -0.3, 0.24, 2.9])
    u = np.tile(q, (3, 3, 3, 1))
    c = np.sqrt(1.4 * 0.4 * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]) / q[0])
    hh = (0.1, 0.2, 0.05)
    want = 0.4 / 3 * min(hh[d] / (abs(q[1 + d] / q[0]) + c) for d in range(3))
    ok &= abs(fv3d.fv3d_dt(e3, u, hh, 0.4) - want) <= 1e-15 * want
    # conservation of the five totals
    v0 = W.euler3d_sine_averages(5, 4, 3)
    vn, _, _ = fv3d.fv3d_step(ops, e3, v0, 0.002, (1 / 5, 1 / 4, 1 / 3))
    ok &= np.abs(vn.sum(axis=(0, 1, 2)) - v0.sum(axis=(0, 1, 2))).max() <= 1e-12
    return bool(ok)


def test_unmutated_fv3d_oracle_passes_its_pins():
    assert _pins_fv3d()


def test_planted_fv3d_mistakes_break_a_pin(monkeypatch):
    from oracle import fv3d

    def no_z_sweep(v, ops):        # the z sweep forgotten: the x-y reconstruction broadcast along z
        wy = fv3d._along(fv3d._along(v, ops, 0), ops, 1)
        return np.repeat(wy[..., None, :], ops.n, axis=-2)
    monkeypatch.setattr(fv3d, "reconstruct3d", no_z_sweep)
    assert not _pins_fv3d()
    monkeypatch.undo()
    orig_rs = fv3d.rusanov
    monkeypatch.setattr(fv3d, "rusanov", lambda pde, qm, qp, d: orig_rs(pde, qp, qm, d))   # face states swapped
    assert not _pins_fv3d()
    monkeypatch.undo()
    monkeypatch.setattr(fv3d, "fv3d_dt", lambda pde, v, h, cfl: cfl / 2.0 * min(
        h[d] / float(pde.speed(v, d).max()) for d in range(3)))                               # d = 2 factor
    assert not _pins_fv3d()
