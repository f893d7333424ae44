"""The limited 2-D step (include/aderdg_lim2d.h) on the GPU against the
oracle (oracle/limiter2d.py), through the C ABI.

* The cylindrical explosion of Sec. 2.2 (troubled cells along the circle),
  periodic and free-outflow boundaries, N = 1, 2, 3, 5 and 9, and on cells of
  unequal sides: the state, the subcell averages and the time after several
  steps to 1e-12 relative (max norm), the troubled cells of the last step
  equal.
* A Table 9 Riemann problem constant along y (and along x): the same.
* A uniform state: kept, nothing troubled.
* Invalid configurations are refused.
"""

import ctypes

import numpy as np
import pytest

from oracle import basis, dg2d, limiter2d
from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import BIG, torch_dev

pytestmark = pytest.mark.gpu
E2 = dg2d.Euler2D()


def _say(*a):
    print("[case]", *a, flush=True)


def gpu_lim(u0, N, bc, nsteps, extent=(-1.0, 1.0, -1.0, 1.0), t_end=BIG):
    torch, dev = torch_dev()
    cx, cy = u0.shape[:2]
    Ns = 2 * N + 1
    h = abi.aderdg2d_lim_init(abi.lim2d_config(N, cx, cy, bc=bc, extent=extent))
    try:
        u = torch.tensor(np.ascontiguousarray(u0), dtype=torch.float64, device=dev)
        v = torch.zeros((cx, cy, Ns, Ns, 4), dtype=torch.float64, device=dev)
        tr = torch.zeros((cx, cy), dtype=torch.int32, device=dev)
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        te = torch.tensor([t_end], dtype=torch.float64, device=dev)
        dt = torch.zeros(1, dtype=torch.float64, device=dev)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        abi.aderdg2d_lim_project(h, u, v)
        abi.aderdg2d_lim_step(h, u, v, tr, t, te, dt, st, nsteps)
        torch.cuda.synchronize()
        cnt = abi.aderdg2d_lim_counters(h)
        return (u.cpu().numpy(), v.cpu().numpy(), tr.cpu().numpy().astype(bool), float(t[0]), int(st[0]), cnt)
    finally:
        abi.aderdg2d_lim_free(h)


def oracle_lim(u0, N, bc, nsteps, extent=(-1.0, 1.0, -1.0, 1.0)):
    ops = basis.build_operators(N)
    u = np.array(u0, dtype=np.float64)
    x0, x1, y0, y1 = extent
    dx, dy = (x1 - x0) / u.shape[0], (y1 - y0) / u.shape[1]
    t, v, bad, total = 0.0, None, None, 0
    for _ in range(nsteps):
        dt = dg2d.cfl_dt2d(ops, E2, u, dx, dy, 0.4)
        with np.errstate(all="ignore"):
            u, bad, v = limiter2d.limited_step2d(ops, E2, u, dt, dx, dy, "periodic" if bc == abi.LIM_PERIODIC
                                                 else "transmissive", 1, v)
        total += int(bad.sum())
        t += dt
    return u, v, bad, t, total


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _check(u0, N, bc, nsteps, extent=(-1.0, 1.0, -1.0, 1.0)):
    u, v, tr, t, st, cnt = gpu_lim(u0, N, bc, nsteps, extent)
    ru, rv, rbad, rt, total = oracle_lim(u0, N, bc, nsteps, extent)
    assert st == 0
    assert t == pytest.approx(rt, rel=1e-13)
    assert (tr == rbad).all()
    assert cnt[0] == total
    assert _rel(u, ru) <= 1e-12
    assert _rel(v, rv) <= 1e-12
    return total


@pytest.mark.parametrize("N,C,bc,nsteps", [(2, 10, abi.LIM_PERIODIC, 4), (2, 10, abi.LIM_TRANSMISSIVE, 4),
                                           (1, 12, abi.LIM_TRANSMISSIVE, 5), (3, 8, abi.LIM_TRANSMISSIVE, 3),
                                           (5, 6, abi.LIM_TRANSMISSIVE, 2), (9, 4, abi.LIM_TRANSMISSIVE, 1)])
def test_explosion_matches_oracle(N, C, bc, nsteps):
    _say("lim2d explosion", N, C, bc, nsteps)
    total = _check(W.euler2d_explosion_nodal(C, C, N), N, bc, nsteps)
    assert total > 0


def _rows(u1, Cy):
    C, n, _ = u1.shape
    u2 = np.zeros((C, Cy, n, n, 4))
    u2[..., 0], u2[..., 1], u2[..., 3] = (u1[:, None, :, None, k] for k in range(3))
    return u2


@pytest.mark.parametrize("axis", [0, 1])
def test_riemann_problem_along_each_axis(axis):
    _say("lim2d riemann", axis)
    N, C, Cy = 3, 24, 3
    u2 = _rows(W.riemann_nodal(C, N, 1), Cy)
    extent = (0.0, 1.0, 0.0, 0.7)
    if axis == 1:
        u2 = np.ascontiguousarray(np.swapaxes(np.swapaxes(u2, 0, 1), 2, 3)[..., [0, 2, 1, 3]])
        extent = (0.0, 0.7, 0.0, 1.0)
    assert _check(u2, N, abi.LIM_TRANSMISSIVE, 3, extent) > 0


def test_uniform_state_is_kept():
    _say("lim2d uniform")
    N = 3
    u0 = np.tile([1.2, 0.3, -0.2, 2.9], (5, 6, N + 1, N + 1, 1))
    for bc in (abi.LIM_PERIODIC, abi.LIM_TRANSMISSIVE):
        u, v, tr, t, st, cnt = gpu_lim(u0, N, bc, 4, extent=(0.0, 1.0, 0.0, 1.0))
        assert st == 0 and not tr.any() and cnt[0] == 0
        assert np.abs(u - u0).max() <= 1e-13


def test_invalid_configs_are_refused():
    lib = abi.load()
    for mut in (lambda c: setattr(c, "N", 0), lambda c: setattr(c, "N", 10), lambda c: setattr(c, "bc", 5),
                lambda c: setattr(c, "cells_x", 2), lambda c: setattr(c, "cfl", 0.0),
                lambda c: setattr(c, "gamma", 1.0), lambda c: setattr(c, "reserved", 1),
                lambda c: setattr(c, "x1", -2.0)):
        cfg = abi.lim2d_config(2, 8, 8)
        mut(cfg)
        h = ctypes.c_void_p()
        assert lib.aderdg2d_lim_init(ctypes.byref(cfg), None, ctypes.byref(h)) == abi.ADERDG_E_INVAL


@pytest.mark.parametrize("bc", [abi.LIM_PERIODIC, abi.LIM_TRANSMISSIVE])
def test_explosion_to_the_final_time(bc):
    """N = 2 on 21^2 cells to t_final = 0.25 (Sec. 2.2): status 0, every node and
    subcell admissible, the totals kept to rounding with periodic boundaries."""
    _say("lim2d explosion to t_final", bc)
    torch, dev = torch_dev()
    N, C = 2, 21
    Ns = 2 * N + 1
    u0 = W.euler2d_explosion_nodal(C, C, N)
    h = abi.aderdg2d_lim_init(abi.lim2d_config(N, C, C, bc=bc))
    try:
        u = torch.tensor(u0, device=dev)
        v = torch.zeros((C, C, Ns, Ns, 4), dtype=torch.float64, device=dev)
        tr = torch.zeros((C, C), dtype=torch.int32, device=dev)
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        te = torch.full((1,), 0.25, dtype=torch.float64, device=dev)
        dt = torch.zeros(1, dtype=torch.float64, device=dev)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        abi.aderdg2d_lim_project(h, u, v)
        for _ in range(40):
            abi.aderdg2d_lim_step(h, u, v, tr, t, te, dt, st, 64)
            torch.cuda.synchronize()
            if float(t[0]) >= 0.25 or int(st[0]) != 0:
                break
        assert int(st[0]) == 0 and float(t[0]) == 0.25
        cnt = abi.aderdg2d_lim_counters(h)
        assert cnt[0] > 0
    finally:
        abi.aderdg2d_lim_free(h)
    un, vn = u.cpu().numpy(), v.cpu().numpy()
    assert E2.admissible(un).all() and E2.admissible(vn).all()
    if bc == abi.LIM_PERIODIC:
        ops = basis.build_operators(N)
        h2 = 2.0 / C
        a, b = dg2d.conserved_totals2d(ops, u0, h2, h2), dg2d.conserved_totals2d(ops, un, h2, h2)
        assert np.abs(b - a).max() <= 1e-12 * np.abs(a).max()


# L1 density error of the 1-D oracle at N = 9, 50 cells, CFL 0.4, d = 2, t = 0.15
# (the limited 1-D step's Table 9 runs; the 2-D oracle reduces to it on data
# constant along y)
ORACLE_L1_1D = {1: 1.26e-3, 2: 4.64e-3, 3: 2.60e-3, 4: 1.40e-3}


@pytest.mark.parametrize("test", [1, 2, 3, 4])
def test_table9_on_the_papers_two_dimensional_mesh(test):
    """Table 9 as the paper runs it (Sec. 2.2): the one-dimensional Riemann
    problem on a 50 x 10 two-dimensional mesh, N = 9, free outflow, t = 0.15:
    status 0, rho v small, and the L1 density error of every row against the
    exact solution within 1.5x of the 1-D oracle's.  The rows are not bitwise
    equal: (P (x) P) u of data constant along y is constant only to rounding
    across a cell's subcell rows, the boundary rows see their mirrored halo in
    reverse order (7e-16 after the first step), and the limiter's threshold
    decisions amplify such differences over the 1600 steps (measured: 3e-2
    at one node of the shock, 8.7e-4 in L1 between rows in the Sod problem,
    against its L1 error of 1.3e-3); so the rows are compared in the L1 norm
    against the error itself: they differ from each other by less than from
    the exact solution."""
    from oracle import riemann
    _say("lim2d Table 9 on 50 x 10", test)
    torch, dev = torch_dev()
    N, C, Cy, T_END = 9, 50, 10, 0.15
    Ns = 2 * N + 1
    u0 = _rows(W.riemann_nodal(C, N, test), Cy)
    h = abi.aderdg2d_lim_init(abi.lim2d_config(N, C, Cy, extent=(0.0, 1.0, 0.0, 0.2)))
    try:
        u = torch.tensor(u0, device=dev)
        v = torch.zeros((C, Cy, Ns, Ns, 4), dtype=torch.float64, device=dev)
        tr = torch.zeros((C, Cy), dtype=torch.int32, device=dev)
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        te = torch.full((1,), T_END, dtype=torch.float64, device=dev)
        dt = torch.zeros(1, dtype=torch.float64, device=dev)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        abi.aderdg2d_lim_project(h, u, v)
        for _ in range(40):
            abi.aderdg2d_lim_step(h, u, v, tr, t, te, dt, st, 256)
            torch.cuda.synchronize()
            if float(t[0]) >= T_END or int(st[0]) != 0:
                break
        cnt = abi.aderdg2d_lim_counters(h)
    finally:
        abi.aderdg2d_lim_free(h)
    assert int(st[0]) == 0 and float(t[0]) == pytest.approx(T_END, abs=1e-14)
    gu = u.cpu().numpy()
    assert E2.admissible(gu).all()
    ops = basis.build_operators(N)
    L, R = W.RIEMANN_TESTS[test]
    exact = riemann.density(L, R, W.cell_points(C, N + 1), float(t[0]))          # [C, n]
    rows = np.einsum("j,cyij->yci", ops.w, gu[..., 0])                           # y-mean of rho per row
    errs = [np.einsum("k,ck->c", ops.w, np.abs(r - exact)).mean() for r in rows]
    spread = max(np.einsum("k,ck->c", ops.w, np.abs(r - rows[0])).mean() for r in rows)
    assert max(errs) <= 1.5 * ORACLE_L1_1D[test]
    assert spread <= ORACLE_L1_1D[test]
    assert np.abs(gu[..., 2]).max() <= 0.1 * np.abs(gu[..., 1]).max()
    print(f"[result] 2-D mesh, test {test}: troubled cell-steps {cnt[0]}, first-order redo steps {cnt[1]}, "
          f"L1(rho) per row {min(errs):.3e}..{max(errs):.3e}, row spread {spread:.2e}, "
          f"max |rho v| {np.abs(gu[..., 2]).max():.2e}", flush=True)


def test_khi_matches_oracle():
    """The Kelvin-Helmholtz problem of Sec. 2.2 (periodic, [0, 2] x [0, 1]) on
    16 x 8 cells, N = 2, 3 steps: state, averages and time to 1e-12."""
    _say("lim2d KHI")
    u0 = W.euler2d_khi_nodal(16, 8, 2)
    _check(u0, 2, abi.LIM_PERIODIC, 3, extent=(0.0, 2.0, 0.0, 1.0))


@pytest.mark.parametrize("bc", [abi.LIM_PERIODIC, abi.LIM_TRANSMISSIVE])
def test_explosion_on_cells_of_unequal_sides(bc):
    """The explosion on 12 x 8 cells of [-1, 1] x [-0.7, 0.7] (dx = 1/6,
    dy = 0.175), N = 3, 3 steps: state, averages and time to 1e-12."""
    _say("lim2d explosion, unequal sides", bc)
    extent = (-1.0, 1.0, -0.7, 0.7)
    u0 = W.euler2d_explosion_nodal(12, 8, 3, extent=extent)
    assert _check(u0, 3, bc, 3, extent=extent) > 0
