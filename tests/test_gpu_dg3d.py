"""3-D ADER-DG (Euler gas) on the GPU against the FP64 oracle, through the C ABI.

* predictor alone: q of every cell and each cell's sweep count;
* fused steps for every degree 1..9 in FP64 and with the FP32 predictor, on
  meshes of unequal sides whose cell counts leave the last workgroup partly
  empty (from N = 6 in FP64 and N = 7 in FP32 the predictor's tiles live in a
  device buffer instead of LDS);
* the paper's 3-D timing mesh (Sec. 3, the 3-D DG table: 4^3 cells) at
  N = 6 and 9 for a few steps;
* edge cases: a single cell (its own neighbour on all six sides), one-cell
  slabs, zero steps, a fixed step, the last step clamped to t_end;
* full size (48^3 and 64^3 cells at N = 3, 40^3 at N = 5 in FP64 and with the
  FP32 predictor, 24^3 at N = 7 and 16^3 at N = 9): a wave of period 4 cells
  equals, on every cell, the oracle's 4^3 run repeated.
"""

import numpy as np
import pytest

from oracle import basis, dg3d
from paper_2409_12483_amd import abi
from paper_2409_12483_amd import workloads as W

from gpu_util import BIG, rel_l2, torch_dev

pytestmark = pytest.mark.gpu
E3 = dg3d.Euler3D()


def _say(*a):
    print("[case]", *a, flush=True)


def gpu_run(u0, N, nsteps, extent=(1.0, 1.0, 1.0), cfl=0.4, fixed_dt=0.0, prec=abi.FP64, t0=0.0,
            t_end=BIG):
    torch, dev = torch_dev()
    h = abi.aderdg3d_init(abi.config3d(N, u0.shape[:3], extent=extent, cfl=cfl, fixed_dt=fixed_dt,
                                       precision=prec))
    try:
        u = torch.tensor(np.ascontiguousarray(u0), dtype=torch.float64, device=dev)
        t = torch.tensor([t0], dtype=torch.float64, device=dev)
        te = torch.tensor([t_end], dtype=torch.float64, device=dev)
        dt = torch.zeros(1, dtype=torch.float64, device=dev)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        abi.aderdg3d_step(h, u, t, te, dt, st, nsteps)
        torch.cuda.synchronize()
        return u.cpu().numpy(), float(t[0]), float(dt[0]), int(st[0]), abi.aderdg3d_sweep_count(h)
    finally:
        abi.aderdg3d_free(h)


@pytest.mark.parametrize("N,cells", [(1, (5, 4, 3)), (2, (3, 2, 3)), (3, (2, 3, 2)), (5, (2, 1, 2)),
                                     (6, (2, 2, 1)), (7, (1, 2, 2)), (9, (2, 1, 1))])
def test_predictor_matches_oracle(N, cells):
    _say("3d predictor", N, cells)
    torch, dev = torch_dev()
    ops = basis.build_operators(N)
    ext = (1.0, 0.8, 0.6)
    u0 = W.euler3d_sine_wave(*cells, N, noise=2e-2, seed=N, velocity=(0.8, -0.5, 0.3), extent=ext)
    h3 = tuple(ext[d] / cells[d] for d in range(3))
    dt = 0.3 * min(h3) / (3 * (2 * N + 1)) / 2.5
    qref, sw, _ = dg3d.predict3d(ops, E3, u0, dt, h3)
    h = abi.aderdg3d_init(abi.config3d(N, cells, extent=ext))
    try:
        u = torch.tensor(u0, dtype=torch.float64, device=dev)
        q = torch.zeros(qref.shape, dtype=torch.float64, device=dev)
        it = torch.zeros(int(np.prod(cells)), dtype=torch.int32, device=dev)
        abi.aderdg3d_predict(h, u, 0.0, dt, q, it)
        torch.cuda.synchronize()
        assert rel_l2(q.cpu().numpy(), qref) <= 1e-12
        assert np.array_equal(it.cpu().numpy(), sw.reshape(-1))
    finally:
        abi.aderdg3d_free(h)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_fused_steps_match_oracle(N):
    cells = {1: (5, 4, 3), 2: (3, 4, 3), 3: (3, 2, 3), 4: (3, 2, 2), 5: (2, 2, 2), 6: (2, 2, 2),
             7: (2, 1, 2), 8: (1, 2, 2), 9: (2, 2, 1)}[N]
    _say("3d steps", N, cells)
    ops = basis.build_operators(N)
    ext = (1.0, 0.9, 0.7)
    u0 = W.euler3d_sine_wave(*cells, N, noise=1e-2, seed=20 + N, velocity=(1.0, 0.6, -0.4), extent=ext)
    ref, t_ref, info = dg3d.dg3d_run(ops, E3, u0, extent=ext, nsteps=3)
    u, t, dt, st, sweeps = gpu_run(u0, N, 3, extent=ext)
    assert st == 0
    assert rel_l2(u, ref) <= 1e-12
    assert abs(t - t_ref) <= 1e-14 * t_ref
    assert abs(dt - info["dts"][-1]) <= 1e-14 * dt
    assert sweeps == sum(k * v for k, v in info["sweep_hist"].items())


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_fp32_predictor_within_1e5(N):
    _say("3d fp32", N)
    ops = basis.build_operators(N)
    cells = (2, 2, 1) if N >= 7 else (2, 2, 2) if N >= 5 else (3, 3, 2)
    u0 = W.euler3d_sine_wave(*cells, N, noise=1e-2, seed=3)
    ref, t_ref, _ = dg3d.dg3d_run(ops, E3, u0, nsteps=2)
    u, t, _, st, _ = gpu_run(u0, N, 2, prec=abi.FP32_PREDICTOR)
    assert st == 0
    assert 0.0 < rel_l2(u, ref) <= 1e-5
    assert abs(t - t_ref) <= 1e-5 * t_ref


@pytest.mark.parametrize("N,cells", [(2, (1, 1, 1)), (3, (1, 3, 1)), (1, (4, 1, 2))])
def test_tiny_meshes(N, cells):
    _say("3d tiny mesh", N, cells)
    ops = basis.build_operators(N)
    u0 = W.euler3d_sine_wave(*cells, N, amp=0.2, noise=1e-3, seed=1)
    ref, t_ref, _ = dg3d.dg3d_run(ops, E3, u0, nsteps=2)
    u, t, _, st, _ = gpu_run(u0, N, 2)
    assert st == 0
    assert rel_l2(u, ref) <= 1e-12
    assert abs(t - t_ref) <= 1e-14 * t_ref


@pytest.mark.parametrize("N", [6, 9])
def test_paper_timing_mesh_high_degree(N):
    """The sine wave of the paper's 3-D timing runs on its smallest mesh (4^3
    cells, unit cube), three steps at the degrees whose tiles live in device
    memory."""
    _say("3d timing mesh", N)
    ops = basis.build_operators(N)
    u0 = W.euler3d_sine_wave(4, 4, 4, N)
    ref, t_ref, info = dg3d.dg3d_run(ops, E3, u0, nsteps=3)
    u, t, _, st, sweeps = gpu_run(u0, N, 3)
    assert st == 0
    assert rel_l2(u, ref) <= 1e-12
    assert abs(t - t_ref) <= 1e-14 * t_ref
    assert sweeps == sum(k * v for k, v in info["sweep_hist"].items())


def test_zero_steps_fixed_dt_and_clamp():
    _say("3d zero steps / fixed dt / clamp")
    N = 2
    ops = basis.build_operators(N)
    u0 = W.euler3d_sine_wave(3, 3, 3, N, noise=1e-3, seed=2)
    u, t, dt, st, sw = gpu_run(u0, N, 0, t0=0.25)
    assert np.array_equal(u, u0) and t == 0.25 and dt == 0.0 and st == 0 and sw == 0
    ref, _, _ = dg3d.dg3d_run(ops, E3, u0, fixed_dt=1e-3, nsteps=2)
    u, t, dt, st, _ = gpu_run(u0, N, 2, fixed_dt=1e-3)
    assert rel_l2(u, ref) <= 1e-12 and dt == 1e-3
    ref, t_ref, _ = dg3d.dg3d_run(ops, E3, u0, t_end=1e-3, nsteps=4)
    u, t, dt, st, _ = gpu_run(u0, N, 4, t_end=1e-3)
    assert rel_l2(u, ref) <= 1e-12 and t == 1e-3 and t_ref == 1e-3 and dt == 1e-3


@pytest.mark.parametrize("N,C,prec", [(3, 48, abi.FP64), (3, 64, abi.FP64), (5, 40, abi.FP64),
                                       (5, 40, abi.FP32_PREDICTOR), (7, 24, abi.FP64),
                                       (9, 16, abi.FP64), (9, 16, abi.FP32_PREDICTOR)])
def test_full_size_periodic_wave_equals_repeated_oracle(N, C, prec):
    """The mesh sizes, degrees, precisions and CFL number of the timed 3-D
    runs, with a wave of period 4 cells: every 4^3 block of the GPU result
    equals the oracle's run on one block, and the sweep total is k^3 times the
    oracle's (FP64)."""
    per = 4
    _say("3d full size tiled", N, C, prec)
    ops = basis.build_operators(N)
    k = C // per
    big = W.euler3d_sine_wave(C, C, C, N, k=(k, k, k))
    small = W.euler3d_sine_wave(per, per, per, N, k=(k, k, k), extent=(per / C,) * 3)
    ref, t_ref, info = dg3d.dg3d_run(ops, E3, small, extent=(per / C,) * 3, nsteps=2)
    u, t, _, st, sweeps = gpu_run(big, N, 2, prec=prec)
    assert st == 0
    tiled = np.tile(ref, (k, k, k, 1, 1, 1, 1))
    if prec == abi.FP64:
        assert np.abs(u - tiled).max() <= 1e-12 * np.abs(ref).max()
        assert abs(t - t_ref) <= 1e-14 * t_ref
        assert sweeps == k ** 3 * sum(c * v for c, v in info["sweep_hist"].items())
    else:
        assert 0.0 < rel_l2(u, tiled) <= 1e-5
        assert abs(t - t_ref) <= 1e-5 * t_ref
