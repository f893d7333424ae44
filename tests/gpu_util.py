"""Helpers shared by the GPU tests: run the HIP path through the C ABI, and
evaluate the oracle on windows of a large mesh (sampled parity)."""

import numpy as np

from oracle import basis, dg, fv, predictor
from oracle import pde as OP
from paper_2409_12483_amd import abi

BIG = 1.0e300

ORACLE_PDE = {
    abi.PDE_EULER: lambda d: OP.Euler(d.gamma),
    abi.PDE_EULER_REACT: lambda d: OP.EulerReact(d.gamma, d.omega),
    abi.PDE_SWE: lambda d: OP.ShallowWater(d.g),
    abi.PDE_ADVECTION: lambda d: OP.Advection(d.adv_speed),
}


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def tensor(a, dtype=None):
    torch, dev = torch_dev()
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device=dev)


def run_steps(descs, cfgs, states, nsteps, t0=None, t_end=None, fv_scheme=False):
    """Advance a batch on the GPU; returns (states, t, dt, status, handle-sweeps)."""
    torch, dev = torch_dev()
    n = len(descs)
    h = abi.aderdg_init(descs, cfgs)
    try:
        us = [tensor(s) for s in states]
        t = tensor(np.zeros(n) if t0 is None else t0)
        te = tensor(np.full(n, BIG) if t_end is None else t_end)
        dt = tensor(np.zeros(n))
        st = torch.zeros(n, dtype=torch.int32, device=dev)
        step = abi.aderweno_step if fv_scheme else abi.aderdg_step
        step(h, us, t, te, dt, st, nsteps)
        torch.cuda.synchronize()
        sweeps = [abi.aderdg_sweep_count(h, k) for k in range(n)]
        return ([u.cpu().numpy() for u in us], t.cpu().numpy(), dt.cpu().numpy(),
                st.cpu().numpy(), sweeps)
    finally:
        abi.aderdg_free(h)


def oracle_dg_window(ops, pde, u, dt, dx, x0, idx, t0=0.0):
    """u^{n+1} of the cells idx of a periodic mesh, each from a 3-cell window."""
    C = u.shape[0]
    win = (np.asarray(idx)[:, None] + np.arange(-1, 2)[None, :]) % C      # [S, 3]
    flat = win.reshape(-1)
    x_left = x0 + dx * flat
    q, _, _ = predictor.predict(ops, pde, u[flat], dt, dx, x_left, t0)
    out = []
    for s in range(len(idx)):
        sl = slice(3 * s, 3 * s + 3)
        un = dg.dg_correct(ops, pde, u[flat[sl]], q[sl], dt, dx, x_left[sl], t0)
        out.append(un[1])
    return np.array(out)


def oracle_fv_window(ops, pde, v, dt, dx, x0, idx, t0=0.0):
    """v^{n+1} of the cells idx of a periodic mesh, each from an 11-cell window."""
    C = v.shape[0]
    reach = ops.N + 1
    offs = np.arange(-reach, reach + 1)
    out = []
    for i in idx:
        win = (i + offs) % C
        vn, _, _ = fv.fv_step(ops, pde, v[win], t0, dt, dx, x0 + dx * win)
        out.append(vn[reach])
    return np.array(out)


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
