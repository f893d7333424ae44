"""Seeded synthetic inputs shaped like the paper's workloads.

This module only samples analytic initial states; it holds none of the
method's arithmetic (no operators, fluxes, Riemann solvers or time
stepping), so both the HIP library's callers and the CPU oracle's tests can
consume its output.  Initial DG data are nodal values of the conserved
variables at the Gauss-Legendre points of each cell (sampling points taken
from numpy's Gauss-Legendre routine); finite-volume data are 16-point
Gauss-Legendre cell averages.

Workloads (1-D restatements of the paper's test problems, Sec. 2.1):
  * Euler density wave: rho = 1 + A sin(2 pi k x) (+ seeded uniform noise on
    the nodal rho), u = 1, p = 1, gamma = 1.4, periodic [0, 1]; the exact
    solution is the translate rho(x - t).
  * Euler with two reacting species, uniform state (ODE test): rho = 1,
    u = 1, p = 1, c1 = 1, c2 = 0.
  * Shallow water over a Gaussian bump: h = 1 + 0.1 sin(2 pi x),
    b = 0.2 exp(-100 (x - 0.5)^2), u = 0.
"""

import numpy as np


def gl_points_01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def cell_points(ncells, n, x0=0.0, x1=1.0):
    """Physical coordinates of the n Gauss-Legendre points of every cell: [C, n]."""
    xi, _ = gl_points_01(n)
    dx = (x1 - x0) / ncells
    return x0 + dx * (np.arange(ncells)[:, None] + xi[None, :])


def _euler_conserved(rho, u, p, gamma):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u], axis=-1)


def euler_density_wave(ncells, N, amp=0.2, k=1, noise=0.0, seed=0, gamma=1.4,
                       x0=0.0, x1=1.0, phase=0.0, velocity=1.0, pressure=1.0):
    """Nodal conserved state u[C, N+1, 3] of the 1-D density wave."""
    xs = cell_points(ncells, N + 1, x0, x1)
    rho = 1.0 + amp * np.sin(2.0 * np.pi * k * xs + phase)
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        rho = rho + rng.uniform(-noise, noise, size=rho.shape)
    return _euler_conserved(rho, np.full_like(rho, velocity), np.full_like(rho, pressure), gamma)


def euler_density_wave_exact(x, t, amp=0.2, k=1, velocity=1.0):
    return 1.0 + amp * np.sin(2.0 * np.pi * k * (x - velocity * t))


def euler_react_uniform(ncells, N, gamma=1.4, c1=1.0, c2=0.0):
    """Uniform state of the ODE test: u[C, N+1, 5]."""
    shape = (ncells, N + 1)
    base = _euler_conserved(np.ones(shape), np.ones(shape), np.ones(shape), gamma)
    return np.concatenate([base, np.full(shape + (1,), c1), np.full(shape + (1,), c2)], axis=-1)


def swe_bump_fields(x):
    h = 1.0 + 0.1 * np.sin(2.0 * np.pi * x)
    b = 0.2 * np.exp(-100.0 * (x - 0.5) ** 2)
    return h, np.zeros_like(h), b


def swe_bump_nodal(ncells, N, x0=0.0, x1=1.0):
    """Nodal (h, hu, b) at the GL points: u[C, N+1, 3]."""
    h, hu, b = swe_bump_fields(cell_points(ncells, N + 1, x0, x1))
    return np.stack([h, hu, b], axis=-1)


def swe_bump_averages(ncells, x0=0.0, x1=1.0, npts=16):
    """16-point Gauss-Legendre cell averages of (h, hu, b): v[C, 3]."""
    xs = cell_points(ncells, npts, x0, x1)
    _, w = gl_points_01(npts)
    h, hu, b = swe_bump_fields(xs)
    return np.stack([h @ w, hu @ w, b @ w], axis=-1)


def smooth_averages(ncells, func, x0=0.0, x1=1.0, npts=16):
    """16-point GL cell averages of an arbitrary scalar function."""
    xs = cell_points(ncells, npts, x0, x1)
    _, w = gl_points_01(npts)
    return func(xs) @ w


def advection_nodal(ncells, N, func, x0=0.0, x1=1.0):
    return func(cell_points(ncells, N + 1, x0, x1))[..., None]


def batched_euler_problems(nprob=256, seed=0, cmin=1_000, cmax=100_000, degrees=range(1, 8)):
    """Specs of independent Euler density-wave problems: log-uniform cell counts,
    uniform degrees, seeded wave numbers 1..4 and phases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    degrees = list(degrees)
    out = []
    for i in range(nprob):
        ncells = int(round(np.exp(rng.uniform(np.log(cmin), np.log(cmax)))))
        N = int(degrees[rng.integers(len(degrees))])
        k = int(rng.integers(1, 5))
        phase = float(rng.uniform(0.0, 2.0 * np.pi))
        out.append({"id": i, "pde": "euler", "N": N, "ncells": ncells, "k": k, "phase": phase})
    return out


def request_trace(nreq=2000, rate=200.0, seed=0, degrees=range(2, 10), cmin=1_000,
                  cmax=200_000, smin=50, smax=500):
    """Poisson arrival trace of solve requests (Euler or shallow-water DG)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    degrees = list(degrees)
    t = 0.0
    out = []
    for i in range(nreq):
        t += rng.exponential(1.0 / rate)
        out.append({
            "id": i, "arrival": t,
            "pde": "euler" if rng.uniform() < 0.5 else "swe",
            "N": int(degrees[rng.integers(len(degrees))]),
            "ncells": int(round(np.exp(rng.uniform(np.log(cmin), np.log(cmax))))),
            "steps": int(rng.integers(smin, smax + 1)),
            "k": int(rng.integers(1, 5)),
            "phase": float(rng.uniform(0.0, 2.0 * np.pi)),
        })
    return out


def euler2d_sine_wave(cx, cy, N, amp=0.5, kx=1, ky=1, velocity=(1.0, 1.0), pressure=1.0, gamma=1.4,
                      noise=0.0, seed=0, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
    """Nodal conserved state u[Cx, Cy, N+1, N+1, 4] of the 2-D sine wave.

    rho = 1 + amp sin(2 pi (kx x + ky y)) (+ seeded uniform noise on the nodal
    rho), velocity (u, v), pressure p, U = (rho, rho u, rho v, E).  The paper's
    2-D accuracy and timing problem (Sec. 2.1) is amp = 0.5, kx = ky = 1,
    velocity (1, 1), p = 1, gamma = 1.4 on the unit square; its exact solution
    is the translate rho(x - u t, y - v t).  Node index order [x node][y node].
    """
    n = N + 1
    xs = cell_points(cx, n, x0, x1)                     # [Cx, n]
    ys = cell_points(cy, n, y0, y1)                     # [Cy, n]
    X = xs[:, None, :, None]
    Y = ys[None, :, None, :]
    rho = 1.0 + amp * np.sin(2.0 * np.pi * (kx * X + ky * Y))
    rho = np.broadcast_to(rho, (cx, cy, n, n)).copy()
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        rho = rho + rng.uniform(-noise, noise, size=rho.shape)
    u = np.full_like(rho, velocity[0])
    v = np.full_like(rho, velocity[1])
    E = pressure / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E], axis=-1)


def euler2d_sine_wave_exact(x, y, t, amp=0.5, kx=1, ky=1, velocity=(1.0, 1.0)):
    return 1.0 + amp * np.sin(2.0 * np.pi * (kx * (x - velocity[0] * t) + ky * (y - velocity[1] * t)))


def euler3d_sine_wave(cx, cy, cz, N, amp=0.5, k=(1, 1, 1), velocity=(1.0, 1.0, 1.0), pressure=1.0,
                      gamma=1.4, noise=0.0, seed=0, extent=(1.0, 1.0, 1.0)):
    """Nodal conserved state u[Cx, Cy, Cz, N+1, N+1, N+1, 5] of the 3-D sine wave.

    rho = 1 + amp sin(2 pi (kx x + ky y + kz z)) (+ seeded uniform noise on the
    nodal rho), velocity (u, v, w), pressure p, U = (rho, rho u, rho v, rho w, E).
    The paper's 3-D problem (Sec. 2.1) is amp = 0.5, k = (1, 1, 1), velocity
    (1, 1, 1), p = 1, gamma = 1.4 on the unit cube.  Node order [x][y][z].
    """
    n = N + 1
    xs = cell_points(cx, n, 0.0, extent[0])
    ys = cell_points(cy, n, 0.0, extent[1])
    zs = cell_points(cz, n, 0.0, extent[2])
    X = xs[:, None, None, :, None, None]
    Y = ys[None, :, None, None, :, None]
    Z = zs[None, None, :, None, None, :]
    rho = 1.0 + amp * np.sin(2.0 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z))
    rho = np.broadcast_to(rho, (cx, cy, cz, n, n, n)).copy()
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        rho = rho + rng.uniform(-noise, noise, size=rho.shape)
    vel = [np.full_like(rho, v) for v in velocity]
    E = pressure / (gamma - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    return np.stack([rho, rho * vel[0], rho * vel[1], rho * vel[2], E], axis=-1)


def euler3d_sine_wave_exact(x, y, z, t, amp=0.5, k=(1, 1, 1), velocity=(1.0, 1.0, 1.0)):
    return 1.0 + amp * np.sin(2.0 * np.pi * (k[0] * (x - velocity[0] * t) + k[1] * (y - velocity[1] * t)
                                             + k[2] * (z - velocity[2] * t)))


def swe_lake_at_rest_nodal(ncells, N, kind="linear", x0=0.0, x1=1.0, amp=0.2, seed=0):
    """Shallow water at rest over a bathymetry, nodal (h, hu, b): u[C, N+1, 3].

    h + b = 1 and hu = 0 everywhere.  kind = "linear": b is continuous and
    piecewise linear between seeded edge values (kinks at the cell edges);
    kind = "step": b is constant in every cell (seeded values), so it jumps
    at every edge.  Periodic: the edge value at x1 equals the one at x0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = cell_points(ncells, N + 1, x0, x1)
    if kind == "linear":
        edges = 0.1 + amp * rng.uniform(0.0, 1.0, ncells)           # b at the left edge of each cell
        left, right = edges, np.roll(edges, -1)
        xi, _ = gl_points_01(N + 1)
        b = left[:, None] + (right - left)[:, None] * xi[None, :]
    elif kind == "step":
        b = np.broadcast_to((0.1 + amp * rng.uniform(0.0, 1.0, ncells))[:, None], xs.shape).copy()
    else:
        raise ValueError(kind)
    return np.stack([1.0 - b, np.zeros_like(b), b], axis=-1)


def swe_lake_at_rest_averages(ncells, x0=0.0, x1=1.0, npts=16):
    """Cell averages of the lake at rest over the Gaussian bump of the shallow-water
    workload: b = 0.2 exp(-100 (x - 0.5)^2), h = 1 - b, hu = 0: v[C, 3]."""
    xs = cell_points(ncells, npts, x0, x1)
    _, w = gl_points_01(npts)
    b = 0.2 * np.exp(-100.0 * (xs - 0.5) ** 2)
    return np.stack([(1.0 - b) @ w, np.zeros(ncells), b @ w], axis=-1)


# Table 9 (Sec. 2.2): primitive states (rho, u, p) left and right of the initial
# discontinuity at x_c = 0.5 of the four classical Riemann tests (Sod, Lax,
# two shocks, two rarefactions); gamma = 1.4, free outflow, t_final = 0.15.
RIEMANN_TESTS = {
    1: ((1.000, 0.000, 1.000), (0.125, 0.000, 0.100)),
    2: ((0.445, 0.698, 3.528), (0.500, 0.000, 0.571)),
    3: ((1.000, 1.000, 1.000), (1.000, -1.000, 1.000)),
    4: ((1.000, -1.000, 1.000), (1.000, 1.000, 1.000)),
}


def riemann_nodal(ncells, N, test, x0=0.0, x1=1.0, xc=0.5, gamma=1.4):
    """Conserved nodal data [C, N+1, 3] of a Table 9 Riemann problem: the left
    state at nodes x <= x_c, the right state elsewhere."""
    (rl, ul, pl), (rr, ur, pr) = RIEMANN_TESTS[test]
    xs = cell_points(ncells, N + 1, x0, x1)
    left = xs <= xc
    return _euler_conserved(np.where(left, rl, rr), np.where(left, ul, ur), np.where(left, pl, pr), gamma)


def riemann_array_nodal(ncells, N, test=1, period=64, gamma=1.4):
    """A periodic row of Table 9 Riemann problems: every block of `period`
    cells holds the left state in its first half and the right state in its
    second half (two discontinuities per block, at cell faces)."""
    (rl, ul, pl), (rr, ur, pr) = RIEMANN_TESTS[test]
    left = (np.arange(ncells) % period < period // 2)[:, None] & np.ones((1, N + 1), dtype=bool)
    return _euler_conserved(np.where(left, rl, rr), np.where(left, ul, ur), np.where(left, pl, pr), gamma)


def euler2d_explosion_nodal(cx, cy, N, r0=0.5, inside=(1.0, 1.0), outside=(0.125, 0.1), gamma=1.4,
                            extent=(-1.0, 1.0, -1.0, 1.0)):
    """Conserved nodal data [cx, cy, N+1, N+1, 4] of the cylindrical explosion of
    Sec. 2.2 (a two-dimensional Sod problem): (rho, p) = inside where the node's
    distance to the centre of the square is at most r0, outside elsewhere; the
    gas at rest; the square [-1, 1]^2 by default.  A cell that the circle
    r = r0 cuts (nodes on both sides) takes the constant state of the
    Gauss-Legendre mean of its nodal values (positive weights, so admissible),
    instead of the overshooting interpolant of a jump."""
    x0, x1, y0, y1 = extent
    xs = cell_points(cx, N + 1, x0, x1)
    ys = cell_points(cy, N + 1, y0, y1)
    X = xs[:, None, :, None]
    Y = ys[None, :, None, :]
    r = np.sqrt((X - 0.5 * (x0 + x1)) ** 2 + (Y - 0.5 * (y0 + y1)) ** 2)
    rho = np.where(r <= r0, inside[0], outside[0])
    p = np.where(r <= r0, inside[1], outside[1])
    z = np.zeros_like(rho)
    u = np.stack([rho, z, z, p / (gamma - 1.0)], axis=-1)
    inner = r <= r0
    cut = inner.any(axis=(2, 3)) & ~inner.all(axis=(2, 3))
    _, w = gl_points_01(N + 1)
    mean = np.einsum("i,j,xyijr->xyr", w, w, u)
    u[cut] = mean[cut][:, None, None, :]
    return u


def euler2d_khi_nodal(cx, cy, N, v0=0.1, sigma=0.05 / np.sqrt(2.0), gamma=1.4):
    """Conserved nodal data [cx, cy, N+1, N+1, 4] of the Kelvin-Helmholtz
    problem of Sec. 2.2 on [0, 2] x [0, 1]: p = 2.5; rho = 2 and u = -0.5 in
    the band 0.25 < y < 0.75, rho = 1 and u = +0.5 outside; v = v0 sin(4 pi x)
    (exp(-(y - 0.25)^2 / (2 sigma^2)) + exp(-(y - 0.75)^2 / (2 sigma^2)))."""
    xs = cell_points(cx, N + 1, 0.0, 2.0)
    ys = cell_points(cy, N + 1, 0.0, 1.0)
    X = np.broadcast_to(xs[:, None, :, None], (cx, cy, N + 1, N + 1))
    Y = np.broadcast_to(ys[None, :, None, :], (cx, cy, N + 1, N + 1))
    band = (Y > 0.25) & (Y < 0.75)
    rho = np.where(band, 2.0, 1.0)
    u = np.where(band, -0.5, 0.5)
    v = v0 * np.sin(4.0 * np.pi * X) * (np.exp(-(Y - 0.25) ** 2 / (2 * sigma ** 2))
                                        + np.exp(-(Y - 0.75) ** 2 / (2 * sigma ** 2)))
    p = np.full_like(rho, 2.5)
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)], axis=-1)


def euler2d_sine_averages(cx, cy, amp=0.5, kx=1, ky=1, velocity=(1.0, 1.0), pressure=1.0, gamma=1.4,
                          npts=16, t=0.0):
    """Cell averages v[Cx, Cy, 4] of the 2-D sine wave (conserved variables) at
    time t of its translation, by an npts x npts Gauss-Legendre rule per cell
    (the state is linear in rho, so the averages of rho u, rho v, E follow)."""
    xs = cell_points(cx, npts)
    ys = cell_points(cy, npts)
    _, w = gl_points_01(npts)
    X = xs[:, None, :, None]
    Y = ys[None, :, None, :]
    rho = euler2d_sine_wave_exact(X, Y, t, amp, kx, ky, velocity)
    rbar = np.einsum("i,j,xyij->xy", w, w, np.broadcast_to(rho, (cx, cy, npts, npts)))
    u, v = velocity
    E = pressure / (gamma - 1.0) + 0.5 * rbar * (u * u + v * v)
    return np.stack([rbar, rbar * u, rbar * v, E], axis=-1)


def euler3d_sine_averages(cx, cy, cz, amp=0.5, k=(1, 1, 1), velocity=(1.0, 1.0, 1.0), pressure=1.0,
                          gamma=1.4, npts=8, t=0.0):
    """Cell averages v[Cx, Cy, Cz, 5] of the 3-D sine wave at time t of its
    translation, by an npts^3 Gauss-Legendre rule per cell (unit cube)."""
    _, w = gl_points_01(npts)
    X = cell_points(cx, npts)[:, None, None, :, None, None]
    Y = cell_points(cy, npts)[None, :, None, None, :, None]
    Z = cell_points(cz, npts)[None, None, :, None, None, :]
    rho = euler3d_sine_wave_exact(X, Y, Z, t, amp, k, velocity)
    rbar = np.einsum("i,j,k,xyzijk->xyz", w, w, w, np.broadcast_to(rho, (cx, cy, cz, npts, npts, npts)))
    E = pressure / (gamma - 1.0) + 0.5 * rbar * sum(vv * vv for vv in velocity)
    return np.stack([rbar, rbar * velocity[0], rbar * velocity[1], rbar * velocity[2], E], axis=-1)
