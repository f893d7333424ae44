"""Point-wise PDE models of the form dU/dt + dF(U)/dx + B(U) dU/dx = S(U, x, t).

Problem statement: Sec. 1, eq. (pde_src) / (pde_src_cart), specialised to
one space dimension.  Models:
  * Euler          - Sec. 2, eq. (system_of_equations); 1-D: U = (rho, rho u, E)
  * EulerReact     - Sec. 2.1 "ODE system problem", eq. (pdes_2_comps); 1-D:
                     U = (rho, rho u, E, rho c1, rho c2), S = (0,0,0, rho c2, -w^2 rho c1)
  * ShallowWater   - not defined in the paper (named only among its
                     applications).  Reading: U = (h, hu, b), F = (hu, hu^2/h + g h^2/2, 0),
                     B(U) dU/dx = (0, g h db/dx, 0), S = 0.
  * Advection      - dq/dt + a dq/dx = 0 (scalar), used for exactness tests.
The maximum signal speed |lambda| = |u| + c follows Sec. 1.5.
The numerical flux (Rusanov) and the path-conservative jump term are readings
of a Riemann solver the paper never specifies (Sec. 1.2): parity unpinned.
Test infrastructure only.
"""

import numpy as np


class Euler:
    """1-D Euler equations of an ideal gas, eq. (system_of_equations)."""

    M = 3
    has_source = False
    has_ncp = False

    def __init__(self, gamma=1.4):
        self.gamma = float(gamma)

    def primitives(self, Q):
        rho, m, E = Q[..., 0], Q[..., 1], Q[..., 2]
        u = m / rho
        p = (self.gamma - 1.0) * (E - 0.5 * m * u)
        return rho, u, p

    def flux(self, Q):
        rho, m, E = Q[..., 0], Q[..., 1], Q[..., 2]
        u = m / rho
        p = (self.gamma - 1.0) * (E - 0.5 * m * u)
        return np.stack([m, m * u + p, u * (E + p)], axis=-1)

    def max_speed(self, Q):
        rho, u, p = self.primitives(Q)
        return np.abs(u) + np.sqrt(self.gamma * p / rho)

    def admissible(self, Q):
        rho, u, p = self.primitives(Q)
        return np.isfinite(Q).all(axis=-1) & (rho > 0) & (p > 0)

    def dissipation_mask(self):
        return np.ones(self.M)


class EulerReact(Euler):
    """Euler + two reacting species, eq. (pdes_2_comps), in 1-D (M = 5)."""

    M = 5
    has_source = True

    def __init__(self, gamma=1.4, omega=1.0):
        super().__init__(gamma)
        self.omega = float(omega)

    def flux(self, Q):
        base = super().flux(Q[..., :3])
        u = Q[..., 1] / Q[..., 0]
        return np.concatenate([base, (Q[..., 3] * u)[..., None],
                               (Q[..., 4] * u)[..., None]], axis=-1)

    def source(self, Q, x, t):
        S = np.zeros_like(Q)
        S[..., 3] = Q[..., 4]
        S[..., 4] = -self.omega ** 2 * Q[..., 3]
        return S

    def source_jacobian(self, Q, x, t):
        """dS/dQ at every point: [..., M, M] (row = component of S)."""
        J = np.zeros(Q.shape + (self.M,))
        J[..., 3, 4] = 1.0
        J[..., 4, 3] = -self.omega ** 2
        return J

    def max_speed(self, Q):
        return super().max_speed(Q[..., :3])

    def admissible(self, Q):
        return super().admissible(Q[..., :3]) & np.isfinite(Q).all(axis=-1)


class ShallowWater:
    """Shallow water with bathymetry as a non-conservative product (reading)."""

    M = 3
    has_source = False
    has_ncp = True

    def __init__(self, g=9.81):
        self.g = float(g)

    def flux(self, Q):
        h, hu = Q[..., 0], Q[..., 1]
        u = hu / h
        return np.stack([hu, hu * u + 0.5 * self.g * h * h, np.zeros_like(h)], axis=-1)

    def ncp(self, Q, dQ):
        """B(Q) . dQ = (0, g h db, 0)."""
        out = np.zeros_like(Q)
        out[..., 1] = self.g * Q[..., 0] * dQ[..., 2]
        return out

    def ncp_jump(self, qm, qp):
        """int_0^1 B(qm + s (qp - qm)) ds . (qp - qm) for the straight-line path.

        Only the momentum row is non-zero: g * (hm + hp) / 2 * (bp - bm)
        (exact, since the integrand is linear in s)."""
        out = np.zeros_like(qm)
        out[..., 1] = self.g * 0.5 * (qm[..., 0] + qp[..., 0]) * (qp[..., 2] - qm[..., 2])
        return out

    def max_speed(self, Q):
        h, hu = Q[..., 0], Q[..., 1]
        return np.abs(hu / h) + np.sqrt(self.g * h)

    def admissible(self, Q):
        return np.isfinite(Q).all(axis=-1) & (Q[..., 0] > 0)

    def dissipation_mask(self):
        # no numerical dissipation on the bathymetry component (b is static)
        return np.array([1.0, 1.0, 0.0])


class Advection:
    """Scalar linear advection dq/dt + a dq/dx = 0."""

    M = 1
    has_source = False
    has_ncp = False

    def __init__(self, a=1.0):
        self.a = float(a)

    def flux(self, Q):
        return self.a * Q

    def max_speed(self, Q):
        return np.full(Q.shape[:-1], abs(self.a))

    def admissible(self, Q):
        return np.isfinite(Q).all(axis=-1)

    def dissipation_mask(self):
        return np.ones(1)


class Burgers:
    """Inviscid Burgers equation dq/dt + d(q^2/2)/dx = 0 (scalar).  Not one of
    the paper's models: it is the test model of the runtime-compiled user
    models (a flux that is not compiled into the library)."""

    M = 1
    has_source = False
    has_ncp = False

    def flux(self, Q):
        return 0.5 * Q * Q

    def max_speed(self, Q):
        return np.abs(Q[..., 0])

    def admissible(self, Q):
        return np.isfinite(Q).all(axis=-1)

    def dissipation_mask(self):
        return np.ones(1)


def rusanov(pde, qm, qp):
    """Rusanov (local Lax-Friedrichs) flux F^(qm, qp), unscaled.

    F^ = (F(qm) + F(qp))/2 - s/2 * D (qp - qm), s = max(lambda(qm), lambda(qp)),
    D the per-component dissipation mask.  Reading of the unspecified Riemann
    solver of Sec. 1.2 / Sec. 1.3: parity unpinned.
    """
    s = np.maximum(pde.max_speed(qm), pde.max_speed(qp))
    D = pde.dissipation_mask()
    return 0.5 * (pde.flux(qm) + pde.flux(qp)) - 0.5 * s[..., None] * D * (qp - qm)


def make_pde(name, **kw):
    name = name.lower()
    if name == "euler":
        return Euler(kw.get("gamma", 1.4))
    if name in ("euler_react", "eulerreact"):
        return EulerReact(kw.get("gamma", 1.4), kw.get("omega", 1.0))
    if name in ("swe", "shallow_water"):
        return ShallowWater(kw.get("g", 9.81))
    if name == "advection":
        return Advection(kw.get("a", 1.0))
    raise ValueError(name)
