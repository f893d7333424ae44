"""Closed form of one ADER-DG step for a linear ODE: the (N, N+1) Pade approximant.

Sec. 2.1 "ODE system problem": for a spatially uniform state of
eq. (pdes_2_comps) the spatial terms vanish and each step of the ADER-DG-P_N
method is a DG-in-time step of degree N for the linear ODE u' = A u,
A = [[0, 1], [-omega^2, 0]] (eq. harm_osc).  A DG-in-time step of degree N
(upwind in time, exact quadrature of the linear source) advances by the
rational function R(dt A), where R is the (N, N+1) Pade approximant of exp:

   P(z) = sum_{i=0..k} (k+j-i)! k! / ((k+j)! i! (k-i)!) z^i,
   Q(z) = sum_{i=0..j} (k+j-i)! j! / ((k+j)! i! (j-i)!) (-z)^i,   k = N, j = N+1,

the textbook stability function of the Radau IIA / DG time discretisation.
This module is the closed form the oracle's predictor + corrector must
reproduce on the ODE test; it does not use the oracle's operators.
Test infrastructure only.
"""

from math import factorial

import numpy as np


def pade_coefficients(k, j):
    p = np.array([factorial(k + j - i) * factorial(k) / (factorial(k + j) * factorial(i) * factorial(k - i))
                  for i in range(k + 1)])
    q = np.array([factorial(k + j - i) * factorial(j) / (factorial(k + j) * factorial(i) * factorial(j - i))
                  * (-1.0) ** i for i in range(j + 1)])
    return p, q


def _matpoly(coef, Z):
    out = np.zeros_like(Z)
    Zi = np.eye(Z.shape[0])
    for c in coef:
        out = out + c * Zi
        Zi = Zi @ Z
    return out


def step_matrix(N, dt, A):
    """R_{N,N+1}(dt A) = Q(dt A)^-1 P(dt A)."""
    p, q = pade_coefficients(N, N + 1)
    Z = dt * np.asarray(A, dtype=np.float64)
    return np.linalg.solve(_matpoly(q, Z), _matpoly(p, Z))


def oscillator_trajectory(N, nsteps, omega=1.0, t_final=2 * np.pi, u0=(1.0, 0.0)):
    """States u^0..u^nsteps of the harmonic-oscillator ODE under R_{N,N+1}."""
    A = np.array([[0.0, 1.0], [-omega ** 2, 0.0]])
    R = step_matrix(N, t_final / nsteps, A)
    out = [np.array(u0, dtype=np.float64)]
    for _ in range(nsteps):
        out.append(R @ out[-1])
    return np.array(out)
