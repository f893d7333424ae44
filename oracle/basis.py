"""Nodal Lagrange basis on Gauss-Legendre points and the 1-D operator matrices.

Follows Sec. 1.1 (LST-DG predictor): the nodal basis of eq. (lst_dg_repr),
the Gauss-Legendre rule of eq. (gl_rule), the mass/stiffness matrices of
eq. (m_and_kappa_matrices), the derived matrices kappa~ = Upsilon^-1 Lambda,
k~ = Lambda^-1 Xi and the gradient matrix D^phi; Sec. 1.2 (ADER-DG, "Using
the BLAS interface") for D~_kl = w_l D^phi_kl and psi_k = phi_k(0),
psi~_k = phi_k(1); Sec. 1.4 for the subcell projection matrix P.

Everything is built from first principles on [0, 1]:
  * Gauss-Legendre nodes/weights by the Golub-Welsch eigenvalue method
    (symmetric Jacobi matrix of the Legendre recurrence);
  * Lagrange polynomials and their derivatives by explicit products;
  * integrals by an independent, finer Gauss-Legendre rule (n + 5 points),
    so that Lambda, Xi and P are the definitions written out rather than
    consequences of collocation.
Test infrastructure only (see package docstring).
"""

from dataclasses import dataclass

import numpy as np


def gauss_legendre_01(n):
    """n-point Gauss-Legendre rule on [0, 1] (eq. gl_rule: sum of weights = 1).

    Golub-Welsch: the nodes are the eigenvalues of the symmetric tridiagonal
    Jacobi matrix of the monic Legendre recurrence on [-1, 1], with
    off-diagonal entries k / sqrt(4k^2 - 1); the weights are 2 v_0^2 where v_0
    is the first component of each normalised eigenvector.  Mapped to [0, 1].
    """
    if n == 1:
        return np.array([0.5]), np.array([1.0])
    k = np.arange(1, n, dtype=np.float64)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    jac = np.diag(beta, 1) + np.diag(beta, -1)
    x, vec = np.linalg.eigh(jac)
    w = 2.0 * vec[0, :] ** 2
    order = np.argsort(x)
    x, w = x[order], w[order]
    # symmetrise (the rule is exactly symmetric about 0)
    x = 0.5 * (x - x[::-1])
    w = 0.5 * (w + w[::-1])
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_eval(nodes, x):
    """phi_k(x) for every node k: array [len(x), n].  phi_k(xi_l) = delta_kl."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(x), n))
    for k in range(n):
        for m in range(n):
            if m != k:
                out[:, k] *= (x - nodes[m]) / (nodes[k] - nodes[m])
    return out


def lagrange_deriv(nodes, x):
    """phi_k'(x) for every node k: array [len(x), n] (product rule, term by term)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(x), n))
    for k in range(n):
        for i in range(n):
            if i == k:
                continue
            term = np.full(len(x), 1.0 / (nodes[k] - nodes[i]))
            for m in range(n):
                if m != k and m != i:
                    term = term * (x - nodes[m]) / (nodes[k] - nodes[m])
            out[:, k] += term
    return out


def lagrange_nth_deriv(nodes, x, order):
    """d^order phi_k / dx^order at x, via the monomial coefficients of phi_k."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(x), n))
    for k in range(n):
        others = [nodes[m] for m in range(n) if m != k]
        coeffs = np.poly(others) / np.prod([nodes[k] - o for o in others])
        d = np.polyder(coeffs, order) if order > 0 else coeffs
        out[:, k] = np.polyval(d, x)
    return out


@dataclass
class Operators:
    """All 1-D matrices of Secs. 1.1, 1.2 and 1.4 for degree N (n = N + 1)."""

    N: int
    n: int
    xi: np.ndarray        # GL nodes on [0,1] (space and time share them)
    w: np.ndarray         # GL weights, sum = 1
    Lam: np.ndarray       # Lambda_kl = int phi_k phi_l
    Xi: np.ndarray        # Xi_kl = int phi_k phi_l'
    Ups: np.ndarray       # Upsilon_kl = phi_k(1) phi_l(1) - Xi_lk
    kappa: np.ndarray     # kappa~ = Upsilon^-1 Lambda   (time contraction)
    ktil: np.ndarray      # k~ = Lambda^-1 Xi            (space contraction)
    Dphi: np.ndarray      # D^phi_kl = phi_k'(xi_l)
    Dtil: np.ndarray      # D~_kl = w_l D^phi_kl
    psi0: np.ndarray      # psi_k = phi_k(0)
    psi1: np.ndarray      # psi~_k = phi_k(1)
    P: np.ndarray         # subcell projection, N_s x n, N_s = 2N+1
    Ns: int


def build_operators(N):
    """Operator matrices for degree N, each from its defining integral."""
    if N < 0:
        raise ValueError("N must be >= 0")
    n = N + 1
    xi, w = gauss_legendre_01(n)
    # independent finer rule for the defining integrals (exact to degree 2n+9)
    xq, wq = gauss_legendre_01(n + 5)
    phi_q = lagrange_eval(xi, xq)          # [Q, n]
    dphi_q = lagrange_deriv(xi, xq)        # [Q, n]
    Lam = np.einsum("q,qk,ql->kl", wq, phi_q, phi_q)
    Xi = np.einsum("q,qk,ql->kl", wq, phi_q, dphi_q)
    psi0 = lagrange_eval(xi, 0.0)[0]
    psi1 = lagrange_eval(xi, 1.0)[0]
    Ups = np.outer(psi1, psi1) - Xi.T
    kappa = np.linalg.solve(Ups, Lam)
    ktil = np.linalg.solve(Lam, Xi)
    Dphi = lagrange_deriv(xi, xi).T        # Dphi[k, l] = phi_k'(xi_l)
    Dtil = Dphi * w[None, :]
    Ns = 2 * N + 1
    P = np.zeros((Ns, n))
    for j in range(Ns):
        a, b = j / Ns, (j + 1) / Ns
        xs = a + (b - a) * xq
        P[j] = Ns * (b - a) * np.einsum("q,qk->k", wq, lagrange_eval(xi, xs))
    return Operators(N=N, n=n, xi=xi, w=w, Lam=Lam, Xi=Xi, Ups=Ups,
                     kappa=kappa, ktil=ktil, Dphi=Dphi, Dtil=Dtil,
                     psi0=psi0, psi1=psi1, P=P, Ns=Ns)
