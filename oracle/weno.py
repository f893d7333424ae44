"""Polynomial WENO reconstruction from cell averages to nodal values (1-D).

The paper states only that a WENO reconstruction w^n(xi) of degree N is
computed from the cell averages of the neighbouring cells (Sec. 1,
eq. weno_reconstr) and is then used as the predictor's initial data
(Sec. 1.1, remark after the predictor's weak form).  No stencils, weights or
constants are given, so this module is a reading (parity unpinned beyond
its mathematical pins):

  * degree N even: three stencils of N+1 cells around cell i,
        left  {i-N .. i},  central {i-N/2 .. i+N/2},  right {i .. i+N};
    degree N odd, N >= 3 (N = 3: the paper's ADER-WENO4): four stencils,
        left  {i-N .. i},  two central {i-(N+1)/2 .. i+(N-1)/2} and
        {i-(N-1)/2 .. i+(N+1)/2},  right {i .. i+N};
    degree 1 (the second-order ADER-WENO2 of the paper's ADER-WENO(N+1)
    naming): the two stencils {i-1, i} and {i, i+1}, both sided;
  * on each stencil the unique degree-N polynomial p_s whose averages over
    the stencil cells equal the given averages (reference coordinate xi of
    cell i, cell i+o spans [o, o+1]);
  * oscillation indicator sigma_s = sum_{alpha=1..N} int_0^1 (d^alpha p_s / dxi^alpha)^2 dxi;
  * nonlinear weights  omega~_s = lambda_s / (sigma_s + eps)^r,
    lambda_central = 1e5, lambda_sided = 1, eps = 1e-14, r = 8, normalised;
  * w^_k = sum_s omega_s p_s(xi_k) at the Gauss-Legendre nodes, component-wise.
Test infrastructure only.
"""

import numpy as np

from .basis import gauss_legendre_01

LAMBDA_CENTRAL = 1.0e5
LAMBDA_SIDED = 1.0
EPSILON = 1.0e-14
POWER = 8


def stencil_offsets(N):
    if N == 1:
        return [[-1, 0], [0, 1]]
    if N % 2:
        lo, hi = (N + 1) // 2, (N - 1) // 2
        return [list(range(-N, 1)), list(range(-lo, hi + 1)), list(range(-hi, lo + 1)), list(range(0, N + 1))]
    h = N // 2
    return [list(range(-N, 1)), list(range(-h, h + 1)), list(range(0, N + 1))]


def linear_weights(N):
    """lambda_s of the stencils of stencil_offsets(N), in the same order."""
    if N == 1:
        return np.array([LAMBDA_SIDED, LAMBDA_SIDED])
    if N % 2:
        return np.array([LAMBDA_SIDED, LAMBDA_CENTRAL, LAMBDA_CENTRAL, LAMBDA_SIDED])
    return np.array([LAMBDA_SIDED, LAMBDA_CENTRAL, LAMBDA_SIDED])


def _monomial_cell_average(o, m):
    """average over [o, o+1] of (xi - 1/2)^m."""
    return ((o + 0.5) ** (m + 1) - (o - 0.5) ** (m + 1)) / (m + 1)


def stencil_polynomials(v, N):
    """Monomial coefficients (in xi - 1/2) of every stencil polynomial.

    v: [C, M] cell averages (periodic).  Returns coeff [S, C, N+1, M], S stencils.
    """
    out = []
    for offs in stencil_offsets(N):
        A = np.array([[_monomial_cell_average(o, m) for m in range(N + 1)] for o in offs])
        vs = np.stack([np.roll(v, -o, axis=0) for o in offs], axis=1)   # [C, N+1, M]
        coeff = np.linalg.solve(A[None, :, :], vs)                      # A c = v_s per cell, var
        out.append(coeff)
    return np.stack(out, axis=0)


def oscillation_indicators(coeff, N):
    """sigma_s = sum_alpha int_0^1 (p^(alpha))^2 for every stencil: [S, C, M]."""
    xq, wq = gauss_legendre_01(N + 2)
    sig = np.zeros(coeff.shape[:2] + coeff.shape[3:])
    for alpha in range(1, N + 1):
        # d^alpha/dxi^alpha of (xi - 1/2)^m  at the quadrature points
        D = np.zeros((len(xq), N + 1))
        for m in range(alpha, N + 1):
            fac = np.prod(np.arange(m - alpha + 1, m + 1, dtype=np.float64))
            D[:, m] = fac * (xq - 0.5) ** (m - alpha)
        vals = np.einsum("qm,scmr->scqr", D, coeff)
        sig += np.einsum("q,scqr->scr", wq, vals * vals)
    return sig


def weights(sig, N=None):
    if N is None:
        N = {2: 1, 3: 2, 4: 3}[sig.shape[0]]
    lam = linear_weights(N)[:, None, None]
    wt = lam / (sig + EPSILON) ** POWER
    return wt / wt.sum(axis=0, keepdims=True)


def reconstruct(v, ops):
    """Nodal values w^[c, k, r] of the WENO polynomial at the GL nodes of ops."""
    N = ops.N
    coeff = stencil_polynomials(v, N)
    omega = weights(oscillation_indicators(coeff, N), N)
    Vn = np.stack([(ops.xi - 0.5) ** m for m in range(N + 1)], axis=1)   # [n, N+1]
    nodal = np.einsum("km,scmr->sckr", Vn, coeff)
    return np.einsum("scr,sckr->ckr", omega, nodal)
