"""Error norms and empirical convergence orders.

Sec. 2.1, eq. (epsilons): L1, L2 and L_inf errors of the DG solution against
the exact solution, the integrals taken cell by cell with a 25-point
Gauss-Legendre rule on the DG polynomial; order p = ln(e1/e2) / ln(h1/h2).
In 1-D the sup is taken over the same quadrature points.
Test infrastructure only.
"""

import numpy as np

from .basis import gauss_legendre_01, lagrange_eval


def dg_errors(ops, u, exact, x0, x1, var=0, npts=25):
    """(L1, L2, Linf) of component `var` of the DG solution u[C, n, M] vs exact(x)."""
    C = u.shape[0]
    dx = (x1 - x0) / C
    xq, wq = gauss_legendre_01(npts)
    phi = lagrange_eval(ops.xi, xq)                    # [Q, n]
    uh = np.einsum("qk,ck->cq", phi, u[:, :, var])     # [C, Q]
    xs = x0 + dx * (np.arange(C)[:, None] + xq[None, :])
    err = np.abs(uh - exact(xs))
    l1 = dx * np.einsum("q,cq->", wq, err)
    l2 = np.sqrt(dx * np.einsum("q,cq->", wq, err ** 2))
    return l1, l2, err.max()


def fv_errors(v, exact_avg, var=0):
    """Errors of cell averages v[C, M] against exact cell averages (C,)."""
    err = np.abs(v[:, var] - exact_avg)
    C = len(err)
    return err.sum() / C, np.sqrt((err ** 2).sum() / C), err.max()


def order(e1, e2, h1, h2):
    return np.log(e1 / e2) / np.log(h1 / h2)
