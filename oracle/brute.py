"""Brute-force solve of the LST-DG predictor system, independent of the Picard loop.

Sec. 1.1: the predictor equations after point-wise evaluation read, for one cell,

    sum_q ( K^tau_pq q_q + K^xi_pq f_q - M_pq (s_q - b_q) ) = sum_k F^0_pk u_k

with the matrices of eq. (lst_dg_predictor_src_matrices)

    K^tau_pq = [Theta_p, Theta_q](1) - <dTheta_p/dtau, Theta_q>,   M_pq = <Theta_p, Theta_q>,
    F^0_pk   = [Theta_p, Phi_k](0),   K^xi_pq = <Theta_p, dTheta_q/dxi>,
    b_p      = B(q_p) sum_r D^xi_pr q_r,   D^xi_pr = dTheta_r/dxi (tau_p, xi_p).

Here these matrices are assembled directly from their definitions by a
tensor Gauss-Legendre quadrature of the space-time basis functions
Theta_p(tau, xi) = phi_p0(tau) phi_p1(xi) -- not from the Kronecker forms of
Sec. 1.1 "Using the BLAS interface" -- and the nonlinear system is solved by
Newton's method with a finite-difference Jacobian.  Agreement with the
Picard predictor therefore checks the Kronecker factorisation, the operators
kappa~ and k~, the L^0 broadcast and the iteration together.
Test infrastructure only.
"""

import numpy as np

from .basis import gauss_legendre_01, lagrange_deriv, lagrange_eval


def assemble(ops):
    n = ops.n
    xq, wq = gauss_legendre_01(n + 5)
    ph = lagrange_eval(ops.xi, xq)          # [Q, n]
    dph = lagrange_deriv(ops.xi, xq)
    ph0 = lagrange_eval(ops.xi, 0.0)[0]
    ph1 = lagrange_eval(ops.xi, 1.0)[0]

    # Theta_p at the tensor quadrature points, p = p0 * n + p1 ; point (i, j) = (tau_i, xi_j)
    def theta(tfac, xfac):
        return np.einsum("ia,jl->ijal", tfac, xfac).reshape(len(xq), len(xq), n * n)

    T = theta(ph, ph)
    Tt = theta(dph, ph)
    Tx = theta(ph, dph)
    W = np.outer(wq, wq)
    M = np.einsum("ij,ijp,ijq->pq", W, T, T)
    Kxi = np.einsum("ij,ijp,ijq->pq", W, T, Tx)
    vol_t = np.einsum("ij,ijp,ijq->pq", W, Tt, T)
    # boundary term [.,.](1): integral over xi at tau = 1
    T1 = np.einsum("a,jl->jal", ph1, ph).reshape(len(xq), n * n)
    Ktau = np.einsum("j,jp,jq->pq", wq, T1, T1) - vol_t
    T0 = np.einsum("a,jl->jal", ph0, ph).reshape(len(xq), n * n)
    F0 = np.einsum("j,jp,jk->pk", wq, T0, ph)
    # D^xi_pr = d Theta_r / dxi at the nodes (tau_p0, xi_p1)
    pt = lagrange_eval(ops.xi, ops.xi)      # [node, basis] = identity up to rounding
    pd = lagrange_deriv(ops.xi, ops.xi)
    Dxi = np.einsum("ab,lj->albj", pt, pd).reshape(n * n, n * n)
    return {"Ktau": Ktau, "M": M, "Kxi": Kxi, "F0": F0, "Dxi": Dxi}


def solve_cell(ops, pde, u_cell, dt, dx, x_left, t0, mats=None, tol=1e-15, max_newton=50):
    """Predictor coefficients q[a, l, r] of one cell by Newton's method."""
    mats = mats or assemble(ops)
    n, M = ops.n, pde.M
    dtdx = dt / dx
    xs = x_left + dx * ops.xi
    ts = t0 + dt * ops.xi
    xnode = np.tile(xs, n)                  # node p = a*n + l  ->  x_l
    tnode = np.repeat(ts, n)                # -> t_a
    rhs = mats["F0"] @ u_cell               # [n*n, M]

    def residual(Qflat):
        Q = Qflat.reshape(n * n, M)
        res = mats["Ktau"] @ Q + mats["Kxi"] @ (dtdx * pde.flux(Q)) - rhs
        sb = np.zeros_like(Q)
        if pde.has_source:
            sb += dt * pde.source(Q, xnode[:, None], tnode[:, None])
        if pde.has_ncp:
            sb -= dtdx * pde.ncp(Q, mats["Dxi"] @ Q)
        return (res - mats["M"] @ sb).ravel()

    Q = np.tile(u_cell, (n, 1)).ravel().copy()
    for _ in range(max_newton):
        r = residual(Q)
        J = np.empty((Q.size, Q.size))
        for i in range(Q.size):
            h = 1e-6 * max(1.0, abs(Q[i]))
            e = np.zeros_like(Q)
            e[i] = h
            J[:, i] = (residual(Q + e) - residual(Q - e)) / (2 * h)
        dQ = np.linalg.solve(J, -r)
        Q = Q + dQ
        if np.abs(dQ).max() <= tol * max(1.0, np.abs(Q).max()):
            break
    return Q.reshape(n, n, M)
