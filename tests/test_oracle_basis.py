"""Pins of the oracle's basis and operator matrices (Sec. 1.1, 1.2, 1.4)."""

import numpy as np
import pytest

from oracle import basis

NS = list(range(0, 10))


@pytest.mark.parametrize("N", NS)
def test_gauss_legendre_matches_library_and_is_exact(N):
    n = N + 1
    ops = basis.build_operators(N)
    x, w = np.polynomial.legendre.leggauss(n)
    assert np.allclose(ops.xi, 0.5 * (x + 1), atol=2e-16, rtol=0)
    assert np.allclose(ops.w, 0.5 * w, atol=1e-15, rtol=0)
    assert abs(ops.w.sum() - 1.0) < 1e-15                       # eq. gl_rule
    for m in range(2 * N + 2):                                   # exact to degree 2N+1
        assert abs(ops.w @ ops.xi ** m - 1.0 / (m + 1)) < 1e-14
    m = 2 * N + 2
    assert abs(ops.w @ ops.xi ** m - 1.0 / (m + 1)) > 1e-13     # and no further


@pytest.mark.parametrize("N", NS)
def test_lagrange_basis_properties(N):
    ops = basis.build_operators(N)
    assert np.allclose(basis.lagrange_eval(ops.xi, ops.xi), np.eye(ops.n), atol=1e-13)
    xs = np.linspace(0, 1, 17)
    assert np.allclose(basis.lagrange_eval(ops.xi, xs).sum(1), 1.0, atol=1e-12)
    assert np.allclose(basis.lagrange_deriv(ops.xi, xs).sum(1), 0.0, atol=1e-9)
    # derivative by finite differences of the basis itself
    h = 1e-6
    fd = (basis.lagrange_eval(ops.xi, xs + h) - basis.lagrange_eval(ops.xi, xs - h)) / (2 * h)
    assert np.allclose(basis.lagrange_deriv(ops.xi, xs), fd, atol=1e-5 * max(1, N ** 3))


@pytest.mark.parametrize("N", NS)
def test_mass_matrix_is_diagonal_with_weights(N):
    # eq. m_and_kappa_matrices: Lambda_kl = Lambda_k delta_kl; GL collocation gives Lambda_k = w_k
    ops = basis.build_operators(N)
    assert np.allclose(ops.Lam, np.diag(ops.w), atol=1e-15)
    # w_k = int phi_k^2 (eq. gl_rule)
    assert np.allclose(np.diag(ops.Lam), ops.w, atol=1e-15)


@pytest.mark.parametrize("N", NS)
def test_ktilde_is_transposed_derivative_matrix(N):
    # k~ = Lambda^-1 Xi equals (D^phi)^T because GL is exact to degree 2N-1
    ops = basis.build_operators(N)
    scale = max(1.0, np.abs(ops.Dphi).max())
    assert np.allclose(ops.ktil, ops.Dphi.T, atol=1e-14 * scale)
    # k~ differentiates polynomials of degree <= N exactly (nodal values -> nodal derivative)
    for d in range(N + 1):
        assert np.allclose(ops.ktil @ ops.xi ** d, d * ops.xi ** max(d - 1, 0) if d else 0 * ops.xi,
                           atol=1e-12 * scale)


@pytest.mark.parametrize("N", NS)
def test_L0_broadcast_property(N):
    # eq. ind_prop: L^0 = (Upsilon^-1 psi) (x) I with Upsilon^-1 psi = 1
    ops = basis.build_operators(N)
    assert np.allclose(np.linalg.solve(ops.Ups, ops.psi0), 1.0, atol=1e-13)


@pytest.mark.parametrize("N", NS)
def test_Lxi_is_nilpotent(N):
    # Sec. 1.1: the eigenvalues of L^xi = kappa~ (x) k~ are zero
    ops = basis.build_operators(N)
    Lxi = np.kron(ops.kappa, ops.ktil)
    P = np.linalg.matrix_power(Lxi, ops.n)
    assert np.abs(P).max() < 1e-9 * max(1.0, np.abs(Lxi).max()) ** ops.n
    assert np.abs(np.linalg.matrix_power(ops.ktil, ops.n)).max() < 1e-8 * max(1, N) ** (2 * ops.n)


@pytest.mark.parametrize("N", NS)
def test_Dtilde_and_traces(N):
    ops = basis.build_operators(N)
    # sum_l D~_kl = int phi_k' = phi_k(1) - phi_k(0)
    assert np.allclose(ops.Dtil.sum(1), ops.psi1 - ops.psi0, atol=1e-12)
    assert abs(ops.psi0.sum() - 1) < 1e-13 and abs(ops.psi1.sum() - 1) < 1e-13
    # traces reproduce the boundary value of x^d
    for d in range(N + 1):
        assert abs(ops.psi0 @ ops.xi ** d - (1.0 if d == 0 else 0.0)) < 1e-12
        assert abs(ops.psi1 @ ops.xi ** d - 1.0) < 1e-12


@pytest.mark.parametrize("N", NS)
def test_subcell_projection_exact_on_polynomials(N):
    # Sec. 1.4: P_jk = N_s int_{j/N_s}^{(j+1)/N_s} phi_k, N_s = 2N+1
    ops = basis.build_operators(N)
    Ns = ops.Ns
    assert ops.P.shape == (2 * N + 1, N + 1)
    for d in range(N + 1):
        exact = Ns * (((np.arange(Ns) + 1) / Ns) ** (d + 1) - (np.arange(Ns) / Ns) ** (d + 1)) / (d + 1)
        assert np.allclose(ops.P @ ops.xi ** d, exact, atol=1e-13)
    # averaging the subcells gives the cell integral: (1/N_s) sum_j P_jk = w_k
    assert np.allclose(ops.P.mean(0), ops.w, atol=1e-14)
