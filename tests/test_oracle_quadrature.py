"""Pins of the oracle's quadrature and interpolation steps (Prop. 2.4, Def. 2.2,
eq. TEI2, eq. chebcheb) against exact mathematics."""
import math

import numpy as np
import pytest

from oracle import tairef as T


@pytest.mark.parametrize("nq", [1, 2, 5, 16, 24, 32, 64])
def test_gauss_legendre_exact_on_monomials(nq):
    # Gauss rule with nq nodes integrates t^j exactly for j <= 2 nq - 1
    omega = 0.7
    t, w = T.time_nodes(omega, nq)
    for j in range(2 * nq):
        exact = omega ** (j + 1) / (j + 1)
        got = np.sum(w * t ** j)
        assert abs(got - exact) <= 4e-15 * exact * max(1, j), (nq, j, got, exact)
    # one degree higher the remainder is the one of Prop. 2.4 with
    # f^(2nq) = (2nq)!: omega^(2nq+1) (nq!)^4 / ((2nq+1) ((2nq)!)^2)
    if nq <= 5:
        j = 2 * nq
        rem = omega ** (j + 1) / (j + 1) - np.sum(w * t ** j)
        expect = omega ** (j + 1) * math.factorial(nq) ** 4 / ((j + 1) * math.factorial(j) ** 2)
        assert abs(rem - expect) <= 1e-9 * expect, (rem, expect)


@pytest.mark.parametrize("nq", [3, 16, 32])
def test_gauss_legendre_symmetry_and_golub_welsch(nq):
    z, zw = T.gauss_legendre(nq)
    assert np.all(np.diff(z) > 0)
    np.testing.assert_allclose(z, -z[::-1], atol=1e-15)
    np.testing.assert_allclose(zw, zw[::-1], rtol=1e-14)
    assert abs(np.sum(zw) - 2.0) < 1e-14
    # independent route: eigenvalues of the Jacobi matrix of Legendre
    # polynomials (Golub-Welsch), computed here from its definition
    k = np.arange(1, nq)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    J = np.diag(beta, 1) + np.diag(beta, -1)
    ev, V = np.linalg.eigh(J)
    np.testing.assert_allclose(z, ev, atol=2e-15)
    np.testing.assert_allclose(zw, 2.0 * V[0, :] ** 2, rtol=1e-12)


@pytest.mark.parametrize("kind", [T.NODES_LOBATTO, T.NODES_GAUSS])
@pytest.mark.parametrize("n", [2, 3, 8, 24, 48])
def test_lagrange_basis_identities(kind, n):
    L = 7.5
    xi, beta = T.cheb_nodes(n, L, kind)
    assert np.all(np.abs(xi) <= L + 1e-12)
    # l_a(xi_b) = delta_ab exactly at the nodes
    np.testing.assert_array_equal(T.lagrange_basis(xi, beta, xi), np.eye(n))
    rng = np.random.default_rng(n)
    x = rng.uniform(-L, L, 200)
    ell = T.lagrange_basis(xi, beta, x)
    # partition of unity
    np.testing.assert_allclose(ell.sum(axis=1), 1.0, atol=1e-13)
    # reproduces every polynomial of degree <= n-1: sum_a xi_a^j l_a(x) = x^j
    for j in range(n):
        got = ell @ (xi / L) ** j
        np.testing.assert_allclose(got, (x / L) ** j, atol=5e-13 * (1 + j))
    # independent product form l_a(x) = prod_{b != a} (x - xi_b)/(xi_a - xi_b)
    if n <= 24:
        prod = np.ones((len(x), n))
        for a in range(n):
            for b in range(n):
                if b != a:
                    prod[:, a] *= (x - xi[b]) / (xi[a] - xi[b])
        np.testing.assert_allclose(ell, prod, atol=1e-11)


def test_chebyshev_nodes_closed_form():
    # Def. 2.2: Lobatto x_k = cos((k-1) pi/(N-1)), Gauss x_k = cos((2k-1) pi/(2N))
    xi, _ = T.cheb_nodes(5, 1.0, T.NODES_LOBATTO)
    np.testing.assert_allclose(xi, [1.0, math.sqrt(0.5), 0.0, -math.sqrt(0.5), -1.0], atol=1e-16)
    xi, _ = T.cheb_nodes(2, 3.0, T.NODES_GAUSS)
    np.testing.assert_allclose(xi, [3.0 * math.sqrt(0.5), -3.0 * math.sqrt(0.5)], atol=1e-15)


def _cheb_T(k, u):
    return np.cos(k * np.arccos(np.clip(u, -1.0, 1.0)))


@pytest.mark.parametrize("kind", [T.NODES_LOBATTO, T.NODES_GAUSS])
def test_lagrange_form_equals_coefficient_form(kind):
    """The node-value (Lagrange) interpolant of exp(-t^2 (x-y)^2) on the n x n
    Chebyshev grid is the same polynomial as the paper's coefficient form
    sum alpha_nm T_n(x) T_m(y) (eqs. chebpoly, chebcoeff).  For first-kind
    nodes the coefficients are those of eq. chebcoeff (c = 1, 2, 4); for
    Lobatto nodes they are the discrete cosine coefficients of the second
    kind (end weights halved)."""
    n, L, t = 20, 6.0, 0.4
    xi, beta = T.cheb_nodes(n, L, kind)
    u = xi / L
    F = np.exp(-t * t * (xi[:, None] - xi[None, :]) ** 2)
    kk = np.arange(n)
    Tk = _cheb_T(kk[:, None], u[None, :])          # Tk[j, a] = T_j(u_a)
    if kind == T.NODES_GAUSS:
        c = np.where(kk == 0, 1.0, 2.0) / n
        alpha = (c[:, None] * Tk) @ F @ (c[:, None] * Tk).T
    else:
        N = n - 1
        e = np.ones(n)
        e[0] = e[-1] = 0.5
        c = (2.0 / N) * e                          # halve j = 0 and j = N
        alpha = (c[:, None] * Tk * e[None, :]) @ F @ (c[:, None] * Tk * e[None, :]).T
    rng = np.random.default_rng(3)
    x = rng.uniform(-L, L, 50)
    y = rng.uniform(-L, L, 50)
    lx = T.lagrange_basis(xi, beta, x)
    ly = T.lagrange_basis(xi, beta, y)
    lag = np.einsum("ia,ab,ib->i", lx, F, ly)
    Tx = _cheb_T(kk[None, :], x[:, None] / L)
    Ty = _cheb_T(kk[None, :], y[:, None] / L)
    coef = np.einsum("in,nm,im->i", Tx, alpha, Ty)
    np.testing.assert_allclose(lag, coef, atol=1e-13)
    # and both approximate the function itself
    exact = np.exp(-t * t * (x - y) ** 2)
    assert np.max(np.abs(lag - exact)) < 1e-5


def test_ktables():
    t, _ = T.time_nodes(0.5, 8)
    xi, _ = T.cheb_nodes(12, 8.0)
    K = T.ktables(t, xi)
    assert K.shape == (8, 12, 12)
    np.testing.assert_array_equal(K, np.transpose(K, (0, 2, 1)))
    np.testing.assert_array_equal(np.diagonal(K, axis1=1, axis2=2), 1.0)
    assert K[3, 2, 7] == math.exp(-t[3] ** 2 * (xi[2] - xi[7]) ** 2)
    # each K_k is a Gaussian-kernel Gram matrix on distinct nodes: SPD
    for k in range(8):
        assert np.linalg.eigvalsh(K[k]).min() > -1e-14
