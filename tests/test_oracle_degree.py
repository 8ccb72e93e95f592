"""Pins of the oracle's per-node degree form (eq. chebcheb with N_i points for
node i, and the nested coefficient moments of section 3.2): Chebyshev
coefficients against a library evaluation of known expansions, the truncation
against the sup-norm bound it promises, the coefficient route against the
node-form route, and the change of B against a bound that uses only the
moments and the tolerance."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import exact as X
from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


@pytest.mark.parametrize("kind", [T.NODES_LOBATTO, T.NODES_GAUSS])
def test_cheb_coefficients_of_known_expansion(kind):
    n, L = 12, 5.0
    xi, _ = T.cheb_nodes(n, L, kind)
    want = np.zeros((n, n))
    want[2, 5] = 3.0
    want[0, 1] = -0.5
    want[11, 11] = 0.25
    want[7, 0] = 1.5
    # node values from numpy's own Chebyshev series evaluation
    F = C.chebgrid2d(xi / L, xi / L, want)
    got = T.cheb_coefficients(F, T.cheb_vandermonde(xi, L))
    assert np.max(np.abs(got - want)) <= 1e-13


def test_tail_sums_match_masked_sums():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((9, 9))
    tail = T.tail_sums(a)
    i, j = np.indices(a.shape)
    for m in range(10):
        assert abs(tail[m] - np.abs(a)[np.maximum(i, j) >= m].sum()) <= 1e-13
    assert tail[9] == 0.0


@pytest.mark.parametrize("omega,nq,n,L,tol", [(0.3, 32, 40, 16.0, 1e-8), (1.0, 16, 24, 8.0, 1e-6),
                                              (0.5, 24, 32, 12.0, 1e-10)])
def test_truncated_polynomial_within_tol_on_dense_grid(omega, nq, n, L, tol):
    t, _ = T.time_nodes(omega, nq)
    xi, beta = T.cheb_nodes(n, L)
    N, ahat, Kt = T.truncated_tables(t, xi, L, tol)
    K = T.ktables(t, xi)
    x = np.linspace(-L, L, 241)
    ell = T.lagrange_basis(xi, beta, x)             # independent of the coefficients
    for k in range(nq):
        p_full = ell @ K[k] @ ell.T                 # the n-node interpolant
        p_trunc = C.chebgrid2d(x / L, x / L, ahat[k])
        assert np.max(np.abs(p_full - p_trunc)) <= tol * (1 + 1e-9) + 1e-14, k
        # node values of the truncated polynomial
        assert np.max(np.abs(C.chebgrid2d(xi / L, xi / L, ahat[k]) - Kt[k])) <= 1e-13
    assert np.all((N >= 1) & (N <= n))


def test_degree_is_the_smallest_within_tol():
    t, _ = T.time_nodes(0.3, 32)
    xi, _ = T.cheb_nodes(40, 16.0)
    V = T.cheb_vandermonde(xi, 16.0)
    K = T.ktables(t, xi)
    for tol in (1e-6, 1e-9, 1e-12):
        N, _, _ = T.truncated_tables(t, xi, 16.0, tol)
        for k in range(len(t)):
            tail = T.tail_sums(T.cheb_coefficients(K[k], V))
            assert tail[N[k]] <= tol
            if N[k] > 1:
                assert tail[N[k] - 1] > tol


def test_degrees_grow_with_t_and_shrink_with_tol():
    t, _ = T.time_nodes(0.3, 32)
    xi, _ = T.cheb_nodes(40, 16.0)
    prev = None
    for tol in (1e-13, 1e-10, 1e-8, 1e-6, 1e-3):
        N, _, _ = T.truncated_tables(t, xi, 16.0, tol)
        assert np.all(np.diff(N) >= 0)              # smoother factor at smaller t
        if prev is not None:
            assert np.all(N <= prev)
        prev = N
    assert prev[0] < 5 and prev[-1] < 40


def test_tiny_tol_keeps_all_degrees_and_reproduces_K():
    t, _ = T.time_nodes(0.5, 16)
    xi, _ = T.cheb_nodes(24, 8.0)
    N, _, Kt = T.truncated_tables(t, xi, 8.0, 1e-300)
    assert np.all(N == 24)
    assert np.max(np.abs(Kt - T.ktables(t, xi))) <= 1e-13
    N0, _, K0 = T.truncated_tables(t, xi, 8.0, 0.0)
    assert np.all(N0 == 24)
    np.testing.assert_array_equal(K0, T.ktables(t, xi))


def _setup(basis, omega, nq, n, L, tol):
    M = T.moments(basis.center, basis.alpha, basis.lxyz, L, n)
    t, w = T.time_nodes(omega, nq)
    xi, _ = T.cheb_nodes(n, L)
    N, ahat, Kt = T.truncated_tables(t, xi, L, tol)
    return M, w, N, ahat, Kt, T.cheb_vandermonde(xi, L), T.ktables(t, xi)


def test_coefficient_route_equals_node_route():
    basis = I.small_random(3, natoms=4, shells=("s", "p", "d"), box=4.0, alpha_lo=0.2, alpha_hi=8.0)
    M, w, N, ahat, Kt, V, K = _setup(basis, 0.5, 16, 24, 8.0, 1e-7)
    assert N.min() < 24
    mu = T.coefficient_moments(M, V)
    Bc = T.B_full_degrees(mu, ahat, N, w)
    Bn = T.B_full(M, Kt, w)
    assert np.max(np.abs(Bc - Bn)) <= 1e-13 * np.max(np.abs(Bn))
    # with every degree at n the coefficient route is the Lagrange form itself
    alphas = np.array([T.cheb_coefficients(Kk, V) for Kk in K])
    Bf = T.B_full_degrees(mu, alphas, np.full(16, 24), w)
    B = T.B_full(M, K, w)
    assert np.max(np.abs(Bf - B)) <= 1e-13 * np.max(np.abs(B))


@pytest.mark.parametrize("tol", [1e-9, 1e-6, 1e-4])
def test_B_change_within_bound_s_type(tol):
    # For s-type pairs both 1D factors are positive, so int |g_p| over the box
    # is prod_d sum_a m_{p,d}(a) (the Lagrange basis sums to one).  Each
    # truncated factor moves by at most tol and every factor is bounded by the
    # sum of its coefficient magnitudes S_k, so each node's product of three
    # moves by at most (S_k + tol)^3 - S_k^3.
    b, P = I.tiny_s()
    M, w, N, ahat, Kt, V, K = _setup(b, P.omega, P.nq, P.n, P.L, tol)
    B = T.B_full(M, K, w)
    Bt = T.B_full(M, Kt, w)
    S = np.array([T.tail_sums(T.cheb_coefficients(Kk, V))[0] for Kk in K])
    u = np.prod(M.sum(axis=1), axis=0)
    bound = (2.0 / math.sqrt(math.pi)) * np.sum(w * ((S + tol) ** 3 - S ** 3)) * np.outer(u, u)
    assert np.all(np.abs(Bt - B) <= bound * (1 + 1e-9))
    assert np.max(np.abs(Bt - B)) > 0.0


def test_converged_degrees_keep_physics_accuracy_s_type():
    # at converged parameters, the per-node degrees at a tight tolerance keep
    # the error against the exact integrals at the fixed-degree level while
    # contracting far fewer coefficients on average (below about 1e-13 the
    # tail sums reach the rounding floor of the coefficients themselves)
    b, _ = I.tiny_s()
    M, w, N, ahat, Kt, V, K = _setup(b, 0.5, 32, 64, 12.0, 1e-12)
    Bt = T.B_full(M, Kt, w)
    Bc = X.B_closed_form_s(b.center, b.alpha, 0.5)
    assert np.max(np.abs(Bt - Bc)) <= 1e-12 * np.max(np.abs(Bc))
    assert N.mean() < 0.7 * 64


def test_J_grid_with_truncated_tables_equals_coefficient_rows():
    basis = I.small_random(4, natoms=3, shells=("s", "p"), box=3.0)
    M, w, N, ahat, Kt, V, K = _setup(basis, 0.5, 12, 16, 8.0, 1e-6)
    D = I.random_density(np.random.default_rng(7), basis)
    Jg = T.J_grid(M, Kt, w, D)
    Bc = T.B_full_degrees(T.coefficient_moments(M, V), ahat, N, w)
    Jd = T.unpack_pairs(Bc @ T.density_pairs(D), basis.nb)
    assert np.max(np.abs(Jg - Jd)) <= 1e-13 * np.max(np.abs(Jd))
