"""Pins of the oracle's Coulomb-matrix route through the Chebyshev grid tensor
(eqs. Coul, coulapprox with the mode products of eq. ig1)."""
import numpy as np

from oracle import exact as X
from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


def _ta(basis, omega, nq, n, L):
    M = T.moments(basis.center, basis.alpha, basis.lxyz, L, n)
    t, w = T.time_nodes(omega, nq)
    xi, _ = T.cheb_nodes(n, L)
    return M, T.ktables(t, xi), w


def _density(basis, seed):
    return I.random_density(np.random.default_rng(seed), basis)


def test_density_pairs_fold_ordered_sum():
    # sum over ordered (k,l) of X(k,l) D(k,l) = sum over pairs of X_q Dt_q for
    # any X symmetric in (k,l)
    rng = np.random.default_rng(0)
    nb = 7
    A = rng.standard_normal((nb, nb))
    D = A + A.T
    Xs = rng.standard_normal((nb, nb))
    Xs = Xs + Xs.T
    mu, nu = T.pair_list(nb)
    assert abs(np.sum(Xs * D) - np.dot(Xs[mu, nu], T.density_pairs(D))) < 1e-12


def test_grid_route_equals_B_times_density():
    for basis, (omega, nq, n, L) in [(I.tiny_s()[0], (0.5, 16, 24, 8.0)),
                                     (I.small_random(1, natoms=3, shells=("s", "p", "d")), (0.4, 12, 16, 8.0))]:
        M, K, w = _ta(basis, omega, nq, n, L)
        D = _density(basis, 3)
        Jg = T.J_grid(M, K, w, D)
        B = T.B_full(M, K, w)
        Jd = T.unpack_pairs(B @ T.density_pairs(D), basis.nb)
        assert np.max(np.abs(Jg - Jd)) <= 1e-13 * np.max(np.abs(Jd))
        np.testing.assert_array_equal(Jg, Jg.T)
        rows = np.array([0, 3, basis.npair - 1])
        np.testing.assert_allclose(T.J_direct_rows(M, K, w, D, rows), (B @ T.density_pairs(D))[rows],
                                   rtol=1e-14, atol=1e-16)


def test_grid_route_matches_closed_form_J_s():
    # J from the exact s-type integrals, at converged TA parameters
    b, _ = I.tiny_s()
    M, K, w = _ta(b, 0.5, 32, 64, 12.0)
    D = _density(b, 4)
    Jg = T.J_grid(M, K, w, D)
    Bc = X.B_closed_form_s(b.center, b.alpha, 0.5)
    Jc = T.unpack_pairs(Bc @ T.density_pairs(D), b.nb)
    assert np.linalg.norm(Jg - Jc, 2) <= 1e-12 * np.linalg.norm(Jc, 2)


def test_J_linear_in_density():
    basis = I.small_random(2, natoms=2, shells=("s", "p"))
    M, K, w = _ta(basis, 0.5, 8, 12, 8.0)
    D1 = _density(basis, 5)
    D2 = _density(basis, 6)
    J12 = T.J_grid(M, K, w, 2.0 * D1 - 0.5 * D2)
    ref = 2.0 * T.J_grid(M, K, w, D1) - 0.5 * T.J_grid(M, K, w, D2)
    assert np.max(np.abs(J12 - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_coulomb_mo_equals_B_contracted_with_orbital_densities():
    # J(i,j) = <q_i q_i^T, B (q_j q_j^T)> against the full B written out over
    # all ordered index pairs, on a tiny basis
    basis = I.small_random(81, natoms=2, shells=("s", "p"), box=2.0)
    M, K, w = _ta(basis, 0.5, 8, 12, 8.0)
    rng = np.random.default_rng(12)
    Q = rng.standard_normal((3, basis.nb))
    Jmo = T.coulomb_mo(M, K, w, Q)
    B = T.B_full(M, K, w)
    nb = basis.nb
    Bfull = np.zeros((nb, nb, nb, nb))
    mu, nu = T.pair_list(nb)
    for p in range(basis.npair):
        for q in range(basis.npair):
            for (a, b_) in {(mu[p], nu[p]), (nu[p], mu[p])}:
                for (c, d) in {(mu[q], nu[q]), (nu[q], mu[q])}:
                    Bfull[a, b_, c, d] = B[p, q]
    ref = np.einsum("ia,ib,abcd,jc,jd->ij", Q, Q, Bfull, Q, Q)
    assert np.max(np.abs(Jmo - ref)) <= 1e-12 * np.max(np.abs(ref))
    np.testing.assert_allclose(Jmo, Jmo.T, rtol=1e-12, atol=1e-14 * np.max(np.abs(ref)))
    # B is positive semidefinite, so the diagonal of the MO Coulomb matrix is >= 0
    assert np.all(np.diag(Jmo) >= -1e-14 * np.max(np.abs(ref)))


def test_coulomb_mo_closed_form_s():
    # s-type basis at converged TA parameters: the MO Coulomb matrix from the
    # exact long-range integrals
    b, _ = I.tiny_s()
    M, K, w = _ta(b, 0.5, 32, 64, 12.0)
    rng = np.random.default_rng(13)
    Q = rng.standard_normal((4, b.nb))
    Jmo = T.coulomb_mo(M, K, w, Q)
    Bc = X.B_closed_form_s(b.center, b.alpha, 0.5)
    ref = np.zeros((4, 4))
    for j in range(4):
        Jao = T.unpack_pairs(Bc @ T.density_pairs(np.outer(Q[j], Q[j])), b.nb)
        for i in range(4):
            ref[i, j] = np.sum(np.outer(Q[i], Q[i]) * Jao)
    assert np.max(np.abs(Jmo - ref)) <= 1e-11 * np.max(np.abs(ref))
