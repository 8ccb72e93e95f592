"""Pins of the oracle's long-range exchange matrix (appendix B, eq.
exchange): the factorized grid form equals the equation written out over the
oracle's B; at converged parameters both equal the exchange matrix of the
closed-form s-type integrals; the matrix is symmetric and positive
semi-definite; for one orbital its expectation value is twice the Coulomb
self-energy; swapping the roles of the index pairs is caught."""
import numpy as np

from oracle import exact as X
from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


def _ta(b, omega, nq, n, L):
    t, w = T.time_nodes(omega, nq)
    xi, _ = T.cheb_nodes(n, L)
    return T.moments(b.center, b.alpha, b.lxyz, L, n), T.ktables(t, xi), w


def test_grid_form_equals_the_equation_over_B():
    b = I.small_random(41, natoms=3, shells=("s", "p"), box=2.0)
    M, K, w = _ta(b, 0.5, 6, 12, 6.0)
    Q = np.random.default_rng(1).standard_normal((3, b.nb))
    Kg = T.exchange_grid(M, K, w, Q)
    Kd = T.exchange_direct(T.B_full(M, K, w), Q)
    assert np.max(np.abs(Kg - Kd)) <= 1e-12 * np.max(np.abs(Kd))


def test_closed_form_s_type():
    b, _ = I.tiny_s()
    M, K, w = _ta(b, 0.5, 32, 64, 12.0)
    Q = np.random.default_rng(2).standard_normal((3, b.nb))
    Kx = T.exchange_direct(X.B_closed_form_s(b.center, b.alpha, 0.5), Q)
    Kg = T.exchange_grid(M, K, w, Q)
    assert np.max(np.abs(Kg - Kx)) <= 1e-11 * np.max(np.abs(Kx))
    # the Coulomb-type pairing (mu nu | lambda kappa) gives a different matrix
    Bc = X.B_closed_form_s(b.center, b.alpha, 0.5)
    P = T.pair_index_matrix(b.nb)
    D = Q.T @ Q
    Jlike = 2.0 * np.einsum("mnlk,lk->mn", Bc[P[:, :, None, None], P[None, None, :, :]], D)
    assert np.max(np.abs(Jlike - Kx)) > 1e-3 * np.max(np.abs(Kx))


def test_symmetric_psd_and_single_orbital_identity():
    b = I.small_random(42, natoms=3, shells=("s", "p"), box=2.5)
    M, K, w = _ta(b, 0.4, 8, 12, 7.0)
    Q = np.random.default_rng(3).standard_normal((2, b.nb))
    Kg = T.exchange_grid(M, K, w, Q)
    assert np.max(np.abs(Kg - Kg.T)) <= 1e-13 * np.max(np.abs(Kg))
    assert np.min(np.linalg.eigvalsh(0.5 * (Kg + Kg.T))) >= -1e-12 * np.max(np.abs(Kg))
    q = Q[:1]
    K1 = T.exchange_grid(M, K, w, q)
    J1 = T.J_grid(M, K, w, np.outer(q[0], q[0]))
    assert abs(q[0] @ K1 @ q[0] - 2.0 * (q[0] @ J1 @ q[0])) <= 1e-12 * abs(q[0] @ K1 @ q[0])
