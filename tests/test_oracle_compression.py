"""Pins of the oracle's low-rank compression of the moments (section 6.1,
eqs. SVD and approxepsilon): the compressed B against the uncompressed one
at full rank, against the projector form computed by Algorithm 1 on P m,
exact recovery of moments of known rank, invariance under rotations of the
kept basis, the singular values against the eigenvalues of the Gram matrix,
and the per-factor truncation bound."""
import numpy as np
import pytest

from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


def _setup(b, P):
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L, P.nodes)
    K = T.ktables(t, xi)
    M = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, kind=P.nodes)
    return M, K, w


def _normwise(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def small():
    b = I.small_random(71, natoms=4, shells=("s", "p", "d"), box=3.0, alpha_lo=0.2, alpha_hi=20.0)
    P = I.Params(omega=0.5, nq=8, n=16, L=8.0)
    return (b, P) + _setup(b, P)


def test_full_rank_is_the_uncompressed_method(small):
    b, P, M, K, w = small
    V, sigma, R = T.compression_basis(M, 0.0)
    assert R == P.n and V.shape == (P.n, P.n)
    U, Kc = T.compress(M, K, V)
    assert _normwise(T.B_full(U, Kc, w), T.B_full(M, K, w)) <= 1e-13
    D = I.random_density(np.random.default_rng(3), b)
    Jc, J = T.J_grid(U, Kc, w, D), T.J_grid(M, K, w, D)
    assert np.max(np.abs(Jc - J)) <= 1e-13 * np.max(np.abs(J))


@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-6])
def test_compressed_B_is_the_projected_method(small, tol):
    """u_p^T Kc_k u_q = (P m_p)^T K_k (P m_q): Algorithm 1 on the projected
    moments, entry by entry, without U or Kc."""
    b, P, M, K, w = small
    V, _, R = T.compression_basis(M, tol)
    assert R < P.n
    U, Kc = T.compress(M, K, V)
    Pm = np.stack([V @ (V.T @ M[d]) for d in range(3)])
    rng = np.random.default_rng(11)
    p = rng.integers(0, M.shape[2], 200)
    q = rng.integers(0, M.shape[2], 200)
    ref = T.B_entries(Pm, K, w, p, q)
    got = T.B_full(U, Kc, w)[p, q]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_exact_low_rank_moments_are_recovered():
    """Moments of rank r by construction (M_d = V0 X_d, V0 orthonormal n x r):
    the rank is r at any small tolerance and the compressed B is exact."""
    rng = np.random.default_rng(5)
    n, r, npair, nq = 20, 7, 60, 5
    V0, _ = np.linalg.qr(rng.standard_normal((n, r)))
    M = np.stack([V0 @ rng.standard_normal((r, npair)) for _ in range(3)])
    t, w = T.time_nodes(0.5, nq)
    xi, _ = T.cheb_nodes(n, 6.0)
    K = T.ktables(t, xi)
    V, sigma, R = T.compression_basis(M, 1e-10)
    assert R == r
    assert sigma[r] <= 1e-13 * sigma[0]
    U, Kc = T.compress(M, K, V)
    assert U.shape == (3, r, npair) and Kc.shape == (nq, r, r)
    assert _normwise(T.B_full(U, Kc, w), T.B_full(M, K, w)) <= 1e-12
    # the kept basis spans the range of V0
    assert np.max(np.abs(V @ V.T - V0 @ V0.T)) <= 1e-12


def test_rotation_of_the_kept_basis_changes_nothing(small):
    b, P, M, K, w = small
    V, _, R = T.compression_basis(M, 1e-5)
    Qr, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((R, R)))
    B1 = T.B_full(*T.compress(M, K, V), w)
    B2 = T.B_full(*T.compress(M, K, V @ Qr), w)
    assert _normwise(B2, B1) <= 1e-13


def test_singular_values_are_the_gram_eigenvalues(small):
    """sigma^2 are the eigenvalues of sum_d M_d M_d^T, the Gram matrix of the
    stacked moments; a transposed or missing direction changes them."""
    b, P, M, K, w = small
    _, sigma, _ = T.compression_basis(M, 0.0)
    G = sum(M[d] @ M[d].T for d in range(3))
    lam = np.sort(np.linalg.eigvalsh(G))[::-1]
    np.testing.assert_allclose(sigma ** 2, np.maximum(lam, 0), rtol=1e-10, atol=1e-13 * lam[0])
    _, sigma2, _ = T.compression_basis(M[[0, 0, 0]], 0.0)
    assert np.max(np.abs(sigma2 - sigma)) > 1e-3 * sigma[0]


@pytest.mark.parametrize("tol", [1e-3, 1e-5, 1e-7])
def test_per_factor_truncation_bound(small, tol):
    """|m_p^T K m_q - u_p^T Kc u_q| <= ||K||_2 (||r_p|| ||m_q|| + ||m_p|| ||r_q||)
    with r = (I - P) m, for every node, direction and sampled pair of pairs."""
    b, P, M, K, w = small
    V, _, _ = T.compression_basis(M, tol)
    U, Kc = T.compress(M, K, V)
    rng = np.random.default_rng(13)
    p = rng.integers(0, M.shape[2], 100)
    q = rng.integers(0, M.shape[2], 100)
    for k in range(K.shape[0]):
        kn = np.linalg.norm(K[k], 2)
        for d in range(3):
            g = np.einsum("ae,ab,be->e", M[d][:, p], K[k], M[d][:, q])
            gc = np.einsum("ae,ab,be->e", U[d][:, p], Kc[k], U[d][:, q])
            rp = np.linalg.norm(M[d][:, p] - V @ U[d][:, p], axis=0)
            rq = np.linalg.norm(M[d][:, q] - V @ U[d][:, q], axis=0)
            mp = np.linalg.norm(M[d][:, p], axis=0)
            mq = np.linalg.norm(M[d][:, q], axis=0)
            bound = kn * (rp * mq + mp * rq)
            assert np.all(np.abs(g - gc) <= bound * (1 + 1e-9) + 1e-15 * kn * mp * mq)


def test_rank_is_the_count_above_the_relative_cut(small):
    """Section 6.1 keeps the singular directions with sigma_r > tol * sigma_1:
    the rank is that count (at least one), with sigma taken here from the
    eigenvalues of the Gram matrix sum_d M_d M_d^T (an eigensolver, not the
    SVD the oracle calls).  Tolerances are placed between singular values so
    that the count is no rounding decision."""
    b, P, M, K, w = small
    G = sum(M[d] @ M[d].T for d in range(3))
    s = np.sqrt(np.maximum(np.sort(np.linalg.eigvalsh(G))[::-1], 0.0))
    s = s / s[0]
    for r in (1, 2, 3, 5, 8, 11):
        tol = float(np.sqrt(s[r - 1] * s[r]))       # between sigma_r and sigma_{r+1}
        assert s[r - 1] > tol * (1 + 1e-6) and s[r] < tol * (1 - 1e-6)
        V, sigma, R = T.compression_basis(M, tol)
        assert R == r and V.shape == (P.n, r)
    # a cut above every direction but the first keeps exactly one
    assert T.compression_basis(M, 0.999)[2] == 1
    assert T.compression_basis(M, 0.0)[2] == P.n


def test_rank_and_error_fall_with_the_tolerance():
    """On the sp16 workload the rank grows and the normwise error of B falls
    as the tolerance is tightened; the error stays within a small multiple of
    the tolerance."""
    b, P = I.sp16()
    M, K, w = _setup(b, P)
    B = T.B_full(M, K, w)
    ranks, errs = [], []
    for tol in (1e-3, 1e-5, 1e-7):
        V, _, R = T.compression_basis(M, tol)
        ranks.append(R)
        errs.append(_normwise(T.B_full(*T.compress(M, K, V), w), B))
        assert errs[-1] <= 10 * tol, (tol, R, errs[-1])
    assert ranks[0] < ranks[1] < ranks[2] < P.n
    assert errs[0] > errs[1] > errs[2]
