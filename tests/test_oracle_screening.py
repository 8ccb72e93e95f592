"""Pins of the oracle's pair screening (section 6.3, compression by screening):
the kept list against a plain double loop over the criterion, its
monotonicity, and the size of everything screening drops against bounds that
use only the overlaps of the dropped pairs."""
import math

import numpy as np
import pytest

from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


def _loop_screen(b, tau):
    if tau <= 0:
        return np.arange(b.npair, dtype=np.int64)
    kept = []
    p = 0
    for mu in range(b.nb):
        for nu in range(mu, b.nb):
            a, c = b.alpha[mu], b.alpha[nu]
            r2 = sum((b.center[mu, d] - b.center[nu, d]) ** 2 for d in range(3))
            if math.exp(-a * c / (a + c) * r2) > tau:
                kept.append(p)
            p += 1
    return np.array(kept, dtype=np.int64)


@pytest.mark.parametrize("tau", [1e-4, 1e-8, 1e-12, 0.0])
def test_screen_matches_double_loop(tau):
    b = I.small_random(71, natoms=6, shells=("s", "p"), box=6.0, alpha_lo=0.2, alpha_hi=30.0)
    np.testing.assert_array_equal(T.screened_pairs(b.center, b.alpha, tau), _loop_screen(b, tau))


def test_screen_keeps_diagonal_and_is_monotone():
    b, _ = I.sp16()
    prev = None
    diag = np.array([T.pair_index(b.nb, m, m) for m in range(b.nb)])
    for tau in (0.0, 1e-14, 1e-10, 1e-6, 1e-2):
        kept = T.screened_pairs(b.center, b.alpha, tau)
        assert np.all(np.diff(kept) > 0)
        assert np.all(np.isin(diag, kept))
        if prev is not None:
            assert np.all(np.isin(kept, prev))
        prev = kept
    assert len(T.screened_pairs(b.center, b.alpha, 0.0)) == b.npair
    assert len(prev) < b.npair


def _setup(b, P):
    M = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n)
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L)
    K = T.ktables(t, xi)
    V = T.cheb_vandermonde(xi, P.L)
    S = np.array([T.tail_sums(T.cheb_coefficients(Kk, V))[0] for Kk in K])
    return M, K, w, S


@pytest.mark.parametrize("tau", [1e-3, 1e-6])
def test_dropped_entries_bounded_s_type(tau):
    # s-type pairs are positive: int |g_p| over the box = prod_d sum_a m_{p,d}(a),
    # and |B(p,q)| <= (2/sqrt(pi)) sum_k w_k S_k^3 u_p u_q with S_k the sum of
    # the node's coefficient magnitudes; a dropped pair's u_p carries its
    # prefactor, at most tau
    rng = np.random.default_rng(5)
    b = I.random_molecule(rng, 6, 4.0, ["s", "s"], 0.3, 20.0)
    P = I.Params(omega=0.5, nq=16, n=24, L=9.0)
    M, K, w, S = _setup(b, P)
    B = T.B_full(M, K, w)
    kept = T.screened_pairs(b.center, b.alpha, tau)
    dropped = np.setdiff1d(np.arange(b.npair), kept)
    assert len(dropped) > 0
    u = np.prod(M.sum(axis=1), axis=0)
    c = (2.0 / math.sqrt(math.pi)) * np.sum(w * S ** 3)
    bound = c * np.outer(u[dropped], u)
    assert np.all(np.abs(B[dropped]) <= bound * (1 + 1e-9))
    # and u of a dropped pair is its prefactor times the product of the two
    # unit-normalised Gaussians' box integrals, at most prefactor * (pi/p)^(3/2) * N N'
    mu, nu = T.pair_list(b.nb)
    a, g = b.alpha[mu[dropped]], b.alpha[nu[dropped]]
    pref = np.exp(-a * g / (a + g) * np.sum((b.center[mu[dropped]] - b.center[nu[dropped]]) ** 2, axis=1))
    NN = (2 * a / np.pi) ** 0.75 * (2 * g / np.pi) ** 0.75
    assert np.all(pref <= tau)
    assert np.all(u[dropped] <= pref * (np.pi / (a + g)) ** 1.5 * NN * (1 + 1e-9))


def test_J_restricted_to_kept_pairs():
    b = I.small_random(72, natoms=5, shells=("s", "p"), box=5.0, alpha_lo=0.3, alpha_hi=20.0)
    P = I.Params(omega=0.5, nq=12, n=20, L=9.0)
    M, K, w, _ = _setup(b, P)
    D = I.random_density(np.random.default_rng(3), b)
    kept = T.screened_pairs(b.center, b.alpha, 1e-6)
    assert len(kept) < b.npair
    Jk = T.J_grid_pairs(M[:, :, kept], K, w, D, kept)
    # the kept-pair route is B restricted to kept x kept applied to D~
    B = T.B_full(M, K, w)
    Jp = np.zeros(b.npair)
    Jp[kept] = B[np.ix_(kept, kept)] @ T.density_pairs(D)[kept]
    ref = T.unpack_pairs(Jp, b.nb)
    assert np.max(np.abs(Jk - ref)) <= 1e-13 * np.max(np.abs(ref))
    # and it differs from the full J by no more than the dropped columns and rows carry
    Jf = T.J_grid(M, K, w, D)
    assert np.max(np.abs(Jk - Jf)) <= 1e-5 * np.max(np.abs(Jf))
