"""Pins of the oracle's B (Algorithm 1, Theorem 3.1, eq. tensors) against the
exact long-range integral and against invariants that the method preserves."""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


def _ta(basis, omega, nq, n, L, kind=T.NODES_LOBATTO):
    M = T.moments(basis.center, basis.alpha, basis.lxyz, L, n, kind=kind)
    t, w = T.time_nodes(omega, nq)
    xi, _ = T.cheb_nodes(n, L, kind)
    return M, T.ktables(t, xi), w


def test_closed_form_pinned_by_bruteforce_6d():
    # the s-type closed form is itself checked against direct 6D product
    # Gauss-Hermite integration of erf(w r)/r (no t-integral involved)
    b, P = I.tiny_s()
    fn = [X.basis_function(b.center, b.alpha, b.lxyz, m) for m in range(b.nb)]
    N = (2 * b.alpha / np.pi) ** 0.75
    for (m1, m2, m3, m4) in [(0, 1, 2, 3), (0, 0, 0, 0), (1, 5, 2, 7), (3, 3, 6, 6), (4, 7, 4, 7)]:
        c = X.eri_lr_ss(b.center[m1], b.alpha[m1], b.center[m2], b.alpha[m2],
                        b.center[m3], b.alpha[m3], b.center[m4], b.alpha[m4], P.omega)
        c *= N[m1] * N[m2] * N[m3] * N[m4]
        bf = X.eri_lr_bruteforce([fn[m1], fn[m2], fn[m3], fn[m4]], P.omega, m=14)
        assert abs(bf - c) <= 1e-12 * abs(c), (m1, m2, m3, m4, bf, c)
        semi = X.eri_lr_semi([fn[m1], fn[m2], fn[m3], fn[m4]], P.omega)
        assert abs(semi - c) <= 1e-13 * abs(c)


def test_semi_analytic_pd_pinned_by_bruteforce():
    bas = I.small_random(7, natoms=3, shells=("s", "p", "d"), box=2.0, alpha_lo=0.4, alpha_hi=4.0)
    fn = [X.basis_function(bas.center, bas.alpha, bas.lxyz, m) for m in range(bas.nb)]
    rng = np.random.default_rng(2)
    for _ in range(4):
        m = rng.integers(0, bas.nb, 4)
        semi = X.eri_lr_semi([fn[i] for i in m], 0.5)
        bf = X.eri_lr_bruteforce([fn[i] for i in m], 0.5, m=14)
        assert abs(semi - bf) <= 1e-11 * max(abs(semi), 1e-3), (m, semi, bf)


def test_algorithm1_equals_theorem31_matrix_form():
    b, P = I.sp16()
    M, K, w = _ta(b, P.omega, P.nq, P.n, P.L)
    rng = np.random.default_rng(0)
    rows = rng.choice(b.npair, 40, replace=False)
    Bm = T.B_full(M, K, w, rows=rows)
    cols = rng.integers(0, b.npair, 400)
    r = np.repeat(rows, 10)
    c = cols[:len(r)]
    e = T.B_entries(M, K, w, r, c)
    ref = Bm[np.repeat(np.arange(40), 10), c]
    assert np.max(np.abs(e - ref)) <= 1e-14 * np.max(np.abs(Bm))


def test_hadamard_form_equals_kronecker_form():
    # Prop. 2.5: (A<>B)(C(x)D) and (A<>B)(C*D) identities turn eq. tensors
    # into the Hadamard form of Theorem 3.1; compare on a tiny case
    bas = I.small_random(3, natoms=2, shells=("s", "p"), box=1.5)
    M, K, w = _ta(bas, 0.6, 4, 6, 5.0)
    Bh = T.B_full(M, K, w)
    Bk = T.B_kronecker(M, K, w)
    assert np.max(np.abs(Bh - Bk)) <= 1e-14 * np.max(np.abs(Bk))


def test_tight_parameters_match_closed_form_s():
    # the whole TA chain against physics at converged parameters
    b, _ = I.tiny_s()
    M, K, w = _ta(b, 0.5, 32, 64, 12.0)
    B = T.B_full(M, K, w)
    Bc = X.B_closed_form_s(b.center, b.alpha, 0.5)
    assert np.max(np.abs(B - Bc)) <= 1e-12 * np.max(np.abs(Bc))
    assert np.max(np.abs(B - Bc) / np.abs(Bc)) <= 1e-12


def test_tight_parameters_match_closed_form_s_gauss_nodes():
    b, _ = I.tiny_s()
    M, K, w = _ta(b, 0.5, 32, 64, 12.0, kind=T.NODES_GAUSS)
    B = T.B_full(M, K, w)
    Bc = X.B_closed_form_s(b.center, b.alpha, 0.5)
    assert np.max(np.abs(B - Bc)) <= 1e-12 * np.max(np.abs(Bc))


def test_tight_parameters_match_semi_analytic_pd():
    bas = I.small_random(7, natoms=3, shells=("s", "p", "d"), box=2.0, alpha_lo=0.4, alpha_hi=4.0)
    M, K, w = _ta(bas, 0.5, 32, 64, 12.0)
    mu, nu = T.pair_list(bas.nb)
    fn = [X.basis_function(bas.center, bas.alpha, bas.lxyz, m) for m in range(bas.nb)]
    rng = np.random.default_rng(0)
    ps = rng.integers(0, bas.npair, 16)
    qs = rng.integers(0, bas.npair, 16)
    ta = T.B_entries(M, K, w, ps, qs)
    ref = np.array([X.eri_lr_semi([fn[mu[p]], fn[nu[p]], fn[mu[q]], fn[nu[q]]], 0.5) for p, q in zip(ps, qs)])
    diag = T.B_entries(M, K, w, np.arange(bas.npair), np.arange(bas.npair))
    assert np.max(np.abs(ta - ref)) <= 1e-12 * np.max(np.abs(diag))


def test_config_params_error_and_convergence_in_n():
    # tiny_s at its own parameters (n=24, L=8, nq=16): the interpolation error
    # dominates; it must fall as n grows (paper section 6.1)
    b, P = I.tiny_s()
    Bc = X.B_closed_form_s(b.center, b.alpha, P.omega)
    errs = []
    for n in (24, 32, 40):
        M, K, w = _ta(b, P.omega, P.nq, n, P.L)
        errs.append(np.max(np.abs(T.B_full(M, K, w) - Bc) / np.abs(Bc)))
    assert errs[0] < 5e-5
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-10


def test_convergence_in_nq():
    b, _ = I.tiny_s()
    Bc = X.B_closed_form_s(b.center, b.alpha, 0.5)
    errs = []
    for nq in (2, 4, 8, 12):
        M, K, w = _ta(b, 0.5, nq, 64, 12.0)
        errs.append(np.max(np.abs(T.B_full(M, K, w) - Bc)) / np.max(np.abs(Bc)))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-10


def test_symmetry_psd_cauchy_schwarz():
    b, P = I.sp16()
    M, K, w = _ta(b, P.omega, P.nq, P.n, P.L)
    B = T.B_full(M, K, w)
    scale = np.max(np.abs(B))
    assert np.max(np.abs(B - B.T)) <= 1e-15 * scale * 4
    ev = np.linalg.eigvalsh(0.5 * (B + B.T))
    assert ev.min() >= -1e-13 * ev.max()
    d = np.sqrt(np.maximum(np.diag(B), 0))
    assert np.all(np.abs(B) <= np.outer(d, d) * (1 + 1e-12) + 1e-15 * scale)


def test_eightfold_index_symmetry():
    # B(mu nu, kl) is invariant under mu<->nu, k<->l and (mu nu)<->(k l); with
    # pairs mu<=nu the first two are built in, the third is B = B^T, and the
    # unfolded Nb^4 tensor built from B has all eight symmetries
    bas = I.small_random(9, natoms=2, shells=("s", "p"), box=2.0)
    M, K, w = _ta(bas, 0.5, 8, 16, 8.0)
    B = T.B_full(M, K, w)
    nb = bas.nb
    idx = np.zeros((nb, nb), dtype=np.int64)
    mu, nu = T.pair_list(nb)
    idx[mu, nu] = np.arange(len(mu))
    idx[nu, mu] = np.arange(len(mu))
    G = B[idx[:, :, None, None], idx[None, None, :, :]]
    scale = np.max(np.abs(G))
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.max(np.abs(G - np.transpose(G, perm))) <= 4e-15 * scale


def test_small_omega_limit():
    # erf(w r)/r -> 2w/sqrt(pi) as w -> 0, so B/w -> (2/sqrt(pi)) S_p S_q with
    # S the box-truncated overlaps; relative deviation is O(w^2)
    b, P = I.tiny_s()
    omega = 1e-3
    M, K, w = _ta(b, omega, 4, P.n, P.L)
    B = T.B_full(M, K, w)
    S = np.prod(M.sum(axis=1), axis=0)
    ref = omega * 2 / math.sqrt(math.pi) * np.outer(S, S)
    assert np.max(np.abs(B - ref)) <= 1e-4 * np.max(np.abs(ref))


def test_large_omega_is_reported_not_asserted(capsys):
    # the paper finds TA degrades as omega grows (section 6.1); report it
    b, _ = I.tiny_s()
    Bc = X.B_closed_form_s(b.center, b.alpha, 1.0)
    M, K, w = _ta(b, 1.0, 32, 40, 16.0)
    err = np.max(np.abs(T.B_full(M, K, w) - Bc)) / np.max(np.abs(Bc))
    print(f"omega=1.0 n=40 L=16 normwise error vs closed form: {err:.3e}")
    assert np.isfinite(err)
