"""GPU parity of the long-range exchange matrix (appendix B, eq. exchange)
through the C ABI: FP64 and FP32 against the oracle's factorized grid form and
the equation written out over B, over all pairs and over a screened pair
list, and with the compressed moments."""
import dataclasses

import numpy as np
import pytest

from oracle import tairef as T
from paper_2210_13069_amd import inputs as I

pytestmark = pytest.mark.gpu


def _tables(P):
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L)
    return T.ktables(t, xi), w


@pytest.mark.parametrize("prec", [0, 1])
def test_exchange_matches_oracle(tai, prec):
    import torch
    b = I.small_random(101, natoms=4, shells=("s", "p"), box=3.0, alpha_lo=0.2, alpha_hi=20.0)
    P = I.Params(omega=0.4, nq=10, n=24, L=8.0)
    Q = np.random.default_rng(7).standard_normal((3, b.nb))
    K, w = _tables(P)
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n)
    ref = T.exchange_grid(Mr, K, w, Q)
    assert np.max(np.abs(ref - T.exchange_direct(T.B_full(Mr, K, w), Q))) <= 1e-12 * np.max(np.abs(ref))
    Mg = tai.moments(b, P)
    got = tai.exchange(Mg, b.nb, torch.as_tensor(Q, device=Mg.device), P, prec=prec).cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= (1e-10 if prec == 0 else 1e-6), err
    assert np.max(np.abs(got - got.T)) <= (1e-13 if prec == 0 else 1e-6) * np.max(np.abs(got))


def test_exchange_screened_pairs(tai):
    """Over the pairs kept by screening: the equation over B with the dropped
    pairs' rows and columns set to zero."""
    import torch
    b = I.small_random(102, natoms=6, shells=("s", "p"), box=5.0, alpha_lo=0.3, alpha_hi=30.0)
    P = I.Params(omega=0.4, nq=8, n=16, L=9.0)
    Q = np.random.default_rng(8).standard_normal((2, b.nb))
    pairs = tai.screen_pairs(b, 1e-6)
    kept = pairs.cpu().numpy().astype(np.int64)
    assert len(kept) < b.npair
    K, w = _tables(P)
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n)
    B = T.B_full(Mr, K, w)
    mask = np.zeros(b.npair, dtype=bool)
    mask[kept] = True
    B[~mask, :] = 0.0
    B[:, ~mask] = 0.0
    ref = T.exchange_direct(B, Q)
    Mk = tai.moments_pairs(b, P, pairs)
    got = tai.exchange(Mk, b.nb, torch.as_tensor(Q, device=Mk.device), P, pairs=pairs).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_exchange_compressed(tai):
    import torch
    b = I.small_random(103, natoms=4, shells=("s", "p", "d"), box=3.0, alpha_lo=0.2, alpha_hi=20.0)
    P = I.Params(omega=0.4, nq=10, n=24, L=8.0, rank_tol=1e-6)
    Q = np.random.default_rng(9).standard_normal((2, b.nb))
    K, w = _tables(P)
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n)
    V, s, R = T.compression_basis(Mr, P.rank_tol)
    assert np.all(np.abs(s / s[0] - P.rank_tol) > 1e-6 * P.rank_tol)
    ref = T.exchange_grid(*T.compress(Mr, K, V), w, Q)
    Mg = tai.moments(b, P)
    got = tai.exchange(Mg, b.nb, torch.as_tensor(Q, device=Mg.device), P).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.fixture(scope="module")
def multi_tile():
    """nb = 92: two lambda batches per X tensor, two 64-row tiles of the
    final product, a ragged tail in both."""
    b = I.small_random(104, natoms=23, shells=("s", "p"), box=5.0, alpha_lo=0.2, alpha_hi=20.0)
    P = I.Params(omega=0.5, nq=8, n=16, L=9.0)
    Q = np.random.default_rng(10).standard_normal((3, b.nb)) / np.sqrt(b.nb)
    K, w = _tables(P)
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n)
    return b, P, Q, T.exchange_grid(Mr, K, w, Q)


@pytest.mark.parametrize("prec", [0, 1])
def test_exchange_multi_tile(tai, multi_tile, prec):
    import torch
    b, P, Q, ref = multi_tile
    assert b.nb == 92
    Mg = tai.moments(b, P)
    got = tai.exchange(Mg, b.nb, torch.as_tensor(Q, device=Mg.device), P, prec=prec).cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= (1e-10 if prec == 0 else 1e-6), err
    # each entry and its mirror come from the same partial sums (the tiles on
    # and above the diagonal), across the two 64-row tiles too
    assert np.array_equal(got, got.T)


def test_exchange_chunked_tensors_bit_equal(tai, multi_tile, monkeypatch):
    """The mode products taken a few tensors at a time (TAI_EXCHANGE_CHUNK)
    give the same bits as in one chunk, and the call is deterministic."""
    import torch
    b, P, Q, ref = multi_tile
    Mg = tai.moments(b, P)
    Qg = torch.as_tensor(Q, device=Mg.device)
    one = tai.exchange(Mg, b.nb, Qg, P)
    assert torch.equal(one, tai.exchange(Mg, b.nb, Qg, P))
    monkeypatch.setenv("TAI_EXCHANGE_CHUNK", "7")
    chunked = tai.exchange(Mg, b.nb, Qg, P)
    assert torch.equal(one, chunked)


@pytest.mark.parametrize("n", [37, 40])
def test_exchange_two_slab_products(tai, n, monkeypatch):
    """33 <= n <= 40 takes the slab products two slabs per work group (the
    products K [X X'] and [U; U'] K^T packed side by side). 5 s functions
    and 3 orbitals give 15 tensors: at n = 37 the slab count is odd, so the
    last work group holds one slab, and for n < 40 the inner index runs past
    n against the zero columns of K. Against the oracle's grid form, and
    bit-equal when the tensors run in chunks of 7."""
    import torch
    b = I.small_random(105, natoms=5, shells=("s",), box=4.0, alpha_lo=0.2, alpha_hi=20.0)
    assert b.nb == 5
    P = I.Params(omega=0.5, nq=6, n=n, L=8.0)
    Q = np.random.default_rng(11).standard_normal((3, b.nb)) / np.sqrt(b.nb)
    K, w = _tables(P)
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n)
    ref = T.exchange_grid(Mr, K, w, Q)
    Mg = tai.moments(b, P)
    Qg = torch.as_tensor(Q, device=Mg.device)
    got = tai.exchange(Mg, b.nb, Qg, P)
    err = np.max(np.abs(got.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err <= 1e-10, (n, err)
    monkeypatch.setenv("TAI_EXCHANGE_CHUNK", "7")
    assert torch.equal(tai.exchange(Mg, b.nb, Qg, P), got)
