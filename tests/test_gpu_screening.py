"""GPU parity of pair screening (section 6.3, compression by screening): the
kept list exactly, the moments of the kept pairs, B over them in every
arithmetic and J with the pair sums restricted to them, through the C ABI
against the oracle on the same seeded inputs.  Tolerances are those of the
unscreened paths."""
import numpy as np
import pytest

from oracle import tairef as T
from paper_2210_13069_amd import inputs as I

pytestmark = pytest.mark.gpu

LOWP_TOL = {1: 1e-6, 2: 3e-5, 3: 1e-6, 4: 1e-6}


def _normwise(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _not_a_tie(b, tau):
    # the keep decision is an FP64 comparison on both sides; the lists are
    # compared exactly where no prefactor lies within rounding of tau
    mu, nu = T.pair_list(b.nb)
    a, g = b.alpha[mu], b.alpha[nu]
    pref = np.exp(-a * g / (a + g) * np.sum((b.center[mu] - b.center[nu]) ** 2, axis=1))
    assert not np.any(np.abs(pref - tau) <= 1e-12 * tau)


@pytest.mark.parametrize("case", ["sp16", "spd400", "jbuild1000"])
@pytest.mark.parametrize("tau", [0.0, 1e-8, 1e-12])
def test_screen_matches_oracle(tai, case, tau):
    if case == "sp16":
        b, _ = I.sp16()
    elif case == "spd400":
        b, _ = I.spd400()
    else:
        b, _, _ = I.jbuild1000()
    if tau > 0:
        _not_a_tie(b, tau)
    kept = tai.screen_pairs(b, tau).cpu().numpy()
    np.testing.assert_array_equal(kept, T.screened_pairs(b.center, b.alpha, tau))


def _moments_check(Mg, Mr):
    scale = np.max(np.abs(Mr), axis=1, keepdims=True)
    assert np.all(np.abs(Mg - Mr) <= 1e-12 * scale + 1e-300)


def test_moments_pairs_match_oracle(tai):
    b, P = I.sp16()
    pairs = tai.screen_pairs(b, 1e-10)
    kept = pairs.cpu().numpy().astype(np.int64)
    assert len(kept) < b.npair
    Mg = tai.moments_pairs(b, P, pairs).cpu().numpy()
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, pairs=kept)
    _moments_check(Mg, Mr)
    # an arbitrary (unsorted, repeated) list works too
    import torch
    lst = torch.as_tensor(np.array([5, 0, b.npair - 1, 5, 17], dtype=np.int32), device=pairs.device)
    Mg2 = tai.moments_pairs(b, P, lst).cpu().numpy()
    _moments_check(Mg2, T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, pairs=[5, 0, b.npair - 1, 5, 17]))


@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4])
def test_assemble_B_screened(tai, prec):
    b = I.small_random(73, natoms=10, shells=("s", "p", "d"), box=6.0, alpha_lo=0.2, alpha_hi=40.0)
    P = I.Params(omega=0.4, nq=16, n=32, L=10.0)
    pairs = tai.screen_pairs(b, 1e-8)
    kept = pairs.cpu().numpy().astype(np.int64)
    assert 64 < len(kept) < b.npair
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, pairs=kept)
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L)
    Br = T.B_full(Mr, T.ktables(t, xi), w)
    Mg = tai.moments_pairs(b, P, pairs)
    Bg = tai.assemble_B(Mg, P, prec=prec).cpu().numpy().astype(np.float64)
    tol = 1e-10 if prec == 0 else LOWP_TOL[prec]
    assert _normwise(Bg, Br) <= tol, (prec, _normwise(Bg, Br))


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_J_pairs(tai, prec):
    import torch
    b = I.small_random(74, natoms=8, shells=("s", "p", "d"), box=5.0, alpha_lo=0.2, alpha_hi=30.0)
    P = I.Params(omega=0.4, nq=12, n=40, L=9.0)
    D = I.random_density(np.random.default_rng(9), b)
    pairs = tai.screen_pairs(b, 1e-8)
    kept = pairs.cpu().numpy().astype(np.int64)
    assert len(kept) < b.npair
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, pairs=kept)
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L)
    Jr = T.J_grid_pairs(Mr, T.ktables(t, xi), w, D, kept)
    Mg = tai.moments_pairs(b, P, pairs)
    Jg = tai.apply_J_pairs(Mg, torch.as_tensor(D, device=Mg.device), pairs, P, prec=prec).cpu().numpy()
    err = np.linalg.norm(Jg - Jr, 2) / np.linalg.norm(Jr, 2)
    assert err <= (1e-10 if prec == 0 else 1e-6), err
    np.testing.assert_array_equal(Jg, Jg.T)
    mu, nu = T.pair_list(b.nb)
    dropped = np.setdiff1d(np.arange(b.npair), kept)
    assert np.all(Jg[mu[dropped], nu[dropped]] == 0.0)


def test_screened_J_full_size_close_to_unscreened(tai):
    """Nb = 1000 at tau = 1e-12: J over the kept pairs (19% of them) against
    the unscreened GPU J, a property that holds at any size: the dropped
    pairs carry prefactors below 1e-12."""
    import torch
    b, P, D = I.jbuild1000()
    Dg = torch.as_tensor(D, device="cuda")
    Jf = tai.apply_J(tai.moments(b, P), Dg, P)
    pairs = tai.screen_pairs(b, 1e-12)
    assert len(pairs) < 0.25 * b.npair
    Js = tai.apply_J_pairs(tai.moments_pairs(b, P, pairs), Dg, pairs, P)
    rel = float(torch.linalg.matrix_norm(Js - Jf, 2) / torch.linalg.matrix_norm(Jf, 2))
    assert rel <= 1e-9, rel


def test_screen_keeps_only_diagonal(tai):
    """tau just below 1 keeps exactly the nb diagonal pairs of well separated
    functions; B over them in FP64 against the oracle."""
    b = I.small_random(75, natoms=4, shells=("s",), box=6.0, alpha_lo=2.0, alpha_hi=8.0)
    pairs = tai.screen_pairs(b, 0.999999)
    kept = pairs.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(kept, T.screened_pairs(b.center, b.alpha, 0.999999))
    np.testing.assert_array_equal(kept, [T.pair_index(b.nb, m, m) for m in range(b.nb)])
    P = I.Params(omega=0.5, nq=8, n=16, L=10.0)
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, pairs=kept)
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L)
    Br = T.B_full(Mr, T.ktables(t, xi), w)
    Bg = tai.assemble_B(tai.moments_pairs(b, P, pairs), P, prec=0).cpu().numpy()
    assert np.max(np.abs(Bg - Br)) <= 1e-10 * np.max(np.abs(Br))
