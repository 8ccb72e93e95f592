"""Pins of the oracle's contracted basis functions (eq. basis with I_mu > 1
primitives each): B over contracted pairs against a plain four-fold loop over
the exact s-type integrals of the primitives, J over contracted functions
against B_c applied to the contracted density, and the trivial contraction."""
import math

import numpy as np

from oracle import exact as X
from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


def _contracted_s(seed):
    # 5 contracted s functions with 1..3 primitives each at 4 centres
    rng = np.random.default_rng(seed)
    nprim = [3, 1, 2, 3, 2]
    centres = rng.uniform(-2.0, 2.0, size=(5, 3))
    fmap, center, alpha, coef = [], [], [], []
    for f, k in enumerate(nprim):
        a = np.exp(rng.uniform(np.log(0.3), np.log(12.0), size=k))
        c = rng.uniform(0.2, 1.0, size=k)
        for j in range(k):
            fmap.append(f)
            center.append(centres[f])
            alpha.append(a[j])
            coef.append(c[j])
    return np.array(fmap), np.array(center), np.array(alpha), np.array(coef)


def test_contracted_B_matches_fourfold_loop_s_type():
    fmap, center, alpha, coef = _contracted_s(3)
    nb = int(fmap[-1]) + 1
    omega = 0.5
    # TA over the primitive pairs at converged parameters, then contracted
    lxyz = np.zeros((len(alpha), 3), dtype=np.int64)
    M = T.moments(center, alpha, lxyz, 12.0, 64, coef=coef)
    t, w = T.time_nodes(omega, 32)
    xi, _ = T.cheb_nodes(64, 12.0)
    Bc = T.contract_pairs(T.B_full(M, T.ktables(t, xi), w), fmap)
    # exact: sum over every primitive of each of the four functions
    members = [np.nonzero(fmap == f)[0] for f in range(nb)]
    mu, nu = T.pair_list(nb)
    ref = np.zeros((len(mu), len(mu)))
    for P in range(len(mu)):
        for Q in range(P, len(mu)):
            s = 0.0
            for i in members[mu[P]]:
                for j in members[nu[P]]:
                    for k in members[mu[Q]]:
                        for l in members[nu[Q]]:
                            s += coef[i] * coef[j] * coef[k] * coef[l] * X.eri_lr_ss(
                                center[i], alpha[i], center[j], alpha[j], center[k], alpha[k], center[l], alpha[l],
                                omega)
            ref[P, Q] = ref[Q, P] = s
    assert np.max(np.abs(Bc - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_contracted_J_equals_contracted_B_times_density():
    rng = np.random.default_rng(4)
    prim = I.random_molecule(rng, 3, 2.0, ["s", "s", "p"], 0.3, 8.0)
    # contract: the two s primitives of each atom form one function; p stays
    fmap, f = [], -1
    for a in range(3):
        f += 1
        fmap += [f, f]          # s, s
        for _ in range(3):      # px, py, pz
            f += 1
            fmap.append(f)
    fmap = np.array(fmap)
    nb = f + 1
    coef = rng.uniform(0.3, 1.0, prim.nb)
    M = T.moments(prim.center, prim.alpha, prim.lxyz, 8.0, 16, coef=coef)
    t, w = T.time_nodes(0.5, 12)
    xi, _ = T.cheb_nodes(16, 8.0)
    K = T.ktables(t, xi)
    A = rng.standard_normal((nb, nb))
    D = A + A.T
    Jc = T.contract_functions(T.J_grid(M, K, w, T.expand_density(D, fmap)), fmap)
    Bc = T.contract_pairs(T.B_full(M, K, w), fmap)
    ref = T.unpack_pairs(Bc @ T.density_pairs(D), nb)
    assert np.max(np.abs(Jc - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_trivial_contraction_is_identity():
    b = I.small_random(5, natoms=2, shells=("s", "p"))
    fmap = np.arange(b.nb)
    rng = np.random.default_rng(6)
    Bp = rng.standard_normal((b.npair, b.npair))
    np.testing.assert_array_equal(T.contract_pairs(Bp, fmap), Bp)
    Jp = rng.standard_normal((b.nb, b.nb))
    np.testing.assert_array_equal(T.contract_functions(Jp, fmap), Jp)
    P, w = T.contraction_pairs(fmap)
    np.testing.assert_array_equal(P, np.arange(b.npair))
    assert np.all(w == 1.0)
