"""Pins of the oracle's 1D moments (eq. defV in Lagrange form) against closed
forms and an independent adaptive quadrature."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf

from oracle import exact as X
from oracle import tairef as T
from paper_2210_13069_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def _factor(center, alpha, lxyz, mu, d, x):
    """One unit-normalised Cartesian factor of g_mu in direction d."""
    l = int(lxyz[mu, d])
    return X.norm_factor(alpha[mu], l) * (x - center[mu, d]) ** l * np.exp(-alpha[mu] * (x - center[mu, d]) ** 2)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("alpha", [0.07, 1.3, 45.0])
def test_unit_norm_constant(alpha, l):
    """The oracle's constant (2l-1)!! formula against its definition: the
    squared factor integrates to one by adaptive quadrature, and it equals
    the Gauss-Hermite value of the independent checker."""
    c = T.norm_1d(alpha, l)
    val, err = integrate.quad(lambda x: (c * x ** l * math.exp(-alpha * x * x)) ** 2, -np.inf, np.inf,
                              epsabs=0.0, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) <= 1e-11
    assert abs(c - X.norm_factor(alpha, l)) <= 1e-13 * c


def test_unit_norm_constant_catches_a_wrong_double_factorial():
    """A plausible slip, (2l-1)! in place of (2l-1)!!, moves the constant for
    l >= 2 far outside the tolerance above."""
    for l in (2, 3):
        wrong = math.sqrt(math.sqrt(2.0 * 1.3 / math.pi) * (4.0 * 1.3) ** l / math.factorial(2 * l - 1))
        assert abs(wrong - X.norm_factor(1.3, l)) > 1e-3 * wrong


def test_sum_of_moments_is_truncated_overlap_s_type():
    # sum_a l_a = 1, so sum_a m_{p,d}(a) is the box-truncated 1D overlap;
    # for s functions it is an erf expression (Prop. 2.1 + eq. compact)
    b, P = I.tiny_s()
    M = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n)
    mu, nu = T.pair_list(b.nb)
    for d in range(3):
        a = b.alpha[mu]
        bb = b.alpha[nu]
        A = b.center[mu, d]
        B = b.center[nu, d]
        p = a + bb
        Pc = (a * A + bb * B) / p
        E = np.exp(-a * bb / p * (A - B) ** 2)
        Nn = (2 * a / np.pi) ** 0.25 * (2 * bb / np.pi) ** 0.25
        exact = Nn * E * 0.5 * np.sqrt(np.pi / p) * (erf(np.sqrt(p) * (P.L - Pc)) - erf(np.sqrt(p) * (-P.L - Pc)))
        np.testing.assert_allclose(M[d].sum(axis=0), exact, rtol=2e-14, atol=1e-300)


def test_box_truncation_near_edge():
    # a diffuse s function centred near the box edge: the truncated integral
    # differs from the full-line one, and the moments follow the truncated one
    L, n = 4.0, 16
    center = np.array([[3.5, 0.0, 0.0]])
    alpha = np.array([0.3])
    lxyz = np.zeros((1, 3), dtype=np.int32)
    M = T.moments(center, alpha, lxyz, L, n)
    p = 0.6
    Nn = math.sqrt(2 * 0.3 / math.pi)
    trunc = Nn * 0.5 * math.sqrt(math.pi / p) * (erf(math.sqrt(p) * (L - 3.5)) - erf(math.sqrt(p) * (-L - 3.5)))
    full = Nn * math.sqrt(math.pi / p)
    assert abs(M[0].sum() - trunc) < 1e-14 * trunc
    assert abs(trunc - full) > 1e-2 * full


@pytest.mark.parametrize("kind", [T.NODES_LOBATTO, T.NODES_GAUSS])
def test_moments_against_adaptive_quadrature(kind):
    # m_{p,d}(a) and the power moments sum_a xi_a^j m(a) = int x^j g g,
    # j <= n-1, against scipy's adaptive Gauss-Kronrod with the Lagrange
    # basis in product form (no barycentric formula)
    bas = I.small_random(11, natoms=3, shells=("s", "p", "d"), box=2.5, alpha_lo=0.2, alpha_hi=30.0)
    L, n = 6.0, 12
    M = T.moments(bas.center, bas.alpha, bas.lxyz, L, n, kind=kind)
    xi, _ = T.cheb_nodes(n, L, kind)
    mu, nu = T.pair_list(bas.nb)
    rng = np.random.default_rng(4)
    for p in rng.choice(len(mu), 25, replace=False):
        for d in range(3):
            def f(x, p=p, d=d):
                return (_factor(bas.center, bas.alpha, bas.lxyz, mu[p], d, x)
                        * _factor(bas.center, bas.alpha, bas.lxyz, nu[p], d, x))
            scale = integrate.quad(lambda x: abs(f(x)), -L, L, epsabs=0, epsrel=1e-13, limit=400)[0]
            for a in (0, n // 2, n - 1):
                def la(x, a=a):
                    v = 1.0
                    for bnode in range(n):
                        if bnode != a:
                            v *= (x - xi[bnode]) / (xi[a] - xi[bnode])
                    return v
                ref = integrate.quad(lambda x: f(x) * la(x), -L, L, epsabs=0, epsrel=1e-13, limit=400)[0]
                assert abs(M[d, a, p] - ref) <= 1e-12 * scale, (p, d, a, M[d, a, p], ref)
            for j in (0, 1, 3, n - 1):
                ref = integrate.quad(lambda x: f(x) * (x / L) ** j, -L, L, epsabs=0, epsrel=1e-13, limit=400)[0]
                got = np.sum((xi / L) ** j * M[d, :, p])
                assert abs(got - ref) <= 1e-12 * scale, (p, d, j, got, ref)


def test_moments_pair_subset_and_symmetry():
    bas = I.small_random(5, natoms=2, shells=("s", "p"), box=2.0)
    L, n = 8.0, 16
    M = T.moments(bas.center, bas.alpha, bas.lxyz, L, n)
    sel = np.array([5, 0, 17, 3])
    Ms = T.moments(bas.center, bas.alpha, bas.lxyz, L, n, pairs=sel)
    np.testing.assert_array_equal(Ms, M[:, :, sel])
    # g_mu g_nu = g_nu g_mu: swapping the functions of a pair gives the same
    # moments (compute the swapped pair by reversing the basis order)
    perm = np.arange(bas.nb)[::-1]
    M2 = T.moments(bas.center[perm], bas.alpha[perm], bas.lxyz[perm], L, n)
    mu, nu = T.pair_list(bas.nb)
    nb = bas.nb
    for p in range(len(mu)):
        q = T.pair_index(nb, nb - 1 - nu[p], nb - 1 - mu[p])
        np.testing.assert_allclose(M2[:, :, q], M[:, :, p], rtol=1e-13, atol=1e-15)


def test_coef_multiplies_the_function():
    bas = I.small_random(6, natoms=2, shells=("s", "p"), box=2.0)
    L, n = 8.0, 10
    M = T.moments(bas.center, bas.alpha, bas.lxyz, L, n)
    c, nd = T.basis_scale(bas.alpha, bas.lxyz, None)
    coef = np.prod(nd, axis=1) * np.linspace(0.5, 2.0, bas.nb)
    Mc = T.moments(bas.center, bas.alpha, bas.lxyz, L, n, coef=coef)
    mu, nu = T.pair_list(bas.nb)
    s = np.linspace(0.5, 2.0, bas.nb)
    ref = np.prod(M, axis=0) * (s[mu] * s[nu])[None, :]
    np.testing.assert_allclose(np.prod(Mc, axis=0), ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
