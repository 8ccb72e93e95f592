"""Exact long-range integrals that the tensorized approximation converges to.

TEST INFRASTRUCTURE ONLY.  These references pin the oracle in `tairef` to
mathematics that does not pass through any of its steps (no Chebyshev
interpolation, no moments, no K tables):

* `eri_lr_ss`: closed form of the erf-attenuated Coulomb integral over four
  s-type Gaussians, from the Gaussian product rule (Prop. 2.1) and the kernel
  identity erf(w r)/r = (2/sqrt(pi)) int_0^w exp(-s^2 r^2) ds (eq. kernel):
      (ss|ss)_w = E_ab E_cd 2 pi^(5/2) / (p q sqrt(p+q)) * sqrt(w^2/(w^2+rho))
                  * F0(rho w^2/(w^2+rho) |P-Q|^2),  rho = pq/(p+q),
  with the Boys function F0(T) = (1/2) sqrt(pi/T) erf(sqrt(T)).
* `eri_lr_semi`: Cartesian Gaussians of any power.  For each t, each direction
  factorises (the per-direction separability after eq. TEI2) into a 2D
  integral of polynomial x Gaussian, taken exactly by tensor Gauss-Hermite
  after completing the square; the t-integral of eq. kernel is then taken by
  Gauss-Legendre, doubled until converged.
* `eri_lr_bruteforce`: direct 6D product Gauss-Hermite quadrature of
  g g K(x,y) g g with K = erf(w r)/r, no t-integral at all.

The integrals are over all of R^3 x R^3 (no box); tests choose the box large
enough that truncation is far below their tolerance.

Nothing here is taken from `tairef`: the Gauss-Legendre rule of the
t-integral is scipy's, and the unit-norm constant of a Cartesian factor is
computed from its own definition, 1 / sqrt(int (x^l exp(-alpha x^2))^2 dx),
by a Gauss-Hermite rule that is exact for that integrand.
"""
import math

import numpy as np
from scipy.special import erf, roots_hermite, roots_legendre

SQRT_PI = math.sqrt(math.pi)


def norm_factor(alpha, l):
    """Constant c with int (c x^l exp(-alpha x^2))^2 dx = 1, from that
    integral itself: with u = sqrt(2 alpha) x it is
    (2 alpha)^(-l-1/2) int u^(2l) exp(-u^2) du, which the (l+1)-point
    Gauss-Hermite rule integrates exactly (degree 2l <= 2(l+1) - 1)."""
    u, wu = roots_hermite(l + 1)
    integral = (2.0 * alpha) ** (-l - 0.5) * float(np.sum(wu * u ** (2 * l)))
    return 1.0 / math.sqrt(integral)


def boys_f0(T):
    """F0(T) = int_0^1 exp(-T u^2) du; series for small T."""
    T = np.asarray(T, dtype=np.float64)
    out = np.empty_like(T)
    small = T < 1e-6
    Ts = T[small]
    out[small] = 1.0 - Ts / 3.0 + Ts * Ts / 10.0
    Tl = T[~small]
    out[~small] = 0.5 * np.sqrt(np.pi / Tl) * erf(np.sqrt(Tl))
    return out


def _pair_gauss(A, a, B, b):
    p = a + b
    P = (a * A + b * B) / p
    E = np.exp(-a * b / p * np.sum((A - B) ** 2, axis=-1))
    return p, P, E


def eri_lr_ss(cA, aA, cB, aB, cC, aC, cD, aD, omega):
    """(ab|erf(w r)/r|cd) for four unnormalised s-type Gaussians
    exp(-a|x-A|^2) (scalars; centres are 3-vectors)."""
    cA, cB, cC, cD = (np.asarray(v, dtype=np.float64) for v in (cA, cB, cC, cD))
    p, P, Eab = _pair_gauss(cA, aA, cB, aB)
    q, Q, Ecd = _pair_gauss(cC, aC, cD, aD)
    rho = p * q / (p + q)
    R2 = float(np.sum((P - Q) ** 2))
    att = omega * omega / (omega * omega + rho)
    return float(Eab * Ecd * 2.0 * math.pi ** 2.5 / (p * q * math.sqrt(p + q))
                 * math.sqrt(att) * boys_f0(np.array([rho * att * R2]))[0])


def B_closed_form_s(center, alpha, omega, rows=None, cols=None):
    """Pair matrix B(p,q) of unit-normalised s-type functions by the closed
    form, over all pairs (or the given pair rows/cols)."""
    center = np.asarray(center, dtype=np.float64).reshape(-1, 3)
    alpha = np.asarray(alpha, dtype=np.float64)
    nb = len(alpha)
    mu, nu = np.triu_indices(nb)
    r = np.arange(len(mu)) if rows is None else np.asarray(rows)
    c = np.arange(len(mu)) if cols is None else np.asarray(cols)
    N = (2.0 * alpha / math.pi) ** 0.75

    def pair_data(sel):
        a = alpha[mu[sel]]
        b = alpha[nu[sel]]
        A = center[mu[sel]]
        Bc = center[nu[sel]]
        p = a + b
        P = (a[:, None] * A + b[:, None] * Bc) / p[:, None]
        E = np.exp(-a * b / p * np.sum((A - Bc) ** 2, axis=1))
        return p, P, E * N[mu[sel]] * N[nu[sel]]

    pr, Pr, Er = pair_data(r)
    pc, Pc, Ec = pair_data(c)
    p = pr[:, None]
    q = pc[None, :]
    rho = p * q / (p + q)
    R2 = np.sum((Pr[:, None, :] - Pc[None, :, :]) ** 2, axis=-1)
    att = omega * omega / (omega * omega + rho)
    return (Er[:, None] * Ec[None, :] * 2.0 * math.pi ** 2.5 / (p * q * np.sqrt(p + q))
            * np.sqrt(att) * boys_f0(rho * att * R2))


# ---------------------------------------------------------------------------
# Semi-analytic reference for Cartesian Gaussians of any power
# ---------------------------------------------------------------------------
def _poly_gauss_2d(t2, fx, fy, gh_u, gh_w):
    """int int Px(x) Py(y) exp(-p(x-P)^2 - q(y-Q)^2 - t2 (x-y)^2) dx dy.

    fx = (A, a, la, B, b, lb) for the x-pair, fy likewise for y.  The
    quadratic form is diagonalised by its Cholesky factor; tensor
    Gauss-Hermite of order m is exact for polynomial degree <= 2m-1.
    """
    A, a, la, B, b, lb = fx
    C, c, lc, D, dd, ld = fy
    p = a + b
    P = (a * A + b * B) / p
    Exy = math.exp(-a * b / p * (A - B) ** 2)
    q = c + dd
    Q = (c * C + dd * D) / q
    Ezy = math.exp(-c * dd / q * (C - D) ** 2)
    # exponent: -(z-c0)^T S (z-c0) - const
    S = np.array([[p + t2, -t2], [-t2, q + t2]])
    rhs = np.array([p * P, q * Q])
    c0 = np.linalg.solve(S, rhs)
    const = p * P * P + q * Q * Q - rhs @ c0
    Lc = np.linalg.cholesky(S)          # S = Lc Lc^T
    LinvT = np.linalg.inv(Lc).T         # z = c0 + LinvT u
    U1, U2 = np.meshgrid(gh_u, gh_u, indexing="ij")
    W = np.outer(gh_w, gh_w)
    X = c0[0] + LinvT[0, 0] * U1 + LinvT[0, 1] * U2
    Y = c0[1] + LinvT[1, 0] * U1 + LinvT[1, 1] * U2
    poly = (X - A) ** la * (X - B) ** lb * (Y - C) ** lc * (Y - D) ** ld
    det = Lc[0, 0] * Lc[1, 1]
    return Exy * Ezy * math.exp(-const) * np.sum(W * poly) / det


def eri_lr_semi(fns, omega, gh_order=8, tol=1e-15, n0=32, nmax=1024):
    """(mu nu|erf(w r)/r|kappa lambda) for four Cartesian Gaussians.

    fns: four tuples (center[3], alpha, l[3], norm) -- norm multiplies the
    function.  Returns the integral over R^3 x R^3.
    """
    gh_u, gh_w = roots_hermite(gh_order)
    (cA, aA, lA, nA), (cB, aB, lB, nB), (cC, aC, lC, nC), (cD, aD, lD, nD) = fns

    def integrand(t):
        t2 = t * t
        v = 1.0
        for d in range(3):
            v *= _poly_gauss_2d(t2, (cA[d], aA, lA[d], cB[d], aB, lB[d]),
                                (cC[d], aC, lC[d], cD[d], aD, lD[d]), gh_u, gh_w)
        return v

    prev = None
    m = n0
    while m <= nmax:
        z, zw = roots_legendre(m)
        t = 0.5 * omega * (1.0 + z)
        s = 0.5 * omega * np.sum(zw * np.array([integrand(tt) for tt in t]))
        val = 2.0 / SQRT_PI * s * nA * nB * nC * nD
        if prev is not None and abs(val - prev) <= tol * max(abs(val), 1e-300):
            return val
        prev = val
        m *= 2
    return prev


def basis_function(center, alpha, lxyz, mu):
    """Tuple (center, alpha, l, norm) of unit-normalised function mu."""
    l = [int(v) for v in lxyz[mu]]
    nrm = 1.0
    for d in range(3):
        nrm *= norm_factor(float(alpha[mu]), l[d])
    return (np.asarray(center[mu], dtype=np.float64), float(alpha[mu]), l, nrm)


def eri_lr_bruteforce(fns, omega, m=16):
    """Direct 6D product Gauss-Hermite quadrature of
    g_mu(x) g_nu(x) erf(w|x-y|)/|x-y| g_k(y) g_l(y) over R^3 x R^3."""
    (cA, aA, lA, nA), (cB, aB, lB, nB), (cC, aC, lC, nC), (cD, aD, lD, nD) = fns
    u, wu = roots_hermite(m)
    p = aA + aB
    P = (aA * cA + aB * cB) / p
    Exy = math.exp(-aA * aB / p * np.sum((cA - cB) ** 2))
    q = aC + aD
    Q = (aC * cC + aD * cD) / q
    Ezy = math.exp(-aC * aD / q * np.sum((cC - cD) ** 2))
    sp = 1.0 / math.sqrt(p)
    sq = 1.0 / math.sqrt(q)
    xs = [P[d] + sp * u for d in range(3)]
    ys = [Q[d] + sq * u for d in range(3)]
    px = [((xs[d] - cA[d]) ** lA[d] * (xs[d] - cB[d]) ** lB[d]) for d in range(3)]
    py = [((ys[d] - cC[d]) ** lC[d] * (ys[d] - cD[d]) ** lD[d]) for d in range(3)]
    # x grid (m^3), y grid (m^3)
    X = np.stack(np.meshgrid(*xs, indexing="ij"), -1).reshape(-1, 3)
    Y = np.stack(np.meshgrid(*ys, indexing="ij"), -1).reshape(-1, 3)
    WX = (np.einsum("i,j,k->ijk", wu * px[0], wu * px[1], wu * px[2])).reshape(-1)
    WY = (np.einsum("i,j,k->ijk", wu * py[0], wu * py[1], wu * py[2])).reshape(-1)
    total = 0.0
    for s in range(0, len(X), 256):
        Xs = X[s:s + 256]
        r = np.sqrt(np.sum((Xs[:, None, :] - Y[None, :, :]) ** 2, axis=-1))
        with np.errstate(divide="ignore", invalid="ignore"):
            kern = np.where(r > 1e-300, erf(omega * r) / r, 2.0 * omega / SQRT_PI)
        small = r < 1e-8
        kern[small] = 2.0 * omega / SQRT_PI * (1.0 - (omega * r[small]) ** 2 / 3.0)
        total += WX[s:s + 256] @ (kern @ WY)
    return Exy * Ezy * total * (sp ** 3) * (sq ** 3) * nA * nB * nC * nD
