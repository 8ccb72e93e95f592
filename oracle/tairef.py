"""Plain FP64 oracle of the tensorized approximation (TA) of the long-range
two-electron integrals tensor (Badreddine, Chollet, Grigori, arXiv 2210.13069).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's
CPU-baseline leg.  It shares no code with the GPU library.

What the method computes (paper section 3, eqs. kernel/TEI2/chebcheb and
Theorem 3.1 with eq. tensors):

  erf(w r)/r = (2/sqrt(pi)) * int_0^w exp(-s^2 r^2) ds                (eq. kernel)
             ~ (2/sqrt(pi)) * sum_k w_k exp(-t_k^2 r^2)                   (eq. TEI2)

with Gauss-Legendre nodes t_k and weights w_k mapped to [0, omega].  Each 1D
factor exp(-t_k^2 (x-y)^2) on [-L,L]^2 is replaced by its tensor Chebyshev
interpolant (eq. chebcheb).  We keep that interpolant in Lagrange (node-value)
form, which is the same polynomial as the paper's coefficient form:

  exp(-t_k^2 (x-y)^2) ~ sum_{a,b} K_k(a,b) l_a(x) l_b(y),   K_k(a,b) = exp(-t_k^2 (xi_a-xi_b)^2)

The 1D moment of a basis pair against the Lagrange basis (eq. defV, node form)

  m_{p,d}(a) = int_{-L}^{L} g_mu,d(x) g_nu,d(x) l_a(x) dx

gives Theorem 3.1 in node form:

  B(p,q) = (2/sqrt(pi)) sum_k w_k prod_{d=1..3} m_{p,d}^T K_k m_{q,d}

With a degree per quadrature node (the paper's N_i, eq. chebcheb and the
nested coefficient moments of section 3.2) node k keeps only the Chebyshev
coefficients of its factor below N_k; `truncated_tables` gives both that
coefficient form and its node-value form.

Every function below cites the passage it follows.  All arithmetic is FP64.
Notation: nb basis functions, pairs p=(mu,nu) with mu<=nu in row-major upper
triangle order, npair = nb(nb+1)/2; n Chebyshev nodes per direction; nq
quadrature nodes in t.
"""
import math

import numpy as np

SQRT_PI = math.sqrt(math.pi)

NODES_LOBATTO = 0
NODES_GAUSS = 1


# ---------------------------------------------------------------------------
# Quadrature in t (section 3.1, eq. TEI2; Gauss quadrature, Prop. 2.4)
# ---------------------------------------------------------------------------
def gauss_legendre(nq):
    """Gauss-Legendre nodes z_i and weights on [-1, 1] (Prop. 2.4).

    Newton iteration on the Legendre polynomial P_nq, evaluated with the
    three-term recurrence (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}, started from
    the classical estimate cos(pi (i - 1/4) / (nq + 1/2)).  Returned in
    increasing order of z.
    """
    if nq < 1:
        raise ValueError("nq must be >= 1")
    i = np.arange(1, nq + 1, dtype=np.float64)
    x = np.cos(np.pi * (i - 0.25) / (nq + 0.5))
    for _ in range(100):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for j in range(1, nq):
            p0, p1 = p1, ((2 * j + 1) * x * p1 - j * p0) / (j + 1)
        # p1 = P_nq(x), p0 = P_{nq-1}(x)
        dp = nq * (x * p1 - p0) / (x * x - 1.0)
        dx = p1 / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-15:
            break
    # final derivative at the converged nodes for the weights
    p0 = np.ones_like(x)
    p1 = x.copy()
    for j in range(1, nq):
        p0, p1 = p1, ((2 * j + 1) * x * p1 - j * p0) / (j + 1)
    dp = nq * (x * p1 - p0) / (x * x - 1.0)
    wts = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], wts[order]


def time_nodes(omega, nq):
    """Nodes t_k and weights w_k of int_0^omega f(s) ds (eq. TEI2).

    t_k = (omega/2)(1 + z_k), w_k = (omega/2) zw_k.  With these weights the
    paper's prefactor (omega/sqrt(pi)) sum_i zw_i equals (2/sqrt(pi)) sum_k w_k.
    """
    z, zw = gauss_legendre(nq)
    return 0.5 * omega * (1.0 + z), 0.5 * omega * zw


# ---------------------------------------------------------------------------
# Chebyshev nodes and the Lagrange basis (Def. 2.2; Lobatto nodes for TA per
# the remark closing section 4.3)
# ---------------------------------------------------------------------------
def cheb_nodes(n, L, kind=NODES_LOBATTO):
    """Chebyshev nodes xi_a on [-L, L] and their barycentric weights beta_a.

    Lobatto (second kind): xi_a = L cos(pi (a-1)/(n-1)), beta_a = (-1)^(a-1),
    halved at both ends.  Gauss (first kind): xi_a = L cos((2a-1) pi / (2n)),
    beta_a = (-1)^(a-1) sin((2a-1) pi / (2n)).  a = 1..n (Def. 2.2).  The
    barycentric weights are those of Berrut and Trefethen (SIAM Review 2004).
    """
    if n < 2:
        raise ValueError("n must be >= 2")
    a = np.arange(n, dtype=np.float64)
    sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    if kind == NODES_LOBATTO:
        xi = L * np.cos(np.pi * a / (n - 1))
        beta = sign.copy()
        beta[0] *= 0.5
        beta[-1] *= 0.5
    elif kind == NODES_GAUSS:
        theta = (2.0 * a + 1.0) * np.pi / (2.0 * n)
        xi = L * np.cos(theta)
        beta = sign * np.sin(theta)
    else:
        raise ValueError("unknown node kind")
    return xi, beta


def lagrange_basis(xi, beta, x):
    """Values l_a(x) of the Lagrange basis on the nodes xi, shape (len(x), n).

    Barycentric formula of the second kind:
    l_a(x) = (beta_a / (x - xi_a)) / sum_b beta_b / (x - xi_b),
    with l_a(xi_b) = delta_ab taken exactly when x hits a node.
    """
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    diff = x[:, None] - xi[None, :]
    hit = diff == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        terms = beta[None, :] / diff
        ell = terms / np.sum(terms, axis=1, keepdims=True)
    rows = np.any(hit, axis=1)
    if np.any(rows):
        ell[rows] = hit[rows].astype(np.float64)
    return ell


def ktables(t, xi):
    """Node-value interpolation matrices K_k(a,b) = exp(-t_k^2 (xi_a - xi_b)^2).

    These are the values of each 1D factor of eq. TEI2 on the n x n Chebyshev
    grid, i.e. the Lagrange-form counterpart of the coefficient matrices A^(i)
    of eq. chebcheb.  Shape (nq, n, n).
    """
    d2 = (xi[:, None] - xi[None, :]) ** 2
    return np.exp(-(np.asarray(t)[:, None, None] ** 2) * d2[None, :, :])


# ---------------------------------------------------------------------------
# Per-node degree N_i (eq. chebcheb with N_i interpolation points for node i;
# the nested coefficient moments of section 3.2, fast evaluation of tensor
# products: the moments of node i are the leading N_i of those at N = max N_i)
# ---------------------------------------------------------------------------
def cheb_vandermonde(xi, L):
    """V[a, j] = T_j(xi_a / L) for j < n: the Chebyshev polynomials (Def. 2.2)
    of the box variable on the grid, T_j(u) = cos(j arccos u)."""
    u = np.clip(np.asarray(xi, dtype=np.float64) / L, -1.0, 1.0)
    return np.cos(np.outer(np.arccos(u), np.arange(len(u))))


def cheb_coefficients(F, V):
    """Coefficients alpha of the tensor Chebyshev interpolant of node values F
    (n x n), eq. chebcheb: the polynomial sum_ij alpha_ij T_i(x/L) T_j(y/L)
    equal to F at every grid point, i.e. V alpha V^T = F (two linear solves)."""
    X = np.linalg.solve(V, F)            # V X = F, X = alpha V^T
    return np.linalg.solve(V, X.T).T     # V alpha^T = X^T


def tail_sums(alpha):
    """tail[m] = sum of |alpha_ij| over max(i, j) >= m (m = 0..n, tail[n] = 0),
    summed shell by shell from the outside in.  Dropping those coefficients
    moves the polynomial by at most tail[m] anywhere on the box, |T_j| <= 1."""
    a = np.abs(np.asarray(alpha, dtype=np.float64))
    n = a.shape[0]
    tail = np.zeros(n + 1)
    for s in range(n - 1, -1, -1):
        shell = a[s, :s + 1].sum() + a[:s, s].sum()
        tail[s] = tail[s + 1] + shell
    return tail


def node_degrees(alphas, tol):
    """N_k for each node: the smallest m >= 1 with tail(m) <= tol, the reading
    taken here of the paper's adaptive choice of N_i (which it delegates to
    chebfun2).  tol <= 0 keeps every node at n."""
    n = alphas.shape[1]
    if tol <= 0:
        return np.full(alphas.shape[0], n, dtype=np.int64)
    out = []
    for a in alphas:
        tail = tail_sums(a)
        out.append(next(m for m in range(1, n + 1) if tail[m] <= tol))
    return np.asarray(out, dtype=np.int64)


def truncated_tables(t, xi, L, tol):
    """Per-node degree form of the interpolation tables.

    For node k the coefficients alpha_k of its factor exp(-t_k^2 (x-y)^2)
    (eq. chebcheb on the n x n grid) are kept for i, j < N_k and dropped
    elsewhere (alpha_hat_k).  Returns (N, alpha_hat, Kt): N[k], the kept
    coefficients [nq][n][n] and Kt_k = V alpha_hat_k V^T, the node values of
    the truncated polynomial, which every node-form route (Theorem 3.1, the
    grid route of J) takes in place of K_k.  tol <= 0 returns the full tables.
    """
    K = ktables(t, xi)
    V = cheb_vandermonde(xi, L)
    alphas = np.array([cheb_coefficients(Kk, V) for Kk in K])
    N = node_degrees(alphas, tol)
    ahat = np.zeros_like(alphas)
    for k, m in enumerate(N):
        ahat[k, :m, :m] = alphas[k, :m, :m]
    Kt = np.einsum("ai,kij,bj->kab", V, ahat, V) if tol > 0 else K
    return N, ahat, Kt


def coefficient_moments(M, V):
    """mu_d = V^T M_d: the moments against T_j(x/L), j < n (eq. defV in the
    coefficient basis).  Exact counterpart of the Lagrange moments, since
    T_j = sum_a T_j(xi_a) l_a for every j < n."""
    return np.einsum("aj,dap->djp", V, M)


def B_full_degrees(mu, ahat, N, w, rows=None):
    """B by eq. tensors with a degree per node: node k contracts only the
    leading N_k coefficient moments of every pair with the N_k x N_k block of
    its coefficient matrix,
    B = (2/sqrt(pi)) sum_k w_k prod_d mu_d[:N_k]^T alpha_hat_k mu_d[:N_k]."""
    npair = mu.shape[2]
    r = np.arange(npair) if rows is None else np.asarray(rows, dtype=np.int64)
    B = np.zeros((len(r), npair))
    for k in range(len(N)):
        m = int(N[k])
        A = ahat[k, :m, :m]
        F = np.ones((len(r), npair))
        for d in range(3):
            F *= mu[d][:m, r].T @ (A @ mu[d][:m])
        B += w[k] * F
    return (2.0 / SQRT_PI) * B


# ---------------------------------------------------------------------------
# Basis and pairs (eqs. basis, primi; Prop. 2.1; symmetric pairs, section 6.3)
# ---------------------------------------------------------------------------
def _double_factorial_odd(l):
    """(2l-1)!! with (-1)!! = 1."""
    r = 1
    for k in range(2 * l - 1, 0, -2):
        r *= k
    return float(r)


def norm_1d(alpha, l):
    """Constant making one Cartesian factor (x^l exp(-alpha x^2)) unit-norm.

    N = [ (2 alpha/pi)^(1/2) (4 alpha)^l / (2l-1)!! ]^(1/2).  The paper only
    names c_j a normalisation constant (eq. primi); per-factor unit norm is the
    reading taken here.
    """
    return math.sqrt(math.sqrt(2.0 * alpha / math.pi) * (4.0 * alpha) ** l
                     / _double_factorial_odd(l))


def pair_list(nb):
    """(mu, nu) of every pair mu <= nu, row-major upper triangle.

    Pair index p(mu,nu) = mu*nb - mu(mu-1)/2 + (nu - mu) (0-based), which is the
    order of this list.  Pair symmetry g_mu g_nu = g_nu g_mu (section 6.3).
    """
    mu, nu = np.triu_indices(nb)
    return mu.astype(np.int64), nu.astype(np.int64)


def pair_index(nb, mu, nu):
    """Pair index of (mu, nu) with mu <= nu."""
    return mu * nb - (mu * (mu - 1)) // 2 + (nu - mu)


def screened_pairs(center, alpha, tau):
    """Pair indices p(mu, nu), mu <= nu, ascending, that survive screening
    (section 6.3, compression by screening): a pair is dropped when its
    Gaussian product prefactor exp(-ab/(a+b) |A - B|^2) is at most tau.
    tau <= 0 keeps every pair; diagonal pairs (prefactor 1) are always kept
    for tau < 1."""
    center = np.asarray(center, dtype=np.float64).reshape(-1, 3)
    alpha = np.asarray(alpha, dtype=np.float64).reshape(-1)
    mu, nu = pair_list(len(alpha))
    if tau <= 0:
        return np.arange(len(mu), dtype=np.int64)
    a, b = alpha[mu], alpha[nu]
    r2 = np.sum((center[mu] - center[nu]) ** 2, axis=1)
    pref = np.exp(-a * b / (a + b) * r2)
    return np.nonzero(pref > tau)[0].astype(np.int64)


def contraction_pairs(fmap):
    """Contracted basis functions (eq. basis, I_mu primitives each): the
    primitive basis is listed function by function and fmap[i] is the
    contracted function of primitive i (non-decreasing).  For each primitive
    pair p = (i, j), i <= j, returns the contracted pair index P = p(fmap[i],
    fmap[j]) and the weight w_p with which it enters the contracted pair's
    product g_mu g_nu = sum over ordered (i in mu, j in nu) of g_i g_j: 2 for
    i != j within one function (both orders), else 1."""
    fmap = np.asarray(fmap, dtype=np.int64)
    nb = int(fmap[-1]) + 1
    i, j = pair_list(len(fmap))
    P = pair_index(nb, fmap[i], fmap[j])
    w = np.where((fmap[i] == fmap[j]) & (i != j), 2.0, 1.0)
    return P, w


def contract_pairs(Bp, fmap):
    """B over contracted pairs from B over primitive pairs:
    B_c(P, Q) = sum_{p -> P} sum_{q -> Q} w_p w_q Bp(p, q)."""
    P, w = contraction_pairs(fmap)
    nb = int(np.asarray(fmap)[-1]) + 1
    npc = nb * (nb + 1) // 2
    rows = np.zeros((npc, Bp.shape[1]))
    np.add.at(rows, P, w[:, None] * Bp)
    out = np.zeros((npc, npc))
    np.add.at(out.T, P, w[:, None] * rows.T)
    return out


def expand_density(D, fmap):
    """Density over the primitives of a contracted basis: D_prim(i, j) =
    D(fmap[i], fmap[j])."""
    fmap = np.asarray(fmap, dtype=np.int64)
    return np.asarray(D, dtype=np.float64)[np.ix_(fmap, fmap)]


def contract_functions(Jp, fmap):
    """nb x nb matrix over contracted functions from one over primitives:
    J(mu, nu) = sum_{i in mu, j in nu} Jp(i, j)."""
    fmap = np.asarray(fmap, dtype=np.int64)
    nb = int(fmap[-1]) + 1
    F = np.zeros((len(fmap), nb))
    F[np.arange(len(fmap)), fmap] = 1.0
    return F.T @ Jp @ F


def basis_scale(alpha, lxyz, coef):
    """Per-function scale s_mu and per-direction unit-norm factors.

    Returns (c, nd): nd[mu, d] = norm_1d(alpha_mu, l_mu,d) when coef is None;
    otherwise nd = 1 and c = coef (multiplier of the whole 3D function).
    """
    nb = len(alpha)
    if coef is None:
        nd = np.empty((nb, 3))
        for m in range(nb):
            for d in range(3):
                nd[m, d] = norm_1d(alpha[m], int(lxyz[m, d]))
        return np.ones(nb), nd
    return np.asarray(coef, dtype=np.float64), np.ones((nb, 3))


# ---------------------------------------------------------------------------
# 1D moments (eq. defV, with the Lagrange basis in place of T_n)
# ---------------------------------------------------------------------------
def moments(center, alpha, lxyz, L, n, kind=NODES_LOBATTO, coef=None,
            pairs=None, panels=8, order=48, cutoff=9.0):
    """Moments M[d, a, p] = int_{-L}^{L} g_mu,d(x) g_nu,d(x) l_a(x) dx.

    Follows eq. defV: the 1D factor of the pair product, by the Gaussian
    product rule (Prop. 2.1, eq. gauss_prod),
        g_mu,d g_nu,d (x) = N N' (x-A)^l (x-B)^l' E exp(-p (x-P)^2),
        p = a+b, P = (aA+bB)/p, E = exp(-ab/p (A-B)^2),
    is integrated against each Lagrange basis function over the box [-L,L]
    (eq. compact).  The integral is taken by composite Gauss-Legendre
    (`panels` panels of `order` nodes) on [-L,L] intersected with
    [P - cutoff/sqrt(p), P + cutoff/sqrt(p)]; outside it the Gaussian is below
    exp(-cutoff^2) of its peak.  A non-None `coef` multiplies the pair's
    d = 0 factor by coef_mu coef_nu.

    `pairs` optionally restricts to a list of pair indices (columns are then
    in that order).  Returns shape (3, n, npair_selected).
    """
    center = np.asarray(center, dtype=np.float64).reshape(-1, 3)
    alpha = np.asarray(alpha, dtype=np.float64).reshape(-1)
    lxyz = np.asarray(lxyz, dtype=np.int64).reshape(-1, 3)
    nb = len(alpha)
    xi, beta = cheb_nodes(n, L, kind)
    c, nd = basis_scale(alpha, lxyz, coef)
    mu_all, nu_all = pair_list(nb)
    if pairs is None:
        sel = np.arange(len(mu_all))
    else:
        sel = np.asarray(pairs, dtype=np.int64)
    mu = mu_all[sel]
    nu = nu_all[sel]
    z, zw = gauss_legendre(order)
    M = np.zeros((3, n, len(sel)))
    chunk = 512
    for d in range(3):
        for s in range(0, len(sel), chunk):
            m_ = mu[s:s + chunk]
            n_ = nu[s:s + chunk]
            A = center[m_, d]
            B = center[n_, d]
            a = alpha[m_]
            b = alpha[n_]
            la = lxyz[m_, d]
            lb = lxyz[n_, d]
            p = a + b
            P = (a * A + b * B) / p
            E = np.exp(-a * b / p * (A - B) ** 2)
            pref = nd[m_, d] * nd[n_, d] * E
            if d == 0:
                pref = pref * c[m_] * c[n_]
            lo = np.maximum(-L, P - cutoff / np.sqrt(p))
            hi = np.minimum(L, P + cutoff / np.sqrt(p))
            empty = lo >= hi
            hi = np.where(empty, lo, hi)
            h = (hi - lo) / panels
            # quadrature points x[j, i]: pair j, point i
            k = np.arange(panels)
            mid = lo[:, None] + (k[None, :] + 0.5) * h[:, None]
            x = (mid[:, :, None] + 0.5 * h[:, None, None] * z[None, None, :]).reshape(len(m_), -1)
            wq = (0.5 * h[:, None, None] * np.ones((1, panels, 1)) * zw[None, None, :]).reshape(len(m_), -1)
            f = (pref[:, None] * (x - A[:, None]) ** la[:, None] * (x - B[:, None]) ** lb[:, None]
                 * np.exp(-p[:, None] * (x - P[:, None]) ** 2))
            ell = lagrange_basis(xi, beta, x.reshape(-1)).reshape(len(m_), -1, n)
            M[d, :, s:s + chunk] = np.einsum("ji,jia->aj", f * wq, ell)
            M[d, :, s:s + chunk][:, empty] = 0.0
    return M


# ---------------------------------------------------------------------------
# B: Algorithm 1 (entry-wise) and Theorem 3.1 in matrix form
# ---------------------------------------------------------------------------
def B_entries(M, K, w, p_idx, q_idx):
    """Entries B(p,q) by Algorithm 1: loop over quadrature nodes k, form
    F = prod_d m_{p,d}^T K_k m_{q,d} (the Hadamard product of Theorem 3.1 for a
    single pair of pairs), accumulate s += w_k F, return (2/sqrt(pi)) s.

    M has shape (3, n, npair); p_idx/q_idx index its columns.
    """
    p_idx = np.asarray(p_idx, dtype=np.int64).reshape(-1)
    q_idx = np.asarray(q_idx, dtype=np.int64).reshape(-1)
    s = np.zeros(len(p_idx))
    for k in range(K.shape[0]):
        F = np.ones(len(p_idx))
        for d in range(3):
            mp = M[d][:, p_idx]                      # (n, e)
            mq = M[d][:, q_idx]
            F *= np.einsum("ae,ab,be->e", mp, K[k], mq)
        s += w[k] * F
    return (2.0 / SQRT_PI) * s


def B_full(M, K, w, rows=None):
    """B (npair x npair, or the given rows) by Theorem 3.1 in matrix form:
    B = (2/sqrt(pi)) sum_k w_k  (M_1^T K_k M_1) o (M_2^T K_k M_2) o (M_3^T K_k M_3)
    where o is the Hadamard product (eq. Fi with Prop. 2.5)."""
    npair = M.shape[2]
    r = np.arange(npair) if rows is None else np.asarray(rows, dtype=np.int64)
    B = np.zeros((len(r), npair))
    for k in range(K.shape[0]):
        F = np.ones((len(r), npair))
        for d in range(3):
            F *= M[d][:, r].T @ (K[k] @ M[d])
        B += w[k] * F
    return (2.0 / SQRT_PI) * B


def B_kronecker(M, K, w):
    """B by eq. tensors: B = (2/sqrt(pi)) sum_k w_k Mt (K_k (x) K_k (x) K_k) Mt^T,
    Mt(p, a1 a2 a3) = prod_d m_{p,d}(a_d).  Forms the n^3 x n^3 Kronecker
    product explicitly: tiny inputs only."""
    n = M.shape[1]
    npair = M.shape[2]
    Mt = np.einsum("ap,bp,cp->pabc", M[0], M[1], M[2]).reshape(npair, n ** 3)
    B = np.zeros((npair, npair))
    for k in range(K.shape[0]):
        kron = np.kron(np.kron(K[k], K[k]), K[k])
        B += w[k] * (Mt @ kron @ Mt.T)
    return (2.0 / SQRT_PI) * B


# ---------------------------------------------------------------------------
# Low-rank compression of the moments (section 6.1, eqs. SVD and approxepsilon)
# ---------------------------------------------------------------------------
def compression_basis(M, tol):
    """Truncated SVD of the moments (section 6.1, eq. SVD).  The moment
    matrices of the three directions are stacked side by side,
    W = [M_1 | M_2 | M_3] (n x 3 npair), one orthonormal basis V of its leading
    left singular vectors serves the three directions and every quadrature
    node (with one degree n the moments of all nodes coincide).  The rank is
    the number of singular values above the relative cut of section 6.1,
    R = #{r : sigma_r > tol * sigma_1}, and at least 1.

    Returns (V[:, :R], sigma (all n), R)."""
    W = np.concatenate([M[0], M[1], M[2]], axis=1)
    V, sigma, _ = np.linalg.svd(W, full_matrices=False)
    R = max(1, int(np.sum(sigma > tol * sigma[0])))
    return V[:, :R], sigma, R


def compress(M, K, V):
    """The compressed operands of eq. approxepsilon: moments U_d = V^T M_d
    (R x npair per direction) and tables Kc_k = V^T K_k V (R x R per node),
    so that m_p^T K_k m_q becomes u_p^T Kc_k u_q = m_p^T P K_k P m_q with the
    projector P = V V^T."""
    U = np.stack([V.T @ M[d] for d in range(3)])
    Kc = np.stack([V.T @ K[k] @ V for k in range(K.shape[0])])
    return U, Kc


# ---------------------------------------------------------------------------
# Coulomb matrix J (section 5, eqs. Coul and coulapprox, with eq. ig1)
# ---------------------------------------------------------------------------
def density_pairs(D):
    """Pair vector Dt_q = D(k,l) (2 - delta_kl) for q = (k,l), k <= l.

    J(mu,nu) = sum over ALL ordered (k,l) of B(mu nu, k l) D(k,l); with a
    symmetric D the two orders of an off-diagonal pair are folded into one
    pair term.  Only the upper triangle of D is read.
    """
    D = np.asarray(D, dtype=np.float64)
    mu, nu = pair_list(D.shape[0])
    return D[mu, nu] * np.where(mu == nu, 1.0, 2.0)


def unpack_pairs(v, nb):
    """Symmetric nb x nb matrix from a pair vector."""
    mu, nu = pair_list(nb)
    J = np.zeros((nb, nb))
    J[mu, nu] = v
    J[nu, mu] = v
    return J


def J_grid(M, K, w, D):
    """J through the n^3 Chebyshev grid tensor, B never formed.

    Follows eq. coulapprox with the mode-product evaluation of eq. ig1:
      rho(a1,a2,a3) = sum_q Dt_q prod_d m_{q,d}(a_d)          (Dt^T Mt)
      Phi = (2/sqrt(pi)) sum_k w_k rho x_1 K_k x_2 K_k x_3 K_k   ((x) K_k applied)
      J_p = sum_a prod_d m_{p,d}(a_d) Phi(a)                     (Mt Phi)
    and unpacks J_p into the symmetric nb x nb matrix.
    """
    nb = D.shape[0]
    Dt = density_pairs(D)
    rho = np.einsum("q,aq,bq,cq->abc", Dt, M[0], M[1], M[2], optimize=True)
    Phi = np.zeros_like(rho)
    for k in range(K.shape[0]):
        Kk = K[k]
        T = np.einsum("ia,abc->ibc", Kk, rho, optimize=True)
        T = np.einsum("jb,ibc->ijc", Kk, T, optimize=True)
        T = np.einsum("kc,ijc->ijk", Kk, T, optimize=True)
        Phi += w[k] * T
    Phi *= 2.0 / SQRT_PI
    Jp = np.einsum("ap,bp,cp,abc->p", M[0], M[1], M[2], Phi, optimize=True)
    return unpack_pairs(Jp, nb)


def J_grid_pairs(M, K, w, D, pairs):
    """J through the grid with the pair sums restricted to the kept pairs of
    screening (M holds their moments, columns in the order of `pairs`);
    entries of dropped pairs are zero."""
    nb = D.shape[0]
    Dt = density_pairs(D)[pairs]
    rho = np.einsum("q,aq,bq,cq->abc", Dt, M[0], M[1], M[2], optimize=True)
    Phi = np.zeros_like(rho)
    for k in range(K.shape[0]):
        Kk = K[k]
        T = np.einsum("ia,abc->ibc", Kk, rho, optimize=True)
        T = np.einsum("jb,ibc->ijc", Kk, T, optimize=True)
        T = np.einsum("kc,ijc->ijk", Kk, T, optimize=True)
        Phi += w[k] * T
    Phi *= 2.0 / SQRT_PI
    Jp = np.zeros(nb * (nb + 1) // 2)
    Jp[pairs] = np.einsum("ap,bp,cp,abc->p", M[0], M[1], M[2], Phi, optimize=True)
    return unpack_pairs(Jp, nb)


def coulomb_mo(M, K, w, Q):
    """Coulomb matrix in the molecular-orbital basis (section 5, eq. Coul):
    J(i,j) = < q_i q_i^T, B (q_j q_j^T) >, the sum over all ordered
    (mu, nu) and (kappa, lambda) of q_i(mu) q_i(nu) B(mu nu, kappa lambda)
    q_j(kappa) q_j(lambda), for the orbitals Q[i] (rows, length nb).  Each
    B (q_j q_j^T) is the AO Coulomb matrix of the density q_j q_j^T, taken by
    the grid route."""
    Q = np.asarray(Q, dtype=np.float64)
    norb = Q.shape[0]
    Dm = [np.outer(Q[i], Q[i]) for i in range(norb)]
    Jao = [J_grid(M, K, w, Dm[j]) for j in range(norb)]
    return np.array([[np.sum(Dm[i] * Jao[j]) for j in range(norb)] for i in range(norb)])


def pair_index_matrix(nb):
    """P[mu][nu] = index of the unordered pair (min, max) in the pair list."""
    mu, nu = np.meshgrid(np.arange(nb), np.arange(nb), indexing="ij")
    lo, hi = np.minimum(mu, nu), np.maximum(mu, nu)
    return lo * nb - lo * (lo - 1) // 2 + (hi - lo)


def exchange_direct(B, Q):
    """Long-range exchange matrix (appendix B, eq. exchange) written out over
    the pair matrix: K(mu, nu) = 2 sum_j sum_{lambda, kappa} q_j(lambda)
    q_j(kappa) B(mu lambda, kappa nu), with B over ordered index pairs read
    from the unordered pair matrix B (npair x npair)."""
    Q = np.asarray(Q, dtype=np.float64)
    nb = Q.shape[1]
    P = pair_index_matrix(nb)
    B4 = B[P[:, :, None, None], P[None, None, :, :]]     # [mu, lambda, kappa, nu]
    D = Q.T @ Q                                          # sum_j q_j q_j^T
    return 2.0 * np.einsum("mlkn,lk->mn", B4, D)


def exchange_grid(M, K, w, Q):
    """The exchange matrix by the factorized form of appendix B: for orbital
    j and function mu the n^3 tensor X_{j mu} = sum_lambda q_j(lambda)
    prod_d m_{(mu lambda), d} (the product of the orbital's coefficients with
    the moment rows of mu), then K(mu, nu) = 2 sum_j < X_{j mu}, Phi_{j nu} >
    with Phi = (2/sqrt(pi)) sum_k w_k X x_1 K_k x_2 K_k x_3 K_k."""
    Q = np.asarray(Q, dtype=np.float64)
    norb, nb = Q.shape
    P = pair_index_matrix(nb)
    n = M.shape[1]
    X = np.zeros((norb, nb, n, n, n))
    for mu in range(nb):
        cols = P[mu]                                     # pairs (mu, lambda), lambda = 0..nb-1
        X[:, mu] = np.einsum("jl,al,bl,cl->jabc", Q, M[0][:, cols], M[1][:, cols], M[2][:, cols], optimize=True)
    Phi = np.zeros_like(X)
    for k in range(K.shape[0]):
        T = np.einsum("ia,jmabc->jmibc", K[k], X, optimize=True)
        T = np.einsum("jb,xmibc->xmijc", K[k], T, optimize=True)
        T = np.einsum("kc,xmijc->xmijk", K[k], T, optimize=True)
        Phi += w[k] * T
    Phi *= 2.0 / SQRT_PI
    return 2.0 * np.einsum("jmabc,jnabc->mn", X, Phi, optimize=True)


def J_direct_rows(M, K, w, D, rows):
    """J_p = sum_q B(p,q) Dt_q for the given pair rows, with the rows of B
    from Theorem 3.1 (eq. Coul in the atomic-orbital basis)."""
    Dt = density_pairs(D)
    return B_full(M, K, w, rows=rows) @ Dt


# ---------------------------------------------------------------------------
# Adaptive integration boxes (section 6.2): a box [-b_s, b_s] per cluster of
# pairs, with the J of eq. coulapprox summed over the pairs of clusters
# ---------------------------------------------------------------------------
def pair_supports(center, alpha, tau):
    """Half-width b_p of the centred box [-b_p, b_p]^3 that holds the numerical
    support of pair p = (mu, nu), mu <= nu (section 6.2).  By the Gaussian
    product rule the pair's exponential factor in direction d is
    sigma(x) = exp(-p (x - P_d)^2), p = a + b, P = (a A + b B) / p, and
    sigma(x) <= tau exactly when |x - P_d| >= r = sqrt(ln(1/tau) / p); the box
    must reach P_d +- r in every direction, so b_p = max_d |P_d| + r."""
    center = np.asarray(center, dtype=np.float64).reshape(-1, 3)
    alpha = np.asarray(alpha, dtype=np.float64)
    mu, nu = pair_list(len(alpha))
    a, b = alpha[mu], alpha[nu]
    p = a + b
    P = (a[:, None] * center[mu] + b[:, None] * center[nu]) / p[:, None]
    r = np.sqrt(math.log(1.0 / tau) / p)
    return np.max(np.abs(P), axis=1) + r


def adaptive_partitions(supports, nparts):
    """Clusters the pair supports into nparts boxes (section 6.2, which leaves
    the clustering rule open).  Reading: equal-count quantiles of the sorted
    supports.  With v_s the ceil(s npair / nparts)-th smallest support
    (s = 1..nparts), partition s holds the pairs with v_{s-1} < b_p <= v_s
    (v_0 = 0) and its box is [-v_s, v_s]: the smallest of the boxes that holds
    the pair's support.  Equal supports stay together, so a partition can be
    empty.  Returns (part [npair] int64, boxes [nparts])."""
    b = np.asarray(supports, dtype=np.float64)
    npair = len(b)
    srt = np.sort(b)
    ranks = [-(-s * npair // nparts) for s in range(1, nparts + 1)]   # ceil(s npair / nparts)
    boxes = np.array([srt[k - 1] for k in ranks])
    part = np.searchsorted(boxes, b, side="left").astype(np.int64)    # first s with b_p <= v_s
    return part, boxes


def cross_tables(t, xi_out, xi_in):
    """K_k(a, b) = exp(-t_k^2 (xi_out[a] - xi_in[b])^2): node values of the
    tensor Chebyshev interpolant of exp(-t_k^2 (x - y)^2) with x on the grid of
    one box and y on the grid of another (eq. chebcheb on the rectangle
    [-b_s, b_s] x [-b_s', b_s'])."""
    d = xi_out[:, None] - xi_in[None, :]
    return np.exp(-(t[:, None, None] ** 2) * d[None, :, :] ** 2)


def partition_moments(center, alpha, lxyz, part, boxes, n, kind=NODES_LOBATTO, coef=None):
    """Moments of each partition's pairs on the Chebyshev grid of its own box
    (eq. defV with [-b, b] = [-b_s, b_s]): list of (pairs_s ascending,
    M_s [3][n][len(pairs_s)])."""
    out = []
    for s in range(len(boxes)):
        sel = np.flatnonzero(part == s)
        M = moments(center, alpha, lxyz, boxes[s], n, kind=kind, coef=coef, pairs=sel) if len(sel) else \
            np.zeros((3, n, 0))
        out.append((sel, M))
    return out


def J_partitioned(pm, boxes, t, w, n, D, kind=NODES_LOBATTO):
    """J of eq. coulapprox with adaptive boxes (section 6.2).  Every pair p of
    partition s carries its moments on the grid of box s; the interaction of
    pairs in partitions s and s' interpolates exp(-t_k^2 (x - y)^2) on
    [-b_s, b_s] x [-b_s', b_s'], so with rho_s' = sum_{q in s'} Dt_q
    (x)_d m_{q,d} on grid s',
        Phi_s = (2/sqrt(pi)) sum_k w_k sum_s' rho_s' x_1 K_k^(s,s') x_2 K_k^(s,s') x_3 K_k^(s,s'),
        J_p   = < (x)_d m_{p,d}, Phi_s >,   p in s,
    the partition-wise form of the grid route (eq. ig1)."""
    nb = D.shape[0]
    Dt = density_pairs(D)
    grids = [cheb_nodes(n, boxes[s], kind)[0] for s in range(len(boxes))]
    rho = []
    for sel, M in pm:
        rho.append(np.einsum("q,aq,bq,cq->abc", Dt[sel], M[0], M[1], M[2], optimize=True))
    Jp = np.zeros(len(Dt))
    for s, (sel, M) in enumerate(pm):
        if len(sel) == 0:
            continue
        Phi = np.zeros((n, n, n))
        for s2 in range(len(pm)):
            Kx = cross_tables(t, grids[s], grids[s2])
            for k in range(len(t)):
                Kk = Kx[k]
                T = np.einsum("ia,abc->ibc", Kk, rho[s2], optimize=True)
                T = np.einsum("jb,ibc->ijc", Kk, T, optimize=True)
                T = np.einsum("kc,ijc->ijk", Kk, T, optimize=True)
                Phi += w[k] * T
        Phi *= 2.0 / SQRT_PI
        Jp[sel] = np.einsum("ap,bp,cp,abc->p", M[0], M[1], M[2], Phi, optimize=True)
    return unpack_pairs(Jp, nb)


def B_partitioned_entries(pm, boxes, t, w, n, p_idx, q_idx, kind=NODES_LOBATTO):
    """Entries B(p, q) of the adaptive-box approximation by Algorithm 1:
    B(p,q) = (2/sqrt(pi)) sum_k w_k prod_d m_{p,d}^T K_k^(s,s') m_{q,d}, p in
    partition s, q in s' (pair indices into the full list)."""
    where = {}
    for s, (sel, _) in enumerate(pm):
        for i, p in enumerate(sel):
            where[int(p)] = (s, i)
    grids = [cheb_nodes(n, boxes[s], kind)[0] for s in range(len(boxes))]
    out = np.zeros(len(p_idx))
    for e, (p, q) in enumerate(zip(p_idx, q_idx)):
        s, i = where[int(p)]
        s2, i2 = where[int(q)]
        Kx = cross_tables(t, grids[s], grids[s2])
        acc = 0.0
        for k in range(len(t)):
            f = 1.0
            for d in range(3):
                f *= pm[s][1][d][:, i] @ Kx[k] @ pm[s2][1][d][:, i2]
            acc += w[k] * f
        out[e] = (2.0 / SQRT_PI) * acc
    return out


def J_partitioned_rows(pm, boxes, t, w, n, D, rows, kind=NODES_LOBATTO):
    """J_p = sum_q B(p, q) Dt_q for the given pairs p (indices into the full
    list) with adaptive boxes: the direct route, rows of B from Theorem 3.1
    on the pairs' boxes (the same entries as B_partitioned_entries, a pair p
    against every pair of one partition at a time)."""
    Dt = density_pairs(D)
    where = {}
    for s, (sel, _) in enumerate(pm):
        for i, p in enumerate(sel):
            where[int(p)] = (s, i)
    grids = [cheb_nodes(n, boxes[s], kind)[0] for s in range(len(boxes))]
    out = np.zeros(len(rows))
    for e, p in enumerate(rows):
        s, i = where[int(p)]
        acc = 0.0
        for s2, (sel2, M2) in enumerate(pm):
            if len(sel2) == 0:
                continue
            Kx = cross_tables(t, grids[s], grids[s2])
            F = np.zeros(len(sel2))
            for k in range(len(t)):
                f = np.ones(len(sel2))
                for d in range(3):
                    f *= (pm[s][1][d][:, i] @ Kx[k]) @ M2[d]
                F += w[k] * f
            acc += F @ Dt[sel2]
        out[e] = (2.0 / SQRT_PI) * acc
    return out
