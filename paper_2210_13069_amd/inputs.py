"""Seeded synthetic inputs for the long-range TEI workloads.

This module only draws random molecules and densities; it holds none of the
method's arithmetic, so the GPU path and the CPU oracle can both consume it.

A molecule is a set of atoms, each carrying shells of primitive Cartesian
Gaussians with one exponent per shell shared by its components.  Component
order per atom: s; px, py, pz; dxx, dxy, dxz, dyy, dyz, dzz.  Draw order:
atom centres, then one exponent per shell (atom-major, s -> p -> d), then
(for densities) the density matrix.  Exponents are log-uniform.
"""
from dataclasses import dataclass, field

import numpy as np

SHELL_COMPONENTS = {
    "s": [(0, 0, 0)],
    "p": [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
    "d": [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)],
}


@dataclass
class Basis:
    """Primitive Cartesian Gaussian basis: nb functions."""
    center: np.ndarray          # (nb, 3) float64, bohr
    alpha: np.ndarray           # (nb,) float64
    lxyz: np.ndarray            # (nb, 3) int32
    atom_of: np.ndarray = field(default=None)  # (nb,) int32

    @property
    def nb(self):
        return int(self.alpha.shape[0])

    @property
    def npair(self):
        return self.nb * (self.nb + 1) // 2


@dataclass
class Params:
    omega: float
    nq: int
    n: int
    L: float
    nodes: int = 0              # 0 = Chebyshev-Lobatto, 1 = Chebyshev-Gauss
    degree_tol: float = 0.0     # > 0: per-node degrees N_k within this tolerance
    rank_tol: float = 0.0       # > 0: low-rank compression of the moments at this tolerance


def random_molecule(rng, natoms, box, shells, alpha_lo, alpha_hi):
    """Atoms uniform in [-box, box]^3; per atom the given shells, one
    log-uniform exponent in [alpha_lo, alpha_hi] per shell."""
    centers = rng.uniform(-box, box, size=(natoms, 3))
    exps = np.exp(rng.uniform(np.log(alpha_lo), np.log(alpha_hi),
                              size=(natoms, len(shells))))
    c, a, l, at = [], [], [], []
    for i in range(natoms):
        for s, sh in enumerate(shells):
            for comp in SHELL_COMPONENTS[sh]:
                c.append(centers[i])
                a.append(exps[i, s])
                l.append(comp)
                at.append(i)
    return Basis(np.array(c, dtype=np.float64), np.array(a, dtype=np.float64),
                 np.array(l, dtype=np.int32), np.array(at, dtype=np.int32))


def random_density(rng, basis, decay=4.0):
    """Symmetric density D(mu,nu) = N(0,1) exp(-|R_mu - R_nu|/decay), drawn
    for mu <= nu in row-major upper-triangle order and mirrored."""
    nb = basis.nb
    mu, nu = np.triu_indices(nb)
    g = rng.standard_normal(len(mu))
    r = np.linalg.norm(basis.center[mu] - basis.center[nu], axis=1)
    D = np.zeros((nb, nb))
    D[mu, nu] = g * np.exp(-r / decay)
    D[nu, mu] = D[mu, nu]
    return D


# ---------------------------------------------------------------------------
# The five workloads.  Seeds: workload c uses seed c; molecule i of the
# batched workload uses seed 4000 + i.
# ---------------------------------------------------------------------------
def tiny_s(seed=1):
    """4 atoms in [-3,3]^3, two s shells each (Nb=8, 36 pairs);
    omega=0.5, nq=16, n=24, L=8."""
    rng = np.random.default_rng(seed)
    b = random_molecule(rng, 4, 3.0, ["s", "s"], 0.2, 20.0)
    return b, Params(omega=0.5, nq=16, n=24, L=8.0)


def sp16(seed=2):
    """16 atoms in [-5,5]^3, s+p shells (Nb=64, 2080 pairs);
    omega=0.5, nq=24, n=32, L=12."""
    rng = np.random.default_rng(seed)
    b = random_molecule(rng, 16, 5.0, ["s", "p"], 0.1, 50.0)
    return b, Params(omega=0.5, nq=24, n=32, L=12.0)


def spd400(seed=3, omega=0.3):
    """40 atoms in [-8,8]^3, s+p+d shells (Nb=400, 80200 pairs);
    omega in {0.3, 1.0}, nq=32, n=40, L=16."""
    rng = np.random.default_rng(seed)
    b = random_molecule(rng, 40, 8.0, ["s", "p", "d"], 0.1, 100.0)
    return b, Params(omega=omega, nq=32, n=40, L=16.0)


def batch64(nmol=64, seed0=4000):
    """Batch of molecules: atoms uniform in {5..30} in [-5,5]^3, s+p shells
    (Nb in [20,120]); omega drawn from {0.3, 0.5, 1.0}; nq=24, n=32, L=12."""
    out = []
    for i in range(nmol):
        rng = np.random.default_rng(seed0 + i)
        natoms = int(rng.integers(5, 31))
        b = random_molecule(rng, natoms, 5.0, ["s", "p"], 0.1, 50.0)
        omega = float(rng.choice([0.3, 0.5, 1.0]))
        out.append((b, Params(omega=omega, nq=24, n=32, L=12.0)))
    return out


def jbuild1000(seed=5):
    """100 atoms in [-12,12]^3, s+p+d shells (Nb=1000, 500500 pairs), with a
    random symmetric density; omega=0.4, nq=32, n=48, L=24."""
    rng = np.random.default_rng(seed)
    b = random_molecule(rng, 100, 12.0, ["s", "p", "d"], 0.1, 100.0)
    D = random_density(rng, b)
    return b, Params(omega=0.4, nq=32, n=48, L=24.0), D


def small_random(seed, natoms=3, shells=("s", "p"), box=2.0, alpha_lo=0.3, alpha_hi=5.0):
    """Small random molecule for property tests."""
    rng = np.random.default_rng(seed)
    return random_molecule(rng, natoms, box, list(shells), alpha_lo, alpha_hi)
