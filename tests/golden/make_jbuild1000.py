"""Write tests/golden/jbuild1000_J.json: the oracle's Coulomb matrix entries on
the Nb = 1000 J workload at sampled pairs (calls only oracle/).

    python tests/golden/make_jbuild1000.py [workers]

Workload: 100 atoms in [-12,12]^3, s+p+d shells (Nb = 1000, 500 500 pairs),
exponents log-uniform in [0.1, 100], the random symmetric density
D = N(0,1) exp(-|R_mu - R_nu| / 4), seed 5; omega = 0.4, nq = 32, n = 48,
L = 24, Chebyshev-Lobatto nodes.

J at a pair p = (mu, nu) is J_p = sum_q B(p, q) Dt_q (eq. Coul in the atomic-
orbital basis, the ordered sum folded onto pairs), with the rows B(p, :) from
Theorem 3.1 over all 500 500 pairs: the direct route, which shares no step
with the grid route the library takes.  The moments of every pair are needed,
so they are computed in parallel chunks by the oracle's own moment function
(about two minutes on eight cores).

Sampled pairs: 24 diagonal pairs (mu, mu), 24 pairs of two functions on one
atom, 16 pairs drawn uniformly from all pairs (rng seed 11).
"""
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import tairef as T  # noqa: E402
from paper_2210_13069_amd import inputs as I  # noqa: E402


def _one_thread():
    # the moment workers run side by side: one BLAS thread each
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _chunk_moments(args):
    lo, hi = args
    b, P, _ = I.jbuild1000()
    return lo, T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, kind=P.nodes, pairs=np.arange(lo, hi))


def sampled_pairs(b):
    rng = np.random.default_rng(11)
    nb = b.nb
    diag_mu = rng.choice(nb, 24, replace=False)
    same = []
    while len(same) < 24:
        mu, nu = sorted(rng.integers(0, nb, 2))
        if mu != nu and b.atom_of[mu] == b.atom_of[nu] and (mu, nu) not in same:
            same.append((int(mu), int(nu)))
    rand = []
    while len(rand) < 16:
        mu, nu = sorted(rng.integers(0, nb, 2))
        if (mu, nu) not in rand:
            rand.append((int(mu), int(nu)))
    pairs = [(int(m), int(m)) for m in diag_mu] + same + rand
    return pairs


def main(workers=8):
    b, P, D = I.jbuild1000()
    npair = b.npair
    t0 = time.time()
    step = 4096
    chunks = [(lo, min(npair, lo + step)) for lo in range(0, npair, step)]
    M = np.empty((3, P.n, npair))
    with Pool(workers, initializer=_one_thread) as pool:
        for lo, Mc in pool.imap_unordered(_chunk_moments, chunks):
            M[:, :, lo:lo + Mc.shape[2]] = Mc
    print(f"moments of {npair} pairs: {time.time() - t0:.1f} s", flush=True)
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L, P.nodes)
    K = T.ktables(t, xi)
    pairs = sampled_pairs(b)
    rows = np.array([T.pair_index(b.nb, mu, nu) for mu, nu in pairs], dtype=np.int64)
    t1 = time.time()
    Jp = T.J_direct_rows(M, K, w, D, rows)
    print(f"J at {len(rows)} pairs by the direct route: {time.time() - t1:.1f} s", flush=True)
    out = {
        "workload": "jbuild1000: 100 atoms in [-12,12]^3, s+p+d shells (Nb=1000, 500500 pairs), "
                    "exponents log-uniform in [0.1,100], density N(0,1) exp(-|R_mu-R_nu|/4), seed 5; "
                    "omega=0.4, nq=32, n=48, L=24, Chebyshev-Lobatto nodes",
        "writer": "tests/golden/make_jbuild1000.py (oracle only: moments, then J_p = sum_q B(p,q) Dt_q "
                  "with the rows of B from Theorem 3.1)",
        "nb": b.nb, "npair": npair, "omega": P.omega, "nq": P.nq, "n": P.n, "L": P.L,
        "pairs": pairs,
        "J": [float(v) for v in Jp],
    }
    with open(os.path.join(HERE, "jbuild1000_J.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("wrote jbuild1000_J.json", len(pairs), "entries")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
