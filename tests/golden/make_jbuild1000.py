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

    python tests/golden/make_jbuild1000.py [workers] parts

writes tests/golden/jbuild1000_Jparts.json instead: the same sampled entries
of J with adaptive boxes (section 6.2; supports at tau = 1e-20, four
equal-count quantile boxes), each pair's moments on its own box and the rows
of B from Theorem 3.1 on the two pairs' boxes.
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


PARTS_TAU, PARTS_N = 1e-20, 4


def _chunk_moments(args):
    lo, hi, L, sel = args
    b, P, _ = I.jbuild1000()
    pairs = np.arange(lo, hi) if sel is None else sel[lo:hi]
    return lo, T.moments(b.center, b.alpha, b.lxyz, L, P.n, kind=P.nodes, pairs=pairs)


def _all_moments(pool, L, sel, count):
    step = 4096
    M = np.empty((3, I.jbuild1000()[1].n, count))
    for lo, Mc in pool.imap_unordered(_chunk_moments, [(lo, min(count, lo + step), L, sel)
                                                       for lo in range(0, count, step)]):
        M[:, :, lo:lo + Mc.shape[2]] = Mc
    return M


def main_parts(workers=8):
    b, P, D = I.jbuild1000()
    t0 = time.time()
    sup = T.pair_supports(b.center, b.alpha, PARTS_TAU)
    part, boxes = T.adaptive_partitions(sup, PARTS_N)
    pm = []
    with Pool(workers, initializer=_one_thread) as pool:
        for s in range(PARTS_N):
            sel = np.flatnonzero(part == s)
            pm.append((sel, _all_moments(pool, boxes[s], sel, len(sel)) if len(sel) else np.zeros((3, P.n, 0))))
    print(f"moments of {b.npair} pairs on {PARTS_N} boxes: {time.time() - t0:.1f} s", flush=True)
    t, w = T.time_nodes(P.omega, P.nq)
    pairs = sampled_pairs(b)
    rows = np.array([T.pair_index(b.nb, mu, nu) for mu, nu in pairs], dtype=np.int64)
    t1 = time.time()
    Jp = T.J_partitioned_rows(pm, boxes, t, w, P.n, D, rows, kind=P.nodes)
    print(f"J at {len(rows)} pairs by the direct route: {time.time() - t1:.1f} s", flush=True)
    out = {
        "workload": "jbuild1000 (as jbuild1000_J.json) with adaptive boxes: supports at tau = 1e-20, "
                    "four equal-count quantile boxes",
        "writer": "tests/golden/make_jbuild1000.py parts (oracle only: supports, boxes, moments on each box, "
                  "then J_p = sum_q B(p,q) Dt_q with the rows of B from Theorem 3.1 on the pairs' boxes)",
        "nb": b.nb, "npair": b.npair, "omega": P.omega, "nq": P.nq, "n": P.n,
        "tau": PARTS_TAU, "nparts": PARTS_N, "boxes": boxes.tolist(),
        "counts": np.bincount(part, minlength=PARTS_N).tolist(),
        "pairs": pairs,
        "J": [float(v) for v in Jp],
    }
    with open(os.path.join(HERE, "jbuild1000_Jparts.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("wrote jbuild1000_Jparts.json", len(pairs), "entries")


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
    with Pool(workers, initializer=_one_thread) as pool:
        M = _all_moments(pool, P.L, None, npair)
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
    nw = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    if len(sys.argv) > 2 and sys.argv[2] == "parts":
        main_parts(nw)
    else:
        main(nw)
