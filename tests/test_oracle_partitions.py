"""Pins of the oracle's adaptive integration boxes (section 6.2): the pair
supports against the cut they are defined by, the clustering against a plain
loop, one partition against the plain method, the partition-wise grid route
against Algorithm 1 written out over partition pairs, and convergence to the
closed-form s-type integrals (while a fixed box that cuts supports stays off
by its truncation, as the paper's table of J errors shows for b = 10)."""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


def test_support_is_where_the_factor_reaches_the_cut():
    """b_p - |P_d| is the distance at which exp(-p (x - P_d)^2) falls to tau
    (found here by bisection on the factor itself) for the direction of the
    largest |P_d|, and the factor is below tau at +-b_p in every direction."""
    b = I.small_random(11, natoms=5, shells=("s", "p"), box=4.0, alpha_lo=0.1, alpha_hi=50.0)
    tau = 1e-12
    sup = T.pair_supports(b.center, b.alpha, tau)
    mu, nu = T.pair_list(b.nb)
    for i in range(0, b.npair, 7):
        a, c = b.alpha[mu[i]], b.alpha[nu[i]]
        p = a + c
        P = (a * b.center[mu[i]] + c * b.center[nu[i]]) / p
        lo, hi = 0.0, 100.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if math.exp(-p * mid * mid) > tau:
                lo = mid
            else:
                hi = mid
        dmax = int(np.argmax(np.abs(P)))
        assert abs((sup[i] - abs(P[dmax])) - lo) <= 1e-12 * lo
        for d in range(3):
            for x in (sup[i], -sup[i]):
                assert math.exp(-p * (x - P[d]) ** 2) <= tau * (1 + 1e-9)


def test_partitions_against_a_plain_loop():
    b = I.small_random(12, natoms=9, shells=("s", "p"), box=5.0, alpha_lo=0.1, alpha_hi=50.0)
    sup = T.pair_supports(b.center, b.alpha, 1e-20)
    for nparts in (1, 2, 3, 5):
        part, boxes = T.adaptive_partitions(sup, nparts)
        srt = sorted(sup.tolist())
        ref_boxes = []
        for s in range(1, nparts + 1):
            k = (s * len(srt) + nparts - 1) // nparts
            ref_boxes.append(srt[k - 1])
        assert boxes.tolist() == ref_boxes
        for i, v in enumerate(sup):
            s = 0
            while ref_boxes[s] < v:
                s += 1
            assert part[i] == s
        # every support inside its box, and no smaller box would hold it
        assert np.all(sup <= boxes[part])
        assert np.all((part == 0) | (sup > boxes[np.maximum(part - 1, 0)]))
        # equal-count quantiles: no partition above ceil(npair / nparts) + ties
        assert np.bincount(part, minlength=nparts).sum() == b.npair


def test_one_partition_is_the_plain_method():
    b = I.small_random(13, natoms=4, shells=("s", "p", "d"), box=3.0, alpha_lo=0.2, alpha_hi=20.0)
    n, omega, nq = 16, 0.5, 10
    sup = T.pair_supports(b.center, b.alpha, 1e-16)
    part, boxes = T.adaptive_partitions(sup, 1)
    assert boxes[0] == np.max(sup) and np.all(part == 0)
    t, w = T.time_nodes(omega, nq)
    D = I.random_density(np.random.default_rng(2), b)
    pm = T.partition_moments(b.center, b.alpha, b.lxyz, part, boxes, n)
    J = T.J_partitioned(pm, boxes, t, w, n, D)
    M = T.moments(b.center, b.alpha, b.lxyz, boxes[0], n)
    xi, _ = T.cheb_nodes(n, boxes[0])
    Jp = T.J_grid(M, T.ktables(t, xi), w, D)
    assert np.max(np.abs(J - Jp)) <= 1e-13 * np.max(np.abs(Jp))


def test_grid_route_equals_algorithm_1_over_partition_pairs():
    """J from the partition-wise grid tensors equals sum_q B(p, q) Dt_q with
    every entry from Algorithm 1 on the two pairs' boxes."""
    b = I.small_random(14, natoms=3, shells=("s", "p"), box=3.0, alpha_lo=0.2, alpha_hi=20.0)
    n, omega, nq = 10, 0.6, 6
    sup = T.pair_supports(b.center, b.alpha, 1e-14)
    part, boxes = T.adaptive_partitions(sup, 3)
    assert len(set(part.tolist())) == 3
    t, w = T.time_nodes(omega, nq)
    D = I.random_density(np.random.default_rng(3), b)
    pm = T.partition_moments(b.center, b.alpha, b.lxyz, part, boxes, n)
    J = T.J_partitioned(pm, boxes, t, w, n, D)
    npair = b.npair
    P, Q = np.meshgrid(np.arange(npair), np.arange(npair), indexing="ij")
    B = T.B_partitioned_entries(pm, boxes, t, w, n, P.ravel(), Q.ravel()).reshape(npair, npair)
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    ref = T.unpack_pairs(B @ T.density_pairs(D), b.nb)
    assert np.max(np.abs(J - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the row form of the direct route (the full-size fixture's writer)
    rows = np.arange(0, npair, 3)
    mu, nu = T.pair_list(b.nb)
    jr = T.J_partitioned_rows(pm, boxes, t, w, n, D, rows)
    assert np.max(np.abs(jr - ref[mu[rows], nu[rows]])) <= 1e-12 * np.max(np.abs(ref))


def test_converges_to_the_closed_form_and_fixed_boxes_truncate():
    """s-type functions: with partitions the J of eq. coulapprox reaches the
    exact long-range J (Boys F0) at n = 64, nq = 32; a single fixed box at the
    median support cuts the larger pairs and stays about 1e-3 off."""
    b = I.small_random(7, natoms=5, shells=("s", "s"), box=3.0, alpha_lo=0.3, alpha_hi=30.0)
    omega = 0.5
    D = I.random_density(np.random.default_rng(1), b)
    Bx = X.B_closed_form_s(b.center, b.alpha, omega)
    Jx = T.unpack_pairs(Bx @ T.density_pairs(D), b.nb)
    sup = T.pair_supports(b.center, b.alpha, 1e-30)
    n, nq = 64, 32
    t, w = T.time_nodes(omega, nq)
    part, boxes = T.adaptive_partitions(sup, 3)
    pm = T.partition_moments(b.center, b.alpha, b.lxyz, part, boxes, n)
    J = T.J_partitioned(pm, boxes, t, w, n, D)
    assert np.linalg.norm(J - Jx, 2) <= 1e-12 * np.linalg.norm(Jx, 2)
    L = float(np.median(sup))
    pm1 = T.partition_moments(b.center, b.alpha, b.lxyz, np.zeros(b.npair, dtype=np.int64), np.array([L]), n)
    J1 = T.J_partitioned(pm1, np.array([L]), t, w, n, D)
    assert np.linalg.norm(J1 - Jx, 2) >= 1e-4 * np.linalg.norm(Jx, 2)
