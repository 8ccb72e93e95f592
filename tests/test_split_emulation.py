"""The split 16-bit arithmetics, emulated on the host from their definition,
reach the accuracy the library is held to, independently of the GPU code.

Definition (the readings of the split): each operand column (one pair, one
direction) is scaled by a power of two that brings its largest magnitude into
[0.5, 1); the scaled value x is cut into round-to-nearest slices
s0 = r(fl32(x)), s1 = r(fl32(x - s0)), s2 = r(fl32(x - s0 - s1)) with r the
FP16 or BF16 rounding; the products of slices are exact in FP32; the slice
products kept per direction are (0,0), (0,1), (1,0) for the X3 forms and also
(0,2), (1,1), (2,0) for BF16X6; per node the direction results are rounded to
FP32, multiplied (Hadamard) and summed over groups of sixteen nodes in FP32,
and the groups in FP64.  Against the FP64 tensorized approximation on the
same inputs the normwise error must be <= 1e-6 for F16X3 and BF16X6; BF16X3
lands near 1e-5 (it is reported, and held to 3e-5).  Without the per-column
power-of-two scaling, FP16 slices underflow on the small moments: the
element-wise error on the small entries grows, which is why the scaling is
part of the form.  The quadrature weight w_k goes into the direction-2
operand of each node together with a power of two that brings the largest
weight near [8, 16): w_k alone (1e-3 .. 3e-2) pushes the low FP16 slices into
the subnormals, which costs F16X3 several times its element-wise accuracy.
"""
import math

import numpy as np

from oracle import tairef as T
from paper_2210_13069_amd import inputs as I


def _bf16(x32):
    """Round float32 values to bfloat16 (round to nearest even), as float32."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _round(x64, kind):
    x32 = x64.astype(np.float32)
    return x32.astype(np.float16).astype(np.float64) if kind == "f16" else _bf16(x32).astype(np.float64)


def _slices(x, kind, ns):
    out, rem = [], x.copy()
    for _ in range(ns):
        s = _round(rem, kind)
        out.append(s)
        rem = rem - s
    return out


PAIRS = {"x3": [(0, 0), (0, 1), (1, 0)], "x6": [(0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0)]}


def _weight_shift(w):
    """Exponent s with max_k w_k 2^s in [8, 16)."""
    return 3 - (math.frexp(float(np.max(w)))[1] - 1)


def _emulate(M, K, w, rows, kind, form, scale=True, wshift=True):
    """B[rows, :] in the emulated split arithmetic."""
    n, npair = M.shape[1], M.shape[2]
    sh = _weight_shift(w) if wshift else 0
    ns = 3 if form == "x6" else 2
    ex = np.zeros((3, npair))
    if scale:
        for d in range(3):
            mx = np.max(np.abs(M[d]), axis=0)
            ex[d] = np.where(mx > 0, np.frexp(np.where(mx > 0, mx, 1.0))[1], 0)
    A = [_slices(M[d][:, rows] * 2.0 ** -ex[d][rows], kind, ns) for d in range(3)]
    acc32 = np.zeros((len(rows), npair), dtype=np.float32)
    acc64 = np.zeros((len(rows), npair))
    for k in range(len(w)):
        G = []
        for d in range(3):
            Y = (K[k] @ M[d]) * 2.0 ** -ex[d]
            if d == 2:
                Y = Y * (w[k] * 2.0 ** sh)
            Ys = _slices(Y, kind, ns)
            g = sum(A[d][i].T @ Ys[j] for i, j in PAIRS[form])
            G.append(g.astype(np.float32))
        acc32 = acc32 + (G[0] * G[1]) * G[2]
        if (k + 1) % 16 == 0 or k + 1 == len(w):
            acc64 += acc32.astype(np.float64)
            acc32[:] = 0
    e = ex[0] + ex[1] + ex[2]
    return acc64 * (2.0 / np.sqrt(np.pi)) * 2.0 ** (e[rows][:, None] + e[None, :] - sh)


def _setup():
    b, P = I.sp16()
    M = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, kind=P.nodes)
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L, P.nodes)
    K = T.ktables(t, xi)
    rows = np.arange(0, M.shape[2], 7)
    ref = T.B_full(M, K, w, rows=rows)
    return M, K, w, rows, ref


def _normwise(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def test_split_forms_meet_the_precision_target():
    M, K, w, rows, ref = _setup()
    err = {name: _normwise(_emulate(M, K, w, rows, kind, form), ref)
           for name, kind, form in [("f16x3", "f16", "x3"), ("bf16x3", "bf16", "x3"), ("bf16x6", "bf16", "x6")]}
    print("emulated normwise error vs FP64:", {k: f"{v:.2e}" for k, v in err.items()})
    assert err["f16x3"] <= 1e-6
    assert err["bf16x6"] <= 1e-6
    assert err["bf16x3"] <= 3e-5
    # the slices are genuinely 16-bit: none of the forms is exact
    assert min(err.values()) > 1e-12


def test_f16_slices_need_the_power_of_two_scaling():
    """Normwise the scaling changes nothing here (the entries it protects are
    small), but element-wise, over entries with |B| >= 1e-8 max|B| (the
    paper's element-wise measure), unscaled FP16 slices lose the small
    moments to underflow: the mean relative error grows by more than 10x."""
    M, K, w, rows, ref = _setup()
    big = np.abs(ref) >= 1e-8 * np.max(np.abs(ref))
    mean_rel = {}
    for scale in (True, False):
        B = _emulate(M, K, w, rows, "f16", "x3", scale=scale)
        mean_rel[scale] = float(np.mean(np.abs(B - ref)[big] / np.abs(ref[big])))
        assert _normwise(B, ref) <= 1e-6
    print(f"f16x3 mean element-wise error: scaled {mean_rel[True]:.2e}, unscaled {mean_rel[False]:.2e}")
    assert mean_rel[True] * 10 < mean_rel[False]


def _mean_rel(B, ref):
    big = np.abs(ref) >= 1e-8 * np.max(np.abs(ref))
    return float(np.mean(np.abs(B - ref)[big] / np.abs(ref[big])))


def test_f16_weight_shift_keeps_the_low_slices_normal():
    """With w_k folded in unshifted, the low FP16 slices of the direction-2
    operand are subnormal and the mean element-wise error is several times
    that of the shifted form; the shifted form stays within 2e-6 mean, with
    the normwise bar met either way.  BF16 has FP32's exponent range: the
    shift changes its results only where FP32 products underflow."""
    M, K, w, rows, ref = _setup()
    B1 = _emulate(M, K, w, rows, "f16", "x3", wshift=True)
    B0 = _emulate(M, K, w, rows, "f16", "x3", wshift=False)
    m1, m0 = _mean_rel(B1, ref), _mean_rel(B0, ref)
    print(f"f16x3 mean element-wise error: weight shift {m1:.2e}, none {m0:.2e}")
    assert _normwise(B1, ref) <= 1e-6 and _normwise(B0, ref) <= 1e-6
    assert m1 <= 2e-6
    assert 3 * m1 < m0
    Bb1 = _emulate(M, K, w, rows, "bf16", "x3", wshift=True)
    Bb0 = _emulate(M, K, w, rows, "bf16", "x3", wshift=False)
    assert _normwise(Bb1, Bb0) <= 1e-12
    assert abs(_mean_rel(Bb1, ref) - _mean_rel(Bb0, ref)) <= 0.05 * _mean_rel(Bb0, ref)
