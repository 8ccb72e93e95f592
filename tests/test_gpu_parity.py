"""GPU parity: every step of the hot path, called through the C ABI, against
the FP64 oracle on the same seeded inputs.

Tolerances (relative, normwise = max|diff| / max|oracle|):
  nodes, weights, K tables              1e-14  (same FP64 formulas, rounding)
  moments (per (pair, direction) column) 1e-12 of the column's max |m|
  B, FP64 MFMA                           1e-10  (the FP64 target)
  B, FP32 / BF16X6 / F16X3               1e-6   (the low-precision target)
  B, BF16X3                              3e-5   (reported; misses 1e-6 by design)
  J, FP64                                1e-10 relative 2-norm
  J, FP32 / BF16X6                       1e-6 relative 2-norm
  J, BF16X3                              3e-5 (reported)
Element-wise (|diff| / |oracle| over entries with |oracle| >= 1e-8 max|oracle|,
the paper's element-wise measure), F16X3: mean <= 8e-6, and max <= 2e-5 over
entries >= 1e-3 max (smaller entries carry the absolute error of the form as
relative error).  The host emulation of the form gives 5.2e-6 and 1.2e-5 on
the whole Nb = 64 matrix (1.4e-5 and 3.3e-5 without the power of two that
keeps the weighted low slices out of the FP16 subnormals).
"""
import numpy as np
import pytest

from oracle import tairef as T
from paper_2210_13069_amd import inputs as I

pytestmark = pytest.mark.gpu

LOWP_TOL = {1: 1e-6, 2: 3e-5, 3: 1e-6, 4: 1e-6}


def _oracle(basis, P, pairs=None):
    M = T.moments(basis.center, basis.alpha, basis.lxyz, P.L, P.n, kind=P.nodes, pairs=pairs)
    t, w = T.time_nodes(P.omega, P.nq)
    xi, _ = T.cheb_nodes(P.n, P.L, P.nodes)
    return M, T.ktables(t, xi), w


def _normwise(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _check_elementwise_f16x3(got, ref, scale=None):
    scale = np.max(np.abs(ref)) if scale is None else scale
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    big = np.abs(ref) >= 1e-8 * scale
    mean = float(np.mean(rel[big]))
    assert mean <= 8e-6, f"F16X3 mean element-wise {mean:.3e}"
    big3 = np.abs(ref) >= 1e-3 * scale
    if np.any(big3):
        mx = float(np.max(rel[big3]))
        assert mx <= 2e-5, f"F16X3 max element-wise (>= 1e-3 max) {mx:.3e}"


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("nq,n", [(1, 2), (16, 24), (32, 40), (128, 64)])
def test_quadrature_tables(tai, kind, nq, n):
    P = I.Params(omega=0.7, nq=nq, n=n, L=9.0, nodes=kind)
    t, w, xi, K = (x.cpu().numpy() for x in tai.quadrature(P))
    tr, wr = T.time_nodes(P.omega, nq)
    xr, _ = T.cheb_nodes(n, P.L, kind)
    np.testing.assert_allclose(t, tr, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(w, wr, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(xi, xr, rtol=0, atol=1e-14 * P.L)
    np.testing.assert_allclose(K, T.ktables(tr, xr), rtol=1e-13, atol=1e-15)


def _check_moments(Mg, Mr):
    scale = np.max(np.abs(Mr), axis=1, keepdims=True)
    err = np.abs(Mg - Mr)
    bad = err > 1e-12 * scale + 1e-300
    assert not np.any(bad), f"max column-relative error {np.max(err / np.maximum(scale, 1e-300)):.3e}"


@pytest.mark.parametrize("case", ["tiny_s", "sp16", "spd_small", "gauss_nodes", "edge"])
def test_moments(tai, case):
    coef = None
    if case == "tiny_s":
        b, P = I.tiny_s()
    elif case == "sp16":
        b, P = I.sp16()
    elif case == "spd_small":
        b = I.small_random(21, natoms=5, shells=("s", "p", "d"), box=3.0, alpha_lo=0.1, alpha_hi=100.0)
        P = I.Params(omega=0.4, nq=12, n=48, L=6.0)
    elif case == "gauss_nodes":
        b = I.small_random(22, natoms=3, shells=("s", "p"), box=2.0)
        P = I.Params(omega=0.5, nq=8, n=33, L=7.0, nodes=1)
    else:
        # centres outside the box, a pair straddling the edge, coef given
        b = I.small_random(23, natoms=3, shells=("s", "p", "d"), box=5.0, alpha_lo=0.05, alpha_hi=2.0)
        P = I.Params(omega=0.5, nq=8, n=20, L=4.0)
        coef = np.linspace(0.3, 1.7, b.nb)
    Mg = tai.moments(b, P, coef=coef).cpu().numpy()
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, kind=P.nodes, coef=coef)
    _check_moments(Mg, Mr)


def test_moments_full_size_sampled(tai):
    # 500500 pairs, n = 48: sampled columns against the oracle
    b, P, _ = I.jbuild1000()
    Mg = tai.moments(b, P)
    rng = np.random.default_rng(0)
    sel = np.concatenate([[0, b.npair - 1], rng.choice(b.npair, 400, replace=False)])
    Mr = T.moments(b.center, b.alpha, b.lxyz, P.L, P.n, pairs=sel)
    _check_moments(Mg[:, :, sel].cpu().numpy(), Mr)


@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("case", ["tiny_s", "sp16"])
def test_assemble_B_small(tai, prec, case):
    b, P = I.tiny_s() if case == "tiny_s" else I.sp16()
    Mr, K, w = _oracle(b, P)
    Br = T.B_full(Mr, K, w)
    Mg = tai.moments(b, P)
    Bg = tai.assemble_B(Mg, P, prec=prec).cpu().numpy().astype(np.float64)
    tol = 1e-10 if prec == 0 else LOWP_TOL[prec]
    err = _normwise(Bg, Br)
    assert err <= tol, f"prec {prec}: normwise {err:.3e} > {tol}"
    # every entry written, both triangles
    assert np.all(np.isfinite(Bg))
    if prec == 4:
        _check_elementwise_f16x3(Bg, Br)
    # mirrored tiles are exact copies; diagonal tiles are symmetric to the
    # arithmetic's own accuracy
    assert _normwise(Bg, Bg.T) <= (1e-14 if prec == 0 else tol)


@pytest.mark.parametrize("n", [5, 12, 16, 29, 40, 41, 56])
def test_assemble_fp64_fp32_inner_lengths(tai, n):
    """FP64 and FP32 at inner lengths 8 .. 56 (n rounded up to 8) of the
    persistent ring kernels, whose row blocks per wave change with the inner
    length, on a ragged pair count (npair = 465, not a multiple of any panel)."""
    b = I.small_random(51, natoms=3, shells=("s", "p", "d"), box=2.0, alpha_lo=0.2, alpha_hi=8.0)
    P = I.Params(omega=0.5, nq=6, n=n, L=7.0)
    Mr, K, w = _oracle(b, P)
    Br = T.B_full(Mr, K, w)
    Mg = tai.moments(b, P)
    for prec in (0, 1):
        Bg = tai.assemble_B(Mg, P, prec=prec).cpu().numpy().astype(np.float64)
        tol = 1e-10 if prec == 0 else LOWP_TOL[prec]
        assert _normwise(Bg, Br) <= tol, (n, prec, _normwise(Bg, Br))
        assert _normwise(Bg, Bg.T) <= (1e-14 if prec == 0 else tol)


@pytest.mark.parametrize("n", [24, 40])
@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5, 6, 7, 8, 9, 17, 18, 33])
def test_assemble_16bit_node_counts(tai, nq, n):
    """Split 16-bit forms at node counts around the LDS ring depth (too few
    nodes take the generic kernel), around the two-node steps (odd counts
    and counts below twice the ring depth fall back to single-node shapes;
    n = 40 has two-node shapes, n = 24 none) and around the FP32 group of
    sixteen nodes, with column blocks ending anywhere within a group of steps."""
    b = I.small_random(41, natoms=6, shells=("s", "p"), box=3.0)   # nb = 24, npair = 300
    P = I.Params(omega=0.6, nq=nq, n=n, L=8.0)
    Mr, K, w = _oracle(b, P)
    Br = T.B_full(Mr, K, w)
    Mg = tai.moments(b, P)
    for prec in (4, 2):
        Bg = tai.assemble_B(Mg, P, prec=prec).cpu().numpy().astype(np.float64)
        assert _normwise(Bg, Br) <= LOWP_TOL[prec], (nq, n, prec)
        assert np.array_equal(Bg, Bg.T) or _normwise(Bg, Bg.T) <= LOWP_TOL[prec]


def test_assemble_ldb_and_ragged_tail(tai):
    import torch
    b = I.small_random(31, natoms=4, shells=("s", "p"), box=2.5)   # nb = 16, npair = 136 (ragged)
    P = I.Params(omega=0.5, nq=10, n=20, L=8.0)
    Mg = tai.moments(b, P)
    npair = b.npair
    for prec, dt in [(0, torch.float64), (4, torch.float32)]:
        ldb = npair + 13
        out = torch.full((npair, ldb), 7.0, dtype=dt, device=Mg.device)
        tai.assemble_B(Mg, P, prec=prec, ldb=ldb, out=out)
        o = out.cpu().numpy()
        assert np.all(o[:, npair:] == 7.0), "columns beyond npair were written"
        Mr, K, w = _oracle(b, P)
        Br = T.B_full(Mr, K, w)
        assert _normwise(o[:, :npair].astype(np.float64), Br) <= (1e-10 if prec == 0 else 1e-6)


def test_assemble_matches_stored_tiny_s(tai):
    """The tiny 36-pair workload against the stored oracle matrix
    (tests/golden/tiny_s.json), every precision form."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_s.json")))
    ref = np.array(g["B_ta"])
    b, P = I.tiny_s()
    Mg = tai.moments(b, P)
    for prec in (0, 1, 2, 3, 4):
        Bg = tai.assemble_B(Mg, P, prec=prec).cpu().numpy().astype(np.float64)
        assert Bg.shape == ref.shape
        assert _normwise(Bg, ref) <= (1e-10 if prec == 0 else LOWP_TOL[prec]), prec


@pytest.mark.parametrize("case", ["sp16", "spd_small", "spd_small_odd"])
def test_assemble_shapes_agree_bitwise(tai, case):
    """Every compiled 16-bit kernel shape (forced through TAI_ASM16_SHAPE)
    gives the same bits, so the autotuner's choice never changes results."""
    import os
    if case == "sp16":
        b, P = I.sp16()                                   # n = 32: kc 96
    else:
        # n = 40: kc 128; an odd node count leaves out the two-node-step
        # shapes (the host falls back to the first shape that fits)
        b = I.small_random(45, natoms=8, shells=("s", "p", "d"), box=3.0)
        P = I.Params(omega=0.4, nq=7 if case == "spd_small_odd" else 8, n=40, L=8.0)
    Mg = tai.moments(b, P)
    old = os.environ.get("TAI_ASM16_SHAPE")
    try:
        outs = []
        for pick in range(8):
            os.environ["TAI_ASM16_SHAPE"] = str(pick)
            outs.append(tai.assemble_B(Mg, P, prec=4).cpu().numpy())
    finally:
        if old is None:
            os.environ.pop("TAI_ASM16_SHAPE", None)
        else:
            os.environ["TAI_ASM16_SHAPE"] = old
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_autotune_keeps_results(tai):
    """A tuned call (first call of its signature) and later calls agree
    bitwise with the table default shape."""
    import torch
    b, P = I.sp16()
    ctx = tai.Context(0)
    Mg = tai.moments(b, P)
    params = tai.make_params(P, tai.F16X3)
    outs = []
    for mode in (0, 1, 1):
        ctx.tune(mode)
        B = torch.empty((b.npair, b.npair), dtype=torch.float32, device=Mg.device)
        ctx.assemble_B(Mg, b.npair, params, B)
        outs.append(B.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


def test_assemble_deterministic(tai):
    b, P = I.sp16()
    Mg = tai.moments(b, P)
    for prec in (0, 4):
        B1 = tai.assemble_B(Mg, P, prec=prec).cpu().numpy()
        B2 = tai.assemble_B(Mg, P, prec=prec).cpu().numpy()
        assert np.array_equal(B1, B2)


@pytest.mark.parametrize("omega", [0.3, 1.0])
def test_assemble_B_full_size_sampled(tai, omega):
    """Nb = 400 (80200 pairs, 6.43e9 entries) in the bench's launch
    configuration; sampled entries against Algorithm 1 of the oracle."""
    import torch
    b, P = I.spd400(omega=omega)
    Mg = tai.moments(b, P)
    rng = np.random.default_rng(7)
    p = np.concatenate([rng.integers(0, b.npair, 300), [0, b.npair - 1, b.npair - 1]])
    q = np.concatenate([rng.integers(0, b.npair, 300), [b.npair - 1, 0, b.npair - 1]])
    sel = np.unique(np.concatenate([p, q]))
    Mr, K, w = _oracle(b, P, pairs=sel)
    ref = T.B_entries(Mr, K, w, np.searchsorted(sel, p), np.searchsorted(sel, q))
    diag = T.B_entries(Mr, K, w, np.arange(len(sel)), np.arange(len(sel)))
    scale = np.max(np.abs(diag))
    pt = torch.as_tensor(p, device=Mg.device)
    qt = torch.as_tensor(q, device=Mg.device)
    for prec in (4, 0):
        B = tai.assemble_B(Mg, P, prec=prec, ldb=tai.aligned_ldb(b.npair))
        got = B[pt, qt].cpu().numpy().astype(np.float64)
        tol = 1e-10 if prec == 0 else 1e-6
        err = np.max(np.abs(got - ref)) / scale
        assert err <= tol, f"prec {prec}: {err:.3e}"
        if prec == 4:
            _check_elementwise_f16x3(got, ref, scale)
        del B
        torch.cuda.empty_cache()


J_TOL = {0: 1e-10, 1: 1e-6, 3: 1e-6, 2: 3e-5}


@pytest.mark.parametrize("prec", [0, 1, 3, 2])
@pytest.mark.parametrize("case", ["tiny_s", "sp16", "spd_small", "spd_n64", "sp_n40_gauss"])
def test_apply_J(tai, case, prec):
    import torch
    if case == "tiny_s":
        b, P = I.tiny_s()
    elif case == "sp16":
        b, P = I.sp16()
    elif case == "spd_small":
        b = I.small_random(41, natoms=6, shells=("s", "p", "d"), box=3.0)
        P = I.Params(omega=0.4, nq=12, n=48, L=8.0)
    elif case == "spd_n64":
        b = I.small_random(43, natoms=5, shells=("s", "p", "d"), box=3.0)
        P = I.Params(omega=0.4, nq=6, n=64, L=8.0)
    else:
        # n = 40: the split forms pad their inner length (6 n = 240 -> 256)
        b = I.small_random(44, natoms=7, shells=("s", "p"), box=4.0)
        P = I.Params(omega=0.6, nq=10, n=40, L=9.0, nodes=1)
    D = I.random_density(np.random.default_rng(3), b)
    Mr, K, w = _oracle(b, P)
    Jr = T.J_grid(Mr, K, w, D)
    Mg = tai.moments(b, P)
    Jg = tai.apply_J(Mg, torch.as_tensor(D, device=Mg.device), P, prec=prec).cpu().numpy()
    err = np.linalg.norm(Jg - Jr, 2) / np.linalg.norm(Jr, 2)
    # FP64 target 1e-10; FP32 and BF16X6 1e-6; BF16X3 keeps 16 bits (reported)
    assert err <= J_TOL[prec], err
    np.testing.assert_array_equal(Jg, Jg.T)


def test_apply_J_equals_B_times_density(tai):
    import torch
    b, P = I.sp16()
    D = I.random_density(np.random.default_rng(9), b)
    Mg = tai.moments(b, P)
    Dg = torch.as_tensor(D, device=Mg.device)
    Jg = tai.apply_J(Mg, Dg, P)
    Bg = tai.assemble_B(Mg, P, prec=0)
    mu, nu = T.pair_list(b.nb)
    Dt = torch.as_tensor(T.density_pairs(D), device=Mg.device)
    Jp = (Bg @ Dt).cpu().numpy()
    ref = T.unpack_pairs(Jp, b.nb)
    assert np.max(np.abs(Jg.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("prec", [4, 0, 1])
def test_batched_equals_per_molecule(tai, graph, prec):
    """Direct launches (default stream) and hipGraph replays (a side stream):
    every replay, with eager work and synchronization in between, equals the
    per-molecule calls bit for bit (split 16-bit persistent kernel; FP64 and
    FP32 tile queue)."""
    import torch
    mols = I.batch64(nmol=6)
    ctx = tai.context(0)
    outs, Ms, keep = [], [], []
    structs = []
    dt = torch.float64 if prec == tai.FP64 else torch.float32
    for b, P in mols:
        ba = tai.BasisArrays(b)
        keep.append(ba)
        M = torch.empty((3, P.n, b.npair), dtype=torch.float64, device="cuda")
        B = torch.full((b.npair, b.npair), float("nan"), dtype=dt, device="cuda")
        Ms.append(M)
        outs.append(B)
        structs.append(tai.tai_mol(ba.struct, tai.make_params(P, prec), M.data_ptr(), B.data_ptr(), b.npair))
    stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()
    for rep in range(3):
        for B in outs:
            B.fill_(float("nan"))
        torch.cuda.synchronize()
        ctx.assemble_B_batched(structs, stream=stream)
        torch.cuda.synchronize()
        for (b, P), M, B in zip(mols, Ms, outs):
            Mref = tai.moments(b, P)
            assert torch.equal(M, Mref)
            Bref = tai.assemble_B(Mref, P, prec=prec)
            assert torch.equal(B, Bref), f"replay {rep}"


@pytest.mark.parametrize("case", ["one_function", "n2_nq1", "n64_nq128", "gauss_nodes_d"])
def test_assemble_and_J_edge_cases(tai, case):
    """Degenerate and extreme sizes for every arithmetic: a single basis
    function (one pair), the smallest degree and node count, the largest
    degree with the largest node count (BF16X6 then exceeds the persistent
    kernel's inner length and takes the generic kernel), and Gauss-Chebyshev
    nodes with d functions; J in FP64 and FP32 for the same inputs."""
    import torch
    rng = np.random.default_rng(77)
    if case == "one_function":
        b = I.random_molecule(rng, 1, 1.0, ["s"], 0.5, 2.0)
        P = I.Params(omega=0.5, nq=8, n=16, L=6.0)
    elif case == "n2_nq1":
        b = I.small_random(51, natoms=2, shells=("s",), box=1.0)
        P = I.Params(omega=0.3, nq=1, n=2, L=4.0)
    elif case == "n64_nq128":
        b = I.small_random(52, natoms=2, shells=("s", "p"), box=2.0)
        P = I.Params(omega=1.0, nq=128, n=64, L=6.0)
    else:
        b = I.small_random(53, natoms=3, shells=("s", "d"), box=2.0)
        P = I.Params(omega=0.5, nq=10, n=30, L=7.0, nodes=1)
    Mr, K, w = _oracle(b, P)
    Br = T.B_full(Mr, K, w)
    Mg = tai.moments(b, P)
    for prec in (0, 1, 2, 3, 4):
        Bg = tai.assemble_B(Mg, P, prec=prec).cpu().numpy().astype(np.float64)
        assert Bg.shape == (b.npair, b.npair)
        tol = 1e-10 if prec == 0 else LOWP_TOL[prec]
        assert _normwise(Bg, Br) <= tol, (case, prec, _normwise(Bg, Br))
    D = I.random_density(np.random.default_rng(4), b)
    Jr = T.J_grid(Mr, K, w, D)
    for prec, tol in ((0, 1e-10), (1, 1e-6)):
        Jg = tai.apply_J(Mg, torch.as_tensor(D, device=Mg.device), P, prec=prec).cpu().numpy()
        err = np.linalg.norm(Jg - Jr) / np.linalg.norm(Jr)
        assert err <= tol, (case, prec, err)


@pytest.mark.parametrize("n", [24, 32, 40, 48, 56])
def test_bf16x6_layouts_and_shapes(tai, n):
    """BF16X6 at every operand layout: segment-major (n = 24) and the
    duplicated-chunk layout with and without index tails (32, 40, 48, 56:
    inner lengths 192, 256, 288, 352); every compiled shape of the inner
    length gives the same bits and matches the oracle; odd node counts take
    the three-deep rings."""
    import os
    b = I.small_random(47, natoms=5, shells=("s", "p", "d"), box=3.0, alpha_lo=0.2, alpha_hi=10.0)
    for nq in (7, 8):
        P = I.Params(omega=0.5, nq=nq, n=n, L=8.0)
        Mr, K, w = _oracle(b, P)
        Br = T.B_full(Mr, K, w)
        Mg = tai.moments(b, P)
        old = os.environ.get("TAI_ASM16_SHAPE")
        try:
            outs = []
            for pick in range(4):
                os.environ["TAI_ASM16_SHAPE"] = str(pick)
                outs.append(tai.assemble_B(Mg, P, prec=3).cpu().numpy())
        finally:
            if old is None:
                os.environ.pop("TAI_ASM16_SHAPE", None)
            else:
                os.environ["TAI_ASM16_SHAPE"] = old
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])
        assert _normwise(outs[0].astype(np.float64), Br) <= LOWP_TOL[3], (n, nq, _normwise(outs[0], Br))


@pytest.mark.parametrize("n", [12, 40, 64])
def test_ring_and_tile_kernels_agree(tai, n):
    """FP64 and FP32: the persistent ring kernels and the tile kernels
    (TAI_TILE_ASSEMBLY) compute the same B to their arithmetic's accuracy."""
    import os
    b = I.small_random(48, natoms=4, shells=("s", "p", "d"), box=2.5, alpha_lo=0.2, alpha_hi=8.0)
    P = I.Params(omega=0.5, nq=5, n=n, L=7.0)
    Mg = tai.moments(b, P)
    for prec in (0, 1):
        ring = tai.assemble_B(Mg, P, prec=prec).cpu().numpy().astype(np.float64)
        old = os.environ.get("TAI_TILE_ASSEMBLY")
        os.environ["TAI_TILE_ASSEMBLY"] = "1"
        try:
            tile = tai.assemble_B(Mg, P, prec=prec).cpu().numpy().astype(np.float64)
        finally:
            if old is None:
                os.environ.pop("TAI_TILE_ASSEMBLY", None)
            else:
                os.environ["TAI_TILE_ASSEMBLY"] = old
        assert _normwise(ring, tile) <= (1e-13 if prec == 0 else 1e-6), (n, prec)


def test_binding_rejects_a_wrong_output_buffer(tai):
    """The binding checks the output buffer before the call: an FP32 buffer
    for the FP64 arithmetic (half the bytes B needs), or one too short, is
    refused with ValueError and no kernel runs."""
    import torch
    b, P = I.sp16()
    ctx = tai.Context(0)
    Mg = tai.moments(b, P)
    small = torch.empty((b.npair, b.npair), dtype=torch.float32, device=Mg.device)
    with pytest.raises(ValueError):
        ctx.assemble_B(Mg, b.npair, tai.make_params(P, tai.FP64), small)
    short = torch.empty((b.npair - 1, b.npair), dtype=torch.float32, device=Mg.device)
    with pytest.raises(ValueError):
        ctx.assemble_B(Mg, b.npair, tai.make_params(P, tai.F16X3), short)
