"""tai_apply_J_noalloc, the J entry point that allocates nothing (its
intermediates live in the library's static device scratch), through the C
ABI against tai_apply_J on the same inputs: equal bit for bit, on two calls in
a row with the second on a smaller basis (the scratch keeps the first call's
contents), in FP64 and FP32, with a degree per node, and sizes beyond the
scratch rejected before any device work."""
import ctypes

import numpy as np
import pytest

from paper_2210_13069_amd import inputs as I

pytestmark = pytest.mark.gpu


def _j_pair(tai, ctx, b, P, prec, seed):
    import torch
    Mg = tai.moments(b, P)
    D = torch.as_tensor(I.random_density(np.random.default_rng(seed), b), device=Mg.device)
    params = tai.make_params(P, prec)
    Jref = torch.empty((b.nb, b.nb), dtype=torch.float64, device=Mg.device)
    ctx.apply_J(Mg, b.nb, params, D, Jref)
    J = torch.full((b.nb, b.nb), float("nan"), dtype=torch.float64, device=Mg.device)
    ctx.check(ctx.lib.tai_apply_J_noalloc(ctx.h, tai._ptr(Mg), int(b.nb), ctypes.byref(params), tai._ptr(D),
                                          tai._ptr(J), tai._stream(None)), "tai_apply_J_noalloc")
    torch.cuda.synchronize()
    return J, Jref


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_apply_J_twice_shrinking(tai, prec):
    import torch
    ctx = tai.context(0)
    big = (I.small_random(61, natoms=8, shells=("s", "p", "d"), box=4.0, alpha_lo=0.1, alpha_hi=40.0),
           I.Params(omega=0.4, nq=16, n=40, L=10.0))
    small = (I.small_random(62, natoms=3, shells=("s", "p"), box=2.0), I.Params(omega=0.5, nq=8, n=24, L=7.0))
    for (b, P), seed in ((big, 1), (small, 2)):
        J, Jref = _j_pair(tai, ctx, b, P, prec, seed)
        assert bool(torch.all(torch.isfinite(J)))
        assert torch.equal(J, Jref), float((J - Jref).abs().max())


def test_noalloc_per_node_degrees_and_full_size(tai):
    """With a degree per node, and at the Nb = 1000 workload (207 MiB of
    scratch in FP64), after a small call."""
    import torch
    ctx = tai.context(0)
    b, P = I.sp16()
    P = I.Params(omega=P.omega, nq=P.nq, n=P.n, L=P.L, degree_tol=1e-8)
    J, Jref = _j_pair(tai, ctx, b, P, 0, 3)
    assert torch.equal(J, Jref)
    jb, jP, _ = I.jbuild1000()
    J, Jref = _j_pair(tai, ctx, jb, jP, 0, 4)
    assert torch.equal(J, Jref)
    del J, Jref
    torch.cuda.empty_cache()


def test_noalloc_rejects_what_does_not_fit(tai):
    """Sizes beyond the static scratch and the compression are refused on the
    host with nothing written."""
    import torch
    ctx = tai.context(0)
    jb, jP, _ = I.jbuild1000()
    dev = torch.device("cuda", 0)
    M = torch.zeros(1, dtype=torch.float64, device=dev)    # never read: the call fails first
    J = torch.zeros((4, 4), dtype=torch.float64, device=dev)
    p32 = tai.make_params(jP, tai.FP32)   # FP32 adds its FP32 copy of the moments: 494 MiB
    r = ctx.lib.tai_apply_J_noalloc(ctx.h, tai._ptr(M), int(jb.nb), ctypes.byref(p32), tai._ptr(J), tai._ptr(J),
                                    tai._stream(None))
    assert r == tai.TAI_ERR_INVALID_ARG
    assert b"scratch" in ctx.lib.tai_last_error(ctx.h)
    pc = tai.make_params(I.Params(omega=0.5, nq=8, n=24, L=7.0, rank_tol=1e-6), tai.FP64)
    r = ctx.lib.tai_apply_J_noalloc(ctx.h, tai._ptr(M), 4, ctypes.byref(pc), tai._ptr(J), tai._ptr(J),
                                    tai._stream(None))
    assert r == tai.TAI_ERR_UNSUPPORTED
    assert bool(torch.all(J == 0))
