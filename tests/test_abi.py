"""The C-ABI library loads, exports every entry point of include/tai.h, and
validates arguments before any device work (host-only context, no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2210_13069_amd import tai
from paper_2210_13069_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "tai.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tai_[a-zA-Z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tai.LIB_PATH):
        pytest.fail("libtai.so is not built; run `python -m paper_2210_13069_amd.build`")
    return tai.load_library()


@pytest.fixture()
def hctx(lib):
    c = tai.Context(device=-1)
    yield c
    c.close()


def test_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert set(declared) == set(tai.SYMBOLS), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_tune_modes(lib, hctx):
    for mode in (0, 1, 2):
        assert lib.tai_tune(hctx.h, mode) == tai.TAI_OK
    for mode in (-1, 3):
        assert lib.tai_tune(hctx.h, mode) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_tune(None, 1) == tai.TAI_ERR_INVALID_ARG


def test_peak_probe_argument_checks(lib, hctx):
    v = ctypes.c_double()
    assert lib.tai_peak_probe(None, 0, ctypes.byref(v), None) == tai.TAI_ERR_INVALID_ARG
    for what in (-1, 3):
        assert lib.tai_peak_probe(hctx.h, what, ctypes.byref(v), None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_peak_probe(hctx.h, 0, None, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_peak_probe(hctx.h, 0, ctypes.byref(v), None) == tai.TAI_ERR_NOT_READY


def test_status_strings(lib):
    for st in (0, -1, -2, -3, -4, -5, 7):
        s = lib.tai_status_string(st)
        assert s is not None and len(s) > 0


def test_null_context_rejected(lib):
    p = tai.tai_params(0.5, 8, 8, 4.0, 0, 0, 0.0)
    assert lib.tai_quadrature(None, ctypes.byref(p), None, None, None, None, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_sync(None, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_destroy(None) == tai.TAI_OK
    assert lib.tai_last_error(None) == b""
    assert lib.tai_create(None, 0) == tai.TAI_ERR_INVALID_ARG


def _params(**kw):
    base = dict(omega=0.5, nq=8, n=16, L=8.0, nodes=0, prec=0, degree_tol=0.0, rank_tol=0.0)
    base.update(kw)
    return tai.tai_params(base["omega"], base["nq"], base["n"], base["L"], base["nodes"], base["prec"],
                          base["degree_tol"], base["rank_tol"])


@pytest.mark.parametrize("bad", [dict(omega=0.0), dict(omega=-1.0), dict(omega=float("nan")),
                                 dict(omega=float("inf")), dict(nq=0), dict(nq=129), dict(n=1),
                                 dict(n=65), dict(L=0.0), dict(L=float("nan")), dict(nodes=2),
                                 dict(prec=5), dict(prec=-1), dict(degree_tol=-1e-9),
                                 dict(degree_tol=float("nan")), dict(degree_tol=float("inf")),
                                 dict(rank_tol=-1e-9), dict(rank_tol=1.0), dict(rank_tol=float("nan")),
                                 dict(rank_tol=float("inf"))])
def test_invalid_params(hctx, bad):
    p = _params(**bad)
    st = hctx.lib.tai_quadrature(hctx.h, ctypes.byref(p), None, None, None, None, None)
    assert st == tai.TAI_ERR_INVALID_ARG
    assert len(hctx.lib.tai_last_error(hctx.h)) > 0


def test_valid_params_host_only_not_ready(hctx):
    p = _params()
    assert hctx.lib.tai_quadrature(hctx.h, ctypes.byref(p), None, None, None, None, None) == tai.TAI_ERR_NOT_READY
    p = _params(degree_tol=1e-8)
    assert hctx.lib.tai_quadrature(hctx.h, ctypes.byref(p), None, None, None, None, None) == tai.TAI_ERR_NOT_READY


def test_degrees_argument_checks(hctx):
    dummy = ctypes.c_void_p(16)
    p = _params(degree_tol=1e-8)
    assert hctx.lib.tai_degrees(hctx.h, ctypes.byref(p), None, None, None) == tai.TAI_ERR_INVALID_ARG
    assert hctx.lib.tai_degrees(hctx.h, None, dummy, None, None) == tai.TAI_ERR_INVALID_ARG
    bad = _params(degree_tol=-1.0)
    assert hctx.lib.tai_degrees(hctx.h, ctypes.byref(bad), dummy, None, None) == tai.TAI_ERR_INVALID_ARG
    assert hctx.lib.tai_degrees(hctx.h, ctypes.byref(p), dummy, None, None) == tai.TAI_ERR_NOT_READY
    assert hctx.lib.tai_degrees(hctx.h, ctypes.byref(p), None, dummy, None) == tai.TAI_ERR_NOT_READY


def test_compress_argument_checks(hctx):
    dummy = ctypes.c_void_p(16)
    rank = ctypes.c_int32(-7)
    p = _params(rank_tol=1e-6)
    lib, h = hctx.lib, hctx.h
    assert lib.tai_compress(h, None, 10, ctypes.byref(p), ctypes.byref(rank), None, None, None, None, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_compress(h, dummy, 10, ctypes.byref(p), None, None, None, None, None, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_compress(h, dummy, 0, ctypes.byref(p), ctypes.byref(rank), None, None, None, None, None) == tai.TAI_ERR_INVALID_ARG
    off = _params()
    assert lib.tai_compress(h, dummy, 10, ctypes.byref(off), ctypes.byref(rank), None, None, None, None, None) == tai.TAI_ERR_INVALID_ARG
    # compression together with per-node degrees is accepted
    both = _params(rank_tol=1e-6, degree_tol=1e-8)
    assert lib.tai_compress(h, dummy, 10, ctypes.byref(both), ctypes.byref(rank), None, None, None, None, None) == tai.TAI_ERR_NOT_READY
    assert lib.tai_assemble_B(h, dummy, 10, ctypes.byref(both), dummy, 10, None) == tai.TAI_ERR_NOT_READY
    assert lib.tai_compress(h, dummy, 10, ctypes.byref(p), ctypes.byref(rank), None, None, None, None, None) == tai.TAI_ERR_NOT_READY
    assert rank.value == -7
    assert lib.tai_assemble_B(h, dummy, 10, ctypes.byref(p), dummy, 10, None) == tai.TAI_ERR_NOT_READY


def test_apply_J_compressed_argument_checks(hctx):
    dummy = ctypes.c_void_p(16)
    lib, h = hctx.lib, hctx.h
    p = _params()
    call = lambda U=dummy, nb=4, pairs=None, npk=0, R=8, Kc=dummy, params=p, D=dummy, J=dummy: \
        lib.tai_apply_J_compressed(h, U, nb, pairs, npk, R, Kc, ctypes.byref(params), D, J, None)
    assert call(U=None) == tai.TAI_ERR_INVALID_ARG
    assert call(Kc=None) == tai.TAI_ERR_INVALID_ARG
    assert call(nb=0) == tai.TAI_ERR_INVALID_ARG
    assert call(R=0) == tai.TAI_ERR_INVALID_ARG
    assert call(R=1) == tai.TAI_ERR_NOT_READY               # rank 1 is valid (padded to 8)
    assert call(R=17) == tai.TAI_ERR_INVALID_ARG           # n = 16
    assert call(pairs=dummy, npk=0) == tai.TAI_ERR_INVALID_ARG
    assert call(params=_params(prec=4)) == tai.TAI_ERR_UNSUPPORTED
    assert call() == tai.TAI_ERR_NOT_READY
    assert call(pairs=dummy, npk=5) == tai.TAI_ERR_NOT_READY


def _basis(**mut):
    b, _ = I.tiny_s()
    center = b.center.copy()
    alpha = b.alpha.copy()
    lxyz = b.lxyz.copy()
    if "alpha" in mut:
        alpha[2] = mut["alpha"]
    if "center" in mut:
        center[1, 2] = mut["center"]
    if "l" in mut:
        lxyz[0, 1] = mut["l"]
    return I.Basis(center, alpha, lxyz)


@pytest.mark.parametrize("mut", [dict(alpha=0.0), dict(alpha=-2.0), dict(alpha=float("nan")),
                                 dict(center=float("inf")), dict(l=-1), dict(l=5)])
def test_invalid_basis(hctx, mut):
    ba = tai.BasisArrays(_basis(**mut))
    p = _params()
    dummy = ctypes.c_void_p(16)
    st = hctx.lib.tai_moments(hctx.h, ctypes.byref(ba.struct), ctypes.byref(p), dummy, None)
    assert st == tai.TAI_ERR_INVALID_ARG


def test_invalid_coef_and_nb(hctx):
    b = _basis()
    coef = np.ones(b.nb)
    coef[3] = np.nan
    ba = tai.BasisArrays(b, coef)
    p = _params()
    dummy = ctypes.c_void_p(16)
    assert hctx.lib.tai_moments(hctx.h, ctypes.byref(ba.struct), ctypes.byref(p), dummy, None) == tai.TAI_ERR_INVALID_ARG
    ba = tai.BasisArrays(b)
    ba.struct.nb = 0
    assert hctx.lib.tai_moments(hctx.h, ctypes.byref(ba.struct), ctypes.byref(p), dummy, None) == tai.TAI_ERR_INVALID_ARG
    ba.struct.nb = 70000  # npair > 2^31 - 1
    assert hctx.lib.tai_moments(hctx.h, ctypes.byref(ba.struct), ctypes.byref(p), dummy, None) == tai.TAI_ERR_INVALID_ARG
    ba = tai.BasisArrays(b)
    assert hctx.lib.tai_moments(hctx.h, ctypes.byref(ba.struct), ctypes.byref(p), None, None) == tai.TAI_ERR_INVALID_ARG
    assert hctx.lib.tai_moments(hctx.h, ctypes.byref(ba.struct), ctypes.byref(p), dummy, None) == tai.TAI_ERR_NOT_READY


def test_assemble_argument_checks(hctx):
    p = _params()
    d = ctypes.c_void_p(16)
    L = hctx.lib
    assert L.tai_assemble_B(hctx.h, None, 36, ctypes.byref(p), d, 36, None) == tai.TAI_ERR_INVALID_ARG
    assert L.tai_assemble_B(hctx.h, d, 36, ctypes.byref(p), None, 36, None) == tai.TAI_ERR_INVALID_ARG
    assert L.tai_assemble_B(hctx.h, d, 0, ctypes.byref(p), d, 36, None) == tai.TAI_ERR_INVALID_ARG
    assert L.tai_assemble_B(hctx.h, d, 36, ctypes.byref(p), d, 35, None) == tai.TAI_ERR_INVALID_ARG
    assert L.tai_assemble_B(hctx.h, d, 36, ctypes.byref(_params(n=1)), d, 36, None) == tai.TAI_ERR_INVALID_ARG
    assert L.tai_assemble_B(hctx.h, d, 36, ctypes.byref(p), d, 36, None) == tai.TAI_ERR_NOT_READY


def test_apply_j_argument_checks(hctx):
    d = ctypes.c_void_p(16)
    L = hctx.lib
    p = _params()
    assert L.tai_apply_J(hctx.h, d, 0, ctypes.byref(p), d, d, None) == tai.TAI_ERR_INVALID_ARG
    assert L.tai_apply_J(hctx.h, d, 8, ctypes.byref(p), None, d, None) == tai.TAI_ERR_INVALID_ARG
    assert L.tai_apply_J(hctx.h, d, 8, ctypes.byref(_params(prec=4)), d, d, None) == tai.TAI_ERR_UNSUPPORTED
    for prec in (2, 3):    # the split-BF16 forms of J are valid
        assert L.tai_apply_J(hctx.h, d, 8, ctypes.byref(_params(prec=prec)), d, d, None) == tai.TAI_ERR_NOT_READY
    assert L.tai_apply_J(hctx.h, d, 8, ctypes.byref(p), d, d, None) == tai.TAI_ERR_NOT_READY


def test_batched_argument_checks(hctx):
    b1 = tai.BasisArrays(_basis())
    mk = lambda nq, ldb: tai.tai_mol(b1.struct, _params(nq=nq), 16, 16, ldb)
    L = hctx.lib
    arr = (tai.tai_mol * 2)(mk(8, 36), mk(9, 36))
    assert L.tai_assemble_B_batched(hctx.h, 2, arr, None) == tai.TAI_ERR_INVALID_ARG  # nq differs
    arr = (tai.tai_mol * 2)(mk(8, 36), mk(8, 10))
    assert L.tai_assemble_B_batched(hctx.h, 2, arr, None) == tai.TAI_ERR_INVALID_ARG  # ldb < npair
    assert L.tai_assemble_B_batched(hctx.h, 0, arr, None) == tai.TAI_ERR_INVALID_ARG
    arr = (tai.tai_mol * 2)(mk(8, 36), mk(8, 36))
    assert L.tai_assemble_B_batched(hctx.h, 2, arr, None) == tai.TAI_ERR_NOT_READY


def test_device_context_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert lib.tai_create(ctypes.byref(h), 0) == tai.TAI_ERR_HIP
    assert not h.value


def test_screening_argument_checks(hctx):
    lib, h = hctx.lib, hctx.h
    ba = tai.BasisArrays(_basis())
    dummy = ctypes.c_void_p(16)
    cnt = ctypes.c_int32(-7)
    for tau in (float("nan"), float("inf"), 1.0, 2.0):
        assert lib.tai_screen_pairs(h, ctypes.byref(ba.struct), tau, dummy, ctypes.byref(cnt), None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_screen_pairs(h, ctypes.byref(ba.struct), 1e-8, None, ctypes.byref(cnt), None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_screen_pairs(h, ctypes.byref(ba.struct), 1e-8, dummy, None, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_screen_pairs(h, ctypes.byref(ba.struct), 1e-8, dummy, ctypes.byref(cnt), None) == tai.TAI_ERR_NOT_READY
    assert cnt.value == -7  # nothing written on a host-only context
    p = _params()
    npair = ba.alpha.shape[0] * (ba.alpha.shape[0] + 1) // 2
    for npk in (0, -1, npair + 1):
        assert lib.tai_moments_pairs(h, ctypes.byref(ba.struct), ctypes.byref(p), dummy, npk, dummy, None) == tai.TAI_ERR_INVALID_ARG
        assert lib.tai_apply_J_pairs(h, dummy, ba.alpha.shape[0], dummy, npk, ctypes.byref(p), dummy, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_moments_pairs(h, ctypes.byref(ba.struct), ctypes.byref(p), None, 3, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_apply_J_pairs(h, dummy, ba.alpha.shape[0], None, 3, ctypes.byref(p), dummy, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_moments_pairs(h, ctypes.byref(ba.struct), ctypes.byref(p), dummy, npair, dummy, None) == tai.TAI_ERR_NOT_READY
    assert lib.tai_apply_J_pairs(h, dummy, ba.alpha.shape[0], dummy, 3, ctypes.byref(p), dummy, dummy, None) == tai.TAI_ERR_NOT_READY


def test_coulomb_mo_argument_checks(hctx):
    lib, h = hctx.lib, hctx.h
    dummy = ctypes.c_void_p(16)
    p = _params()
    assert lib.tai_coulomb_mo(h, None, 8, None, 0, ctypes.byref(p), dummy, 2, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_coulomb_mo(h, dummy, 8, None, 0, ctypes.byref(p), None, 2, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_coulomb_mo(h, dummy, 8, None, 0, ctypes.byref(p), dummy, 2, None, None) == tai.TAI_ERR_INVALID_ARG
    for norb in (0, -3, 1025):
        assert lib.tai_coulomb_mo(h, dummy, 8, None, 0, ctypes.byref(p), dummy, norb, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_coulomb_mo(h, dummy, 0, None, 0, ctypes.byref(p), dummy, 2, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_coulomb_mo(h, dummy, 8, dummy, 0, ctypes.byref(p), dummy, 2, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_coulomb_mo(h, dummy, 8, dummy, 37, ctypes.byref(p), dummy, 2, dummy, None) == tai.TAI_ERR_INVALID_ARG
    p16 = _params(prec=4)
    assert lib.tai_coulomb_mo(h, dummy, 8, None, 0, ctypes.byref(p16), dummy, 2, dummy, None) == tai.TAI_ERR_UNSUPPORTED
    assert lib.tai_coulomb_mo(h, dummy, 8, None, 0, ctypes.byref(p), dummy, 2, dummy, None) == tai.TAI_ERR_NOT_READY
    assert lib.tai_coulomb_mo(h, dummy, 8, dummy, 36, ctypes.byref(p), dummy, 2, dummy, None) == tai.TAI_ERR_NOT_READY


def test_contraction_argument_checks(hctx):
    lib, h = hctx.lib, hctx.h
    dummy = ctypes.c_void_p(16)
    i32p = ctypes.POINTER(ctypes.c_int32)

    def fm(lst):
        return (ctypes.c_int32 * len(lst))(*lst)

    good = fm([0, 0, 1, 2, 2])      # nb = 3 from 5 primitives: npair 6 from 15
    for bad in ([1, 1, 2, 3, 3], [0, 2, 2, 3, 3], [0, 1, 0, 1, 2]):
        assert lib.tai_contract_pairs(h, dummy, 15, 5, fm(bad), 0, dummy, 6, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_contract_pairs(h, dummy, 15, 5, None, 0, dummy, 6, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_contract_pairs(h, dummy, 14, 5, good, 0, dummy, 6, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_contract_pairs(h, dummy, 15, 5, good, 0, dummy, 5, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_contract_pairs(h, None, 15, 5, good, 0, dummy, 6, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_contract_pairs(h, dummy, 15, 5, good, 9, dummy, 6, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_contract_pairs(h, dummy, 15, 5, good, 0, dummy, 6, None) == tai.TAI_ERR_NOT_READY
    p = _params()
    assert lib.tai_apply_J_contracted(h, dummy, 5, fm([0, 1, 1, 3, 3]), ctypes.byref(p), dummy, dummy, None) == tai.TAI_ERR_INVALID_ARG
    assert lib.tai_apply_J_contracted(h, None, 5, good, ctypes.byref(p), dummy, dummy, None) == tai.TAI_ERR_INVALID_ARG
    p16 = _params(prec=4)
    assert lib.tai_apply_J_contracted(h, dummy, 5, good, ctypes.byref(p16), dummy, dummy, None) == tai.TAI_ERR_UNSUPPORTED
    assert lib.tai_apply_J_contracted(h, dummy, 5, good, ctypes.byref(p), dummy, dummy, None) == tai.TAI_ERR_NOT_READY


def test_exchange_argument_checks(hctx):
    dummy = ctypes.c_void_p(16)
    lib, h = hctx.lib, hctx.h
    p = _params()
    call = lambda M=dummy, nb=4, pairs=None, npk=0, params=p, Q=dummy, norb=2, Kx=dummy: \
        lib.tai_exchange(h, M, nb, pairs, npk, ctypes.byref(params), Q, norb, Kx, None)
    assert call(M=None) == tai.TAI_ERR_INVALID_ARG
    assert call(Q=None) == tai.TAI_ERR_INVALID_ARG
    assert call(Kx=None) == tai.TAI_ERR_INVALID_ARG
    assert call(nb=0) == tai.TAI_ERR_INVALID_ARG
    assert call(norb=0) == tai.TAI_ERR_INVALID_ARG
    assert call(norb=1025) == tai.TAI_ERR_INVALID_ARG
    assert call(pairs=dummy, npk=0) == tai.TAI_ERR_INVALID_ARG
    assert call(nb=60000, norb=1024, params=_params(n=64)) == tai.TAI_ERR_INVALID_ARG   # tensors > 64 GiB
    assert call(params=_params(prec=4)) == tai.TAI_ERR_UNSUPPORTED
    assert call() == tai.TAI_ERR_NOT_READY


def test_partition_argument_checks(hctx):
    lib, h = hctx.lib, hctx.h
    b = I.small_random(3, natoms=2, shells=("s", "p"))
    ba = tai.BasisArrays(b)
    dummy = ctypes.c_void_p(16)
    cnt = (ctypes.c_int32 * 16)()
    box = (ctypes.c_double * 16)()
    call = lambda tau=1e-12, k=3, pairs=dummy, c=cnt, bx=box: \
        lib.tai_partition_pairs(h, ctypes.byref(ba.struct), tau, k, pairs, c, bx, None)
    for tau in (0.0, 1.0, -1e-3, float("nan")):
        assert call(tau=tau) == tai.TAI_ERR_INVALID_ARG
    for k in (0, 17):
        assert call(k=k) == tai.TAI_ERR_INVALID_ARG
    assert call(pairs=None) == tai.TAI_ERR_INVALID_ARG
    assert call(c=None) == tai.TAI_ERR_INVALID_ARG
    assert call(bx=None) == tai.TAI_ERR_INVALID_ARG
    assert call() == tai.TAI_ERR_NOT_READY


def test_apply_J_partitioned_argument_checks(hctx):
    lib, h = hctx.lib, hctx.h
    dummy = ctypes.c_void_p(16)
    nb = 4                        # npair = 10
    mk = lambda vals, t: (t * len(vals))(*vals)
    good_c = mk([4, 6], ctypes.c_int32)
    good_b = mk([3.0, 5.0], ctypes.c_double)
    p = _params()
    call = lambda c=good_c, bx=good_b, k=2, params=p, M=dummy: \
        lib.tai_apply_J_partitioned(h, M, nb, dummy, c, bx, k, ctypes.byref(params), dummy, dummy, None)
    assert call(c=mk([4, 5], ctypes.c_int32)) == tai.TAI_ERR_INVALID_ARG       # does not add up to npair
    assert call(c=mk([-1, 11], ctypes.c_int32)) == tai.TAI_ERR_INVALID_ARG
    assert call(bx=mk([0.0, 5.0], ctypes.c_double)) == tai.TAI_ERR_INVALID_ARG
    assert call(k=0) == tai.TAI_ERR_INVALID_ARG
    assert call(M=None) == tai.TAI_ERR_INVALID_ARG
    assert call(params=_params(prec=4)) == tai.TAI_ERR_UNSUPPORTED
    assert call(params=_params(rank_tol=1e-6)) == tai.TAI_ERR_UNSUPPORTED
    assert call(params=_params(degree_tol=1e-8)) == tai.TAI_ERR_UNSUPPORTED
    assert call() == tai.TAI_ERR_NOT_READY
    # the boxes give the half-widths: params->L is not read
    assert call(params=_params(L=0.0)) == tai.TAI_ERR_NOT_READY


def test_moments_partitioned_argument_checks(hctx):
    lib, h = hctx.lib, hctx.h
    b = I.small_random(3, natoms=2, shells=("s", "p"))   # nb = 8, npair = 36
    ba = tai.BasisArrays(b)
    dummy = ctypes.c_void_p(16)
    mk = lambda vals, t: (t * len(vals))(*vals)
    good_c = mk([10, 20], ctypes.c_int32)
    good_b = mk([3.0, 5.0], ctypes.c_double)
    p = _params()
    call = lambda c=good_c, bx=good_b, k=2, params=p, M=dummy, pairs=dummy: \
        lib.tai_moments_partitioned(h, ctypes.byref(ba.struct), ctypes.byref(params), pairs, c, bx, k, M, None)
    assert call(c=mk([-1, 20], ctypes.c_int32)) == tai.TAI_ERR_INVALID_ARG
    assert call(c=mk([0, 0], ctypes.c_int32)) == tai.TAI_ERR_INVALID_ARG          # no pairs at all
    assert call(c=mk([30, 7], ctypes.c_int32)) == tai.TAI_ERR_INVALID_ARG         # more than npair
    assert call(bx=mk([3.0, float("inf")], ctypes.c_double)) == tai.TAI_ERR_INVALID_ARG
    assert call(bx=mk([-1.0, 5.0], ctypes.c_double)) == tai.TAI_ERR_INVALID_ARG
    for k in (0, 17):
        assert call(k=k) == tai.TAI_ERR_INVALID_ARG
    assert call(M=None) == tai.TAI_ERR_INVALID_ARG
    assert call(pairs=None) == tai.TAI_ERR_INVALID_ARG
    assert call() == tai.TAI_ERR_NOT_READY
    # the boxes give the half-widths: params->L is not read
    assert call(params=_params(L=0.0)) == tai.TAI_ERR_NOT_READY


def test_assemble_B_partitioned_argument_checks(hctx):
    lib, h = hctx.lib, hctx.h
    dummy = ctypes.c_void_p(16)
    mk = lambda vals, t: (t * len(vals))(*vals)
    good_c = mk([4, 6], ctypes.c_int32)
    good_b = mk([3.0, 5.0], ctypes.c_double)
    p = _params()
    call = lambda c=good_c, bx=good_b, k=2, params=p, M=dummy, B=dummy, ldb=10: \
        lib.tai_assemble_B_partitioned(h, M, c, bx, k, ctypes.byref(params), B, ldb, None)
    assert call(c=mk([-1, 6], ctypes.c_int32)) == tai.TAI_ERR_INVALID_ARG
    assert call(c=mk([0, 0], ctypes.c_int32)) == tai.TAI_ERR_INVALID_ARG
    assert call(bx=mk([0.0, 5.0], ctypes.c_double)) == tai.TAI_ERR_INVALID_ARG
    assert call(bx=mk([3.0, float("nan")], ctypes.c_double)) == tai.TAI_ERR_INVALID_ARG
    for k in (0, 17):
        assert call(k=k) == tai.TAI_ERR_INVALID_ARG
    assert call(M=None) == tai.TAI_ERR_INVALID_ARG
    assert call(B=None) == tai.TAI_ERR_INVALID_ARG
    assert call(ldb=9) == tai.TAI_ERR_INVALID_ARG
    assert call(params=_params(rank_tol=1e-6)) == tai.TAI_ERR_UNSUPPORTED
    assert call(params=_params(degree_tol=1e-8)) == tai.TAI_ERR_UNSUPPORTED
    assert call() == tai.TAI_ERR_NOT_READY
    assert call(params=_params(L=0.0)) == tai.TAI_ERR_NOT_READY   # params->L is not read
