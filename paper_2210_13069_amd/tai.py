"""ctypes binding of libtai (include/tai.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch supplies device buffers and the current HIP stream.
The binding refuses to run when the library is missing: there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtai.so")

TAI_OK = 0
TAI_ERR_INVALID_ARG = -1
TAI_ERR_NOMEM = -2
TAI_ERR_HIP = -3
TAI_ERR_UNSUPPORTED = -4
TAI_ERR_NOT_READY = -5

NODES_LOBATTO = 0
NODES_GAUSS = 1

FP64, FP32, BF16X3, BF16X6, F16X3 = 0, 1, 2, 3, 4
PREC_NAMES = {FP64: "fp64", FP32: "fp32", BF16X3: "bf16x3", BF16X6: "bf16x6", F16X3: "f16x3"}
PREC_BY_NAME = {v: k for k, v in PREC_NAMES.items()}

# exported symbols declared in include/tai.h
SYMBOLS = ["tai_create", "tai_destroy", "tai_status_string", "tai_last_error", "tai_sync",
           "tai_quadrature", "tai_degrees", "tai_compress", "tai_moments", "tai_screen_pairs", "tai_moments_pairs",
           "tai_apply_J_pairs", "tai_apply_J_compressed", "tai_coulomb_mo", "tai_exchange", "tai_contract_pairs", "tai_apply_J_contracted", "tai_assemble_B", "tai_assemble_B_batched", "tai_apply_J", "tai_apply_J_noalloc",
           "tai_partition_pairs", "tai_moments_partitioned", "tai_apply_J_partitioned", "tai_assemble_B_partitioned", "tai_tune", "tai_profile_enable", "tai_profile_read", "tai_peak_probe"]
STAGES = ["nodes", "moments", "pack", "project", "assemble", "apply_J", "batched", "compress"]


class TaiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class tai_basis(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int32),
                ("center", ctypes.POINTER(ctypes.c_double)),
                ("alpha", ctypes.POINTER(ctypes.c_double)),
                ("lxyz", ctypes.POINTER(ctypes.c_int32)),
                ("coef", ctypes.POINTER(ctypes.c_double))]


class tai_params(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double),
                ("nq", ctypes.c_int32),
                ("n", ctypes.c_int32),
                ("L", ctypes.c_double),
                ("nodes", ctypes.c_int32),
                ("prec", ctypes.c_int32),
                ("degree_tol", ctypes.c_double),
                ("rank_tol", ctypes.c_double)]


class tai_mol(ctypes.Structure):
    _fields_ = [("basis", tai_basis),
                ("params", tai_params),
                ("M", ctypes.c_void_p),
                ("B", ctypes.c_void_p),
                ("ldb", ctypes.c_int64)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libtai.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2210_13069_amd.build`")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.tai_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.tai_destroy.argtypes = [vp]
    lib.tai_status_string.argtypes = [ctypes.c_int]
    lib.tai_status_string.restype = ctypes.c_char_p
    lib.tai_last_error.argtypes = [vp]
    lib.tai_last_error.restype = ctypes.c_char_p
    lib.tai_sync.argtypes = [vp, vp]
    lib.tai_quadrature.argtypes = [vp, ctypes.POINTER(tai_params), vp, vp, vp, vp, vp]
    lib.tai_degrees.argtypes = [vp, ctypes.POINTER(tai_params), vp, vp, vp]
    lib.tai_compress.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(tai_params), ctypes.POINTER(ctypes.c_int32),
                                 vp, vp, vp, vp, vp]
    lib.tai_exchange.argtypes = [vp, vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.POINTER(tai_params), vp,
                                 ctypes.c_int32, vp, vp]
    lib.tai_apply_J_compressed.argtypes = [vp, vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int32, vp,
                                           ctypes.POINTER(tai_params), vp, vp, vp]
    lib.tai_screen_pairs.argtypes = [vp, ctypes.POINTER(tai_basis), ctypes.c_double, vp,
                                     ctypes.POINTER(ctypes.c_int32), vp]
    lib.tai_moments_pairs.argtypes = [vp, ctypes.POINTER(tai_basis), ctypes.POINTER(tai_params), vp, ctypes.c_int32,
                                      vp, vp]
    lib.tai_apply_J_pairs.argtypes = [vp, vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.POINTER(tai_params), vp,
                                      vp, vp]
    lib.tai_coulomb_mo.argtypes = [vp, vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.POINTER(tai_params), vp,
                                   ctypes.c_int32, vp, vp]
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.tai_contract_pairs.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, i32p, ctypes.c_int32, vp,
                                       ctypes.c_int64, vp]
    lib.tai_apply_J_contracted.argtypes = [vp, vp, ctypes.c_int32, i32p, ctypes.POINTER(tai_params), vp, vp, vp]
    lib.tai_moments.argtypes = [vp, ctypes.POINTER(tai_basis), ctypes.POINTER(tai_params), vp, vp]
    lib.tai_assemble_B.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(tai_params), vp, ctypes.c_int64, vp]
    lib.tai_assemble_B_batched.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(tai_mol), vp]
    lib.tai_apply_J.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(tai_params), vp, vp, vp]
    lib.tai_partition_pairs.argtypes = [vp, ctypes.POINTER(tai_basis), ctypes.c_double, ctypes.c_int32, vp,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), vp]
    lib.tai_moments_partitioned.argtypes = [vp, ctypes.POINTER(tai_basis), ctypes.POINTER(tai_params), vp,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                            ctypes.c_int32, vp, vp]
    lib.tai_apply_J_partitioned.argtypes = [vp, vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                            ctypes.POINTER(tai_params), vp, vp, vp]
    lib.tai_assemble_B_partitioned.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                               ctypes.c_int32, ctypes.POINTER(tai_params), vp, ctypes.c_int64, vp]
    lib.tai_apply_J_noalloc.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(tai_params), vp, vp, vp]
    lib.tai_peak_probe.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp]
    lib.tai_profile_enable.argtypes = [vp, ctypes.c_int]
    lib.tai_profile_read.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]
    for name in SYMBOLS:
        if name not in ("tai_status_string", "tai_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def make_params(p, prec=None):
    """tai_params from an object with omega, nq, n, L, nodes (and prec,
    degree_tol, rank_tol)."""
    return tai_params(float(p.omega), int(p.nq), int(p.n), float(p.L), int(getattr(p, "nodes", 0)),
                      int(prec if prec is not None else getattr(p, "prec", FP64)),
                      float(getattr(p, "degree_tol", 0.0)), float(getattr(p, "rank_tol", 0.0)))


class BasisArrays:
    """Keeps the contiguous host arrays of a basis alive for a call."""

    def __init__(self, basis, coef=None):
        self.center = np.ascontiguousarray(basis.center, dtype=np.float64)
        self.alpha = np.ascontiguousarray(basis.alpha, dtype=np.float64)
        self.lxyz = np.ascontiguousarray(basis.lxyz, dtype=np.int32)
        self.coef = None if coef is None else np.ascontiguousarray(coef, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        self.struct = tai_basis(int(self.alpha.shape[0]),
                                self.center.ctypes.data_as(dp),
                                self.alpha.ctypes.data_as(dp),
                                self.lxyz.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                None if self.coef is None else self.coef.ctypes.data_as(dp))


class Context:
    """One libtai context on a HIP device (device=-1: validation only)."""

    def __init__(self, device=0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.tai_create(ctypes.byref(h), int(device))
        if st != TAI_OK:
            raise TaiError(st, f"tai_create failed: {self.lib.tai_status_string(st).decode()}")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self.lib.tai_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st, what):
        if st != TAI_OK:
            raise TaiError(st, f"{what}: {self.lib.tai_status_string(st).decode()}: "
                               f"{self.lib.tai_last_error(self.h).decode()}")

    def sync(self, stream=None):
        self.check(self.lib.tai_sync(self.h, _stream(stream)), "tai_sync")

    # ---- raw entry points (device tensors in, device tensors out) ----------
    def quadrature(self, params, t=None, w=None, xi=None, K=None, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_quadrature(self.h, ctypes.byref(p), _ptr(t), _ptr(w), _ptr(xi), _ptr(K),
                                           _stream(stream)), "tai_quadrature")

    def degrees(self, params, nk=None, C=None, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_degrees(self.h, ctypes.byref(p), _ptr(nk), _ptr(C), _stream(stream)),
                   "tai_degrees")

    def compress(self, M, npair, params, sigma=None, V=None, U=None, Kc=None, stream=None):
        """Rank of the low-rank compression of M (params.rank_tol > 0); the
        singular values and vectors go into sigma [n] and V [n][n], the
        compressed operands into U (room for [3][n][npair]) and Kc (room for
        [nq][n][n]) if given."""
        p = params if isinstance(params, tai_params) else make_params(params)
        rank = ctypes.c_int32()
        self.check(self.lib.tai_compress(self.h, _ptr(M), int(npair), ctypes.byref(p), ctypes.byref(rank),
                                         _ptr(sigma), _ptr(V), _ptr(U), _ptr(Kc), _stream(stream)), "tai_compress")
        return rank.value

    def apply_J_compressed(self, U, nb, R, Kc, params, D, J, pairs=None, npk=0, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_apply_J_compressed(self.h, _ptr(U), int(nb), _ptr(pairs), int(npk), int(R), _ptr(Kc),
                                                   ctypes.byref(p), _ptr(D), _ptr(J), _stream(stream)),
                   "tai_apply_J_compressed")

    def screen_pairs(self, basis_arrays, tau, pairs, stream=None):
        """Kept pair indices into `pairs` (int32 device tensor of npair
        entries); returns their count."""
        cnt = ctypes.c_int32()
        self.check(self.lib.tai_screen_pairs(self.h, ctypes.byref(basis_arrays.struct), float(tau), _ptr(pairs),
                                             ctypes.byref(cnt), _stream(stream)), "tai_screen_pairs")
        return cnt.value

    def moments_pairs(self, basis_arrays, params, pairs, npk, M, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_moments_pairs(self.h, ctypes.byref(basis_arrays.struct), ctypes.byref(p),
                                              _ptr(pairs), int(npk), _ptr(M), _stream(stream)), "tai_moments_pairs")

    def moments_partitioned(self, basis_arrays, params, pairs, counts, boxes, M, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        k = len(counts)
        cnt = (ctypes.c_int32 * k)(*[int(x) for x in counts])
        box = (ctypes.c_double * k)(*[float(x) for x in boxes])
        self.check(self.lib.tai_moments_partitioned(self.h, ctypes.byref(basis_arrays.struct), ctypes.byref(p),
                                                    _ptr(pairs), cnt, box, k, _ptr(M), _stream(stream)),
                   "tai_moments_partitioned")

    def assemble_B_partitioned(self, M, counts, boxes, params, B, ldb=None, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        k = len(counts)
        total = int(sum(counts))
        ldb = total if ldb is None else ldb
        esize = 8 if p.prec == FP64 else 4
        if B.element_size() != esize or B.numel() < (total - 1) * int(ldb) + total:
            raise ValueError(f"B must hold total x ldb {'FP64' if esize == 8 else 'FP32'} entries "
                             f"(got {B.dtype}, {B.numel()} entries)")
        cnt = (ctypes.c_int32 * k)(*[int(x) for x in counts])
        box = (ctypes.c_double * k)(*[float(x) for x in boxes])
        self.check(self.lib.tai_assemble_B_partitioned(self.h, _ptr(M), cnt, box, k, ctypes.byref(p), _ptr(B),
                                                       int(ldb), _stream(stream)), "tai_assemble_B_partitioned")

    def apply_J_pairs(self, M, nb, pairs, npk, params, D, J, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_apply_J_pairs(self.h, _ptr(M), int(nb), _ptr(pairs), int(npk), ctypes.byref(p),
                                              _ptr(D), _ptr(J), _stream(stream)), "tai_apply_J_pairs")

    def exchange(self, M, nb, params, Q, norb, Kx, pairs=None, npk=0, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_exchange(self.h, _ptr(M), int(nb), _ptr(pairs), int(npk), ctypes.byref(p), _ptr(Q),
                                         int(norb), _ptr(Kx), _stream(stream)), "tai_exchange")

    def coulomb_mo(self, M, nb, params, Q, norb, Jmo, pairs=None, npk=0, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_coulomb_mo(self.h, _ptr(M), int(nb), _ptr(pairs), int(npk), ctypes.byref(p), _ptr(Q),
                                           int(norb), _ptr(Jmo), _stream(stream)), "tai_coulomb_mo")

    def contract_pairs(self, Bp, nbp, fmap, prec, B, ldbp=None, ldb=None, stream=None):
        fm = np.ascontiguousarray(fmap, dtype=np.int32)
        ldbp = int(Bp.shape[1]) if ldbp is None else ldbp
        ldb = int(B.shape[1]) if ldb is None else ldb
        self.check(self.lib.tai_contract_pairs(self.h, _ptr(Bp), int(ldbp), int(nbp),
                                               fm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(prec), _ptr(B),
                                               int(ldb), _stream(stream)), "tai_contract_pairs")

    def apply_J_contracted(self, M, nbp, fmap, params, D, J, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        fm = np.ascontiguousarray(fmap, dtype=np.int32)
        self.check(self.lib.tai_apply_J_contracted(self.h, _ptr(M), int(nbp),
                                                   fm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(p),
                                                   _ptr(D), _ptr(J), _stream(stream)), "tai_apply_J_contracted")

    def moments(self, basis_arrays, params, M, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_moments(self.h, ctypes.byref(basis_arrays.struct), ctypes.byref(p), _ptr(M),
                                        _stream(stream)), "tai_moments")

    def assemble_B(self, M, npair, params, B, ldb=None, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        ldb = npair if ldb is None else ldb
        # the library cannot see the size of the caller's buffer: B holds
        # npair rows of ldb entries, FP64 for TAI_FP64 and FP32 otherwise
        esize = 8 if p.prec == FP64 else 4
        if B is not None and (B.element_size() != esize or B.numel() < (int(npair) - 1) * int(ldb) + int(npair)):
            raise ValueError(f"B must hold npair x ldb {'FP64' if esize == 8 else 'FP32'} entries "
                             f"(got {B.dtype}, {B.numel()} entries)")
        self.check(self.lib.tai_assemble_B(self.h, _ptr(M), int(npair), ctypes.byref(p), _ptr(B), int(ldb),
                                           _stream(stream)), "tai_assemble_B")

    def assemble_B_batched(self, mols, stream=None):
        arr = (tai_mol * len(mols))(*mols)
        self.check(self.lib.tai_assemble_B_batched(self.h, len(mols), arr, _stream(stream)),
                   "tai_assemble_B_batched")

    def tune(self, mode):
        """0: table default shapes, 1: tune each new signature once, 2: forget choices."""
        self.check(self.lib.tai_tune(self.h, int(mode)), "tai_tune")

    def peak_probe(self, what, stream=None):
        """Sustained device peak: 0 FP16 MFMA, 1 FP64 MFMA (TFLOP/s), 2 HBM copy (GB/s)."""
        v = ctypes.c_double()
        self.check(self.lib.tai_peak_probe(self.h, int(what), ctypes.byref(v), _stream(stream)), "tai_peak_probe")
        return v.value

    def profile_enable(self, enable=True):
        self.check(self.lib.tai_profile_enable(self.h, int(bool(enable))), "tai_profile_enable")

    def profile_read(self, stage):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self.check(self.lib.tai_profile_read(self.h, stage.encode(), ctypes.byref(ms), ctypes.byref(cnt)),
                   "tai_profile_read")
        return ms.value, cnt.value

    def apply_J(self, M, nb, params, D, J, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_apply_J(self.h, _ptr(M), int(nb), ctypes.byref(p), _ptr(D), _ptr(J),
                                        _stream(stream)), "tai_apply_J")

    def partition_pairs(self, basis_arrays, tau, nparts, pairs, stream=None):
        """Adaptive boxes: the partitions' pair lists into `pairs` (int32 device
        tensor of npair entries); returns (counts, boxes) as lists."""
        cnt = (ctypes.c_int32 * int(nparts))()
        box = (ctypes.c_double * int(nparts))()
        self.check(self.lib.tai_partition_pairs(self.h, ctypes.byref(basis_arrays.struct), float(tau), int(nparts),
                                                _ptr(pairs), cnt, box, _stream(stream)), "tai_partition_pairs")
        return list(cnt), list(box)

    def apply_J_partitioned(self, M, nb, pairs, counts, boxes, params, D, J, stream=None):
        p = params if isinstance(params, tai_params) else make_params(params)
        k = len(counts)
        cnt = (ctypes.c_int32 * k)(*[int(x) for x in counts])
        box = (ctypes.c_double * k)(*[float(x) for x in boxes])
        self.check(self.lib.tai_apply_J_partitioned(self.h, _ptr(M), int(nb), _ptr(pairs), cnt, box, k, ctypes.byref(p),
                                                    _ptr(D), _ptr(J), _stream(stream)), "tai_apply_J_partitioned")

    def apply_J_noalloc(self, M, nb, params, D, J, stream=None):
        """tai_apply_J with every intermediate in the library's static device
        scratch (no allocation)."""
        p = params if isinstance(params, tai_params) else make_params(params)
        self.check(self.lib.tai_apply_J_noalloc(self.h, _ptr(M), int(nb), ctypes.byref(p), _ptr(D), _ptr(J),
                                                _stream(stream)), "tai_apply_J_noalloc")


# ---- convenience wrappers allocating torch outputs ---------------------------
_default = {}


def context(device=0):
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def quadrature(params, device=0):
    import torch
    nq, n = int(params.nq), int(params.n)
    dev = torch.device("cuda", device)
    t = torch.empty(nq, dtype=torch.float64, device=dev)
    w = torch.empty(nq, dtype=torch.float64, device=dev)
    xi = torch.empty(n, dtype=torch.float64, device=dev)
    K = torch.empty((nq, n, n), dtype=torch.float64, device=dev)
    context(device).quadrature(params, t, w, xi, K)
    return t, w, xi, K


def degrees(params, device=0):
    """Per-node degrees N_k [nq] (int32) and kept coefficients C [nq][n][n]."""
    import torch
    nq, n = int(params.nq), int(params.n)
    dev = torch.device("cuda", device)
    nk = torch.empty(nq, dtype=torch.int32, device=dev)
    C = torch.empty((nq, n, n), dtype=torch.float64, device=dev)
    context(device).degrees(params, nk, C)
    return nk, C


def compress(M, params, device=0):
    """(rank, sigma [n], V [n][n]) of the low-rank compression of M."""
    import torch
    n = int(params.n)
    dev = torch.device("cuda", device)
    sigma = torch.empty(n, dtype=torch.float64, device=dev)
    V = torch.empty((n, n), dtype=torch.float64, device=dev)
    rank = context(device).compress(M, M.shape[2], params, sigma, V)
    return rank, sigma, V


def padded_rank(R, n):
    """Inner length min(n, 8 ceil(R / 8)) the compressed operands of rank R
    are laid out at (the rows and columns from R on are zero)."""
    return min(int(n), (int(R) + 7) // 8 * 8)


def compress_operands(M, params, device=0):
    """(rank R, U [3][Rp][npair], Kc [nq][Rp][Rp]): the compressed operands of
    M at the padded length Rp = padded_rank(R, n)."""
    import torch
    n, nq, npair = int(params.n), int(params.nq), int(M.shape[2])
    dev = torch.device("cuda", device)
    U = torch.empty(3 * n * npair, dtype=torch.float64, device=dev)
    Kc = torch.empty(nq * n * n, dtype=torch.float64, device=dev)
    R = context(device).compress(M, npair, params, U=U, Kc=Kc)
    Rp = padded_rank(R, n)
    return R, U[:3 * Rp * npair].view(3, Rp, npair), Kc[:nq * Rp * Rp].view(nq, Rp, Rp)


def apply_J_compressed(U, Kc, D, params, R, prec=FP64, pairs=None, device=0):
    """J (nb x nb FP64) from prepared compressed operands of rank R."""
    import torch
    nb = int(D.shape[0])
    J = torch.empty((nb, nb), dtype=torch.float64, device=U.device)
    npk = 0 if pairs is None else int(pairs.shape[0])
    context(device).apply_J_compressed(U, nb, int(R), Kc, make_params(params, prec), D, J, pairs, npk)
    return J


def partition_pairs(basis, tau, nparts, device=0):
    """(pairs int32 [npair] on the device, counts, boxes) of the adaptive
    boxes of a basis."""
    import torch
    ba = BasisArrays(basis)
    nb = ba.alpha.shape[0]
    pairs = torch.empty(nb * (nb + 1) // 2, dtype=torch.int32, device=torch.device("cuda", device))
    counts, boxes = context(device).partition_pairs(ba, tau, nparts, pairs)
    return pairs, counts, boxes


def moments_partitioned(basis, params, pairs, counts, boxes, device=0):
    """The partitions' moment blocks, block s on box boxes[s], concatenated."""
    import torch
    ba = BasisArrays(basis)
    n = int(params.n)
    total = int(sum(counts))
    M = torch.empty(3 * n * total, dtype=torch.float64, device=torch.device("cuda", device))
    context(device).moments_partitioned(ba, params, pairs, counts, boxes, M)
    return M


def assemble_B_partitioned(M, counts, boxes, params, prec=FP64, ldb=None, device=0):
    """B over adaptive boxes (total x total, FP64 for prec FP64 else FP32),
    rows and columns in the order of the concatenated partition lists."""
    import torch
    total = int(sum(counts))
    ldb = total if ldb is None else ldb
    dt = torch.float64 if prec == FP64 else torch.float32
    B = torch.empty((total, ldb), dtype=dt, device=M.device)
    context(device).assemble_B_partitioned(M, counts, boxes, make_params(params, prec), B, ldb)
    return B


def apply_J_partitioned(M, D, pairs, counts, boxes, params, prec=FP64, device=0):
    """J (nb x nb FP64) over adaptive boxes."""
    import torch
    nb = int(D.shape[0])
    J = torch.empty((nb, nb), dtype=torch.float64, device=M.device)
    context(device).apply_J_partitioned(M, nb, pairs, counts, boxes, make_params(params, prec), D, J)
    return J


def moments(basis, params, coef=None, device=0):
    """M[3][n][npair] (FP64, on the device) of a basis."""
    import torch
    ba = BasisArrays(basis, coef)
    npair = ba.alpha.shape[0] * (ba.alpha.shape[0] + 1) // 2
    M = torch.empty((3, int(params.n), npair), dtype=torch.float64, device=torch.device("cuda", device))
    context(device).moments(ba, params, M)
    return M


def aligned_ldb(npair):
    """A row stride for B (>= npair, a multiple of 16 entries) that starts
    every row on a 64-byte boundary, so that the assembly's 64-byte row
    pieces each fill whole memory segments."""
    return (int(npair) + 15) // 16 * 16


def assemble_B(M, params, prec=FP64, ldb=None, out=None, device=0):
    """Full npair x npair B (FP64 for prec FP64, else FP32) on the device."""
    import torch
    npair = int(M.shape[2])
    ldb = npair if ldb is None else ldb
    dt = torch.float64 if prec == FP64 else torch.float32
    B = out if out is not None else torch.empty((npair, ldb), dtype=dt, device=M.device)
    context(device).assemble_B(M, npair, make_params(params, prec), B, ldb)
    return B


def apply_J(M, D, params, prec=FP64, device=0):
    import torch
    nb = int(D.shape[0])
    J = torch.empty((nb, nb), dtype=torch.float64, device=M.device)
    context(device).apply_J(M, nb, make_params(params, prec), D, J)
    return J


def screen_pairs(basis, tau, device=0):
    """Pair indices kept by screening at tau (int32 device tensor, ascending)."""
    import torch
    ba = BasisArrays(basis)
    npair = ba.alpha.shape[0] * (ba.alpha.shape[0] + 1) // 2
    pairs = torch.empty(npair, dtype=torch.int32, device=torch.device("cuda", device))
    cnt = context(device).screen_pairs(ba, tau, pairs)
    return pairs[:cnt].clone()


def moments_pairs(basis, params, pairs, coef=None, device=0):
    """M[3][n][len(pairs)] (FP64, on the device) of the listed pairs."""
    import torch
    ba = BasisArrays(basis, coef)
    npk = int(pairs.shape[0])
    M = torch.empty((3, int(params.n), npk), dtype=torch.float64, device=torch.device("cuda", device))
    context(device).moments_pairs(ba, params, pairs, npk, M)
    return M


def apply_J_pairs(M, D, pairs, params, prec=FP64, device=0):
    """J (nb x nb FP64) with the pair sums restricted to `pairs`."""
    import torch
    nb = int(D.shape[0])
    J = torch.empty((nb, nb), dtype=torch.float64, device=M.device)
    context(device).apply_J_pairs(M, nb, pairs, int(pairs.shape[0]), make_params(params, prec), D, J)
    return J


def coulomb_mo(M, nb, Q, params, prec=FP64, pairs=None, device=0):
    """Orbital-basis Coulomb matrix [norb][norb] (FP64) for orbitals Q [norb][nb]."""
    import torch
    norb = int(Q.shape[0])
    Jmo = torch.empty((norb, norb), dtype=torch.float64, device=M.device)
    context(device).coulomb_mo(M, nb, make_params(params, prec), Q, norb, Jmo, pairs=pairs,
                               npk=0 if pairs is None else int(pairs.shape[0]))
    return Jmo


def contract_pairs(Bp, nbp, fmap, prec=FP64, device=0):
    """B over contracted pairs from B over the primitive pairs (see tai_contract_pairs)."""
    import torch
    nb = int(np.asarray(fmap)[-1]) + 1
    npc = nb * (nb + 1) // 2
    B = torch.empty((npc, npc), dtype=Bp.dtype, device=Bp.device)
    context(device).contract_pairs(Bp, nbp, fmap, prec, B)
    return B


def exchange(M, nb, Q, params, prec=FP64, pairs=None, device=0):
    """Long-range exchange matrix [nb][nb] (FP64) for orbitals Q [norb][nb]."""
    import torch
    norb = int(Q.shape[0])
    Kx = torch.empty((nb, nb), dtype=torch.float64, device=M.device)
    npk = 0 if pairs is None else int(pairs.shape[0])
    context(device).exchange(M, nb, make_params(params, prec), Q.contiguous(), norb, Kx, pairs, npk)
    return Kx


def apply_J_contracted(M, nbp, fmap, D, params, prec=FP64, device=0):
    """J over contracted functions from the primitive moments (see tai_apply_J_contracted)."""
    import torch
    nb = int(D.shape[0])
    J = torch.empty((nb, nb), dtype=torch.float64, device=M.device)
    context(device).apply_J_contracted(M, nbp, fmap, make_params(params, prec), D, J)
    return J
