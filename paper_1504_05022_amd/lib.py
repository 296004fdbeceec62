"""ctypes binding of libspgemm (include/spgemm.h).

Argument marshalling only: every stage runs in the HIP library.  PyTorch
supplies device memory (through the library's allocator callback, backed by
torch's caching allocator on the current stream) and the stream itself.
Importing works without a GPU; calling into the library needs the built
``libspgemm.so`` and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspgemm.so")

F32, F64 = 0, 1
NBINS = 38
NSTAGES = 12
STAGES = ("upper", "bin", "tiny", "medium", "long", "scan", "copy", "backward", "long_wave",
          "combine", "combine_wave", "long_sym")

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EOVERFLOW", -4: "EHIP", -5: "ESTATE"}


class SpgemmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "?"), code, msg))
        self.code = code
        self.name = _STATUS.get(code, "?")


class CsrDesc(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("dtype", ctypes.c_int32)]


class CsrOut(ctypes.Structure):
    _fields_ = CsrDesc._fields_


class Options(ctypes.Structure):
    _fields_ = [("bin_edges", ctypes.c_int32 * 5), ("long_slot", ctypes.c_int32),
                ("l1_cap", ctypes.c_int32), ("seg", ctypes.c_int64),
                ("pool_entries", ctypes.c_int64), ("validate", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("timing_mask", ctypes.c_int32),
                ("tiny_heap", ctypes.c_int32), ("long_path", ctypes.c_int32),
                ("long_direct", ctypes.c_int32),
                ("batch_shapes", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("k", ctypes.c_int64), ("n", ctypes.c_int64),
                ("flops", ctypes.c_int64), ("nnz_hat", ctypes.c_int64),
                ("nnz_tilde", ctypes.c_int64), ("nnz_c", ctypes.c_int64),
                ("max_u", ctypes.c_int64), ("bin_count", ctypes.c_int64 * NBINS),
                ("long_items", ctypes.c_int64), ("bytes_scratch", ctypes.c_int64),
                ("pool_entries", ctypes.c_int64), ("pool_used", ctypes.c_int64),
                ("realloc_rounds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("stage_ms", ctypes.c_float * NSTAGES), ("long_kernel_ms", ctypes.c_float),
                ("long_launches", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("bin_count", "stage_ms", "reserved")}
        d["bin_count"] = list(self.bin_count)
        d["stage_ms"] = dict(zip(STAGES, list(self.stage_ms)))
        return d


class BatchStats(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("shapes", ctypes.c_int32),
                ("items", ctypes.c_int64), ("flops", ctypes.c_int64), ("nnz_c", ctypes.c_int64),
                ("bin_edges", ctypes.c_int32 * 5), ("tune_ms", ctypes.c_float * 12),
                ("bytes_scratch", ctypes.c_int64)]

    def as_dict(self):
        return {"count": self.count, "fallback": self.fallback, "grid": self.grid,
                "shapes": self.shapes, "items": self.items, "flops": self.flops,
                "nnz_c": self.nnz_c, "bin_edges": list(self.bin_edges),
                "tune_ms": list(self.tune_ms), "bytes_scratch": self.bytes_scratch}


# exported symbols declared in include/spgemm.h
EXPORTS = ("spgemm_default_options", "spgemm_strerror", "spgemm_last_error", "spgemm_analyze",
           "spgemm_compute", "spgemm_backward", "spgemm_backward_static", "spgemm_plan_info",
           "spgemm_plan_destroy",
           "spgemm_batch_create", "spgemm_batch_run", "spgemm_batch_stats_get",
           "spgemm_batch_destroy", "spgemm_batch_multiply", "spgemm_merge_pairs",
           "spgemm_multiply")

_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_live: dict = {}


def _torch_alloc(nbytes, ctx, stream):
    try:
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    except RuntimeError:
        return None
    p = t.data_ptr()
    _live[p] = t
    return p


def _torch_free(ptr, ctx, stream):
    _live.pop(ptr, None)


_alloc_cb = _ALLOC_T(_torch_alloc)
_free_cb = _FREE_T(_torch_free)


def load(path: str = LIB_PATH):
    """Load libspgemm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libspgemm.so not found at %s: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.spgemm_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.spgemm_default_options.restype = None
    lib.spgemm_strerror.argtypes = [ctypes.c_int]
    lib.spgemm_strerror.restype = ctypes.c_char_p
    lib.spgemm_last_error.argtypes = []
    lib.spgemm_last_error.restype = ctypes.c_char_p
    lib.spgemm_analyze.argtypes = [ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc),
                                   ctypes.POINTER(Options), _ALLOC_T, _FREE_T, P, P,
                                   ctypes.POINTER(P), ctypes.POINTER(Info)]
    lib.spgemm_analyze.restype = ctypes.c_int
    lib.spgemm_compute.argtypes = [P, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc),
                                   ctypes.POINTER(CsrOut), P, ctypes.POINTER(Info)]
    lib.spgemm_compute.restype = ctypes.c_int
    lib.spgemm_backward.argtypes = [P, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc),
                                    ctypes.POINTER(CsrDesc), P, P, P]
    lib.spgemm_backward.restype = ctypes.c_int
    lib.spgemm_backward_static.argtypes = [P, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc),
                                           ctypes.POINTER(CsrDesc), P, P, P]
    lib.spgemm_backward_static.restype = ctypes.c_int
    lib.spgemm_plan_info.argtypes = [P, ctypes.POINTER(Info)]
    lib.spgemm_plan_info.restype = ctypes.c_int
    lib.spgemm_plan_destroy.argtypes = [P]
    lib.spgemm_plan_destroy.restype = ctypes.c_int
    lib.spgemm_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(CsrDesc),
                                        ctypes.POINTER(CsrDesc), ctypes.POINTER(Options),
                                        _ALLOC_T, _FREE_T, P, P, ctypes.POINTER(P),
                                        ctypes.POINTER(BatchStats)]
    lib.spgemm_batch_create.restype = ctypes.c_int
    lib.spgemm_batch_run.argtypes = [P, ctypes.POINTER(CsrOut), P]
    lib.spgemm_batch_run.restype = ctypes.c_int
    lib.spgemm_batch_stats_get.argtypes = [P, ctypes.POINTER(BatchStats)]
    lib.spgemm_batch_stats_get.restype = ctypes.c_int
    lib.spgemm_batch_destroy.argtypes = [P]
    lib.spgemm_batch_destroy.restype = ctypes.c_int
    lib.spgemm_batch_multiply.argtypes = [ctypes.c_int32, ctypes.POINTER(CsrDesc),
                                          ctypes.POINTER(CsrDesc), ctypes.POINTER(Options),
                                          _ALLOC_T, _FREE_T, P, P, ctypes.POINTER(CsrOut),
                                          ctypes.POINTER(P), ctypes.POINTER(BatchStats)]
    lib.spgemm_batch_multiply.restype = ctypes.c_int
    lib.spgemm_merge_pairs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int, P, P, P, P, P]
    lib.spgemm_merge_pairs.restype = ctypes.c_int
    lib.spgemm_multiply.argtypes = [ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc),
                                    ctypes.POINTER(Options), _ALLOC_T, _FREE_T, P, P,
                                    ctypes.POINTER(CsrOut), ctypes.POINTER(Info)]
    lib.spgemm_multiply.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise SpgemmError(rc, _lib.spgemm_last_error().decode(errors="replace"))


def default_options(**kw) -> Options:
    """The library defaults; keyword arguments override single fields."""
    o = Options()
    load().spgemm_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "bin_edges":
            for i, e in enumerate(v):
                o.bin_edges[i] = int(e)
        elif v is not None:
            setattr(o, k, int(v))
    return o


_DT = {torch.float32: F32, torch.float64: F64}


class CsrMatrix:
    """A CSR matrix on the GPU: int32 row_ptr / col_idx, float32/64 values."""

    def __init__(self, shape, row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor):
        self.shape = (int(shape[0]), int(shape[1]))
        self.row_ptr = row_ptr
        self.col_idx = col_idx
        self.val = val

    @property
    def nnz(self):
        return int(self.col_idx.numel())

    @property
    def dtype(self):
        return self.val.dtype

    @classmethod
    def from_host(cls, M, device="cuda"):
        """From a ``synthetic.Csr`` (or (rows, cols, row_ptr, col_idx, val))."""
        if hasattr(M, "as_tuple"):
            M = M.as_tuple()
        rows, cols, rp, ci, v = M
        return cls((rows, cols),
                   torch.as_tensor(rp).to(device=device, dtype=torch.int32),
                   torch.as_tensor(ci).to(device=device, dtype=torch.int32),
                   torch.as_tensor(v).to(device=device))

    @classmethod
    def from_torch(cls, t: torch.Tensor):
        """From a torch.sparse_csr_tensor."""
        return cls(tuple(t.shape), t.crow_indices().to(torch.int32).contiguous(),
                   t.col_indices().to(torch.int32).contiguous(), t.values().contiguous())

    def to_torch(self) -> torch.Tensor:
        return torch.sparse_csr_tensor(self.row_ptr, self.col_idx, self.val, self.shape)

    def to_host(self):
        return (self.shape[0], self.shape[1], self.row_ptr.cpu().numpy(),
                self.col_idx.cpu().numpy(), self.val.cpu().numpy())

    def with_values(self, val: torch.Tensor) -> "CsrMatrix":
        return CsrMatrix(self.shape, self.row_ptr, self.col_idx, val)

    def desc(self) -> CsrDesc:
        if self.val.dtype not in _DT:
            raise TypeError("values must be float32 or float64")
        for t in (self.row_ptr, self.col_idx, self.val):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous CUDA tensors")
        if self.row_ptr.dtype != torch.int32 or self.col_idx.dtype != torch.int32:
            raise TypeError("index arrays must be int32")
        return CsrDesc(self.shape[0], self.shape[1], self.nnz, self.row_ptr.data_ptr(),
                       self.col_idx.data_ptr(), self.val.data_ptr(), _DT[self.val.dtype])


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _take(ptr, nbytes, dtype):
    buf = _live.pop(ptr)
    return buf[:nbytes].view(dtype)


class Plan:
    """spgemm_analyze on construction; compute() / backward() reuse it."""

    def __init__(self, A: CsrMatrix, B: CsrMatrix, options: Options | None = None, **kw):
        lib = load()
        self.A, self.B = A, B
        self._da, self._db = A.desc(), B.desc()
        opts = options if options is not None else default_options(**kw)
        self._h = ctypes.c_void_p()
        info = Info()
        rc = lib.spgemm_analyze(ctypes.byref(self._da), ctypes.byref(self._db), ctypes.byref(opts),
                                _alloc_cb, _free_cb, None, _stream_handle(),
                                ctypes.byref(self._h), ctypes.byref(info))
        _check(rc)
        self.info = info

    def compute(self) -> CsrMatrix:
        out = CsrOut()
        info = Info()
        rc = _lib.spgemm_compute(self._h, ctypes.byref(self._da), ctypes.byref(self._db),
                                 ctypes.byref(out), _stream_handle(), ctypes.byref(info))
        _check(rc)
        self.info = info
        return _out_matrix(out)

    def backward(self, C: CsrMatrix, dC: torch.Tensor, want_a=True, want_b=True):
        """(dA, dB) value tensors on A's and B's patterns (None where not wanted)."""
        dA = torch.empty_like(self.A.val) if want_a else None
        dB = torch.empty_like(self.B.val) if want_b else None
        dc = C.with_values(dC.contiguous()).desc()
        rc = _lib.spgemm_backward(self._h, ctypes.byref(self._da), ctypes.byref(self._db),
                                  ctypes.byref(dc), dA.data_ptr() if want_a else None,
                                  dB.data_ptr() if want_b else None, _stream_handle())
        _check(rc)
        return dA, dB

    def backward_static(self, C: CsrMatrix, dC: torch.Tensor, dA=None, dB=None):
        """backward() through the entry point that allocates no device memory
        (its scratch is a fixed area in the library): the caller passes the
        output tensors dA / dB (None to skip one)."""
        dc = C.with_values(dC.contiguous()).desc()
        rc = _lib.spgemm_backward_static(self._h, ctypes.byref(self._da), ctypes.byref(self._db),
                                         ctypes.byref(dc), dA.data_ptr() if dA is not None else None,
                                         dB.data_ptr() if dB is not None else None,
                                         _stream_handle())
        _check(rc)
        return dA, dB

    def refresh_info(self):
        info = Info()
        _check(_lib.spgemm_plan_info(self._h, ctypes.byref(info)))
        self.info = info
        return info

    def close(self):
        if self._h:
            _lib.spgemm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _out_matrix(out: CsrOut) -> CsrMatrix:
    """Tensors over the three arrays the library allocated for C."""
    m, nnz = int(out.rows), int(out.nnz)
    vt = torch.float64 if out.dtype == F64 else torch.float32
    rp = _take(out.row_ptr, 4 * (m + 1), torch.int32)
    ci = _take(out.col_idx, 4 * nnz, torch.int32)
    va = _take(out.val, vt.itemsize * nnz, vt)
    return CsrMatrix((m, int(out.cols)), rp, ci, va)


def spgemm(A: CsrMatrix, B: CsrMatrix, return_info=False, **kw):
    """C = A*B (analyze + compute + release in one library call)."""
    lib = load()
    da, db = A.desc(), B.desc()
    opts = default_options(**kw)
    out = CsrOut()
    info = Info()
    _check(lib.spgemm_multiply(ctypes.byref(da), ctypes.byref(db), ctypes.byref(opts), _alloc_cb,
                               _free_cb, None, _stream_handle(), ctypes.byref(out),
                               ctypes.byref(info)))
    C = _out_matrix(out)
    return (C, info) if return_info else C


MERGE_ALGORITHMS = ("ranking", "merge_path", "odd_even", "bitonic", "bitonic_advanced")


def merge_pairs(keys: torch.Tensor, vals, l: int, algorithm: str, threads: int = 256):
    """spgemm_merge_pairs on device tensors: ``keys`` (int32 holding the
    32-bit unsigned keys) stores pairs of ascending length-``l`` runs, 2l
    entries per pair; ``vals`` is None or an int32 / int64 tensor of the same
    length.  Returns new (keys, vals) tensors, every pair merged."""
    lib = load()
    if keys.dtype != torch.int32 or not keys.is_cuda:
        raise TypeError("keys must be a CUDA int32 tensor")
    n = keys.numel()
    if n % (2 * l):
        raise ValueError("keys must hold whole pairs of 2l entries")
    vb = 0 if vals is None else vals.element_size()
    if vals is not None and (vals.numel() != n or vb not in (4, 8)):
        raise ValueError("vals must be None or 4- or 8-byte values, one per key")
    ko = torch.empty_like(keys)
    vo = None if vals is None else torch.empty_like(vals)
    _check(lib.spgemm_merge_pairs(MERGE_ALGORITHMS.index(algorithm), vb, l, n // (2 * l), threads,
                                  keys.data_ptr(), None if vals is None else vals.data_ptr(),
                                  ko.data_ptr(), None if vo is None else vo.data_ptr(),
                                  _stream_handle()))
    return ko, vo


def _view(ptr, nbytes, dtype):
    """A tensor view of library-owned memory that came from the allocator."""
    return _live[ptr][:nbytes].view(dtype)


class Batch:
    """Many independent products C_p = A_p * B_p replayed from one HIP graph
    (one kernel launch per capacity class over the rows of every problem).

    ``pairs``: list of (A_p, B_p) CsrMatrix pairs (binary32 and binary64 may
    be mixed).  The matrices must stay alive and keep their patterns.
    """

    def __init__(self, pairs, options: Options | None = None, **kw):
        lib = load()
        self.pairs = list(pairs)
        n = len(self.pairs)
        self._A = (CsrDesc * max(n, 1))(*[a.desc() for a, _ in self.pairs])
        self._B = (CsrDesc * max(n, 1))(*[b.desc() for _, b in self.pairs])
        opts = options if options is not None else default_options(**kw)
        self._h = ctypes.c_void_p()
        st = BatchStats()
        rc = lib.spgemm_batch_create(n, self._A, self._B, ctypes.byref(opts), _alloc_cb,
                                     _free_cb, None, _stream_handle(), ctypes.byref(self._h),
                                     ctypes.byref(st))
        _check(rc)
        self.stats = st
        self._outs = (CsrOut * max(n, 1))()

    def run(self, views=True):
        """Recompute every C_p; returns CsrMatrix views of the batch-owned outputs."""
        _check(_lib.spgemm_batch_run(self._h, self._outs, _stream_handle()))
        if not views:
            return None
        res = []
        for p in range(len(self.pairs)):
            o = self._outs[p]
            m, nnz = int(o.rows), int(o.nnz)
            vt = torch.float64 if o.dtype == F64 else torch.float32
            res.append(CsrMatrix((m, int(o.cols)), _view(o.row_ptr, 4 * (m + 1), torch.int32),
                                 _view(o.col_idx, 4 * nnz, torch.int32),
                                 _view(o.val, vt.itemsize * nnz, vt)))
        return res

    def close(self):
        if self._h:
            _lib.spgemm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_multiply(pairs, options: Options | None = None, return_stats=False, **kw):
    """Every C_p = A_p * B_p of ``pairs`` (list of (A_p, B_p) CsrMatrix
    pairs, binary32 and binary64 mixed) in one spgemm_batch_multiply call:
    no plan is kept.  The outputs are views into one device block, which
    lives as long as any of them."""
    lib = load()
    pairs = list(pairs)
    n = len(pairs)
    da = (CsrDesc * max(n, 1))(*[a.desc() for a, _ in pairs])
    db = (CsrDesc * max(n, 1))(*[b.desc() for _, b in pairs])
    opts = options if options is not None else default_options(**kw)
    outs = (CsrOut * max(n, 1))()
    mem = ctypes.c_void_p()
    st = BatchStats()
    _check(lib.spgemm_batch_multiply(n, da, db, ctypes.byref(opts), _alloc_cb, _free_cb, None,
                                     _stream_handle(), outs, ctypes.byref(mem), ctypes.byref(st)))
    res = []
    if mem.value:
        block = _live.pop(mem.value)
        base = mem.value
        for p in range(n):
            o = outs[p]
            m, nnz = int(o.rows), int(o.nnz)
            vt = torch.float64 if o.dtype == F64 else torch.float32

            def part(ptr, nbytes, dt):
                off = ptr - base
                return block[off:off + nbytes].view(dt)

            res.append(CsrMatrix((m, int(o.cols)), part(o.row_ptr, 4 * (m + 1), torch.int32),
                                 part(o.col_idx, 4 * nnz, torch.int32),
                                 part(o.val, vt.itemsize * nnz, vt)))
    return (res, st) if return_stats else res
