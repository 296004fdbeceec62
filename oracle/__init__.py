"""Reference SpGEMM (the oracle) -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded C code in ``oracle.c`` (Gustavson's method, Algorithm 1
of Liu & Vinter, with a dense binary64 accumulator), wrapped here with ctypes
and numpy.  Only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the GPU library never does, and the
two share no code.

Matrices are passed as ``(rows, cols, row_ptr, col_idx, val)`` tuples of numpy
arrays (any integer dtype for the index arrays).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc: -O2, no FMA contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Result(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("val", ctypes.POINTER(ctypes.c_double)),
        ("val32", ctypes.POINTER(ctypes.c_float)),
        ("absval", ctypes.POINTER(ctypes.c_double)),
        ("u", ctypes.POINTER(ctypes.c_int64)),
    ]


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_free.argtypes = [ctypes.POINTER(_Result)]
        lib.oracle_free.restype = None
        lib.oracle_upper_bound.argtypes = [I64, P, P, P, P]
        lib.oracle_upper_bound.restype = I64
        lib.oracle_bin.argtypes = [I64, P, P, P]
        lib.oracle_bin.restype = I64
        for name in ("oracle_spgemm_f64", "oracle_spgemm_f32acc"):
            f = getattr(lib, name)
            f.argtypes = [I64, I64, I64, P, P, P, P, P, P]
            f.restype = ctypes.POINTER(_Result)
        lib.oracle_grad_f64.argtypes = [I64, I64, I64, P, P, P, P, P, P, P, P, P,
                                        P, I64, P, P, I64, P]
        lib.oracle_grad_f64.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(M, vdtype):
    rows, cols, rp, ci, v = M
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=vdtype)
    assert rp.shape == (rows + 1,) and ci.shape == v.shape == (int(rp[-1]),)
    return int(rows), int(cols), rp, ci, v


@dataclass
class OracleResult:
    """C = A*B in CSR, plus the per-row upper bounds of Algorithm 2."""
    rows: int
    cols: int
    row_ptr: np.ndarray   # int64, rows+1
    col_idx: np.ndarray   # int32
    val: np.ndarray       # float64 (or float32 for the binary32 variant)
    absval: np.ndarray    # float64, (|A||B|)_ik
    u: np.ndarray         # int64, rows

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def flops(self) -> int:
        return 2 * int(self.u.sum())


def spgemm(A, B, acc32: bool = False) -> OracleResult:
    """C = A*B.  binary64 accumulator; binary32 inputs are widened exactly.

    With ``acc32=True`` the inputs are taken as binary32 and every product and
    partial sum is rounded to binary32 (same order as the binary64 version).
    """
    lib = _load()
    vd = np.float32 if acc32 else np.float64
    m, k, arp, aci, av = _prep(A, vd)
    k2, n, brp, bci, bv = _prep(B, vd)
    if k != k2:
        raise ValueError("inner dimensions differ: %d vs %d" % (k, k2))
    f = lib.oracle_spgemm_f32acc if acc32 else lib.oracle_spgemm_f64
    r = f(m, k, n, _ptr(arp), _ptr(aci), _ptr(av), _ptr(brp), _ptr(bci), _ptr(bv))
    if not r:
        raise MemoryError("oracle allocation failed")
    try:
        res = r.contents
        nnz = int(res.nnz)
        rp = np.ctypeslib.as_array(res.row_ptr, shape=(m + 1,)).copy()
        u = np.ctypeslib.as_array(res.u, shape=(max(m, 1),))[:m].copy()
        if nnz:
            col = np.ctypeslib.as_array(res.col, shape=(nnz,)).copy()
            absval = np.ctypeslib.as_array(res.absval, shape=(nnz,)).copy()
            if acc32:
                val = np.ctypeslib.as_array(res.val32, shape=(nnz,)).copy()
            else:
                val = np.ctypeslib.as_array(res.val, shape=(nnz,)).copy()
        else:
            col = np.zeros(0, np.int32)
            absval = np.zeros(0, np.float64)
            val = np.zeros(0, vd)
    finally:
        lib.oracle_free(r)
    return OracleResult(m, n, rp, col, val, absval, u)


def upper_bound(A, B):
    """Algorithm 2: u_i = sum of nnz(b_j*) over the stored a_ij.  Returns (u, sum u)."""
    lib = _load()
    m, _, arp, aci, _ = _prep(A, np.float64)
    _, _, brp, _, _ = _prep(B, np.float64)
    u = np.zeros(max(m, 1), np.int64)
    tot = lib.oracle_upper_bound(m, _ptr(arp), _ptr(aci), _ptr(brp), _ptr(u))
    return u[:m], int(tot)


def bins(u: np.ndarray):
    """Algorithm 3 (paper thresholds): returns (bin id per row, C~ row sizes, nnz(C~))."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.int64)
    m = u.shape[0]
    b = np.zeros(max(m, 1), np.int32)
    h = np.zeros(max(m, 1), np.int64)
    tot = lib.oracle_bin(m, _ptr(u if m else np.zeros(1, np.int64)), _ptr(b), _ptr(h))
    return b[:m], h[:m], int(tot)


def grad(A, B, C_row_ptr, C_col_idx, dC, sample_a=None, sample_b=None,
         want_a=True, want_b=True):
    """Gradient of <dC, A*B> w.r.t. A's and B's stored values (binary64).

    ``sample_a`` / ``sample_b``: optional arrays of positions in A's / B's
    value arrays; only those entries are computed (the rest are NaN).
    Returns (dA, dB) as float64 arrays of nnz(A) and nnz(B) (or None).
    """
    lib = _load()
    m, k, arp, aci, av = _prep(A, np.float64)
    k2, n, brp, bci, bv = _prep(B, np.float64)
    assert k == k2
    crp = np.ascontiguousarray(C_row_ptr, dtype=np.int64)
    cci = np.ascontiguousarray(C_col_idx, dtype=np.int32)
    dc = np.ascontiguousarray(dC, dtype=np.float64)
    dA = np.full(max(av.shape[0], 1), np.nan) if want_a else None
    dB = np.full(max(bv.shape[0], 1), np.nan) if want_b else None
    sa = None if sample_a is None else np.ascontiguousarray(sample_a, dtype=np.int64)
    sb = None if sample_b is None else np.ascontiguousarray(sample_b, dtype=np.int64)
    nsa = -1 if sa is None else sa.shape[0]
    nsb = -1 if sb is None else sb.shape[0]
    z = np.zeros(1, np.int64)
    rc = lib.oracle_grad_f64(
        m, k, n, _ptr(arp), _ptr(aci), _ptr(av if av.size else np.zeros(1)),
        _ptr(brp), _ptr(bci), _ptr(bv if bv.size else np.zeros(1)),
        _ptr(crp), _ptr(cci if cci.size else np.zeros(1, np.int32)),
        _ptr(dc if dc.size else np.zeros(1)),
        _ptr(dA) if want_a else None, nsa if want_a else 0, _ptr(sa if sa is not None and sa.size else z),
        _ptr(dB) if want_b else None, nsb if want_b else 0, _ptr(sb if sb is not None and sb.size else z))
    if rc == -1:
        raise MemoryError("oracle allocation failed")
    if rc == -2:
        raise ValueError("dC pattern does not contain S(A*B)")
    return (dA[:av.shape[0]] if want_a else None, dB[:bv.shape[0]] if want_b else None)


def value_error(val, ref: OracleResult):
    """Componentwise scaled error max |c - c*| / (|A||B|)_ik (entries with a zero
    magnitude sum must be exactly zero), and the plain relative error over
    entries with |c*| >= 1e-8 (|A||B|)_ik.  Returns (scaled, plain)."""
    val = np.asarray(val, dtype=np.float64)
    ref_v = np.asarray(ref.val, dtype=np.float64)
    d = np.abs(val - ref_v)
    s = ref.absval
    zero = s == 0
    if np.any(d[zero] != 0):
        return float("inf"), float("inf")
    nz = ~zero
    scaled = float(np.max(d[nz] / s[nz])) if np.any(nz) else 0.0
    big = np.abs(ref_v) >= 1e-8 * s
    big &= nz
    plain = float(np.max(d[big] / np.abs(ref_v[big]))) if np.any(big) else 0.0
    return scaled, plain


def merge_pairs(keys: np.ndarray, vals, l: int):
    """Merge of sorted sequences (Section 3.2, the merge microbenchmark):
    ``keys`` holds pairs of ascending length-``l`` runs, each pair as 2l
    consecutive entries; every pair comes back in ascending key order, the
    first run's entries before the second's among equal keys (the stable
    sort of the pair's entries, a library sort standing for the merge).
    ``vals`` (or None) moves with the keys.  Returns (keys, vals)."""
    k = np.asarray(keys).reshape(-1, 2 * l)
    order = np.argsort(k, axis=1, kind="stable")
    ko = np.take_along_axis(k, order, axis=1).reshape(-1)
    if vals is None:
        return ko, None
    v = np.asarray(vals).reshape(-1, 2 * l)
    return ko, np.take_along_axis(v, order, axis=1).reshape(-1)
