"""Small CSR helpers for the tests (no SpGEMM arithmetic here)."""
import numpy as np

from synthetic import Csr


def random_csr(rng, rows, cols, density, dtype=np.float64, ints=False):
    """Random pattern with the given density; values either small integers
    (so every sum is exact in binary64) or U[-1, 1]."""
    mask = rng.random((rows, cols)) < density
    r, c = np.nonzero(mask)
    if ints:
        v = rng.integers(-4, 5, r.size).astype(dtype)
    else:
        v = rng.uniform(-1, 1, r.size).astype(dtype)
    counts = np.bincount(r, minlength=rows)
    rp = np.zeros(rows + 1, np.int32)
    np.cumsum(counts, out=rp[1:])
    return Csr(rows, cols, rp, c.astype(np.int32), v)


def transpose(M: Csr) -> Csr:
    r = np.repeat(np.arange(M.rows), np.diff(M.row_ptr))
    order = np.lexsort((r, M.col_idx))
    counts = np.bincount(M.col_idx, minlength=M.cols)
    rp = np.zeros(M.cols + 1, np.int32)
    np.cumsum(counts, out=rp[1:])
    return Csr(M.cols, M.rows, rp, r[order].astype(np.int32), M.val[order])


def identity(n, dtype=np.float64) -> Csr:
    return Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               np.ones(n, dtype=dtype))


def from_rows(rows, cols, entries, dtype=np.float64) -> Csr:
    """entries: list of (row, col, value)."""
    entries = sorted(entries)
    r = np.array([e[0] for e in entries], dtype=np.int64)
    counts = np.bincount(r, minlength=rows) if r.size else np.zeros(rows, np.int64)
    rp = np.zeros(rows + 1, np.int32)
    np.cumsum(counts, out=rp[1:])
    return Csr(rows, cols, rp, np.array([e[1] for e in entries], dtype=np.int32),
               np.array([e[2] for e in entries], dtype=dtype))


def read_golden(path):
    """Parse a golden file of 'NAME rows cols' headers followed by 'r c v' lines."""
    mats = {}
    cur = None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split()
            if parts[0][0].isalpha():
                cur = parts[0]
                mats[cur] = (int(parts[1]), int(parts[2]), [])
            else:
                mats[cur][2].append((int(parts[0]), int(parts[1]), float(parts[2])))
    return {k: from_rows(r, c, e) for k, (r, c, e) in mats.items()}


def csr_equal_structure(rp1, ci1, rp2, ci2):
    return (np.array_equal(np.asarray(rp1, np.int64), np.asarray(rp2, np.int64))
            and np.array_equal(np.asarray(ci1, np.int32), np.asarray(ci2, np.int32)))
