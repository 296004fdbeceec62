"""Seeded generators of CSR matrices for the SpGEMM workloads.

Workloads (they stand in for the paper's University of Florida matrices and
CUSP AMG hierarchies, which are not available):

1. uniform squaring: A is 2000 x 2000 with exactly 10 distinct uniformly drawn
   columns per row, values U[-1, 1] in binary64; C = A*A.
2. irregular squaring: A is 200000 x 200000 with power-law row degrees
   (exponent 2.1, mean 16, capped at 20000), distinct uniform columns, values
   U[-1, 1] in binary64; C = A*A.
3. Galerkin product R*(A*P) of algebraic multigrid: A is the 27-point stencil
   on a 64^3 grid (diagonal 26, off-diagonals -1, truncated at the boundary),
   P aggregates 2x2x2 blocks (entries 1.0), R = P^T, all binary64.  The
   multigrid experiment's other problems (2D 5- and 9-point stencils on
   1024^2, 3D 7- and 27-point stencils on 101^3, both multiplication orders)
   use the same construction (`galerkin`).
4. 512 independent banded products A_i*B_i, n_i log-uniform in [1024, 65536],
   per-row degree uniform in {4..32}, columns in a band of width ceil(0.05 n)
   around the diagonal, binary64 for even i and binary32 for odd i,
   values U[-1, 1].
5. A (500000 x 500000, power-law degrees, exponent 2.2, mean 20, truncated
   at n) times B (500000 x 4096, 32 distinct uniform columns per row), values
   N(0, 1) in binary32; an upstream gradient dC ~ N(0, 1) on C's pattern.

Every generator takes its sizes as arguments (defaulting to the full
workload) so that tests can draw small matrices of the same structure.
Random streams: numpy PCG64 seeded with SEED_BASE + workload number and a
per-matrix sub-stream key.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 150405022


@dataclass
class Csr:
    rows: int
    cols: int
    row_ptr: np.ndarray  # int32 (int64 only if nnz >= 2^31)
    col_idx: np.ndarray  # int32, strictly increasing within each row
    val: np.ndarray      # float64 or float32

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def dtype(self):
        return self.val.dtype

    def as_tuple(self):
        return (self.rows, self.cols, self.row_ptr, self.col_idx, self.val)

    def astype(self, dtype) -> "Csr":
        return Csr(self.rows, self.cols, self.row_ptr, self.col_idx,
                   self.val.astype(dtype))

    def row_slice(self, r0: int, r1: int) -> "Csr":
        """Rows [r0, r1) as a new CSR (same column space)."""
        a, b = int(self.row_ptr[r0]), int(self.row_ptr[r1])
        rp = (self.row_ptr[r0:r1 + 1] - a).astype(self.row_ptr.dtype)
        return Csr(r1 - r0, self.cols, rp, self.col_idx[a:b], self.val[a:b])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.rows, self.cols), dtype=np.float64)
        r = np.repeat(np.arange(self.rows), np.diff(self.row_ptr))
        d[r, self.col_idx] = self.val
        return d

    def pattern_dense(self) -> np.ndarray:
        d = np.zeros((self.rows, self.cols), dtype=bool)
        r = np.repeat(np.arange(self.rows), np.diff(self.row_ptr))
        d[r, self.col_idx] = True
        return d


def rng_for(workload: int, *sub: int) -> np.random.Generator:
    """PCG64 stream for a workload number and sub-stream key."""
    ss = np.random.SeedSequence(SEED_BASE + workload, spawn_key=tuple(sub))
    return np.random.Generator(np.random.PCG64(ss))


def _row_ptr(counts: np.ndarray) -> np.ndarray:
    rp = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    if rp[-1] < 2**31:
        rp = rp.astype(np.int32)
    return rp


def distinct_columns(rng: np.random.Generator, degrees: np.ndarray, ncols: int,
                     lo: np.ndarray | None = None, width: np.ndarray | int | None = None):
    """Distinct uniformly drawn columns for every row, sorted ascending.

    Row r receives ``degrees[r]`` distinct columns from [lo[r], lo[r] + width[r])
    (the whole column range by default).  Draws with replacement, drops
    duplicates and tops up until every row has its exact count.
    Returns (row_ptr, col_idx).
    """
    m = degrees.shape[0]
    if lo is None:
        lo = np.zeros(m, dtype=np.int64)
    if width is None:
        width = np.full(m, ncols, dtype=np.int64)
    width = np.broadcast_to(np.asarray(width, dtype=np.int64), (m,))
    degrees = np.minimum(degrees.astype(np.int64), width)
    keys = np.zeros(0, dtype=np.int64)
    need = degrees.copy()
    have = np.zeros(m, dtype=np.int64)
    rows_all = np.arange(m, dtype=np.int64)
    while True:
        draw_rows = np.repeat(rows_all, need)
        if draw_rows.size == 0:
            break
        c = lo[draw_rows] + (rng.random(draw_rows.size) * width[draw_rows]).astype(np.int64)
        c = np.minimum(c, lo[draw_rows] + width[draw_rows] - 1)
        keys = np.unique(np.concatenate([keys, draw_rows * ncols + c]))
        have = np.bincount(keys // ncols, minlength=m).astype(np.int64)
        need = degrees - have
        if not np.any(need > 0):
            break
        need = np.maximum(need, 0)
    # rows can only exceed their degree if a top-up overshot: never happens
    # because every draw is for the exact deficit and duplicates are dropped.
    rows = keys // ncols
    cols = (keys - rows * ncols).astype(np.int32)
    counts = np.bincount(rows, minlength=m)
    return _row_ptr(counts), cols


def powerlaw_degrees(rng: np.random.Generator, m: int, gamma: float, mean: float,
                     cap: int) -> np.ndarray:
    """Row degrees d = round(X), X a truncated Pareto variable with density
    proportional to x^-gamma on [x_min, cap].  x_min is found by bisection on
    this stream's own uniform draws so the realised mean of d equals ``mean``
    (to within 0.5%)."""
    u = rng.random(m)
    e = 1.0 - gamma

    def degrees_for(xmin):
        a = xmin ** e
        b = float(cap) ** e
        x = (a - u * (a - b)) ** (1.0 / e)
        return np.clip(np.rint(x), 1, cap).astype(np.int64)

    lo, hi = 1.0, float(mean)
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if degrees_for(mid).mean() < mean:
            lo = mid
        else:
            hi = mid
    d = degrees_for(hi)
    return d


def _values(rng, n, dist, dtype):
    if dist == "uniform":
        v = rng.uniform(-1.0, 1.0, n)
    elif dist == "normal":
        v = rng.standard_normal(n)
    else:
        raise ValueError(dist)
    return v.astype(dtype)


def uniform_csr(rows, cols, degree, workload=1, sub=0, dtype=np.float64, dist="uniform") -> Csr:
    """Exactly ``degree`` distinct uniform columns per row."""
    rng = rng_for(workload, sub)
    rp, ci = distinct_columns(rng, np.full(rows, degree, dtype=np.int64), cols)
    return Csr(rows, cols, rp, ci, _values(rng, ci.size, dist, dtype))


def powerlaw_csr(n, gamma, mean, cap, workload, sub=0, dtype=np.float64, dist="uniform",
                 cols=None) -> Csr:
    """Square (or n x cols) matrix with power-law row degrees and distinct
    uniform columns."""
    cols = n if cols is None else cols
    rng = rng_for(workload, sub)
    d = powerlaw_degrees(rng, n, gamma, mean, min(cap, cols))
    rp, ci = distinct_columns(rng, d, cols)
    return Csr(n, cols, rp, ci, _values(rng, ci.size, dist, dtype))


def _grid_coords(g):
    f = np.arange(g ** 3, dtype=np.int64)
    return f % g, (f // g) % g, f // (g * g)


def stencil27(g=64, diag=26.0, off=-1.0, dtype=np.float64) -> Csr:
    """27-point stencil on a g^3 grid, fine index x + g*(y + g*z), truncated
    at the boundary (no wrap-around)."""
    x, y, z = _grid_coords(g)
    n = g ** 3
    cols, rows, vals = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok = ((x + dx >= 0) & (x + dx < g) & (y + dy >= 0) & (y + dy < g)
                      & (z + dz >= 0) & (z + dz < g))
                r = np.nonzero(ok)[0]
                c = (x[r] + dx) + g * ((y[r] + dy) + g * (z[r] + dz))
                rows.append(r)
                cols.append(c)
                vals.append(np.full(r.size, diag if (dx, dy, dz) == (0, 0, 0) else off))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    counts = np.bincount(r, minlength=n)
    return Csr(n, n, _row_ptr(counts), c[order].astype(np.int32), v[order].astype(dtype))


def aggregation_p(g=64, dtype=np.float64) -> Csr:
    """Piecewise-constant prolongation: fine point (x,y,z) -> aggregate
    (x//2, y//2, z//2) with coarse index X + (g/2)*(Y + (g/2)*Z), value 1."""
    x, y, z = _grid_coords(g)
    h = g // 2
    agg = (x // 2) + h * ((y // 2) + h * (z // 2))
    n = g ** 3
    return Csr(n, h ** 3, _row_ptr(np.ones(n, dtype=np.int64)), agg.astype(np.int32),
               np.ones(n, dtype=dtype))


def aggregation_r(g=64, dtype=np.float64) -> Csr:
    """Restriction R = P^T, built directly: coarse row I lists its 8 fine
    points in ascending fine index, value 1."""
    h = g // 2
    nc = h ** 3
    X = np.arange(nc, dtype=np.int64) % h
    Y = (np.arange(nc, dtype=np.int64) // h) % h
    Z = np.arange(nc, dtype=np.int64) // (h * h)
    cols = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                cols.append((2 * X + dx) + g * ((2 * Y + dy) + g * (2 * Z + dz)))
    c = np.stack(cols, axis=1)
    c.sort(axis=1)
    return Csr(nc, g ** 3, _row_ptr(np.full(nc, 8, dtype=np.int64)),
               c.reshape(-1).astype(np.int32), np.ones(nc * 8, dtype=dtype))


def stencil(g, dim, points, dtype=np.float64) -> Csr:
    """Constant-coefficient stencil on a grid of g points per side in `dim`
    dimensions (fine index x + g*y, or x + g*(y + g*z)), truncated at the
    boundary.  points = 2*dim + 1 couples each point to its axis neighbours
    (2D 5-point, 3D 7-point); points = 3**dim to every point of its unit cube
    (2D 9-point, 3D 27-point).  Off-diagonals are -1 and the diagonal is the
    neighbour count (4, 6, 8 or 26), so interior rows sum to zero."""
    if points not in (2 * dim + 1, 3 ** dim):
        raise ValueError("points must be 2*dim+1 or 3**dim")
    n = g ** dim
    f = np.arange(n, dtype=np.int64)
    coord = [(f // g ** k) % g for k in range(dim)]
    nb = points - 1
    rows, cols, vals = [], [], []
    for off in itertools.product((-1, 0, 1), repeat=dim):
        if points == 2 * dim + 1 and sum(abs(o) for o in off) > 1:
            continue
        ok = np.ones(n, dtype=bool)
        for k in range(dim):
            ok &= (coord[k] + off[k] >= 0) & (coord[k] + off[k] < g)
        r = np.nonzero(ok)[0]
        c = np.zeros(r.size, dtype=np.int64)
        for k in range(dim):
            c += (coord[k][r] + off[k]) * g ** k
        rows.append(r)
        cols.append(c)
        vals.append(np.full(r.size, float(nb) if not any(off) else -1.0))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    return Csr(n, n, _row_ptr(np.bincount(r, minlength=n)), c[order].astype(np.int32),
               v[order].astype(dtype))


def aggregates(g, dim):
    """Aggregate of every fine point of the g^dim grid: blocks of 2 points per
    side (the last block of an odd side holds one), coarse index
    X + h*Y (+ h^2*Z) with h = ceil(g/2) coarse points per side."""
    h = (g + 1) // 2
    f = np.arange(g ** dim, dtype=np.int64)
    agg = np.zeros(f.size, dtype=np.int64)
    for k in range(dim):
        agg += ((f // g ** k) % g // 2) * h ** k
    return agg, h ** dim


def aggregation_p_grid(g, dim, dtype=np.float64) -> Csr:
    """Piecewise-constant prolongation of unsmoothed aggregation: fine point
    i -> its aggregate, value 1."""
    agg, nc = aggregates(g, dim)
    n = agg.size
    return Csr(n, nc, _row_ptr(np.ones(n, dtype=np.int64)), agg.astype(np.int32),
               np.ones(n, dtype=dtype))


def aggregation_r_grid(g, dim, dtype=np.float64) -> Csr:
    """Restriction R = P^T, built directly: coarse row I lists the fine points
    of aggregate I in ascending fine index, value 1."""
    agg, nc = aggregates(g, dim)
    fine = np.arange(agg.size, dtype=np.int64)
    order = np.lexsort((fine, agg))
    return Csr(nc, agg.size, _row_ptr(np.bincount(agg, minlength=nc)),
               fine[order].astype(np.int32), np.ones(agg.size, dtype=dtype))


# Galerkin problems of the multigrid experiment: name -> (dim, points, grid
# points per side at the measured size)
GALERKIN = {"2d-5pt": (2, 5, 1024), "2d-9pt": (2, 9, 1024), "3d-7pt": (3, 7, 101),
            "3d-27pt": (3, 27, 101)}


def galerkin(name, g=None, dtype=np.float64):
    """(A, P, R) of a Galerkin product R*A*P: the named stencil and
    unsmoothed 2^dim aggregation, at g points per side (default: the
    measured size)."""
    dim, points, g0 = GALERKIN[name]
    g = g0 if g is None else g
    return (stencil(g, dim, points, dtype), aggregation_p_grid(g, dim, dtype),
            aggregation_r_grid(g, dim, dtype))


def banded_csr(n, dmin, dmax, band_frac, rng, dtype) -> Csr:
    """Per-row degree uniform in {dmin..dmax}; distinct uniform columns in a
    window of width ceil(band_frac*n) centred on the diagonal, shifted to
    stay inside [0, n)."""
    w = int(math.ceil(band_frac * n))
    d = rng.integers(dmin, dmax + 1, n)
    i = np.arange(n, dtype=np.int64)
    lo = np.clip(i - w // 2, 0, n - w)
    rp, ci = distinct_columns(rng, d, n, lo=lo, width=w)
    return Csr(n, n, rp, ci, _values(rng, ci.size, "uniform", dtype))


# ---------------------------------------------------------------- workloads

def config1(n=2000, degree=10):
    """Workload 1: uniform A, C = A*A (binary64)."""
    A = uniform_csr(n, n, degree, workload=1)
    return A, A


def config2(n=200000, gamma=2.1, mean=16.0, cap=20000):
    """Workload 2: power-law A, C = A*A (binary64)."""
    A = powerlaw_csr(n, gamma, mean, cap, workload=2)
    return A, A


def config3(g=64):
    """Workload 3: (A, P, R) of the 27-point Galerkin product R*(A*P)."""
    return stencil27(g), aggregation_p(g), aggregation_r(g)


def config4_sizes(count=512, nmin=1024, nmax=65536):
    """Matrix sizes of workload 4 (log-uniform in [nmin, nmax])."""
    sizes = rng_for(4, 0)
    return np.exp(sizes.uniform(math.log(nmin), math.log(nmax), count)).round().astype(np.int64)


def config4(count=512, nmin=1024, nmax=65536, dmin=4, dmax=32, band=0.05, only=None):
    """Workload 4: list of (A_i, B_i); binary64 for even i, binary32 for odd i.
    ``only``: generate just these problem indices (same matrices as in the
    full batch)."""
    ns = config4_sizes(count, nmin, nmax)
    out = []
    for p in (range(count) if only is None else only):
        dt = np.float64 if p % 2 == 0 else np.float32
        rng = rng_for(4, 1, p)
        A = banded_csr(int(ns[p]), dmin, dmax, band, rng, dt)
        B = banded_csr(int(ns[p]), dmin, dmax, band, rng, dt)
        out.append((A, B))
    return out


def config5(n=500000, gamma=2.2, mean=20.0, ncols=4096, bdeg=32):
    """Workload 5: (A, B) of the differentiable product, binary32, N(0,1)."""
    A = powerlaw_csr(n, gamma, mean, n, workload=5, sub=0, dtype=np.float32, dist="normal")
    B = uniform_csr(n, ncols, bdeg, workload=5, sub=1, dtype=np.float32, dist="normal")
    return A, B


def config5_dc(nnz_c, dtype=np.float32):
    """Upstream gradient dC ~ N(0,1), one value per entry of C in CSR order."""
    return rng_for(5, 2).standard_normal(nnz_c).astype(dtype)


def crafted_rows(targets, n=4096, workload=9, dtype=np.float64, col_range=None,
                 empty_refs=0):
    """A and B such that row i of A*B has exactly ``targets[i]`` products.

    B holds 16 copies each of rows of length 2^p (p = 0..12, capped at
    ``col_range``) plus 16 empty rows; row i of A references B rows chosen
    greedily (longest first) so their lengths sum to its target, plus
    ``empty_refs`` references to empty B rows.  ``col_range`` limits B's columns to [0, col_range) to force
    duplicate columns in C's rows.  Returns (A, B).
    """
    rng = rng_for(workload, 0)
    cr = n if col_range is None else min(col_range, n)
    copies = 16
    lengths = []
    for p in range(13):
        lengths += [min(2 ** p, cr)] * copies
    lengths += [0] * copies
    lengths = np.array(lengths, dtype=np.int64)
    kb = lengths.size
    brp, bci = distinct_columns(rng, lengths, n, lo=np.zeros(kb, np.int64),
                                width=np.full(kb, cr, np.int64))
    B = Csr(kb, n, brp, bci, _values(rng, bci.size, "uniform", dtype))
    by_len = {}
    for j, L in enumerate(lengths.tolist()):
        by_len.setdefault(L, []).append(j)
    empty = by_len[0]
    rows = []
    for t in targets:
        t = int(t)
        refs = set()
        rem = t
        for L in sorted((x for x in by_len if x > 0), reverse=True):
            free = [j for j in by_len[L] if j not in refs]
            c = min(rem // L, len(free))
            if c:
                for j in rng.choice(free, size=c, replace=False).tolist():
                    refs.add(j)
                rem -= c * L
        if rem:
            raise ValueError("target %d cannot be composed from the crafted B rows" % t)
        for e in rng.choice(empty, size=min(empty_refs, len(empty)), replace=False).tolist():
            refs.add(e)
        rows.append(sorted(refs))
    counts = np.array([len(r) for r in rows], dtype=np.int64)
    aci = np.array([j for r in rows for j in r], dtype=np.int32)
    A = Csr(len(targets), kb, _row_ptr(counts), aci, _values(rng, aci.size, "uniform", dtype))
    return A, B
