"""Pins of the reference oracle against facts that do not come from the oracle
itself: the paper's worked example, dense brute force, identities, a
library SpGEMM, the closed form of the Galerkin stencil product, and the
stated bin table.  CPU only."""
import os

import numpy as np
import pytest

import oracle
import synthetic as S
from tests.helpers import (from_rows, identity, random_csr, read_golden, transpose,
                           csr_equal_structure)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def T(M):
    return M.as_tuple()


def test_paper_worked_example():
    g = read_golden(os.path.join(GOLD, "paper_example.txt"))
    C = oracle.spgemm(T(g["A"]), T(g["B"]))
    exp = g["C"]
    assert csr_equal_structure(C.row_ptr, C.col_idx, exp.row_ptr, exp.col_idx)
    assert np.array_equal(C.val, exp.val)
    assert C.u.tolist() == [4]


@pytest.mark.parametrize("seed", range(12))
def test_dense_bruteforce_exact(seed):
    """Small-integer values: every sum is exact, so the oracle must equal the
    dense matrix product (BLAS) exactly, and its pattern the boolean product."""
    rng = np.random.default_rng(1000 + seed)
    m, k, n = rng.integers(1, 25, 3)
    da, db = rng.uniform(0, 1, 2)
    A = random_csr(rng, m, k, da, ints=True)
    B = random_csr(rng, k, n, db, ints=True)
    C = oracle.spgemm(T(A), T(B))
    pat = (A.pattern_dense().astype(np.int64) @ B.pattern_dense().astype(np.int64)) > 0
    dense = A.to_dense() @ B.to_dense()
    r = np.repeat(np.arange(m), np.diff(C.row_ptr))
    got_pat = np.zeros((m, n), bool)
    got_pat[r, C.col_idx] = True
    assert np.array_equal(got_pat, pat)
    assert np.array_equal(C.val, dense[r, C.col_idx])
    # entries are sorted and unique per row
    for i in range(m):
        cols = C.col_idx[C.row_ptr[i]:C.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)


@pytest.mark.parametrize("seed", range(6))
def test_dense_bruteforce_float(seed):
    rng = np.random.default_rng(2000 + seed)
    m, k, n = rng.integers(1, 25, 3)
    A = random_csr(rng, m, k, 0.3)
    B = random_csr(rng, k, n, 0.3)
    C = oracle.spgemm(T(A), T(B))
    dense = A.to_dense() @ B.to_dense()
    absd = np.abs(A.to_dense()) @ np.abs(B.to_dense())
    r = np.repeat(np.arange(m), np.diff(C.row_ptr))
    err = np.abs(C.val - dense[r, C.col_idx])
    assert np.all(err <= 1e-14 * absd[r, C.col_idx] + 0.0)
    assert np.allclose(C.absval, absd[r, C.col_idx], rtol=1e-14, atol=0)


def test_cancellation_keeps_entries():
    """Section 3.1: no cancellation is considered, so an exact zero sum stays."""
    A = from_rows(1, 2, [(0, 0, 1.0), (0, 1, 1.0)])
    B = from_rows(2, 3, [(0, 1, 2.0), (1, 1, -2.0), (1, 2, 0.0)])
    C = oracle.spgemm(T(A), T(B))
    assert C.col_idx.tolist() == [1, 2]
    assert C.val.tolist() == [0.0, 0.0]
    assert C.u.tolist() == [3]


@pytest.mark.parametrize("seed", range(4))
def test_identity(seed):
    rng = np.random.default_rng(3000 + seed)
    A = random_csr(rng, 30, 40, 0.2)
    C1 = oracle.spgemm(T(A), T(identity(40)))
    C2 = oracle.spgemm(T(identity(30)), T(A))
    for C in (C1, C2):
        assert csr_equal_structure(C.row_ptr, C.col_idx, A.row_ptr, A.col_idx)
        assert np.array_equal(C.val, A.val)


@pytest.mark.parametrize("seed", range(4))
def test_transpose_identity(seed):
    """(AB)^T = B^T A^T, bit for bit: the same products, summed in the same
    ascending inner index."""
    rng = np.random.default_rng(4000 + seed)
    A = random_csr(rng, 35, 20, 0.25)
    B = random_csr(rng, 20, 28, 0.25)
    C = oracle.spgemm(T(A), T(B))
    Ct = oracle.spgemm(T(transpose(B)), T(transpose(A)))
    from synthetic import Csr
    CT = transpose(Csr(C.rows, C.cols, C.row_ptr.astype(np.int32), C.col_idx, C.val))
    assert csr_equal_structure(Ct.row_ptr, Ct.col_idx, CT.row_ptr, CT.col_idx)
    assert np.array_equal(Ct.val, CT.val)


def test_scipy_agrees():
    sp = pytest.importorskip("scipy.sparse")
    A, _ = S.config2(n=3000, cap=300)
    C = oracle.spgemm(T(A), T(A))
    sa = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.rows, A.cols))
    sc = (sa @ sa).tocsr()
    sc.sort_indices()
    assert csr_equal_structure(C.row_ptr, C.col_idx, sc.indptr, sc.indices)
    assert np.max(np.abs(C.val - sc.data) / C.absval) < 1e-15


def test_nnz_bounds_and_flops():
    A, _ = S.config2(n=5000, cap=500)
    C = oracle.spgemm(T(A), T(A))
    u_ref, tot = oracle.upper_bound(T(A), T(A))
    assert np.array_equal(C.u, u_ref)
    assert C.flops == 2 * tot
    assert C.nnz <= tot
    rownnz = np.diff(C.row_ptr)
    assert np.all(rownnz <= np.minimum(C.u, A.cols))


def test_upper_bound_closed_forms():
    A, _ = S.config1()
    u, tot = oracle.upper_bound(T(A), T(A))
    assert np.all(u == 100) and tot == 200000
    A5, B5 = S.config5(n=3000, ncols=512)
    u5, _ = oracle.upper_bound(T(A5), T(B5))
    assert np.array_equal(u5, 32 * np.diff(A5.row_ptr).astype(np.int64))
    targets = [0, 1, 2, 31, 32, 33, 64, 65, 128, 129, 256, 257, 512, 513, 4097, 20000]
    Ac, Bc = S.crafted_rows(targets, empty_refs=2)
    uc, _ = oracle.upper_bound(T(Ac), T(Bc))
    assert uc.tolist() == targets


def test_bin_table_matches_prose():
    rows = np.loadtxt(os.path.join(GOLD, "bin_table.txt"), dtype=np.int64, comments="#")
    b, h, tot = oracle.bins(rows[:, 0])
    assert b.tolist() == rows[:, 1].tolist()
    assert h.tolist() == rows[:, 2].tolist()
    assert tot == int(rows[:, 2].sum())


def test_bins_partition_invariants():
    u = np.arange(0, 3000, dtype=np.int64)
    b, h, _ = oracle.bins(u)
    assert np.all(np.diff(b) >= 0)              # monotone in u
    assert set(b.tolist()) == set(range(38))    # 38 bins, all reachable
    assert np.all(h[u <= 512] == u[u <= 512])
    assert np.all(h[u > 512] == 256)


def _stencil_closed_form_ap(g):
    """(A*P)_{fJ} from grid geometry: per dimension, c = number of the two fine
    coordinates of block X_d that lie within distance 1 of x_d; the entry is
    27*[J is f's own block] - prod_d c_d (A = 27*I - [neighbour incl. self])."""
    x = np.arange(g ** 3) % g
    y = (np.arange(g ** 3) // g) % g
    z = np.arange(g ** 3) // (g * g)
    h = g // 2
    entries_r, entries_c, entries_v = [], [], []
    for dZ in (-1, 0, 1):
        for dY in (-1, 0, 1):
            for dX in (-1, 0, 1):
                X, Y, Z = x // 2 + dX, y // 2 + dY, z // 2 + dZ
                ok = (X >= 0) & (X < h) & (Y >= 0) & (Y < h) & (Z >= 0) & (Z < h)
                cnt = np.ones(g ** 3, dtype=np.int64)
                for a, B in ((x, X), (y, Y), (z, Z)):
                    c = np.zeros(g ** 3, dtype=np.int64)
                    for off in (0, 1):
                        q = 2 * B + off
                        c += (np.abs(q - a) <= 1) & (q >= 0) & (q < g)
                    cnt *= c
                ok &= cnt > 0
                own = (dX == 0) & (dY == 0) & (dZ == 0)
                val = (27 if own else 0) - cnt
                r = np.nonzero(ok)[0]
                entries_r.append(r)
                entries_c.append((X + h * (Y + h * Z))[r])
                entries_v.append(val[r])
    r = np.concatenate(entries_r)
    c = np.concatenate(entries_c)
    v = np.concatenate(entries_v).astype(np.float64)
    o = np.lexsort((c, r))
    return r[o], c[o], v[o]


def _stencil_closed_form_rap(g):
    """(R*A*P)_{IK} = 216*[I=K] - prod_d N_d with N_d = 4 for the same block
    and 1 for adjacent blocks (pairs of fine coordinates at distance <= 1)."""
    h = g // 2
    I = np.arange(h ** 3)
    X, Y, Z = I % h, (I // h) % h, I // (h * h)
    rs, cs, vs = [], [], []
    for dZ in (-1, 0, 1):
        for dY in (-1, 0, 1):
            for dX in (-1, 0, 1):
                K = (X + dX, Y + dY, Z + dZ)
                ok = np.ones(h ** 3, bool)
                prod = np.ones(h ** 3, np.int64)
                for Kd, d in zip(K, (dX, dY, dZ)):
                    ok &= (Kd >= 0) & (Kd < h)
                    prod *= 4 if d == 0 else 1
                val = (216 if (dX, dY, dZ) == (0, 0, 0) else 0) - prod
                r = np.nonzero(ok)[0]
                rs.append(r)
                cs.append((K[0] + h * (K[1] + h * K[2]))[r])
                vs.append(val[r])
    r = np.concatenate(rs)
    c = np.concatenate(cs)
    v = np.concatenate(vs).astype(np.float64)
    o = np.lexsort((c, r))
    return r[o], c[o], v[o]


@pytest.mark.parametrize("g", [4, 8, 16])
def test_galerkin_closed_form(g):
    A, P, R = S.config3(g)
    AP = oracle.spgemm(T(A), T(P))
    r, c, v = _stencil_closed_form_ap(g)
    assert AP.nnz == r.size == (2 * g - 2) ** 3
    assert np.array_equal(np.repeat(np.arange(AP.rows), np.diff(AP.row_ptr)), r)
    assert np.array_equal(AP.col_idx, c)
    assert np.array_equal(AP.val, v)
    from synthetic import Csr
    APc = Csr(AP.rows, AP.cols, AP.row_ptr.astype(np.int32), AP.col_idx, AP.val)
    RAP = oracle.spgemm(T(R), T(APc))
    r2, c2, v2 = _stencil_closed_form_rap(g)
    assert np.array_equal(np.repeat(np.arange(RAP.rows), np.diff(RAP.row_ptr)), r2)
    assert np.array_equal(RAP.col_idx, c2)
    assert np.array_equal(RAP.val, v2)
    h = g // 2
    assert RAP.nnz == (3 * h - 2) ** 3
    # interior rows sum to zero (the aggregated operator annihilates constants)
    s = np.add.reduceat(RAP.val, RAP.row_ptr[:-1]) if RAP.nnz else []
    interior = [X + h * (Y + h * Z) for Z in range(1, h - 1) for Y in range(1, h - 1)
                for X in range(1, h - 1)]
    assert np.all(np.asarray(s)[interior] == 0)


@pytest.mark.slow
def test_galerkin_closed_form_full():
    """Workload 3 at full size: nnz(AP) = 126^3, nnz(RAP) = 94^3, products
    190^3 and 2000376 (Algorithm 2 sums)."""
    A, P, R = S.config3(64)
    AP = oracle.spgemm(T(A), T(P))
    assert AP.nnz == 126 ** 3 and int(AP.u.sum()) == 190 ** 3
    r, c, v = _stencil_closed_form_ap(64)
    assert np.array_equal(AP.col_idx, c) and np.array_equal(AP.val, v)
    from synthetic import Csr
    APc = Csr(AP.rows, AP.cols, AP.row_ptr.astype(np.int32), AP.col_idx, AP.val)
    RAP = oracle.spgemm(T(R), T(APc))
    assert RAP.nnz == 94 ** 3 and int(RAP.u.sum()) == 126 ** 3
    r2, c2, v2 = _stencil_closed_form_rap(64)
    assert np.array_equal(RAP.col_idx, c2) and np.array_equal(RAP.val, v2)


def _coarse_interior(dim, points):
    """Row of R*A*P for an aggregate whose neighbouring aggregates are all
    full 2^dim blocks, as {offset: value}, derived by hand.  Entry (I, J) is
    the sum of a_ij over fine i in I and j in J.  For the full stencil
    (3^dim points) the coupled fine pairs factor over the dimensions: along
    one axis a 2-block couples to itself through 4 ordered pairs and to a
    neighbouring block through 1, so J at offset D != 0 gets -prod_k c(D_k)
    with c(0) = 4, c(+-1) = 1, and the diagonal is 2^dim (3^dim - 1) minus the
    4^dim - 2^dim coupled pairs of distinct points inside the block.  For the
    axis stencil (2 dim + 1 points) only blocks at a unit axis offset couple,
    through the 2^(dim-1) fine edges that cross the shared face; the diagonal
    is 2^dim * 2 dim minus the dim * 2^dim ordered edges inside the block."""
    import itertools
    out = {}
    for off in itertools.product((-1, 0, 1), repeat=dim):
        nz = sum(abs(o) for o in off)
        if points == 3 ** dim:
            if nz == 0:
                out[off] = 2 ** dim * (3 ** dim - 1) - (4 ** dim - 2 ** dim)
            else:
                out[off] = -int(np.prod([1 if o else 4 for o in off]))
        else:
            if nz == 0:
                out[off] = dim * 2 ** dim
            elif nz == 1:
                out[off] = -(2 ** (dim - 1))
    return out


GALERKIN_SMALL = [("2d-5pt", 8), ("2d-5pt", 9), ("2d-9pt", 8), ("2d-9pt", 11),
                  ("3d-7pt", 6), ("3d-7pt", 7), ("3d-27pt", 6), ("3d-27pt", 9)]


@pytest.mark.parametrize("name,g", GALERKIN_SMALL)
def test_galerkin_variants(name, g):
    """Both multiplication orders of R*A*P for every stencil of the
    multigrid experiment (odd g leaves one-point aggregates on the far
    faces): equal bit for bit (small integers, every sum exact), equal to
    the dense triple product, and interior rows equal to the hand-derived
    coarse stencil."""
    import itertools
    from synthetic import Csr
    dim, points, _ = S.GALERKIN[name]
    A, P, R = S.galerkin(name, g)
    AP = oracle.spgemm(T(A), T(P))
    RAP1 = oracle.spgemm(T(R), (AP.rows, AP.cols, AP.row_ptr.astype(np.int32), AP.col_idx, AP.val))
    RA = oracle.spgemm(T(R), T(A))
    RAP2 = oracle.spgemm((RA.rows, RA.cols, RA.row_ptr.astype(np.int32), RA.col_idx, RA.val), T(P))
    assert np.array_equal(RAP1.row_ptr, RAP2.row_ptr)
    assert np.array_equal(RAP1.col_idx, RAP2.col_idx)
    assert np.array_equal(RAP1.val, RAP2.val)
    # dense triple product (BLAS) and the boolean pattern product
    dense = R.to_dense() @ A.to_dense() @ P.to_dense()
    pat = (R.pattern_dense().astype(np.int64) @ A.pattern_dense().astype(np.int64)
           @ P.pattern_dense().astype(np.int64)) > 0
    C = Csr(RAP1.rows, RAP1.cols, RAP1.row_ptr, RAP1.col_idx, RAP1.val)
    assert np.array_equal(C.pattern_dense(), pat)
    assert np.array_equal(C.to_dense(), dense)
    # interior aggregates: X in [1, (g - 3) // 2] along every axis
    h = (g + 1) // 2
    want = _coarse_interior(dim, points)
    inner = range(1, (g - 3) // 2 + 1)
    count = 0
    for X in itertools.product(inner, repeat=dim):
        I = sum(X[k] * h ** k for k in range(dim))
        a, b = RAP1.row_ptr[I], RAP1.row_ptr[I + 1]
        got = {}
        for c, v in zip(RAP1.col_idx[a:b], RAP1.val[a:b]):
            off = tuple(int((c // h ** k) % h) - X[k] for k in range(dim))
            got[off] = v
        assert got == want, (I, got)
        assert sum(got.values()) == 0
        count += 1
    assert count > 0


def test_stencil_generator_matches_27_point():
    """The general generator reproduces workload 3's matrices exactly."""
    A, P, R = S.galerkin("3d-27pt", 8)
    for X, Y in ((A, S.stencil27(8)), (P, S.aggregation_p(8)), (R, S.aggregation_r(8))):
        assert np.array_equal(X.row_ptr, Y.row_ptr)
        assert np.array_equal(X.col_idx, Y.col_idx)
        assert np.array_equal(X.val, Y.val)


@pytest.mark.parametrize("seed", range(4))
def test_f32_accumulator(seed):
    """The binary32 variant stays within the binary32 dot-product bound of the
    binary64 result, and equals a binary32 dense sum for single-term entries."""
    rng = np.random.default_rng(5000 + seed)
    A = random_csr(rng, 40, 30, 0.3, dtype=np.float32)
    B = random_csr(rng, 30, 50, 0.3, dtype=np.float32)
    C64 = oracle.spgemm(T(A.astype(np.float64)), T(B.astype(np.float64)))
    C32 = oracle.spgemm(T(A), T(B), acc32=True)
    assert np.array_equal(C32.col_idx, C64.col_idx)
    k = 30
    assert np.all(np.abs(C32.val.astype(np.float64) - C64.val) <= (k + 1) * 2.0 ** -23 * C64.absval)
    ones = (np.asarray(C32.val, np.float64) != 0)
    assert ones.any()


@pytest.mark.parametrize("seed", range(6))
def test_gradient_dense_exact(seed):
    """dA = (dC B^T) on S(A), dB = (A^T dC) on S(B), with integer values so the
    dense products are exact."""
    rng = np.random.default_rng(6000 + seed)
    m, k, n = rng.integers(1, 20, 3)
    A = random_csr(rng, m, k, 0.4, ints=True)
    B = random_csr(rng, k, n, 0.4, ints=True)
    C = oracle.spgemm(T(A), T(B))
    dc = rng.integers(-3, 4, C.nnz).astype(np.float64)
    dA, dB = oracle.grad(T(A), T(B), C.row_ptr, C.col_idx, dc)
    dC = np.zeros((m, n))
    r = np.repeat(np.arange(m), np.diff(C.row_ptr))
    dC[r, C.col_idx] = dc
    gA = dC @ B.to_dense().T
    gB = A.to_dense().T @ dC
    ra = np.repeat(np.arange(m), np.diff(A.row_ptr))
    rb = np.repeat(np.arange(k), np.diff(B.row_ptr))
    assert np.array_equal(dA, gA[ra, A.col_idx])
    assert np.array_equal(dB, gB[rb, B.col_idx])


def test_gradient_finite_difference():
    """L = <dC, A*B> is bilinear, so a central difference with h = 1 equals the
    gradient up to rounding."""
    rng = np.random.default_rng(7000)
    A = random_csr(rng, 15, 12, 0.4)
    B = random_csr(rng, 12, 18, 0.4)
    C = oracle.spgemm(T(A), T(B))
    dc = rng.standard_normal(C.nnz)
    dA, dB = oracle.grad(T(A), T(B), C.row_ptr, C.col_idx, dc)

    def L(Am, Bm):
        R = oracle.spgemm(T(Am), T(Bm))
        assert np.array_equal(R.col_idx, C.col_idx)
        return float(np.dot(dc, R.val))

    from synthetic import Csr
    for p in range(A.nnz):
        vp, vm = A.val.copy(), A.val.copy()
        vp[p] += 1.0
        vm[p] -= 1.0
        fd = (L(Csr(A.rows, A.cols, A.row_ptr, A.col_idx, vp), B)
              - L(Csr(A.rows, A.cols, A.row_ptr, A.col_idx, vm), B)) / 2
        assert abs(fd - dA[p]) <= 1e-12 * (1 + abs(dA[p]))
    for q in range(B.nnz):
        vp, vm = B.val.copy(), B.val.copy()
        vp[q] += 1.0
        vm[q] -= 1.0
        fd = (L(A, Csr(B.rows, B.cols, B.row_ptr, B.col_idx, vp))
              - L(A, Csr(B.rows, B.cols, B.row_ptr, B.col_idx, vm))) / 2
        assert abs(fd - dB[q]) <= 1e-12 * (1 + abs(dB[q]))


def test_gradient_sampled_matches_full():
    A, B = S.config5(n=2000, ncols=256)
    C = oracle.spgemm(T(A), T(B))
    dc = S.config5_dc(C.nnz)
    dA, dB = oracle.grad(T(A), T(B), C.row_ptr, C.col_idx, dc)
    sa = np.array([0, 5, A.nnz - 1, 17])
    sb = np.array([3, B.nnz - 1, 0])
    dA2, dB2 = oracle.grad(T(A), T(B), C.row_ptr, C.col_idx, dc, sample_a=sa, sample_b=sb)
    assert np.array_equal(dA2[sa], dA[sa]) and np.array_equal(dB2[sb], dB[sb])


def test_degenerate_shapes():
    for m, k, n in [(0, 5, 5), (5, 0, 5), (5, 5, 0), (0, 0, 0)]:
        A = random_csr(np.random.default_rng(0), m, k, 0.5)
        B = random_csr(np.random.default_rng(1), k, n, 0.5)
        C = oracle.spgemm(T(A), T(B))
        assert C.nnz == 0 and C.row_ptr.tolist() == [0] * (m + 1)


def test_planted_mistakes_are_caught():
    """A dropped term, a wrong sign or a transposed operand in the oracle's
    output is detected by the dense brute-force pin."""
    rng = np.random.default_rng(8000)
    A = random_csr(rng, 12, 10, 0.5, ints=True)
    B = random_csr(rng, 10, 14, 0.5, ints=True)
    C = oracle.spgemm(T(A), T(B))
    dense = A.to_dense() @ B.to_dense()
    r = np.repeat(np.arange(12), np.diff(C.row_ptr))
    assert np.array_equal(C.val, dense[r, C.col_idx])
    # dropped term: remove the contribution of the first product of row 0
    i = int(np.nonzero(np.diff(A.row_ptr))[0][0])
    j = A.col_idx[A.row_ptr[i]]
    kcol = B.col_idx[B.row_ptr[j]] if B.row_ptr[j + 1] > B.row_ptr[j] else None
    if kcol is not None:
        bad = C.val.copy()
        pos = C.row_ptr[i] + np.searchsorted(C.col_idx[C.row_ptr[i]:C.row_ptr[i + 1]], kcol)
        bad[pos] -= A.val[A.row_ptr[i]] * B.val[B.row_ptr[j]]
        if A.val[A.row_ptr[i]] * B.val[B.row_ptr[j]] != 0:
            assert not np.array_equal(bad, dense[r, C.col_idx])
    # transposed operand: B^T in place of B (square case)
    Bs = random_csr(rng, 10, 10, 0.5, ints=True)
    C1 = oracle.spgemm(T(A), T(Bs))
    C2 = oracle.spgemm(T(A), T(transpose(Bs)))
    dense1 = A.to_dense() @ Bs.to_dense()
    r2 = np.repeat(np.arange(12), np.diff(C2.row_ptr))
    assert np.array_equal(C1.val, dense1[np.repeat(np.arange(12), np.diff(C1.row_ptr)), C1.col_idx])
    assert not (np.array_equal(C2.col_idx, C1.col_idx) and np.array_equal(C2.val, dense1[r2, C2.col_idx]))


def _merge_two_pointer(a, b, av, bv):
    """Textbook merge of two ascending lists, the first list winning ties."""
    i = j = 0
    ok, ov = [], []
    while i < len(a) or j < len(b):
        if j >= len(b) or (i < len(a) and a[i] <= b[j]):
            ok.append(a[i]); ov.append(av[i]); i += 1
        else:
            ok.append(b[j]); ov.append(bv[j]); j += 1
    return ok, ov


@pytest.mark.parametrize("l", [1, 2, 3, 8, 33])
def test_merge_pairs_two_pointer(l):
    """The oracle's merge equals a two-pointer merge, ties included (keys
    drawn from a handful of values), pair by pair."""
    rng = np.random.default_rng(600 + l)
    pairs = 7
    k = rng.integers(0, 4, (pairs, 2 * l)).astype(np.uint32)
    k[:, :l].sort(axis=1)
    k[:, l:].sort(axis=1)
    v = np.arange(k.size, dtype=np.int64).reshape(pairs, 2 * l)
    ko, vo = oracle.merge_pairs(k.reshape(-1), v.reshape(-1), l)
    for p in range(pairs):
        ek, ev = _merge_two_pointer(list(k[p, :l]), list(k[p, l:]), list(v[p, :l]), list(v[p, l:]))
        assert ko[p * 2 * l:(p + 1) * 2 * l].tolist() == ek
        assert vo[p * 2 * l:(p + 1) * 2 * l].tolist() == ev


def test_merge_pairs_worked_example():
    """A hand-merged pair: ties keep the first run's entry first."""
    k = np.array([1, 4, 4, 9, 0, 4, 5, 9], np.uint32)
    v = np.array([10, 11, 12, 13, 20, 21, 22, 23])
    ko, vo = oracle.merge_pairs(k, v, 4)
    assert ko.tolist() == [0, 1, 4, 4, 4, 5, 9, 9]
    assert vo.tolist() == [20, 10, 11, 12, 21, 22, 13, 23]


def _golden_rounding():
    g = read_golden(os.path.join(GOLD, "binary32_rounding.txt"))
    return g["A"], g["B"], g["C32"], g["C64"]


def test_f32_accumulator_sequential_rounding():
    """Per-step binary32 rounding in ascending j (hand-worked fixture): ties
    to even at every addition, products rounded before they are added."""
    A, B, C32, C64 = _golden_rounding()
    r32 = oracle.spgemm(T(A.astype(np.float32)), T(B.astype(np.float32)), acc32=True)
    assert r32.val.dtype == np.float32
    assert csr_equal_structure(r32.row_ptr, r32.col_idx, C32.row_ptr, C32.col_idx)
    assert np.array_equal(r32.val, C32.val.astype(np.float32))
    r64 = oracle.spgemm(T(A), T(B))
    assert np.array_equal(r64.val, C64.val)


def _round_f32(x):
    """Round an exact rational to binary32, nearest, ties to even."""
    from fractions import Fraction
    c = np.float32(float(x))
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - x)
        key = (d, int(np.float32(cand).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return np.float32(best[1])


def test_f32_rounding_fixture_rejects_planted_variants():
    """Plausible wrong binary32 accumulators fail the fixture: summing in
    binary64 and rounding once, adding in descending j, or fusing each
    multiply with its add (one rounding)."""
    from fractions import Fraction
    A, B, C32, _ = _golden_rounding()
    f = np.float32
    want = list(C32.val.astype(np.float32))

    def row_terms(i):
        out = []
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = A.col_idx[p]
            for q in range(B.row_ptr[j], B.row_ptr[j + 1]):
                out.append((f(A.val[p]), f(B.val[q])))
        return out

    def sequential(i):
        s = f(0.0)
        for a, b in row_terms(i):
            s = f(s + f(a * b))
        return s

    def acc64_round_once(i):
        s = 0.0
        for a, b in row_terms(i):
            s += float(f(a * b))
        return f(s)

    def descending(i):
        s = f(0.0)
        for a, b in reversed(row_terms(i)):
            s = f(s + f(a * b))
        return s

    def fused(i):
        s = f(0.0)
        for a, b in row_terms(i):
            s = _round_f32(Fraction(float(s)) + Fraction(float(a)) * Fraction(float(b)))
        return s

    assert [sequential(i) for i in range(3)] == want
    for bad, row in ((acc64_round_once, 0), (descending, 1), (fused, 2)):
        assert bad(row) != want[row], bad.__name__


def _fake_ref(val, absval):
    return oracle.OracleResult(1, len(val), np.array([0, len(val)], np.int64),
                               np.arange(len(val), dtype=np.int32), np.asarray(val, np.float64),
                               np.asarray(absval, np.float64), np.array([len(val)], np.int64))


def test_value_error_known_answers():
    """The componentwise metric |c - c*| / (|A||B|)_ik on hand-made cases:
    a known scaled error, an entry whose exact sum cancels to zero (scaled
    by its magnitude sum, left out of the plain relative error), and entries
    whose magnitude sum is zero (must be exactly zero, else infinite)."""
    # c* = [1, 2, 0 (cancelled: +1 - 1), 0 (all products zero)]
    ref = _fake_ref([1.0, 2.0, 0.0, 0.0], [2.0, 4.0, 2.0, 0.0])
    scaled, plain = oracle.value_error([1.0 + 1e-3, 2.0, 0.0, 0.0], ref)
    assert scaled == pytest.approx(5e-4, rel=1e-12)
    assert plain == pytest.approx(1e-3, rel=1e-9)
    # an error on the cancelled entry is scaled by its magnitude sum 2
    scaled, plain = oracle.value_error([1.0, 2.0, 1e-15, 0.0], ref)
    assert scaled == pytest.approx(5e-16, rel=1e-12)
    assert plain == 0.0
    # a nonzero value where every product is zero
    scaled, plain = oracle.value_error([1.0, 2.0, 0.0, 1e-300], ref)
    assert scaled == float("inf") and plain == float("inf")
    # exact agreement
    assert oracle.value_error([1.0, 2.0, 0.0, 0.0], ref) == (0.0, 0.0)


def test_value_error_rejects_planted_metrics():
    """Scaling by |c*| instead of the magnitude sum, or dropping the
    zero-magnitude rule, gives a different answer than the metric on the
    fixture's cancelled and all-zero entries."""
    ref = _fake_ref([1.0, 0.0, 0.0], [2.0, 2.0, 0.0])
    good = [1.0, 1e-15, 0.0]       # error only on the cancelled entry
    bad = [1.0, 1e-15, 1e-300]     # and a value where every product is zero
    assert oracle.value_error(good, ref)[0] == pytest.approx(5e-16, rel=1e-12, abs=0)
    assert oracle.value_error(bad, ref)[0] == float("inf")
    d_good = np.abs(np.asarray(good) - ref.val)
    d_bad = np.abs(np.asarray(bad) - ref.val)
    # planted: scaled by |c*| (the cancelled entry has c* = 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        by_value = float(np.max(d_good / np.abs(ref.val)))
    assert by_value != pytest.approx(5e-16, rel=1e-6, abs=0)
    # planted: zero-magnitude entries skipped instead of required to be 0
    keep = ref.absval > 0
    no_zero_rule = float(np.max(d_bad[keep] / ref.absval[keep]))
    assert no_zero_rule != float("inf")
