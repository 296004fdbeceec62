"""Parity of the HIP path (through the C ABI) with the oracle.

Structure (row_ptr, col_idx) must match bit for bit; values within the
componentwise bound |c - c*| <= tol * (|A||B|)_ik with tol = 1e-12 (binary64)
and 1e-5 (binary32).  Rows that are neither split nor spilled are summed in
the oracle's order, so their values must match exactly; the tests check
exact equality wherever that holds.
"""
import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu

TOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}


def _run(A, B, **opts):
    import torch
    from paper_1504_05022_amd import CsrMatrix, Plan
    dA = CsrMatrix.from_host(A)
    dB = dA if B is A else CsrMatrix.from_host(B)
    plan = Plan(dA, dB, **opts)
    C = plan.compute()
    torch.cuda.synchronize()
    info = plan.info
    plan.close()
    return C, info


def check(A, B, exact=True, **opts):
    """Run the GPU path and compare with the oracle.  Returns (C host tuple, info)."""
    print("case: A %dx%d nnz %d, B %dx%d nnz %d, %s, opts %s" %
          (A.rows, A.cols, A.nnz, B.rows, B.cols, B.nnz, A.val.dtype, opts), flush=True)
    C, info = _run(A, B, **opts)
    _, _, rp, ci, v = C.to_host()
    ref = oracle.spgemm(A.astype(np.float64).as_tuple(), B.astype(np.float64).as_tuple())
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr), "row_ptr differs"
    assert np.array_equal(ci, ref.col_idx), "col_idx differs"
    assert info.nnz_c == ref.nnz
    assert info.flops == ref.flops
    assert info.nnz_hat == int(ref.u.sum())
    if "bin_edges" not in opts and "long_slot" not in opts:
        # Algorithm 3 with the paper's thresholds: bins and the size of C~
        b, _, nnz_tilde = oracle.bins(ref.u)
        assert list(info.bin_count) == np.bincount(b, minlength=38).tolist()
        assert info.nnz_tilde == nnz_tilde
    err, rel = oracle.value_error(v, ref)
    print("  nnz(C) %d, flops %d, max scaled err %.3g, max rel err %.3g" %
          (ref.nnz, ref.flops, err, rel), flush=True)
    assert err <= TOL[np.dtype(A.val.dtype)]
    if exact:
        u = ref.u
        seg = opts.get("seg", 0)
        lp = opts.get("long_path", 0)
        dense_w = 2048 if A.val.dtype == np.float64 else 4096
        if not seg and (lp == 2 or (lp == 0 and B.cols <= dense_w)):
            # column windows (chosen automatically when B has at most
            # dense_w columns): every row in Gustavson's order, except rows
            # of more than 16384 products into one dense window of columns
            # (product ranges added in range order)
            ok_rows = ~((B.cols <= dense_w) & (u > 16384))
        else:
            # rows summed in the oracle's order: not split into segments and
            # not spilling out of the level-1 sequence
            l1cap = opts.get("l1_cap") or (5120 if A.val.dtype == np.float64 else 7168)
            segp = np.inf if seg is not None and seg < 0 else (seg or 1024)
            ok_rows = (u <= segp) & (np.minimum(u, B.cols) <= l1cap - 1024)
        mask = np.repeat(ok_rows, np.diff(ref.row_ptr))
        if A.val.dtype == np.float64:
            assert np.array_equal(v[mask], ref.val[mask]), "binary64 values differ from sequential sums"
        else:
            r32 = oracle.spgemm(A.as_tuple(), B.as_tuple(), acc32=True)
            assert np.array_equal(v[mask], r32.val[mask]), "binary32 values differ from sequential sums"
    return (rp, ci, v), info


EDGE_U = [0, 1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255,
          256, 257, 511, 512, 513, 1000, 1023, 1024, 1025, 2048, 4097]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("col_range", [None, 40, 700])
def test_bin_edges(dtype, col_range):
    targets = [t for t in EDGE_U if col_range is None or t <= 16 * 1024]
    A, B = S.crafted_rows(targets * 3, col_range=col_range, empty_refs=2, dtype=dtype)
    _, info = check(A, B)
    b, _, _ = oracle.bins(np.array(targets * 3))
    assert list(info.bin_count) == np.bincount(b, minlength=38).tolist()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("col_range", [None, 6])
@pytest.mark.parametrize("edge0", [32, 16])
def test_tiny_rows_heap_method(dtype, col_range, edge0):
    """The paper's heap method for bin group 3 (one thread per row, one
    kernel per exact size): structure bit for bit, values within tolerance
    (duplicates are added in heap order); few distinct columns exercise the
    fusing step; every other bin is unchanged."""
    targets = list(range(0, 40)) + ([100, 700, 3000] if col_range is None else [60])
    A, B = S.crafted_rows(targets * 20, col_range=col_range, empty_refs=1, dtype=dtype)
    edges = (edge0, 64, 128, 256, 512)
    (rp0, ci0, v0), i0 = check(A, B, exact=False, bin_edges=edges)
    (rp1, ci1, v1), i1 = check(A, B, exact=False, bin_edges=edges, tiny_heap=1)
    assert np.array_equal(rp0, rp1) and np.array_equal(ci0, ci1)
    assert list(i0.bin_count) == list(i1.bin_count)
    # rows outside bin group 3 are computed exactly as before
    c = oracle.spgemm(A.astype(np.float64).as_tuple(), B.astype(np.float64).as_tuple())
    keep = np.repeat((c.u < 2) | (c.u > edge0), np.diff(c.row_ptr))
    assert np.array_equal(v0[keep], v1[keep])


def test_tiny_rows_heap_method_scaled():
    A, _ = S.config2(n=20000, cap=400)
    check(A, A, exact=False, tiny_heap=1)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_long_rows_that_spill(dtype):
    """Results longer than the LDS level-1 sequence: spills into growing pool
    blocks (values then within tolerance, structure exact)."""
    A, B = S.crafted_rows([20000, 9000, 70000, 513, 30000], n=60000, dtype=dtype)
    check(A, B, exact=False)


def test_config1_full():
    A, _ = S.config1()
    check(A, A)


@pytest.mark.parametrize("n,cap", [(3000, 300), (20000, 2000), (50000, 20000)])
def test_config2_scaled(n, cap):
    A, _ = S.config2(n=n, cap=cap)
    check(A, A, exact=False)


def test_config3_chain_full():
    """Both products of the Galerkin chain, checked against the oracle and,
    through it, against the closed form."""
    from synthetic import Csr
    A, P, R = S.config3(64)
    (rp, ci, v), _ = check(A, P)
    AP = Csr(A.rows, P.cols, rp, ci, v)
    check(R, AP)


def _galerkin_orders(name, g, dtype):
    """R*(A*P) and (R*A)*P on the GPU, every product checked against the
    oracle; the two orders must agree bit for bit (small-integer values make
    every sum exact)."""
    from synthetic import Csr
    A, P, R = S.galerkin(name, g, dtype)
    (rp, ci, v), _ = check(A, P)
    (rp1, ci1, v1), _ = check(R, Csr(A.rows, P.cols, rp, ci, v))
    (rp, ci, v), _ = check(R, A)
    (rp2, ci2, v2), _ = check(Csr(R.rows, A.cols, rp, ci, v), P)
    assert np.array_equal(rp1, rp2) and np.array_equal(ci1, ci2) and np.array_equal(v1, v2)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("name,g", [("2d-5pt", 301), ("2d-9pt", 256), ("3d-7pt", 33),
                                    ("3d-27pt", 30)])
def test_galerkin_orders(name, g, dtype):
    _galerkin_orders(name, g, dtype)


@pytest.mark.parametrize("name", ["2d-5pt", "2d-9pt", "3d-7pt", "3d-27pt"])
def test_galerkin_orders_full(name):
    """The multigrid experiment's sizes (1024^2 and 101^3 grids)."""
    _galerkin_orders(name, None, np.float64)


@pytest.mark.parametrize("n", [2000, 20000])
def test_config5_scaled_f32(n):
    A, B = S.config5(n=n, ncols=512)
    check(A, B)


def test_config4_sample():
    probs = S.config4(count=6, nmax=8192)
    for A, B in probs:
        check(A, B)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_wide_column_space(dtype):
    """2^27 columns: the sort keys of the short-row kernels, of the long-row
    segments and of the column ranges of rows with up to about 2000 products
    need more than 32 bits (the 64-bit key variants of every kernel)."""
    A = S.powerlaw_csr(3000, 2.1, 16.0, 600, workload=11, dtype=dtype)
    B = S.uniform_csr(3000, 1 << 27, 24, workload=11, sub=1, dtype=dtype)
    check(A, B)


def test_degenerate_shapes():
    from tests.helpers import random_csr
    rng = np.random.default_rng(5)
    for m, k, n in [(0, 5, 7), (6, 0, 7), (6, 5, 0), (0, 0, 0), (1, 1, 1)]:
        A = random_csr(rng, m, k, 0.5)
        B = random_csr(rng, k, n, 0.5)
        if A.nnz == 0 and B.nnz == 0 and m * k * n > 0:
            continue
        check(A, B)
    # rows that reference only empty rows of B, and an all-empty product
    A, B = S.crafted_rows([0, 0, 5, 0], empty_refs=4)
    check(A, B)


def test_zero_products_and_signed_zeros():
    """Explicit zeros are stored entries; a single product -0.0 must come out
    as +0.0 (the sum starts from +0.0)."""
    from tests.helpers import from_rows
    A = from_rows(3, 3, [(0, 0, -1.0), (0, 1, 0.0), (1, 2, 2.0), (2, 0, 0.0)])
    B = from_rows(3, 4, [(0, 0, 0.0), (0, 3, 1.0), (1, 0, -3.0), (2, 1, -0.0), (2, 2, 5.0)])
    (rp, ci, v), _ = check(A, B)
    assert np.all(np.signbit(v) == np.signbit(oracle.spgemm(A.as_tuple(), B.as_tuple()).val))


def test_pool_exhaustion_relaunch():
    """A pool far too small forces the checkpoint / 2x growth / relaunch path
    (segments longer than one tile go through the level-1 merge method, which
    spills into pool blocks); the result must not change."""
    A, B = S.crafted_rows([20000, 9000, 3000, 700, 40000, 600], n=60000)
    (rp0, ci0, v0), i0 = check(A, B, exact=False, seg=8192)
    (rp1, ci1, v1), i1 = check(A, B, exact=False, seg=8192, pool_entries=300)
    assert i1.realloc_rounds > 0
    assert np.array_equal(ci0, ci1) and np.array_equal(v0, v1)


@pytest.mark.parametrize("seg", [1024, 2048, 4096, -1])
def test_long_row_splitting(seg):
    """Rows cut into product segments (phase 1) and combined per column range
    (phase 2), or never cut (seg = -1, L1 spills into growing pool blocks):
    identical structure, values within tolerance."""
    A, B = S.crafted_rows([20000, 9000, 70000, 513, 30000, 3000, 600], n=60000)
    check(A, B, exact=False, seg=seg)
    A2, _ = S.config2(n=30000, cap=5000)
    check(A2, A2, exact=False, seg=seg)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("seg", [0, 1024, 2048, 4096])
def test_split_rows_are_exact(dtype, seg):
    """Long rows cut into segments (512 products by default, or `seg`) and
    column ranges that all fit one tile: phase 1 only orders each segment and
    phase 2 folds every column in (segment, position) order, which is
    Gustavson's order -- every value is the oracle's sequential sum."""
    from paper_1504_05022_amd import CsrMatrix, Plan
    import torch
    A, B = S.crafted_rows([1500, 5000, 20000, 60000, 700, 3000], n=60000, dtype=dtype)
    print("case: split rows exact,", dtype, "seg", seg, flush=True)
    dA, dB = CsrMatrix.from_host(A), CsrMatrix.from_host(B)
    plan = Plan(dA, dB, seg=seg)
    C = plan.compute()
    torch.cuda.synchronize()
    assert plan.info.long_items > 6  # the rows were split
    _, _, rp, ci, v = C.to_host()
    plan.close()
    if dtype == np.float32:
        ref = oracle.spgemm(A.as_tuple(), B.as_tuple(), acc32=True)
    else:
        ref = oracle.spgemm(A.as_tuple(), B.as_tuple())
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr)
    assert np.array_equal(ci, ref.col_idx)
    assert np.array_equal(v.astype(np.float64), ref.val.astype(np.float64))


def test_collision_heavy_rows_split():
    """Workload-5-like rows (u >> n): many segments whose partials overlap in
    almost every column."""
    A, B = S.config5(n=20000, ncols=256)
    check(A, B, exact=False, seg=1024)


def test_never_split_with_tiny_pool():
    """The paper's progressive scheme alone: unsplit long rows spill L1 into
    pool blocks that grow 2x; a tiny pool forces checkpoint + relaunch."""
    A, B = S.crafted_rows([20000, 9000, 3000, 700, 40000, 600], n=60000)
    (_, ci0, v0), _ = check(A, B, exact=False, seg=-1)
    (_, ci1, v1), i1 = check(A, B, exact=False, seg=-1, pool_entries=500)
    assert i1.realloc_rounds > 0
    assert np.array_equal(ci0, ci1) and np.array_equal(v0, v1)


def test_one_call_multiply_matches_plan():
    """spgemm_multiply (analyze, compute and release in one call) gives the
    plan path's C bit for bit, and its info."""
    import torch
    from paper_1504_05022_amd import lib as L
    A, _ = S.config2(n=8000, cap=300)
    (rp, ci, v), info = check(A, A)
    dA = L.CsrMatrix.from_host(A)
    C, i2 = L.spgemm(dA, dA, return_info=True)
    torch.cuda.synchronize()
    _, _, rp2, ci2, v2 = C.to_host()
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2) and np.array_equal(v, v2)
    assert i2.nnz_c == info.nnz_c and i2.flops == info.flops
    assert list(i2.bin_count) == list(info.bin_count)


@pytest.mark.parametrize("seg,long_path", [(0, 0), (4096, 0), (0, 2)])
def test_options_do_not_change_result(seg, long_path):
    """Bin thresholds, level-1 size and stage timers change neither the
    structure nor any value: with the default options (what the benchmark
    runs), with 4096-product segments and with column windows."""
    A, _ = S.config2(n=8000, cap=300)
    o = dict(seg=seg, long_path=long_path)
    (rp0, ci0, v0), _ = check(A, A, **o)
    (rp1, ci1, v1), _ = check(A, A, bin_edges=(16, 48, 100, 300, 700), **o)
    (rp2, ci2, v2), _ = check(A, A, bin_edges=(8, 16, 32, 64, 128), l1_cap=7168, **o)
    # stage timers (all, then two) do not change the result
    (rp4, ci4, v4), _ = check(A, A, timing=1, **o)
    (rp5, ci5, v5), _ = check(A, A, timing=1, timing_mask=(1 << 8) | (1 << 10), **o)
    for ci, v in ((ci1, v1), (ci2, v2), (ci4, v4), (ci5, v5)):
        assert np.array_equal(ci, ci0) and np.array_equal(v, v0)
    if seg or long_path:
        return
    # a smaller level-1 sequence spills more often: same structure, values
    # within tolerance (checked inside check())
    (rp3, ci3, v3), _ = check(A, A, exact=False, long_slot=8, l1_cap=2048)
    assert np.array_equal(ci3, ci0)


def test_row_permutation_equivariance():
    """Permuting A's rows permutes C's rows; every row is computed the same
    way, so even spilled rows match bit for bit."""
    A, _ = S.config2(n=6000, cap=600)
    (rp, ci, v), _ = check(A, A, exact=False)
    perm = np.random.default_rng(3).permutation(A.rows)
    counts = np.diff(A.row_ptr)[perm]
    rpp = np.zeros(A.rows + 1, np.int32)
    np.cumsum(counts, out=rpp[1:])
    idx = np.concatenate([np.arange(A.row_ptr[i], A.row_ptr[i + 1]) for i in perm])
    from synthetic import Csr
    Ap = Csr(A.rows, A.cols, rpp, A.col_idx[idx], A.val[idx])
    (rq, cq, vq), _ = check(Ap, A, exact=False)
    for newi, oldi in enumerate(perm):
        a, b = rp[oldi], rp[oldi + 1]
        c, d = rq[newi], rq[newi + 1]
        assert np.array_equal(ci[a:b], cq[c:d]) and np.array_equal(v[a:b], vq[c:d])


def test_errors():
    import torch
    from paper_1504_05022_amd import CsrMatrix, Plan, SpgemmError
    A, _ = S.config1(n=50, degree=3)
    dA = CsrMatrix.from_host(A)
    B = CsrMatrix.from_host(S.uniform_csr(40, 30, 3))
    with pytest.raises(SpgemmError) as e:
        Plan(dA, B)
    assert e.value.name == "EINVAL"
    d32 = CsrMatrix.from_host(A.astype(np.float32))
    with pytest.raises(SpgemmError):
        Plan(dA, d32)
    # unsorted columns caught by validation
    bad_ci = A.col_idx.copy()
    bad_ci[0], bad_ci[1] = bad_ci[1], bad_ci[0]
    from synthetic import Csr
    bad = CsrMatrix.from_host(Csr(A.rows, A.cols, A.row_ptr, bad_ci, A.val))
    with pytest.raises(SpgemmError) as e:
        Plan(bad, dA, validate=1)
    assert e.value.name == "EINVAL"
    # out-of-range column
    oor = A.col_idx.copy()
    oor[-1] = A.cols + 5
    bad2 = CsrMatrix.from_host(Csr(A.rows, A.cols, A.row_ptr, oor, A.val))
    with pytest.raises(SpgemmError):
        Plan(bad2, dA, validate=1)
    # valid input passes validation
    Plan(dA, dA, validate=1).close()
    # options out of range
    with pytest.raises(SpgemmError):
        Plan(dA, dA, bin_edges=(40, 64, 128, 256, 512))
    with pytest.raises(SpgemmError):
        Plan(dA, dA, timing=1, timing_mask=1 << 20)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("ncols", [256, 9000])
def test_backward_matches_oracle(dtype, ncols):
    """Few columns: dC rows held densely on chip; many: binary searches in C."""
    import torch
    from paper_1504_05022_amd import CsrMatrix, Plan
    A, B = S.config5(n=3000, ncols=ncols)
    A, B = A.astype(dtype), B.astype(dtype)
    dA, dB = CsrMatrix.from_host(A), CsrMatrix.from_host(B)
    plan = Plan(dA, dB)
    C = plan.compute()
    dc = torch.as_tensor(S.config5_dc(C.nnz, dtype=dtype)).cuda()
    gA, gB = plan.backward(C, dc)
    torch.cuda.synchronize()
    ref = oracle.spgemm(A.astype(np.float64).as_tuple(), B.astype(np.float64).as_tuple())
    ra, rb = oracle.grad(A.as_tuple(), B.as_tuple(), ref.row_ptr, ref.col_idx,
                         dc.cpu().numpy().astype(np.float64))
    # componentwise bound: |g - g*| <= tol * sum |terms|
    absA = np.abs(A.astype(np.float64).val)
    absB = np.abs(B.astype(np.float64).val)
    sa, sb = oracle.grad(A.astype(np.float64).as_tuple(),
                         (B.rows, B.cols, B.row_ptr, B.col_idx, absB),
                         ref.row_ptr, ref.col_idx, np.abs(dc.cpu().numpy().astype(np.float64)))
    _, sb = oracle.grad((A.rows, A.cols, A.row_ptr, A.col_idx, absA), B.astype(np.float64).as_tuple(),
                        ref.row_ptr, ref.col_idx, np.abs(dc.cpu().numpy().astype(np.float64)))
    tol = TOL[np.dtype(dtype)]
    assert np.all(np.abs(gA.cpu().numpy().astype(np.float64) - ra) <= tol * sa + 0.0)
    assert np.all(np.abs(gB.cpu().numpy().astype(np.float64) - rb) <= tol * sb + 0.0)
    plan.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_window_method_row_plans(dtype):
    """Long rows by column windows (long_path 2), one case per row plan,
    every value Gustavson's sequential sum: rows of up to 1024 products as
    one sparse window; longer rows partitioned into pieces of 2^shift
    columns -- pieces of one wavefront's staging, and pieces whose products
    crowd into few columns and overflow it (then swept by a work-group in
    dense sub-windows)."""
    targets = [513, 700, 1024, 1025, 1500, 2048, 2049, 3000, 5000, 20000, 60000]
    A, B = S.crafted_rows(targets * 2, n=60000, dtype=dtype)
    check(A, B, long_path=2)
    # products crowded into columns [0, 3000) of 60000: overflowing pieces
    A, B = S.crafted_rows([2500, 5000, 9000, 30000], n=60000, col_range=3000, dtype=dtype)
    check(A, B, long_path=2)
    # many duplicates in few columns (large buckets of the counting sort)
    A, B = S.crafted_rows([3000, 5000, 1200], n=60000, col_range=40, dtype=dtype)
    check(A, B, long_path=2)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_window_method_dense_rows(dtype):
    """C with at most 2048 (binary64) / 4096 (binary32) columns: column
    windows are chosen automatically and every long row is one dense window
    in LDS; rows above 16384 products are cut into product ranges whose
    dense partial rows are added in range order (values within tolerance),
    the others are exact.  The merge method (long_path 1) gives the same
    structure."""
    n, big = (1500, 80000) if dtype == np.float64 else (3500, 120000)
    A, B = S.crafted_rows([600, 3000, 16384, 16385, 40000, 70000, big, 513], n=n, dtype=dtype)
    (rp, ci, v), info = check(A, B, exact=False)
    (rp1, ci1, v1), _ = check(A, B, exact=False, long_path=1)
    assert np.array_equal(rp, rp1) and np.array_equal(ci, ci1)
    ref = oracle.spgemm(A.astype(np.float64).as_tuple(), B.astype(np.float64).as_tuple())
    exact_rows = ref.u <= 16384
    mask = np.repeat(exact_rows, np.diff(ref.row_ptr))
    if dtype == np.float64:
        assert np.array_equal(v[mask], ref.val[mask])
    else:
        r32 = oracle.spgemm(A.as_tuple(), B.as_tuple(), acc32=True)
        assert np.array_equal(v[mask], r32.val[mask])


def test_window_method_matches_segment_method():
    """The two long-row methods give the same structure, and the same values
    wherever both sum in Gustavson's order (workload-2 structure)."""
    A, _ = S.config2(n=30000, cap=5000)
    (rp0, ci0, v0), i0 = check(A, A, long_path=2)
    (rp1, ci1, v1), i1 = check(A, A, long_path=1)
    assert np.array_equal(rp0, rp1) and np.array_equal(ci0, ci1)
    assert np.array_equal(v0, v1)


@pytest.mark.parametrize("case", ["workload2", "crowded", "duplicates"])
def test_direct_output_matches_copy(case):
    """Merge method with long_direct = 1: the pieces of split rows are sized
    by a counting pass over phase 1's sorted segments and written straight
    into C (no range buffer); C equals the default's bit for bit, on less
    device memory.  Crowded and duplicate-heavy columns send ranges through
    the larger-tile and level-1 kernels too."""
    if case == "workload2":
        A, _ = S.config2(n=30000, cap=5000)
        B = A
    elif case == "crowded":
        A, B = S.crafted_rows([1500, 3000, 9000, 30000, 2049], n=60000, col_range=3000)
    else:
        A, B = S.crafted_rows([3000, 5000, 1200], n=60000, col_range=40)
    (rp0, ci0, v0), i0 = check(A, B, exact=False, long_path=1)
    (rp1, ci1, v1), i1 = check(A, B, exact=False, long_path=1, long_direct=1)
    assert np.array_equal(rp0, rp1) and np.array_equal(ci0, ci1) and np.array_equal(v0, v1)
    assert i1.bytes_scratch < i0.bytes_scratch
