"""Batched products (spgemm_batch_*) through the C ABI.

Every C_p of a batch must equal the single-product path bit for bit (same
structure, same values: both sum each row in ascending (column, product
index) order), and the oracle to the usual componentwise bound.  Problems
that the class kernels do not take (rows with more than 1024
products) are recomputed with the single-product path and counted in the
statistics.
"""
import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu

TOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}


def _plain(A, B):
    from paper_1504_05022_amd import CsrMatrix, spgemm
    C = spgemm(CsrMatrix.from_host(A), CsrMatrix.from_host(B))
    return C.to_host()


def _oracle_check(A, B, host):
    _, _, rp, ci, v = host
    ref = oracle.spgemm(A.astype(np.float64).as_tuple(), B.astype(np.float64).as_tuple())
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr)
    assert np.array_equal(ci, ref.col_idx)
    err, _ = oracle.value_error(v, ref)
    assert err <= TOL[np.dtype(A.val.dtype)]


def _same(h1, h2):
    for x, y in zip(h1[2:], h2[2:]):
        assert x.dtype == y.dtype and np.array_equal(x, y)


def _batch(problems, **opts):
    from paper_1504_05022_amd import Batch, CsrMatrix
    dev = [(CsrMatrix.from_host(A), CsrMatrix.from_host(B)) for A, B in problems]
    return dev, Batch(dev, **opts)


def test_batch_mixed_precision_against_plain_and_oracle():
    import torch
    problems = S.config4(count=40, nmin=200, nmax=3000)
    print("case: config4-shaped batch, 40 problems, n in [200, 3000]", flush=True)
    dev, b = _batch(problems)
    st = b.stats.as_dict()
    print("  stats", st, flush=True)
    assert st["count"] == 40 and st["fallback"] == 0 and st["items"] > 0
    outs = b.run()
    torch.cuda.synchronize()
    flops = 0
    for p, (A, B) in enumerate(problems):
        h = outs[p].to_host()
        assert outs[p].dtype == (torch.float64 if p % 2 == 0 else torch.float32)
        _same(h, _plain(A, B))
        if p % 5 == 0:
            _oracle_check(A, B, h)
        flops += oracle.upper_bound(A.as_tuple(), B.as_tuple())[1] * 2
    assert st["flops"] == flops
    assert st["nnz_c"] == sum(o.nnz for o in outs)
    b.close()


def test_batch_replay_recomputes_values():
    """Clearing the outputs between replays: every replay writes them again."""
    import torch
    problems = S.config4(count=12, nmin=100, nmax=2000)
    dev, b = _batch(problems)
    first = [o.to_host() for o in b.run()]
    for rep in range(3):
        outs = b.run(views=True)
        for o in outs:
            o.val.zero_()
            o.col_idx.fill_(-1)
        torch.cuda.synchronize()
        outs = b.run()
        torch.cuda.synchronize()
        print("  replay", rep, flush=True)
        for p in range(len(problems)):
            _same(outs[p].to_host(), first[p])
    b.close()


def test_batch_fixed_edges_no_tuning():
    """Thresholds fixed by the caller: only the three tile-shape sets are
    timed, under those thresholds."""
    import torch
    problems = S.config4(count=8, nmin=300, nmax=1500)
    dev, b = _batch(problems, bin_edges=[16, 64, 256, 512, 1024])
    st = b.stats.as_dict()
    assert st["bin_edges"] == [16, 64, 256, 512, 1024]
    assert all(t > 0 for t in st["tune_ms"][:3]) and st["tune_ms"][3:] == [0.0] * 9
    assert st["shapes"] in (0, 1, 2)
    outs = b.run()
    torch.cuda.synchronize()
    for p, (A, B) in enumerate(problems):
        _same(outs[p].to_host(), _plain(A, B))
    b.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batch_fallback_and_degenerate_problems(dtype):
    """A problem with long rows (taken by the single-product path), a
    product with no rows, one whose rows are all empty, one 1x1, next to
    ordinary problems."""
    import torch
    from tests.helpers import from_rows, identity
    longp = S.crafted_rows([5, 1500, 3000, 0, 17], n=2048, dtype=dtype)
    empty_rows = (S.Csr(0, 50, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, dtype)),
                  S.Csr(50, 40, np.zeros(51, np.int32), np.zeros(0, np.int32), np.zeros(0, dtype)))
    zero_a = S.Csr(30, 60, np.zeros(31, np.int32), np.zeros(0, np.int32), np.zeros(0, dtype))
    one = from_rows(1, 1, [(0, 0, 3.0)], dtype)
    problems = [S.config4(count=2, nmin=500, nmax=800)[0], longp, empty_rows,
                (zero_a, identity(60, dtype)), (one, one), S.config4(count=2, nmin=500, nmax=800)[1]]
    print("case: fallback + degenerate problems,", dtype, flush=True)
    dev, b = _batch(problems)
    st = b.stats.as_dict()
    print("  stats", st, flush=True)
    assert st["fallback"] == 1
    for rep in range(2):
        outs = b.run()
        torch.cuda.synchronize()
        for p, (A, B) in enumerate(problems):
            h = outs[p].to_host()
            assert outs[p].shape == (A.rows, B.cols)
            _oracle_check(A, B, h)
            if p != 1:
                _same(h, _plain(A, B))
    b.close()


def test_batch_empty_and_errors():
    import ctypes
    from paper_1504_05022_amd import Batch, SpgemmError
    from paper_1504_05022_amd import lib as L
    b = Batch([])
    assert b.stats.count == 0 and b.stats.items == 0
    assert b.run() == []
    b.close()
    L.load()
    h = ctypes.c_void_p()
    rc = L._lib.spgemm_batch_create(-1, None, None, None, L._alloc_cb, L._free_cb, None,
                                    L._stream_handle(), ctypes.byref(h), None)
    assert rc == -1 and not h
    assert L._lib.spgemm_batch_run(None, None, None) == -1
    # shape mismatch inside one problem is reported by its analysis
    A = S.Csr(4, 5, np.arange(5, dtype=np.int32), np.zeros(4, np.int32), np.ones(4))
    with pytest.raises(SpgemmError):
        _batch([(A, A)])


def test_config4_full_batch_sampled():
    """Workload 4 at its full size (512 problems, n log-uniform in
    [1024, 65536]): every problem against the single-product path, and 16
    of them against the oracle."""
    import torch
    problems = S.config4()
    dev, b = _batch(problems)
    st = b.stats.as_dict()
    print("  stats", st, flush=True)
    assert st["fallback"] == 0
    outs = b.run()
    torch.cuda.synchronize()
    pick = set(range(0, 512, 32))
    for p, (A, B) in enumerate(problems):
        h = outs[p].to_host()
        if p in pick:
            _oracle_check(A, B, h)
        if p % 4 == 0:
            _same(h, _plain(A, B))
    b.close()


@pytest.mark.parametrize("shapes", [1, 2, 3])
def test_batch_every_tile_shape_set(shapes):
    """Each tile-shape set (lanes per row against products per lane of every
    capacity class), fixed by batch_shapes, gives C bit for bit equal to the
    plain path; with the thresholds fixed too nothing is timed."""
    import torch
    problems = S.config4(count=12, nmin=300, nmax=3000)
    dev, b = _batch(problems, bin_edges=[16, 64, 256, 512, 1024], batch_shapes=shapes)
    st = b.stats.as_dict()
    assert st["shapes"] == shapes - 1 and st["tune_ms"] == [0.0] * 12
    outs = b.run()
    torch.cuda.synchronize()
    for p, (A, B) in enumerate(problems):
        _same(outs[p].to_host(), _plain(A, B))
    b.close()


# ---- one-shot batched products (spgemm_batch_multiply): no plan, no graph


def _multiply(problems, **opts):
    from paper_1504_05022_amd import CsrMatrix, batch_multiply
    dev = [(CsrMatrix.from_host(A), CsrMatrix.from_host(B)) for A, B in problems]
    outs, st = batch_multiply(dev, return_stats=True, **opts)
    return dev, outs, st.as_dict()


def test_batch_multiply_against_plain_and_oracle():
    import torch
    problems = S.config4(count=40, nmin=200, nmax=3000)
    print("case: one-shot batch, 40 problems, n in [200, 3000]", flush=True)
    dev, outs, st = _multiply(problems)
    print("  stats", st, flush=True)
    torch.cuda.synchronize()
    assert st["count"] == 40 and st["fallback"] == 0 and st["items"] > 0
    assert 0 < st["grid"] <= 11 and st["shapes"] == 0
    flops = 0
    for p, (A, B) in enumerate(problems):
        h = outs[p].to_host()
        assert outs[p].dtype == (torch.float64 if p % 2 == 0 else torch.float32)
        _same(h, _plain(A, B))
        if p % 5 == 0:
            _oracle_check(A, B, h)
        flops += oracle.upper_bound(A.as_tuple(), B.as_tuple())[1] * 2
    assert st["flops"] == flops
    assert st["nnz_c"] == sum(o.nnz for o in outs)
    # scratch: at least C~ (4 + 8 bytes per product) and the entry scan
    nprod = flops // 2
    nnz_a = sum(A.nnz for A, _ in problems)
    assert st["bytes_scratch"] >= 12 * nprod + 12 * nnz_a


@pytest.mark.parametrize("shapes", [1, 2, 3])
def test_batch_multiply_every_tile_shape_set(shapes):
    import torch
    problems = S.config4(count=10, nmin=300, nmax=2500)
    dev, outs, st = _multiply(problems, batch_shapes=shapes)
    torch.cuda.synchronize()
    assert st["shapes"] == shapes - 1
    for p, (A, B) in enumerate(problems):
        _same(outs[p].to_host(), _plain(A, B))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batch_multiply_fallback_and_degenerate_problems(dtype):
    """Long rows (plain path, moved into the output block), no rows, only
    empty rows, an all-zero A, 1x1, duplicates-heavy rows, next to ordinary
    problems."""
    import torch
    from tests.helpers import from_rows, identity
    longp = S.crafted_rows([5, 1500, 3000, 0, 17], n=2048, dtype=dtype)
    empty_rows = (S.Csr(0, 50, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, dtype)),
                  S.Csr(50, 40, np.zeros(51, np.int32), np.zeros(0, np.int32), np.zeros(0, dtype)))
    zero_a = S.Csr(30, 60, np.zeros(31, np.int32), np.zeros(0, np.int32), np.zeros(0, dtype))
    one = from_rows(1, 1, [(0, 0, 3.0)], dtype)
    crowded = S.crafted_rows([1024, 1000, 600, 1, 0, 2, 513], n=700, dtype=dtype, col_range=40)
    problems = [S.config4(count=2, nmin=500, nmax=800)[0], longp, empty_rows,
                (zero_a, identity(60, dtype)), (one, one), crowded,
                S.config4(count=2, nmin=500, nmax=800)[1]]
    print("case: one-shot fallback + degenerate problems,", dtype, flush=True)
    dev, outs, st = _multiply(problems)
    print("  stats", st, flush=True)
    torch.cuda.synchronize()
    assert st["fallback"] == 1
    for p, (A, B) in enumerate(problems):
        h = outs[p].to_host()
        assert outs[p].shape == (A.rows, B.cols)
        _oracle_check(A, B, h)
        _same(h, _plain(A, B))


def test_batch_multiply_only_fallbacks_and_empty():
    import torch
    from paper_1504_05022_amd import batch_multiply
    outs, st = batch_multiply([], return_stats=True)
    assert outs == [] and st.count == 0 and st.items == 0
    problems = [S.crafted_rows([2000, 1100], n=4096), S.crafted_rows([1025], n=2048)]
    dev, outs, st = _multiply(problems)
    torch.cuda.synchronize()
    assert st["fallback"] == 2 and st["items"] == 0 and st["grid"] == 0
    for p, (A, B) in enumerate(problems):
        _same(outs[p].to_host(), _plain(A, B))


def test_batch_multiply_errors():
    import ctypes
    from paper_1504_05022_amd import SpgemmError
    from paper_1504_05022_amd import lib as L
    L.load()
    mem = ctypes.c_void_p()
    rc = L._lib.spgemm_batch_multiply(-1, None, None, None, L._alloc_cb, L._free_cb, None,
                                      L._stream_handle(), None, ctypes.byref(mem), None)
    assert rc == -1 and not mem
    rc = L._lib.spgemm_batch_multiply(0, None, None, None, L._alloc_cb, L._free_cb, None,
                                      L._stream_handle(), None, None, None)
    assert rc == -1
    A = S.Csr(4, 5, np.arange(5, dtype=np.int32), np.zeros(4, np.int32), np.ones(4))
    with pytest.raises(SpgemmError):
        _multiply([(A, A)])
    good = S.config4(count=2, nmin=100, nmax=200)
    with pytest.raises(SpgemmError):
        _multiply(good, batch_shapes=4)


def test_config4_full_batch_multiply_sampled():
    """Workload 4 at full size through the one-shot form: every fourth
    problem against the single-product path, 16 against the oracle."""
    import torch
    problems = S.config4()
    dev, outs, st = _multiply(problems)
    print("  stats", st, flush=True)
    torch.cuda.synchronize()
    assert st["fallback"] == 0
    pick = set(range(0, 512, 32))
    for p, (A, B) in enumerate(problems):
        h = outs[p].to_host()
        if p in pick:
            _oracle_check(A, B, h)
        if p % 4 == 0:
            _same(h, _plain(A, B))
