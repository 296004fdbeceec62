"""Parity at the full workload sizes, in the configuration the benchmark
times (default options): whole results against the oracle (workload 5 in
row blocks), gradients on sampled entries against the oracle's gradient and
against central differences."""
import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu


def test_config2_full_against_oracle():
    """Workload 2 at full size (200000 rows, 51M products): whole result."""
    import torch
    from paper_1504_05022_amd import CsrMatrix, spgemm
    A, _ = S.config2()
    dA = CsrMatrix.from_host(A)
    C, info = spgemm(dA, dA, return_info=True)
    torch.cuda.synchronize()
    _, _, rp, ci, v = C.to_host()
    ref = oracle.spgemm(A.as_tuple(), A.as_tuple())
    assert info.flops == ref.flops and info.nnz_c == ref.nnz
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr)
    assert np.array_equal(ci, ref.col_idx)
    err, rel = oracle.value_error(v, ref)
    print("workload 2: nnz(C) %d, max scaled error %.3g, max relative error %.3g" %
          (ref.nnz, err, rel))
    assert err <= 1e-12


@pytest.fixture(scope="module")
def config5_full():
    A, B = S.config5()
    return A, B


def _rows_csr(A, r0, r1):
    from synthetic import Csr
    a, b = int(A.row_ptr[r0]), int(A.row_ptr[r1])
    rp = (A.row_ptr[r0:r1 + 1].astype(np.int64) - a)
    return Csr(r1 - r0, A.cols, rp, A.col_idx[a:b], A.val[a:b])


def test_config5_full_forward_all_rows(config5_full):
    """Workload 5 at full size (500000 rows, 320M products): every row of C
    against the oracle, computed in row blocks of 50000 -- row sizes and
    columns bit for bit, values within 1e-5 of the magnitude sums; the
    largest error over the whole result is reported."""
    import torch
    from paper_1504_05022_amd import CsrMatrix, spgemm
    A, B = config5_full
    dA, dB = CsrMatrix.from_host(A), CsrMatrix.from_host(B)
    C, info = spgemm(dA, dB, return_info=True)
    torch.cuda.synchronize()
    _, _, rp, ci, v = C.to_host()
    del C
    u, tot = oracle.upper_bound(A.as_tuple(), B.as_tuple())
    assert info.flops == 2 * tot
    rp = rp.astype(np.int64)
    A64, B64 = A.astype(np.float64), B.astype(np.float64).as_tuple()
    worst, worst_rel = 0.0, 0.0
    for r0 in range(0, A.rows, 50000):
        r1 = min(A.rows, r0 + 50000)
        ref = oracle.spgemm(_rows_csr(A64, r0, r1).as_tuple(), B64)
        assert np.array_equal(np.diff(rp[r0:r1 + 1]), np.diff(ref.row_ptr)), (r0, r1)
        a, b = int(rp[r0]), int(rp[r1])
        assert np.array_equal(ci[a:b], ref.col_idx), (r0, r1)
        err, rel = oracle.value_error(v[a:b], ref)
        worst, worst_rel = max(worst, err), max(worst_rel, rel)
        assert err <= 1e-5, (r0, r1, err)
        del ref
    print("workload 5 forward: nnz(C) %d, max scaled error %.3g, max relative error %.3g" %
          (int(rp[-1]), worst, worst_rel))


@pytest.fixture(scope="module")
def config5_grad(config5_full):
    """Autograd gradients of <dC, A*B> on the full workload (GPU)."""
    import torch
    from paper_1504_05022_amd import CsrMatrix, matmul
    A, B = config5_full
    dA, dB = CsrMatrix.from_host(A), CsrMatrix.from_host(B)
    av = dA.val.clone().requires_grad_(True)
    bv = dB.val.clone().requires_grad_(True)
    C = matmul(dA.with_values(av), dB.with_values(bv))
    dc = S.config5_dc(C.nnz)
    (C.val * torch.as_tensor(dc).cuda()).sum().backward()
    torch.cuda.synchronize()
    out = dict(dA=dA, dB=dB, crp=C.row_ptr.cpu().numpy(), cci=C.col_idx.cpu().numpy(), dc=dc,
               ga=av.grad.cpu().numpy().astype(np.float64),
               gb=bv.grad.cpu().numpy().astype(np.float64))
    del C, av, bv
    return out


def test_config5_full_backward_sampled(config5_full, config5_grad):
    """Gradient on the full workload against the oracle's gradient on 1000
    sampled entries of dA and 1000 of dB (componentwise bound)."""
    A, B = config5_full
    g = config5_grad
    crp, cci, dc = g["crp"], g["cci"], g["dc"]
    rng = np.random.default_rng(18)
    sa = rng.choice(A.nnz, 1000, replace=False)
    sb = rng.choice(B.nnz, 1000, replace=False)
    dc64 = dc.astype(np.float64)
    ga, gb = oracle.grad(A.astype(np.float64).as_tuple(), B.astype(np.float64).as_tuple(), crp,
                         cci, dc64, sample_a=sa, sample_b=sb)
    absA = (A.rows, A.cols, A.row_ptr, A.col_idx, np.abs(A.val.astype(np.float64)))
    absB = (B.rows, B.cols, B.row_ptr, B.col_idx, np.abs(B.val.astype(np.float64)))
    ma, _ = oracle.grad(A.astype(np.float64).as_tuple(), absB, crp, cci, np.abs(dc64),
                        sample_a=sa, want_b=False)
    _, mb = oracle.grad(absA, B.astype(np.float64).as_tuple(), crp, cci, np.abs(dc64),
                        sample_b=sb, want_a=False)
    assert np.all(np.abs(g["ga"][sa] - ga[sa]) <= 1e-5 * ma[sa])
    assert np.all(np.abs(g["gb"][sb] - gb[sb]) <= 1e-5 * mb[sb])


def test_config5_full_finite_differences(config5_full, config5_grad):
    """Central differences on the full workload, 1000 sampled entries of dA
    and 1000 of dB.  L = <dC, A*B> is bilinear, so h = 1 has no truncation
    error; each difference evaluates the GPU forward of only the rows of C
    that the entry touches (row i for a_ij, the rows of A's column j for
    b_jk), and must agree with the gradient within 1e-3 of the magnitude of
    its terms (binary32 forward)."""
    import torch
    from paper_1504_05022_amd import CsrMatrix, spgemm
    from synthetic import Csr
    A, B = config5_full
    g = config5_grad
    crp, dc, ga, gb = g["crp"], g["dc"], g["ga"], g["gb"]
    dB = g["dB"]
    rng = np.random.default_rng(1018)

    def slice_loss(rows, avals, Bd):
        idx = np.concatenate([np.arange(A.row_ptr[r], A.row_ptr[r + 1]) for r in rows])
        rp = np.zeros(len(rows) + 1, np.int32)
        np.cumsum([A.row_ptr[r + 1] - A.row_ptr[r] for r in rows], out=rp[1:])
        As = CsrMatrix.from_host(Csr(len(rows), A.cols, rp, A.col_idx[idx],
                                     A.val[idx] if avals is None else avals))
        C = spgemm(As, Bd)
        dcr = np.concatenate([dc[crp[i]:crp[i + 1]] for i in rows]).astype(np.float64)
        return float(np.dot(dcr, C.val.cpu().numpy().astype(np.float64))), dcr

    worst = 0.0
    for p in rng.choice(A.nnz, 1000, replace=False):
        i = int(np.searchsorted(A.row_ptr, p, side="right") - 1)
        base = A.val[A.row_ptr[i]:A.row_ptr[i + 1]].copy()
        k = p - A.row_ptr[i]
        vp, vm = base.copy(), base.copy()
        vp[k] += 1
        vm[k] -= 1
        lp, dci = slice_loss([i], vp, dB)
        lm, _ = slice_loss([i], vm, dB)
        j = A.col_idx[p]
        scale = float(np.sum(np.abs(B.val[B.row_ptr[j]:B.row_ptr[j + 1]]).astype(np.float64))
                      * np.max(np.abs(dci)))
        d = abs((lp - lm) / 2 - ga[p])
        worst = max(worst, d / max(scale, 1e-30))
        assert d <= 1e-3 * scale + 1e-6, p
    # rows of every column of A, for the dB entries
    order = np.argsort(A.col_idx, kind="stable")
    col_start = np.searchsorted(A.col_idx[order], np.arange(A.cols + 1))
    row_of = np.repeat(np.arange(A.rows), np.diff(A.row_ptr))
    for q in rng.choice(B.nnz, 1000, replace=False):
        j = int(np.searchsorted(B.row_ptr, q, side="right") - 1)
        ents = order[col_start[j]:col_start[j + 1]]
        rows = sorted(set(row_of[ents].tolist()))
        if not rows:
            assert gb[q] == 0
            continue
        bp = dB.val.clone()
        bp[int(q)] += 1
        bm = dB.val.clone()
        bm[int(q)] -= 1
        lp, dcr = slice_loss(rows, None, dB.with_values(bp))
        lm, _ = slice_loss(rows, None, dB.with_values(bm))
        scale = float(np.sum(np.abs(A.val[ents]).astype(np.float64)) * np.max(np.abs(dcr)))
        d = abs((lp - lm) / 2 - gb[q])
        worst = max(worst, d / max(scale, 1e-30))
        assert d <= 1e-3 * scale + 1e-6, q
    torch.cuda.synchronize()
    print("workload 5 finite differences: max |fd - g| / scale = %.3g" % worst)


def test_config4_full_size_problems():
    """Workload 4: the largest and smallest problems of the batch at their
    full sizes, and every 64th one, against the oracle."""
    from tests.test_gpu_parity import check
    sizes = S.config4_sizes()
    pick = sorted(set([int(np.argmax(sizes)), int(np.argmin(sizes))] + list(range(0, 512, 64))))
    for A, B in S.config4(only=pick):
        check(A, B)
