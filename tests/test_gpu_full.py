"""Parity at the full workload sizes, in the configuration the benchmark
times (default options).  Where the oracle can handle the whole product it
checks everything; otherwise sampled rows (forward) and sampled entries
(gradient) are compared one by one."""
import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu


def _compare_rows(C_host, ref, rows, tol):
    _, _, rp, ci, v = C_host
    for k, i in enumerate(rows):
        a, b = int(rp[i]), int(rp[i + 1])
        ra, rb = int(ref.row_ptr[k]), int(ref.row_ptr[k + 1])
        assert np.array_equal(ci[a:b], ref.col_idx[ra:rb]), i
        d = np.abs(v[a:b].astype(np.float64) - ref.val[ra:rb])
        s = ref.absval[ra:rb]
        assert np.all(d <= tol * s + (s == 0) * 0.0), i


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


def test_config5_full_forward_sampled(config5_full):
    """Workload 5 at full size: 400 sampled rows (the 40 longest, the rest
    uniform) against the oracle; row_ptr checked in full against Algorithm 2
    bounds and the row sizes of those rows."""
    import torch
    from paper_1504_05022_amd import CsrMatrix, spgemm
    A, B = config5_full
    dA, dB = CsrMatrix.from_host(A), CsrMatrix.from_host(B)
    C, info = spgemm(dA, dB, return_info=True)
    torch.cuda.synchronize()
    host = C.to_host()
    u, tot = oracle.upper_bound(A.as_tuple(), B.as_tuple())
    assert info.flops == 2 * tot
    rn = np.diff(host[2].astype(np.int64))
    assert np.all(rn <= np.minimum(u, B.cols))
    rng = np.random.default_rng(5)
    longest = np.argsort(u)[-40:]
    rows = np.unique(np.concatenate([longest, rng.choice(A.rows, 360, replace=False)]))
    from synthetic import Csr
    idx = np.concatenate([np.arange(A.row_ptr[r], A.row_ptr[r + 1]) for r in rows])
    rp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(np.diff(A.row_ptr)[rows], out=rp[1:])
    As = Csr(rows.size, A.cols, rp, A.col_idx[idx], A.val[idx])
    ref = oracle.spgemm(As.astype(np.float64).as_tuple(), B.astype(np.float64).as_tuple())
    _compare_rows(host, ref, rows, 1e-5)


def test_config5_full_backward_sampled(config5_full):
    """Gradient on the full workload against the oracle's gradient on 1000
    sampled entries of dA and 1000 of dB (componentwise bound)."""
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
    crp = C.row_ptr.cpu().numpy()
    cci = C.col_idx.cpu().numpy()
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
    g_a = av.grad.cpu().numpy().astype(np.float64)
    g_b = bv.grad.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g_a[sa] - ga[sa]) <= 1e-5 * ma[sa])
    assert np.all(np.abs(g_b[sb] - gb[sb]) <= 1e-5 * mb[sb])


def test_config4_full_size_problems():
    """Workload 4: the largest and smallest problems of the batch at their
    full sizes, and every 64th one, against the oracle."""
    from tests.test_gpu_parity import check
    sizes = S.config4_sizes()
    pick = sorted(set([int(np.argmax(sizes)), int(np.argmin(sizes))] + list(range(0, 512, 64))))
    for A, B in S.config4(only=pick):
        check(A, B)
