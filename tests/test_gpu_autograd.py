"""The differentiable extension: torch.autograd through spgemm_backward.

Checks: torch.autograd.gradcheck in binary64 on tiny inputs (a library
routine's finite differences as the pin); the gradient against the oracle's
gradient (componentwise bound); and central finite differences of the GPU
forward on sampled entries of dA and dB.  The loss L = <dC, A*B> is bilinear,
so a central difference with h = 1 has no truncation error; it is evaluated
on the slice of rows the perturbed entry affects.
"""
import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu


def _dev(M, dtype=None):
    from paper_1504_05022_amd import CsrMatrix
    return CsrMatrix.from_host(M if dtype is None else M.astype(dtype))


@pytest.mark.parametrize("seed", range(3))
def test_gradcheck_f64(seed):
    import torch
    from paper_1504_05022_amd import matmul
    from tests.helpers import random_csr
    rng = np.random.default_rng(900 + seed)
    A = _dev(random_csr(rng, 7, 6, 0.5))
    B = _dev(random_csr(rng, 6, 8, 0.5))
    av = A.val.clone().requires_grad_(True)
    bv = B.val.clone().requires_grad_(True)

    def f(x, y):
        return matmul(A.with_values(x), B.with_values(y)).val

    assert torch.autograd.gradcheck(f, (av, bv), eps=1e-6, atol=1e-9, rtol=1e-7)


def test_autograd_matches_oracle_gradient():
    import torch
    from paper_1504_05022_amd import matmul
    A, B = S.config5(n=6000, ncols=512)
    dA, dB = _dev(A), _dev(B)
    av = dA.val.clone().requires_grad_(True)
    bv = dB.val.clone().requires_grad_(True)
    C = matmul(dA.with_values(av), dB.with_values(bv))
    dc = torch.as_tensor(S.config5_dc(C.nnz)).cuda()
    (C.val * dc).sum().backward()
    torch.cuda.synchronize()
    crp = C.row_ptr.cpu().numpy()
    cci = C.col_idx.cpu().numpy()
    ga, gb = oracle.grad(A.as_tuple(), B.as_tuple(), crp, cci, dc.cpu().numpy().astype(np.float64))
    absA = (A.rows, A.cols, A.row_ptr, A.col_idx, np.abs(A.val.astype(np.float64)))
    absB = (B.rows, B.cols, B.row_ptr, B.col_idx, np.abs(B.val.astype(np.float64)))
    adc = np.abs(dc.cpu().numpy().astype(np.float64))
    sa, _ = oracle.grad(A.as_tuple(), absB, crp, cci, adc, want_b=False)
    _, sb = oracle.grad(absA, B.as_tuple(), crp, cci, adc, want_a=False)
    ea = np.abs(av.grad.cpu().numpy().astype(np.float64) - ga)
    eb = np.abs(bv.grad.cpu().numpy().astype(np.float64) - gb)
    print("max scaled grad error dA %.3g dB %.3g" % (np.max(ea / np.maximum(sa, 1e-300)),
                                                    np.max(eb / np.maximum(sb, 1e-300))))
    assert np.all(ea <= 1e-5 * sa) and np.all(eb <= 1e-5 * sb)


def _row_slice_loss(A, rows, Bd, dC_rows, aval_override=None):
    """<dC restricted to `rows`, (A[rows] * B)> evaluated on the GPU."""
    import torch
    from paper_1504_05022_amd import CsrMatrix, spgemm
    from synthetic import Csr
    idx = np.concatenate([np.arange(A.row_ptr[r], A.row_ptr[r + 1]) for r in rows])
    counts = np.array([A.row_ptr[r + 1] - A.row_ptr[r] for r in rows])
    rp = np.zeros(len(rows) + 1, np.int32)
    np.cumsum(counts, out=rp[1:])
    vals = A.val[idx] if aval_override is None else aval_override
    As = CsrMatrix.from_host(Csr(len(rows), A.cols, rp, A.col_idx[idx], vals))
    C = spgemm(As, Bd)
    torch.cuda.synchronize()
    return float(np.dot(dC_rows, C.val.cpu().numpy().astype(np.float64))), C


def test_finite_differences_sampled():
    """Central differences (h = 1) of the GPU forward on 100 sampled entries of
    dA and 100 of dB, binary32, workload-5 structure."""
    import torch
    from paper_1504_05022_amd import matmul
    A, B = S.config5(n=4000, ncols=512)
    dA, dB = _dev(A), _dev(B)
    av = dA.val.clone().requires_grad_(True)
    bv = dB.val.clone().requires_grad_(True)
    C = matmul(dA.with_values(av), dB.with_values(bv))
    dc = S.config5_dc(C.nnz)
    (C.val * torch.as_tensor(dc).cuda()).sum().backward()
    ga = av.grad.cpu().numpy()
    gb = bv.grad.cpu().numpy()
    crp = C.row_ptr.cpu().numpy()
    rng = np.random.default_rng(18)
    # dA_ij: only row i of C changes
    for p in rng.choice(A.nnz, 100, replace=False):
        i = int(np.searchsorted(A.row_ptr, p, side="right") - 1)
        dci = dc[crp[i]:crp[i + 1]].astype(np.float64)
        base = A.val[A.row_ptr[i]:A.row_ptr[i + 1]].copy()
        k = p - A.row_ptr[i]
        vp, vm = base.copy(), base.copy()
        vp[k] += 1
        vm[k] -= 1
        lp, _ = _row_slice_loss(A, [i], dB, dci, vp)
        lm, _ = _row_slice_loss(A, [i], dB, dci, vm)
        j = A.col_idx[p]
        scale = np.sum(np.abs(B.val[B.row_ptr[j]:B.row_ptr[j + 1]]).astype(np.float64)
                       * np.max(np.abs(dci)))
        assert abs((lp - lm) / 2 - ga[p]) <= 1e-3 * scale + 1e-6, p
    # dB_jk: the rows i with a_ij stored change
    colsA = {}
    for q in rng.choice(B.nnz, 100, replace=False):
        j = int(np.searchsorted(B.row_ptr, q, side="right") - 1)
        if j not in colsA:
            colsA[j] = np.nonzero(A.col_idx == j)[0]
        ents = colsA[j]
        rows = sorted(set(int(np.searchsorted(A.row_ptr, e, side="right") - 1) for e in ents))
        if not rows:
            assert gb[q] == 0
            continue
        dcr = np.concatenate([dc[crp[i]:crp[i + 1]] for i in rows]).astype(np.float64)
        from paper_1504_05022_amd import CsrMatrix
        bp, bm = B.val.copy(), B.val.copy()
        bp[q] += 1
        bm[q] -= 1
        from synthetic import Csr
        Bp = CsrMatrix.from_host(Csr(B.rows, B.cols, B.row_ptr, B.col_idx, bp))
        Bm = CsrMatrix.from_host(Csr(B.rows, B.cols, B.row_ptr, B.col_idx, bm))
        lp, _ = _row_slice_loss(A, rows, Bp, dcr)
        lm, _ = _row_slice_loss(A, rows, Bm, dcr)
        scale = sum(abs(float(A.val[e])) for e in ents) * np.max(np.abs(dcr))
        assert abs((lp - lm) / 2 - gb[q]) <= 1e-3 * scale + 1e-6, q
