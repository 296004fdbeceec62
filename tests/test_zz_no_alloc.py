"""The backward entry point that allocates no device memory
(spgemm_backward_static): its gradients equal spgemm_backward's bit for bit
(the same kernels and summation order), on two calls in a row -- the second
with a smaller input, so that the fixed scratch area holds the first call's
contents -- for the staged dB products and for dB summed without staging,
and an input whose transposed pattern exceeds the area is refused."""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20  # SPGEMM_STATIC_SCRATCH_BYTES


def _grads(A, B, seed, dtype):
    import torch
    from paper_1504_05022_amd import CsrMatrix, Plan
    dA_ = CsrMatrix.from_host(A.astype(dtype))
    dB_ = CsrMatrix.from_host(B.astype(dtype))
    plan = Plan(dA_, dB_)
    C = plan.compute()
    g = torch.Generator(device="cuda").manual_seed(seed)
    dC = torch.randn(C.nnz, generator=g, device="cuda", dtype=C.val.dtype)
    ga, gb = plan.backward(C, dC)
    sa = torch.full_like(ga, float("nan"))
    sb = torch.full_like(gb, float("nan"))
    plan.backward_static(C, dC, sa, sb)
    # one output skipped: the other is unchanged
    sa2 = torch.full_like(ga, float("nan"))
    plan.backward_static(C, dC, sa2, None)
    torch.cuda.synchronize()
    info = plan.info
    plan.close()
    return ([x.cpu().numpy() for x in (ga, gb, sa, sb, sa2)], int(info.nnz_hat))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_static_backward_matches_backward(dtype):
    # first call: staged dB products; second call, smaller: the area still
    # holds the first call's pattern and products
    for n, seed in ((20000, 1), (3000, 2)):
        print("case: workload-2 structure n=%d %s" % (n, np.dtype(dtype).name), flush=True)
        A, _ = S.config2(n=n, cap=2000)
        (ga, gb, sa, sb, sa2), nprod = _grads(A, A, seed, dtype)
        assert nprod * np.dtype(dtype).itemsize < SCRATCH - (8 << 20)  # staged
        assert np.array_equal(sa, ga) and np.array_equal(sb, gb)
        assert np.array_equal(sa2, ga)


def test_static_backward_unstaged_db():
    # nnz(hat C) products too many to stage in the area: dB is summed
    # without staging, to the same values
    for n, seed in ((120000, 3), (30000, 4)):
        print("case: workload-2 structure n=%d float64" % n, flush=True)
        A, _ = S.config2(n=n)
        (ga, gb, sa, sb, sa2), nprod = _grads(A, A, seed, np.float64)
        assert np.array_equal(sa, ga) and np.array_equal(sb, gb)
        assert np.array_equal(sa2, ga)
        if n == 120000:
            assert nprod * 8 > SCRATCH


def test_static_backward_rejects_oversize():
    import torch
    from paper_1504_05022_amd import CsrMatrix, Plan, SpgemmError
    # A 4 x k with k = 6M columns: its transposed pattern needs 12 k bytes
    k = 6_000_000
    rng = np.random.default_rng(5)
    cols = np.sort(rng.choice(k, 40, replace=False)).astype(np.int32)
    A = S.Csr(4, k, np.arange(0, 41, 10, dtype=np.int32), cols, rng.standard_normal(40))
    brp = np.zeros(k + 1, np.int32)
    brp[cols + 1] = 1
    brp = np.cumsum(brp).astype(np.int32)
    B = S.Csr(k, 8, brp, rng.integers(0, 8, 40).astype(np.int32), rng.standard_normal(40))
    print("case: A 4 x %d, transposed pattern above the scratch area" % k, flush=True)
    dA_, dB_ = CsrMatrix.from_host(A), CsrMatrix.from_host(B)
    plan = Plan(dA_, dB_)
    C = plan.compute()
    dC = torch.ones(C.nnz, device="cuda", dtype=torch.float64)
    ga, gb = plan.backward(C, dC)
    sb = torch.empty_like(gb)
    with pytest.raises(SpgemmError):
        plan.backward_static(C, dC, None, sb)
    # dA alone needs no scratch
    sa = torch.full_like(ga, float("nan"))
    plan.backward_static(C, dC, sa, None)
    torch.cuda.synchronize()
    assert torch.equal(sa, ga)
    plan.close()
