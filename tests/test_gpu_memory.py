"""Device memory of a plan: spgemm_info.bytes_scratch is the most memory
the plan held at once during its latest call, as the caller's allocator saw
it (C excluded) -- for analyze, for compute with both long-row methods, on a
dense-window product and with long-row pool growth, and for a backward (A's
transposed pattern plus the staged products) -- and after the plan is
destroyed nothing it allocated is left."""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


class _Tracked(dict):
    """The binding's table of live allocations, with the current and the
    largest total size."""

    def __init__(self, base):
        super().__init__(base)
        self.cur = sum(t.numel() for t in base.values())
        self.peak = self.cur

    def __setitem__(self, k, v):
        super().__setitem__(k, v)
        self.cur += v.numel()
        self.peak = max(self.peak, self.cur)

    def pop(self, k, *default):
        v = super().pop(k, *default)
        if v is not None and not (default and v is default[0]):
            self.cur -= v.numel()
        return v


def _alloc_size(b):
    b = (b + 255) & ~255
    return b if b else 256


@pytest.mark.parametrize("case", ["workload1", "merge", "direct", "windows", "dense", "pool_growth"])
def test_bytes_scratch_is_the_plans_peak(case):
    import torch
    from paper_1504_05022_amd import lib as L
    opts = {}
    if case == "workload1":
        A, _ = S.config1()
        B = A
    elif case in ("merge", "direct", "windows"):
        A, _ = S.config2(n=20000, cap=3000)
        B = A
        opts = {"long_path": 2 if case == "windows" else 1, "long_direct": int(case == "direct")}
    elif case == "dense":
        A, B = S.crafted_rows([600, 3000, 40000, 513, 20], n=3000, dtype=np.float32)
    else:
        A, _ = S.config2(n=8000, cap=2000)
        B = A
        opts = {"seg": -1, "pool_entries": 300}
    print("case:", case, A.rows, A.nnz, opts, flush=True)
    dA, dB = L.CsrMatrix.from_host(A), L.CsrMatrix.from_host(B)
    torch.cuda.synchronize()
    saved = L._live
    L._live = tr = _Tracked(saved)
    try:
        base = tr.cur
        plan = L.Plan(dA, dB, **opts)
        assert plan.info.bytes_scratch == tr.peak - base  # analysis arrays
        tr.peak = tr.cur
        C = plan.compute()
        torch.cuda.synchronize()
        info = plan.info
        if case == "pool_growth":
            assert info.realloc_rounds > 0
        s = C.val.element_size()
        c_bytes = _alloc_size(4 * (A.rows + 1)) + _alloc_size(4 * C.nnz) + _alloc_size(s * C.nnz)
        assert info.bytes_scratch == tr.peak - base - c_bytes
        assert info.nnz_c == C.nnz <= info.nnz_hat
        tr.peak = tr.cur
        plan.backward(C, torch.ones(C.nnz, device="cuda", dtype=C.val.dtype))
        torch.cuda.synchronize()
        assert plan.refresh_info().bytes_scratch == tr.peak - base
        plan.close()
        assert tr.cur == base
    finally:
        L._live = saved
        for k, v in tr.items():
            if k not in saved:
                saved[k] = v
