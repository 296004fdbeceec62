"""Differentiable C = A*B on fixed sparsity patterns.

``matmul(A, B)`` returns C whose value tensor carries autograd history with
respect to A's and B's value tensors.  The backward pass calls
``spgemm_backward``: dA = (dC B^T) restricted to A's pattern and
dB = (A^T dC) restricted to B's pattern, both computed by masked gather
kernels in the HIP library (no dense intermediate, no atomics).
"""
from __future__ import annotations

import torch

from .lib import CsrMatrix, Plan


class _SpGEMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a_val, b_val, A, B, opts):
        plan = Plan(A.with_values(a_val.detach()), B.with_values(b_val.detach()), **opts)
        C = plan.compute()
        ctx.plan = plan
        ctx.C = C
        ctx.mark_non_differentiable(C.row_ptr, C.col_idx)
        return C.val, C.row_ptr, C.col_idx

    @staticmethod
    def backward(ctx, grad_val, _g_rp, _g_ci):
        plan = ctx.plan
        want_a = ctx.needs_input_grad[0]
        want_b = ctx.needs_input_grad[1]
        dA = dB = None
        if grad_val is not None and (want_a or want_b):
            dA, dB = plan.backward(ctx.C, grad_val.contiguous(), want_a, want_b)
        # the plan stays alive with the graph (backward may run again with
        # retain_graph); it is released when the graph is freed
        return dA, dB, None, None, None


def matmul(A: CsrMatrix, B: CsrMatrix, **opts) -> CsrMatrix:
    """C = A*B, differentiable in A.val and B.val (patterns are fixed)."""
    val, rp, ci = _SpGEMM.apply(A.val, B.val, A, B, opts)
    return CsrMatrix((A.shape[0], B.shape[1]), rp, ci, val)


def matmul_torch(a: torch.Tensor, b: torch.Tensor, **opts) -> torch.Tensor:
    """Same for torch.sparse_csr_tensor operands (int32 or int64 indices)."""
    A = CsrMatrix.from_torch(a)
    B = CsrMatrix.from_torch(b)
    A.val = a.values()
    B.val = b.values()
    C = matmul(A, B, **opts)
    return torch.sparse_csr_tensor(C.row_ptr, C.col_idx, C.val, C.shape)
