"""MI355X-native general sparse matrix-matrix multiplication (C = A*B, CSR).

Liu & Vinter's SpGEMM framework (upper bounds, binning, hybrid allocation,
per-bin insert kernels, compaction) as hand-written HIP kernels for gfx950
behind the C ABI in include/spgemm.h; this package is its Python binding.
"""
from .lib import (  # noqa: F401
    Batch,
    CsrMatrix,
    Plan,
    batch_multiply,
    SpgemmError,
    default_options,
    load,
    spgemm,
)
from .autograd import matmul, matmul_torch  # noqa: F401
