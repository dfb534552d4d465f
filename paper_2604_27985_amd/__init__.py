"""MI355X-native SpMM and SDDMM (C = A B, S = A (.) (U V^T)) with A in CSR.

The library's computations run in hand-written HIP kernels for gfx950 behind a
C ABI (include/spk.h); this package is its Python binding.  Importing it does
not load the library; the first call does, and fails loudly when it is not
built.
"""
from ._lib import (BF16, F32, F64, OP_BACKWARD, OP_SDDMM, OP_SPMM, OP_TRANSPOSE, VAR_BSR4, VAR_COO, VAR_DCSR, VAR_MERGE,
                   VAR_ROWS, VAR_SLAB, VAR_SLAB16, VAR_TILE, SpkError)

__all__ = [
    "CSR", "Plan", "spmm", "sddmm", "csr_transpose", "spmm_backward", "spmm_autograd", "validate",
    "validate_rules", "backward_workspace_bytes", "workspace_bytes", "SpkError", "F32", "BF16", "F64", "OP_SPMM", "OP_SDDMM", "OP_BACKWARD", "OP_TRANSPOSE",
    "VAR_ROWS", "VAR_MERGE", "VAR_BSR4", "VAR_SLAB", "VAR_TILE", "VAR_SLAB16", "Slab16", "csr_to_slab16",
    "spmm_slab16", "sddmm_slab16", "attention", "attention_unfused", "csr_row_softmax", "VAR_DCSR", "VAR_COO",
    "csr_nonempty_order", "csr_row_index",
]


def __getattr__(name):
    # torch-dependent API is imported lazily so that the generator subpackage
    # can be used without touching torch or the HIP library.
    if name in ("CSR", "Plan", "spmm", "sddmm", "csr_transpose", "spmm_backward", "spmm_autograd", "validate",
                "validate_rules", "backward_workspace_bytes", "workspace_bytes", "SpMMFunction", "BSR4", "csr_to_bsr4", "spmm_bsr4", "Slab16", "csr_to_slab16", "spmm_slab16",
                "sddmm_slab16", "attention", "attention_unfused", "csr_row_softmax", "attention_workspace_bytes", "csr_nonempty_order", "csr_row_index"):
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
