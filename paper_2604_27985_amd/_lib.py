"""ctypes loader for libspk.so: the C ABI declared in include/spk.h.

Loading fails loudly when the library is not built: there is no fallback
path of any kind.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspk.so")

# enum spk_dtype
F32, BF16, F64 = 0, 1, 2
# enum spk_op
OP_SPMM, OP_SDDMM, OP_BACKWARD, OP_TRANSPOSE, OP_BSR4, OP_SELECT = 0, 1, 2, 3, 4, 5
# enum spk_variant
VAR_ROWS, VAR_MERGE, VAR_BSR4, VAR_SLAB, VAR_TILE, VAR_SLAB16, VAR_DCSR, VAR_COO = 0, 1, 2, 3, 4, 5, 6, 7

STATUS = {
    0: "SPK_OK", -1: "SPK_ERR_NULL", -2: "SPK_ERR_SIZE", -3: "SPK_ERR_DTYPE", -4: "SPK_ERR_LD",
    -5: "SPK_ERR_WORKSPACE", -6: "SPK_ERR_PLAN", -7: "SPK_ERR_HIP", -8: "SPK_ERR_STRUCTURE",
    -9: "SPK_ERR_OP", -10: "SPK_ERR_NO_MODEL",
}


class spk_csr(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("vals_dtype", ctypes.c_int32)]


class spk_plan(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("lanes", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("flags", ctypes.c_int32)]

    def __repr__(self):
        return f"spk_plan(variant={self.variant}, lanes={self.lanes}, chunk={self.chunk}, flags={self.flags})"


class spk_bsr4(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nblocks", ctypes.c_int64),
                ("b_row_ptr", ctypes.c_void_p), ("b_col", ctypes.c_void_p), ("b_vals", ctypes.c_void_p)]


class spk_slab16(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("width", ctypes.c_int64),
                ("nslabs", ctypes.c_int64), ("seg", ctypes.c_void_p), ("apos", ctypes.c_void_p),
                ("col16", ctypes.c_void_p)]


class spk_dcsr(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("nrows", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("order", ctypes.c_void_p)]


class SpkError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({strerror(status)})")


# Every exported symbol with its (argtypes, restype); tests check that each
# one declared in include/spk.h is exported.
_P = ctypes.c_void_p
_I32, _I64, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_CSR_P = ctypes.POINTER(spk_csr)
_PLAN_P = ctypes.POINTER(spk_plan)
SIGNATURES = {
    "spk_workspace_bytes": ([_I32, _CSR_P, _I64, _PLAN_P], _SZ),
    "spk_strerror": ([_I32], ctypes.c_char_p),
    "spmm_csr": ([_CSR_P, _P, _I64, _I32, _I64, _P, _I64, _PLAN_P, _P, _SZ, _P], _I32),
    "spmm_csr_noalloc": ([_CSR_P, _P, _I64, _I32, _I64, _P, _I64, _PLAN_P, _P], _I32),
    "spmm_csr_noalloc_max_bytes": ([], _SZ),
    "sddmm_csr": ([_CSR_P, _P, _I64, _P, _I64, _I32, _I64, _P, _PLAN_P, _P, _SZ, _P], _I32),
    "csr_transpose": ([_CSR_P, _P, _P, _P, _P, _SZ, _P], _I32),
    "spmm_csr_backward": ([_CSR_P, _P, _P, _P, _P, _I64, _P, _I64, _I32, _I64, _P, _I64, _P, _PLAN_P, _PLAN_P,
                           _P, _SZ, _P], _I32),
    "spk_csr_validate": ([_CSR_P, ctypes.POINTER(_I32), _P, _SZ, _P], _I32),
    "csr_to_bsr4_count": ([_CSR_P, _P, ctypes.POINTER(ctypes.c_int64), _P, _SZ, _P], _I32),
    "csr_to_bsr4_fill": ([_CSR_P, _P, _P, _P, _P], _I32),
    "spmm_bsr4": ([ctypes.POINTER(spk_bsr4), _P, _I64, _I32, _I64, _P, _I64, _P], _I32),
    "slab16_workspace_bytes": ([_CSR_P, _I64], _SZ),
    "csr_to_slab16": ([_CSR_P, _I64, _P, _P, _P, _P, _SZ, _P], _I32),
    "spmm_slab16": ([ctypes.POINTER(spk_slab16), _P, _P, _I64, _I32, _I64, _P, _I64, _PLAN_P, _P], _I32),
    "sddmm_slab16": ([ctypes.POINTER(spk_slab16), _P, _P, _I64, _P, _I64, _I32, _I64, _P, _PLAN_P, _P], _I32),
    "sddmm_softmax_spmm": ([_CSR_P, _P, _I64, _P, _I64, _I64, _P, _I64, _I64, _I32, _P, _I64, _P, _PLAN_P, _P, _SZ,
                            _P], _I32),
    "attention_workspace_bytes": ([_CSR_P, _I64, _PLAN_P], _SZ),
    "csr_row_softmax": ([_CSR_P, _P, _P, _P, _SZ, _P], _I32),
    "row_softmax_workspace_bytes": ([_CSR_P], _SZ),
    "nonempty_order_workspace_bytes": ([_CSR_P], _SZ),
    "csr_nonempty_order": ([_CSR_P, _P, ctypes.POINTER(ctypes.c_int64), _P, _SZ, _P], _I32),
    "spmm_dcsr": ([ctypes.POINTER(spk_dcsr), _P, _I64, _I32, _I64, _P, _I64, _PLAN_P, _P], _I32),
    "sddmm_dcsr": ([ctypes.POINTER(spk_dcsr), _P, _I64, _P, _I64, _I32, _I64, _P, _PLAN_P, _P], _I32),
    "csr_row_index": ([_CSR_P, _P, _P], _I32),
    "sddmm_coo": ([_CSR_P, _P, _P, _I64, _P, _I64, _I32, _I64, _P, _PLAN_P, _P], _I32),
    "plan_count": ([_I32], _I32),
    "plan_of_index": ([_I32, _I32, _I64, _I32, _PLAN_P, ctypes.POINTER(_I32)], _I32),
    "csr_features": ([_CSR_P, _P, _P, _SZ, _P], _I32),
    "selector_inputs": ([_P, _I64, _I32, _P, _P], _I32),
    "mlp_forward": ([_P, _I64, _I64, _I64, _P, _I64, _P, _P], _I32),
    "mlp_workspace_bytes": ([_I64, _I64, _I64, _I64], _SZ),
    "mlp_loss_grad": ([_P, _I64, _I64, _I64, _P, _P, _P, _I64, _P, _P, _P, _SZ, _P], _I32),
    "adam_update": ([_P, _P, _P, _P, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _I64,
                     _P], _I32),
    "selector_load": ([_I32, _P, _I64, _I64, _I64], _I32),
    "plan_select": ([_CSR_P, _I64, _I32, _I32, _PLAN_P, _P, _SZ, _P], _I32),
    "plan_rank": ([_CSR_P, _I64, _I32, _I32, _I32, _PLAN_P, ctypes.POINTER(_I32), _P, _SZ, _P], _I32),
}

_lib = None


def load():
    """Load libspk.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def strerror(status: int) -> str:
    try:
        return load().spk_strerror(status).decode()
    except Exception:  # noqa: BLE001 - only used to decorate an error message
        return "?"


def check(status: int, what: str) -> None:
    if status != 0:
        raise SpkError(status, what)
