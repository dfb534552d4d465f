"""Python binding of the sparse-product library: argument marshalling only.

Every computation runs in the HIP kernels behind the C ABI (include/spk.h);
torch supplies device memory and the current stream.  Nothing here computes
on the host or falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import weakref
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import BF16, F32, F64, OP_BACKWARD, OP_SDDMM, OP_SPMM, OP_TRANSPOSE, VAR_MERGE, VAR_ROWS, VAR_SLAB

_DT = {torch.float32: F32, torch.bfloat16: BF16, torch.float64: F64}


@dataclass(frozen=True)
class Plan:
    """Execution plan (mirrors spk_plan)."""

    variant: int = VAR_ROWS
    lanes: int = 16
    chunk: int = 0
    flags: int = 0

    def c(self) -> _lib.spk_plan:
        return _lib.spk_plan(self.variant, self.lanes, self.chunk, self.flags)

    def name(self) -> str:
        v = {VAR_ROWS: "rows", VAR_MERGE: "merge", 2: "bsr4", VAR_SLAB: "slab", 4: "tile", 5: "slab16", 6: "dcsr",
             7: "coo"}[self.variant]
        s = f"{v}/l{self.lanes}"
        if self.chunk:
            s += f"/c{self.chunk}"
        if self.flags:
            s += f"/f{self.flags}"
        return s

    @classmethod
    def from_name(cls, name: str) -> "Plan":
        """Inverse of name(): "tile/l16/c64/f6" and the like."""
        parts = name.split("/")
        v = {"rows": VAR_ROWS, "merge": VAR_MERGE, "bsr4": 2, "slab": VAR_SLAB, "tile": 4, "slab16": 5, "dcsr": 6,
             "coo": 7}[parts[0]]
        fields = {p[0]: int(p[1:]) for p in parts[1:]}
        return cls(v, fields.get("l", 16), fields.get("c", 0), fields.get("f", 0))


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p | None:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _require_device(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("operands must be device tensors (the library runs on the GPU only)")


def _rowmajor(t: torch.Tensor, name: str) -> None:
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1) or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be a row-major 2-D tensor with unit column stride")


@dataclass
class CSR:
    """A CSR matrix in device memory (int32 indices; vals float32/float64 or None)."""

    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    vals: torch.Tensor | None
    shape: tuple
    _transpose: tuple | None = field(default=None, repr=False)

    @property
    def m(self) -> int:
        return int(self.shape[0])

    @property
    def n(self) -> int:
        return int(self.shape[1])

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @classmethod
    def from_host(cls, A, vals=None, device="cuda", vals_dtype=torch.float32) -> "CSR":
        """From a host pattern (row_ptr, col_idx numpy arrays) and optional values."""
        rp = torch.from_numpy(A.row_ptr).to(device)
        ci = torch.from_numpy(A.col_idx).to(device)
        v = None if vals is None else torch.as_tensor(vals).to(device=device, dtype=vals_dtype)
        return cls(rp, ci, v, (A.m, A.n))

    def with_vals(self, vals: torch.Tensor | None) -> "CSR":
        out = CSR(self.row_ptr, self.col_idx, vals, self.shape)
        out._transpose = self._transpose
        return out

    def c(self, vals: torch.Tensor | None = None, use_vals: bool = True) -> _lib.spk_csr:
        v = self.vals if vals is None else vals
        if not use_vals:
            v = None
        if v is not None:
            if v.dtype not in (torch.float32, torch.float64) or not v.is_contiguous() or v.numel() != self.nnz:
                raise ValueError("vals must be a contiguous float32/float64 tensor with nnz entries")
        for t in (self.row_ptr, self.col_idx):
            if t.dtype != torch.int32 or not t.is_contiguous():
                raise ValueError("row_ptr and col_idx must be contiguous int32 tensors")
        return _lib.spk_csr(self.m, self.n, self.nnz, self.row_ptr.data_ptr(),
                            self.col_idx.data_ptr() if self.nnz else None,
                            None if v is None else v.data_ptr(), F64 if (v is not None and v.dtype == torch.float64) else F32)

    def transpose(self):
        """(at_row_ptr, at_col_idx, perm), computed once per pattern on the GPU."""
        if self._transpose is None:
            self._transpose = csr_transpose(self)
        return self._transpose

    def nonempty_order(self):
        """(order [m] int32, nrows): non-empty rows first, built on the GPU once
        per pattern and cached."""
        if getattr(self, "_order", None) is None:
            self._order = csr_nonempty_order(self)
        return self._order

    def row_index(self) -> torch.Tensor:
        """COO row index of the entries, built on the GPU once per pattern."""
        if getattr(self, "_rowidx", None) is None:
            self._rowidx = csr_row_index(self)
        return self._rowidx

    def dcsr(self, vals: torch.Tensor | None = None, use_vals: bool = True) -> "_lib.spk_dcsr":
        order, nr = self.nonempty_order()
        ca = self.c(vals, use_vals=use_vals)
        if ca.vals is not None and ca.vals_dtype != F32:
            raise ValueError("the hyper-sparse products take float32 values")
        return _lib.spk_dcsr(self.m, self.n, self.nnz, nr, ca.row_ptr, ca.col_idx, ca.vals,
                             order.data_ptr() if order.numel() else None)

    def slab16_form(self, width: int) -> "Slab16":
        """Column-slab form with 16-bit columns at this slab width, built on the
        GPU once per pattern and width and cached (values are not part of it)."""
        cache = getattr(self, "_slab16", None)
        if cache is None:
            cache = self._slab16 = {}
        if width not in cache:
            cache[width] = csr_to_slab16(self, width)
        return cache[width]

    def block_form(self, vals: torch.Tensor | None = None) -> "BSR4":
        """4x4 block form for these values, built on the GPU once and cached.

        The cache is keyed on the values tensor itself (a weak reference, so
        it holds no memory) and its in-place version counter: another tensor,
        even one the allocator placed at the same address, or an in-place
        update of the same tensor, rebuilds the tiles."""
        v = self.vals if vals is None else vals
        cache = getattr(self, "_bsr4", None)
        if cache is not None:
            ref, version, form = cache
            same = (v is None and ref is None) or (v is not None and ref is not None and ref() is v
                                                   and version == v._version)
            if same:
                return form
        form = csr_to_bsr4(self, vals)
        self._bsr4 = (None if v is None else weakref.ref(v), None if v is None else v._version, form)
        return form


def workspace_bytes(op: int, A: CSR, K: int, plan: Plan | None = None) -> int:
    lib = _lib.load()
    ca = A.c(use_vals=False)
    cp = plan.c() if plan is not None else None
    return int(lib.spk_workspace_bytes(op, ctypes.byref(ca), K, ctypes.byref(cp) if cp else None))


def _workspace(op, A, K, plan, device):
    nb = workspace_bytes(op, A, K, plan)
    if nb == 0:
        return None, 0
    return torch.empty(nb, dtype=torch.uint8, device=device), nb


def spmm(A: CSR, B: torch.Tensor, plan: Plan | None = None, out: torch.Tensor | None = None,
         vals: torch.Tensor | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """C = A B (Eq. 1).  B: [n, K] float32/bfloat16 (float64 with float64 values)."""
    lib = _lib.load()
    _require_device(A.row_ptr, B)
    _rowmajor(B, "B")
    if B.shape[0] != A.n:
        raise ValueError(f"B has {B.shape[0]} rows, A has {A.n} columns")
    K = int(B.shape[1])
    odt = torch.float64 if B.dtype == torch.float64 else torch.float32
    C = out if out is not None else torch.empty((A.m, K), dtype=odt, device=B.device)
    _rowmajor(C, "C")
    if plan is not None and plan.variant == _lib.VAR_BSR4:
        # the block form is per-pattern (and per-values) preprocessing, cached on A
        return spmm_bsr4(A.block_form(vals), B, out=C)
    if plan is not None and plan.variant == _lib.VAR_DCSR:
        cd, cp = A.dcsr(vals), plan.c()
        st = lib.spmm_dcsr(ctypes.byref(cd), _ptr(B), B.stride(0), _DT[B.dtype], K, _ptr(C), C.stride(0),
                           ctypes.byref(cp), _stream())
        _lib.check(st, "spmm_dcsr")
        return C
    if plan is not None and plan.variant == _lib.VAR_SLAB16:
        # the slab form is per-pattern preprocessing, cached on A; values stay A's
        F = A.slab16_form(slab16_width(plan, K, B.dtype))
        v = A.vals if vals is None else vals
        return spmm_slab16(F, B, v, plan=Plan(plan.variant, plan.lanes, 0, plan.flags), out=C)
    ca = A.c(vals)
    cp = plan.c() if plan is not None else None
    ws, nb = (workspace, workspace.numel()) if workspace is not None else _workspace(OP_SPMM, A, K, plan, B.device)
    st = lib.spmm_csr(ctypes.byref(ca), _ptr(B), B.stride(0), _DT[B.dtype], K, _ptr(C), C.stride(0),
                      ctypes.byref(cp) if cp else None, _ptr(ws), nb, _stream())
    _lib.check(st, "spmm_csr")
    return C


def sddmm(A: CSR, U: torch.Tensor, V: torch.Tensor, plan: Plan | None = None, out: torch.Tensor | None = None,
          vals: torch.Tensor | None = None, pattern: bool = False,
          workspace: torch.Tensor | None = None) -> torch.Tensor:
    """S[p] = a_p <U[row p], V[col p]> (Eq. 2); pattern=True uses a_p = 1."""
    lib = _lib.load()
    _require_device(A.row_ptr, U, V)
    _rowmajor(U, "U")
    _rowmajor(V, "V")
    if U.shape[0] != A.m or V.shape[0] != A.n or U.shape[1] != V.shape[1] or U.dtype != V.dtype:
        raise ValueError("U must be [m, K] and V [n, K] of one dtype")
    K = int(U.shape[1])
    odt = torch.float64 if U.dtype == torch.float64 else torch.float32
    S = out if out is not None else torch.empty(A.nnz, dtype=odt, device=U.device)
    if plan is not None and plan.variant in (_lib.VAR_DCSR, _lib.VAR_COO):
        cp = plan.c()
        if plan.variant == _lib.VAR_DCSR:
            cd = A.dcsr(vals, use_vals=not pattern)
            st = lib.sddmm_dcsr(ctypes.byref(cd), _ptr(U), U.stride(0), _ptr(V), V.stride(0), _DT[U.dtype], K,
                                _ptr(S), ctypes.byref(cp), _stream())
        else:
            ca = A.c(vals, use_vals=not pattern)
            st = lib.sddmm_coo(ctypes.byref(ca), _ptr(A.row_index()), _ptr(U), U.stride(0), _ptr(V), V.stride(0),
                               _DT[U.dtype], K, _ptr(S), ctypes.byref(cp), _stream())
        _lib.check(st, "sddmm_dcsr" if plan.variant == _lib.VAR_DCSR else "sddmm_coo")
        return S
    if plan is not None and plan.variant == _lib.VAR_SLAB16:
        F = A.slab16_form(slab16_width(plan, K, U.dtype))
        v = None if pattern else (A.vals if vals is None else vals)
        return sddmm_slab16(F, U, V, v, plan=Plan(plan.variant, plan.lanes, 0, plan.flags), out=S)
    ca = A.c(vals, use_vals=not pattern)
    cp = plan.c() if plan is not None else None
    ws, nb = (workspace, workspace.numel()) if workspace is not None else _workspace(OP_SDDMM, A, K, plan, U.device)
    st = lib.sddmm_csr(ctypes.byref(ca), _ptr(U), U.stride(0), _ptr(V), V.stride(0), _DT[U.dtype], K, _ptr(S),
                       ctypes.byref(cp) if cp else None, _ptr(ws), nb, _stream())
    _lib.check(st, "sddmm_csr")
    return S


def csr_transpose(A: CSR):
    """Stable transpose of A's pattern: (at_row_ptr [n+1], at_col_idx [nnz], perm [nnz])."""
    lib = _lib.load()
    _require_device(A.row_ptr)
    dev = A.row_ptr.device
    trp = torch.empty(A.n + 1, dtype=torch.int32, device=dev)
    tci = torch.empty(A.nnz, dtype=torch.int32, device=dev)
    perm = torch.empty(A.nnz, dtype=torch.int32, device=dev)
    ca = A.c(use_vals=False)
    ws, nb = _workspace(OP_TRANSPOSE, A, 0, None, dev)
    st = lib.csr_transpose(ctypes.byref(ca), _ptr(trp), _ptr(tci), _ptr(perm), _ptr(ws), nb, _stream())
    _lib.check(st, "csr_transpose")
    return trp, tci, perm


def backward_workspace_bytes(A: CSR, K: int, plan: Plan | None = None, dvals_plan: Plan | None = None) -> int:
    """Workspace of spmm_backward: its two products run in order and share it."""
    return max(workspace_bytes(OP_BACKWARD, A, K, plan), workspace_bytes(OP_SDDMM, A, K, dvals_plan))


def spmm_backward(A: CSR, B: torch.Tensor, G: torch.Tensor, need_dB: bool = True, need_dvals: bool = True,
                  plan: Plan | None = None, vals: torch.Tensor | None = None, dvals_plan: Plan | None = None,
                  out_dB: torch.Tensor | None = None, out_dvals: torch.Tensor | None = None,
                  workspace: torch.Tensor | None = None):
    """(dB, dvals) of C = A B for dL/dC = G: dB = A^T G, dvals = SDDMM(pattern, G, B).

    plan is a plan for the A^T product (one chosen for A^T, not for A);
    dvals_plan one for the pattern SDDMM on A.  BSR4 plans are not accepted."""
    lib = _lib.load()
    _require_device(A.row_ptr, B, G)
    _rowmajor(B, "B")
    _rowmajor(G, "G")
    if B.dtype != G.dtype or B.dtype not in (torch.float32, torch.float64):
        raise ValueError("B and G must share dtype float32 or float64")
    K = int(B.shape[1])
    trp, tci, perm = A.transpose() if need_dB else (None, None, None)
    dB = None
    if need_dB:
        dB = out_dB if out_dB is not None else torch.empty((A.n, K), dtype=B.dtype, device=B.device)
        _rowmajor(dB, "dB")
    dv = None
    if need_dvals:
        dv = out_dvals if out_dvals is not None else torch.empty(A.nnz, dtype=B.dtype, device=B.device)
    ca = A.c(vals)
    cp = plan.c() if plan is not None else None
    cq = dvals_plan.c() if dvals_plan is not None else None
    if workspace is not None:
        ws, nb = workspace, workspace.numel()
    else:
        nb = backward_workspace_bytes(A, K, plan, dvals_plan)
        ws = torch.empty(nb, dtype=torch.uint8, device=B.device) if nb else None
    st = lib.spmm_csr_backward(ctypes.byref(ca), _ptr(trp), _ptr(tci), _ptr(perm), _ptr(B), B.stride(0), _ptr(G),
                               G.stride(0), _DT[B.dtype], K, _ptr(dB), dB.stride(0) if dB is not None else K,
                               _ptr(dv), ctypes.byref(cp) if cp else None, ctypes.byref(cq) if cq else None,
                               _ptr(ws), nb, _stream())
    _lib.check(st, "spmm_csr_backward")
    return dB, dv


@dataclass
class BSR4:
    """4x4 block-sparse form of a CSR matrix (device arrays)."""

    b_row_ptr: torch.Tensor
    b_col: torch.Tensor
    b_vals: torch.Tensor  # [nblocks, 4, 4] float32
    shape: tuple

    @property
    def nblocks(self) -> int:
        return int(self.b_col.numel())

    def c(self) -> _lib.spk_bsr4:
        return _lib.spk_bsr4(int(self.shape[0]), int(self.shape[1]), self.nblocks, self.b_row_ptr.data_ptr(),
                             self.b_col.data_ptr() if self.nblocks else None,
                             self.b_vals.data_ptr() if self.nblocks else None)


def csr_to_bsr4(A: CSR, vals: torch.Tensor | None = None) -> BSR4:
    """Block form of A on the GPU (count pass synchronises to size the arrays)."""
    lib = _lib.load()
    _require_device(A.row_ptr)
    dev = A.row_ptr.device
    mb = (A.m + 3) // 4
    brp = torch.empty(mb + 1, dtype=torch.int32, device=dev)
    ca = A.c(vals)
    if ca.vals is not None and ca.vals_dtype != F32:
        raise ValueError("the block form holds float32 values")
    ws, nb = _workspace(_lib.OP_BSR4, A, 0, None, dev)
    count = ctypes.c_int64(0)
    _lib.check(lib.csr_to_bsr4_count(ctypes.byref(ca), _ptr(brp), ctypes.byref(count), _ptr(ws), nb, _stream()),
               "csr_to_bsr4_count")
    bcol = torch.empty(count.value, dtype=torch.int32, device=dev)
    bval = torch.empty((count.value, 4, 4), dtype=torch.float32, device=dev)
    _lib.check(lib.csr_to_bsr4_fill(ctypes.byref(ca), _ptr(brp), _ptr(bcol), _ptr(bval), _stream()),
               "csr_to_bsr4_fill")
    return BSR4(brp, bcol, bval, A.shape)


def spmm_bsr4(Ab: BSR4, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """C = A B on matrix cores from the block form."""
    lib = _lib.load()
    _require_device(Ab.b_row_ptr, B)
    _rowmajor(B, "B")
    if B.shape[0] != Ab.shape[1] or B.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("B must be [n, K] float32 or bfloat16")
    K = int(B.shape[1])
    C = out if out is not None else torch.empty((Ab.shape[0], K), dtype=torch.float32, device=B.device)
    _rowmajor(C, "C")
    cb = Ab.c()
    _lib.check(lib.spmm_bsr4(ctypes.byref(cb), _ptr(B), B.stride(0), _DT[B.dtype], K, _ptr(C), C.stride(0),
                             _stream()), "spmm_bsr4")
    return C


@dataclass
class Slab16:
    """Column-slab form with 16-bit slab-relative columns (device arrays).

    seg[S m + 1] run starts (slab-major), apos[S m] A positions of the runs,
    col16[nnz] column offsets (uint16 bits held in an int16 tensor)."""

    seg: torch.Tensor
    apos: torch.Tensor
    col16: torch.Tensor
    shape: tuple
    nnz: int
    width: int
    nslabs: int

    def c(self) -> _lib.spk_slab16:
        return _lib.spk_slab16(int(self.shape[0]), int(self.shape[1]), self.nnz, self.width, self.nslabs,
                               self.seg.data_ptr(), self.apos.data_ptr() if self.apos.numel() else None,
                               self.col16.data_ptr() if self.nnz else None)

    def nbytes(self) -> int:
        """Bytes of the pattern form (values are A's own array)."""
        return 4 * self.seg.numel() + 4 * self.apos.numel() + 2 * self.col16.numel()


def csr_to_slab16(A: CSR, width: int) -> Slab16:
    """Build the slab form of A's pattern on the GPU (once per pattern)."""
    lib = _lib.load()
    _require_device(A.row_ptr)
    dev = A.row_ptr.device
    S = max(1, -(-A.n // width)) if width > 0 else 0
    seg = torch.empty(S * A.m + 1, dtype=torch.int32, device=dev)
    apos = torch.empty(S * A.m, dtype=torch.int32, device=dev)
    col16 = torch.empty(A.nnz, dtype=torch.int16, device=dev)
    ca = A.c(use_vals=False)
    nb = int(lib.slab16_workspace_bytes(ctypes.byref(ca), width))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    _lib.check(lib.csr_to_slab16(ctypes.byref(ca), width, _ptr(seg), _ptr(apos) if apos.numel() else None,
                                 _ptr(col16) if A.nnz else None, _ptr(ws), nb, _stream()), "csr_to_slab16")
    return Slab16(seg, apos, col16, A.shape, A.nnz, width, S)


def slab16_width(plan: Plan, K: int, dtype: torch.dtype) -> int:
    """Slab width of a SLAB16 plan: its chunk, else the power of two (>= 256)
    whose slab of the dense operand takes at most 2 MiB, capped at 65536."""
    if plan.chunk > 0:
        return int(plan.chunk)
    row = max(K, 1) * (2 if dtype == torch.bfloat16 else 4)
    w = 256
    while w * 2 * row <= (2 << 20) and w < 65536:
        w *= 2
    return w


def _slab16_plan(plan: Plan | None):
    if plan is not None and plan.variant != _lib.VAR_SLAB16:
        raise ValueError("slab16 products take SLAB16 plans (variant 5) or None")
    return plan.c() if plan is not None else None


def spmm_slab16(F: Slab16, B: torch.Tensor, vals: torch.Tensor | None, plan: Plan | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """C = A B on the slab form; vals: A's values in A's storage order (None: pattern)."""
    lib = _lib.load()
    _require_device(F.seg, B)
    _rowmajor(B, "B")
    if B.shape[0] != F.shape[1] or B.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("B must be [n, K] float32 or bfloat16")
    if vals is not None and (vals.dtype != torch.float32 or not vals.is_contiguous() or vals.numel() != F.nnz):
        raise ValueError("vals must be a contiguous float32 tensor with nnz entries")
    K = int(B.shape[1])
    C = out if out is not None else torch.empty((F.shape[0], K), dtype=torch.float32, device=B.device)
    _rowmajor(C, "C")
    cf, cp = F.c(), _slab16_plan(plan)
    _lib.check(lib.spmm_slab16(ctypes.byref(cf), _ptr(vals), _ptr(B), B.stride(0), _DT[B.dtype], K, _ptr(C),
                               C.stride(0), ctypes.byref(cp) if cp else None, _stream()), "spmm_slab16")
    return C


def sddmm_slab16(F: Slab16, U: torch.Tensor, V: torch.Tensor, vals: torch.Tensor | None, plan: Plan | None = None,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """S[p] = a_p <U[row p], V[col p]> on the slab form, in A's storage order (vals None: a_p = 1)."""
    lib = _lib.load()
    _require_device(F.seg, U, V)
    _rowmajor(U, "U")
    _rowmajor(V, "V")
    if U.shape[0] != F.shape[0] or V.shape[0] != F.shape[1] or U.shape[1] != V.shape[1] or U.dtype != V.dtype:
        raise ValueError("U must be [m, K] and V [n, K] of one dtype")
    if vals is not None and (vals.dtype != torch.float32 or not vals.is_contiguous() or vals.numel() != F.nnz):
        raise ValueError("vals must be a contiguous float32 tensor with nnz entries")
    K = int(U.shape[1])
    S = out if out is not None else torch.empty(F.nnz, dtype=torch.float32, device=U.device)
    cf, cp = F.c(), _slab16_plan(plan)
    _lib.check(lib.sddmm_slab16(ctypes.byref(cf), _ptr(vals), _ptr(U), U.stride(0), _ptr(V), V.stride(0),
                                _DT[U.dtype], K, _ptr(S), ctypes.byref(cp) if cp else None, _stream()),
               "sddmm_slab16")
    return S


def attention_workspace_bytes(A: CSR, K2: int, plan: Plan | None = None) -> int:
    lib = _lib.load()
    ca = A.c(use_vals=False)
    cp = plan.c() if plan is not None else None
    return int(lib.attention_workspace_bytes(ctypes.byref(ca), K2, ctypes.byref(cp) if cp else None))


def attention(A: CSR, U: torch.Tensor, V: torch.Tensor, B: torch.Tensor, plan: Plan | None = None,
              vals: torch.Tensor | None = None, pattern: bool = False, out: torch.Tensor | None = None,
              with_lse: bool = False, workspace: torch.Tensor | None = None):
    """O = softmax_rows(A (.) U V^T) B in one pass (the probabilities stay on
    chip).  Returns O, or (O, lse) with with_lse."""
    lib = _lib.load()
    _require_device(A.row_ptr, U, V, B)
    for t, nm in ((U, "U"), (V, "V"), (B, "B")):
        _rowmajor(t, nm)
    if U.shape[0] != A.m or V.shape[0] != A.n or B.shape[0] != A.n or U.shape[1] != V.shape[1]:
        raise ValueError("U must be [m, K1], V [n, K1] and B [n, K2]")
    if not (U.dtype == V.dtype == B.dtype) or U.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("U, V and B must share dtype float32 or bfloat16")
    K1, K2 = int(U.shape[1]), int(B.shape[1])
    O = out if out is not None else torch.empty((A.m, K2), dtype=torch.float32, device=B.device)
    _rowmajor(O, "O")
    lse = torch.empty(A.m, dtype=torch.float32, device=B.device) if with_lse else None
    ca = A.c(vals, use_vals=not pattern)
    cp = plan.c() if plan is not None else None
    if workspace is not None:
        ws, nb = workspace, workspace.numel()
    else:
        nb = int(lib.attention_workspace_bytes(ctypes.byref(ca), K2, ctypes.byref(cp) if cp else None))
        ws = torch.empty(nb, dtype=torch.uint8, device=B.device) if nb else None
    _lib.check(lib.sddmm_softmax_spmm(ctypes.byref(ca), _ptr(U), U.stride(0), _ptr(V), V.stride(0), K1, _ptr(B),
                                      B.stride(0), K2, _DT[U.dtype], _ptr(O), O.stride(0), _ptr(lse),
                                      ctypes.byref(cp) if cp else None, _ptr(ws), nb, _stream()),
               "sddmm_softmax_spmm")
    return (O, lse) if with_lse else O


def csr_row_softmax(A: CSR, S: torch.Tensor, with_lse: bool = False, workspace: torch.Tensor | None = None):
    """Row softmax of stored scores S (nnz, A's order) in place; returns S (and lse)."""
    lib = _lib.load()
    _require_device(A.row_ptr, S)
    if S.dtype != torch.float32 or not S.is_contiguous() or S.numel() != A.nnz:
        raise ValueError("S must be a contiguous float32 tensor with nnz entries")
    lse = torch.empty(A.m, dtype=torch.float32, device=S.device) if with_lse else None
    ca = A.c(use_vals=False)
    if workspace is not None:
        ws, nb = workspace, workspace.numel()
    else:
        nb = int(lib.row_softmax_workspace_bytes(ctypes.byref(ca)))
        ws = torch.empty(nb, dtype=torch.uint8, device=S.device) if nb else None
    _lib.check(lib.csr_row_softmax(ctypes.byref(ca), _ptr(S), _ptr(lse), _ptr(ws), nb, _stream()), "csr_row_softmax")
    return (S, lse) if with_lse else S


def attention_unfused(A: CSR, U: torch.Tensor, V: torch.Tensor, B: torch.Tensor, sddmm_plan: Plan | None = None,
                      spmm_plan: Plan | None = None, vals: torch.Tensor | None = None, pattern: bool = False,
                      S: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """The same chain as three launches: sddmm_csr, csr_row_softmax, spmm_csr
    with the probabilities as values (S is written to and read from HBM)."""
    S = sddmm(A, U, V, plan=sddmm_plan, vals=vals, pattern=pattern, out=S)
    csr_row_softmax(A, S)
    return spmm(A, B, plan=spmm_plan, vals=S, out=out)


def csr_nonempty_order(A: CSR):
    """(order [m] int32, nrows): rows holding an entry first, then empty rows."""
    lib = _lib.load()
    _require_device(A.row_ptr)
    dev = A.row_ptr.device
    order = torch.empty(A.m, dtype=torch.int32, device=dev)
    ca = A.c(use_vals=False)
    nb = int(lib.nonempty_order_workspace_bytes(ctypes.byref(ca)))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    nr = ctypes.c_int64(0)
    _lib.check(lib.csr_nonempty_order(ctypes.byref(ca), _ptr(order) if A.m else None, ctypes.byref(nr), _ptr(ws), nb,
                                      _stream()), "csr_nonempty_order")
    return order, int(nr.value)


def csr_row_index(A: CSR) -> torch.Tensor:
    """COO row index of A's entries."""
    lib = _lib.load()
    _require_device(A.row_ptr)
    rowidx = torch.empty(A.nnz, dtype=torch.int32, device=A.row_ptr.device)
    ca = A.c(use_vals=False)
    _lib.check(lib.csr_row_index(ctypes.byref(ca), _ptr(rowidx) if A.nnz else None, _stream()), "csr_row_index")
    return rowidx


def validate_rules(A: CSR) -> int:
    """Opt-in structural check on the GPU (synchronises the stream): the OR of
    the canonical-CSR rules A breaks (spk_csr_rule bits), 0 when canonical."""
    lib = _lib.load()
    ws = torch.empty(16, dtype=torch.uint8, device=A.row_ptr.device)
    ca = A.c(use_vals=False)
    rules = ctypes.c_int32(0)
    st = lib.spk_csr_validate(ctypes.byref(ca), ctypes.byref(rules), _ptr(ws), 16, _stream())
    if st not in (0, -8):
        _lib.check(st, "spk_csr_validate")
    return int(rules.value)


def validate(A: CSR) -> bool:
    """True when A is canonical CSR (see validate_rules)."""
    return validate_rules(A) == 0


class SpMMFunction(torch.autograd.Function):
    """C = A(vals) B with gradients for vals and B from the library's backward.

    The forward plan is chosen for A; the backward's A^T product and pattern
    SDDMM take their own plans (NULL, the plain ones, by default), since a
    plan picked for A says nothing of A^T and a block plan has no transposed
    form."""

    @staticmethod
    def forward(ctx, vals, B, A, plan, backward_plan, dvals_plan):
        C = spmm(A, B, plan=plan, vals=vals)
        ctx.save_for_backward(vals, B)
        ctx.A, ctx.backward_plan, ctx.dvals_plan = A, backward_plan, dvals_plan
        return C

    @staticmethod
    def backward(ctx, G):
        vals, B = ctx.saved_tensors
        G = G.contiguous()
        dB, dv = spmm_backward(ctx.A, B, G, need_dB=ctx.needs_input_grad[1], need_dvals=ctx.needs_input_grad[0],
                               plan=ctx.backward_plan, vals=vals, dvals_plan=ctx.dvals_plan)
        return dv, dB, None, None, None, None


def spmm_autograd(A: CSR, vals: torch.Tensor, B: torch.Tensor, plan: Plan | None = None,
                  backward_plan: Plan | None = None, dvals_plan: Plan | None = None) -> torch.Tensor:
    """Differentiable SpMM in vals and B.  plan: the forward's (any SpMM plan,
    BSR4 included); backward_plan: the A^T product's; dvals_plan: the pattern
    SDDMM's."""
    if backward_plan is not None and backward_plan.variant == _lib.VAR_BSR4:
        raise ValueError("the A^T product has no block plan")
    return SpMMFunction.apply(vals, B, A, plan, backward_plan, dvals_plan)
