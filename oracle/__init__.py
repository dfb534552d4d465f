"""FP64 CPU oracle for the sparse products (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library never does, and this
package imports nothing from the library: the two share no code.

Each function is a thin numpy wrapper over the plain C loops in ``oracle.c``
(definitions written out in double precision; see that file for the passage
of the paper each one follows).  Inputs are converted to float64 exactly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
NFEAT = 28
_lib = None


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    src = os.path.join(_HERE, "oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-fno-fast-math",
           "-ffp-contract=off", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    global _lib
    _lib = None
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, dbl = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
    lib.oracle_spmm.argtypes = [i64, i64, vp, vp, vp, vp, i64, vp, i64, vp]
    lib.oracle_spmm.restype = None
    lib.oracle_sddmm.argtypes = [i64, i64, vp, vp, vp, vp, i64, vp, i64, vp, vp]
    lib.oracle_sddmm.restype = None
    lib.oracle_csr_transpose.argtypes = [i64, i64, vp, vp, vp, vp, vp]
    lib.oracle_csr_transpose.restype = None
    lib.oracle_spmm_t.argtypes = [i64, i64, i64, vp, vp, vp, vp, i64, vp, i64, vp]
    lib.oracle_spmm_t.restype = None
    lib.oracle_round_bf16.argtypes = [vp, vp, i64]
    lib.oracle_round_bf16.restype = None
    lib.oracle_features.argtypes = [i64, i64, vp, vp, vp]
    lib.oracle_features.restype = None
    lib.oracle_csr_to_bsr4.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
    lib.oracle_csr_to_bsr4.restype = i64
    lib.oracle_mlp_forward.argtypes = [i64, i64, i64] + [vp] * 6 + [i64, vp, vp]
    lib.oracle_mlp_forward.restype = None
    lib.oracle_mlp_loss_grad.argtypes = [i64, i64, i64] + [vp] * 6 + [i64, vp, vp, vp] + [vp] * 6
    lib.oracle_mlp_loss_grad.restype = dbl
    lib.oracle_adam.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, dbl, i64]
    lib.oracle_adam.restype = None
    lib.oracle_selector_inputs.argtypes = [vp, i64, ctypes.c_int32, vp]
    lib.oracle_selector_inputs.restype = None
    lib.oracle_csr_to_slab16.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp]
    lib.oracle_csr_to_slab16.restype = i64
    lib.oracle_sddmm_softmax_spmm.argtypes = [i64, i64, i64, vp, vp, vp, vp, i64, vp, i64, vp, i64, vp, i64, vp, vp, vp]
    lib.oracle_sddmm_softmax_spmm.restype = None
    lib.oracle_nonempty_order.argtypes = [i64, vp, vp]
    lib.oracle_nonempty_order.restype = i64
    lib.oracle_row_index.argtypes = [i64, vp, vp]
    lib.oracle_row_index.restype = None
    lib.oracle_csr_canonical.argtypes = [i64, i64, i64, vp, vp]
    lib.oracle_csr_canonical.restype = ctypes.c_int32
    _lib = lib
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def spmm(row_ptr, col_idx, vals, B, with_bound: bool = True):
    """C = A B in FP64 (Eq. 1).  Returns (C, bound) with bound = |A| |B|."""
    lib = _load()
    rp, ci = _i32(row_ptr), _i32(col_idx)
    m = rp.shape[0] - 1
    B64 = _f64(B)
    K = B64.shape[1]
    v64 = _f64(vals)
    C = np.empty((m, K), np.float64)
    M = np.empty((m, K), np.float64) if with_bound else None
    lib.oracle_spmm(m, K, _p(rp), _p(ci), _p(v64), _p(B64), K, _p(C), K, _p(M))
    return C, M


def sddmm(row_ptr, col_idx, vals, U, V, with_bound: bool = True):
    """S[p] = v_p <U[row p], V[col p]> in FP64 (Eq. 2).  Returns (S, bound)."""
    lib = _load()
    rp, ci = _i32(row_ptr), _i32(col_idx)
    m = rp.shape[0] - 1
    U64, V64 = _f64(U), _f64(V)
    K = U64.shape[1]
    nnz = ci.shape[0]
    S = np.zeros(nnz, np.float64)
    M = np.zeros(nnz, np.float64) if with_bound else None
    v64 = _f64(vals)
    lib.oracle_sddmm(m, K, _p(rp), _p(ci), _p(v64), _p(U64), K, _p(V64), K, _p(S), _p(M))
    return S, M


def csr_transpose(row_ptr, col_idx, n: int):
    """Stable transpose: returns (t_row_ptr[n+1], t_col_idx, perm)."""
    lib = _load()
    rp, ci = _i32(row_ptr), _i32(col_idx)
    m = rp.shape[0] - 1
    nnz = ci.shape[0]
    trp = np.empty(n + 1, np.int32)
    tci = np.empty(nnz, np.int32)
    perm = np.empty(nnz, np.int32)
    lib.oracle_csr_transpose(m, n, _p(rp), _p(ci), _p(trp), _p(tci), _p(perm))
    return trp, tci, perm


def spmm_t(row_ptr, col_idx, vals, G, n: int, with_bound: bool = True):
    """A^T G in FP64, by scatter over A's entries.  Returns (D, bound)."""
    lib = _load()
    rp, ci = _i32(row_ptr), _i32(col_idx)
    m = rp.shape[0] - 1
    G64 = _f64(G)
    K = G64.shape[1]
    D = np.empty((n, K), np.float64)
    M = np.empty((n, K), np.float64) if with_bound else None
    v64 = _f64(vals)
    lib.oracle_spmm_t(m, n, K, _p(rp), _p(ci), _p(v64), _p(G64), K, _p(D), K, _p(M))
    return D, M


def spmm_backward(row_ptr, col_idx, vals, B, G, n: int):
    """Gradients of <A B, G>: returns (dB, dB_bound, dvals, dvals_bound)."""
    dB, dBM = spmm_t(row_ptr, col_idx, vals, G, n)
    dv, dvM = sddmm(row_ptr, col_idx, None, G, B)
    return dB, dBM, dv, dvM


def sddmm_softmax_spmm(row_ptr, col_idx, vals, U, V, B):
    """Attention on A's pattern in FP64: O = softmax_rows(A (.) U V^T) B.
    Returns (O, bound, escale, lse); see oracle.c."""
    lib = _load()
    rp, ci = _i32(row_ptr), _i32(col_idx)
    m = rp.shape[0] - 1
    U64, V64, B64 = _f64(U), _f64(V), _f64(B)
    K1, K2 = U64.shape[1], B64.shape[1]
    O = np.empty((m, K2), np.float64)
    M = np.empty((m, K2), np.float64)
    E = np.empty(m, np.float64)
    L = np.empty(m, np.float64)
    v64 = _f64(vals)
    lib.oracle_sddmm_softmax_spmm(m, K1, K2, _p(rp), _p(ci), _p(v64), _p(U64), K1, _p(V64), K1, _p(B64), K2,
                                  _p(O), K2, _p(M), _p(E), _p(L))
    return O, M, E, L


def nonempty_order(row_ptr):
    """(order[m], nr): non-empty rows ascending, then empty rows ascending."""
    lib = _load()
    rp = _i32(row_ptr)
    m = rp.shape[0] - 1
    order = np.empty(m, np.int32)
    nr = int(lib.oracle_nonempty_order(m, _p(rp), _p(order)))
    return order, nr


def row_index(row_ptr):
    """COO row index of every stored entry."""
    lib = _load()
    rp = _i32(row_ptr)
    m = rp.shape[0] - 1
    out = np.empty(int(rp[m]), np.int32)
    lib.oracle_row_index(m, _p(rp), _p(out))
    return out


def csr_to_slab16(row_ptr, col_idx, n: int, width: int):
    """Slab-major form with 16-bit slab-relative columns: (seg[S m + 1],
    apos[S m], col16[nnz] uint16, S); see oracle.c."""
    lib = _load()
    rp, ci = _i32(row_ptr), _i32(col_idx)
    m = rp.shape[0] - 1
    S = int(lib.oracle_csr_to_slab16(m, n, width, _p(rp), _p(ci), None, None, None))
    seg = np.empty(S * m + 1, np.int32)
    apos = np.empty(S * m, np.int32)
    col16 = np.empty(ci.shape[0], np.uint16)
    lib.oracle_csr_to_slab16(m, n, width, _p(rp), _p(ci), _p(seg), _p(apos), _p(col16))
    return seg, apos, col16, S


# Rules of canonical CSR (bit values of csr_canonical's result).
CSR_BAD_START, CSR_BAD_END, CSR_BAD_ORDER, CSR_BAD_COL, CSR_BAD_SORT, CSR_BAD_DUP = 1, 2, 4, 8, 16, 32


def csr_canonical(row_ptr, col_idx, m: int, n: int, nnz: int | None = None) -> int:
    """OR of the canonical-CSR rules the arrays break (0: canonical); see oracle.c."""
    lib = _load()
    rp = None if row_ptr is None else _i32(row_ptr)
    ci = _i32(col_idx if col_idx is not None else np.zeros(0, np.int32))
    nnz = ci.shape[0] if nnz is None else nnz
    return int(lib.oracle_csr_canonical(m, n, nnz, _p(rp), _p(ci)))


def round_bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (RNE); returned as float32."""
    lib = _load()
    a = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty_like(a)
    lib.oracle_round_bf16(_p(a), _p(out), a.size)
    return out


def features(row_ptr, col_idx, n: int) -> np.ndarray:
    """Integer structural features (see oracle.c for the 28 entries)."""
    lib = _load()
    rp, ci = _i32(row_ptr), _i32(col_idx)
    f = np.zeros(NFEAT, np.int64)
    lib.oracle_features(rp.shape[0] - 1, n, _p(rp), _p(ci), _p(f))
    return f


NIN = 33


def selector_inputs(f, K: int, dtype: int = 0) -> np.ndarray:
    """The 33 scaled selector inputs of integer features f, width K and the
    dense operands' dtype (0 binary32, 1 bfloat16); see oracle.c."""
    lib = _load()
    f64 = np.ascontiguousarray(f, dtype=np.int64)
    x = np.empty(NIN, np.float64)
    lib.oracle_selector_inputs(_p(f64), int(K), int(dtype), _p(x))
    return x


def csr_to_bsr4(row_ptr, col_idx, vals, n: int):
    """4x4 block CSR: returns (b_row_ptr, b_col, b_vals[nb,4,4] float64)."""
    lib = _load()
    rp, ci = _i32(row_ptr), _i32(col_idx)
    m = rp.shape[0] - 1
    mb = (m + 3) // 4
    brp = np.empty(mb + 1, np.int32)
    nb = lib.oracle_csr_to_bsr4(m, n, _p(rp), _p(ci), None, _p(brp), None, None)
    bcol = np.empty(nb, np.int32)
    bv = np.empty((nb, 4, 4), np.float64)
    v64 = _f64(vals)
    lib.oracle_csr_to_bsr4(m, n, _p(rp), _p(ci), _p(v64), _p(brp), _p(bcol), _p(bv))
    return brp, bcol, bv


class MLP:
    """FP64 three-layer perceptron weights (row-major [out][in])."""

    def __init__(self, W1, b1, W2, b2, W3, b3):
        self.W1, self.b1 = _f64(W1), _f64(b1)
        self.W2, self.b2 = _f64(W2), _f64(b2)
        self.W3, self.b3 = _f64(W3), _f64(b3)
        self.H, self.F = self.W1.shape
        self.P = self.W3.shape[0]

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]

    def forward(self, X) -> np.ndarray:
        lib = _load()
        X64 = _f64(X)
        Y = np.empty((X64.shape[0], self.P), np.float64)
        lib.oracle_mlp_forward(self.F, self.H, self.P, *[_p(a) for a in self.params()],
                               X64.shape[0], _p(X64), _p(Y))
        return Y

    def loss_grad(self, X, T, mask):
        lib = _load()
        X64, T64, M64 = _f64(X), _f64(T), _f64(mask)
        grads = [np.empty_like(a) for a in self.params()]
        loss = lib.oracle_mlp_loss_grad(self.F, self.H, self.P, *[_p(a) for a in self.params()],
                                        X64.shape[0], _p(X64), _p(T64), _p(M64),
                                        *[_p(g) for g in grads])
        return loss, grads


def adam(w, g, mom, vel, lr, beta1, beta2, eps, t):
    """In-place Adam step on float64 arrays (Kingma and Ba, Algorithm 1)."""
    lib = _load()
    for a in (w, g, mom, vel):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib.oracle_adam(w.size, _p(w), _p(g), _p(mom), _p(vel), lr, beta1, beta2, eps, t)
