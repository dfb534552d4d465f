"""Seeded synthetic inputs: CSR patterns, values and dense operands.

Both the GPU library and the CPU oracle consume what this module writes; it
contains no arithmetic of the sparse products themselves.  All randomness is
counter-based (see ``spgen.c``), so arrays are identical for a given seed on
any machine and thread count.

Workload shapes follow the paper's evaluation (Section IV-A): random square
sparse matrices at 90-99.9% sparsity with uniformly placed nonzeros, FP32
values and 32-bit column indices (Section III-A), plus the power-law graph
adjacencies the library targets for GNN-style layers.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspgen.so")

# Independent random streams per kind of input.
S_PATTERN = 1
S_VALS = 2
S_B = 3
S_U = 4
S_V = 5
S_G = 6
S_DEG = 7
S_MISC = 8

_lib = None


def build(verbose: bool = False) -> str:
    """Compile libspgen.so with the host C compiler (always recompiles)."""
    import subprocess

    src = os.path.join(_HERE, "spgen.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", src, "-o", tmp, "-lm"]
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
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    i64, u64, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    vp = ctypes.c_void_p
    lib.spgen_bernoulli.argtypes = [i64, i64, dbl, i64, u64, u64, vp, vp, vp]
    lib.spgen_block4.argtypes = [i64, i64, dbl, u64, u64, vp, vp, vp]
    lib.spgen_powerlaw_degrees.argtypes = [i64, i64, dbl, dbl, dbl, u64, u64, vp, vp]
    lib.spgen_distinct_cols.argtypes = [i64, i64, vp, u64, u64, vp]
    lib.spgen_normal_f32.argtypes = [u64, u64, i64, vp]
    lib.spgen_uniform_f32.argtypes = [u64, u64, i64, dbl, dbl, vp]
    lib.spgen_randint.argtypes = [u64, u64, i64, i64, vp]
    lib.spgen_u64.argtypes = [u64, u64, u64, u64]
    lib.spgen_u64.restype = u64
    for f in ("spgen_bernoulli", "spgen_block4", "spgen_powerlaw_degrees",
              "spgen_distinct_cols", "spgen_normal_f32", "spgen_uniform_f32",
              "spgen_randint"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


@dataclass
class HostCSR:
    """A CSR pattern in host memory: int32 row_ptr[m+1], int32 col_idx[nnz]."""

    m: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    kind: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _finish(m, n, lens: np.ndarray, fill, kind: str) -> HostCSR:
    rp64 = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=rp64[1:])
    nnz = int(rp64[-1])
    if nnz >= 2**31:
        raise ValueError(f"nnz={nnz} does not fit int32 indices")
    col = np.empty(nnz, dtype=np.int32)
    rc = fill(rp64, col)
    if rc != 0:
        raise RuntimeError(f"generator failed ({rc})")
    return HostCSR(m, n, rp64.astype(np.int32), col, kind)


def bernoulli(m: int, n: int, density: float, seed: int = 0, band: int | None = None,
              stream: int = S_PATTERN) -> HostCSR:
    """Each entry present independently with probability ``density``.

    With ``band`` set, only |i - j| <= band are candidates.
    """
    lib = _load()
    bw = -1 if band is None else int(band)
    lens = np.empty(m, dtype=np.int64)
    rc = lib.spgen_bernoulli(m, n, float(density), bw, seed, stream, _ptr(lens), None, None)
    if rc != 0:
        raise RuntimeError("spgen_bernoulli count failed")
    fill = lambda rp, col: lib.spgen_bernoulli(m, n, float(density), bw, seed, stream, None,
                                               _ptr(rp), _ptr(col))
    kind = "uniform" if band is None else f"banded{band}"
    return _finish(m, n, lens, fill, kind)


def block4(m: int, n: int, density: float, seed: int = 0, stream: int = S_PATTERN) -> HostCSR:
    """Bernoulli(density) over the 4x4 block grid; chosen blocks are dense."""
    lib = _load()
    lens = np.empty(m, dtype=np.int64)
    if lib.spgen_block4(m, n, float(density), seed, stream, _ptr(lens), None, None) != 0:
        raise RuntimeError("spgen_block4 count failed")
    fill = lambda rp, col: lib.spgen_block4(m, n, float(density), seed, stream, None,
                                            _ptr(rp), _ptr(col))
    return _finish(m, n, lens, fill, "block4")


def powerlaw_degrees(m: int, n: int, mean: float, alpha: float = 2.1, seed: int = 0,
                     tol: float = 0.005) -> tuple[np.ndarray, float]:
    """Zipf-like row degrees, shifted (x_min bisected) to the requested mean."""
    lib = _load()
    deg = np.empty(m, dtype=np.int32)
    xmin = ctypes.c_double(0.0)
    rc = lib.spgen_powerlaw_degrees(m, n, float(alpha), float(mean), float(tol), seed,
                                    S_DEG, _ptr(deg), ctypes.byref(xmin))
    if rc != 0:
        raise RuntimeError("spgen_powerlaw_degrees failed")
    return deg, xmin.value


def fixed_degree(n_cols: int, deg: np.ndarray, seed: int = 0, stream: int = S_PATTERN,
                 kind: str = "fixed") -> HostCSR:
    """Row i gets deg[i] distinct uniformly drawn columns (sorted)."""
    lib = _load()
    m = int(deg.shape[0])
    lens = deg.astype(np.int64)
    fill = lambda rp, col: lib.spgen_distinct_cols(m, n_cols, _ptr(rp), seed, stream, _ptr(col))
    return _finish(m, n_cols, lens, fill, kind)


def powerlaw(n: int, mean: float, alpha: float = 2.1, seed: int = 0) -> HostCSR:
    """Square power-law adjacency: Zipf(alpha) degrees with the given mean."""
    deg, _ = powerlaw_degrees(n, n, mean, alpha, seed)
    return fixed_degree(n, deg, seed, S_PATTERN, kind=f"powerlaw{alpha}")


def normal(shape, seed: int, stream: int) -> np.ndarray:
    """Standard normal float32 array (Box-Muller)."""
    lib = _load()
    out = np.empty(shape, dtype=np.float32)
    lib.spgen_normal_f32(seed, stream, out.size, _ptr(out))
    return out


def uniform(shape, seed: int, stream: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform float32 array on [lo, hi)."""
    lib = _load()
    out = np.empty(shape, dtype=np.float32)
    lib.spgen_uniform_f32(seed, stream, out.size, float(lo), float(hi), _ptr(out))
    return out


def randint(count: int, n: int, seed: int, stream: int = S_MISC) -> np.ndarray:
    lib = _load()
    out = np.empty(count, dtype=np.int64)
    lib.spgen_randint(seed, stream, count, n, _ptr(out))
    return out


# --------------------------------------------------------------------------
# Workload recipes.
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """A sparse matrix with values plus the dense operands of both products."""

    A: HostCSR
    vals: np.ndarray  # float32[nnz]
    K: int
    B: np.ndarray | None = None  # [n, K]
    U: np.ndarray | None = None  # [m, K]
    V: np.ndarray | None = None  # [n, K]
    G: np.ndarray | None = None  # [m, K]
    name: str = ""


def uniform_problem(n: int, density: float, K: int, seed: int = 0, m: int | None = None,
                    dense=("B", "U", "V")) -> Problem:
    """Random matrix, uniform columns, vals ~ N(0,1); dense operands N(0,1)."""
    m = n if m is None else m
    A = bernoulli(m, n, density, seed)
    vals = normal(A.nnz, seed, S_VALS)
    p = Problem(A, vals, K, name=f"uniform m={m} n={n} d={density} K={K} seed={seed}")
    _dense(p, m, n, K, seed, dense)
    return p


def powerlaw_problem(n: int, mean: float, K: int, alpha: float = 2.1, seed: int = 0,
                     dense=("B", "U", "V")) -> Problem:
    """Power-law adjacency, vals ~ U(0,1); dense operands N(0,1)."""
    A = powerlaw(n, mean, alpha, seed)
    vals = uniform(A.nnz, seed, S_VALS)
    p = Problem(A, vals, K, name=f"powerlaw n={n} mean={mean} alpha={alpha} K={K} seed={seed}")
    _dense(p, n, n, K, seed, dense)
    return p


def _dense(p: Problem, m: int, n: int, K: int, seed: int, which) -> None:
    if "B" in which:
        p.B = normal((n, K), seed, S_B)
    if "U" in which:
        p.U = normal((m, K), seed, S_U)
    if "V" in which:
        p.V = normal((n, K), seed, S_V)
    if "G" in which:
        p.G = normal((m, K), seed, S_G)
