"""C ABI checks that need no GPU: exported symbols and host-side validation.

Every call here fails its O(1) argument checks, which run before any launch,
so the device pointers passed are never dereferenced.
"""
import ctypes
import os
import re

import pytest

from paper_2604_27985_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x100000)  # stand-in device address, never dereferenced


def header_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libspk.so not built")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert {"spmm_csr", "sddmm_csr", "spmm_csr_backward", "csr_transpose"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no binding signature"


def csr(m=10, n=8, nnz=20, vals=True, dt=0):
    return _lib.spk_csr(m, n, nnz, FAKE.value, FAKE.value, FAKE.value if vals else None, dt)


def spmm(A, B=FAKE, ldb=16, bdt=0, K=16, C=FAKE, ldc=16, plan=None, ws=None, nb=0):
    lib = _lib.load()
    return lib.spmm_csr(ctypes.byref(A) if A is not None else None, B, ldb, bdt, K, C, ldc,
                        ctypes.byref(plan) if plan else None, ws, nb, None)


def test_spmm_argument_errors(lib):
    assert spmm(None) == -1
    assert spmm(csr(m=-1)) == -2
    assert spmm(csr(nnz=2**31)) == -2
    assert spmm(csr(), K=-3) == -2
    assert spmm(csr(), B=None) == -1
    assert spmm(csr(), C=None) == -1
    assert spmm(csr(), ldb=8) == -4
    assert spmm(csr(), ldc=15) == -4
    assert spmm(csr(), bdt=7) == -3
    assert spmm(csr(dt=2), bdt=0) == -3           # F64 values with F32 operand
    assert spmm(csr(dt=0), bdt=2) == -3           # F32 values with F64 operand
    assert spmm(csr(), plan=_lib.spk_plan(5, 16, 0, 0)) == -6
    assert spmm(csr(), plan=_lib.spk_plan(0, 12, 0, 0)) == -6
    assert spmm(csr(), plan=_lib.spk_plan(0, 16, 0, 2)) == -6
    assert spmm(csr(), plan=_lib.spk_plan(1, 16, 0, 0)) == -5  # merge needs a workspace
    A = csr()
    need = lib.spk_workspace_bytes(0, ctypes.byref(A), 16, ctypes.byref(_lib.spk_plan(1, 16, 0, 0)))
    assert need > 0
    assert spmm(A, plan=_lib.spk_plan(1, 16, 0, 0), ws=FAKE, nb=need - 1) == -5
    # no-ops return before touching anything
    assert spmm(csr(m=0)) == 0
    assert spmm(csr(), K=0) == 0


def test_tile_plan_limits(lib):
    """TILE plans are refused before launch when they do not fit: groups of K/4
    lanes at least, slabs within the two-buffer LDS budget, a slab spanning
    less than 4 GiB of the dense operand (32-bit copy offsets), and entry
    positions that stay within 32 bits."""
    tile = lambda lanes, chunk, flags=0: _lib.spk_plan(4, lanes, chunk, flags)  # noqa: E731
    assert spmm(csr(), K=64, ldb=64, ldc=64, plan=tile(8, 16)) == -6            # 8 lanes x 4 < 64
    assert spmm(csr(), K=64, ldb=64, ldc=64, plan=tile(16, 129)) == -6          # 2 x 129 x 256 B > 64 KiB
    assert spmm(csr(), K=64, ldb=1 << 25, ldc=64, plan=tile(16, 32)) == -6      # 32 x 2^25 x 4 B = 4 GiB
    assert spmm(csr(), K=64, ldb=64, ldc=64, plan=tile(16, 16, 16)) == -6       # unknown flag
    f = lib.sddmm_csr
    A = csr()
    assert f(ctypes.byref(A), FAKE, 64, FAKE, 1 << 25, 0, 64, FAKE, ctypes.byref(tile(16, 32)), None, 0,
             None) == -6
    assert f(ctypes.byref(A), FAKE, 64, FAKE, 64, 0, 64, FAKE, ctypes.byref(tile(8, 16)), None, 0, None) == -6
    # entries are read at 32-bit positions plus up to 63 lanes: TILE takes nnz
    # up to 2^31 - 65 and refuses more with SPK_ERR_SIZE
    big = csr(nnz=2**31 - 64)
    assert spmm(big, K=64, ldb=64, ldc=64, plan=tile(16, 32)) == -2
    assert spmm(big, K=64, ldb=64, ldc=64, plan=tile(16, 32, 4)) == -2
    assert f(ctypes.byref(big), FAKE, 64, FAKE, 64, 0, 64, FAKE, ctypes.byref(tile(16, 32)), None, 0, None) == -2


def test_mlp_size_limits(lib):
    """The network kernels take F <= 64, H <= 192, P <= 32; larger sizes are
    refused before anything is launched."""
    assert lib.mlp_workspace_bytes(33, 192, 30, 10) > 0
    assert lib.mlp_workspace_bytes(33, 193, 30, 10) == 0
    assert lib.mlp_forward(FAKE, 33, 193, 30, FAKE, 10, FAKE, None) == -2
    assert lib.mlp_forward(FAKE, 65, 64, 30, FAKE, 10, FAKE, None) == -2
    assert lib.mlp_forward(FAKE, 33, 64, 33, FAKE, 10, FAKE, None) == -2


def test_plan_rank_argument_errors(lib):
    """Checked before the device is touched: null outputs, k outside 1..32, K, op."""
    A = csr()
    out = (_lib.spk_plan * 4)()
    count = ctypes.c_int32(-1)
    f = lib.plan_rank
    assert f(ctypes.byref(A), 64, 0, 0, 4, None, ctypes.byref(count), FAKE, 1 << 20, None) == -1
    assert f(ctypes.byref(A), 64, 0, 0, 4, out, None, FAKE, 1 << 20, None) == -1
    assert f(ctypes.byref(A), 64, 0, 0, 0, out, ctypes.byref(count), FAKE, 1 << 20, None) == -2
    assert f(ctypes.byref(A), 64, 0, 0, 33, out, ctypes.byref(count), FAKE, 1 << 20, None) == -2
    assert f(ctypes.byref(A), -1, 0, 0, 4, out, ctypes.byref(count), FAKE, 1 << 20, None) == -2
    assert f(ctypes.byref(A), 64, 7, 0, 4, out, ctypes.byref(count), FAKE, 1 << 20, None) < 0
    assert f(ctypes.byref(A), 64, 0, 9, 4, out, ctypes.byref(count), FAKE, 1 << 20, None) == -3  # dtype
    assert f(None, 64, 0, 0, 4, out, ctypes.byref(count), FAKE, 1 << 20, None) == -1
    assert count.value == -1  # untouched on errors


def test_sddmm_argument_errors(lib):
    A = csr()
    f = lib.sddmm_csr
    assert f(None, FAKE, 16, FAKE, 16, 0, 16, FAKE, None, None, 0, None) == -1
    assert f(ctypes.byref(A), None, 16, FAKE, 16, 0, 16, FAKE, None, None, 0, None) == -1
    assert f(ctypes.byref(A), FAKE, 8, FAKE, 16, 0, 16, FAKE, None, None, 0, None) == -4
    assert f(ctypes.byref(A), FAKE, 16, FAKE, 16, 5, 16, FAKE, None, None, 0, None) == -3
    bad = _lib.spk_plan(0, 4, 0, 0)  # 4 lanes x 4 wide x 8 slices = 128 < K
    assert f(ctypes.byref(A), FAKE, 4096, FAKE, 4096, 0, 4096, FAKE, ctypes.byref(bad), None, 0, None) == -6
    assert f(ctypes.byref(csr(nnz=0)), None, 16, None, 16, 0, 16, None, None, None, 0, None) == 0


def test_transpose_and_backward_argument_errors(lib):
    A = csr()
    assert lib.csr_transpose(ctypes.byref(A), None, FAKE, FAKE, FAKE, 1 << 30, None) == -1
    need = lib.spk_workspace_bytes(3, ctypes.byref(A), 0, None)
    assert need > 0
    assert lib.csr_transpose(ctypes.byref(A), FAKE, FAKE, FAKE, FAKE, need - 1, None) == -5
    bw = lib.spmm_csr_backward
    assert bw(ctypes.byref(A), FAKE, FAKE, FAKE, FAKE, 16, FAKE, 16, 1, 16, FAKE, 16, None, None, None, None, 0,
              None) == -3  # BF16 backward is not offered
    assert bw(ctypes.byref(A), None, FAKE, FAKE, FAKE, 16, FAKE, 16, 0, 16, FAKE, 16, None, None, None, None, 0,
              None) == -1
    assert bw(ctypes.byref(A), FAKE, FAKE, FAKE, FAKE, 16, FAKE, 8, 0, 16, FAKE, 16, None, None, None, None, 0,
              None) == -4
    assert lib.spk_csr_validate(ctypes.byref(A), None, None, 0, None) == -5


def test_workspace_sizes(lib):
    A = csr(m=1000, n=1000, nnz=50000)
    assert lib.spk_workspace_bytes(0, ctypes.byref(A), 64, None) == 0
    assert lib.spk_workspace_bytes(1, ctypes.byref(A), 64, None) == 0
    merge = _lib.spk_plan(1, 16, 256, 0)
    groups = -(-(1000 + 50000) // 256)
    nb = lib.spk_workspace_bytes(0, ctypes.byref(A), 64, ctypes.byref(merge))
    assert nb >= groups * 64 * 4 + 2 * groups * 4
    assert lib.spk_workspace_bytes(9, ctypes.byref(A), 64, None) == 0
    assert lib.spk_strerror(-5).decode().startswith("workspace")


def test_noalloc_argument_errors(lib):
    """The allocation-free SpMM runs spmm_csr's O(1) checks before touching
    the device; its scratch size is stated."""
    na = lib.spmm_csr_noalloc
    assert na(None, FAKE, 16, 0, 16, FAKE, 16, None, None) == -1
    A = csr()
    assert na(ctypes.byref(A), FAKE, 16, 0, 16, FAKE, 8, None, None) == -4
    assert na(ctypes.byref(A), None, 16, 0, 16, FAKE, 16, None, None) == -1
    assert na(ctypes.byref(A), FAKE, 16, 7, 16, FAKE, 16, None, None) == -3
    bad = _lib.spk_plan(1, 5, 0, 0)
    assert na(ctypes.byref(A), FAKE, 16, 0, 16, FAKE, 16, ctypes.byref(bad), None) == -6
    assert lib.spmm_csr_noalloc_max_bytes() == 64 << 20
