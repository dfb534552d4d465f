"""spmm_csr_noalloc through the C ABI against spmm_csr (GPU).

The allocation-free entry point runs the same kernels as spmm_csr with the
library's per-GPU scratch array in place of a caller's workspace: its output
must equal spmm_csr's bit for bit (both deterministic) and meet the 1e-5 gate
against the FP64 oracle, on two calls in a row (the second on a smaller
input, so that the array keeps the first call's contents), and a plan that
needs more scratch than the array holds is refused before any launch.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import _lib, synth
from spk_testutil import TOL_F32, assert_within

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    import paper_2604_27985_amd as spk

    assert torch.cuda.is_available()
    return spk


def noalloc(dA, B, C, plan):
    lib = _lib.load()
    ca = dA.c()
    cp = plan.c() if plan is not None else None
    dt = {torch.float32: _lib.F32, torch.bfloat16: _lib.BF16}[B.dtype]
    return lib.spmm_csr_noalloc(ctypes.byref(ca), ctypes.c_void_p(B.data_ptr()), B.stride(0), dt, B.shape[1],
                                ctypes.c_void_p(C.data_ptr()), C.stride(0), ctypes.byref(cp) if cp else None,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def case(n, mean, K, seed):
    A = synth.powerlaw(n, mean, 2.1, seed)
    v = synth.normal(A.nnz, seed, synth.S_VALS)
    B = synth.normal((n, K), seed, synth.S_B)
    return A, v, B


@pytest.mark.parametrize("plan_args", [(1, 32, 0), (1, 16, 64), (3, 16, 0), (0, 16, 0), None])
def test_noalloc_matches_spmm_csr_twice(spk, plan_args):
    plan = None if plan_args is None else spk.Plan(*plan_args)
    for n, mean, K, seed in ((60000, 16, 128, 1), (7000, 8, 64, 2)):  # the second call is smaller
        print(f"noalloc case plan={plan} n={n} K={K}", flush=True)
        A, v, B = case(n, mean, K, seed)
        dA = spk.CSR.from_host(A, v)
        Bd = torch.from_numpy(B).cuda()
        ref = spk.spmm(dA, Bd, plan=plan)
        C = torch.full((A.m, K), float("nan"), device="cuda")
        st = noalloc(dA, Bd, C, plan)
        assert st == 0, _lib.STATUS.get(st, st)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), "spmm_csr_noalloc differs from spmm_csr"
        C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
        assert_within(C.cpu().numpy(), C64, M, TOL_F32, f"noalloc {plan} n={n}")


def test_noalloc_refuses_oversize_plans(spk):
    lib = _lib.load()
    cap = int(lib.spmm_csr_noalloc_max_bytes())
    assert cap == 64 << 20
    # merge-path shares of 16 items over 600000 one-entry rows at K = 256:
    # 75000 carries of 1 KiB, more than the array holds
    m, n, K = 600000, 16, 256
    rp = np.arange(m + 1, dtype=np.int32)
    ci = (np.arange(m, dtype=np.int32) % n).astype(np.int32)
    A = synth.HostCSR(m, n, rp, ci)
    dA = spk.CSR.from_host(A, np.ones(m, np.float32))
    plan = spk.Plan(1, 64, 16)
    assert spk.workspace_bytes(spk.OP_SPMM, dA, K, plan) > cap
    Bd = torch.ones((n, K), device="cuda")
    C = torch.zeros((m, K), device="cuda")
    assert noalloc(dA, Bd, C, plan) == -5  # SPK_ERR_WORKSPACE, nothing launched
    torch.cuda.synchronize()
    assert not C.any()
