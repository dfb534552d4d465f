"""BF16 dense operands with FP32 accumulation against the FP64 oracle (GPU).

Workload shape: power-law adjacency (Zipf 2.1 row degrees, mean 32), values
U(0, 1) in FP32, dense operands N(0, 1) rounded to bfloat16, width 256.
Two comparisons per product:
  (i)  against the oracle on the rounded operands: |err| <= 1e-5 |A| |B|;
  (ii) against the oracle on the unrounded FP32 sources: |err| <= 1e-2 |A| |B|
       elementwise (one bf16 rounding per dense factor is at most 2^-8
       relative, two factors in SDDMM at most 2^-8 (2 + 2^-8)), and the
       normwise relative error is reported and bounded the same way.
"""
import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth
from spk_testutil import TOL_BF16_SRC, TOL_F32, assert_within, sub_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    import paper_2604_27985_amd as spk

    assert torch.cuda.is_available()
    return spk


def bf16_dev(x32):
    """Device bf16 tensor holding exactly oracle.round_bf16(x32)."""
    r = oracle.round_bf16(x32)
    t = torch.from_numpy(r).cuda().to(torch.bfloat16)
    assert np.array_equal(t.float().cpu().numpy(), r)  # the conversion is exact on rounded values
    return t, r


def powerlaw_bf16(n, mean, K, seed):
    A = synth.powerlaw(n, mean, 2.1, seed)
    v = synth.uniform(A.nnz, seed, synth.S_VALS)
    B = synth.normal((n, K), seed, synth.S_B)
    U = synth.normal((n, K), seed, synth.S_U)
    return A, v, B, U


@pytest.mark.parametrize("K,plans", [(256, [None, (1, 64, 0), (1, 32, 0), (0, 32, 0), (3, 32, 0), (4, 64, 0),
                                            (4, 64, 33)]),
                                     (64, [None, (1, 8, 0), (0, 16, 0), (4, 16, 0), (4, 16, 5, 2), (4, 16, 0, 4),
                                           (4, 16, 7, 6)]),
                                     (128, [(4, 32, 0, 4), (4, 32, 9, 6)]),  # one entry per quad, 256-byte rows
                                     (36, [None, (1, 8, 0)])])
def test_spmm_bf16(spk, K, plans):
    A, v, B32, _ = powerlaw_bf16(40000, 32, K, 1)
    Bt, Br = bf16_dev(B32)
    C_r, M_r = oracle.spmm(A.row_ptr, A.col_idx, v, Br)
    C_s, M_s = oracle.spmm(A.row_ptr, A.col_idx, v, B32)
    dA = spk.CSR.from_host(A, v)
    for p in plans:
        plan = None if p is None else spk.Plan(*p)
        C = spk.spmm(dA, Bt, plan=plan).cpu().numpy()
        assert_within(C, C_r, M_r, TOL_F32, f"bf16 spmm rounded {plan}")
        assert_within(C, C_s, M_s, TOL_BF16_SRC, f"bf16 spmm vs fp32 sources {plan}")
        rel = np.linalg.norm(C - C_s) / np.linalg.norm(C_s)
        assert rel <= 2.0 ** -8, rel


@pytest.mark.parametrize("K", [256, 64, 128])
def test_sddmm_bf16(spk, K):
    A, v, V32, U32 = powerlaw_bf16(40000, 32, K, 2)
    Ut, Ur = bf16_dev(U32)
    Vt, Vr = bf16_dev(V32)
    S_r, M_r = oracle.sddmm(A.row_ptr, A.col_idx, v, Ur, Vr)
    S_s, M_s = oracle.sddmm(A.row_ptr, A.col_idx, v, U32, V32)
    dA = spk.CSR.from_host(A, v)
    tl = K // 4  # TILE plans: default and odd slab widths, 4 or 8 rows per group
    # flags bit 2: one entry per quad (two-element BF16 dot products) at K = 64 and 128
    quad = [spk.Plan(4, 16, 0, 4), spk.Plan(4, 16, 11, 6)]  # rows of 128, 256 and 512 bytes
    for plan in [None, spk.Plan(1, 16, 256), spk.Plan(1, 64, 256), spk.Plan(0, 32), spk.Plan(3, 16, 0), spk.Plan(4, tl, 0),
                 spk.Plan(4, tl, 9, 2)] + quad:
        S = spk.sddmm(dA, Ut, Vt, plan=plan).cpu().numpy()
        assert_within(S, S_r, M_r, TOL_F32, f"bf16 sddmm rounded {plan}")
        assert_within(S, S_s, M_s, TOL_BF16_SRC, f"bf16 sddmm vs fp32 sources {plan}")
        rel = np.linalg.norm(S - S_s) / np.linalg.norm(S_s)
        assert rel <= 2.0 ** -8 * (2 + 2.0 ** -8), rel


def test_bf16_full_size_sampled(spk):
    """n = 2^20, mean degree 32, K = 256: sampled rows of C and the entries of
    sampled rows of S, against the oracle on the rounded operands, on the
    plans the bench line of this workload runs (merge-path SpMM at 32 lanes,
    the 8-wide BF16 instantiation; merge-path SDDMM at 64 lanes and 256
    entries per group: the recorded profile's plans), on the network's five
    best plans timed once, and on the NULL plans."""
    from paper_2604_27985_amd import selector

    n, K = 1 << 20, 256
    A, v, B32, U32 = powerlaw_bf16(n, 32, K, 0)
    V32 = B32  # V and B share the draw: the products use them independently
    Bt, Br = bf16_dev(B32)
    Ut, Ur = bf16_dev(U32)
    dA = spk.CSR.from_host(A, v)
    rows = np.unique(np.concatenate([synth.randint(400, n, 7), np.argsort(A.row_lengths())[-3:]]))
    srp, sci, idx = sub_rows(A, rows)
    C_r, M_r = oracle.spmm(srp, sci, v[idx], Br)
    S_r, SM_r = oracle.sddmm(srp, sci, v[idx], Ur[rows], Br)
    r = torch.from_numpy(rows).cuda()
    e = torch.from_numpy(idx).cuda()
    spmm_plans = [spk.Plan(1, 32, 0), selector.select(dA, K, spk.OP_SPMM, verify=5, B=Bt), spk.Plan(1, 64, 0), None]
    sddmm_plans = [spk.Plan(1, 64, 256), selector.select(dA, K, spk.OP_SDDMM, verify=5, U=Ut, V=Bt), None]
    for plan in spmm_plans:
        C = spk.spmm(dA, Bt, plan=plan)
        assert_within(C[r].cpu().numpy(), C_r, M_r, TOL_F32, f"bf16 full C {plan}")
        del C
    for plan in sddmm_plans:
        S = spk.sddmm(dA, Ut, Bt, plan=plan)
        assert_within(S[e].cpu().numpy(), S_r, SM_r, TOL_F32, f"bf16 full S {plan}")
        del S
    del dA, Bt, Ut
    torch.cuda.empty_cache()
