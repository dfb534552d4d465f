"""The column-slab form with 16-bit slab-relative columns on the GPU.

The form (the paper's 16-bit in-range column offsets and by-owner packing,
Section III-A, Optimization 1) is integer preprocessing: its GPU build must
equal the oracle's bit for bit.  Products on it compute Eq. 1 and Eq. 2 and
meet the 1e-5 |A||B| gate against the FP64 oracle of the CSR matrix.
"""
import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth
from spk_testutil import TOL_BF16_SRC, TOL_F32, assert_within, host_csr, sub_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    import paper_2604_27985_amd as spk

    assert torch.cuda.is_available()
    return spk


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def pattern(kind, m, n, d, seed):
    if kind == "powerlaw":
        return synth.powerlaw(n, d, 2.1, seed)
    if kind == "block4":
        return synth.block4(m, n, d, seed)
    return synth.bernoulli(m, n, d, seed)


CASES = [("uniform", 3000, 2000, 0.02, 256), ("uniform", 500, 70000, 0.002, 65536), ("powerlaw", 40000, 40000, 16, 4096),
         ("uniform", 333, 777, 0.05, 100), ("uniform", 64, 64, 0.3, 1), ("block4", 1024, 2048, 0.02, 512),
         ("uniform", 7, 5, 0.0, 2)]


@pytest.mark.parametrize("kind,m,n,d,W", CASES)
def test_slab16_build_bit_exact(spk, kind, m, n, d, W):
    A = pattern(kind, m, n, d, 1)
    seg, apos, col16, S = oracle.csr_to_slab16(A.row_ptr, A.col_idx, A.n, W)
    F = spk.csr_to_slab16(spk.CSR.from_host(A), W)
    assert F.nslabs == S
    assert np.array_equal(F.seg.cpu().numpy(), seg)
    assert np.array_equal(F.apos.cpu().numpy(), apos)
    assert np.array_equal(F.col16.cpu().numpy().view(np.uint16), col16)
    assert F.nbytes() == 4 * (S * A.m + 1) + 4 * S * A.m + 2 * A.nnz


@pytest.mark.parametrize("kind,m,n,d,W", CASES)
@pytest.mark.parametrize("K", [64, 36, 1])
def test_spmm_slab16_matches_oracle(spk, kind, m, n, d, W, K):
    A = pattern(kind, m, n, d, 2)
    v = synth.normal(A.nnz, 2, synth.S_VALS)
    B = synth.normal((A.n, K), 2, synth.S_B)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    F = spk.csr_to_slab16(spk.CSR.from_host(A), W)
    Bd, vd = dev(B), dev(v)
    for plan in (None, spk.Plan(5, 4, 0), spk.Plan(5, 16, 0), spk.Plan(5, 64, 0), spk.Plan(5, 16, 0, 1)):
        C = spk.spmm_slab16(F, Bd, vd, plan=plan)
        assert_within(C.cpu().numpy(), C64, M, TOL_F32, f"spmm_slab16 {kind} W={W} K={K} {plan}")
        assert torch.equal(C, spk.spmm_slab16(F, Bd, vd, plan=plan))  # run to run
    P64, PM = oracle.spmm(A.row_ptr, A.col_idx, None, B)
    assert_within(spk.spmm_slab16(F, Bd, None).cpu().numpy(), P64, PM, TOL_F32, "spmm_slab16 pattern")


@pytest.mark.parametrize("kind,m,n,d,W", CASES)
@pytest.mark.parametrize("K", [64, 20, 128])
def test_sddmm_slab16_matches_oracle(spk, kind, m, n, d, W, K):
    A = pattern(kind, m, n, d, 3)
    v = synth.normal(A.nnz, 3, synth.S_VALS)
    U = synth.normal((A.m, K), 3, synth.S_U)
    V = synth.normal((A.n, K), 3, synth.S_V)
    S64, M = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    F = spk.csr_to_slab16(spk.CSR.from_host(A), W)
    Ud, Vd, vd = dev(U), dev(V), dev(v)
    for plan in (None, spk.Plan(5, 8, 0), spk.Plan(5, 32, 0), spk.Plan(5, 16, 0, 1)):
        S = spk.sddmm_slab16(F, Ud, Vd, vd, plan=plan)
        assert_within(S.cpu().numpy(), S64, M, TOL_F32, f"sddmm_slab16 {kind} W={W} K={K} {plan}")
    P64, PM = oracle.sddmm(A.row_ptr, A.col_idx, None, U, V)
    assert_within(spk.sddmm_slab16(F, Ud, Vd, None).cpu().numpy(), P64, PM, TOL_F32, "sddmm_slab16 pattern")


def test_slab16_bf16_strided_and_empty_runs(spk):
    """BF16 dense operands, leading dimensions above K, empty rows and slabs a
    row never reaches (their C rows keep the earlier slabs' sums)."""
    A = host_csr(6, 300, [[], [299], [0, 1, 2, 150], [], [5, 250, 251], [100]])
    v = synth.normal(A.nnz, 4, synth.S_VALS)
    K, ld = 64, 80
    B32 = synth.normal((300, ld), 4, synth.S_B)
    Br = oracle.round_bf16(B32)
    F = spk.csr_to_slab16(spk.CSR.from_host(A), 64)
    Bd = dev(Br).to(torch.bfloat16)[:, :K]
    C = torch.full((6, ld), 5.0, device="cuda")[:, :K]
    spk.spmm_slab16(F, Bd, dev(v), out=C)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, Br[:, :K])
    assert_within(C.cpu().numpy(), C64, M, TOL_F32, "bf16 strided slab16")
    C_s, M_s = oracle.spmm(A.row_ptr, A.col_idx, v, B32[:, :K])
    assert_within(C.cpu().numpy(), C_s, M_s, TOL_BF16_SRC, "bf16 slab16 vs fp32 sources")
    U32 = synth.normal((6, ld), 4, synth.S_U)
    Ur = oracle.round_bf16(U32)
    S = spk.sddmm_slab16(F, dev(Ur).to(torch.bfloat16)[:, :K], Bd, dev(v))
    S64, SM = oracle.sddmm(A.row_ptr, A.col_idx, v, Ur[:, :K], Br[:, :K])
    assert_within(S.cpu().numpy(), S64, SM, TOL_F32, "bf16 slab16 sddmm")


def test_slab16_argument_errors(spk):
    A = synth.bernoulli(100, 100, 0.05, 5)
    dA = spk.CSR.from_host(A)
    with pytest.raises(spk.SpkError):
        spk.csr_to_slab16(dA, 65537)
    F = spk.csr_to_slab16(dA, 32)
    with pytest.raises(ValueError):
        spk.spmm_slab16(F, torch.ones(100, 8, device="cuda"), None, plan=spk.Plan(0, 16, 0))
    with pytest.raises(spk.SpkError):
        spk.spmm_slab16(F, torch.ones(100, 8, device="cuda"), None, plan=spk.Plan(5, 5, 0))


def test_slab16_full_size_99_percent_sampled(spk):
    """n = 65536 at 99% sparsity, K = 64 and 128: the form at two slab widths
    (2 MiB and 8 MiB of the dense operand per slab at K = 64) against the
    oracle on sampled rows of C and the entries of sampled rows of S."""
    n = 65536
    A = synth.bernoulli(n, n, 0.01, 0)
    v = synth.normal(A.nnz, 0, synth.S_VALS)
    dA = spk.CSR.from_host(A)
    vd = dev(v)
    rows = np.unique(np.concatenate([[0, n - 1], synth.randint(48, n, 12)]))
    srp, sci, idx = sub_rows(A, rows)
    r = torch.from_numpy(rows).cuda()
    e = torch.from_numpy(idx).cuda()
    for K in (64, 128):
        B = synth.normal((n, K), 0, synth.S_B)
        U = synth.normal((n, K), 0, synth.S_U)
        C64, CM = oracle.spmm(srp, sci, v[idx], B)
        S64, SM = oracle.sddmm(srp, sci, v[idx], U[rows], B)
        Bd, Ud = dev(B), dev(U)
        for W in (8192, 32768):
            F = spk.csr_to_slab16(dA, W)
            C = spk.spmm_slab16(F, Bd, vd, plan=spk.Plan(5, 16 if K == 64 else 32, 0))
            assert_within(C[r].cpu().numpy(), C64, CM, TOL_F32, f"full-size spmm_slab16 W={W} K={K}")
            S = spk.sddmm_slab16(F, Ud, Bd, vd)
            assert_within(S[e].cpu().numpy(), S64, SM, TOL_F32, f"full-size sddmm_slab16 W={W} K={K}")
            del F, C, S
    torch.cuda.empty_cache()


@pytest.mark.parametrize("sparsity,K,plans", [
    (0.99, 128, [(5, 32, 4096), (5, 16, 4096)]),
    (0.99, 64, [(5, 16, 8192), (5, 8, 8192)]),
    (0.999, 128, [(5, 32, 16384), (5, 16, 16384)]),
])
def test_sparse_bench_plans_full_size_sampled(spk, sparsity, K, plans):
    """The column-slab plans the 99% and 99.9% bench lines run (SpMM, then
    SDDMM, through spmm / sddmm on the CSR), n = 65536, the bench's seed-0
    operands, on sampled rows of C and the entries of sampled rows of S."""
    n = 65536
    p = synth.uniform_problem(n, 1 - sparsity, K, 0)
    A, v = p.A, p.vals
    dA = spk.CSR.from_host(A, v)
    B, U, V = dev(p.B), dev(p.U), dev(p.V)
    rows = np.unique(np.concatenate([[0, n - 1], synth.randint(96, n, 13)]))
    srp, sci, idx = sub_rows(A, rows)
    C64, CM = oracle.spmm(srp, sci, v[idx], p.B)
    S64, SM = oracle.sddmm(srp, sci, v[idx], p.U[rows], p.V)
    r = torch.from_numpy(rows).cuda()
    e = torch.from_numpy(idx).cuda()
    C = spk.spmm(dA, B, plan=spk.Plan(*plans[0]))
    assert_within(C[r].cpu().numpy(), C64, CM, TOL_F32, f"bench spmm {plans[0]}")
    S = spk.sddmm(dA, U, V, plan=spk.Plan(*plans[1]))
    assert_within(S[e].cpu().numpy(), S64, SM, TOL_F32, f"bench sddmm {plans[1]}")
    del dA, B, U, V, C, S
    torch.cuda.empty_cache()
