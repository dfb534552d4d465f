"""Hyper-sparse forms on the GPU: the doubly compressed row order and the
COO row index (integer preprocessing, bit-exact against the oracle), and
the products over them against the FP64 oracle at 1e-5 |A||B|."""
import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth
from spk_testutil import TOL_F32, assert_within, sub_rows

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


CASES = [(200000, 200000, 2e-6), (50000, 3000, 1e-4), (4000, 4000, 0.001), (3000, 2000, 0.0), (1000, 800, 0.05)]


@pytest.mark.parametrize("m,n,d", CASES)
def test_forms_bit_exact(spk, m, n, d):
    A = synth.bernoulli(m, n, d, 1)
    order, nr = oracle.nonempty_order(A.row_ptr)
    dA = spk.CSR.from_host(A)
    g_order, g_nr = spk.csr_nonempty_order(dA)
    assert g_nr == nr and np.array_equal(g_order.cpu().numpy(), order)
    assert np.array_equal(spk.csr_row_index(dA).cpu().numpy(), oracle.row_index(A.row_ptr))


@pytest.mark.parametrize("m,n,d", CASES)
@pytest.mark.parametrize("K", [64, 36])
def test_products_match_oracle(spk, m, n, d, K):
    A = synth.bernoulli(m, n, d, 2)
    v = synth.normal(A.nnz, 2, synth.S_VALS)
    B = synth.normal((n, K), 2, synth.S_B)
    U = synth.normal((m, K), 2, synth.S_U)
    C64, CM = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    S64, SM = oracle.sddmm(A.row_ptr, A.col_idx, v, U, B)
    dA = spk.CSR.from_host(A, v)
    Bd, Ud = dev(B), dev(U)
    for lanes in (4, 16, 64):
        C = torch.full((m, K), float("nan"), device="cuda")
        spk.spmm(dA, Bd, plan=spk.Plan(6, lanes, 0), out=C)
        assert_within(C.cpu().numpy(), C64, CM, TOL_F32, f"spmm_dcsr l{lanes}")
    for plan in (spk.Plan(6, 8, 0), spk.Plan(6, 32, 0), spk.Plan(7, 8, 0), spk.Plan(7, 16, 5), spk.Plan(7, 16, 64, 1)):
        S = spk.sddmm(dA, Ud, Bd, plan=plan)
        assert_within(S.cpu().numpy(), S64, SM, TOL_F32, f"sddmm {plan}")
        assert torch.equal(S, spk.sddmm(dA, Ud, Bd, plan=plan))
    P64, PM = oracle.sddmm(A.row_ptr, A.col_idx, None, U, B)
    for plan in (spk.Plan(6, 16, 0), spk.Plan(7, 16, 0)):
        assert_within(spk.sddmm(dA, Ud, Bd, plan=plan, pattern=True).cpu().numpy(), P64, PM, TOL_F32, f"pattern {plan}")


def test_bf16_and_strides(spk):
    A = synth.bernoulli(20000, 9000, 2e-4, 3)
    v = synth.normal(A.nnz, 3, synth.S_VALS)
    K, ld = 64, 72
    B32 = synth.normal((9000, ld), 3, synth.S_B)
    U32 = synth.normal((20000, ld), 3, synth.S_U)
    Br, Ur = oracle.round_bf16(B32), oracle.round_bf16(U32)
    dA = spk.CSR.from_host(A, v)
    Bd = dev(Br).to(torch.bfloat16)[:, :K]
    Ud = dev(Ur).to(torch.bfloat16)[:, :K]
    C = torch.full((20000, ld), 7.0, device="cuda")[:, :K]
    spk.spmm(dA, Bd, plan=spk.Plan(6, 16, 0), out=C)
    C64, CM = oracle.spmm(A.row_ptr, A.col_idx, v, Br[:, :K])
    assert_within(C.cpu().numpy(), C64, CM, TOL_F32, "bf16 dcsr spmm")
    S64, SM = oracle.sddmm(A.row_ptr, A.col_idx, v, Ur[:, :K], Br[:, :K])
    for plan in (spk.Plan(6, 16, 0), spk.Plan(7, 16, 0)):
        assert_within(spk.sddmm(dA, Ud, Bd, plan=plan).cpu().numpy(), S64, SM, TOL_F32, f"bf16 {plan}")


def test_full_size_sampled(spk):
    """n = 65536 at 99.9% sparsity, K = 64 and 128 (the sweep's hyper-sparse
    end), and n = 2^20 at density 1e-6 (two thirds of the rows empty)."""
    for n, d, Ks in ((65536, 0.001, (64, 128)), (1 << 20, 1e-6, (64,))):
        A = synth.bernoulli(n, n, d, 0)
        v = synth.normal(A.nnz, 0, synth.S_VALS)
        dA = spk.CSR.from_host(A, v)
        rows = np.unique(np.concatenate([[0, n - 1], synth.randint(200, n, 13)]))
        srp, sci, idx = sub_rows(A, rows)
        r = torch.from_numpy(rows).cuda()
        e = torch.from_numpy(idx).cuda()
        for K in Ks:
            B = synth.normal((n, K), 0, synth.S_B)
            U = synth.normal((n, K), 0, synth.S_U)
            C64, CM = oracle.spmm(srp, sci, v[idx], B)
            S64, SM = oracle.sddmm(srp, sci, v[idx], U[rows], B)
            Bd, Ud = dev(B), dev(U)
            C = spk.spmm(dA, Bd, plan=spk.Plan(6, 16, 0))
            assert_within(C[r].cpu().numpy(), C64, CM, TOL_F32, f"dcsr spmm n={n} K={K}")
            for plan in (spk.Plan(6, 8, 0), spk.Plan(7, 16, 0)):
                S = spk.sddmm(dA, Ud, Bd, plan=plan)
                assert_within(S[e].cpu().numpy(), S64, SM, TOL_F32, f"{plan} n={n} K={K}")
            del Bd, Ud, C, S
        del dA
        torch.cuda.empty_cache()


def test_slab16_past_one_grid(spk):
    """n = 2^21 at density 1e-7, K = 64, on the 2 MiB column-slab plan
    (W = 8192, 8 lanes): its 256 slabs of 65536 row blocks hold 2^32 threads,
    past one grid's 32-bit work-item count, so the SDDMM takes two launches of
    whole slabs.  Every row with an entry in the last slab (the second launch),
    the first and last rows and sampled rows against the oracle, for the SDDMM
    and for the SpMM on the same plan."""
    n, K, W = 1 << 21, 64, 8192
    A = synth.bernoulli(n, n, 1e-7, 0)
    v = synth.normal(A.nnz, 0, synth.S_VALS)
    row_of = np.repeat(np.arange(n), np.diff(A.row_ptr.astype(np.int64)))
    last = np.unique(row_of[A.col_idx >= n - W])
    assert len(last) > 0
    rows = np.unique(np.concatenate([[0, n - 1], last, synth.randint(4000, n, 13)]))
    srp, sci, idx = sub_rows(A, rows)
    U = synth.normal((n, K), 0, synth.S_U)
    V = synth.normal((n, K), 0, synth.S_V)
    S64, SM = oracle.sddmm(srp, sci, v[idx], U[rows], V)
    C64, CM = oracle.spmm(srp, sci, v[idx], V)
    dA = spk.CSR.from_host(A, v)
    Ud, Vd = dev(U), dev(V)
    plan = spk.Plan(5, 8, W)
    S = spk.sddmm(dA, Ud, Vd, plan=plan)
    assert_within(S[torch.from_numpy(idx).cuda()].cpu().numpy(), S64, SM, TOL_F32, "slab16 sddmm n=2^21 W=8192")
    C = spk.spmm(dA, Vd, plan=plan)
    assert_within(C[torch.from_numpy(rows).cuda()].cpu().numpy(), C64, CM, TOL_F32, "slab16 spmm n=2^21 W=8192")
    del dA, Ud, Vd, S, C
    torch.cuda.empty_cache()
