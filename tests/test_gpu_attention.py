"""Attention on A's pattern (SDDMM -> row softmax -> SpMM) on the GPU.

The fused kernel keeps the probabilities on chip; the unfused chain runs
sddmm_csr, csr_row_softmax and spmm_csr.  Both are compared with the FP64
oracle's three-step definition.  The gate follows the arithmetic: a score
carries at most about K1 u E_i of absolute error (E_i the row's largest
|a_p| sum |U||V|, u = 2^-24), which perturbs each probability by a relative
twice that, so |O - O64| <= (1e-5 + 4 K1 u E_i) * sum_p P_p |B_p| elementwise
(the 1e-5 term covers the FP32 sum over the row, as for SpMM).
"""
import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth
from spk_testutil import assert_within, host_csr, sub_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U_ROUND = 2.0 ** -24


@pytest.fixture(scope="module")
def spk():
    import paper_2604_27985_amd as spk

    assert torch.cuda.is_available()
    return spk


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def operands(A, K1, K2, seed):
    """Scores of unit scale: U and V ~ N(0,1) / K1^(1/4), values U(0, 1)."""
    v = synth.uniform(A.nnz, seed, synth.S_VALS)
    s = float(K1) ** -0.25 if K1 > 0 else 1.0
    U = (synth.normal((A.m, K1), seed, synth.S_U) * s).astype(np.float32)
    V = (synth.normal((A.n, K1), seed, synth.S_V) * s).astype(np.float32)
    B = synth.normal((A.n, K2), seed, synth.S_B)
    return v, U, V, B


def check(O, lse, ref, K1, what):
    O64, M, E, L = ref
    tol = (1e-5 + 4 * K1 * U_ROUND * E)[:, None]
    err = np.abs(O.astype(np.float64) - O64)
    bad = err > tol * M
    assert not bad.any(), f"{what}: {int(bad.sum())} of {bad.size} outside; worst {float((err / np.maximum(M, 1e-300)).max())}"
    if lse is not None:
        fin = np.isfinite(L)
        assert np.array_equal(np.isneginf(lse), ~fin), what
        lim = 4 * K1 * U_ROUND * E[fin] + 8 * U_ROUND * np.abs(L[fin]) + 1e-6
        assert np.all(np.abs(lse[fin].astype(np.float64) - L[fin]) <= lim), what


def pattern(kind, m, n, d, seed):
    if kind == "powerlaw":
        return synth.powerlaw(n, d, 2.1, seed)
    return synth.bernoulli(m, n, d, seed)


@pytest.mark.parametrize("kind,m,n,d", [("uniform", 2000, 1500, 0.02), ("powerlaw", 30000, 30000, 16),
                                        ("uniform", 300, 5000, 0.001), ("uniform", 64, 64, 1.0)])
@pytest.mark.parametrize("K1,K2", [(64, 64), (32, 128), (20, 36), (8, 256)])
def test_attention_matches_oracle(spk, kind, m, n, d, K1, K2):
    A = pattern(kind, m, n, d, 1)
    v, U, V, B = operands(A, K1, K2, 1)
    ref = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, v, U, V, B)
    dA = spk.CSR.from_host(A, v)
    Ud, Vd, Bd = dev(U), dev(V), dev(B)
    # NULL = runs of 512 entries; small runs cut most rows into pieces
    plans = [None, spk.Plan(0, 4, 0), spk.Plan(0, 16, 0), spk.Plan(0, 64, 0), spk.Plan(0, 8, 0, 1),
             spk.Plan(1, 8, 7), spk.Plan(1, 16, 64), spk.Plan(1, 4, 1000), spk.Plan(1, 32, 3, 1)]
    for plan in plans:
        try:
            O, lse = spk.attention(dA, Ud, Vd, Bd, plan=plan, with_lse=True)
        except spk.SpkError:
            vec = 1 if (plan is not None and plan.flags & 1) or K1 % 4 or K2 % 4 else 4
            assert plan is not None and plan.lanes * vec * 8 < max(K1, K2), plan  # too wide for the plan
            continue
        check(O.cpu().numpy(), lse.cpu().numpy(), ref, K1, f"fused {kind} K1={K1} K2={K2} {plan}")
        assert torch.equal(O, spk.attention(dA, Ud, Vd, Bd, plan=plan))  # run to run
    if K1 % 4 == 0:
        O = spk.attention_unfused(dA, Ud, Vd, Bd)
        check(O.cpu().numpy(), None, ref, K1, f"unfused {kind} K1={K1} K2={K2}")
    ref1 = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, None, U, V, B)
    check(spk.attention(dA, Ud, Vd, Bd, pattern=True).cpu().numpy(), None, ref1, K1, "fused pattern")


def test_attention_fold_boundaries(spk):
    """Runs of 16 entries: a row of exactly 64 pieces (combined directly), rows
    of 65 and 66 pieces (folded 64 at a time, then a partial fold), a short
    row, an empty row and a row of 188 pieces, against the oracle."""
    n = 4096
    lens = [1024, 1040, 1041, 5, 0, 3000]
    A = host_csr(len(lens), n, [list(range(k)) for k in lens])
    rp = A.row_ptr.astype(np.int64)
    pieces = [(rp[i + 1] - 1) // 16 + 1 - rp[i] // 16 if lens[i] else 0 for i in range(len(lens))]
    assert pieces[:3] == [64, 65, 66] and pieces[5] > 64
    v, U, V, B = operands(A, 64, 64, 5)
    ref = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, v, U, V, B)
    dA = spk.CSR.from_host(A, v)
    O, lse = spk.attention(dA, dev(U), dev(V), dev(B), plan=spk.Plan(1, 8, 16), with_lse=True)
    check(O.cpu().numpy(), lse.cpu().numpy(), ref, 64, "fold boundaries")


def test_attention_many_folds(spk):
    """A row of 80000 entries in runs of 3: 26667 pieces, 417 folds of 64,
    which the fix-up combines in several batches; beside it short and empty
    rows."""
    rows = [[3, 9], list(range(80000)), [], [79999], list(range(0, 80000, 1000))]
    A = host_csr(len(rows), 80000, rows)
    v, U, V, B = operands(A, 16, 16, 9)
    ref = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, v, U, V, B)
    dA = spk.CSR.from_host(A, v)
    for plan in (spk.Plan(1, 8, 3), spk.Plan(1, 4, 5)):
        O, lse = spk.attention(dA, dev(U), dev(V), dev(B), plan=plan, with_lse=True)
        check(O.cpu().numpy(), lse.cpu().numpy(), ref, 16, f"many folds {plan}")


def test_attention_and_softmax_workspace_sizes(spk):
    """Caller workspaces: one byte short is refused before any launch; the
    exact size gives the same bits as the library-sized call (entry-split
    attention with runs of 16, so the long rows' folds are in use)."""
    A = synth.powerlaw(3000, 16, 2.1, 7)
    v, U, V, B = operands(A, 32, 32, 7)
    dA = spk.CSR.from_host(A, v)
    Ud, Vd, Bd = dev(U), dev(V), dev(B)
    plan = spk.Plan(1, 8, 16)
    nb = spk.attention_workspace_bytes(dA, 32, plan)
    assert nb > 0
    ref = spk.attention(dA, Ud, Vd, Bd, plan=plan)
    with pytest.raises(spk.SpkError):
        spk.attention(dA, Ud, Vd, Bd, plan=plan, workspace=torch.empty(nb - 1, dtype=torch.uint8, device="cuda"))
    O = spk.attention(dA, Ud, Vd, Bd, plan=plan, workspace=torch.empty(nb, dtype=torch.uint8, device="cuda"))
    assert torch.equal(O, ref)
    S = spk.sddmm(dA, Ud, Vd)
    P_ref = spk.csr_row_softmax(dA, S.clone())
    from paper_2604_27985_amd import _lib
    import ctypes
    ns = int(_lib.load().row_softmax_workspace_bytes(ctypes.byref(dA.c(use_vals=False))))
    with pytest.raises(spk.SpkError):
        spk.csr_row_softmax(dA, S.clone(), workspace=torch.empty(ns - 1, dtype=torch.uint8, device="cuda"))
    P = spk.csr_row_softmax(dA, S.clone(), workspace=torch.empty(ns, dtype=torch.uint8, device="cuda"))
    assert torch.equal(P, P_ref)


def test_attention_bf16_empty_rows_and_strides(spk):
    A = host_csr(7, 40, [[], [3], [0, 1, 2, 39], [], [5, 6, 30], [7], list(range(0, 40, 2))])
    K1, K2, ld = 32, 64, 72
    v, U, V, B = operands(A, K1, K2, 2)
    Ur, Vr, Br = oracle.round_bf16(U), oracle.round_bf16(V), oracle.round_bf16(B)
    ref = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, v, Ur, Vr, Br)
    pad = lambda x: np.pad(x, ((0, 0), (0, ld - x.shape[1])))  # noqa: E731
    Ud = dev(pad(Ur)).to(torch.bfloat16)[:, :K1]
    Vd = dev(pad(Vr)).to(torch.bfloat16)[:, :K1]
    Bd = dev(pad(Br)).to(torch.bfloat16)[:, :K2]
    O = torch.full((7, ld), 9.0, device="cuda")[:, :K2]
    for plan in (None, spk.Plan(1, 8, 2), spk.Plan(0, 8, 0)):
        O.fill_(9.0)
        _, lse = spk.attention(spk.CSR.from_host(A, v), Ud, Vd, Bd, out=O, with_lse=True, plan=plan)
        check(O.cpu().numpy(), lse.cpu().numpy(), ref, K1, f"bf16 strided {plan}")
        assert not O[0].any() and not O[3].any()
    # no stored entries at all
    E = synth.HostCSR(5, 9, np.zeros(6, np.int32), np.zeros(0, np.int32))
    O, lse = spk.attention(spk.CSR.from_host(E, np.zeros(0, np.float32)), dev(U[:5]), dev(V[:9]), dev(B[:9]),
                           with_lse=True)
    assert not O.any() and bool(torch.isneginf(lse).all())


@pytest.mark.parametrize("kind", ["powerlaw", "short", "hub", "long"])
def test_row_softmax_matches_oracle(spk, kind):
    """Every row's probabilities and log-normaliser.  "short": rows of about
    three entries and many empty rows, so one run of scores spans hundreds of
    rows; "hub": one row of every column beside single-entry rows; "long": a
    row of 80000 entries, cut into more than 256 runs, whose pieces the
    fix-up combines in several batches."""
    if kind == "powerlaw":
        A = synth.powerlaw(20000, 16, 2.1, 3)
    elif kind == "short":
        A = synth.bernoulli(30000, 30000, 1e-4, 3)
    elif kind == "hub":
        rows = [[j] for j in range(0, 3000, 7)] + [list(range(3000))] + [[], [5]] * 50
        A = host_csr(len(rows), 3000, rows)
    else:
        rows = [[3, 9], list(range(80000)), [], [79999]]
        A = host_csr(len(rows), 80000, rows)
    v, U, V, B = operands(A, 16, 4, 3)
    S64, _ = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    dA = spk.CSR.from_host(A, v)
    S = spk.sddmm(dA, dev(U), dev(V))
    P, lse = spk.csr_row_softmax(dA, S, with_lse=True)
    _, _, E, L = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, v, U, V, B)
    fin = np.isfinite(L)
    assert np.array_equal(np.isneginf(lse.cpu().numpy()), ~fin)
    assert np.all(np.abs(lse.cpu().numpy()[fin] - L[fin]) <= 4 * 16 * U_ROUND * E[fin] + 8 * U_ROUND * np.abs(L[fin]) + 1e-6)
    # reference probabilities of every entry, row by row in FP64
    lens = A.row_lengths()
    rows = np.repeat(np.arange(A.m), lens)
    nz = lens > 0
    mx = np.full(A.m, -np.inf)
    mx[nz] = np.maximum.reduceat(S64, A.row_ptr[:-1][nz])
    ex = np.exp(S64 - mx[rows])
    tot = np.zeros(A.m)
    tot[nz] = np.add.reduceat(ex, A.row_ptr[:-1][nz])
    p = ex / tot[rows]
    got = P.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - p) <= (1e-5 + 4 * 16 * U_ROUND * E[rows]) * p + 1e-7)


def test_attention_full_size_sampled(spk):
    """Power-law graph n = 262144, mean degree 16, K = 64: sampled rows
    (with the longest ones) of the fused and unfused chains."""
    n, K = 262144, 64
    A = synth.powerlaw(n, 16, 2.1, 0)
    v, U, V, B = operands(A, K, K, 0)
    dA = spk.CSR.from_host(A, v)
    Ud, Vd, Bd = dev(U), dev(V), dev(B)
    rows = np.unique(np.concatenate([synth.randint(300, n, 9), np.argsort(A.row_lengths())[-4:]]))
    srp, sci, idx = sub_rows(A, rows)
    ref = oracle.sddmm_softmax_spmm(srp, sci, v[idx], U[rows], V, B)
    r = torch.from_numpy(rows).cuda()
    for plan in (None, spk.Plan(1, 8, 128), spk.Plan(0, 16, 0)):
        O, lse = spk.attention(dA, Ud, Vd, Bd, plan=plan, with_lse=True)
        check(O[r].cpu().numpy(), lse[r].cpu().numpy(), ref, K, f"full-size fused {plan}")
    O = spk.attention_unfused(dA, Ud, Vd, Bd)
    check(O[r].cpu().numpy(), None, ref, K, "full-size unfused")
    del dA, Ud, Vd, Bd, O
    torch.cuda.empty_cache()
