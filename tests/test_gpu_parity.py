"""Parity of the HIP kernels with the FP64 oracle (GPU).

Every product is called through the C ABI (via the binding) and compared
element by element with the oracle on the same seeded inputs.
"""
import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth
from spk_testutil import TOL_F32, TOL_F64, assert_within, host_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPMM_PLANS = [(v, l) for v in (0, 1, 3) for l in (4, 8, 16, 32, 64)]
CHUNK = {0: 0, 1: 96, 3: 100}  # merge: entries + rows per group; slab: columns per slab


@pytest.fixture(scope="module")
def spk():
    import paper_2604_27985_amd as spk

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return spk


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def problem(m, n, d, K, seed, kind="uniform"):
    if kind == "uniform":
        A = synth.bernoulli(m, n, d, seed)
    elif kind == "powerlaw":
        A = synth.powerlaw(n, d, 2.1, seed)
    elif kind == "banded":
        A = synth.bernoulli(m, n, d, seed, band=64)
    else:
        A = synth.block4(m, n, d, seed)
    v = synth.normal(A.nnz, seed, synth.S_VALS)
    B = synth.normal((A.n, K), seed, synth.S_B)
    U = synth.normal((A.m, K), seed, synth.S_U)
    return A, v, B, U


def run_spmm(spk, A, v, B, plan=None, pattern=False):
    dA = spk.CSR.from_host(A, None if pattern else v)
    C = spk.spmm(dA, dev(B), plan=plan)
    torch.cuda.synchronize()
    return C.cpu().numpy()


# ------------------------------------------------------------------ SpMM
@pytest.mark.parametrize("variant,lanes", SPMM_PLANS)
def test_spmm_config1_every_plan(spk, variant, lanes):
    """1024 x 1024 at 90% sparsity, K = 64, seed 0: every row-split and merge plan."""
    A, v, B, _ = problem(1024, 1024, 0.1, 64, 0)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    for flags in (0, 1):
        plan = spk.Plan(variant, lanes, CHUNK[variant], flags)
        C = run_spmm(spk, A, v, B, plan)
        assert_within(C, C64, M, TOL_F32, f"spmm {plan.name()}")
    if variant == 3:  # default slab width (one slab here) and a width of 1 column
        for chunk in (0, 1):
            assert_within(run_spmm(spk, A, v, B, spk.Plan(3, lanes, chunk)), C64, M, TOL_F32, f"slab c{chunk}")


@pytest.mark.parametrize("m,n,d,K", [(1000, 777, 0.02, 1), (333, 1000, 0.05, 3), (517, 517, 0.03, 36),
                                     (2049, 1500, 0.01, 100), (700, 900, 0.02, 128), (300, 4000, 0.01, 256),
                                     (257, 513, 0.05, 300), (5, 3, 0.5, 7)])
def test_spmm_ragged_shapes(spk, m, n, d, K):
    A, v, B, _ = problem(m, n, d, K, 3)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    for plan in (None, spk.Plan(1, 8, 64), spk.Plan(0, 64), spk.Plan(3, 16, 128)):
        C = run_spmm(spk, A, v, B, plan)
        assert_within(C, C64, M, TOL_F32, f"spmm {m}x{n} K={K} {plan}")


@pytest.mark.parametrize("K,lanes", [(64, 16), (128, 32), (32, 8), (256, 64), (36, 16), (64, 64), (8, 4)])
@pytest.mark.parametrize("kind,m,n,d", [("uniform", 3001, 2500, 0.05), ("powerlaw", 6000, 6000, 12),
                                        ("block4", 1024, 4096, 0.02), ("uniform", 7, 5, 0.5)])
def test_spmm_tile(spk, K, lanes, kind, m, n, d):
    """LDS-staged slabs: default, odd and one-column slab widths; 4 or 8 rows per lane group."""
    A, v, B, _ = problem(m, n, d, K, 8, kind)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    for chunk in (0, 7, 1, 31):  # widths within the two-buffer LDS budget (32 rows at K = 256)
        for flags in (0, 2):
            C = run_spmm(spk, A, v, B, spk.Plan(4, lanes, chunk, flags))
            assert_within(C, C64, M, TOL_F32, f"tile K={K} lanes={lanes} chunk={chunk} flags={flags}")


@pytest.mark.parametrize("K", [64, 32, 128])
@pytest.mark.parametrize("kind,m,n,d", [("uniform", 3001, 2500, 0.05), ("powerlaw", 6000, 6000, 12),
                                        ("block4", 1024, 4096, 0.02), ("uniform", 7, 5, 0.5)])
def test_spmm_tile_quad_split(spk, K, kind, m, n, d):
    """One entry per 4-lane quad (flags bit 2), 4 or 8 rows per group: default, odd and one-row slabs."""
    A, v, B, _ = problem(m, n, d, K, 13, kind)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    # flags 12: 512-thread workgroups with two rows per group
    for chunk in (0, 7, 1, 31):
        for flags in (4, 6, 12):
            plan = spk.Plan(4, 16, chunk, flags)
            assert_within(run_spmm(spk, A, v, B, plan), C64, M, TOL_F32, f"quad spmm K={K} {plan.name()}")
    P64, PM = oracle.spmm(A.row_ptr, A.col_idx, None, B)
    assert_within(run_spmm(spk, A, v, B, spk.Plan(4, 16, 5, 4), pattern=True), P64, PM, TOL_F32,
                  "quad spmm pattern")


@pytest.mark.parametrize("kind", ["uniform", "powerlaw"])
def test_tile_quad_wide_slabs(spk, kind):
    """Wide quad plans (flags 12): slabs above 32 KiB run in 1024-thread
    workgroups (512-byte rows always), up to 64 KiB of B per slab (128 KiB of
    LDS for the two buffers), also ragged last slabs; other plans keep the
    64 KiB budget."""
    for K, chunks in ((128, (128, 100, 64)), (64, (256, 200, 128)), (32, (512, 300))):
        A, v, B, U = problem(3000, 2500, 0.05 if kind == "uniform" else 8, K, 16, kind)
        C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
        S64, SM = oracle.sddmm(A.row_ptr, A.col_idx, v, U, B)
        for chunk in chunks:
            plan = spk.Plan(4, 16, chunk, 12)
            assert_within(run_spmm(spk, A, v, B, plan), C64, M, TOL_F32, f"wide quad spmm K={K} {plan.name()}")
            assert_within(run_sddmm(spk, A, v, U, B, plan), S64, SM, TOL_F32, f"wide quad sddmm K={K} {plan.name()}")
        for plan in (spk.Plan(4, 16, chunks[0], 4), spk.Plan(4, 16, chunks[0] + 1, 12)):
            with pytest.raises(spk.SpkError) as e:
                run_spmm(spk, A, v, B, plan)
            assert e.value.status == -6


@pytest.mark.parametrize("K,lanes", [(48, 16), (256, 64), (16, 4), (8, 4)])
def test_tile_quad_flag_falls_back_to_plain_split(spk, K, lanes):
    """Rows other than 128, 256 or 512 bytes run the plain TILE split with the plan's lanes."""
    A, v, B, U = problem(1500, 1200, 0.03, K, 14)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    for flags in (4, 6):
        assert_within(run_spmm(spk, A, v, B, spk.Plan(4, lanes, 0, flags)), C64, M, TOL_F32, f"fallback K={K}")
    S64, SM = oracle.sddmm(A.row_ptr, A.col_idx, v, U, B)
    sl = max(lanes, 16)
    assert_within(run_sddmm(spk, A, v, U, B, spk.Plan(4, sl, 0, 6)), S64, SM, TOL_F32, f"fallback sddmm K={K}")


def test_spmm_tile_rejects_unfit_plans(spk):
    A, v, B, _ = problem(100, 100, 0.1, 64, 1)
    for plan in (spk.Plan(4, 8, 0),      # 8 lanes x 4 < K
                 spk.Plan(4, 16, 1 << 20),  # slab larger than the LDS budget
                 spk.Plan(4, 16, 129, 4),   # one entry per quad: 2 x 129 x 256 B > 64 KiB
                 spk.Plan(4, 16, 0, 16)):   # unknown flag
        with pytest.raises(spk.SpkError) as e:
            run_spmm(spk, A, v, B, plan)
        assert e.value.status == -6
    with pytest.raises(spk.SpkError):  # K not a multiple of 4 floats
        A2, v2, B2, _ = problem(100, 100, 0.1, 30, 1)
        run_spmm(spk, A2, v2, B2, spk.Plan(4, 16, 0))


def test_spmm_pattern_mode_and_empty_rows(spk):
    # rows 0, 3, 4 and the last are empty
    A = host_csr(6, 9, [[], [0, 4, 8], [2], [], [], [1, 2, 3, 4, 5, 6, 7]])
    B = synth.normal((9, 20), 1, synth.S_B)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, None, B)
    for plan in (None, spk.Plan(1, 4, 3), spk.Plan(1, 8, 1), spk.Plan(0, 4), spk.Plan(3, 4, 2), spk.Plan(4, 8, 3),
                 spk.Plan(4, 8, 2, 2)):
        C = run_spmm(spk, A, None, B, plan, pattern=True)
        assert_within(C, C64, M, TOL_F32, "pattern")
        assert not C[[0, 3, 4]].any()


def test_spmm_special_cases_bit_exact(spk):
    """One product per output is a single rounding: identity, permutation, diagonal."""
    n, K = 3000, 64
    B = synth.normal((n, K), 2, synth.S_B)
    eye = synth.HostCSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32))
    pi = np.random.default_rng(0).permutation(n).astype(np.int32)
    perm = synth.HostCSR(n, n, np.arange(n + 1, dtype=np.int32), pi)
    dvals = synth.normal(n, 2, synth.S_VALS)
    for plan in (None, spk.Plan(1, 16, 7), spk.Plan(0, 4, 0, 1), spk.Plan(3, 16, 256), spk.Plan(4, 16, 32),
                 spk.Plan(4, 16, 0, 2)):
        assert np.array_equal(run_spmm(spk, eye, np.ones(n, np.float32), B, plan), B)
        assert np.array_equal(run_spmm(spk, perm, None, B, plan, pattern=True), B[pi])
        C = run_spmm(spk, eye, dvals, B, plan)
        assert np.array_equal(C, (dvals[:, None] * B).astype(np.float32))


def test_spmm_nnz_zero_and_noops(spk):
    A = synth.HostCSR(10, 7, np.zeros(11, np.int32), np.zeros(0, np.int32))
    dA = spk.CSR.from_host(A, np.zeros(0, np.float32))
    C = torch.full((10, 5), 7.0, device="cuda")
    spk.spmm(dA, torch.randn(7, 5, device="cuda"), out=C)
    assert not C.cpu().numpy().any()
    # m = 0 and K = 0 are no-ops
    E = synth.HostCSR(0, 7, np.zeros(1, np.int32), np.zeros(0, np.int32))
    out = spk.spmm(spk.CSR.from_host(E, np.zeros(0, np.float32)), torch.randn(7, 5, device="cuda"))
    assert out.shape == (0, 5)
    A2, v2, _, _ = problem(20, 20, 0.2, 1, 1)
    out = spk.spmm(spk.CSR.from_host(A2, v2), torch.zeros(20, 0, device="cuda"))
    assert out.shape == (20, 0)


def test_spmm_strided_operands(spk):
    """Leading dimensions larger than K (views of wider tensors)."""
    A, v, B, _ = problem(400, 300, 0.05, 40, 4)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    dA = spk.CSR.from_host(A, v)
    Bw = torch.zeros(300, 52, device="cuda")
    Bw[:, :40] = dev(B)
    Cw = torch.full((400, 44), 9.0, device="cuda")
    spk.spmm(dA, Bw[:, :40], out=Cw[:, :40])
    torch.cuda.synchronize()
    out = Cw.cpu().numpy()
    assert_within(out[:, :40], C64, M, TOL_F32, "strided")
    assert (out[:, 40:] == 9.0).all()


@pytest.mark.parametrize("K,lanes", [(64, 16), (128, 32), (32, 8)])
def test_tile_strided_operands(spk, K, lanes):
    """TILE plans, plain and one entry per quad, on views of wider tensors: ldb, ldc, ldu and
    ldv above K (multiples of 16 bytes), outputs outside the view untouched."""
    A, v, B, U = problem(700, 600, 0.05, K, 15)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    S64, SM = oracle.sddmm(A.row_ptr, A.col_idx, v, U, B)
    dA = spk.CSR.from_host(A, v)
    Bw = torch.zeros(600, K + 12, device="cuda")
    Bw[:, :K] = dev(B)
    Uw = torch.zeros(700, K + 20, device="cuda")
    Uw[:, :K] = dev(U)
    for flags in (0, 2, 4, 6):
        Cw = torch.full((700, K + 8), 9.0, device="cuda")
        spk.spmm(dA, Bw[:, :K], plan=spk.Plan(4, lanes, 0, flags), out=Cw[:, :K])
        S = spk.sddmm(dA, Uw[:, :K], Bw[:, :K], plan=spk.Plan(4, max(lanes, 16), 0, flags))
        torch.cuda.synchronize()
        out = Cw.cpu().numpy()
        assert_within(out[:, :K], C64, M, TOL_F32, f"strided tile spmm K={K} flags={flags}")
        assert (out[:, K:] == 9.0).all()
        assert_within(S.cpu().numpy(), S64, SM, TOL_F32, f"strided tile sddmm K={K} flags={flags}")


@pytest.mark.parametrize("kind,n,d", [("powerlaw", 20000, 16), ("banded", 5000, 0.2), ("block4", 4096, 0.01)])
def test_spmm_structured_patterns(spk, kind, n, d):
    A, v, B, _ = problem(n, n, d, 64, 5, kind)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    for plan in (None, spk.Plan(1, 16), spk.Plan(1, 64, 256), spk.Plan(0, 8), spk.Plan(3, 16, 1000)):
        assert_within(run_spmm(spk, A, v, B, plan), C64, M, TOL_F32, f"{kind} {plan}")


def test_spmm_deterministic(spk):
    A, v, B, _ = problem(3000, 3000, 16, 128, 6, "powerlaw")
    for plan in (spk.Plan(0, 32), spk.Plan(1, 32, 100), spk.Plan(3, 32, 300)):
        c1 = run_spmm(spk, A, v, B, plan)
        c2 = run_spmm(spk, A, v, B, plan)
        assert np.array_equal(c1.view(np.uint32), c2.view(np.uint32))


# ------------------------------------------------------------------ SDDMM
def run_sddmm(spk, A, v, U, V, plan=None, pattern=False):
    dA = spk.CSR.from_host(A, v)
    S = spk.sddmm(dA, dev(U), dev(V), plan=plan, pattern=pattern)
    torch.cuda.synchronize()
    return S.cpu().numpy()


@pytest.mark.parametrize("variant", [0, 1, 3])
@pytest.mark.parametrize("lanes", [4, 8, 16, 32, 64])
def test_sddmm_config1_every_plan(spk, variant, lanes):
    """1024 x 1024 at 90% sparsity, U, V 1024 x 64, seed 0: rows, entry-split, slab."""
    A, v, V, U = problem(1024, 1024, 0.1, 64, 0)
    S64, M = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    for chunk in (0, 5, 1000):
        for flags in (0, 1):
            plan = spk.Plan(variant, lanes, chunk, flags)
            if -(-64 // (lanes * (1 if flags else 4))) > 8:
                # more than 8 register slices per lane: the plan is refused before launch
                with pytest.raises(spk.SpkError) as e:
                    run_sddmm(spk, A, v, U, V, plan)
                assert e.value.status == -6
                continue
            S = run_sddmm(spk, A, v, U, V, plan)
            assert_within(S, S64, M, TOL_F32, f"sddmm lanes={lanes} chunk={chunk} flags={flags}")


@pytest.mark.parametrize("m,n,d,K", [(1000, 777, 0.02, 1), (333, 1000, 0.05, 3), (517, 517, 0.03, 36),
                                     (700, 900, 0.02, 128), (300, 4000, 0.01, 256), (257, 513, 0.05, 300)])
def test_sddmm_ragged_and_pattern(spk, m, n, d, K):
    A, v, V, U = problem(m, n, d, K, 7)
    S64, M = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    P64, PM = oracle.sddmm(A.row_ptr, A.col_idx, None, U, V)
    assert_within(run_sddmm(spk, A, v, U, V), S64, M, TOL_F32, "sddmm")
    assert_within(run_sddmm(spk, A, v, U, V, pattern=True), P64, PM, TOL_F32, "sddmm pattern")


def test_sddmm_powerlaw_and_empty_rows(spk):
    A, v, V, U = problem(20000, 20000, 16, 64, 8, "powerlaw")
    S64, M = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    for plan in (None, spk.Plan(1, 16, 64), spk.Plan(1, 4, 1024), spk.Plan(0, 8), spk.Plan(3, 16, 3000)):
        assert_within(run_sddmm(spk, A, v, U, V, plan), S64, M, TOL_F32, f"powerlaw {plan}")
    E = host_csr(7, 5, [[], [], [1, 3], [], [0, 1, 2, 3, 4], [], [4]])
    Ue = synth.normal((7, 12), 1, synth.S_U)
    Ve = synth.normal((5, 12), 1, synth.S_V)
    ve = synth.normal(E.nnz, 1, synth.S_VALS)
    S64, M = oracle.sddmm(E.row_ptr, E.col_idx, ve, Ue, Ve)
    for plan in (None, spk.Plan(1, 4, 1), spk.Plan(1, 4, 3), spk.Plan(0, 4), spk.Plan(3, 4, 2)):
        assert_within(run_sddmm(spk, E, ve, Ue, Ve, plan), S64, M, TOL_F32, "empty rows")


@pytest.mark.parametrize("K,lanes", [(64, 16), (128, 32), (32, 16), (256, 64), (48, 16), (64, 64), (8, 16)])
@pytest.mark.parametrize("kind,m,n,d", [("uniform", 3001, 2500, 0.05), ("powerlaw", 6000, 6000, 12),
                                        ("block4", 1024, 4096, 0.02), ("uniform", 7, 5, 0.5)])
def test_sddmm_tile(spk, K, lanes, kind, m, n, d):
    """LDS-staged slabs of V: default, odd and one-row slab widths; 4 or 8 rows per group; pattern mode."""
    A, v, V, U = problem(m, n, d, K, 11, kind)
    S64, M = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    P64, PM = oracle.sddmm(A.row_ptr, A.col_idx, None, U, V)
    for chunk in (0, 7, 1, 31):  # within the two-buffer LDS budget (32 rows of V at K = 256)
        for flags in (0, 2):
            plan = spk.Plan(4, lanes, chunk, flags)
            assert_within(run_sddmm(spk, A, v, U, V, plan), S64, M, TOL_F32, f"tile sddmm K={K} {plan.name()}")
    assert_within(run_sddmm(spk, A, v, U, V, spk.Plan(4, lanes, 5), pattern=True), P64, PM, TOL_F32,
                  "tile sddmm pattern")


@pytest.mark.parametrize("K", [64, 32, 128])
@pytest.mark.parametrize("kind,m,n,d", [("uniform", 3001, 2500, 0.05), ("powerlaw", 6000, 6000, 12),
                                        ("block4", 1024, 4096, 0.02), ("uniform", 7, 5, 0.5)])
def test_sddmm_tile_quad_split(spk, K, kind, m, n, d):
    """One entry per 4-lane quad (flags bit 2): rows of 128, 256 and 512 bytes, odd and one-row slabs."""
    A, v, V, U = problem(m, n, d, K, 12, kind)
    S64, M = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    for chunk in (0, 7, 1, 31):
        for flags in (4, 6, 12):
            plan = spk.Plan(4, 16, chunk, flags)
            assert_within(run_sddmm(spk, A, v, U, V, plan), S64, M, TOL_F32, f"quad sddmm K={K} {plan.name()}")
    # the quad split uses 16-lane groups whatever the plan's lanes
    assert_within(run_sddmm(spk, A, v, U, V, spk.Plan(4, 64, 0, 4)), S64, M, TOL_F32, "quad sddmm lanes 64")
    P64, PM = oracle.sddmm(A.row_ptr, A.col_idx, None, U, V)
    assert_within(run_sddmm(spk, A, v, U, V, spk.Plan(4, 16, 5, 4), pattern=True), P64, PM, TOL_F32,
                  "quad sddmm pattern")


def test_sddmm_tile_rejects_unfit_plans(spk):
    A, v, V, U = problem(100, 100, 0.1, 64, 1)
    for plan in (spk.Plan(4, 8, 0),      # groups narrower than a 16-lane row
                 spk.Plan(4, 16, 1 << 20),  # slab beyond the LDS budget
                 spk.Plan(4, 16, 0, 1),     # scalar loads are not a TILE option
                 spk.Plan(4, 16, 129, 4),   # one entry per quad: 2 x 129 x 256 B > 64 KiB
                 spk.Plan(4, 16, 0, 16)):   # unknown flag
        with pytest.raises(spk.SpkError) as e:
            run_sddmm(spk, A, v, U, V, plan)
        assert e.value.status == -6
    with pytest.raises(spk.SpkError):  # K above 4 x lanes
        A2, v2, V2, U2 = problem(100, 100, 0.1, 96, 1)
        run_sddmm(spk, A2, v2, U2, V2, spk.Plan(4, 16, 0))


def test_sddmm_tile_empty_rows_and_single_entries(spk):
    E = host_csr(7, 5, [[], [], [1, 3], [], [0, 1, 2, 3, 4], [], [4]])
    Ue = synth.normal((7, 16), 1, synth.S_U)
    Ve = synth.normal((5, 16), 1, synth.S_V)
    ve = synth.normal(E.nnz, 1, synth.S_VALS)
    S64, M = oracle.sddmm(E.row_ptr, E.col_idx, ve, Ue, Ve)
    for plan in (spk.Plan(4, 16, 1), spk.Plan(4, 16, 3), spk.Plan(4, 16, 0, 2), spk.Plan(4, 64, 2)):
        assert_within(run_sddmm(spk, E, ve, Ue, Ve, plan), S64, M, TOL_F32, f"empty rows {plan.name()}")


def test_sddmm_deterministic(spk):
    A, v, V, U = problem(3000, 3000, 0.02, 64, 9)
    s1 = run_sddmm(spk, A, v, U, V)
    s2 = run_sddmm(spk, A, v, U, V)
    assert np.array_equal(s1.view(np.uint32), s2.view(np.uint32))


# ------------------------------------------------------------------ adjoint
def test_adjoint_identity_on_gpu(spk):
    """<SpMM(A, B), G> = <vals, SDDMM(pattern, G, B)> within the summed bounds."""
    A, v, B, _ = problem(2000, 1800, 0.01, 32, 10)
    G = synth.normal((2000, 32), 10, synth.S_G)
    C = run_spmm(spk, A, v, B).astype(np.float64)
    S = run_sddmm(spk, A, v, G, B, pattern=True).astype(np.float64)
    lhs, rhs = float((C * G).sum()), float((v * S).sum())
    _, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    _, PM = oracle.sddmm(A.row_ptr, A.col_idx, None, G, B)
    scale = float((M * np.abs(G)).sum() + (np.abs(v) * PM).sum())
    assert abs(lhs - rhs) <= 2 * TOL_F32 * scale


@pytest.mark.parametrize("K", [40, 100, 200, 300])
def test_merge_fixup_long_runs(spk, K):
    """One row of 5000 entries among short and empty rows, merge-path shares
    of 16 (rows + entries): the long row's carries span hundreds of shares,
    summed in batches of 1, 2 or 4 column blocks of 64 by K (300: one more
    pass over the columns); F32, F64 and BF16 dense operands."""
    n = 6000
    rows = [list(range(0, 5000))] + [[7, 900, 5999], [], [1], list(range(100, 160))] * 20
    A = host_csr(len(rows), n, rows)
    v = synth.normal(A.nnz, 13, synth.S_VALS)
    B = synth.normal((n, K), 13, synth.S_B)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    dA = spk.CSR.from_host(A, v)
    for plan in (spk.Plan(1, 16, 16), spk.Plan(1, 64, 16), spk.Plan(1, 8, 40)):
        C = spk.spmm(dA, dev(B), plan=plan)
        assert_within(C.cpu().numpy(), C64, M, TOL_F32, f"merge long runs K={K} {plan.name()}")
        assert torch.equal(C, spk.spmm(dA, dev(B), plan=plan))  # run to run
    dA64 = spk.CSR.from_host(A, v, vals_dtype=torch.float64)
    C = spk.spmm(dA64, dev(B, torch.float64), plan=spk.Plan(1, 16, 16)).cpu().numpy()
    assert_within(C, C64, M, TOL_F64, f"f64 merge long runs K={K}")
    Br = oracle.round_bf16(B)
    Cr64, Mr = oracle.spmm(A.row_ptr, A.col_idx, v, Br)
    C = spk.spmm(dA, dev(Br).to(torch.bfloat16), plan=spk.Plan(1, 16, 16)).cpu().numpy()
    assert_within(C, Cr64, Mr, TOL_F32, f"bf16 merge long runs K={K}")


# ------------------------------------------------------------------ FP64
def test_f64_kernels_match_oracle(spk):
    A, v, B, U = problem(900, 700, 0.03, 24, 11)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    dA = spk.CSR.from_host(A, v, vals_dtype=torch.float64)
    for plan in (None, spk.Plan(1, 8, 50)):
        C = spk.spmm(dA, dev(B, torch.float64), plan=plan).cpu().numpy()
        assert_within(C, C64, M, TOL_F64, "f64 spmm")
    V = synth.normal((700, 24), 11, synth.S_V)
    S64, SM = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    S = spk.sddmm(dA, dev(U, torch.float64), dev(V, torch.float64)).cpu().numpy()
    assert_within(S, S64, SM, TOL_F64, "f64 sddmm")


@pytest.mark.parametrize("K", [64, 128])
def test_uniform_90_percent_full_size_sampled(spk, K):
    """n = 65536 at 90% sparsity (4.3e8 entries), K = 64 and 128, seed 0: the
    plans the bench times (the learned ones, best of the network's top five,
    and the wide one-entry-per-quad plans its lines recorded) and LDS-slab
    plans, plain and one entry per quad, on sampled rows of C and the entries
    of sampled rows of S."""
    from paper_2604_27985_amd import selector
    from spk_testutil import sub_rows

    n = 65536
    p = synth.uniform_problem(n, 0.1, K, 0)
    A, v = p.A, p.vals
    dA = spk.CSR.from_host(A, v)
    B, U, V = dev(p.B), dev(p.U), dev(p.V)
    rows = np.unique(np.concatenate([[0, n - 1], synth.randint(64, n, 12)]))
    srp, sci, idx = sub_rows(A, rows)
    C64, CM = oracle.spmm(srp, sci, v[idx], p.B)
    S64, SM = oracle.sddmm(srp, sci, v[idx], p.U[rows], p.V)
    r = torch.from_numpy(rows).cuda()
    lo = torch.from_numpy(A.row_ptr[rows].astype(np.int64)).cuda()
    cnt = torch.from_numpy((A.row_ptr[rows + 1] - A.row_ptr[rows]).astype(np.int64)).cuda()
    ent = torch.cat([torch.arange(int(a), int(a) + int(c), device="cuda") for a, c in zip(lo, cnt)])
    if K == 64:
        fixed_spmm = [spk.Plan(4, 16, 128, 12), spk.Plan(4, 16, 64), spk.Plan(4, 16, 128, 2), spk.Plan(4, 16, 64, 4),
                      spk.Plan(4, 16, 64, 6)]
        fixed_sddmm = [spk.Plan(4, 16, 256, 12), spk.Plan(4, 16, 64), spk.Plan(4, 16, 128, 2),
                       spk.Plan(4, 16, 64, 4), spk.Plan(4, 16, 64, 6)]
    else:  # 512-byte rows: 1024-thread workgroups, 64 KiB slabs
        fixed_spmm = [spk.Plan(4, 32, 128, 12), spk.Plan(4, 32, 64, 12), spk.Plan(4, 32, 32, 4)]
        fixed_sddmm = [spk.Plan(4, 32, 128, 12), spk.Plan(4, 32, 64, 12), spk.Plan(4, 32, 32, 6)]
    for plan in [selector.select(dA, K, spk.OP_SPMM, verify=5, B=B)] + fixed_spmm:
        C = spk.spmm(dA, B, plan=plan)
        assert_within(C[r].cpu().numpy(), C64, CM, TOL_F32, f"full-size spmm K={K} {plan.name()}")
        del C
    for plan in [selector.select(dA, K, spk.OP_SDDMM, verify=5, U=U, V=V)] + fixed_sddmm:
        S = spk.sddmm(dA, U, V, plan=plan)
        assert_within(S[ent].cpu().numpy(), S64, SM, TOL_F32, f"full-size sddmm K={K} {plan.name()}")
        del S
    del dA, B, U, V
    torch.cuda.empty_cache()
