"""Shapes past the 32-bit work-item count of one grid.

A one-dimensional launch counts its threads in 32 bits.  The kernels that give
one wave to each row (validation, the transpose's row ids, the COO row index)
stride over the rows past their grid; a launcher whose grid would still pass
2^32 threads returns SPK_ERR_SIZE instead of launching.  The matrix here has
2^26 + 64 rows (one wave per row: 2^32 + 4096 threads) and a few entries, the
last ones in the last rows, so the rows past the first grid are checked against
the oracle: integer work bit for bit, the products (Eq. 2 and Eq. 1) at the
1e-5 |A||B| gate.
"""
import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth
from spk_testutil import TOL_F32, assert_within, sub_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M = (1 << 26) + 64
N = 8
K = 4
ROWS = np.array([0, 5, 5, 1 << 20, (1 << 26) - 1, M - 2, M - 1, M - 1])
COLS = np.array([3, 0, 6, 7, 2, 1, 2, 6], np.int32)


@pytest.fixture(scope="module")
def spk():
    import paper_2604_27985_amd as spk

    assert torch.cuda.is_available()
    return spk


@pytest.fixture(scope="module")
def tall():
    counts = np.bincount(ROWS, minlength=M)
    rp = np.zeros(M + 1, np.int32)
    np.cumsum(counts, out=rp[1:])
    A = synth.HostCSR(M, N, rp, COLS.copy())
    v = synth.normal(A.nnz, 0, synth.S_VALS)
    return A, v


def test_wave_per_row_kernels_past_one_grid(spk, tall):
    A, v = tall
    dA = spk.CSR.from_host(A, v)
    assert oracle.csr_canonical(A.row_ptr, A.col_idx, M, N) == 0
    assert spk.validate_rules(dA) == 0
    # a duplicate column in the last row, found only by a wave past the first grid
    ci = A.col_idx.copy()
    ci[-1] = ci[-2]
    want = oracle.csr_canonical(A.row_ptr, ci, M, N)
    assert want != 0
    bad = spk.CSR(dA.row_ptr, torch.from_numpy(ci).cuda(), None, (M, N))
    assert spk.validate_rules(bad) == want
    trp, tci, perm = spk.csr_transpose(dA)
    otrp, otci, operm = oracle.csr_transpose(A.row_ptr, A.col_idx, N)
    assert np.array_equal(trp.cpu().numpy(), otrp)
    assert np.array_equal(tci.cpu().numpy(), otci)
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(spk.csr_row_index(dA).cpu().numpy(), oracle.row_index(A.row_ptr))


def test_products_and_size_error_past_one_grid(spk, tall):
    A, v = tall
    dA = spk.CSR.from_host(A, v)
    rows = np.unique(ROWS)
    srp, sci, idx = sub_rows(A, rows)
    U = synth.normal((M, K), 0, synth.S_U)
    V = synth.normal((N, K), 0, synth.S_V)
    S64, SM = oracle.sddmm(srp, sci, v[idx], U[rows], V)
    C64, CM = oracle.spmm(srp, sci, v[idx], V)
    Ud, Vd = torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda()
    r = torch.from_numpy(rows).cuda()
    # 64 lanes per row: M / 4 workgroups of 256 threads pass 2^32 threads
    for call in (lambda: spk.sddmm(dA, Ud, Vd, plan=spk.Plan(0, 64, 0)),
                 lambda: spk.spmm(dA, Vd, plan=spk.Plan(0, 64, 0))):
        with pytest.raises(spk.SpkError) as e:
            call()
        assert e.value.status == -2  # SPK_ERR_SIZE
    for plan in (spk.Plan(0, 4, 0), spk.Plan(7, 16, 0), spk.Plan(6, 8, 0)):
        S = spk.sddmm(dA, Ud, Vd, plan=plan)
        assert_within(S.cpu().numpy(), S64, SM, TOL_F32, f"sddmm {plan} m=2^26+64")
    for plan in (spk.Plan(0, 4, 0), spk.Plan(6, 16, 0)):
        C = spk.spmm(dA, Vd, plan=plan)
        assert_within(C[r].cpu().numpy(), C64, CM, TOL_F32, f"spmm {plan} m=2^26+64")
        C[r] = 0  # every other row of C is empty, so zero
        assert not C.any()
        del C
    del dA, Ud, Vd, S
    torch.cuda.empty_cache()
