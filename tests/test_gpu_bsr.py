"""4x4 block-sparse form and its matrix-core SpMM against the FP64 oracle (GPU)."""
import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth
from spk_testutil import TOL_F32, assert_within

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    import paper_2604_27985_amd as spk

    assert torch.cuda.is_available()
    return spk


@pytest.mark.parametrize("kind,m,n,d", [("block4", 2048, 2048, 0.02), ("block4", 1001, 999, 0.05),
                                        ("uniform", 777, 555, 0.02), ("uniform", 5, 3, 0.5), ("block4", 4, 4, 1.0)])
def test_bsr4_structure_bit_exact(spk, kind, m, n, d):
    A = synth.block4(m, n, d, 1) if kind == "block4" else synth.bernoulli(m, n, d, 1)
    v = synth.normal(A.nnz, 1, synth.S_VALS)
    brp, bcol, bv = oracle.csr_to_bsr4(A.row_ptr, A.col_idx, v, n)
    Ab = spk.csr_to_bsr4(spk.CSR.from_host(A, v))
    assert np.array_equal(Ab.b_row_ptr.cpu().numpy(), brp)
    assert np.array_equal(Ab.b_col.cpu().numpy(), bcol)
    assert np.array_equal(Ab.b_vals.cpu().numpy().astype(np.float64), bv)


@pytest.mark.parametrize("K", [64, 256, 100, 36, 1, 512])
@pytest.mark.parametrize("kind,m,n,d", [("block4", 4096, 4096, 0.01), ("block4", 1001, 999, 0.05),
                                        ("uniform", 3000, 2000, 0.01)])
def test_spmm_bsr4_matches_oracle(spk, K, kind, m, n, d):
    A = synth.block4(m, n, d, 2) if kind == "block4" else synth.bernoulli(m, n, d, 2)
    v = synth.normal(A.nnz, 2, synth.S_VALS)
    B = synth.normal((n, K), 2, synth.S_B)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    Ab = spk.csr_to_bsr4(spk.CSR.from_host(A, v))
    C = spk.spmm_bsr4(Ab, torch.from_numpy(B).cuda()).cpu().numpy()
    assert_within(C, C64, M, TOL_F32, f"bsr4 {kind} K={K}")


def test_spmm_bsr4_pattern_bf16_and_empty(spk):
    A = synth.block4(2048, 1536, 0.02, 3)
    B32 = synth.normal((1536, 256), 3, synth.S_B)
    Br = oracle.round_bf16(B32)
    C64, M = oracle.spmm(A.row_ptr, A.col_idx, None, Br)
    Ab = spk.csr_to_bsr4(spk.CSR.from_host(A, None))
    C = spk.spmm_bsr4(Ab, torch.from_numpy(Br).cuda().to(torch.bfloat16)).cpu().numpy()
    assert_within(C, C64, M, TOL_F32, "bsr4 pattern bf16")
    # no stored entries: C is zero-filled
    E = synth.HostCSR(9, 7, np.zeros(10, np.int32), np.zeros(0, np.int32))
    Eb = spk.csr_to_bsr4(spk.CSR.from_host(E, np.zeros(0, np.float32)))
    assert Eb.nblocks == 0
    out = torch.full((9, 8), 3.0, device="cuda")
    spk.spmm_bsr4(Eb, torch.randn(7, 8, device="cuda"), out=out)
    assert not out.cpu().numpy().any()


def test_spmm_bsr4_full_size_sampled(spk):
    """4x4-block pattern at n = 65536, block density 0.01, K = 64: sampled rows."""
    n, K = 65536, 64
    A = synth.block4(n, n, 0.01, 4)
    v = synth.normal(A.nnz, 4, synth.S_VALS)
    B = synth.normal((n, K), 4, synth.S_B)
    Ab = spk.csr_to_bsr4(spk.CSR.from_host(A, v))
    C = spk.spmm_bsr4(Ab, torch.from_numpy(B).cuda())
    rows = np.unique(synth.randint(500, n, 9))
    from spk_testutil import sub_rows

    srp, sci, idx = sub_rows(A, rows)
    ref, M = oracle.spmm(srp, sci, v[idx], B)
    assert_within(C[torch.from_numpy(rows).cuda()].cpu().numpy(), ref, M, TOL_F32, "bsr4 full")
