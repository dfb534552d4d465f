"""Transpose, backward and autograd on the GPU against the FP64 oracle.

The differentiated layer follows the GCN-style workload: power-law CSR with
mean degree 16, learnable FP32 values, B of width 128; the finite-difference
check runs in FP64 on an ego subgraph of 2048 rows.
"""
import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth
from spk_testutil import TOL_F32, assert_within, host_csr, sub_rows

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


@pytest.mark.parametrize("kind,m,n,d", [("uniform", 1000, 700, 0.02), ("uniform", 300, 70000, 0.001),
                                        ("powerlaw", 50000, 50000, 16), ("uniform", 5, 9, 0.0),
                                        ("uniform", 4097, 3, 0.5), ("block4", 1024, 2048, 0.02)])
def test_transpose_bit_exact(spk, kind, m, n, d):
    if kind == "powerlaw":
        A = synth.powerlaw(n, d, 2.1, 1)
    elif kind == "block4":
        A = synth.block4(m, n, d, 1)
    else:
        A = synth.bernoulli(m, n, d, 1)
    trp, tci, perm = oracle.csr_transpose(A.row_ptr, A.col_idx, A.n)
    dA = spk.CSR.from_host(A)
    g = [t.cpu().numpy() for t in spk.csr_transpose(dA)]
    assert np.array_equal(g[0], trp)
    assert np.array_equal(g[1], tci)
    assert np.array_equal(g[2], perm)


def test_transpose_with_empty_columns_and_rows(spk):
    A = host_csr(6, 10, [[], [9], [0, 9], [], [2, 3, 9], []])
    trp, tci, perm = oracle.csr_transpose(A.row_ptr, A.col_idx, A.n)
    g = [t.cpu().numpy() for t in spk.csr_transpose(spk.CSR.from_host(A))]
    assert np.array_equal(g[0], trp) and np.array_equal(g[1], tci) and np.array_equal(g[2], perm)


def gcn_layer(n=262144, mean=16, K=128, seed=0):
    A = synth.powerlaw(n, mean, 2.1, seed)
    vals = synth.uniform(A.nnz, seed, synth.S_VALS)
    B = synth.normal((n, K), seed, synth.S_B)
    G = synth.normal((n, K), seed, synth.S_G)
    return A, vals, B, G


@pytest.mark.parametrize("plan_args", [None, (1, 32, 0), (0, 16, 0), (3, 32, 1000), (4, 32, 0), (4, 32, 7, 2)])
def test_backward_matches_oracle(spk, plan_args):
    A, v, B, G = gcn_layer(n=30000, mean=16, K=128, seed=2)
    dB64, dBM, dv64, dvM = oracle.spmm_backward(A.row_ptr, A.col_idx, v, B, G, A.n)
    plan = None if plan_args is None else spk.Plan(*plan_args)
    dA = spk.CSR.from_host(A, v)
    dB, dv = spk.spmm_backward(dA, dev(B), dev(G), plan=plan)
    torch.cuda.synchronize()
    assert_within(dB.cpu().numpy(), dB64, dBM, TOL_F32, "dB")
    assert_within(dv.cpu().numpy(), dv64, dvM, TOL_F32, "dvals")


def test_backward_full_size_sampled(spk):
    """n = 262144, mean degree 16, K = 128: sampled rows of dB and entries of dvals."""
    A, v, B, G = gcn_layer()
    dA = spk.CSR.from_host(A, v)
    dB, dv = spk.spmm_backward(dA, dev(B), dev(G), plan=spk.Plan(1, 32, 0))
    torch.cuda.synchronize()
    dB, dv = dB.cpu().numpy(), dv.cpu().numpy()
    # dB rows j: the oracle's A^T G restricted to sampled columns of A
    trp, tci, perm = oracle.csr_transpose(A.row_ptr, A.col_idx, A.n)
    AT = synth.HostCSR(A.n, A.m, trp, tci)
    cols = np.unique(synth.randint(300, A.n, 3))
    srp, sci, idx = sub_rows(AT, cols)
    ref, M = oracle.spmm(srp, sci, v[perm[idx]], G)
    assert_within(dB[cols], ref, M, TOL_F32, "dB sampled")
    ps = np.unique(synth.randint(5000, A.nnz, 4))
    rows = np.searchsorted(A.row_ptr, ps, side="right") - 1
    exact = np.einsum("ik,ik->i", G[rows].astype(np.float64), B[A.col_idx[ps]].astype(np.float64))
    bound = np.einsum("ik,ik->i", np.abs(G[rows]).astype(np.float64), np.abs(B[A.col_idx[ps]]).astype(np.float64))
    assert_within(dv[ps], exact, bound, TOL_F32, "dvals sampled")


def test_autograd_function(spk):
    A, v, B, G = gcn_layer(n=8000, mean=16, K=64, seed=3)
    dA = spk.CSR.from_host(A)
    vt = dev(v).requires_grad_(True)
    Bt = dev(B).requires_grad_(True)
    C = spk.spmm_autograd(dA, vt, Bt)
    C.backward(dev(G))
    dB64, dBM, dv64, dvM = oracle.spmm_backward(A.row_ptr, A.col_idx, v, B, G, A.n)
    assert_within(Bt.grad.cpu().numpy(), dB64, dBM, TOL_F32, "autograd dB")
    assert_within(vt.grad.cpu().numpy(), dv64, dvM, TOL_F32, "autograd dvals")
    # only one input needing a gradient
    vt2 = dev(v).requires_grad_(True)
    spk.spmm_autograd(dA, vt2, dev(B)).sum().backward()
    assert vt2.grad is not None


def ego_subgraph(A, vals, B, rows):
    """2048 sampled rows with all their columns, relabelled to a compact CSR."""
    srp, sci, idx = sub_rows(A, rows)
    J, inv = np.unique(sci, return_inverse=True)
    sub = synth.HostCSR(len(rows), len(J), srp, inv.astype(np.int32), "ego")
    return sub, vals[idx], B[J]


def test_finite_differences_fp64_ego_subgraph(spk):
    """FP64 central differences of L1 = <C, G> and L2 = |C|^2 / 2 against the FP64 backward
    kernels.  Along a direction in vals alone or in B alone both losses are at most
    quadratic, so the differences are exact up to rounding."""
    A, v, B, _ = gcn_layer()
    rows = np.sort(np.unique(synth.randint(2048 * 2, A.m, 5))[:2048])
    S, sv, SB = ego_subgraph(A, v, B, rows)
    dA = spk.CSR.from_host(S, sv, vals_dtype=torch.float64)
    v64 = dev(sv.astype(np.float64))
    B64 = dev(SB.astype(np.float64))
    G64 = dev(synth.normal((S.m, B.shape[1]), 5, synth.S_G).astype(np.float64))
    h = 2.0 ** -10

    def C_of(vv, BB):
        return spk.spmm(dA, BB, vals=vv)

    for loss in ("L1", "L2"):
        C = C_of(v64, B64)
        Gl = G64 if loss == "L1" else C
        dB, dv = spk.spmm_backward(dA, B64, Gl.contiguous(), vals=v64)
        L = (lambda vv, BB: float((C_of(vv, BB) * G64).sum())) if loss == "L1" else \
            (lambda vv, BB: float(0.5 * (C_of(vv, BB) ** 2).sum()))
        gmax = max(1.0, float(dv.abs().max()), float(dB.abs().max()))
        rng = np.random.default_rng(6)
        for _ in range(32):  # random directions, in vals alone and in B alone
            dvd = dev(rng.standard_normal(S.nnz))
            dBd = dev(rng.standard_normal(tuple(B64.shape)))
            # each loss is at most quadratic in vals alone and in B alone, so the
            # central difference has no truncation error along either direction
            fd_v = (L(v64 + h * dvd, B64) - L(v64 - h * dvd, B64)) / (2 * h)
            fd_b = (L(v64, B64 + h * dBd) - L(v64, B64 - h * dBd)) / (2 * h)
            an_v = float((dv * dvd).sum())
            an_b = float((dB * dBd).sum())
            assert abs(fd_v - an_v) <= 1e-8 * gmax * float(dvd.abs().sum()) ** 0.5, (loss, fd_v, an_v)
            assert abs(fd_b - an_b) <= 1e-8 * gmax * float(dBd.abs().sum()) ** 0.5, (loss, fd_b, an_b)
        for p in rng.choice(S.nnz, 256, replace=False):  # coordinates of vals
            e = torch.zeros_like(v64)
            e[int(p)] = h
            fd = (L(v64 + e, B64) - L(v64 - e, B64)) / (2 * h)
            assert abs(fd - float(dv[int(p)])) <= 1e-8 * gmax
    # the FP64 gradients also agree with the FP64 oracle
    dB, dv = spk.spmm_backward(dA, B64, G64, vals=v64)
    o_dB, o_dBM, o_dv, o_dvM = oracle.spmm_backward(S.row_ptr, S.col_idx, sv.astype(np.float64), SB.astype(np.float64),
                                                    G64.cpu().numpy(), S.n)
    assert_within(dB.cpu().numpy(), o_dB, o_dBM, 1e-12, "fp64 dB")
    assert_within(dv.cpu().numpy(), o_dv, o_dvM, 1e-12, "fp64 dvals")
