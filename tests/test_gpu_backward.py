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


@pytest.mark.parametrize("plan_args,dvals_args", [(None, None), ((1, 32, 0), (1, 32, 256)), ((0, 16, 0), (0, 32, 0)),
                                                   ((3, 32, 1000), (3, 16, 0)), ((4, 32, 0), (4, 32, 0, 4)),
                                                   ((4, 32, 7, 2), (4, 32, 9, 6))])
def test_backward_matches_oracle(spk, plan_args, dvals_args):
    """Both products of the backward on their own plans (A^T G and the pattern
    SDDMM), the workspace shared as the header states."""
    A, v, B, G = gcn_layer(n=30000, mean=16, K=128, seed=2)
    dB64, dBM, dv64, dvM = oracle.spmm_backward(A.row_ptr, A.col_idx, v, B, G, A.n)
    plan = None if plan_args is None else spk.Plan(*plan_args)
    dplan = None if dvals_args is None else spk.Plan(*dvals_args)
    dA = spk.CSR.from_host(A, v)
    dB, dv = spk.spmm_backward(dA, dev(B), dev(G), plan=plan, dvals_plan=dplan)
    torch.cuda.synchronize()
    assert_within(dB.cpu().numpy(), dB64, dBM, TOL_F32, f"dB {plan}")
    assert_within(dv.cpu().numpy(), dv64, dvM, TOL_F32, f"dvals {dplan}")
    # preallocated outputs and an explicit workspace of exactly the stated size
    nb = spk.backward_workspace_bytes(dA, 128, plan, dplan)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    oB = torch.full((A.n, 128), 7.0, device="cuda")
    ov = torch.full((A.nnz,), 7.0, device="cuda")
    spk.spmm_backward(dA, dev(B), dev(G), plan=plan, dvals_plan=dplan, out_dB=oB, out_dvals=ov, workspace=ws)
    assert torch.equal(oB, dB) and torch.equal(ov, dv)


def test_backward_full_size_sampled(spk):
    """n = 262144, mean degree 16, K = 128: sampled rows of dB and entries of
    dvals, on the plans the GCN bench line runs (the forward's merge-path
    plan, row-split A^T G, merge-path pattern SDDMM: the recorded profile's
    plans) and on the network's five best plans timed once for each product."""
    from paper_2604_27985_amd import selector

    A, v, B, G = gcn_layer()
    K = B.shape[1]
    dA = spk.CSR.from_host(A, v)
    Bd, Gd = dev(B), dev(G)
    trp_d, tci_d, _ = dA.transpose()
    AT_d = spk.CSR(trp_d, tci_d, None, (A.n, A.m))
    # the backward runs the CSR variants (rows, merge-path, column slabs, LDS
    # slabs); the forms built per pattern have calls of their own
    csr_variants = (spk.VAR_ROWS, spk.VAR_MERGE, spk.VAR_SLAB, spk.VAR_TILE)
    cands = [p for p in selector.rank(AT_d, K, spk.OP_SPMM, 16) if p.variant in csr_variants]
    from paper_2604_27985_amd import autotune
    learned_bwd = min(autotune.sweep(AT_d, K, spk.OP_SPMM, B=Gd, plans=cands[:5], reps=2, warmup=1),
                      key=lambda r: r[1])[0]
    dv_cands = [p for p in selector.rank(dA, K, spk.OP_SDDMM, 16) if p.variant in csr_variants]
    learned_dv = min(autotune.sweep(dA, K, spk.OP_SDDMM, U=Gd, V=Bd, plans=dv_cands[:5], reps=2, warmup=1),
                     key=lambda r: r[1])[0]
    # dB rows j: the oracle's SpMM over the sampled rows of A^T (the oracle's
    # own transpose), values gathered through its perm
    trp, tci, perm = oracle.csr_transpose(A.row_ptr, A.col_idx, A.n)
    AT = synth.HostCSR(A.n, A.m, trp, tci)
    cols = np.unique(np.concatenate([synth.randint(300, A.n, 3), np.argsort(np.diff(trp))[-3:]]))
    srp, sci, idx = sub_rows(AT, cols)
    ref_dB, M_dB = oracle.spmm(srp, sci, v[perm[idx]], G)
    # dvals: the entries of sampled rows of A, from the oracle's pattern SDDMM
    rows = np.unique(np.concatenate([synth.randint(400, A.m, 4), np.argsort(A.row_lengths())[-3:]]))
    rrp, rci, ridx = sub_rows(A, rows)
    ref_dv, M_dv = oracle.sddmm(rrp, rci, None, G[rows], B)
    for plan, dplan in ((spk.Plan(0, 32, 0), spk.Plan(1, 32, 256)), (learned_bwd, learned_dv), (None, None)):
        dB, dv = spk.spmm_backward(dA, Bd, Gd, plan=plan, dvals_plan=dplan)
        torch.cuda.synchronize()
        assert_within(dB[torch.from_numpy(cols).cuda()].cpu().numpy(), ref_dB, M_dB, TOL_F32, f"dB sampled {plan}")
        assert_within(dv[torch.from_numpy(ridx).cuda()].cpu().numpy(), ref_dv, M_dv, TOL_F32,
                      f"dvals sampled {dplan}")


@pytest.mark.parametrize("fwd,bwd,dvp", [(None, None, None), ((4, 16, 0, 4), (4, 16, 0), (4, 16, 0, 4)),
                                          ((2, 64, 0), None, (1, 16, 256)), ((1, 16, 0), (1, 16, 0), None)])
def test_autograd_function(spk, fwd, bwd, dvp):
    """Forward on any SpMM plan (TILE, 4x4 blocks, merge-path), backward on
    the plans given for A^T and for the pattern SDDMM (NULL by default)."""
    A, v, B, G = gcn_layer(n=8000, mean=16, K=64, seed=3)
    dA = spk.CSR.from_host(A)
    plan, bplan, dplan = (None if a is None else spk.Plan(*a) for a in (fwd, bwd, dvp))
    vt = dev(v).requires_grad_(True)
    Bt = dev(B).requires_grad_(True)
    C = spk.spmm_autograd(dA, vt, Bt, plan=plan, backward_plan=bplan, dvals_plan=dplan)
    C64, CM = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    assert_within(C.detach().cpu().numpy(), C64, CM, TOL_F32, f"autograd forward {plan}")
    C.backward(dev(G))
    dB64, dBM, dv64, dvM = oracle.spmm_backward(A.row_ptr, A.col_idx, v, B, G, A.n)
    assert_within(Bt.grad.cpu().numpy(), dB64, dBM, TOL_F32, "autograd dB")
    assert_within(vt.grad.cpu().numpy(), dv64, dvM, TOL_F32, "autograd dvals")
    # only one input needing a gradient
    vt2 = dev(v).requires_grad_(True)
    spk.spmm_autograd(dA, vt2, dev(B), plan=plan).sum().backward()
    assert vt2.grad is not None
    with pytest.raises(ValueError):
        spk.spmm_autograd(dA, vt2, dev(B), backward_plan=spk.Plan(2, 64, 0))


def test_bsr4_plan_sees_new_values(spk):
    """The block form cached on a matrix follows its values: a new values
    tensor (here very likely at the freed tensor's address) and an in-place
    update both rebuild it."""
    A = synth.block4(2048, 2048, 0.02, 4)
    B = synth.normal((2048, 64), 4, synth.S_B)
    dA = spk.CSR.from_host(A)
    Bd = dev(B)
    plan = spk.Plan(2, 64, 0)
    for seed in (10, 11, 12):
        v = synth.normal(A.nnz, seed, synth.S_VALS)
        vt = dev(v)
        C = spk.spmm(dA, Bd, plan=plan, vals=vt).cpu().numpy()
        C64, CM = oracle.spmm(A.row_ptr, A.col_idx, v, B)
        assert_within(C, C64, CM, TOL_F32, f"bsr4 values seed {seed}")
        vt.mul_(2.0)
        C = spk.spmm(dA, Bd, plan=plan, vals=vt).cpu().numpy()
        assert_within(C, 2 * C64, 2 * CM, TOL_F32, f"bsr4 values seed {seed} doubled in place")
        del vt, C
    # values held by the matrix itself
    v = synth.normal(A.nnz, 13, synth.S_VALS)
    dV = dA.with_vals(dev(v))
    C64, CM = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    assert_within(spk.spmm(dV, Bd, plan=plan).cpu().numpy(), C64, CM, TOL_F32, "bsr4 matrix values")


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
