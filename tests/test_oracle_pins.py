"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something other than itself: hand-worked
examples, dense brute force through numpy's matmul, closed-form special
cases, identities between the two products, and library routines (scipy's
CSR transpose, torch's bfloat16 conversion).
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_2604_27985_amd import synth


def dense_of(rp, ci, vals, m, n):
    D = np.zeros((m, n), np.float64)
    for i in range(m):
        for p in range(rp[i], rp[i + 1]):
            D[i, ci[p]] += 1.0 if vals is None else float(vals[p])
    return D


def rand_csr(m, n, d, seed):
    A = synth.bernoulli(m, n, d, seed)
    v = synth.normal(A.nnz, seed, synth.S_VALS)
    return A, v


# ---------------------------------------------------------------- hand-worked
def test_spmm_hand_example(golden):
    g = golden["spmm"]
    C, M = oracle.spmm(g["row_ptr"], g["col_idx"], g["vals"], np.array(g["B"], float))
    assert np.array_equal(C, np.array(g["C"], float))
    assert M[1].tolist() == [0.0, 0.0]


def test_sddmm_hand_example(golden):
    g, s = golden["spmm"], golden["sddmm"]
    S, _ = oracle.sddmm(g["row_ptr"], g["col_idx"], g["vals"], np.array(s["U"], float),
                        np.array(s["V"], float))
    assert S.tolist() == s["S"]
    S0, _ = oracle.sddmm(g["row_ptr"], g["col_idx"], None, np.array(s["U"], float),
                         np.array(s["V"], float))
    assert S0.tolist() == s["S_pattern"]


def test_transpose_hand_example(golden):
    g, t = golden["spmm"], golden["transpose"]
    trp, tci, perm = oracle.csr_transpose(g["row_ptr"], g["col_idx"], g["n"])
    assert trp.tolist() == t["t_row_ptr"]
    assert tci.tolist() == t["t_col_idx"]
    assert perm.tolist() == t["perm"]


def test_features_hand_example(golden):
    g = golden["spmm"]
    f = oracle.features(g["row_ptr"], g["col_idx"], g["n"])
    assert f.tolist() == golden["features"]["f"]


def test_mlp_hand_example(golden):
    h = golden["mlp"]
    net = oracle.MLP(np.array(h["W1"], float), np.array(h["b1"], float), np.array(h["W2"], float),
                     np.array(h["b2"], float), np.array(h["W3"], float), np.array(h["b3"], float))
    y = net.forward(np.array([h["x"]], float))
    assert y.tolist() == [h["y"]]


# ---------------------------------------------------------------- brute force
@settings(max_examples=40, deadline=None)
@given(m=st.integers(0, 40), n=st.integers(1, 40), d=st.sampled_from([0.0, 0.05, 0.3, 1.0]),
       K=st.integers(1, 9), seed=st.integers(0, 10_000), pattern=st.booleans())
def test_spmm_matches_dense(m, n, d, K, seed, pattern):
    A, v = rand_csr(m, n, d, seed)
    vals = None if pattern else v
    B = synth.normal((n, K), seed, synth.S_B).astype(np.float64)
    C, M = oracle.spmm(A.row_ptr, A.col_idx, vals, B)
    D = dense_of(A.row_ptr, A.col_idx, vals, m, n)
    ref = D @ B
    assert np.allclose(C, ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(M, np.abs(D) @ np.abs(B), rtol=1e-12, atol=1e-12)


@settings(max_examples=40, deadline=None)
@given(m=st.integers(0, 30), n=st.integers(1, 30), d=st.sampled_from([0.0, 0.1, 0.5, 1.0]),
       K=st.integers(1, 9), seed=st.integers(0, 10_000))
def test_sddmm_matches_dense(m, n, d, K, seed):
    A, v = rand_csr(m, n, d, seed)
    U = synth.normal((m, K), seed, synth.S_U).astype(np.float64)
    V = synth.normal((n, K), seed, synth.S_V).astype(np.float64)
    S, _ = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    full = U @ V.T
    rows = np.repeat(np.arange(m), A.row_lengths())
    ref = v.astype(np.float64) * full[rows, A.col_idx]
    assert np.allclose(S, ref, rtol=1e-12, atol=1e-12)


def test_sddmm_full_pattern_is_hadamard():
    m, n, K = 17, 13, 5
    A, v = rand_csr(m, n, 1.0, 3)
    assert A.nnz == m * n
    U = synth.normal((m, K), 3, synth.S_U)
    V = synth.normal((n, K), 3, synth.S_V)
    S, _ = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    ref = v.reshape(m, n).astype(np.float64) * (U.astype(np.float64) @ V.astype(np.float64).T)
    assert np.allclose(S.reshape(m, n), ref, rtol=1e-12, atol=1e-13)


def test_spmm_t_matches_dense():
    m, n, K = 37, 29, 6
    A, v = rand_csr(m, n, 0.2, 5)
    G = synth.normal((m, K), 5, synth.S_G)
    D, M = oracle.spmm_t(A.row_ptr, A.col_idx, v, G, n)
    Ad = dense_of(A.row_ptr, A.col_idx, v, m, n)
    assert np.allclose(D, Ad.T @ G.astype(np.float64), rtol=1e-12, atol=1e-12)
    assert np.allclose(M, np.abs(Ad).T @ np.abs(G.astype(np.float64)), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- special cases
def test_spmm_special_cases_exact():
    n, K = 50, 7
    B = synth.normal((n, K), 1, synth.S_B).astype(np.float64)
    eye = np.arange(n + 1, dtype=np.int32)
    # identity: C = B
    C, _ = oracle.spmm(eye, np.arange(n, dtype=np.int32), np.ones(n), B)
    assert np.array_equal(C, B)
    # permutation: row gather
    pi = np.random.default_rng(0).permutation(n).astype(np.int32)
    C, _ = oracle.spmm(eye, pi, None, B)
    assert np.array_equal(C, B[pi])
    # diagonal: row scaling, one product per output
    dvals = synth.normal(n, 1, synth.S_VALS).astype(np.float64)
    C, _ = oracle.spmm(eye, np.arange(n, dtype=np.int32), dvals, B)
    assert np.array_equal(C, dvals[:, None] * B)
    # K = 1 is a sparse matrix-vector product; B = ones gives row sums
    A, v = rand_csr(n, n, 0.3, 2)
    C, _ = oracle.spmm(A.row_ptr, A.col_idx, v, np.ones((n, 1)))
    sums = np.array([v[A.row_ptr[i]:A.row_ptr[i + 1]].astype(np.float64).sum() for i in range(n)])
    assert np.allclose(C[:, 0], sums, rtol=1e-13, atol=1e-13)
    # nnz = 0: all zeros
    C, M = oracle.spmm(np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0), B)
    assert not C.any() and not M.any()


def test_sddmm_identity_pattern_rowwise_dot():
    n, K = 40, 9
    U = synth.normal((n, K), 4, synth.S_U).astype(np.float64)
    V = synth.normal((n, K), 4, synth.S_V).astype(np.float64)
    S, _ = oracle.sddmm(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), None, U, V)
    assert np.allclose(S, np.einsum("ik,ik->i", U, V), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- identities
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sddmm_trace_identity(seed):
    """sum_p S_p = <A, U V^T>_F = trace(U^T A V), with A dense."""
    m, n, K = 60, 45, 8
    A, v = rand_csr(m, n, 0.15, seed)
    U = synth.normal((m, K), seed, synth.S_U).astype(np.float64)
    V = synth.normal((n, K), seed, synth.S_V).astype(np.float64)
    S, _ = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    Ad = dense_of(A.row_ptr, A.col_idx, v, m, n)
    assert np.isclose(S.sum(), np.trace(U.T @ Ad @ V), rtol=1e-11)


@pytest.mark.parametrize("seed", [0, 7])
def test_adjoint_identity(seed):
    """<SpMM(A, B), G> = <vals, SDDMM(pattern, G, B)>."""
    m, n, K = 80, 70, 12
    A, v = rand_csr(m, n, 0.1, seed)
    B = synth.normal((n, K), seed, synth.S_B)
    G = synth.normal((m, K), seed, synth.S_G)
    C, _ = oracle.spmm(A.row_ptr, A.col_idx, v, B)
    S, _ = oracle.sddmm(A.row_ptr, A.col_idx, None, G, B)
    lhs = float((C * G.astype(np.float64)).sum())
    rhs = float((v.astype(np.float64) * S).sum())
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))


def test_transpose_against_scipy_and_involution():
    import scipy.sparse as sp

    m, n = 123, 77
    A, v = rand_csr(m, n, 0.07, 11)
    trp, tci, perm = oracle.csr_transpose(A.row_ptr, A.col_idx, n)
    ref = sp.csr_matrix((np.arange(A.nnz), A.col_idx, A.row_ptr), shape=(m, n)).T.tocsr()
    ref.sort_indices()
    assert np.array_equal(trp, ref.indptr) and np.array_equal(tci, ref.indices)
    assert np.array_equal(perm, ref.data)
    assert np.array_equal(np.sort(perm), np.arange(A.nnz))
    rp2, ci2, perm2 = oracle.csr_transpose(trp, tci, m)
    assert np.array_equal(rp2, A.row_ptr) and np.array_equal(ci2, A.col_idx)
    assert np.array_equal(perm[perm2], np.arange(A.nnz))


def test_backward_matches_finite_differences():
    """L(vals, B) = <A B, G> is bilinear, so central differences are exact up to rounding."""
    m, n, K = 20, 16, 4
    A, v = rand_csr(m, n, 0.3, 9)
    B = synth.normal((n, K), 9, synth.S_B).astype(np.float64)
    G = synth.normal((m, K), 9, synth.S_G).astype(np.float64)
    v64 = v.astype(np.float64)
    dB, _, dv, _ = oracle.spmm_backward(A.row_ptr, A.col_idx, v64, B, G, n)

    def L(vv, BB):
        C, _ = oracle.spmm(A.row_ptr, A.col_idx, vv, BB, with_bound=False)
        return float((C * G).sum())

    h = 2.0 ** -10
    for p in range(0, A.nnz, 7):
        e = np.zeros_like(v64); e[p] = h
        fd = (L(v64 + e, B) - L(v64 - e, B)) / (2 * h)
        assert abs(fd - dv[p]) <= 1e-10 * max(1.0, abs(dv).max())
    for (j, k) in [(0, 0), (3, 2), (n - 1, K - 1), (7, 1)]:
        E = np.zeros_like(B); E[j, k] = h
        fd = (L(v64, B + E) - L(v64, B - E)) / (2 * h)
        assert abs(fd - dB[j, k]) <= 1e-10 * max(1.0, abs(dB).max())


# ---------------------------------------------------------------- bf16
def test_bf16_rounding_against_torch_and_ties():
    import torch

    x = synth.normal(100_000, 3, synth.S_MISC) * np.float32(1e3)
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x3F80FFFF, 0x7F7FFFFF, 0x00008000,
                     0x00018000, 0x7F800000, 0xFF800000, 0x00000000, 0x80000000],
                    dtype=np.uint32).view(np.float32)
    x = np.concatenate([x, ties])
    got = oracle.round_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    # by hand: 1 + 2^-8 is a tie, rounds to even (1.0); 1 + 3*2^-8 rounds up
    assert got[-11].view(np.uint32) == 0x3F800000
    assert got[-10].view(np.uint32) == 0x3F820000
    assert not (got.view(np.uint32) & 0xFFFF).any()


# ---------------------------------------------------------------- features, bsr
def test_features_brute_force():
    for (m, n, d, seed, kind) in [(70, 90, 0.05, 1, "u"), (64, 64, 0.1, 2, "b"), (33, 33, 0.0, 0, "u")]:
        A = synth.block4(m, n, d, seed) if kind == "b" else synth.bernoulli(m, n, d, seed)
        f = oracle.features(A.row_ptr, A.col_idx, n)
        L = A.row_lengths()
        rows = np.repeat(np.arange(m), L)
        bins = np.zeros(20, np.int64)
        for l in L:
            b = 0 if l == 0 else min(19, int(np.floor(np.log2(l))) + 1)
            bins[b] += 1
        diff = np.abs(rows - A.col_idx)
        blocks = {(r // 4, c // 4) for r, c in zip(rows.tolist(), A.col_idx.tolist())}
        exp = [m, n, A.nnz, *bins.tolist(), int(L.max(initial=0)), int((L * L).sum()),
               int(diff.max(initial=0)), int(diff.sum()), len(blocks)]
        assert f.tolist() == exp


def test_bsr4_reconstructs_dense():
    for (m, n, kind) in [(30, 22, "u"), (64, 48, "b"), (5, 3, "u")]:
        A = synth.block4(m, n, 0.2, 4) if kind == "b" else synth.bernoulli(m, n, 0.1, 4)
        v = synth.normal(A.nnz, 4, synth.S_VALS)
        brp, bcol, bv = oracle.csr_to_bsr4(A.row_ptr, A.col_idx, v, n)
        D = np.zeros(((m + 3) // 4 * 4, (n + 3) // 4 * 4))
        for I in range(len(brp) - 1):
            assert np.all(np.diff(bcol[brp[I]:brp[I + 1]]) > 0)
            for q in range(brp[I], brp[I + 1]):
                D[4 * I:4 * I + 4, 4 * bcol[q]:4 * bcol[q] + 4] += bv[q]
        assert np.array_equal(D[:m, :n], dense_of(A.row_ptr, A.col_idx, v, m, n))
        assert not D[m:, :].any() and not D[:, n:].any()


def test_selector_inputs_closed_forms(golden):
    """Hand-worked example: m=3, n=4, nnz=5, lengths (2, 0, 3), |i-j| sum 5, one block, K=64."""
    f = golden["features"]["f"]
    x = oracle.selector_inputs(f, 64)
    assert x[0] == np.log2(4) / 20 and x[1] == np.log2(5) / 20 and x[2] == np.log2(6) / 30
    assert x[3] == 1 / 3 and x[5] == 2 / 3 and x[3:23].sum() == 1.0
    mean = 5 / 3
    assert np.isclose(x[24], np.log2(1 + mean) / 20)
    cv = np.sqrt(13 / 3 - mean ** 2) / mean  # lengths 2, 0, 3: E[L^2] = 13/3
    assert np.isclose(x[25], np.log2(1 + cv) / 4)
    assert x[26] == np.log2(4) / 20 and np.isclose(x[27], (5 / 5) / 4)
    assert np.isclose(x[28], 5 / 16) and x[29] == 6 / 8
    assert np.isclose(x[30], 1 + np.log10(5 / 12) / 5) and x[31] == 1.0
    # the dtype input: 0 for binary32 operands, 1 for bfloat16, nothing else moves
    assert x[32] == 0.0
    xb = oracle.selector_inputs(f, 64, 1)
    assert xb[32] == 1.0 and np.array_equal(xb[:32], x[:32])
    # an empty matrix gives finite inputs
    e = np.zeros(28, np.int64)
    e[0], e[1], e[3] = 10, 10, 10
    assert np.isfinite(oracle.selector_inputs(e, 1)).all()


# ---------------------------------------------------------------- mlp
def _rand_mlp(F, H, P, seed):
    r = np.random.default_rng(seed)
    return oracle.MLP(r.normal(size=(H, F)), r.normal(size=H), r.normal(size=(H, H)) / 4,
                      r.normal(size=H), r.normal(size=(P, H)) / 4, r.normal(size=P))


@pytest.mark.parametrize("weighted", [False, True])
def test_mlp_gradients_match_finite_differences(weighted):
    """A 0/1 mask gives the masked mean of squared errors; other mask values
    weigh the terms (count stays the number of nonzero entries)."""
    F, H, P, Bsz = 6, 8, 5, 7
    net = _rand_mlp(F, H, P, 0)
    r = np.random.default_rng(1)
    X, T = r.normal(size=(Bsz, F)), r.normal(size=(Bsz, P))
    mask = (r.random((Bsz, P)) < 0.7).astype(np.float64)
    if weighted:
        mask *= r.uniform(0.1, 5.0, size=(Bsz, 1))
    loss, grads = net.loss_grad(X, T, mask)
    Y = net.forward(X)
    assert np.isclose(loss, ((Y - T) ** 2 * mask).sum() / (2 * (mask != 0).sum()), rtol=1e-13)
    h = 1e-6
    for W, g in zip(net.params(), grads):
        flat, gflat = W.reshape(-1), g.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 11)):
            old = flat[idx]
            flat[idx] = old + h; lp, _ = net.loss_grad(X, T, mask)
            flat[idx] = old - h; lm, _ = net.loss_grad(X, T, mask)
            flat[idx] = old
            assert abs((lp - lm) / (2 * h) - gflat[idx]) <= 1e-6 * max(1.0, abs(gflat).max())


def test_adam_first_step_closed_form():
    """First Adam step: m_hat = g and v_hat = g^2, so w moves by -lr g / (|g| + eps)."""
    r = np.random.default_rng(2)
    w0 = r.normal(size=50); g = r.normal(size=50)
    w = w0.copy(); mom = np.zeros(50); vel = np.zeros(50)
    oracle.adam(w, g, mom, vel, 1e-3, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(w, w0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g, v_hat = g^2 at every step
    oracle.adam(w, g, mom, vel, 1e-3, 0.9, 0.999, 1e-8, 2)
    assert np.allclose(w, w0 - 2e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)


# ---------------------------------------------------------------- canonical CSR
def test_csr_canonical_hand_cases():
    """One hand-worked case per rule of canonical CSR (tests/golden/csr_canonical.json)."""
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "csr_canonical.json")))
    for c in g["cases"]:
        got = oracle.csr_canonical(np.array(c["row_ptr"]), np.array(c["col_idx"], np.int32), c["m"], c["n"], c["nnz"])
        assert got == c["bits"], (c["name"], got)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_csr_canonical_against_scipy_and_single_mutations(seed):
    """Generated patterns are canonical (scipy agrees); a swap of two neighbours
    breaks only the order rule, a copied neighbour only the duplicate rule, a
    column pushed to n only the range rule, and every such matrix is flagged
    exactly when scipy's has_canonical_format (sorted, no duplicates) says no."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    for A in (synth.bernoulli(300, 200, 0.05, seed), synth.powerlaw(500, 8, 2.1, seed),
              synth.block4(64, 96, 0.1, seed), synth.bernoulli(200, 200, 0.05, seed, band=8)):
        assert oracle.csr_canonical(A.row_ptr, A.col_idx, A.m, A.n) == 0
        lens = np.diff(A.row_ptr)
        for kind in ("swap", "dup", "range"):
            ci = A.col_idx.copy()
            rows = np.flatnonzero(lens >= 2)
            i = int(rng.choice(rows))
            p = int(A.row_ptr[i] + rng.integers(0, lens[i] - 1))
            if kind == "swap":
                ci[p], ci[p + 1] = ci[p + 1], ci[p]
                want = oracle.CSR_BAD_SORT
            elif kind == "dup":
                ci[p + 1] = ci[p]
                want = oracle.CSR_BAD_DUP
            else:
                ci[A.row_ptr[i + 1] - 1] = A.n  # the last entry of the row: stays increasing
                want = oracle.CSR_BAD_COL
            assert oracle.csr_canonical(A.row_ptr, ci, A.m, A.n) == want, kind
            if kind != "range":
                M = sp.csr_matrix((np.ones(A.nnz), ci, A.row_ptr), shape=(A.m, A.n))
                assert not M.has_canonical_format
        M = sp.csr_matrix((np.ones(A.nnz), A.col_idx, A.row_ptr), shape=(A.m, A.n))
        assert M.has_canonical_format


# ---------------------------------------------------------------- slab16 form
def test_slab16_hand_examples(golden):
    g = golden["spmm"]
    for c in golden["slab16"]["cases"]:
        seg, apos, col16, S = oracle.csr_to_slab16(g["row_ptr"], g["col_idx"], g["n"], c["width"])
        assert S == c["slabs"]
        assert seg.tolist() == c["seg"] and apos.tolist() == c["apos"] and col16.tolist() == c["col16"], c["width"]


def _slab16_rebuild(seg, apos, col16, S, m, W):
    """Rows of A rebuilt from the slab form: runs in slab order, columns s W + col16."""
    rows = [[] for _ in range(m)]
    positions = [[] for _ in range(m)]
    for s in range(S):
        for i in range(m):
            a, b = int(seg[s * m + i]), int(seg[s * m + i + 1])
            rows[i] += [s * W + int(c) for c in col16[a:b]]
            positions[i] += list(range(int(apos[s * m + i]), int(apos[s * m + i]) + b - a))
    return rows, positions


@pytest.mark.parametrize("kind,m,n,W", [("uniform", 300, 1000, 128), ("uniform", 50, 70000, 65536),
                                        ("powerlaw", 2000, 2000, 100), ("uniform", 40, 30, 1),
                                        ("uniform", 64, 64, 64), ("empty", 9, 17, 4)])
def test_slab16_reconstructs_csr(kind, m, n, W):
    """The runs of every row, read slab by slab, give back the row's columns
    in order and at the positions apos names; every run lies inside its slab
    and 16-bit offsets stay below W."""
    if kind == "powerlaw":
        A = synth.powerlaw(n, 8, 2.1, 3)
    elif kind == "empty":
        A = synth.HostCSR(m, n, np.zeros(m + 1, np.int32), np.zeros(0, np.int32))
    else:
        A = synth.bernoulli(m, n, 0.05, 2)
    seg, apos, col16, S = oracle.csr_to_slab16(A.row_ptr, A.col_idx, A.n, W)
    assert S == max(1, -(-A.n // W))
    assert seg[0] == 0 and seg[-1] == A.nnz and np.all(np.diff(seg.astype(np.int64)) >= 0)
    assert np.all(col16.astype(np.int64) < W)
    rows, positions = _slab16_rebuild(seg, apos, col16, S, A.m, W)
    for i in range(A.m):
        lo, hi = A.row_ptr[i], A.row_ptr[i + 1]
        assert rows[i] == A.col_idx[lo:hi].tolist()
        assert positions[i] == list(range(lo, hi))


# ---------------------------------------------------------------- attention chain
def _dense_attention(A, v, U, V, B):
    """Masked dense attention with scipy's softmax: scores U V^T times A's
    values where A stores an entry, -inf elsewhere; empty rows give zeros."""
    from scipy.special import logsumexp, softmax

    D = dense_of(A.row_ptr, A.col_idx, v, A.m, A.n)
    mask = dense_of(A.row_ptr, A.col_idx, None, A.m, A.n) > 0
    scores = np.where(mask, D * (U.astype(np.float64) @ V.astype(np.float64).T), -np.inf)
    O = np.zeros((A.m, B.shape[1]))
    lse = np.full(A.m, -np.inf)
    rows = mask.any(1)
    if rows.any():
        O[rows] = softmax(scores[rows], axis=1) @ B.astype(np.float64)
        lse[rows] = logsumexp(scores[rows], axis=1)
    return O, lse


@pytest.mark.parametrize("m,n,d,K1,K2,seed", [(30, 40, 0.2, 8, 5, 0), (25, 25, 1.0, 4, 4, 1), (40, 17, 0.05, 3, 9, 2),
                                              (1, 1, 1.0, 2, 2, 3)])
def test_attention_chain_matches_dense_softmax(m, n, d, K1, K2, seed):
    A = synth.bernoulli(m, n, d, seed)
    v = synth.normal(A.nnz, seed, synth.S_VALS)
    U = synth.normal((m, K1), seed, synth.S_U)
    V = synth.normal((n, K1), seed, synth.S_V)
    B = synth.normal((n, K2), seed, synth.S_B)
    O, M, E, L = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, v, U, V, B)
    Od, Ld = _dense_attention(A, v, U, V, B)
    assert np.allclose(O, Od, rtol=1e-12, atol=1e-12)
    assert np.array_equal(np.isinf(L), np.isinf(Ld)) and np.allclose(L[np.isfinite(L)], Ld[np.isfinite(Ld)], rtol=1e-12)
    # pattern mode equals values of one
    O1, _, _, _ = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, None, U, V, B)
    O1d, _ = _dense_attention(A, np.ones(A.nnz), U, V, B)
    assert np.allclose(O1, O1d, rtol=1e-12, atol=1e-12)
    # bound and score scale: brute force from their definitions' pieces
    S, SM = oracle.sddmm(A.row_ptr, A.col_idx, v, U, V)
    for i in range(m):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        assert E[i] == (SM[a:b].max() if b > a else 0.0)


def test_attention_chain_closed_forms():
    """B of ones gives rows of one (probabilities sum to 1); a one-entry row
    copies its B row; a zero row of U gives the mean of the row's B rows."""
    A = synth.bernoulli(50, 60, 0.1, 4)
    U = synth.normal((50, 6), 4, synth.S_U)
    V = synth.normal((60, 6), 4, synth.S_V)
    B = synth.normal((60, 7), 4, synth.S_B)
    lens = np.diff(A.row_ptr)
    O, M, _, _ = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, None, U, V, np.ones((60, 3)))
    assert np.allclose(O[lens > 0], 1.0, rtol=0, atol=1e-14) and not O[lens == 0].any()
    U0 = U.copy()
    U0[::2] = 0.0
    O, M, _, _ = oracle.sddmm_softmax_spmm(A.row_ptr, A.col_idx, None, U0, V, B)
    for i in range(0, 50, 2):
        cols = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        want = B[cols].astype(np.float64).mean(0) if len(cols) else np.zeros(7)
        assert np.allclose(O[i], want, rtol=1e-13, atol=1e-14)
    one = synth.HostCSR(2, 60, np.array([0, 1, 1], np.int32), np.array([17], np.int32))
    O, _, _, L = oracle.sddmm_softmax_spmm(one.row_ptr, one.col_idx, None, U[:2], V, B)
    assert np.array_equal(O[0], B[17].astype(np.float64)) and not O[1].any()
    assert np.isclose(L[0], float(U[0].astype(np.float64) @ V[17].astype(np.float64)), rtol=1e-14, atol=0)
    assert np.isneginf(L[1])


# ---------------------------------------------------------------- hyper-sparse forms
def test_hypersparse_hand_examples(golden):
    for c in golden["hypersparse"]["cases"]:
        order, nr = oracle.nonempty_order(c["row_ptr"])
        assert order.tolist() == c["order"] and nr == c["nr"]
        assert oracle.row_index(c["row_ptr"]).tolist() == c["rowidx"]


@pytest.mark.parametrize("m,n,d,seed", [(5000, 3000, 1e-4, 0), (300, 300, 0.01, 1), (1000, 10, 0.0, 2)])
def test_hypersparse_forms_properties(m, n, d, seed):
    """order is a permutation listing exactly the non-empty rows first, each
    part ascending; rowidx repeats each row number its length, in order
    (numpy's repeat of the row lengths)."""
    A = synth.bernoulli(m, n, d, seed)
    order, nr = oracle.nonempty_order(A.row_ptr)
    lens = np.diff(A.row_ptr)
    assert sorted(order.tolist()) == list(range(m))
    assert nr == int((lens > 0).sum())
    assert np.all(lens[order[:nr]] > 0) and np.all(lens[order[nr:]] == 0)
    assert np.all(np.diff(order[:nr]) > 0) and np.all(np.diff(order[nr:]) > 0)
    assert np.array_equal(oracle.row_index(A.row_ptr), np.repeat(np.arange(m, dtype=np.int32), lens))
