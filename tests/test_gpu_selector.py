"""Selector kernels against the FP64 oracle (GPU): features, inputs, network
forward, gradients, Adam, and plan_select's choice."""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
from paper_2604_27985_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    import paper_2604_27985_amd as spk

    assert torch.cuda.is_available()
    return spk


@pytest.fixture(scope="module")
def sel():
    from paper_2604_27985_amd import selector

    return selector


@pytest.mark.parametrize("kind,n,d", [("uniform", 3000, 0.01), ("banded", 5000, 0.3), ("powerlaw", 20000, 16),
                                      ("block4", 4096, 0.01), ("uniform", 33, 0.0), ("uniform", 1 << 18, 2e-5),
                                      ("block4", 1030, 0.05), ("wide", 3_000_000, 1e-4)])
def test_features_bit_exact(spk, sel, kind, n, d):
    """Feature counts equal the oracle's; the 4x4-block count runs as an LDS
    bitmap per block row up to 2^21 columns and as binary searches beyond."""
    if kind == "wide":  # 257 rows (a ragged last block row) x 3e6 columns: the search path
        A = synth.bernoulli(257, n, d, 1)
    elif kind == "powerlaw":
        A = synth.powerlaw(n, d, 2.1, 1)
    elif kind == "banded":
        A = synth.bernoulli(n, n, d, 1, band=64)
    elif kind == "block4":
        A = synth.block4(n, n, d, 1)
    else:
        A = synth.bernoulli(n, n, d, 1)
    f = sel.features(spk.CSR.from_host(A)).cpu().numpy()
    assert f.tolist() == oracle.features(A.row_ptr, A.col_idx, A.n).tolist()


def test_inputs_match_oracle(spk, sel):
    for (n, d, K) in [(3000, 0.01, 64), (777, 0.2, 33), (10, 0.0, 1)]:
        A = synth.bernoulli(n, n, d, 2)
        f = sel.features(spk.CSR.from_host(A))
        for dt in (0, 1):  # F32 and BF16 dense operands
            x = sel.inputs(f, K, dt).cpu().numpy().astype(np.float64)
            ref = oracle.selector_inputs(f.cpu().numpy(), K, dt)
            assert np.allclose(x, ref, rtol=2e-6, atol=2e-7), (x - ref)


def rand_params(P, H=64, F=33, seed=0):
    r = np.random.default_rng(seed)
    W1, b1 = r.normal(size=(H, F)) / 4, r.normal(size=H) / 4
    W2, b2 = r.normal(size=(H, H)) / 8, r.normal(size=H) / 4
    W3, b3 = r.normal(size=(P, H)) / 8, r.normal(size=P) / 4
    return [a.astype(np.float32) for a in (W1, b1, W2, b2, W3, b3)]


@pytest.mark.parametrize("H", [64, 192])  # one network; three averaged (the largest the kernels take)
def test_mlp_forward_grad_adam_match_oracle(spk, sel, H):
    P, F, N = 16, 33, 300
    parts = rand_params(P, H, F, 1)
    r = np.random.default_rng(2)
    X = r.normal(size=(N, F)).astype(np.float32)
    T = r.normal(size=(N, P)).astype(np.float32)
    # a weighted mask: per-sample weights as the time-weighted training uses
    mask = ((r.random((N, P)) < 0.8) * r.uniform(0.2, 4.0, size=(N, 1))).astype(np.float32)
    net = oracle.MLP(*parts)
    tr = sel.Trainer(P, H)
    tr.params = torch.from_numpy(np.concatenate([a.reshape(-1) for a in parts])).cuda()
    tr.grads = torch.zeros_like(tr.params)
    tr.mom = torch.zeros_like(tr.params)
    tr.vel = torch.zeros_like(tr.params)
    Xd, Td, Md = (torch.from_numpy(a).cuda() for a in (X, T, mask))
    Y = tr.forward(Xd).cpu().numpy()
    Yr = net.forward(X)
    assert np.allclose(Y, Yr, rtol=1e-4, atol=1e-5 * np.abs(Yr).max())
    loss = float(tr.loss_grad(Xd, Td, Md).item())
    lref, gref = net.loss_grad(X, T, mask)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    g = tr.grads.cpu().numpy().astype(np.float64)
    gr = np.concatenate([a.reshape(-1) for a in gref])
    assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max()
    # two gradient evaluations are bitwise equal (fixed summation order)
    g2 = tr.grads.clone()
    tr.loss_grad(Xd, Td, Md)
    assert torch.equal(g2, tr.grads)
    # Adam against the oracle's update on the same gradient
    w = np.concatenate([a.reshape(-1) for a in parts]).astype(np.float64)
    m0, v0 = np.zeros_like(w), np.zeros_like(w)
    gg = tr.grads.cpu().numpy().astype(np.float64)
    for step in (1, 2):
        oracle.adam(w, gg, m0, v0, 1e-3, 0.9, 0.999, 1e-8, step)
        tr.adam(1e-3)
    assert np.allclose(tr.params.cpu().numpy(), w, rtol=0, atol=1e-6)


def test_plan_select_matches_oracle_argmin(spk, sel):
    """plan_select's plan is the argmin, over valid plans, of the FP64 oracle network on
    the same features (near-ties excluded)."""
    P = sel.plan_count(0)
    parts = rand_params(P, seed=3)
    mean = np.linspace(0, 0.5, 33).astype(np.float32)
    scale = np.linspace(0.5, 1.5, 33).astype(np.float32)
    table = {"op": 0, "F": 33, "H": 64, "P": P, "mean": mean.tolist(), "scale": scale.tolist(),
             "params": np.concatenate([a.reshape(-1) for a in parts]).tolist()}
    sel.load_table(table)
    sel._loaded.add(torch.cuda.current_device())  # keep select() from loading the shipped tables
    net = oracle.MLP(*parts)
    checked = 0
    for i, (n, d, K) in enumerate([(3000, 0.01, 64), (8000, 0.001, 256), (2048, 0.1, 32), (20000, 5e-4, 128),
                                   (500, 0.3, 16), (4096, 0.002, 100)]):
        A = synth.bernoulli(n, n, d, i)
        dA = spk.CSR.from_host(A)
        for dt in (0, 1):  # F32 and BF16 dense operands: the dtype input and the valid plans differ
            plan = sel.rank(dA, K, 0, 1, dt)[0]
            x = oracle.selector_inputs(oracle.features(A.row_ptr, A.col_idx, n), K, dt)
            y = net.forward(((x - mean) / scale)[None])[0]
            valid = np.array([ok for _, ok in sel.plan_list(0, K, dt)])
            order = np.argsort(np.where(valid, y, np.inf))
            if y[order[1]] - y[order[0]] < 1e-3:
                continue
            expect = sel.plan_list(0, K, dt)[order[0]][0]
            assert (plan.variant, plan.lanes, plan.chunk, plan.flags) == (expect.variant, expect.lanes, expect.chunk,
                                                                          expect.flags)
            if dt == 0:
                assert sel.select(dA, K, 0, fallback=False) == plan
            checked += 1
    assert checked >= 8
    sel._loaded.clear()


def test_plan_rank_matches_oracle_order(spk, sel):
    """plan_rank lists the valid plans in ascending output of the FP64 oracle network (near-ties
    excluded); its first plan is plan_select's, and select(verify=k) keeps one of the k."""
    P = sel.plan_count(1)
    parts = rand_params(P, seed=4)
    mean = np.linspace(0, 0.5, 33).astype(np.float32)
    scale = np.linspace(0.5, 1.5, 33).astype(np.float32)
    table = {"op": 1, "F": 33, "H": 64, "P": P, "mean": mean.tolist(), "scale": scale.tolist(),
             "params": np.concatenate([a.reshape(-1) for a in parts]).tolist()}
    sel.load_table(table)
    sel._loaded.add(torch.cuda.current_device())
    net = oracle.MLP(*parts)
    checked = 0
    key = lambda p: (p.variant, p.lanes, p.chunk, p.flags)  # noqa: E731
    for i, (n, d, K) in enumerate([(3000, 0.01, 64), (8000, 0.001, 256), (2048, 0.1, 32), (500, 0.3, 16)]):
        A = synth.bernoulli(n, n, d, 20 + i)
        dA = spk.CSR.from_host(A)
        got = sel.rank(dA, K, 1, 6)
        x = oracle.selector_inputs(oracle.features(A.row_ptr, A.col_idx, n), K)
        y = net.forward(((x - mean) / scale)[None])[0]
        plans = sel.plan_list(1, K)
        valid = np.array([ok for _, ok in plans])
        order = [int(j) for j in np.argsort(np.where(valid, y, np.inf), kind="stable") if valid[j]]
        assert len(got) == min(6, len(order))
        for j in range(len(got)):
            if (j > 0 and y[order[j]] - y[order[j - 1]] < 1e-3) or (
                    j + 1 < len(order) and y[order[j + 1]] - y[order[j]] < 1e-3):
                continue
            assert key(got[j]) == key(plans[order[j]][0]), (i, j)
            checked += 1
        assert key(sel.select(dA, K, 1, fallback=False)) == key(got[0])
        assert key(sel.select(dA, K, 1, fallback=False, verify=3)) in {key(p) for p in got[:3]}
    assert checked >= 10
    with pytest.raises(spk.SpkError):
        sel.rank(spk.CSR.from_host(synth.bernoulli(100, 100, 0.1, 1)), 64, 1, 33)
    sel._loaded.clear()


def test_training_reduces_loss(spk, sel):
    """A few hundred full-batch steps on a synthetic regression task."""
    P, N = 16, 512
    r = np.random.default_rng(4)
    X = r.normal(size=(N, 33)).astype(np.float32)
    T = np.abs(np.tanh(X[:, :P] * 0.7 + X[:, P:2 * P] * 0.3)).astype(np.float32)
    mask = np.ones((N, P), np.float32)
    tr = sel.Trainer(P, seed=5)
    hist = tr.fit(X, T, mask, steps=600, lr=3e-3)
    assert hist[-1] < 0.25 * hist[0]
