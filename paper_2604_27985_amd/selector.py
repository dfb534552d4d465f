"""Learned plan selection: data, training and inference around the C ABI.

The network, its training step (forward, hand-derived backward, Adam) and
inference run in the library's HIP kernels; this module only organises the
data:

  specs      seeded descriptions of synthetic matrices (size, density,
             pattern family, dense width K)
  timings    every plan of an op timed on the GPU for each matrix (the
             exhaustive search), appended to a resumable JSONL file
  training   inputs standardised with the training split's mean and scale,
             targets log(t_plan / t_best) on the valid plans, full-batch Adam
  inference  plan_select (features -> inputs -> network -> masked argmin)

The exhaustive search (autotune) stays the fallback when no model is loaded
and is the yardstick of the selector's regret.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import time

import numpy as np
import torch

from . import _lib, api, synth
from ._lib import OP_SDDMM, OP_SELECT, OP_SPMM

F, H = 33, 64
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "selector_weights.json")
PATTERNS = ("uniform", "banded", "powerlaw", "block4")
KS = (32, 64, 128, 256)
NNZ_CAP = 1 << 24


# ---------------------------------------------------------------- plan lists
def plan_count(op: int) -> int:
    return int(_lib.load().plan_count(op))


DTYPES = {"f32": _lib.F32, "bf16": _lib.BF16}
TORCH_DTYPES = {"f32": torch.float32, "bf16": torch.bfloat16}


def dtype_code(t) -> int:
    """spk_dtype of a torch dtype, a tensor, or a record's dtype name (F32 for None)."""
    if t is None:
        return _lib.F32
    if isinstance(t, str):
        return DTYPES[t]
    if isinstance(t, torch.Tensor):
        t = t.dtype
    return {torch.float32: _lib.F32, torch.bfloat16: _lib.BF16, torch.float64: _lib.F64}[t]


def plan_list(op: int, K: int, dtype: int = _lib.F32) -> list[tuple[api.Plan, bool]]:
    """[(plan, valid for K and the dense dtype)] in the op's plan-list order (include/spk.h)."""
    lib = _lib.load()
    out = []
    for i in range(plan_count(op)):
        p = _lib.spk_plan()
        v = ctypes.c_int32(0)
        _lib.check(lib.plan_of_index(op, i, K, dtype, ctypes.byref(p), ctypes.byref(v)), "plan_of_index")
        out.append((api.Plan(p.variant, p.lanes, p.chunk, p.flags), bool(v.value)))
    return out


# ---------------------------------------------------------------- specs
def sample_spec(index: int, cap: int = NNZ_CAP) -> dict:
    """Matrix `index` of the selector set.  Indices below LARGE_FIRST: n
    log-uniform in [4096, 524288] (multiple of 64), density log-uniform in
    [1e-4, 0.1] (redrawn while the expected entry count exceeds `cap`),
    pattern and K uniform.  From LARGE_FIRST on, the regime of the paper's
    workloads (N x N up to N = 65536 at 90-99.9% sparsity, and denser): n
    log-uniform in [8192, 131072], density log-uniform in [1e-3, 0.3] (at most
    LARGE_CAP expected entries), half of them uniform."""
    if index >= BF16_FIRST:
        return _bf16_spec(index)
    if index >= LARGE_FIRST:
        return _large_spec(index)
    rng = np.random.default_rng([2604, 27985, index])
    pattern = PATTERNS[int(rng.integers(len(PATTERNS)))]
    K = KS[int(rng.integers(len(KS)))]
    while True:  # redraw (n, density) until the expected entry count fits the cap
        n = int(round(math.exp(rng.uniform(math.log(4096), math.log(524288))) / 64) * 64)
        d = math.exp(rng.uniform(math.log(1e-4), math.log(0.1)))
        if expected_nnz(n, d, pattern) <= cap:
            break
    return {"index": index, "n": n, "density": d, "pattern": pattern, "K": K, "seed": index,
            "split": "test" if index % 5 == 0 else "train"}


LARGE_FIRST = 2000
LARGE_CAP = 6e8
BF16_FIRST, BF16_LAST = 3000, 3600


def _bf16_spec(index: int) -> dict:
    """BF16 dense operands: the first family's distribution with K in {64, 128,
    256} (the BF16 workload's widths)."""
    rng = np.random.default_rng([2604, 27985, 2, index])
    pattern = PATTERNS[int(rng.integers(len(PATTERNS)))]
    K = (64, 128, 256)[int(rng.integers(3))]
    while True:
        n = int(round(math.exp(rng.uniform(math.log(4096), math.log(524288))) / 64) * 64)
        d = math.exp(rng.uniform(math.log(1e-4), math.log(0.1)))
        if expected_nnz(n, d, pattern) <= NNZ_CAP:
            break
    return {"index": index, "n": n, "density": d, "pattern": pattern, "K": K, "seed": index, "dtype": "bf16",
            "split": "test" if index % 5 == 0 else "train"}


def _large_spec(index: int) -> dict:
    rng = np.random.default_rng([2604, 27985, 1, index])
    pattern = "uniform" if rng.uniform() < 0.5 else PATTERNS[1 + int(rng.integers(len(PATTERNS) - 1))]
    K = KS[int(rng.integers(len(KS)))]
    while True:
        n = int(round(math.exp(rng.uniform(math.log(8192), math.log(131072))) / 64) * 64)
        d = math.exp(rng.uniform(math.log(1e-3), math.log(0.3)))
        if expected_nnz(n, d, pattern) <= LARGE_CAP:
            break
    return {"index": index, "n": n, "density": d, "pattern": pattern, "K": K, "seed": index,
            "split": "test" if index % 5 == 0 else "train"}


def expected_nnz(n: int, d: float, pattern: str) -> float:
    if pattern == "banded":
        return n * 129 * min(1.0, d * n / 129)
    if pattern == "powerlaw":
        return n * max(1.0, d * n)
    return d * n * n


def make_matrix(spec: dict):
    """Host CSR and values of a spec (banded: in-band probability min(1, d n / 129);
    power-law: Zipf 2.1 degrees with mean max(1, d n))."""
    n, d, seed, pat = spec["n"], spec["density"], spec["seed"], spec["pattern"]
    if pat == "uniform":
        A = synth.bernoulli(n, n, d, seed)
    elif pat == "banded":
        A = synth.bernoulli(n, n, min(1.0, d * n / 129), seed, band=64)
    elif pat == "powerlaw":
        A = synth.powerlaw(n, min(float(n), max(1.0, d * n)), 2.1, seed)
    else:
        A = synth.block4(n, n, d, seed)
    return A, synth.normal(A.nnz, seed, synth.S_VALS)


# ---------------------------------------------------------------- features
def features(A: api.CSR) -> torch.Tensor:
    """Integer features (device int64[28]) from the GPU feature kernels."""
    lib = _lib.load()
    dev = A.row_ptr.device
    f = torch.empty(28, dtype=torch.int64, device=dev)
    nb = api.workspace_bytes(OP_SELECT, A, 0)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    ca = A.c(use_vals=False)
    _lib.check(lib.csr_features(ctypes.byref(ca), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nb,
                                api._stream()), "csr_features")
    return f


def inputs(f: torch.Tensor, K: int, dtype: int = _lib.F32) -> torch.Tensor:
    """The 33 network inputs (device float32) of features f, width K and dense dtype."""
    lib = _lib.load()
    x = torch.empty(F, dtype=torch.float32, device=f.device)
    _lib.check(lib.selector_inputs(ctypes.c_void_p(f.data_ptr()), K, dtype, ctypes.c_void_p(x.data_ptr()),
                                   api._stream()), "selector_inputs")
    return x


# ---------------------------------------------------------------- timings
def time_plans(A: api.CSR, K: int, op: int, reps: int = 3, warmup: int = 1,
               indices: list[int] | None = None, dtype: str = "f32") -> list[float | None]:
    """Median ms of every plan of the op's list, or of the plans `indices`
    only (None where invalid for K and dtype), dense operands of `dtype`."""
    from . import autotune

    dev = A.row_ptr.device
    tdt = TORCH_DTYPES[dtype]
    B = torch.randn(A.n, K, device=dev).to(tdt)
    U = torch.randn(A.m, K, device=dev).to(tdt) if op == OP_SDDMM else None
    out = []
    plans = plan_list(op, K, dtype_code(dtype))
    for plan, valid in (plans if indices is None else [plans[i] for i in indices]):
        if not valid:
            out.append(None)
            continue
        if plan.variant == _lib.VAR_BSR4:
            A.block_form()  # conversion is per-pattern preprocessing, not timed
        out.append(autotune.time_plan(A, K, op, plan, B=B, U=U, V=B, reps=reps, warmup=warmup))
    return out


def build_timings(path: str, count: int = 2000, start: int = 0, ops=(OP_SPMM, OP_SDDMM), log=print,
                  time_budget_s: float | None = None) -> int:
    """Append one record per spec index in [start, count) not yet in `path`."""
    done = set()
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                done.add(json.loads(line)["index"])
    t0 = time.time()
    added = 0
    with open(path, "a") as fh:
        for i in range(start, count):
            if i in done:
                continue
            if time_budget_s is not None and time.time() - t0 > time_budget_s:
                break
            spec = sample_spec(i)
            tg = time.time()
            A, v = make_matrix(spec)
            dA = api.CSR.from_host(A, v)
            f = features(dA)
            rec = dict(spec, nnz=A.nnz, features=f.cpu().tolist(), gen_s=round(time.time() - tg, 3))
            for op in ops:
                rec["ms_" + ("spmm" if op == OP_SPMM else "sddmm")] = time_plans(dA, spec["K"], op,
                                                                                 dtype=spec.get("dtype", "f32"))
            fh.write(json.dumps(rec) + "\n")
            fh.flush()
            added += 1
            log(f"[{i}] {spec['pattern']} n={spec['n']} nnz={A.nnz} K={spec['K']} "
                f"best spmm {min(t for t in rec['ms_spmm'] if t is not None):.4f} ms ({time.time() - t0:.0f} s)")
            del dA
    return added


def load_timings(path: str) -> list[dict]:
    with open(path) as fh:
        return [json.loads(line) for line in fh]


def extend_timings(path: str, out_path: str, op: int, indices: list[int], log=print,
                   time_budget_s: float | None = None, min_k: int = 0) -> int:
    """Time plans added to an op's list after `path` was built, or plans whose
    definition changed for widths K >= min_k: every matrix of `path` with
    K >= min_k is generated again from its spec (seeded) and only plans
    `indices` are timed.  Appends {"index", "op", "plans", "ms"} records to
    `out_path` (resumable); merge_timings folds them into the timing set."""
    done = set()
    if os.path.exists(out_path):
        with open(out_path) as fh:
            for line in fh:
                done.add(json.loads(line)["index"])
    t0 = time.time()
    added = 0
    key = "spmm" if op == OP_SPMM else "sddmm"
    with open(out_path, "a") as fh:
        for rec in load_timings(path):
            i = rec["index"]
            if i in done or rec["K"] < min_k:
                continue
            if time_budget_s is not None and time.time() - t0 > time_budget_s:
                break
            spec = {k: rec[k] for k in ("index", "n", "density", "pattern", "K", "seed", "split")}
            A, v = make_matrix(spec)
            assert A.nnz == rec["nnz"], f"matrix {i} does not regenerate"
            dA = api.CSR.from_host(A, v)
            ms = time_plans(dA, spec["K"], op, indices=indices, dtype=rec.get("dtype", "f32"))
            fh.write(json.dumps({"index": i, "op": key, "plans": indices, "ms": ms}) + "\n")
            fh.flush()
            added += 1
            log(f"[{i}] n={spec['n']} nnz={A.nnz} K={spec['K']}: {added} matrices extended ({time.time() - t0:.0f} s)")
            del dA
    return added


def merge_timings(path: str, ext_path: str, out_path: str) -> int:
    """Fold extend_timings records into the timing set: the op's time list of
    each record is widened to the op's plan count with the new plans' times."""
    ext = {}
    with open(ext_path) as fh:
        for line in fh:
            e = json.loads(line)
            ext[(e["index"], e["op"])] = e
    merged = 0
    with open(out_path + ".tmp", "w") as fh:
        for rec in load_timings(path):
            for op in (OP_SPMM, OP_SDDMM):
                key = "spmm" if op == OP_SPMM else "sddmm"
                times = list(rec.get("ms_" + key, []))
                times += [None] * (plan_count(op) - len(times))
                e = ext.get((rec["index"], key))
                if e is not None:
                    for p, t in zip(e["plans"], e["ms"]):
                        times[p] = t
                    merged += 1
                rec["ms_" + key] = times
            fh.write(json.dumps(rec) + "\n")
    os.replace(out_path + ".tmp", out_path)
    return merged


# ---------------------------------------------------------------- dataset
def dataset(records: list[dict], op: int):
    """(X inputs [N, 32], T targets [N, P], mask [N, P], times [N, P]) for an op.
    Inputs come from the GPU input kernel on the recorded integer features."""
    key = "ms_spmm" if op == OP_SPMM else "ms_sddmm"
    P = plan_count(op)
    dev = torch.device("cuda")
    feats = torch.tensor([r["features"] for r in records], dtype=torch.int64, device=dev)
    X = torch.stack([inputs(feats[i].contiguous(), r["K"], dtype_code(r.get("dtype")))
                     for i, r in enumerate(records)]).cpu().numpy()
    times = np.full((len(records), P), np.nan)
    for i, r in enumerate(records):
        for p, t in enumerate(r[key]):
            if t is not None and t > 0:
                times[i, p] = t
    mask = np.isfinite(times).astype(np.float32)
    best = np.nanmin(times, axis=1, keepdims=True)
    T = np.where(mask > 0, np.log(np.where(mask > 0, times, 1.0) / best), 0.0).astype(np.float32)
    return X.astype(np.float32), T, mask, times


# ---------------------------------------------------------------- training
class Trainer:
    """Full-batch training of the selector network with the library's kernels."""

    def __init__(self, P: int, hidden: int = H, seed: int = 0):
        self.P, self.H = P, hidden
        g = torch.Generator().manual_seed(seed)

        def init(o, i):  # He-uniform
            lim = math.sqrt(6.0 / i)
            return (torch.rand(o, i, generator=g) * 2 - 1) * lim

        parts = [init(hidden, F), torch.zeros(hidden), init(hidden, hidden), torch.zeros(hidden),
                 init(P, hidden) * 0.1, torch.zeros(P)]
        self.params = torch.cat([t.reshape(-1) for t in parts]).cuda().contiguous()
        self.mom = torch.zeros_like(self.params)
        self.vel = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, device="cuda")
        self.step_no = 0

    def loss_grad(self, X: torch.Tensor, T: torch.Tensor, mask: torch.Tensor) -> float:
        lib = _lib.load()
        nb = lib.mlp_workspace_bytes(F, self.H, self.P, X.shape[0])
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        _lib.check(lib.mlp_loss_grad(p(self.params), F, self.H, self.P, p(X), p(T), p(mask), X.shape[0],
                                     p(self.grads), p(self.loss), p(ws), nb, api._stream()), "mlp_loss_grad")
        return self.loss

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> None:
        lib = _lib.load()
        self.step_no += 1
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        _lib.check(lib.adam_update(p(self.params), p(self.grads), p(self.mom), p(self.vel), self.params.numel(), lr,
                                   b1, b2, eps, self.step_no, api._stream()), "adam_update")

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        lib = _lib.load()
        Y = torch.empty((X.shape[0], self.P), dtype=torch.float32, device="cuda")
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        _lib.check(lib.mlp_forward(p(self.params), F, self.H, self.P, p(X), X.shape[0], p(Y), api._stream()),
                   "mlp_forward")
        return Y

    def fit(self, X, T, mask, steps: int = 4000, lr: float = 3e-3, log=None) -> list[float]:
        Xd, Td, Md = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, T, mask))
        hist = []
        for s in range(steps):
            lr_s = lr * 0.5 * (1 + math.cos(math.pi * s / steps))  # cosine decay
            self.loss_grad(Xd, Td, Md)
            self.adam(max(lr_s, lr * 0.01))
            if s % 200 == 0 or s == steps - 1:
                hist.append(float(self.loss.item()))
                if log:
                    log(f"step {s} loss {hist[-1]:.5f}")
        return hist


def choose(Y: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """Argmin of predictions over valid plans, per row."""
    return np.where(valid > 0, Y, np.inf).argmin(axis=1)


def best_of_top(Y: np.ndarray, valid: np.ndarray, times: np.ndarray, k: int) -> np.ndarray:
    """Per row, the fastest (by recorded time) of the k valid plans with the
    lowest predictions: what a caller timing the network's k best picks."""
    top = np.argsort(np.where(valid > 0, Y, np.inf), axis=1, kind="stable")[:, :k]
    t = np.take_along_axis(np.where(np.isnan(times), np.inf, times), top, axis=1)
    return top[np.arange(top.shape[0]), t.argmin(axis=1)]


def regret_stats(times: np.ndarray, pick: np.ndarray, plain_idx: np.ndarray) -> dict:
    rows = np.arange(times.shape[0])
    best = np.nanmin(times, axis=1)
    t_pick = times[rows, pick]
    t_plain = times[rows, plain_idx]
    r = t_pick / best
    return {"count": int(len(r)), "geomean_regret": float(np.exp(np.mean(np.log(r)))),
            "median_regret": float(np.median(r)), "p90_regret": float(np.quantile(r, 0.9)),
            "max_regret": float(r.max()), "total_time_ratio": float(t_pick.sum() / best.sum()),
            "geomean_gain_over_plain": float(np.exp(np.mean(np.log(t_plain / t_pick)))),
            "geomean_plain_regret": float(np.exp(np.mean(np.log(t_plain / best))))}


def plain_index(op: int, K: int) -> int:
    """Index of the plan a NULL plan runs (row-split SpMM with the smallest lanes
    >= K/4; entry-split SDDMM with 8 lanes widened to fit K)."""
    if op == OP_SPMM:
        lanes = 4
        while lanes < 64 and lanes * 4 < K:
            lanes <<= 1
        return int(math.log2(lanes)) - 2
    lanes = 8
    while lanes < 64 and -(-K // (lanes * 4)) > 8:
        lanes <<= 1
    return 5 + int(math.log2(lanes)) - 2


def time_weights(times: np.ndarray, rows: np.ndarray, power: float) -> np.ndarray:
    """Per-matrix loss weights (best time / median best time)^power, clipped to
    [1/16, 16] and scaled to mean 1 over `rows`: with power > 0 the network
    weighs the matrices whose time dominates a total more."""
    best = np.nanmin(times, axis=1)
    w = np.clip((best / np.median(best[rows])) ** power, 1.0 / 16, 16.0)
    return (w / w[rows].mean()).astype(np.float32)


def train_op(records: list[dict], op: int, steps: int = 4000, lr: float = 3e-3, seed: int = 0, log=None,
             weight_power: float = 0.0):
    """Train on the train split, evaluate on the test split; returns (table dict, report).
    weight_power > 0 weighs each matrix's squared errors by its best time
    (time_weights), which favours the total-time ratio."""
    X, T, mask, times = dataset(records, op)
    split = np.array([r["split"] for r in records])
    tr, te = split == "train", split == "test"
    mean = X[tr].mean(0)
    scale = X[tr].std(0)
    scale = np.where(scale > 1e-6, scale, 1.0).astype(np.float32)
    Xs = ((X - mean) / scale).astype(np.float32)
    P = plan_count(op)
    trainer = Trainer(P, seed=seed)
    wmask = mask * time_weights(times, tr, weight_power)[:, None] if weight_power > 0 else mask
    hist = trainer.fit(Xs[tr], T[tr], wmask[tr], steps=steps, lr=lr, log=log)
    table = {"op": int(op), "F": F, "H": trainer.H, "P": P, "mean": mean.tolist(), "scale": scale.tolist(),
             "params": trainer.params.cpu().tolist(), "seed": seed, "steps": steps, "lr": lr,
             "plans": [p.name() for p, _ in plan_list(op, 64)]}
    report = evaluate(records, table)
    report.update({"loss_history": hist, "weight_power": weight_power})
    return table, report


def evaluate(records: list[dict], table: dict) -> dict:
    """Regret of a network's picks on the train and test splits (first choice,
    and the best of its first 3 and 5 choices by the recorded times)."""
    op = table["op"]
    X, _, mask, times = dataset(records, op)
    split = np.array([r["split"] for r in records])
    tr, te = split == "train", split == "test"
    mean, scale = np.asarray(table["mean"], np.float32), np.asarray(table["scale"], np.float32)
    Xs = np.ascontiguousarray(((X - mean) / scale).astype(np.float32))
    net = Trainer(table["P"], table["H"])
    net.params = torch.tensor(table["params"], dtype=torch.float32, device="cuda")
    Y = net.forward(torch.from_numpy(Xs).cuda()).cpu().numpy()
    pick = choose(Y, mask)
    plain = np.array([plain_index(op, r["K"]) for r in records])
    report = {"op": "spmm" if op == OP_SPMM else "sddmm",
              "train": regret_stats(times[tr], pick[tr], plain[tr]),
              "test": regret_stats(times[te], pick[te], plain[te])}
    bf = np.array([r.get("dtype", "f32") == "bf16" for r in records])
    if (te & bf).any():
        report["test_bf16"] = regret_stats(times[te & bf], pick[te & bf], plain[te & bf])
        report["test_f32"] = regret_stats(times[te & ~bf], pick[te & ~bf], plain[te & ~bf])
    for k in (3, 5):
        pk = best_of_top(Y, mask, times, k)
        report[f"test_best_of_top{k}"] = regret_stats(times[te], pk[te], plain[te])
    return report


def split_params(table: dict) -> list[np.ndarray]:
    """W1 [H, F], b1 [H], W2 [H, H], b2 [H], W3 [P, H], b3 [P] of a table."""
    F, H, P = table["F"], table["H"], table["P"]
    flat = np.asarray(table["params"], np.float64)
    shapes = [(H, F), (H,), (H, H), (H,), (P, H), (P,)]
    out, at = [], 0
    for s in shapes:
        size = int(np.prod(s))
        out.append(flat[at:at + size].reshape(s))
        at += size
    assert at == flat.size, "parameter count does not match F, H, P"
    return out


def merge_tables(tables: list[dict]) -> dict:
    """One network whose output is the mean of the members' outputs: hidden
    layers stacked (layer 1 rows concatenated, layer 2 block-diagonal, so each
    member's units see only its own), layer 3 side by side scaled by 1/n and
    the output biases averaged.  Members share op, F, P and the input
    standardisation (trained on one split of one timing set)."""
    t0, n = tables[0], len(tables)
    for t in tables[1:]:
        if (t["op"], t["F"], t["P"]) != (t0["op"], t0["F"], t0["P"]) or t["mean"] != t0["mean"] or \
                t["scale"] != t0["scale"]:
            raise ValueError("members differ in op, sizes or input standardisation")
    parts = [split_params(t) for t in tables]
    W1 = np.concatenate([q[0] for q in parts], 0)
    b1 = np.concatenate([q[1] for q in parts])
    Hs = [q[2].shape[0] for q in parts]
    W2 = np.zeros((sum(Hs), sum(Hs)))
    at = 0
    for q, h in zip(parts, Hs):
        W2[at:at + h, at:at + h] = q[2]
        at += h
    b2 = np.concatenate([q[3] for q in parts])
    W3 = np.concatenate([q[4] for q in parts], 1) / n
    b3 = np.mean([q[5] for q in parts], 0)
    out = dict(t0)
    out["H"] = int(sum(Hs))
    out["params"] = np.concatenate([a.reshape(-1) for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float32).tolist()
    out["seed"] = [t["seed"] for t in tables]
    return out


# ---------------------------------------------------------------- inference
def load_table(table: dict) -> None:
    lib = _lib.load()
    host = np.ascontiguousarray(np.concatenate([table["mean"], table["scale"], table["params"]]).astype(np.float32))
    _lib.check(lib.selector_load(table["op"], ctypes.c_void_p(host.ctypes.data), table["F"], table["H"], table["P"]),
               "selector_load")


_loaded = set()


def load_default(path: str = WEIGHTS_PATH) -> bool:
    """Load the trained tables shipped with the package (once per device)."""
    dev = torch.cuda.current_device()
    if dev in _loaded:
        return True
    if not os.path.exists(path):
        return False
    with open(path) as fh:
        tables = json.load(fh)["tables"]
    for t in tables:
        load_table(t)
    _loaded.add(dev)
    return True


def offline_choices(table: dict, records: list[dict]) -> np.ndarray:
    """Plan index the loaded network picks for each recorded matrix (GPU inputs
    kernel on the recorded features, then the GPU network)."""
    op = table["op"]
    X, _, mask, _ = dataset(records, op)
    mean, scale = np.asarray(table["mean"], np.float32), np.asarray(table["scale"], np.float32)
    Xs = np.ascontiguousarray(((X - mean) / scale).astype(np.float32))
    tr = Trainer(table["P"], table["H"])
    tr.params = torch.tensor(table["params"], dtype=torch.float32, device="cuda")
    Y = tr.forward(torch.from_numpy(Xs).cuda()).cpu().numpy()
    valid = np.array([[ok for _, ok in plan_list(op, r["K"], dtype_code(r.get("dtype")))] for r in records],
                     np.float32)
    return choose(Y, valid)


def rank(A: api.CSR, K: int, op: int, k: int, dtype: int = _lib.F32) -> list[api.Plan]:
    """The network's k best plans for (A, K, op) with dense operands of
    `dtype`, best first (plan_rank)."""
    lib = _lib.load()
    load_default()
    nb = api.workspace_bytes(OP_SELECT, A, K)
    ws = torch.empty(nb, dtype=torch.uint8, device=A.row_ptr.device)
    ca = A.c(use_vals=False)
    out = (_lib.spk_plan * k)()
    count = ctypes.c_int32(0)
    st = lib.plan_rank(ctypes.byref(ca), K, op, dtype, k, out, ctypes.byref(count), ctypes.c_void_p(ws.data_ptr()),
                       nb, api._stream())
    _lib.check(st, "plan_rank")
    return [api.Plan(p.variant, p.lanes, p.chunk, p.flags) for p in out[:count.value]]


def select(A: api.CSR, K: int, op: int, fallback: bool = True, verify: int = 1, B=None, U=None,
           V=None) -> api.Plan:
    """Learned plan for (A, K, op) via plan_select; the timed search when no
    model is available.  verify > 1 times the network's `verify` best plans
    on the given operands (random ones of A's shape if None) and keeps the
    fastest: a short timed search that guards against a mispredicted first
    choice."""
    lib = _lib.load()
    dt = dtype_code(B if op == OP_SPMM else U)
    if verify > 1:
        try:
            cands = rank(A, K, op, verify, dt)
        except _lib.SpkError as e:
            if e.status != -10 or not fallback:
                raise
            from . import autotune

            return autotune.best_plan(A, K, op, B=B, U=U, V=V)[0]
        from . import autotune

        if op == OP_SPMM and B is None:
            B = torch.randn(A.n, K, device=A.row_ptr.device)
        if op == OP_SDDMM and (U is None or V is None):
            tdt = U.dtype if U is not None else torch.float32
            U = torch.randn(A.m, K, device=A.row_ptr.device).to(tdt)
            V = torch.randn(A.n, K, device=A.row_ptr.device).to(tdt)
        timed = []
        for p in cands:
            if p.variant == _lib.VAR_BSR4:
                A.block_form()  # per-pattern preprocessing, not timed
            timed.append((autotune.time_plan(A, K, op, p, B=B, U=U, V=V, reps=3, warmup=1), p))
        return min(timed, key=lambda t: t[0])[1]
    load_default()
    nb = api.workspace_bytes(OP_SELECT, A, K)
    ws = torch.empty(nb, dtype=torch.uint8, device=A.row_ptr.device)
    ca = A.c(use_vals=False)
    out = _lib.spk_plan()
    st = lib.plan_select(ctypes.byref(ca), K, op, dt, ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), nb,
                         api._stream())
    if st == -10 and fallback:
        from . import autotune

        return autotune.best_plan(A, K, op)[0]
    _lib.check(st, "plan_select")
    return api.Plan(out.variant, out.lanes, out.chunk, out.flags)


def main(argv=None) -> None:
    """python -m paper_2604_27985_amd.selector build|train ..."""
    import argparse

    ap = argparse.ArgumentParser(prog="python -m paper_2604_27985_amd.selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build", help="time every plan on seeded synthetic matrices (resumable)")
    b.add_argument("--out", required=True)
    b.add_argument("--count", type=int, default=2000)
    b.add_argument("--start", type=int, default=0)
    b.add_argument("--budget", type=float, default=None, help="stop after this many seconds")
    e = sub.add_parser("extend", help="time plans added to an op's list on an existing timing set (resumable)")
    e.add_argument("--timings", required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--op", choices=("spmm", "sddmm"), required=True)
    e.add_argument("--plans", required=True, help="first-last plan indices, e.g. 16-19")
    e.add_argument("--budget", type=float, default=None, help="stop after this many seconds")
    e.add_argument("--min-k", type=int, default=0, help="only matrices with dense width K >= this")
    g = sub.add_parser("merge", help="fold extend records into a timing set")
    g.add_argument("--timings", required=True)
    g.add_argument("--ext", required=True)
    g.add_argument("--out", required=True)
    m = sub.add_parser("ensemble", help="average trained networks of one op into one and evaluate it")
    m.add_argument("--timings", required=True)
    m.add_argument("--members", required=True, nargs="+", help="weight files each holding a table of the op")
    m.add_argument("--op", choices=("spmm", "sddmm"), required=True)
    m.add_argument("--out", default=WEIGHTS_PATH)
    m.add_argument("--report", default=None)
    t = sub.add_parser("train", help="train the selector networks on a timing set")
    t.add_argument("--timings", required=True)
    t.add_argument("--out", default=WEIGHTS_PATH)
    t.add_argument("--report", default=None)
    t.add_argument("--steps", type=int, default=4000)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--weight-power", type=float, default=0.0,
                   help="weigh each matrix by (best time / median)^p in the loss")
    t.add_argument("--ops", default="spmm,sddmm",
                   help="ops to train; the other ops' tables are kept from --out")
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if args.cmd == "build":
        n = build_timings(args.out, count=args.count, start=args.start, time_budget_s=args.budget, log=log)
        print(f"added {n} records", flush=True)
        return
    if args.cmd == "extend":
        lo, hi = (int(x) for x in args.plans.split("-"))
        op = OP_SPMM if args.op == "spmm" else OP_SDDMM
        n = extend_timings(args.timings, args.out, op, list(range(lo, hi + 1)), log=log, time_budget_s=args.budget,
                           min_k=args.min_k)
        print(f"extended {n} records", flush=True)
        return
    if args.cmd == "merge":
        print(f"merged {merge_timings(args.timings, args.ext, args.out)} extensions", flush=True)
        return
    records = load_timings(args.timings)
    if args.cmd == "ensemble":
        op = OP_SPMM if args.op == "spmm" else OP_SDDMM
        members = []
        for path in args.members:
            with open(path) as fh:
                members += [t for t in json.load(fh)["tables"] if t["op"] == op]
        table = merge_tables(members)
        report = evaluate(records, table)
        report["members"] = table["seed"]
        print(json.dumps(report), flush=True)
        tables = [table]
        if os.path.exists(args.out):  # keep the other op's table
            with open(args.out) as fh:
                tables = [t for t in json.load(fh)["tables"] if t["op"] != op] + tables
        with open(args.out, "w") as fh:
            json.dump({"format": 1, "device": torch.cuda.get_device_name(0),
                       "timings": os.path.basename(args.timings), "records": len(records),
                       "tables": sorted(tables, key=lambda t: t["op"])}, fh)
        if args.report:
            kept = []
            if os.path.exists(args.report):
                with open(args.report) as fh:
                    kept = [r for r in json.load(fh) if r["op"] != report["op"]]
            with open(args.report, "w") as fh:
                json.dump(sorted(kept + [report], key=lambda r: r["op"] != "spmm"), fh, indent=1)
        return
    ops = [OP_SPMM if o == "spmm" else OP_SDDMM for o in args.ops.split(",")]
    kept = {}
    if set(ops) != {OP_SPMM, OP_SDDMM} and os.path.exists(args.out):
        with open(args.out) as fh:
            kept = {t["op"]: t for t in json.load(fh)["tables"]}
    tables, reports = [], []
    for op in (OP_SPMM, OP_SDDMM):
        if op not in ops:
            if op in kept:
                tables.append(kept[op])
            continue
        table, report = train_op(records, op, steps=args.steps, lr=args.lr, seed=args.seed, log=log,
                                 weight_power=args.weight_power)
        tables.append(table)
        reports.append(report)
        print(json.dumps({k: v for k, v in report.items() if k != "loss_history"}), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump({"format": 1, "device": torch.cuda.get_device_name(0), "timings": os.path.basename(args.timings),
                   "records": len(records), "tables": tables}, fh)
    if args.report:
        if kept and os.path.exists(args.report):  # keep the reports of ops not retrained
            with open(args.report) as fh:
                fresh = {r["op"] for r in reports}
                reports = [r for r in json.load(fh) if r["op"] not in fresh] + reports
        with open(args.report, "w") as fh:
            json.dump(reports, fh, indent=1)


if __name__ == "__main__":
    main()
