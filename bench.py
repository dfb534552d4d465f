"""Throughput of the SpMM / SDDMM hot path on one MI355X.

A step is one SpMM (C = A B, Eq. 1) plus one SDDMM (S = A (.) (U V^T), Eq. 2)
on the same sparse matrix, with every operand resident in HBM before the
timed region.  The default workload is the paper's headline shape (random
N x N at 90% sparsity, largest N = 65536, Section IV-A) with dense width 64:
uniform column positions, values and dense operands ~ N(0, 1), FP32, seed 0.

Prints ONE JSON line on stdout:
  value      whole-job GFLOP/s (2 nnz K flops per product, both products)
  roofline   for the dominant kernel: algorithmic bytes or flops per launch
             divided by its average launch time (HIP events on the launch
             stream), against the binding MI355X peak
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of rows of the
             same workload on this host's cores (rank 0, one GPU)

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--plan plain|tuned|learned]
  python bench.py --sweep OUT.jsonl    # the n x sparsity x K grid, one record per op
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_VALU_PEAK_TFS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (no packed FP32)

WORKLOADS = {
    # name: (n, density, K, kind)
    "uniform-n65536-s90-K64": (65536, 0.1, 64, "uniform"),
    "uniform-n65536-s90-K128": (65536, 0.1, 128, "uniform"),
    "uniform-n65536-s99-K64": (65536, 0.01, 64, "uniform"),
    "uniform-n65536-s99-K128": (65536, 0.01, 128, "uniform"),
    "uniform-n65536-s99.9-K64": (65536, 0.001, 64, "uniform"),
    "uniform-n65536-s99.9-K128": (65536, 0.001, 128, "uniform"),
    "uniform-n16384-s90-K64": (16384, 0.1, 64, "uniform"),
    "uniform-n16384-s90-K128": (16384, 0.1, 128, "uniform"),
    "uniform-n16384-s99-K64": (16384, 0.01, 64, "uniform"),
    "uniform-n16384-s99-K128": (16384, 0.01, 128, "uniform"),
    "uniform-n16384-s99.9-K64": (16384, 0.001, 64, "uniform"),
    "uniform-n16384-s99.9-K128": (16384, 0.001, 128, "uniform"),
    "uniform-n1024-s90-K64": (1024, 0.1, 64, "uniform"),
}
DEFAULT_WORKLOAD = "uniform-n65536-s90-K64"


def spmm_bytes(m, n, nnz, K, sv=4, sb=4):
    """Compulsory HBM bytes of SpMM: row_ptr, (col, val) per entry, B once, C once."""
    return 4 * (m + 1) + nnz * (4 + sv) + n * K * sb + m * K * 4


def sddmm_bytes(m, n, nnz, K, sv=4, su=4):
    """Compulsory HBM bytes of SDDMM: row_ptr, (col, val, out) per entry, U and V once."""
    return 4 * (m + 1) + nnz * (4 + sv + 4) + m * K * su + n * K * su


def roofline(bytes_, flops, seconds):
    """Binding roof (HBM or FP32 VALU) and the achieved fraction of it."""
    t_hbm = bytes_ / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (FP32_VALU_PEAK_TFS * 1e12)
    if t_hbm >= t_alu:
        ach = bytes_ / seconds / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4)}
    ach = flops / seconds / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_VALU_PEAK_TFS, "unit": "TFLOP/s",
            "frac": round(ach / FP32_VALU_PEAK_TFS, 4)}


def make_problem(name, seed=0):
    from paper_2604_27985_amd import synth

    n, d, K, kind = WORKLOADS[name]
    if kind == "uniform":
        return synth.uniform_problem(n, d, K, seed)
    raise ValueError(kind)


def to_device(p):
    import torch

    import paper_2604_27985_amd as spk

    dA = spk.CSR.from_host(p.A, p.vals)
    B = torch.from_numpy(p.B).cuda()
    U = torch.from_numpy(p.U).cuda()
    V = torch.from_numpy(p.V).cuda()
    return dA, B, U, V


def choose_plans(mode, dA, K, B, U, V):
    """(spmm plan, sddmm plan) for plain (NULL plans), tuned (timed search) or learned."""
    import paper_2604_27985_amd as spk

    if mode == "plain":
        return None, None
    if mode == "learned":
        from paper_2604_27985_amd import selector

        return selector.select(dA, K, spk.OP_SPMM), selector.select(dA, K, spk.OP_SDDMM)
    from paper_2604_27985_amd import autotune

    return autotune.best_plan(dA, K, spk.OP_SPMM, B=B)[0], autotune.best_plan(dA, K, spk.OP_SDDMM, U=U, V=V)[0]


def time_steps(dA, B, U, V, p_spmm, p_sddmm, steps, warmup):
    """Run warmup + timed steps; per-kernel HIP events on the launch stream."""
    import torch

    import paper_2604_27985_amd as spk

    C = torch.empty((dA.m, B.shape[1]), dtype=torch.float32, device="cuda")
    S = torch.empty(dA.nnz, dtype=torch.float32, device="cuda")
    ws_nb = spk.workspace_bytes(spk.OP_SPMM, dA, B.shape[1], p_spmm)
    ws = torch.empty(max(ws_nb, 1), dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        spk.spmm(dA, B, plan=p_spmm, out=C, workspace=ws if ws_nb else None)
        spk.sddmm(dA, U, V, plan=p_sddmm, out=S)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    for s in range(steps):
        ev[s][0].record()
        spk.spmm(dA, B, plan=p_spmm, out=C, workspace=ws if ws_nb else None)
        ev[s][1].record()
        spk.sddmm(dA, U, V, plan=p_sddmm, out=S)
        ev[s][2].record()
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    spmm_ms = [e[0].elapsed_time(e[1]) for e in ev]
    sddmm_ms = [e[1].elapsed_time(e[2]) for e in ev]
    return total_ms, wall, spmm_ms, sddmm_ms, C, S


def cpu_baseline(p, C, S, budget_s=12.0):
    """FP64 oracle on the first rows of the workload, sized to about budget_s of CPU work;
    also reports the scaled error of the GPU results on those rows."""
    import numpy as np

    import oracle

    A = p.A
    K = p.K
    rp = A.row_ptr
    # calibrate on a small slice, then take as many rows as the budget allows
    rows = max(1, min(A.m, 64))
    t0 = time.perf_counter()
    oracle.spmm(rp[:rows + 1], A.col_idx, p.vals, p.B)
    oracle.sddmm(rp[:rows + 1], A.col_idx, p.vals, p.U, p.V)
    dt = max(time.perf_counter() - t0, 1e-4)
    rows = int(min(A.m, max(rows, rows * budget_s / dt)))
    t0 = time.perf_counter()
    C64, CM = oracle.spmm(rp[:rows + 1], A.col_idx, p.vals, p.B)
    S64, SM = oracle.sddmm(rp[:rows + 1], A.col_idx, p.vals, p.U, p.V)
    dt = time.perf_counter() - t0
    nnz_s = int(rp[rows]) - int(rp[0])
    S64, SM = S64[:nnz_s], SM[:nnz_s]  # entries of the sampled rows (row_ptr starts at 0)
    flops = 2.0 * nnz_s * K * 2
    c = C[:rows].cpu().numpy().astype(np.float64)
    s = S[: nnz_s].cpu().numpy().astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ec = np.where(CM > 0, np.abs(c - C64) / CM, np.abs(c - C64))
        es = np.where(SM > 0, np.abs(s - S64) / SM, np.abs(s - S64))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"first {rows} of {A.m} rows ({nnz_s} entries), SpMM + SDDMM in FP64, {dt:.1f} s",
            "gpu_max_scaled_err": float(max(ec.max(initial=0.0), es.max(initial=0.0)))}


def run_workload(args):
    import numpy as np
    import torch

    name = args.workload
    n, d, K, kind = WORKLOADS[name]
    t0 = time.perf_counter()
    p = make_problem(name)
    gen_s = time.perf_counter() - t0
    dA, B, U, V = to_device(p)
    torch.cuda.synchronize()
    p_spmm, p_sddmm = choose_plans(args.plan, dA, K, B, U, V)
    total_ms, wall, spmm_ms, sddmm_ms, C, S = time_steps(dA, B, U, V, p_spmm, p_sddmm, args.steps, args.warmup)
    nnz = p.A.nnz
    flops_step = 2.0 * nnz * K * 2
    ms_step = total_ms / args.steps
    value = flops_step / (ms_step * 1e-3) / 1e9
    t_spmm = float(np.mean(spmm_ms)) * 1e-3
    t_sddmm = float(np.mean(sddmm_ms)) * 1e-3
    b_spmm = spmm_bytes(p.A.m, p.A.n, nnz, K)
    b_sddmm = sddmm_bytes(p.A.m, p.A.n, nnz, K)
    f_one = 2.0 * nnz * K
    dominant = "spmm" if t_spmm >= t_sddmm else "sddmm"
    roof = roofline(b_spmm if dominant == "spmm" else b_sddmm, f_one, max(t_spmm, t_sddmm))
    roof["kernel"] = dominant
    roof["traffic"] = None
    out = {
        "metric": "SpMM/SDDMM GFLOP/s + % HBM roofline; learned-tuned vs plain at 1e-5 rel err",
        "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "n": n, "sparsity": 1 - d, "nnz": nnz, "K": K, "pattern": kind,
                   "ops": "spmm+sddmm", "plan": args.plan,
                   "plans": {"spmm": p_spmm.name() if p_spmm else "plain", "sddmm": p_sddmm.name() if p_sddmm else "plain"}},
        "roofline": roof,
        "kernels": {
            "spmm": {"ms": round(t_spmm * 1e3, 4), "gflops": round(f_one / t_spmm / 1e9, 1),
                     "hbm_frac": round(b_spmm / t_spmm / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": b_spmm},
            "sddmm": {"ms": round(t_sddmm * 1e3, 4), "gflops": round(f_one / t_sddmm / 1e9, 1),
                      "hbm_frac": round(b_sddmm / t_sddmm / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": b_sddmm},
        },
        "host_wall_s": round(wall, 3), "gen_s": round(gen_s, 2),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, C, S, args.cpu_budget)
    print(json.dumps(out), flush=True)


def run_sweep(args):
    """One record per (workload, op, plan mode) of the n x sparsity x K grid."""
    import numpy as np
    import torch

    import paper_2604_27985_amd as spk

    names = [w for w in WORKLOADS if w != "uniform-n1024-s90-K64"]
    with open(args.sweep, "w") as f:
        for name in names:
            n, d, K, kind = WORKLOADS[name]
            p = make_problem(name)
            dA, B, U, V = to_device(p)
            for mode in args.sweep_modes.split(","):
                ps, pd = choose_plans(mode, dA, K, B, U, V)
                total_ms, wall, spmm_ms, sddmm_ms, _, _ = time_steps(dA, B, U, V, ps, pd, args.steps, args.warmup)
                for op, ms, plan, b in (("spmm", spmm_ms, ps, spmm_bytes(p.A.m, n, p.A.nnz, K)),
                                        ("sddmm", sddmm_ms, pd, sddmm_bytes(p.A.m, n, p.A.nnz, K))):
                    t = float(np.median(ms)) * 1e-3
                    rec = {"workload": name, "op": op, "mode": mode, "plan": plan.name() if plan else "plain",
                           "n": n, "sparsity": 1 - d, "K": K, "nnz": p.A.nnz, "ms_median": round(t * 1e3, 4),
                           "gflops": round(2.0 * p.A.nnz * K / t / 1e9, 1), "alg_bytes": b,
                           "hbm_frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4),
                           "roofline": roofline(b, 2.0 * p.A.nnz * K, t)}
                    f.write(json.dumps(rec) + "\n")
                    f.flush()
                    print(json.dumps(rec), file=sys.stderr, flush=True)
            del dA, B, U, V
            torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--plan", default="tuned", choices=["plain", "tuned", "learned"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--sweep", default=None, help="write the grid sweep to this JSONL file")
    ap.add_argument("--sweep-modes", default="plain,tuned")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(row-sharded designs are described but not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.sweep:
        run_sweep(args)
    else:
        run_workload(args)


if __name__ == "__main__":
    main()
