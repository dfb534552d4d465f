"""Throughput of the SpMM / SDDMM hot path on one MI355X.

A step is one pass of the hot path over one synthetic matrix with every
operand resident in HBM before the timed region:
  uniform        SpMM (C = A B, Eq. 1) + SDDMM (S = A (.) (U V^T), Eq. 2), FP32
  powerlaw-bf16  the same two products with BF16 dense operands, FP32 accumulation
  gcn            forward SpMM + backward (dB = A^T G, dvals = SDDMM(pattern, G, B)),
                 FP32; the transpose is per-pattern preprocessing, timed once
The default workload is the largest single-GPU configuration of the scaling
sweep: the paper's headline shape (random N x N at 90% sparsity, the largest
N = 65536, Section IV-A) with dense width 128: uniform column positions,
values and dense operands ~ N(0, 1), FP32, seed 0.

Prints ONE JSON line on stdout:
  value         whole-job GFLOP/s (2 nnz K flops per product, all products)
  roofline      for the dominant kernel: algorithmic bytes or flops per launch
                over its average launch time (HIP events on the launch stream),
                against the binding MI355X peak (HBM 8 TB/s, or the FP32 VALU
                rate of 78.6 TFLOP/s without packed FP32)
  cpu_baseline  the FP64 CPU oracle timed on the first rows of the same
                workload (about --cpu-budget seconds) on this host's cores
  kernels       per part: mean and median time over the timed steps (warm:
                operands the previous step left in L2 and the MALL stay
                there) and cold_ms, the median of five launches each preceded
                by a 1 GiB read that evicts them
  parity        the largest |gpu - oracle| / (|A| |B|) over the oracle's
                sample, against the 1e-5 gate

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
    # name: (n, density or mean degree, K, kind)
    "powerlaw-n1048576-mean32-K256-bf16": (1 << 20, 32, 256, "powerlaw-bf16"),
    "gcn-n262144-mean16-K128": (262144, 16, 128, "gcn"),
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
    # hyper-sparse: most rows of the dense operands are never referenced
    "uniform-n1048576-d1e-06-K64": (1 << 20, 1e-6, 64, "uniform"),
    "uniform-n1048576-d1e-07-K64": (1 << 20, 1e-7, 64, "uniform"),
    "uniform-n2097152-d1e-07-K64": (1 << 21, 1e-7, 64, "uniform"),
    "attention-powerlaw-n262144-mean16-K64": (262144, 16, 64, "attention"),
}
DEFAULT_WORKLOAD = "uniform-n65536-s90-K128"
SWEEP = [w for w, v in WORKLOADS.items() if v[3] == "uniform" and 16384 <= v[0] <= 65536]
HYPER = [w for w, v in WORKLOADS.items() if v[3] == "uniform" and v[0] > 65536]


def touched_bytes(A, K):
    """Bytes of the rows the products actually reference (hyper-sparse
    patterns leave most rows of the dense operands untouched): SpMM reads the
    referenced rows of B and writes all of C; SDDMM reads the rows of U of the
    non-empty rows and the referenced rows of V."""
    import numpy as np

    cols = int(np.unique(A.col_idx).size)
    rows = int(np.count_nonzero(np.diff(A.row_ptr)))
    spmm = 4 * (A.m + 1) + A.nnz * 8 + cols * K * 4 + A.m * K * 4
    sddmm = 4 * (A.m + 1) + A.nnz * 12 + rows * K * 4 + cols * K * 4
    return {"spmm": spmm, "sddmm": sddmm}


def spmm_bytes(m, n, nnz, K, sv=4, sb=4, perm=False):
    """Compulsory HBM bytes of SpMM: row_ptr, (col, val) per entry, B once, C once
    (plus a 4-byte perm entry per stored value for A^T G)."""
    return 4 * (m + 1) + nnz * (4 + sv + (4 if perm else 0)) + n * K * sb + m * K * 4


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


# ------------------------------------------------------------------ profiles
PROFILES = os.path.join(ROOT, "profiles")
# kernels of each part of a step (rocprofv3 names), for attributing counter readings
PART_KERNELS = {"spmm": ("spmm_", "slab_bounds_kernel", "merge_partition_kernel", "merge_fixup_kernel",
                         "gather_vals_kernel", "zero_rows_kernel"),
                "sddmm": ("sddmm_",),
                "attention": ("attn_",),
                "softmax": ("softmax_",)}


def kernel_source_digest():
    """sha256 (16 hex digits) of the HIP sources and the C header: counter
    readings taken from another source state are not reported."""
    import glob
    import hashlib

    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2604_27985_amd", "csrc", "*")))
    for f in files + [os.path.join(ROOT, "include", "spk.h")]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _read_csv(path):
    import csv

    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(d, suffix):
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def _part_of(kernel):
    short = kernel.split("(")[0].split("<")[0].replace("void ", "").replace("spk::", "").strip()
    for part, prefixes in PART_KERNELS.items():
        if any(short.startswith(p) for p in prefixes):
            return part, short
    return None, short


def profile_summary(args):
    """Markdown summary of one rocprofv3 trace pass and two counter passes
    (FETCH_SIZE, WRITE_SIZE) of the same bench command, written to --out.
    DIR also holds cmd.txt (the commands), trace.log (the run's output) and
    digest.txt (kernel_source_digest() of the profiled tree).
    Counter readings (KiB per dispatch) are scaled by what the same counters
    read for the run's device copy of --calib-copy GiB (that many GiB read and
    written), then summed per part of a step and divided by the steps run."""
    d = args.profile_summary
    with open(os.path.join(d, "cmd.txt")) as fh:
        cmds = [ln.rstrip("\n") for ln in fh if ln.strip()]
    line = None
    with open(os.path.join(d, "trace.log")) as fh:
        for ln in fh:
            if ln.startswith("{") and '"metric"' in ln:
                line = json.loads(ln)
    if line is None:
        raise SystemExit("the trace run printed no bench line")
    runs = line["steps"] + line["warmup"]
    stats = _read_csv(_find(os.path.join(d, "trace"), "kernel_stats.csv"))
    per = {}
    for tag, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        for r in _read_csv(_find(os.path.join(d, tag), "counter_collection.csv")):
            if r["Counter_Name"] != counter:
                continue
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            per.setdefault(tag, {}).setdefault(key, 0.0)
            per[tag][key] += float(r["Counter_Value"])
    calib_bytes = float(args.calib_copy << 30)
    factor = {}
    for tag in ("fetch", "write"):
        copies = [v for (_, k), v in per[tag].items() if "copy" in k.lower()]
        factor[tag] = calib_bytes / (max(copies) * 1024.0) if copies and max(copies) > 0 else None
    by_kernel = {}
    for tag in ("fetch", "write"):
        for (_, k), v in per[tag].items():
            e = by_kernel.setdefault(k, {"fetch": [], "write": []})
            e[tag].append(v)
    part_bytes = {}
    rows = []
    for k, e in sorted(by_kernel.items(), key=lambda kv: -sum(kv[1]["fetch"])):
        part, short = _part_of(k)
        nf, nw = len(e["fetch"]), len(e["write"])
        fkib = sum(e["fetch"]) / max(nf, 1)
        wkib = sum(e["write"]) / max(nw, 1)
        scaled = None
        if factor["fetch"] and factor["write"]:
            scaled = fkib * 1024 * factor["fetch"] + wkib * 1024 * factor["write"]
            if part:
                part_bytes[part] = part_bytes.get(part, 0.0) + scaled * nf / runs
        rows.append((short, part or "-", nf, fkib, wkib, scaled))
    # the digest of the sources the profiled run was built from, recorded
    # beside the counters when they were taken
    with open(os.path.join(d, "digest.txt")) as fh:
        digest = fh.read().strip()
    out = [f"# rocprofv3: {line['config']['workload']}", "",
           "Commands (repository root, one MI355X; each counter in a pass of its own):", ""]
    out += ["    " + c for c in cmds]
    out += ["", f"Plans: {json.dumps(line['config']['plans'])}; {line['steps']} timed + {line['warmup']} warmup "
            f"steps; bench line: {line['ms_per_step']} ms per step.", "",
            f"Kernel sources: sha256 {digest} (paper_2604_27985_amd/csrc/*, include/spk.h).", "",
            "## Kernel time (--kernel-trace --stats)", "",
            "| kernel | calls | average us | total ms |", "|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        out.append(f"| {_part_of(r['Name'])[1]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} |")
    fr = "none found" if factor["fetch"] is None else f"{factor['fetch']:.4f}"
    wr = "none found" if factor["write"] is None else f"{factor['write']:.4f}"
    out += ["", "## HBM traffic per dispatch (FETCH_SIZE, WRITE_SIZE)", "",
            f"Calibration: the device copy of {args.calib_copy} GiB (read and written once); "
            f"scale factors FETCH {fr}, WRITE {wr}.", "",
            "| kernel | part | dispatches | FETCH KiB | WRITE KiB | scaled HBM bytes |", "|---|---|---|---|---|---|"]
    for short, part, n, f, w, sc in rows[:14]:
        out.append(f"| {short} | {part} | {n} | {f:.0f} | {w:.0f} | {'-' if sc is None else f'{sc:.4g}'} |")
    out += _counter_tables(d)
    if line["config"]["ops"] in ("spmm+sddmm", "attention"):
        out += ["", "Per step (scaled bytes of a part's kernels over the steps run), read by bench.py while the",
                "kernel sources keep the digest above:", "", "```"]
        for part, b in sorted(part_bytes.items()):
            if part not in line["config"]["plans"]:
                continue  # kernels of a comparison run, not of the step
            plan = line["config"]["plans"][part]
            out.append(f"traffic {line['config']['workload']} {part} {plan} {b:.0f} {digest}")
        out += ["```", ""]
        if line["config"]["ops"] == "attention" and "attention" in part_bytes:
            # the unfused chain the bench line times beside the fused kernel
            chain = {k: part_bytes.get(k, 0.0) for k in ("sddmm", "softmax", "spmm")}
            tot = sum(chain.values())
            out += [f"Fused attention: {part_bytes['attention']:.4g} HBM bytes per step; the unfused chain "
                    f"(SDDMM {chain['sddmm']:.4g}, row softmax {chain['softmax']:.4g}, SpMM {chain['spmm']:.4g}): "
                    f"{tot:.4g} bytes per step ({tot / part_bytes['attention']:.2f}x the fused kernel's).", ""]
    else:  # the backward runs SpMM kernels too: kernel names do not separate the parts
        out += ["", "No per-part traffic: forward and backward share kernel names.", ""]
    with open(args.out, "w") as fh:
        fh.write("\n".join(out))
    print("\n".join(out))


def _counter_medians(d):
    """{kernel: {counter: median per dispatch}} of one counter pass under d."""
    import numpy as np

    vals = {}
    for r in _read_csv(_find(d, "counter_collection.csv")):
        key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
        vals.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], {}).setdefault(key, 0.0)
        vals[r["Kernel_Name"]][r["Counter_Name"]][key] += float(r["Counter_Value"])
    return {k: {c: float(np.median(list(v.values()))) for c, v in cs.items()} for k, cs in vals.items()}


def _counter_tables(d):
    """Optional passes: sq/ (LDS bank conflicts and instruction mix) and tcc/
    (L2-to-fabric read requests by size, which FETCH_SIZE weighs)."""
    out = []
    sq_dir, tcc_dir = os.path.join(d, "sq"), os.path.join(d, "tcc")
    if os.path.isdir(sq_dir):
        med = _counter_medians(sq_dir)
        out += ["", "## LDS bank conflicts and instruction mix (SQ counters, median per dispatch)", "",
                "conflict ratio = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE (the stalled share of the cycles the "
                "LDS serves indexed reads and writes).  waves/SIMD = SQ_WAVE_CYCLES / (8 SQ_BUSY_CYCLES): the mean "
                "number of resident waves, with SQ_WAVE_CYCLES counted in 4-cycle units over all waves and "
                "SQ_BUSY_CYCLES summed over the 32 shader engines of 1024 SIMDs.", "",
                "| kernel | SQ_LDS_BANK_CONFLICT | SQ_LDS_IDX_ACTIVE | conflict ratio | SQ_INSTS_LDS | "
                "SQ_INSTS_VALU | SQ_WAIT_INST_LDS | SQ_WAVES | SQ_WAVE_CYCLES | SQ_BUSY_CYCLES | waves/SIMD |",
                "|---|---|---|---|---|---|---|---|---|---|---|"]
        for k, c in sorted(med.items(), key=lambda kv: -kv[1].get("SQ_WAVE_CYCLES", 0.0)):
            if "copy" in k.lower() or "elementwise" in k:
                continue
            g = lambda n: c.get(n, float("nan"))  # noqa: E731
            ratio = g("SQ_LDS_BANK_CONFLICT") / g("SQ_LDS_IDX_ACTIVE") if g("SQ_LDS_IDX_ACTIVE") else float("nan")
            out.append(f"| {_part_of(k)[1]} | {g('SQ_LDS_BANK_CONFLICT'):.3g} | {g('SQ_LDS_IDX_ACTIVE'):.3g} | "
                       f"{ratio:.3f} | {g('SQ_INSTS_LDS'):.3g} | {g('SQ_INSTS_VALU'):.3g} | "
                       f"{g('SQ_WAIT_INST_LDS'):.3g} | {g('SQ_WAVES'):.3g} | {g('SQ_WAVE_CYCLES'):.3g} | "
                       f"{g('SQ_BUSY_CYCLES'):.3g} | {g('SQ_WAVE_CYCLES') / (8 * g('SQ_BUSY_CYCLES')):.2f} |")
    if os.path.isdir(tcc_dir):
        med = _counter_medians(tcc_dir)
        out += ["", "## Read-request sizes behind FETCH_SIZE (TCC counters, median per dispatch)", "",
                "FETCH_SIZE weighs TCC_BUBBLE requests as 128 B, TCC_EA0_RDREQ_32B as 32 B and the rest as 64 B. "
                "The calibration factor measured on the device copy holds for a kernel whose requests split the "
                "same way.", "",
                "| kernel | TCC_EA0_RDREQ | 32 B share | TCC_BUBBLE share | other (64 B) share |", "|---|---|---|---|---|"]
        for k, c in sorted(med.items(), key=lambda kv: -kv[1].get("TCC_EA0_RDREQ_sum", 0.0)):
            tot = c.get("TCC_EA0_RDREQ_sum", 0.0)
            if tot <= 0:
                continue
            r32 = c.get("TCC_EA0_RDREQ_32B_sum", 0.0) / tot
            rb = c.get("TCC_BUBBLE_sum", 0.0) / tot
            out.append(f"| {_part_of(k)[1]} | {tot:.4g} | {r32:.3f} | {rb:.3f} | {1 - r32 - rb:.3f} |")
    return out


def recorded_traffic(workload, part, plan):
    """HBM bytes per launch of a step part from profiles/, or None when no
    summary matches this workload, part and plan at the current sources."""
    if not os.path.isdir(PROFILES):
        return None
    digest = kernel_source_digest()
    for f in sorted(os.listdir(PROFILES)):
        if not f.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, f)) as fh:
            for ln in fh:
                t = ln.split()
                if len(t) == 6 and t[0] == "traffic" and t[1:4] == [workload, part, plan] and t[5] == digest:
                    return int(float(t[4]))
    return None


def make_problem(name, seed=0):
    from paper_2604_27985_amd import synth

    n, d, K, kind = WORKLOADS[name]
    if kind == "uniform":
        return synth.uniform_problem(n, d, K, seed)
    if kind == "powerlaw-bf16":
        return synth.powerlaw_problem(n, d, K, 2.1, seed)
    if kind == "gcn":
        # vals U(0,1) learnable, B and G ~ N(0,1); SDDMM(pattern, G, B) takes U = G, V = B
        p = synth.powerlaw_problem(n, d, K, 2.1, seed, dense=("B", "G"))
        p.U, p.V = p.G, p.B
        return p
    raise ValueError(kind)


def to_device(p, kind):
    import torch

    import paper_2604_27985_amd as spk

    dA = spk.CSR.from_host(p.A, p.vals)
    dt = torch.bfloat16 if kind == "powerlaw-bf16" else torch.float32
    B = torch.from_numpy(p.B).cuda().to(dt)
    U = torch.from_numpy(p.U).cuda().to(dt)
    V = B if p.V is p.B else torch.from_numpy(p.V).cuda().to(dt)
    return dA, B, U, V


VERIFY = 5  # candidates of the learned ranking timed before the run


# plan variants spmm_csr_backward takes for its A^T product and its pattern
# SDDMM (rows, merge-path, column slabs, LDS slabs); the forms built per
# pattern (blocks, 16-bit slabs, compressed rows, COO) have their own calls
BACKWARD_VARIANTS = (0, 1, 3, 4)


def autotune_sweep(A, K, B, plans):
    import paper_2604_27985_amd as spk
    from paper_2604_27985_amd import autotune

    return autotune.sweep(A, K, spk.OP_SPMM, B=B, plans=plans, reps=3, warmup=1)


def autotune_sweep_sddmm(A, K, U, V, plans):
    import paper_2604_27985_amd as spk
    from paper_2604_27985_amd import autotune

    return autotune.sweep(A, K, spk.OP_SDDMM, U=U, V=V, plans=plans, reps=3, warmup=1)


def choose_plans(mode, dA, K, B, U, V, kind):
    """(spmm plan, sddmm plan): NULL plans (plain), a timed search (tuned), or the selector."""
    import paper_2604_27985_amd as spk

    if mode == "plain":
        return None, None
    if mode == "learned":
        from paper_2604_27985_amd import selector

        # the network's VERIFY best plans, timed once on these operands
        p1 = selector.select(dA, K, spk.OP_SPMM, verify=VERIFY, B=B)
        if kind == "gcn":
            # the backward's product runs on A^T: ask for a plan for that matrix
            # among the variants spmm_csr_backward takes
            trp, tci, _ = dA.transpose()
            AT = spk.CSR(trp, tci, None, (dA.n, dA.m))
            cands = [p for p in selector.rank(AT, K, spk.OP_SPMM, 16) if p.variant in BACKWARD_VARIANTS]
            return p1, min(autotune_sweep(AT, K, U, cands[:VERIFY]), key=lambda r: r[1])[0]
        return p1, selector.select(dA, K, spk.OP_SDDMM, verify=VERIFY, U=U, V=V)
    from paper_2604_27985_amd import autotune

    def log(line):  # the search is long on large patterns: one line per timed plan
        print(line, file=sys.stderr, flush=True)

    p1 = autotune.best_plan(dA, K, spk.OP_SPMM, B=B, log=log)[0]
    if kind == "gcn":
        trp, tci, perm = dA.transpose()
        AT = spk.CSR(trp, tci, None, (dA.n, dA.m))
        plans = [p for p in autotune.plans_for(spk.OP_SPMM, K) if p.variant in BACKWARD_VARIANTS]
        return p1, min(autotune.sweep(AT, K, spk.OP_SPMM, B=U, plans=plans, log=log), key=lambda r: r[1])[0]
    return p1, autotune.best_plan(dA, K, spk.OP_SDDMM, U=U, V=V, log=log)[0]


def choose_dvals_plan(mode, dA, K, U, V):
    """The GCN backward's pattern SDDMM (dvals = SDDMM(pattern, G, B)): NULL
    (plain), the timed search, or the network's best plans timed once."""
    import paper_2604_27985_amd as spk

    if mode == "plain":
        return None
    if mode == "learned":
        from paper_2604_27985_amd import selector

        cands = [p for p in selector.rank(dA, K, spk.OP_SDDMM, 16) if p.variant in BACKWARD_VARIANTS]
        return min(autotune_sweep_sddmm(dA, K, U, V, cands[:VERIFY]), key=lambda r: r[1])[0]
    from paper_2604_27985_amd import autotune

    plans = [p for p in autotune.plans_for(spk.OP_SDDMM, K) if p.variant in BACKWARD_VARIANTS]
    return min(autotune.sweep(dA, K, spk.OP_SDDMM, U=U, V=V, plans=plans), key=lambda r: r[1])[0]


class Step:
    """One pass of the hot path with preallocated outputs and workspaces."""

    def __init__(self, dA, B, U, V, p_spmm, p_sddmm, kind, p_dvals=None):
        import torch

        import paper_2604_27985_amd as spk

        self.spk, self.kind = spk, kind
        self.dA, self.B, self.U, self.V = dA, B, U, V
        self.p_spmm, self.p_sddmm, self.p_dvals = p_spmm, p_sddmm, p_dvals
        K = B.shape[1]
        self.C = torch.empty((dA.m, K), dtype=torch.float32, device="cuda")
        self.S = torch.empty(dA.nnz, dtype=torch.float32, device="cuda")
        nb = spk.workspace_bytes(spk.OP_SPMM, dA, K, p_spmm)
        self.ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        nb = spk.workspace_bytes(spk.OP_SDDMM, dA, K, p_sddmm)
        self.ws2 = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        if kind == "gcn":
            self.G = U
            self.dB = torch.empty((dA.n, K), dtype=torch.float32, device="cuda")
            nb = spk.backward_workspace_bytes(dA, K, p_sddmm, p_dvals)
            self.ws3 = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            spk.csr_transpose(dA)  # warm
            ev0.record()
            t = spk.csr_transpose(dA)  # per-pattern preprocessing, cached on the matrix
            ev1.record()
            torch.cuda.synchronize()
            dA._transpose = t
            self.transpose_ms = ev0.elapsed_time(ev1)

    def first(self):
        self.spk.spmm(self.dA, self.B, plan=self.p_spmm, out=self.C, workspace=self.ws)

    def second(self):
        if self.kind == "gcn":
            # one backward call: p_sddmm is the plan of its A^T product,
            # p_dvals that of its pattern SDDMM
            self.spk.spmm_backward(self.dA, self.B, self.G, plan=self.p_sddmm, dvals_plan=self.p_dvals,
                                   out_dB=self.dB, out_dvals=self.S, workspace=self.ws3)
        else:
            self.spk.sddmm(self.dA, self.U, self.V, plan=self.p_sddmm, out=self.S, workspace=self.ws2)


def time_steps(step, steps, warmup):
    """Warmup, then `steps` timed steps; per-part HIP events on the launch stream."""
    import torch

    for _ in range(warmup):
        step.first()
        step.second()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    for s in range(steps):
        ev[s][0].record()
        step.first()
        ev[s][1].record()
        step.second()
        ev[s][2].record()
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    first_ms = [e[0].elapsed_time(e[1]) for e in ev]
    second_ms = [e[1].elapsed_time(e[2]) for e in ev]
    return total_ms, wall, first_ms, second_ms


def time_cold(step, reps=5, flush_bytes=1 << 30):
    """Median per-part times with the caches cold: before each launch a 1 GiB
    buffer (four times the 256 MB MALL, far beyond the L2s) is read, so the
    launch finds none of its operands cached.  Reading rather than writing
    leaves clean lines behind, so no write-backs compete with the launch."""
    import numpy as np
    import torch

    scratch = torch.ones(flush_bytes // 4, dtype=torch.float32, device="cuda")
    out = []
    for part in (step.first, step.second):
        ts = []
        for _ in range(reps):
            scratch.sum()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            part()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        out.append(float(np.median(ts)))
    del scratch
    torch.cuda.empty_cache()
    return out


def cpu_baseline(p, kind, C, S, budget_s=12.0):
    """FP64 oracle (SpMM + SDDMM) on the first rows of the workload, sized to about
    budget_s of CPU work, timed on this host; also the scaled error of the GPU
    results on those rows."""
    import numpy as np

    import oracle

    A = p.A
    K = p.K
    rp = A.row_ptr
    B, U, V = p.B, p.U, p.V
    if kind == "powerlaw-bf16":  # the GPU consumed the bf16-rounded operands
        B, U = oracle.round_bf16(B), oracle.round_bf16(U)
        V = oracle.round_bf16(V)
    svals = None if kind == "gcn" else p.vals  # the backward's SDDMM is pattern-only
    rows = max(1, min(A.m, 64))
    while True:  # grow the sample until one pass takes at least 1 s, then scale to the budget
        t0 = time.perf_counter()
        oracle.spmm(rp[:rows + 1], A.col_idx, p.vals, B, with_bound=False)
        oracle.sddmm(rp[:rows + 1], A.col_idx, svals, U, V, with_bound=False)
        dt = time.perf_counter() - t0
        if dt >= 1.0 or rows >= A.m:
            break
        rows = min(A.m, rows * 4)
    rows = int(min(A.m, max(rows, rows * budget_s / dt)))
    t0 = time.perf_counter()
    C64, CM = oracle.spmm(rp[:rows + 1], A.col_idx, p.vals, B)
    S64, SM = oracle.sddmm(rp[:rows + 1], A.col_idx, svals, U, V)
    dt = time.perf_counter() - t0
    nnz_s = int(rp[rows]) - int(rp[0])
    S64, SM = S64[:nnz_s], SM[:nnz_s]  # entries of the sampled rows (row_ptr starts at 0)
    flops = 2.0 * nnz_s * K * 2
    c = C[:rows].cpu().numpy().astype(np.float64)
    s = S[:nnz_s].cpu().numpy().astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ec = np.where(CM > 0, np.abs(c - C64) / CM, np.abs(c - C64))
        es = np.where(SM > 0, np.abs(s - S64) / SM, np.abs(s - S64))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"first {rows} of {A.m} rows ({nnz_s} entries): SpMM + SDDMM in FP64, {dt:.1f} s",
            "gpu_max_scaled_err": float(max(ec.max(initial=0.0), es.max(initial=0.0))),
            "gpu_max_scaled_err_parts": {"spmm": float(ec.max(initial=0.0)),
                                         ("dvals" if kind == "gcn" else "sddmm"): float(es.max(initial=0.0))}}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or platform.machine()


def kernel_table(p, kind, K, t1, t2):
    """Per-part time, GFLOP/s and compulsory-byte HBM fraction."""
    m, n, nnz = p.A.m, p.A.n, p.A.nnz
    sb = 2 if kind == "powerlaw-bf16" else 4
    f = 2.0 * nnz * K
    if kind == "gcn":
        # backward = A^T G (with perm) + SDDMM(pattern, G, B)
        b1 = spmm_bytes(m, n, nnz, K)
        b2 = spmm_bytes(n, m, nnz, K, perm=True) + sddmm_bytes(m, n, nnz, K, sv=0)
        names, flops = ("spmm", "backward"), (f, 2 * f)
    else:
        b1 = spmm_bytes(m, n, nnz, K, sb=sb)
        b2 = sddmm_bytes(m, n, nnz, K, su=sb)
        names, flops = ("spmm", "sddmm"), (f, f)
    out = {}
    for name, t, b, fl in zip(names, (t1, t2), (b1, b2), flops):
        out[name] = {"ms": round(t * 1e3, 4), "gflops": round(fl / t / 1e9, 1), "alg_bytes": int(b),
                     "hbm_frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4), "_b": b, "_f": fl, "_t": t}
    return out


def run_workload(args):
    import numpy as np
    import torch

    name = args.workload
    n, d, K, kind = WORKLOADS[name]
    t0 = time.perf_counter()
    p = make_problem(name)
    gen_s = time.perf_counter() - t0
    dA, B, U, V = to_device(p, kind)
    torch.cuda.synchronize()
    p_dvals = None
    if args.plans:  # fixed plans (a profiled run repeats those of a bench line)
        from paper_2604_27985_amd.api import Plan

        named = [None if x == "plain" else Plan.from_name(x) for x in args.plans.split(",")]
        p_spmm, p_sddmm = named[0], named[1]
        if kind == "gcn" and len(named) > 2:
            p_dvals = named[2]
    else:
        p_spmm, p_sddmm = choose_plans(args.plan, dA, K, B, U, V, kind)
        if kind == "gcn":
            p_dvals = choose_dvals_plan(args.plan, dA, K, U, V)
    step = Step(dA, B, U, V, p_spmm, p_sddmm, kind, p_dvals)
    if args.calib_copy:
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE readings
        # calibrate the counters of the kernels profiled in the same run
        src = torch.ones(args.calib_copy << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    total_ms, wall, first_ms, second_ms = time_steps(step, args.steps, args.warmup)
    # a profiled run (--calib-copy) launches only the steps, so that its
    # counters divide by steps + warmup
    cold = [None, None] if args.calib_copy else time_cold(step)
    nnz = p.A.nnz
    kt = kernel_table(p, kind, K, float(np.mean(first_ms)) * 1e-3, float(np.mean(second_ms)) * 1e-3)
    for part, c, ts in zip(kt, cold, (first_ms, second_ms)):
        # warm (the steps above: mean and median) and cold (caches flushed before each launch)
        kt[part]["ms_median"] = round(float(np.median(ts)), 4)
        kt[part]["cold_ms"] = None if c is None else round(c, 4)
    flops_step = sum(v["_f"] for v in kt.values())
    ms_step = total_ms / args.steps
    value = flops_step / (ms_step * 1e-3) / 1e9
    dom = max(kt, key=lambda k: kt[k]["_t"])
    roof = roofline(kt[dom]["_b"], kt[dom]["_f"], kt[dom]["_t"])
    roof["kernel"] = dom
    dom_plan = (p_spmm if dom == "spmm" else p_sddmm)
    roof["traffic"] = recorded_traffic(name, dom, dom_plan.name() if dom_plan else "plain")
    for v in kt.values():
        for key in ("_b", "_f", "_t"):
            v.pop(key)
    cfg = {"workload": name, "n": n, "nnz": nnz, "K": K, "pattern": "uniform" if kind == "uniform" else "powerlaw",
           "ops": "spmm+backward" if kind == "gcn" else "spmm+sddmm",
           "plan": ("fixed" if args.plans else
                    f"learned, best of the top {VERIFY} timed" if args.plan == "learned" else args.plan),
           "plans": {"spmm": p_spmm.name() if p_spmm else "plain",
                     ("backward" if kind == "gcn" else "sddmm"): p_sddmm.name() if p_sddmm else "plain"}}
    if kind == "gcn":
        cfg["plans"]["backward_sddmm"] = p_dvals.name() if p_dvals else "plain"
    if kind == "uniform":
        cfg["sparsity"] = 1 - d
    else:
        cfg["mean_degree"] = d
    out = {
        "metric": "SpMM/SDDMM GFLOP/s + % HBM roofline; learned-tuned vs plain at 1e-5 rel err",
        "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-in/f32-acc" if kind == "powerlaw-bf16" else "f32", "data": "synthetic",
        "config": cfg, "roofline": roof, "kernels": kt,
        "host_wall_s": round(wall, 3), "gen_s": round(gen_s, 2),
    }
    if kind == "gcn":
        out["transpose_ms_once"] = round(step.transpose_ms, 4)
    if args.plan != "plain" and not args.no_compare:
        # the same step with NULL plans (the plain method), for learned-vs-plain
        plain = Step(dA, B, U, V, None, None, kind)
        p_total, _, p1, p2 = time_steps(plain, args.steps, args.warmup)
        p_ms = p_total / args.steps
        out["plain"] = {"ms_per_step": round(p_ms, 4), "value": round(flops_step / (p_ms * 1e-3) / 1e9, 2),
                        "ms": [round(float(np.mean(p1)), 4), round(float(np.mean(p2)), 4)]}
        out["speedup_vs_plain"] = round(p_ms / ms_step, 3)
    if kind in ("uniform", "gcn") and not args.no_compare:
        # F32 operands only: the library takes no BF16 sparse product
        out["library"] = library_times(dA, B, U, V, kt, sddmm=kind == "uniform")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, kind, step.C, step.S, args.cpu_budget)
        out["parity"] = {"max_scaled_err": out["cpu_baseline"]["gpu_max_scaled_err"], "gate": 1e-5,
                         "ok": out["cpu_baseline"]["gpu_max_scaled_err"] <= 1e-5,
                         "sample": out["cpu_baseline"]["sample"].split(":")[0]}
    print(json.dumps(out), flush=True)


def median_ms(f, reps=5, warmup=2):
    """Median milliseconds of `reps` launches of f after `warmup` untimed ones."""
    import torch

    for _ in range(warmup):
        f()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        f()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return sorted(ts)[len(ts) // 2]


def library_times(dA, B, U, V, kt, sddmm=True):
    """The vendor sparse library on the same CSR and F32 operands, as PyTorch
    calls it (torch.sparse.mm and torch.sparse.sampled_addmm, hipSPARSE on
    ROCm, including whatever PyTorch does around the call), against the
    median times of this line's kernels.  The library's sampled product is the
    pattern SDDMM (no multiply by A's values).  Context, not the baseline."""
    import torch

    A = torch.sparse_csr_tensor(dA.row_ptr, dA.col_idx, dA.vals, size=(dA.m, dA.n))
    res = {"what": "torch.sparse.mm / torch.sparse.sampled_addmm (hipSPARSE) on the same CSR, median of 5"}
    t = median_ms(lambda: torch.sparse.mm(A, B))
    res["spmm_ms"] = round(t, 4)
    res["spmm_ratio"] = round(t / kt["spmm"]["ms_median"], 2)
    if sddmm:
        Vt = V.t().contiguous()
        t = median_ms(lambda: torch.sparse.sampled_addmm(A, U, Vt, beta=0.0, alpha=1.0))
        res["sddmm_ms"] = round(t, 4)
        res["sddmm_ratio"] = round(t / kt["sddmm"]["ms_median"], 2)
    del A
    torch.cuda.empty_cache()
    return res


def attention_bytes(m, n, nnz, K1, K2, s=4):
    """Compulsory HBM bytes of the fused chain: row_ptr, (col, val) per entry,
    U, V and B once, O once; the probabilities never leave the chip."""
    return 4 * (m + 1) + nnz * 8 + m * K1 * s + n * K1 * s + n * K2 * s + m * K2 * 4


def attention_problem(name, seed=0):
    """GAT-like scores of unit scale: U, V ~ N(0,1) / K^(1/4), values U(0,1)."""
    from paper_2604_27985_amd import synth

    n, d, K, kind = WORKLOADS[name]
    p = synth.powerlaw_problem(n, d, K, 2.1, seed)
    s = float(K) ** -0.25
    p.U = (p.U * s).astype("float32")
    p.V = (p.V * s).astype("float32")
    return p


def run_attention(args):
    """Attention on A's pattern: the fused one-pass kernel timed as the step,
    the unfused chain (sddmm_csr, csr_row_softmax, spmm_csr) beside it."""
    import numpy as np
    import torch

    import paper_2604_27985_amd as spk
    from paper_2604_27985_amd.api import Plan

    name = args.workload
    n, d, K, kind = WORKLOADS[name]
    t0 = time.perf_counter()
    p = attention_problem(name)
    gen_s = time.perf_counter() - t0
    dA = spk.CSR.from_host(p.A, p.vals)
    U, V, B = (torch.from_numpy(x).cuda() for x in (p.U, p.V, p.B))
    O = torch.empty((p.A.m, K), dtype=torch.float32, device="cuda")
    plan = None
    if args.plans:
        plan = None if args.plans.split(",")[0] == "plain" else Plan.from_name(args.plans.split(",")[0])
    elif args.plan != "plain":
        best = None
        # a short timed choice among entry-split runs and one group per row
        cands = [Plan(1, lanes, chunk) for lanes in (8, 16, 32) for chunk in (256, 512)] + \
                [Plan(0, lanes, 0) for lanes in (8, 16)]
        for cand in cands:
            for _ in range(2):
                spk.attention(dA, U, V, B, plan=cand, out=O)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                spk.attention(dA, U, V, B, plan=cand, out=O)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 5
            if best is None or t < best[1]:
                best = (cand, t)
        plan = best[0]

    nbw = spk.attention_workspace_bytes(dA, K, plan)
    ws_at = torch.empty(nbw, dtype=torch.uint8, device="cuda") if nbw else None

    class _Step:
        def first(self):
            spk.attention(dA, U, V, B, plan=plan, out=O, workspace=ws_at)

        def second(self):
            pass

    step = _Step()
    if args.calib_copy:
        src = torch.ones(args.calib_copy << 28, dtype=torch.float32, device="cuda")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
    total_ms, wall, first_ms, _ = time_steps(step, args.steps, args.warmup)
    nnz = p.A.nnz
    ms = float(np.mean(first_ms))
    flops = 2.0 * nnz * K * 2
    byts = attention_bytes(p.A.m, p.A.n, nnz, K, K)
    roof = roofline(byts, flops, ms * 1e-3)
    roof["kernel"] = "attention"
    roof["traffic"] = recorded_traffic(name, "attention", plan.name() if plan else "plain")
    ms_step = total_ms / args.steps
    out = {
        "metric": "SpMM/SDDMM GFLOP/s + % HBM roofline; learned-tuned vs plain at 1e-5 rel err",
        "value": round(flops / (ms_step * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "n": n, "nnz": nnz, "K": K, "pattern": "powerlaw", "mean_degree": d,
                   "ops": "attention", "plan": "fixed" if args.plans else ("best of 8 timed" if plan else "plain"),
                   "plans": {"attention": plan.name() if plan else "plain"}},
        "roofline": roof,
        "kernels": {"attention": {"ms": round(ms, 4), "ms_median": round(float(np.median(first_ms)), 4),
                                  "gflops": round(flops / (ms * 1e-3) / 1e9, 1), "alg_bytes": int(byts),
                                  "hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}},
        "host_wall_s": round(wall, 3), "gen_s": round(gen_s, 2),
    }
    if not args.no_compare:
        # the unfused chain: S written by the SDDMM, read and rewritten by the
        # softmax, read again as the SpMM's values
        S = torch.empty(nnz, dtype=torch.float32, device="cuda")
        sp_sddmm, sp_spmm = Plan(1, 8, 256), Plan(1, 16, 0)
        from paper_2604_27985_amd import _lib
        import ctypes

        nbs = int(_lib.load().row_softmax_workspace_bytes(ctypes.byref(dA.c(use_vals=False))))
        ws_sm = torch.empty(max(nbs, 1), dtype=torch.uint8, device="cuda")
        parts = (lambda: spk.sddmm(dA, U, V, plan=sp_sddmm, out=S),
                 lambda: spk.csr_row_softmax(dA, S, workspace=ws_sm),
                 lambda: spk.spmm(dA, B, plan=sp_spmm, vals=S, out=O))
        for _ in range(args.warmup):
            for f in parts:
                f()
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        for e in ev:
            for i, f in enumerate(parts):
                e[i].record()
                f()
            e[3].record()
        torch.cuda.synchronize()
        t = [[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in ev]
        um = [float(np.mean([x[i] for x in t])) for i in range(3)]
        ub = (sddmm_bytes(p.A.m, p.A.n, nnz, K) + 4 * (p.A.m + 1) + 8 * nnz
              + spmm_bytes(p.A.m, p.A.n, nnz, K))
        out["unfused"] = {"ms": round(sum(um), 4), "parts_ms": {"sddmm": round(um[0], 4), "softmax": round(um[1], 4),
                                                                "spmm": round(um[2], 4)},
                          "plans": {"sddmm": sp_sddmm.name(), "spmm": sp_spmm.name()}, "alg_bytes": int(ub)}
        out["speedup_vs_unfused"] = round(sum(um) / ms, 3)
        del S
    if not args.no_cpu_baseline:
        import oracle

        rows = 64
        while True:  # about args.cpu_budget seconds of the oracle on the first rows
            t0 = time.perf_counter()
            oracle.sddmm_softmax_spmm(p.A.row_ptr[:rows + 1], p.A.col_idx, p.vals, p.U, p.V, p.B)
            dt = time.perf_counter() - t0
            if dt >= 1.0 or rows >= p.A.m:
                break
            rows = min(p.A.m, rows * 4)
        rows = int(min(p.A.m, max(rows, rows * args.cpu_budget / dt)))
        t0 = time.perf_counter()
        O64, M, E, _ = oracle.sddmm_softmax_spmm(p.A.row_ptr[:rows + 1], p.A.col_idx, p.vals, p.U, p.V, p.B)
        dt = time.perf_counter() - t0
        spk.attention(dA, U, V, B, plan=plan, out=O)
        got = O[:rows].cpu().numpy().astype(np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            err = np.where(M > 0, np.abs(got - O64) / M, np.abs(got - O64))
        nnz_s = int(p.A.row_ptr[rows])
        out["cpu_baseline"] = {"value": round(2.0 * nnz_s * K * 2 / dt / 1e9, 3), "unit": "GFLOP/s",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"first {rows} of {p.A.m} rows ({nnz_s} entries): the three-step chain in "
                                         f"FP64, {dt:.1f} s",
                               "gpu_max_scaled_err": float(err.max(initial=0.0))}
        gate = 1e-5 + 4 * K * 2.0 ** -24 * float(E.max(initial=0.0))
        out["parity"] = {"max_scaled_err": float(err.max(initial=0.0)), "gate": gate,
                         "ok": float(err.max(initial=0.0)) <= gate,
                         "sample": out["cpu_baseline"]["sample"].split(":")[0]}
    print(json.dumps(out), flush=True)


def run_sweep(args):
    """One record per (workload, op, plan mode) of the n x sparsity x K grid."""
    import numpy as np
    import torch

    with open(args.sweep, "w") as f:
        for name in (HYPER if args.sweep_set == "hyper" else SWEEP):
            n, d, K, kind = WORKLOADS[name]
            p = make_problem(name)
            dA, B, U, V = to_device(p, kind)
            touched = touched_bytes(p.A, K) if args.sweep_set == "hyper" else None
            for mode in args.sweep_modes.split(","):
                print(f"{name}: {mode} plans", file=sys.stderr, flush=True)
                ps, pd = choose_plans(mode, dA, K, B, U, V, kind)
                step = Step(dA, B, U, V, ps, pd, kind)
                _, _, first_ms, second_ms = time_steps(step, args.steps, args.warmup)
                kt = kernel_table(p, kind, K, float(np.median(first_ms)) * 1e-3, float(np.median(second_ms)) * 1e-3)
                for op, plan in (("spmm", ps), ("sddmm", pd)):
                    v = kt[op]
                    rec = {"workload": name, "op": op, "mode": mode, "plan": plan.name() if plan else "plain",
                           "n": n, "sparsity": 1 - d, "K": K, "nnz": p.A.nnz, "ms_median": v["ms"],
                           "gflops": v["gflops"], "alg_bytes": v["alg_bytes"], "hbm_frac": v["hbm_frac"],
                           "roofline": roofline(v["_b"], v["_f"], v["_t"])}
                    if touched:
                        rec["touched_bytes"] = touched[op]
                        rec["touched_roofline"] = roofline(touched[op], v["_f"], v["_t"])
                    f.write(json.dumps(rec) + "\n")
                    f.flush()
                    print(json.dumps(rec), file=sys.stderr, flush=True)
                del step
            del dA, B, U, V
            torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--plan", default="learned", choices=["plain", "tuned", "learned"])
    ap.add_argument("--plans", default=None, help="fixed plans SPMM,SDDMM (or SPMM,BACKWARD,BACKWARD_SDDMM) by name, e.g. "
                    "tile/l16/c128/f2,tile/l16/c64/f6; overrides --plan")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain-plan comparison")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="GIB",
                    help="also run one device copy of this many GiB (counter calibration)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--sweep", default=None, help="write the grid sweep to this JSONL file")
    ap.add_argument("--sweep-modes", default="plain,tuned")
    ap.add_argument("--sweep-set", default="grid", choices=["grid", "hyper"],
                    help="the n x sparsity x K grid, or the hyper-sparse patterns (n = 2^20, 2^21)")
    ap.add_argument("--profile-summary", default=None, metavar="DIR",
                    help="summarise the rocprofv3 passes under DIR (cmd.txt, digest.txt, trace.log, trace/, "
                         "fetch/, write/) into --out; no GPU needed")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args)
        return
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
    elif WORKLOADS[args.workload][3] == "attention":
        run_attention(args)
    else:
        run_workload(args)


if __name__ == "__main__":
    if sys.argv[1:] == ["--source-digest"]:  # recorded beside profiles when they are taken
        print(kernel_source_digest())
        sys.exit(0)
    main()
