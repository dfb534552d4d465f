"""Exhaustive plan search: time every plan of the plan space on the GPU.

This is the fallback of the learned selector and the yardstick of its regret:
for a matrix, K and op it launches every valid plan through the C ABI,
times each with HIP events on the launch stream (median of `reps` after
`warmup` launches) and returns the fastest.
"""
from __future__ import annotations

import torch

from . import api
from ._lib import OP_SDDMM, OP_SPMM, VAR_MERGE, VAR_ROWS, VAR_SLAB

LANES = (4, 8, 16, 32, 64)


def spmm_plans(K: int, dtype: torch.dtype = torch.float32) -> list[api.Plan]:
    """Row-split, merge-path and column-slab SpMM plans whose lanes cover at most
    2x the padded K."""
    vec = 2 if dtype == torch.float64 else 4
    cap = max(16, 1 << (max(K, 1) - 1).bit_length())
    plans = []
    for lanes in LANES:
        if lanes * vec > 2 * cap and lanes != 4:
            continue
        plans.append(api.Plan(VAR_ROWS, lanes, 0))
        plans.append(api.Plan(VAR_MERGE, lanes, 0))
        plans.append(api.Plan(VAR_SLAB, lanes, 0))
    return plans


def sddmm_plans(K: int, dtype: torch.dtype = torch.float32) -> list[api.Plan]:
    """SDDMM plans (lanes x entries per group) with at most 8 register slices."""
    vec = 2 if dtype == torch.float64 else 4
    plans = []
    for lanes in LANES:
        if (K + lanes * vec - 1) // (lanes * vec) > 8:
            continue
        if lanes * vec > 2 * max(K, 4) and lanes != 4:
            continue
        for chunk in (64, 256, 1024):
            plans.append(api.Plan(VAR_MERGE, lanes, chunk))
        plans.append(api.Plan(VAR_ROWS, lanes, 0))
        plans.append(api.Plan(VAR_SLAB, lanes, 0))
    return plans


def plans_for(op: int, K: int, dtype: torch.dtype = torch.float32) -> list[api.Plan]:
    """The op's plan list (as the selector sees it) restricted to plans valid for K;
    F64 operands use their own vector width and have no block form."""
    if dtype == torch.float64:
        return spmm_plans(K, dtype) if op == OP_SPMM else sddmm_plans(K, dtype)
    from . import selector

    return [p for p, ok in selector.plan_list(op, K, selector.dtype_code(dtype)) if ok]


def time_plan(A: api.CSR, K: int, op: int, plan: api.Plan | None, B=None, U=None, V=None, reps: int = 5,
              warmup: int = 2) -> float:
    """Median milliseconds of one launch of `plan`."""
    dev = A.row_ptr.device
    if op == OP_SPMM:
        if B is None:
            B = torch.randn(A.n, K, device=dev)
        C = torch.empty((A.m, K), dtype=torch.float32 if B.dtype != torch.float64 else torch.float64, device=dev)
        nb = api.workspace_bytes(OP_SPMM, A, K, plan)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev) if nb else None

        def launch():
            api.spmm(A, B, plan=plan, out=C, workspace=ws)
    else:
        if U is None:
            U = torch.randn(A.m, K, device=dev)
        if V is None:
            V = torch.randn(A.n, K, device=dev)
        S = torch.empty(A.nnz, dtype=torch.float32 if U.dtype != torch.float64 else torch.float64, device=dev)
        nb = api.workspace_bytes(OP_SDDMM, A, K, plan)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev) if nb else None

        def launch():
            api.sddmm(A, U, V, plan=plan, out=S, workspace=ws)
    for _ in range(warmup):
        launch()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        launch()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return ts[len(ts) // 2]


def sweep(A: api.CSR, K: int, op: int, B=None, U=None, V=None, reps: int = 5, warmup: int = 2,
          plans: list[api.Plan] | None = None, log=None) -> list[tuple[api.Plan, float]]:
    """Time every plan; returns [(plan, ms)] in plan-space order.  `log`, if
    given, receives one line per plan as it is timed."""
    dtype = (B if op == OP_SPMM else U).dtype if (B is not None or U is not None) else torch.float32
    plans = plans if plans is not None else plans_for(op, K, dtype)
    out = []
    for p in plans:
        out.append((p, time_plan(A, K, op, p, B=B, U=U, V=V, reps=reps, warmup=warmup)))
        if log is not None:
            log(f"{'spmm' if op == OP_SPMM else 'sddmm'} {p.name()}: {out[-1][1]:.4f} ms")
    return out


def best_plan(A: api.CSR, K: int, op: int, B=None, U=None, V=None, reps: int = 5, log=None) -> tuple[api.Plan, float]:
    res = sweep(A, K, op, B=B, U=U, V=V, reps=reps, log=log)
    return min(res, key=lambda r: r[1])
