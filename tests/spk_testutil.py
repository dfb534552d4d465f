"""Helpers shared by the test modules (host side only)."""
from __future__ import annotations

import numpy as np

from paper_2604_27985_amd import synth

# Elementwise gate for FP32 results: |gpu - exact| <= TOL * (|A| |B|) with the
# exact value and the bound from the FP64 oracle.
TOL_F32 = 1e-5
# BF16 operands rounded from FP32 sources, compared with the unrounded exact
# product: one bf16 rounding (2^-8 relative) per dense factor.
TOL_BF16_SRC = 1e-2
# F64 kernels against the F64 oracle.
TOL_F64 = 1e-12


def assert_within(gpu, exact, bound, tol, what=""):
    gpu = np.asarray(gpu, dtype=np.float64)
    err = np.abs(gpu - exact)
    lim = tol * bound
    bad = err > lim
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {bad.size} outside {tol} x bound; first {idx.tolist()}: "
            f"gpu={gpu[bad][:5]}, exact={exact[bad][:5]}, bound={bound[bad][:5]}")


def sub_rows(A, rows):
    """Host CSR of the selected rows (keeps column numbering)."""
    rp = A.row_ptr.astype(np.int64)
    lens = rp[rows + 1] - rp[rows]
    new_rp = np.zeros(len(rows) + 1, np.int64)
    np.cumsum(lens, out=new_rp[1:])
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows]) if len(rows) else np.zeros(0, np.int64)
    return new_rp.astype(np.int32), A.col_idx[idx], idx


def host_csr(m, n, row_lists):
    """HostCSR from explicit per-row column lists."""
    rp = np.zeros(m + 1, np.int32)
    cols = []
    for i, r in enumerate(row_lists):
        rp[i + 1] = rp[i] + len(r)
        cols.extend(r)
    return synth.HostCSR(m, n, rp, np.asarray(cols, np.int32), "explicit")
