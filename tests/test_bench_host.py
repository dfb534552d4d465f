"""Host-side pieces of bench.py (no GPU): byte and flop accounting, the
roofline choice, the multi-GPU refusal and the traffic lookup in profiles/
(a reading counts only at the kernel sources it was taken from)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes():
    m = n = 1000
    nnz, K = 50_000, 64
    # row_ptr, (col, val) per entry, B read once, C written once
    assert bench.spmm_bytes(m, n, nnz, K) == 4 * (m + 1) + nnz * 8 + n * K * 4 + m * K * 4
    # A^T G reads a 4-byte perm entry per value as well
    assert bench.spmm_bytes(m, n, nnz, K, perm=True) == bench.spmm_bytes(m, n, nnz, K) + 4 * nnz
    # BF16 dense operand
    assert bench.spmm_bytes(m, n, nnz, K, sb=2) == 4 * (m + 1) + nnz * 8 + n * K * 2 + m * K * 4
    # SDDMM: row_ptr, (col, val, out) per entry, U and V once; pattern mode drops the value
    assert bench.sddmm_bytes(m, n, nnz, K) == 4 * (m + 1) + nnz * 12 + m * K * 4 + n * K * 4
    assert bench.sddmm_bytes(m, n, nnz, K, sv=0) == bench.sddmm_bytes(m, n, nnz, K) - 4 * nnz


def test_touched_bytes_counts_referenced_rows_only():
    """Hyper-sparse accounting: 5 x 8 pattern with two empty rows, columns
    {1, 3, 6} referenced (column 3 twice)."""
    import numpy as np
    from types import SimpleNamespace

    A = SimpleNamespace(m=5, n=8, nnz=4, row_ptr=np.array([0, 2, 2, 3, 3, 4], np.int32),
                        col_idx=np.array([1, 3, 3, 6], np.int32))
    K = 16
    t = bench.touched_bytes(A, K)
    # SpMM: row_ptr, (col, val) per entry, 3 referenced rows of B, all 5 rows of C
    assert t["spmm"] == 4 * 6 + 4 * 8 + 3 * K * 4 + 5 * K * 4
    # SDDMM: row_ptr, (col, val, out) per entry, 3 non-empty rows of U, 3 referenced rows of V
    assert t["sddmm"] == 4 * 6 + 4 * 12 + 3 * K * 4 + 3 * K * 4
    # never more than the byte model, which counts every dense row
    assert t["spmm"] <= bench.spmm_bytes(5, 8, 4, K) and t["sddmm"] <= bench.sddmm_bytes(5, 8, 4, K)


def test_roofline_picks_the_binding_roof():
    # 8e9 bytes, tiny flops: HBM binds; 1 s at 8 GB/s of 8 TB/s is 0.1%
    r = bench.roofline(8e9, 1.0, 1.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["frac"] == pytest.approx(0.001)
    # 78.6e12 flops in 2 s with few bytes: the FP32 ALU binds at half its rate
    r = bench.roofline(1.0, 78.6e12, 2.0)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["frac"] == pytest.approx(0.5)


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode != 0 and "one GPU" in (out.stdout + out.stderr)


def test_recorded_traffic_needs_matching_digest(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    (tmp_path / "p.md").write_text(
        f"traffic w1 sddmm tile/l16/c64/f6 123456 {digest}\n"
        "traffic w1 spmm tile/l16/c64 777 0000000000000000\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.recorded_traffic("w1", "sddmm", "tile/l16/c64/f6") == 123456
    assert bench.recorded_traffic("w1", "sddmm", "tile/l16/c64") is None  # another plan
    assert bench.recorded_traffic("w1", "spmm", "tile/l16/c64") is None   # taken from other sources

