"""Host-side logic of the plan selector (CPU only; the C ABI's host-only calls)."""
import json
import math
import os

import numpy as np
import pytest

from paper_2604_27985_amd import _lib

if not os.path.exists(_lib.LIB_PATH):
    pytest.skip("libspk.so not built", allow_module_level=True)

from paper_2604_27985_amd import selector  # noqa: E402


def test_plan_lists():
    assert selector.plan_count(_lib.OP_SPMM) == 30 and selector.plan_count(_lib.OP_SDDMM) == 29
    pl = selector.plan_list(_lib.OP_SPMM, 64)
    assert [p.variant for p, _ in pl[:15]] == [0] * 5 + [1] * 5 + [3] * 5 and pl[15][0].variant == 2
    # LDS slabs of 16 / 32 KiB of F32 rows (K = 64: 256-byte rows), 4 or 8 rows per group, then one
    # entry per quad (flags bit 2) with 16 and 32 KiB slabs
    assert [(p.variant, p.lanes, p.chunk, p.flags) for p, _ in pl[16:24]] == [
        (4, 16, 64, 0), (4, 16, 128, 0), (4, 16, 64, 2), (4, 16, 128, 2), (4, 16, 64, 4), (4, 16, 64, 6),
        (4, 16, 128, 4), (4, 16, 128, 6)]
    # wide quad plans (32 and 64 KiB slabs), the column-slab form (4 and 8 MiB
    # of B per slab), doubly compressed rows (plain lanes, then 4)
    assert [(p.variant, p.lanes, p.chunk, p.flags) for p, _ in pl[24:]] == [
        (4, 16, 128, 12), (4, 16, 256, 12), (5, 16, 16384, 0), (5, 16, 32768, 0), (6, 16, 0, 0), (6, 4, 0, 0)]
    # SDDMM column-slab plans: 2 and 8 MiB, groups of 8 lanes widened until a
    # lane holds at most 8 columns (K = 128: 16 lanes)
    sd = selector.plan_list(_lib.OP_SDDMM, 128)
    assert [(p.variant, p.lanes, p.chunk) for p, _ in sd[25:27]] == [(5, 16, 4096), (5, 16, 16384)]
    # SpMM at K = 128: plain lanes for 4 MiB slabs, 16 lanes for 8 MiB
    sp = selector.plan_list(_lib.OP_SPMM, 128)
    assert [(p.variant, p.lanes, p.chunk) for p, _ in sp[26:28]] == [(5, 32, 8192), (5, 16, 16384)]
    assert all(ok for _, ok in pl[16:])
    for K, ok in ((8, True), (36, False), (256, True), (512, False)):
        assert all(v == ok for _, v in selector.plan_list(_lib.OP_SPMM, K)[16:25]), K
    # 64 KiB wide slabs only where the quad split takes the rows (F32 K 32, 64, 128; BF16 K 64, 128)
    for K, ok32, okbf in ((32, True, False), (64, True, True), (128, True, True), (256, False, False), (8, False, False)):
        assert selector.plan_list(_lib.OP_SPMM, K)[25][1] == ok32, K
        assert selector.plan_list(_lib.OP_SPMM, K, _lib.BF16)[25][1] == okbf, K
    assert selector.plan_list(_lib.OP_SDDMM, 256, _lib.BF16)[24][1]  # SDDMM quad takes 512-byte BF16 rows
    # F64 operands: the first 15 plans only
    assert [ok for _, ok in selector.plan_list(_lib.OP_SPMM, 64, _lib.F64)][15:] == [False] * 15
    assert [p.chunk for p, _ in selector.plan_list(_lib.OP_SPMM, 256)[16:18]] == [16, 32]
    assert [p.lanes for p, _ in pl[:5]] == [4, 8, 16, 32, 64]
    # K = 64: lanes x 4 up to 2 x 64
    assert [ok for _, ok in pl[:5]] == [True, True, True, True, False]
    assert all(ok for _, ok in selector.plan_list(_lib.OP_SPMM, 256)[:5])
    sd = selector.plan_list(_lib.OP_SDDMM, 256)
    # 4 lanes x 4 wide x 8 slices = 128 < 256
    assert not sd[0][1] and sd[1][1]
    assert all(p.chunk == 256 for p, _ in sd[5:10])
    # SDDMM TILE plans: at least 16 lanes (reductions over 16-lane rows)
    assert [(p.variant, p.lanes, p.chunk, p.flags) for p, _ in selector.plan_list(_lib.OP_SDDMM, 32)[15:23]] == [
        (4, 16, 128, 0), (4, 16, 256, 0), (4, 16, 128, 2), (4, 16, 256, 2), (4, 16, 128, 4), (4, 16, 128, 6),
        (4, 16, 256, 4), (4, 16, 256, 6)]
    assert [p.lanes for p, _ in sd[15:25]] == [64] * 10 and all(ok for _, ok in sd[15:24])
    assert not sd[24][1]  # F32 rows of 1 KiB: no quad split, no 64 KiB slabs
    assert [(p.variant, p.lanes, p.chunk, p.flags) for p, _ in selector.plan_list(_lib.OP_SDDMM, 64)[25:]] == [
        (5, 8, 8192, 0), (5, 8, 32768, 0), (6, 8, 0, 0), (7, 16, 16, 0)]


def test_plain_index_matches_null_plan_rule():
    for K in (1, 16, 32, 64, 100, 128, 256, 1024):
        i = selector.plain_index(_lib.OP_SPMM, K)
        lanes = 4 << (i % 5)
        assert i < 5 and (lanes == 64 or lanes * 4 >= K) and (lanes == 4 or (lanes // 2) * 4 < K)
        j = selector.plain_index(_lib.OP_SDDMM, K)
        assert 5 <= j < 10
        lanes = 4 << (j % 5)
        assert lanes >= 8 and (lanes == 64 or -(-K // (lanes * 4)) <= 8)


def test_specs_are_seeded_and_capped():
    a = [selector.sample_spec(i) for i in range(300)]
    b = [selector.sample_spec(i) for i in range(300)]
    assert a == b
    for s in a:
        assert 4096 <= s["n"] <= 524288 and s["n"] % 64 == 0
        assert 1e-4 <= s["density"] <= 0.1
        assert selector.expected_nnz(s["n"], s["density"], s["pattern"]) <= selector.NNZ_CAP
        assert s["split"] == ("test" if s["index"] % 5 == 0 else "train")
    assert {s["pattern"] for s in a} == set(selector.PATTERNS)
    assert {s["K"] for s in a} == set(selector.KS)


def test_make_matrix_families():
    for i in range(12):
        s = dict(selector.sample_spec(i), n=2048)
        A, v = selector.make_matrix(s)
        assert A.m == A.n == 2048 and v.shape == (A.nnz,)
        L = A.row_lengths()
        if s["pattern"] == "banded":
            rows = np.repeat(np.arange(A.m), L)
            assert np.all(np.abs(rows - A.col_idx) <= 64)
        if s["pattern"] == "block4":
            assert np.all(L.reshape(-1, 4) == L.reshape(-1, 4)[:, :1])


def test_regret_stats_and_choice():
    times = np.array([[1.0, 2.0, np.nan], [3.0, 1.5, 1.0], [2.0, 2.0, 4.0]])
    valid = np.isfinite(times).astype(np.float32)
    Y = np.array([[0.5, 0.1, -9.0], [0.0, 1.0, 2.0], [1.0, 0.0, 3.0]])
    pick = selector.choose(Y, valid)
    assert pick.tolist() == [1, 0, 1]  # the invalid plan never wins
    st = selector.regret_stats(times, pick, np.array([0, 0, 0]))
    r = np.array([2.0, 3.0, 1.0])
    assert math.isclose(st["geomean_regret"], float(np.exp(np.log(r).mean())))
    assert st["max_regret"] == 3.0 and st["median_regret"] == 2.0
    # plain = plan 0: times (1, 3, 2) against picks (2, 3, 2)
    assert math.isclose(st["geomean_gain_over_plain"], float(np.exp(np.log(np.array([0.5, 1.0, 1.0])).mean())))


def test_extended_timings_merge(tmp_path):
    """Times of plans added later are folded in at their plan indices."""
    base = tmp_path / "t.jsonl"
    ext = tmp_path / "e.jsonl"
    out = tmp_path / "m.jsonl"
    recs = [{"index": 0, "ms_spmm": [1.0] * 16, "ms_sddmm": [2.0] * 15},
            {"index": 1, "ms_spmm": [3.0] * 16, "ms_sddmm": [4.0] * 15}]
    base.write_text("".join(json.dumps(r) + "\n" for r in recs))
    ext.write_text(json.dumps({"index": 1, "op": "spmm", "plans": [16, 17, 18, 19], "ms": [0.5, None, 0.7, 0.8]}) + "\n")
    assert selector.merge_timings(str(base), str(ext), str(out)) == 1
    m = selector.load_timings(str(out))
    assert m[0]["ms_spmm"] == [1.0] * 16 + [None] * 14
    assert m[1]["ms_spmm"] == [3.0] * 16 + [0.5, None, 0.7, 0.8] + [None] * 10
    assert m[1]["ms_sddmm"] == [4.0] * 15 + [None] * 14  # widened to the SDDMM plan count


def test_plan_names_round_trip():
    """Plan.name() and Plan.from_name() are inverse (bench --plans reads the names bench lines print)."""
    from paper_2604_27985_amd.api import Plan

    for op in (_lib.OP_SPMM, _lib.OP_SDDMM):
        for K in (8, 32, 64, 128, 256):
            for p, _ in selector.plan_list(op, K):
                q = Plan.from_name(p.name())
                assert (q.variant, q.lanes, q.chunk, q.flags) == (p.variant, p.lanes, p.chunk, p.flags)


def test_merged_network_is_the_members_mean():
    """merge_tables stacks three networks into one of 3H hidden units whose
    output is the mean of theirs: checked with the oracle's FP64 forward on
    random inputs (the merged parameters are stored in binary32, so W3 / 3
    carries one rounding)."""
    import oracle

    F, H, P = 33, 64, 30
    rng = np.random.default_rng(7)
    tables = []
    for seed in range(3):
        params = np.concatenate([rng.normal(0, 0.3, H * F), rng.normal(0, 0.1, H), rng.normal(0, 0.2, H * H),
                                 rng.normal(0, 0.1, H), rng.normal(0, 0.2, P * H), rng.normal(0, 0.1, P)])
        tables.append({"op": 1, "F": F, "H": H, "P": P, "mean": [0.0] * F, "scale": [1.0] * F,
                       "params": params.astype(np.float32).tolist(), "seed": seed})
    merged = selector.merge_tables(tables)
    assert merged["H"] == 3 * H and merged["seed"] == [0, 1, 2]
    assert len(merged["params"]) == 3 * H * F + 3 * H + 9 * H * H + 3 * H + P * 3 * H + P
    X = rng.normal(0, 1, (50, F))
    ys = [oracle.MLP(*selector.split_params(t)).forward(X) for t in tables]
    y = oracle.MLP(*selector.split_params(merged)).forward(X)
    want = np.mean(ys, 0)
    assert np.max(np.abs(y - want)) <= 1e-6 * (1 + np.max(np.abs(want)))
    # a member whose standardisation differs cannot be merged
    other = dict(tables[0], mean=[1.0] * F)
    with pytest.raises(ValueError):
        selector.merge_tables([tables[0], other])
