"""spk_csr_validate on the GPU against the oracle's canonical-CSR check.

Canonical CSR is the reading of the paper's CSR input (Section III-A: 32-bit
column indices) taken by the library: row_ptr from 0, rows inside [0, nnz]
and not decreasing, row_ptr[m] = nnz, columns in [0, n) and strictly
increasing within a row.  Both sides return the OR of the rules broken; they
must agree bit for bit on every hand-worked case, on the generators' output
and on single mutations of it.
"""
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


def dev_csr(spk, m, n, rp, ci):
    rp_t = torch.from_numpy(np.asarray(rp, np.int32)).cuda()
    ci_t = torch.from_numpy(np.asarray(ci, np.int32)).cuda()
    return spk.CSR(rp_t, ci_t, None, (m, n))


def test_validate_hand_cases(spk):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "csr_canonical.json")))
    for c in g["cases"]:
        assert len(c["col_idx"]) == c["nnz"]
        want = oracle.csr_canonical(np.array(c["row_ptr"]), np.array(c["col_idx"], np.int32), c["m"], c["n"], c["nnz"])
        assert want == c["bits"]
        got = spk.validate_rules(dev_csr(spk, c["m"], c["n"], c["row_ptr"], c["col_idx"]))
        assert got == want, (c["name"], got, want)
        assert spk.validate(dev_csr(spk, c["m"], c["n"], c["row_ptr"], c["col_idx"])) == (want == 0)


@pytest.mark.parametrize("seed", [0, 1])
def test_validate_generators_and_mutations(spk, seed):
    rng = np.random.default_rng(seed)
    for A in (synth.bernoulli(3000, 2000, 0.02, seed), synth.powerlaw(20000, 16, 2.1, seed),
              synth.block4(1024, 2048, 0.02, seed), synth.bernoulli(5000, 5000, 0.01, seed, band=64),
              synth.HostCSR(7, 5, np.zeros(8, np.int32), np.zeros(0, np.int32))):
        assert spk.validate_rules(dev_csr(spk, A.m, A.n, A.row_ptr, A.col_idx)) == 0
        if A.nnz == 0:
            continue
        lens = np.diff(A.row_ptr)
        rows = np.flatnonzero(lens >= 2)
        for kind in ("swap", "dup", "range", "neg", "start", "end", "order"):
            rp, ci = A.row_ptr.copy(), A.col_idx.copy()
            i = int(rng.choice(rows))
            p = int(rp[i] + rng.integers(0, lens[i] - 1))
            if kind == "swap":
                ci[p], ci[p + 1] = ci[p + 1], ci[p]
            elif kind == "dup":
                ci[p + 1] = ci[p]
            elif kind == "range":
                ci[rp[i + 1] - 1] = A.n
            elif kind == "neg":
                ci[rp[i]] = -1
            elif kind == "start":
                rp[0] = 1
            elif kind == "end":
                rp[A.m] = A.nnz - 1
            else:  # a row range that runs backwards
                rp[i + 1] = rp[i] - 1 if rp[i] > 0 else A.nnz + 1
            want = oracle.csr_canonical(rp, ci, A.m, A.n, A.nnz)
            assert want != 0, kind
            got = spk.validate_rules(dev_csr(spk, A.m, A.n, rp, ci))
            assert got == want, (kind, got, want)
