"""Shared test setup: repository root on sys.path, the gpu marker, built libraries."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running case")


def _ensure_host_libs():
    # Tests load what is built and build only when nothing is.
    from paper_2604_27985_amd import synth
    import oracle

    if not os.path.exists(synth.LIB_PATH):
        synth.build()
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()


_ensure_host_libs()


@pytest.fixture(scope="session")
def golden():
    import json

    with open(os.path.join(ROOT, "tests", "golden", "hand_examples.json")) as f:
        return json.load(f)
