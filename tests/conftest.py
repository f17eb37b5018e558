"""Shared test set-up: import paths, the `gpu` marker and the oracle build."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle._load()
    if os.environ.get("PYTEST_XDIST_WORKER"):
        # parallel test workers share the cores: one oracle thread each, or the OpenMP
        # teams of several workers spin against each other
        oracle.set_num_threads(1)
    return oracle


def read_golden(name="paper_values.txt"):
    """key -> list of string tokens, from a golden file (comments after '#')."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = line.split("=", 1)
            out[k.strip()] = v.split()
    return out
