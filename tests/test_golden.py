"""The oracle still reproduces the frozen fixtures in tests/golden (written by
tests/golden/make_golden.py from the oracle alone)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def _load(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def test_toy_paths_fixture():
    ref = _load("toy_paths.json")
    got = make_golden.toy_paths()
    assert got["candidates"] == ref["candidates"]
    for a, b in zip(got["rx"], ref["rx"]):
        assert [p["faces"] for p in a] == [p["faces"] for p in b]
        for p, q in zip(a, b):
            assert np.allclose(p["a"], q["a"], rtol=1e-12, atol=1e-20)
            assert abs(p["tau"] - q["tau"]) <= 1e-15 * q["tau"]


def test_toy_coverage_fixture():
    ref = _load("toy_coverage.json")
    got = make_golden.toy_coverage()
    assert got["total_hits"] == ref["total_hits"] and got["cells_with_hits"] == ref["cells_with_hits"]
    for c, d in zip(got["cells"], ref["cells"]):
        assert c[:2] == d[:2] and c[3] == d[3]
        assert abs(c[2] - d[2]) <= 1e-12 * max(abs(d[2]), 1e-300)
