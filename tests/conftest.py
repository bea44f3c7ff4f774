import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def golden_rows(name):
    """Non-comment rows of a golden fixture, split on whitespace."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def golden_sheet_rows(name, inputs):
    """Oracle values on sampled rows of a large sheet (tests/golden/make_sheet_rows.py):
    {tag: (rows, values)}.  `inputs` are the workload's inputs as drawn now; their sums must
    equal the ones recorded with the values (the input generator has not changed)."""
    import numpy as np
    out = {}
    for r in golden_rows(name):
        if r[0].startswith("sum_"):
            key = r[0][4:]
            got = float(np.sum(inputs[key]))
            assert got == float(r[1]), f"{name}: inputs changed ({key}: {got!r} != {r[1]})"
        elif r[0] != "workload":
            rows, vals = out.setdefault(r[0], ([], []))
            rows.append(int(r[1]))
            vals.append([float(x) for x in r[2:]])
    return {k: (np.array(v[0]), np.array(v[1])) for k, v in out.items()}
