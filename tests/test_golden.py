"""The paper's worked shapes (tests/golden/paper_shapes.json) with closed-form
expected values, checked against the oracle."""
import json
import os

import numpy as np
import pytest

import oracle

_OPS = {"NONE": 0, "SUM": 1, "MIN": 2, "MAX": 3, "ARGMIN": 4, "ARGMAX": 5}
_DT = {"I32": (0, np.int32), "F32": (1, np.float32)}
_CASES = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_shapes.json")))["cases"]


def fill(case):
    dt = _DT[case["dtype"]][1]
    shape = tuple(case["extents"])
    f = case["fill"]
    if f == "arange":
        return np.arange(int(np.prod(shape)), dtype=dt).reshape(shape)
    if f.startswith("const:"):
        return np.full(shape, float(f[6:]), dtype=dt)
    raise ValueError(f)


def expected(case, n):
    if "expected" in case:
        return np.array(case["expected"], dtype=np.float64)
    i = np.arange(n, dtype=np.float64)
    return eval(case["expected_formula"], {"i": i}) * np.ones(n)


@pytest.mark.parametrize("case", _CASES, ids=[c["name"] for c in _CASES])
def test_golden_oracle(case):
    a = fill(case)
    ops = [_OPS[o] for o in case["ops"]]
    out = oracle.reduce(a, case["extents"], ops, _DT[case["dtype"]][0])
    np.testing.assert_array_equal(out.astype(np.float64), expected(case, out.size))
