import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.set_threads(min(8, max(1, len(os.sched_getaffinity(0)))))
    return oracle


def _hexf(v):
    return float(v) if v in ("inf", "-inf") else float.fromhex(v)


@pytest.fixture(scope="session")
def aux_cases():
    """Plus / Minus / MultiplyWithScalar cases whose results were worked by
    hand from the binary64 rounding rule (tests/golden/aux_worked_values.json):
    (plus, minus, scale) lists of (x, y, result) / (alpha, x, result)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "aux_worked_values.json")) as f:
        doc = json.load(f)
    pm = [[(_hexf(c["x"]), _hexf(c["y"]), _hexf(c["result"])) for c in doc[k]] for k in ("plus", "minus")]
    sc = [(_hexf(c["alpha"]), _hexf(c["x"]), _hexf(c["result"])) for c in doc["multiply_with_scalar"]]
    return pm[0], pm[1], sc
