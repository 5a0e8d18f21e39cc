"""The paper's test program (Tests section) on the GPU, against the oracle.

C = A (8A), N := NaivKahan: every entry of the error column of the paper's
methods must equal the oracle's NormInf(N - C) on the same inputs bit for
bit (every product, the difference and the row sums are rounded in the
paper's order on both sides); the methods beyond the paper stay at the
magnitude of the paper's rows.
"""
import io
import json
from contextlib import redirect_stdout

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1106_1347_amd import papertest

    return papertest


def _oracle_rows(orc):
    return {
        "NaivStandard": orc.naive,
        "NaivOnArray": orc.naive_on_array,
        "NaivLoopUnrollingTwo": lambda A, B: orc.naive_unroll(A, B, 2),
        "NaivLoopUnrollingThree": lambda A, B: orc.naive_unroll(A, B, 3),
        "NaivLoopUnrollingFour": lambda A, B: orc.naive_unroll(A, B, 4),
        "StrassenNaiv": lambda A, B: orc.strassen(A, B, 0, orc.MODE_PAPER),
        "StrassenWinograd": lambda A, B: orc.strassen(A, B, 1, orc.MODE_PAPER),
        "WinogradOriginal": orc.winograd,
        "WinogradScaled": orc.winograd_scaled,
    }


@pytest.mark.parametrize("n", [200, 67, 33])
def test_error_column_equals_oracle(pt, orc, n):
    print("case n =", n, flush=True)
    res = pt.run(n=n, repeats=1, seed=500)
    A, B = synth.paper_test_pair(n, 500)
    Nk = orc.kahan(A, B)
    ref = _oracle_rows(orc)
    labels = [r["label"] for r in res["rows"]]
    assert labels[0].startswith("N := NaivKahan") and labels[1:10] == list(ref)
    for r in res["rows"][1:]:
        if r["label"] in ref:
            want = orc.norm_inf(orc.minus(Nk, ref[r["label"]](A, B)))
            assert r["err"] == want, (n, r["label"], r["err"], want)
        else:
            assert r["beyond_paper"] and 0.0 <= r["err"] <= 1e-9, r
        assert r["seconds"] > 0.0


def test_cli_json_and_table(pt):
    buf = io.StringIO()
    with redirect_stdout(buf):
        assert pt.main(["-O", "48", "-R", "2", "--json", "--no-extras"]) == 0
    res = json.loads(buf.getvalue())
    assert res["n"] == 48 and res["repeats"] == 2 and len(res["rows"]) == 10
    buf = io.StringIO()
    with redirect_stdout(buf):
        assert pt.main(["-O", "40", "-R", "1"]) == 0
    text = buf.getvalue()
    assert "TIME TEST FOR METHODS OF MATRIX MULTIPLICATION" in text and "NaivLoopUnrollingThree" in text
    assert np.isfinite([float(l.split("|")[3]) for l in text.splitlines() if "NaivStandard" in l][0])
