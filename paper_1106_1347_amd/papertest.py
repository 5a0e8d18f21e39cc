"""The paper's test program (Tests section) on the GPU.

C = A (8A) for an n x n random matrix A, N := NaivKahan as the reference,
and for every method the time of one product and NormInf(N - C).  The paper
states neither the distribution nor the seed; A is uniform on [0, 1) from
numpy's PCG64 with a given seed (B = 8A is exact).  Every product,
difference and norm runs in the library's kernels; the host draws A, times
with HIP events and prints.

    python -m paper_1106_1347_amd.papertest [-O n] [-R repeats] [--seed s] [--json] [--no-extras]

-O (matrix size) and -R (repeats) default to 400 and 10 as in the paper.
The time column is the median over the R repeats of one product, in seconds
(the paper does not say whether its column is per product or per R).
"""
import argparse
import json
import sys

import numpy as np
import torch

from ._lib import Config, minus, multiply, norm_inf, workspace_bytes

# (label as printed by the paper, method, config) in the paper's row order;
# Strassen in the paper's embedding mode with its naive leaf
PAPER_ROWS = [
    ("NaivStandard", "naive", Config()),
    ("NaivOnArray", "naive_on_array", Config()),
    ("NaivLoopUnrollingTwo", "naive_unroll2", Config()),
    ("NaivLoopUnrollingThree", "naive_unroll3", Config()),
    ("NaivLoopUnrollingFour", "naive_unroll4", Config()),
    ("StrassenNaiv", "strassen_naive", Config(pad_mode="paper")),
    ("StrassenWinograd", "strassen_winograd", Config(pad_mode="paper")),
    ("WinogradOriginal", "winograd", Config()),
    ("WinogradScaled", "winograd_scaled", Config()),
]
# methods of this library beyond the paper
EXTRA_ROWS = [
    ("DGEMM (FP64 matrix cores)", "dgemm", Config()),
    ("StrassenWinograd L=2, DGEMM", "strassen_winograd", Config(strassen_levels=2)),
    ("Split int8 x7", "split", Config(split_type="int8", split_slices=7)),
    ("Dot2 (compensated, FMA)", "dot2", Config()),
]
REFERENCE = ("N := NaivKahan", "kahan", Config())


def paper_inputs(n: int, seed: int):
    """A ~ U[0, 1) (n x n, float64), B = 8 A, as host arrays."""
    A = np.random.default_rng(seed).random(size=(n, n))
    return A, 8.0 * A


def _timed(A, B, method, cfg, repeats, stream):
    n = A.shape[0]
    C = torch.empty((n, n), dtype=torch.float64, device=A.device)
    ws = torch.empty(max(workspace_bytes(method, n, n, n, cfg), 1), dtype=torch.uint8, device=A.device)
    multiply(A, B, method, cfg, out=C, workspace=ws, stream=stream)  # warm-up
    times = []
    for _ in range(max(repeats, 1)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        multiply(A, B, method, cfg, out=C, workspace=ws, stream=stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    return C, float(np.median(times)), float(np.sum(times))


def run(n: int = 400, repeats: int = 10, seed: int = 500, extras: bool = True, device: str = "cuda"):
    """Rows of the test table: dicts with label, method, seconds (median per
    product), total_seconds (over the repeats) and err = NormInf(N - C)
    (None for the reference row)."""
    Ah, Bh = paper_inputs(n, seed)
    A = torch.from_numpy(Ah).to(device)
    B = torch.from_numpy(Bh).to(device)
    stream = torch.cuda.current_stream(A.device)
    label, method, cfg = REFERENCE
    Nref, t, tt = _timed(A, B, method, cfg, repeats, stream)
    rows = [{"label": label, "method": method, "seconds": t, "total_seconds": tt, "err": None}]
    D = torch.empty_like(Nref)
    todo = [(r, False) for r in PAPER_ROWS] + ([(r, True) for r in EXTRA_ROWS] if extras else [])
    for (label, method, cfg), beyond in todo:
        C, t, tt = _timed(A, B, method, cfg, repeats, stream)
        minus(Nref, C, out=D, stream=stream)
        err = norm_inf(D, stream=stream)
        stream.synchronize()
        rows.append({"label": label, "method": method, "seconds": t, "total_seconds": tt,
                     "err": float(err.item()), "beyond_paper": beyond})
    return {"n": n, "repeats": repeats, "seed": seed, "rows": rows}


def format_table(res) -> str:
    """The table in the layout the paper prints (one box per run)."""
    w = 71
    bar = "+" + "-" * w + "+"
    out = [bar, "|" + "TIME TEST FOR METHODS OF MATRIX MULTIPLICATION".center(w) + "|", "|" + " " * w + "|",
           "|" + (" C = A*(8A), where A is a (n x n) random matrix with n = %10d" % res["n"]).ljust(w) + "|", bar,
           "| %-27s | %16s | %20s |" % ("method", "time (sec)", "NormInf( N-C )"), bar]
    for r in res["rows"]:
        err = "" if r["err"] is None else "%.10f" % r["err"]
        out.append("| %-27s | %16.6f | %20s |" % (r["label"][:27], r["seconds"], err))
    out.append(bar)
    return "\n".join(out)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("-O", dest="n", type=int, default=400, help="matrix size (default 400)")
    ap.add_argument("-R", dest="repeats", type=int, default=10, help="number of repeats (default 10)")
    ap.add_argument("--seed", type=int, default=500)
    ap.add_argument("--json", action="store_true", help="print the rows as one JSON line instead of the table")
    ap.add_argument("--no-extras", action="store_true", help="only the paper's methods")
    a = ap.parse_args(argv)
    if a.n < 1 or a.repeats < 1:
        ap.error("-O and -R must be positive")
    if not torch.cuda.is_available():
        print("papertest: no GPU visible", file=sys.stderr)
        return 2
    res = run(a.n, a.repeats, a.seed, extras=not a.no_extras)
    print(json.dumps(res) if a.json else format_table(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
