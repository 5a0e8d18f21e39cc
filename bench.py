"""Benchmark of the hot path: C = AB by every method of the library on the
N = M = 4096, P in {4096, 4097} FP64 workload (entries uniform on [-1, 1]).

One step = one pass of every method over both shapes (P = 4096 and the odd
P = 4097).  Prints ONE JSON line with the whole-step FP64-grade throughput
(sum of 2NPM over the step's products divided by the step's time), the
per-method median and p99 latency, TFLOP/s and relative infinity-norm error
on sampled rows, the roofline of the dominant kernel measured live with HIP
events on the stream the kernels run on, and the CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64-grade TFLOP/s vs plain FP64 MFMA GEMM at fixed ∞-norm err; p99 latency"
FP64_GRADE = 1e-13

# MI355X published peaks and chip constants.
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 16, 2.4
# non-fused FP64 vector operations per second (each op one flop): one wave64
# instruction per SIMD every 4 clocks
PEAK_FP64_VALU_OPS_T = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_GHZ * 1e9 / 1e12  # 39.3

# (name, method, config kwargs, algorithmic cost per multiply-add, bound, unit of the cost)
#   naive:   1 mul + 1 add (rounded separately)           -> 2 VALU ops / MAC
#   kahan:   1 mul + 4 add/sub                             -> 5 VALU ops / MAC
#   winograd: 2 add + 1 mul + 1 add per pair of MACs       -> 2 VALU ops / MAC
#   dgemm:   2 flop / MAC on FP64 matrix cores
#   split:   s(s+1)/2 digit-pair products x 2 ops / MAC on the bf16 / int8 matrix cores
PEAK_BF16_MFMA_TFLOPS = 2516.6
PEAK_INT8_MFMA_TOPS = 5033.2
METHODS = [
    ("dgemm", "dgemm", {}, 2.0, "mfma"),
    ("naive", "naive", {}, 2.0, "alu"),
    ("kahan", "kahan", {}, 5.0, "alu"),
    ("winograd", "winograd", {}, 2.0, "alu"),
    ("winograd_scaled", "winograd_scaled", {}, 2.0, "alu"),
    ("strassen_winograd_L2", "strassen_winograd", {"strassen_levels": 2}, None, None),
    ("strassen_naive_L2", "strassen_naive", {"strassen_levels": 2}, None, None),
    ("split_int8_s7", "split", {"split_type": "int8", "split_slices": 7}, None, None),
    ("split_bf16_s6", "split", {"split_type": "bf16", "split_slices": 6}, None, None),
]
# the precision comparison at 8192^3 on the wide-range distribution
PRECISION = [
    ("dgemm", "dgemm", {}),
    ("split_int8_s7", "split", {"split_type": "int8", "split_slices": 7}),
    ("split_bf16_s6", "split", {"split_type": "bf16", "split_slices": 6}),
]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="", help="comma-separated subset of methods (for profiling)")
    ap.add_argument("--no-precision", action="store_true", help="skip the 8192^3 split-vs-DGEMM comparison")
    ap.add_argument("--precision-reps", type=int, default=5)
    ap.add_argument("--precision-only", action="store_true", help="run only the 8192^3 comparison (profiling)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the products of the workload "
              "are independent per GPU; see the design notes on sharding). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1106_1347_amd as mmm
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.precision_only:
        stream = torch.cuda.current_stream()
        print(json.dumps({"precision_8192": precision_section(args, mmm, torch, synth, dev, stream,
                                                              errors_needed=not args.no_cpu_baseline)}), flush=True)
        return
    n = args.size
    shapes = [(n, n, n), (n, n + 1, n)]
    methods = [m for m in METHODS if not args.only or m[0] in args.only.split(",")]

    data = {}
    for (N, P, M) in shapes:
        A = synth.uniform((N, P), synth.seed_a(1))
        B = synth.uniform((P, M), synth.seed_b(1))
        Ad = torch.from_numpy(A).to(dev)
        Bd = torch.from_numpy(B).to(dev)
        C = torch.empty((N, M), dtype=torch.float64, device=dev)
        data[P] = (A, B, Ad, Bd, C)
    ws = {}
    for name, method, kw, _, _ in methods:
        cfg = mmm.Config(**kw)
        for (N, P, M) in shapes:
            need = mmm.workspace_bytes(method, N, P, M, cfg)
            ws[(name, P)] = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def one_step(timings):
        for name, method, kw, _, _ in methods:
            cfg = mmm.Config(**kw)
            for (N, P, M) in shapes:
                _, _, Ad, Bd, C = data[P]
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws[(name, P)], stream=stream)
                e1.record(stream)
                if timings is not None:
                    timings.append((name, P, e0, e1))

    for _ in range(args.warmup):
        one_step(None)
    torch.cuda.synchronize()

    timings = []
    step_events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        one_step(timings)
        s1.record(stream)
        step_events.append((s0, s1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    step_ms = [a.elapsed_time(b) for a, b in step_events]
    per = {}
    for name, P, e0, e1 in timings:
        per.setdefault((name, P), []).append(e0.elapsed_time(e1))
    flop_step = sum(2.0 * N * P * M for (N, P, M) in shapes) * len(methods)
    total_s = sum(step_ms) / 1e3
    value = flop_step * args.steps / total_s / 1e12

    # errors on sampled rows, against the oracle (also the CPU baseline sample)
    errors = {}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        # the host cores this process may use (the GPU machine grants 16 per GPU)
        threads = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16")))
        oracle.set_threads(threads)
        rows = np.linspace(0, n - 1, 8 * threads).round().astype(np.int64)
        ref = {}
        cpu_t = 0.0
        cpu_flop = 0.0
        for (N, P, M) in shapes:
            A, B, _, _, _ = data[P]
            t = time.perf_counter()
            ref[P] = oracle.naive_rows(A, B, rows)
            cpu_t += time.perf_counter() - t
            cpu_flop += 2.0 * len(rows) * P * M
        cpu = {"value": cpu_flop / cpu_t / 1e12, "unit": "TFLOP/s", "cores": oracle.get_threads(), "kind": "oracle",
               "sample": "%d of %d rows of C at P=4096 and P=4097 by the naive definition (FP64, k ascending, "
                         "threads split rows), %.1f s wall" % (len(rows), n, cpu_t),
               "cpu_model": platform.processor() or _cpu_model()}
        nrm = {P: (oracle.norm_inf(data[P][0]), oracle.norm_inf(data[P][1])) for (_, P, _) in shapes}
        ridx = torch.from_numpy(rows).to(dev)
        for name, method, kw, _, _ in methods:
            cfg = mmm.Config(**kw)
            worst = 0.0
            for (N, P, M) in shapes:
                _, _, Ad, Bd, C = data[P]
                mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws[(name, P)], stream=stream)
                got = C[ridx].cpu().numpy()
                e = oracle.norm_inf(oracle.minus(got, ref[P])) / (nrm[P][0] * nrm[P][1])
                worst = max(worst, e)
            errors[name] = worst

    precision = None
    if not args.no_precision:
        precision = precision_section(args, mmm, torch, synth, dev, stream, errors_needed=not args.no_cpu_baseline)

    results = {}
    for name, method, kw, cost, bound in methods:
        ms = []
        for (N, P, M) in shapes:
            ms += per[(name, P)]
        ms = np.array(ms)
        fl = np.mean([2.0 * N * P * M for (N, P, M) in shapes])
        med = float(np.median(ms))
        results[name] = {"ms_p50": med, "ms_p99": float(np.percentile(ms, 99)), "ms_mean": float(ms.mean()),
                         "tflops_p50": fl / (med / 1e3) / 1e12,
                         "rel_err_inf_sampled": errors.get(name)}

    # dominant single-kernel method: the largest share of the step
    single = [m for m in methods if m[3] is not None]
    dom = max(single, key=lambda m: results[m[0]]["ms_mean"])
    dname, _, _, dcost, dbound = dom
    dms = results[dname]["ms_mean"]
    macs = np.mean([N * P * M for (N, P, M) in shapes])
    if dbound == "mfma":
        achieved = dcost * macs / (dms / 1e3) / 1e12
        peak = PEAK_FP64_MFMA_TFLOPS
    else:
        achieved = dcost * macs / (dms / 1e3) / 1e12
        peak = PEAK_FP64_VALU_OPS_T
    roofline = {"bound": dbound, "kernel": dname, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "note": "achieved = %g algorithmic FP64 ops per multiply-add x N*P*M / mean launch time; "
                        "alu peak = 256 CU x 4 SIMD x 16 lanes x 2.4 GHz non-fused FP64 ops" % dcost}

    fp64_grade = all((e is None or e <= FP64_GRADE) for e in errors.values()) if errors else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "C = AB, N = M = %d, P in {%d, %d}, entries U[-1,1] (seeds 1001/1002), one product "
                               "per method per shape per step" % (n, n, n + 1),
                   "methods": [m[0] for m in methods], "global_batch": len(shapes) * len(methods),
                   "parallelism": "single GPU"},
        "fp64_grade_all": fp64_grade,
        "step_ms_p50": float(np.median(step_ms)),
        "step_ms_p99": float(np.percentile(step_ms, 99)),
        "wall_s": wall,
        "methods": results,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "precision_8192": precision,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)


def precision_section(args, mmm, torch, synth, dev, stream, errors_needed):
    """DGEMM against the split products at N = P = M = 8192 on the
    wide-range distribution: median time, FP64-grade TFLOP/s (2NPM/t) and
    relative infinity-norm error on sampled rows against the oracle."""
    n = 8192
    A = synth.wide_range((n, n), synth.seed_a(2))
    B = synth.wide_range((n, n), synth.seed_b(2))
    Ad = torch.from_numpy(A).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    out = {"workload": "N = P = M = 8192, entries +-2^u (u ~ U[-20,20]), rows scaled by 2^v (v ~ U{-10..10}), "
                       "seeds 2001/2002", "reps": args.precision_reps}
    rows = np.array([0, 1, 2048, 4095, 6000, 8191])
    ref = None
    if errors_needed:
        import oracle

        ref = oracle.naive_rows(A, B, rows)
        nrm = oracle.norm_inf(A) * oracle.norm_inf(B)
    ridx = torch.from_numpy(rows).to(dev)
    for name, method, kw in PRECISION:
        cfg = mmm.Config(**kw)
        ws = torch.empty(max(mmm.workspace_bytes(method, n, n, n, cfg), 1), dtype=torch.uint8, device=dev)
        mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.precision_reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = float(np.median(ms))
        ent = {"ms_p50": med, "ms_min": float(np.min(ms)), "tflops_fp64_grade": 2.0 * n ** 3 / (med / 1e3) / 1e12}
        if name == "dgemm":
            ent["frac_fp64_mfma_peak"] = ent["tflops_fp64_grade"] / PEAK_FP64_MFMA_TFLOPS
        else:
            s = kw["split_slices"]
            pairs = s * (s + 1) // 2
            peak = PEAK_INT8_MFMA_TOPS if kw["split_type"] == "int8" else PEAK_BF16_MFMA_TFLOPS
            ent["lowprec_ops_per_s_T"] = pairs * 2.0 * n ** 3 / (med / 1e3) / 1e12
            ent["frac_lowprec_mfma_peak"] = ent["lowprec_ops_per_s_T"] / peak
        if ref is not None:
            import oracle

            got = C[ridx].cpu().numpy()
            ent["rel_err_inf_sampled"] = oracle.norm_inf(oracle.minus(got, ref)) / nrm
        out[name] = ent
        del ws
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
