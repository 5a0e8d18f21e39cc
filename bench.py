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
    ("split_fp16_s6", "split", {"split_type": "fp16", "split_slices": 6}),
    ("strassen_winograd_L1", "strassen_winograd", {"strassen_levels": 1}),
    ("strassen_winograd_L2", "strassen_winograd", {"strassen_levels": 2}),
]


# HBM bytes per launch of a kernel, from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by
# what the counters read for a plain 512 MiB device copy (FETCH x 2.0, WRITE x 1.0); valid only while the
# kernel's source is the one measured (sha256 below), otherwise reported as null.
COUNTED_TRAFFIC = {
    "kahan": {"bytes": 3.3577e+09, "file": "paper_1106_1347_amd/csrc/valu_gemm.hip",
              "sha256": "c222f1ed93ef6f95a59b2dd1ad0c3a9a77fe8ea689a6f0462e24b53b7677e36c"},
    "dgemm": {"bytes": 1.8797e+09, "file": "paper_1106_1347_amd/csrc/dgemm.hip",
              "sha256": "6cde41f24dff417abc4b34646945670d8025cd7dcfaed948b7a1f600fb7a36e7"},
}


def counted_traffic(name):
    import hashlib

    rec = COUNTED_TRAFFIC.get(name)
    if not rec:
        return None
    try:
        with open(os.path.join(ROOT, rec["file"]), "rb") as f:
            ok = hashlib.sha256(f.read()).hexdigest() == rec["sha256"]
    except OSError:
        return None
    return rec["bytes"] if ok else None


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
    ap.add_argument("--no-aux", action="store_true", help="skip the auxiliary-kernel bandwidth section")
    ap.add_argument("--no-batch", action="store_true", help="skip the 2048-problem batch section")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--no-paper-test", action="store_true", help="skip the paper's test table (n = 800)")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the products of the workload "
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
    if args.copy_mib:
        src = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

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
    aux = None if args.no_aux else aux_section(mmm, torch, dev, stream)
    batch = None if args.no_batch else batch_section(mmm, torch, synth, dev, stream)
    serving = None if args.no_serve else serve_section(args, mmm, torch, synth, dev)
    paper_test = None if args.no_paper_test else paper_test_section()

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
                "frac": achieved / peak, "traffic": counted_traffic(dname),
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
        "aux_8192": aux,
        "batch_2048": batch,
        "serving": serving,
        "paper_test_800": paper_test,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)


def precision_section(args, mmm, torch, synth, dev, stream, errors_needed):
    """DGEMM against the split products and Strassen-Winograd (DGEMM leaf, 1
    and 2 levels) at N = P = M = 8192 on the wide-range distribution: median
    time, FP64-grade TFLOP/s (2NPM/t) and relative infinity-norm error on
    sampled rows against the oracle."""
    n = 8192
    A = synth.wide_range((n, n), synth.seed_a(2))
    B = synth.wide_range((n, n), synth.seed_b(2))
    Ad = torch.from_numpy(A).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    out = {"workload": "N = P = M = 8192, entries +-2^u (u ~ U[-20,20]), rows scaled by 2^v (v ~ U{-10..10}), "
                       "seeds 2001/2002", "reps": args.precision_reps}
    # fixed rows plus the two rows of A with the largest absolute row sums:
    # every row of this workload has its own 2^v scale, and the normwise
    # error is set by the largest rows
    big = np.argsort(np.abs(A).sum(axis=1))[-2:]
    rows = np.unique(np.concatenate([np.array([0, 1, 2048, 4095, 6000, 8191]), big]))
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
        elif method == "strassen_winograd":
            L = kw["strassen_levels"]
            ent["leaf_flop_share"] = (7.0 / 8.0) ** L  # of 2NPM, on the FP64 matrix cores
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
    # ceilings measured with the vendor library on the same box (context for
    # the peaks, never part of the path): FP64 and BF16 GEMMs of this size
    ceil = {}
    for name, X, Y, peak in (("vendor_fp64_gemm", Ad, Bd, PEAK_FP64_MFMA_TFLOPS),
                             ("vendor_bf16_gemm", Ad.to(torch.bfloat16).contiguous(),
                              Bd.to(torch.bfloat16).contiguous(), PEAK_BF16_MFMA_TFLOPS)):
        Z = torch.empty((n, n), dtype=X.dtype, device=dev)
        with torch.cuda.stream(stream):
            torch.matmul(X, Y, out=Z)
            ms = _time(torch, stream, lambda: torch.matmul(X, Y, out=Z), args.precision_reps)
        tf = 2.0 * n ** 3 / (ms / 1e3) / 1e12
        ceil[name] = {"ms_p50": ms, "tflops": tf, "frac_peak": tf / peak}
        del Z
    out["library_ceilings"] = ceil
    return out


def _time(torch, stream, fn, reps):
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms))


def paper_test_section():
    """The paper's test program at n = 800, R = 10 (C = A (8A), N := NaivKahan):
    per method the median time of one product and NormInf(N - C)."""
    from paper_1106_1347_amd import papertest

    res = papertest.run(n=800, repeats=10, seed=500)
    return {"workload": "C = A (8A), A 800 x 800 ~ U[0,1) (seed 500), N := NaivKahan, R = 10",
            "rows": {r["label"]: {"ms": 1e3 * r["seconds"], "norm_inf_n_minus_c": r["err"]} for r in res["rows"]}}


def aux_section(mmm, torch, dev, stream):
    """Plus, Minus, MultiplyWithScalar and NormInf on 8192 x 8192 operands
    (512 MiB each, above the 256 MB Infinity Cache): algorithmic bytes per
    entry 24, 24, 16 and 8; GB/s against the 8 TB/s HBM peak."""
    n = 8192
    X = torch.rand(n, n, dtype=torch.float64, device=dev)
    Y = torch.rand(n, n, dtype=torch.float64, device=dev)
    Z = torch.empty_like(X)
    out = torch.empty((), dtype=torch.float64, device=dev)
    res = {}
    for name, fn, bpe in (("plus", lambda: mmm.plus(X, Y, out=Z, stream=stream), 24),
                          ("minus", lambda: mmm.minus(X, Y, out=Z, stream=stream), 24),
                          ("multiply_with_scalar", lambda: mmm.multiply_with_scalar(0.5, X, out=Z, stream=stream), 16),
                          ("norm_inf", lambda: mmm.norm_inf(X, out=out, stream=stream), 8)):
        fn()
        ms = _time(torch, stream, fn, 10)
        gbs = bpe * n * n / (ms / 1e3) / 1e9
        res[name] = {"ms_p50": ms, "GB_s": gbs, "frac_hbm_peak": gbs / PEAK_HBM_GBS}
    # ceiling: the runtime's own device-to-device copy of one operand (16 bytes per entry)
    with torch.cuda.stream(stream):
        Z.copy_(X)
        ms = _time(torch, stream, lambda: Z.copy_(X), 10)
    gbs = 16 * n * n / (ms / 1e3) / 1e9
    res["ceiling_device_copy"] = {"ms_p50": ms, "GB_s": gbs, "frac_hbm_peak": gbs / PEAK_HBM_GBS}
    return res


def batch_section(mmm, torch, synth, dev, stream):
    """2048 independent products, N, P, M uniform on 16..512, entries
    U[-1,1]; even index FP64 DGEMM, odd index split (int8 digits, 7): one
    graph launch against 2048 separate calls."""
    shapes = synth.batch_shapes(2048, synth.seed_a(3), 16, 512)
    probs = []
    for g, (N, P, M) in enumerate(shapes):
        gen = torch.Generator(device=dev).manual_seed(3010 + g)
        A = torch.rand((N, P), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
        B = torch.rand((P, M), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
        probs.append((A, B, torch.empty((N, M), dtype=torch.float64, device=dev), "dgemm" if g % 2 == 0 else "split"))
    cfg = mmm.Config(split_type="int8", split_slices=7)
    t0 = time.perf_counter()
    plan = mmm.Batch(probs, cfg, stream=stream)
    create_s = time.perf_counter() - t0
    plan.launch(stream)
    torch.cuda.synchronize()
    ms_graph = _time(torch, stream, lambda: plan.launch(stream), 5)
    def separate():
        for (A, B, C, m) in probs:
            mmm.multiply(A, B, m, cfg, out=C, stream=stream)

    separate()
    ms_sep = _time(torch, stream, separate, 3)
    plan.close()
    flop = sum(2.0 * N * P * M for (N, P, M) in shapes)
    return {"workload": "2048 products, N,P,M ~ U{16..512}, half DGEMM, half split int8 x7, one HIP graph",
            "plan_create_s": create_s, "ms_graph_p50": ms_graph, "ms_separate_calls_p50": ms_sep,
            "tflops_fp64_grade_graph": flop / (ms_graph / 1e3) / 1e12, "speedup_vs_separate": ms_sep / ms_graph,
            "flop": flop}


def serve_section(args, mmm, torch, synth, dev):
    """Poisson request stream, dims log-uniform on 32..4096 (half square),
    tolerance 1e-13 or 1e-10: capacity measured closed-loop, then p50/p99
    latency (arrival to completion event) at 50% and 80% of it."""
    from paper_1106_1347_amd.serve import Server

    n = args.serve_requests
    reqs = synth.serving_requests(n, synth.seed_a(4), rate_per_s=1.0)
    data = []
    for r in reqs:
        N, P, M = r["shape"]
        gen = torch.Generator(device=dev).manual_seed(4010 + r["id"])
        A = torch.rand((N, P), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
        B = torch.rand((P, M), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
        data.append((A, B, r["tol"]))
    torch.cuda.synchronize()
    budget = 64 << 30
    # warm-up and closed-loop capacity
    srv = Server(budget, streams=4)
    for f in [srv.submit(A, B, tol) for (A, B, tol) in data[: min(40, n)]]:
        f.result()
    srv.close()
    srv = Server(budget, streams=4)
    for f in [srv.submit(A, B, tol) for (A, B, tol) in data]:
        f.result()
    cap = srv.stats()
    srv.close()
    out = {"workload": "%d requests, dims log-uniform 32..4096 (half square), tol 1e-13 | 1e-10, HBM budget 64 GiB, "
                       "4 streams" % n, "capacity_req_per_s": cap["req_per_s"], "closed_loop": cap}
    for frac in (0.5, 0.8):
        rate = frac * cap["req_per_s"]
        arrivals = np.cumsum(np.random.default_rng(4004).exponential(1.0 / rate, size=n))
        srv = Server(budget, streams=4)
        t0 = time.perf_counter()
        futs = []
        for (A, B, tol), ta in zip(data, arrivals):
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            futs.append(srv.submit(A, B, tol))
        for f in futs:
            f.result()
        st = srv.stats()
        srv.close()
        st["offered_req_per_s"] = rate
        out["load_%d" % int(frac * 100)] = st
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
