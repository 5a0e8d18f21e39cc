"""Benchmark of the hot path: FP64-grade C = AB on one MI355X.

Headline (one JSON line): the split-precision product against the plain
FP64 matrix-core GEMM at N = P = M = 8192 on the wide-range workload
(entries +-2^u, u ~ U[-20, 20], rows scaled by 2^v, v ~ U{-10..10}).  One
step = one full product (digit extraction, digit GEMM, recombination) with
the operands resident in HBM.  ``value`` is the FP64-grade TFLOP/s (2NPM per
step time) of the fastest split configuration whose relative infinity-norm
error on the sampled rows is <= 1e-13; DGEMM's TFLOP/s, the ratio and the
p99 latency of a step stand beside it, with the serving p99.  ``roofline``
is the digit GEMM kernel of that configuration (the dominant kernel), its
mean launch time measured with HIP events on the stream it runs on, against
the published matrix-core peak of its digit type.  ``cpu_baseline`` is the
CPU oracle (the naive definition, all usable host cores) on a bounded sample
of the rows of the same product.

Extra keys: the 256^3 latency of every method (and the single-core oracle
time), the all-methods step at N = M = 4096, P in {4096, 4097}, the
auxiliaries' HBM bandwidth, the 2048-problem batch graph, the serving loop
at 50% and 80% of its capacity, and the paper's test table at n = 800.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--only SECTIONS]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64-grade TFLOP/s vs plain FP64 MFMA GEMM at fixed ∞-norm err; p99 latency"
FP64_GRADE = 1e-13

# MI355X published peaks and chip constants.
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_BF16_MFMA_TFLOPS = 2516.6   # dense; FP16 the same
PEAK_INT8_MFMA_TOPS = 5033.2     # dense
PEAK_HBM_GBS = 8000.0
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 16, 2.4
# non-fused FP64 vector operations per second (each op one flop): one wave64
# instruction per SIMD every 4 clocks
PEAK_FP64_VALU_OPS_T = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_GHZ * 1e9 / 1e12  # 39.3

SECTIONS = ("headline", "latency", "allmethods", "aux", "batch", "serve", "paper")

# the comparison at 8192^3: (name, method, config kwargs)
HEADLINE = [
    ("dgemm", "dgemm", {}),
    ("split_int8_s7", "split", {"split_type": "int8", "split_slices": 7}),
    ("split_bf16_s6", "split", {"split_type": "bf16", "split_slices": 6}),
    ("split_fp16_s6", "split", {"split_type": "fp16", "split_slices": 6}),
    ("split_fp16_s5", "split", {"split_type": "fp16", "split_slices": 5}),
    ("split_bf16_b9_s5", "split", {"split_type": "bf16", "split_slices": 5, "split_bits": 9}),
    ("split_int8_b8_s6", "split", {"split_type": "int8", "split_slices": 6, "split_bits": 8}),
    ("strassen_winograd_L2", "strassen_winograd", {"strassen_levels": 2}),
    ("strassen_winograd_L3", "strassen_winograd", {"strassen_levels": 3}),
]

# the all-methods step at 4096: (name, method, config kwargs, algorithmic ops per multiply-add, bound)
#   naive: 1 mul + 1 add (rounded separately) -> 2 VALU ops / MAC; kahan: 1 mul + 4 add/sub -> 5;
#   winograd: 2 add + 1 mul + 1 add per pair of MACs -> 2; dgemm: 2 flop / MAC on the FP64 matrix cores
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

LATENCY_METHODS = [
    ("naive", "naive", {}), ("kahan", "kahan", {}), ("winograd", "winograd", {}),
    ("winograd_scaled", "winograd_scaled", {}), ("dgemm", "dgemm", {}),
    ("strassen_naive_L2", "strassen_naive", {"strassen_levels": 2}),
    ("strassen_winograd_L2", "strassen_winograd", {"strassen_levels": 2}),
    ("split_int8_s7", "split", {"split_type": "int8", "split_slices": 7}),
    ("split_int8_b8_s6", "split", {"split_type": "int8", "split_slices": 6, "split_bits": 8}),
    ("split_bf16_s6", "split", {"split_type": "bf16", "split_slices": 6}),
]


# HBM bytes per launch of a kernel at the workload it is reported for (Kahan and DGEMM: the 4096 step;
# the split digit GEMMs: the 8192^3 comparison), from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE)
# scaled by what the counters read for a plain 512 MiB device copy (FETCH x 2.0, WRITE x 1.0); valid only
# while the kernel's source is the one measured (sha256 below), otherwise reported as null.
COUNTED_TRAFFIC = {
    "kahan": {"bytes": 3.3573e+09, "file": "paper_1106_1347_amd/csrc/valu_gemm.hip",
              "sha256": "784fd6af09d049f1b0e0437e1f9ddc7e8f26bb308359eddad475efd03dd2ae02"},
    "dgemm": {"bytes": 1.8793e+09, "file": "paper_1106_1347_amd/csrc/dgemm.hip",
              "sha256": "9d31101e8996d414e7cb07292a174fa4a17b51f0e9da174eb074a984527ad929"},
    "split_int8_s7": {"bytes": 2.8035e+10, "file": "paper_1106_1347_amd/csrc/split.hip",
                      "sha256": "bb68fc774998d9c613771b7561f5f4733392e02503be299b3edd28b35a99e945"},
    "split_int8_b8_s6": {"bytes": 2.0162e+10, "file": "paper_1106_1347_amd/csrc/split.hip",
                         "sha256": "bb68fc774998d9c613771b7561f5f4733392e02503be299b3edd28b35a99e945"},
    "split_bf16_b9_s5": {"bytes": 6.9849e+10, "file": "paper_1106_1347_amd/csrc/split.hip",
                         "sha256": "bb68fc774998d9c613771b7561f5f4733392e02503be299b3edd28b35a99e945"},
    "split_fp16_s5": {"bytes": 7.1554e+10, "file": "paper_1106_1347_amd/csrc/split.hip",
                      "sha256": "bb68fc774998d9c613771b7561f5f4733392e02503be299b3edd28b35a99e945"},
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


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=4096, help="N = M of the all-methods step")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip timing the CPU oracle (errors are still taken on a few sampled rows)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--only", default="", help="comma-separated sections of %s" % (SECTIONS,))
    ap.add_argument("--headline", default="", help="comma-separated subset of the 8192^3 configurations")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-budget-gib", type=float, default=96.0)
    ap.add_argument("--serve-rate", type=float, default=3000.0,
                    help="fixed Poisson arrival rate (requests/s) of the serving run the headline p50/p99 come from")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args(argv)


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time(torch, stream, fn, reps):
    ms = []
    for _ in range(reps):
        e0, e1 = _events(torch)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms))


def _pct(xs, p):
    return float(np.percentile(np.asarray(xs), p))


def _rel_err(oracle, got, ref, nrm):
    return float(oracle.norm_inf(oracle.minus(got, ref)) / nrm) if nrm > 0 else 0.0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads():
    # the host cores this process may use (its CPU affinity, at most OMP_NUM_THREADS)
    return max(1, min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16"))))


# ---------------------------------------------------------------------------------------------------
# the headline: split against DGEMM at 8192^3

def headline_section(args, mmm, torch, synth, dev, stream):
    import oracle

    n = 8192
    A = synth.wide_range((n, n), synth.seed_a(2))
    B = synth.wide_range((n, n), synth.seed_b(2))
    Ad = torch.from_numpy(A).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    flop = 2.0 * n ** 3
    todo = [h for h in HEADLINE if not args.headline or h[0] in args.headline.split(",")]

    # the CPU oracle on sampled rows first: the two rows of A with the
    # largest absolute row sums (each row carries its own 2^v scale, so they
    # set the normwise error) plus evenly spaced rows, extended to about
    # cpu_seconds of oracle work; these rows time the CPU baseline and give
    # every configuration's error
    threads = _host_threads()
    oracle.set_threads(threads)
    big = np.argsort(np.abs(A).sum(axis=1))[-2:]
    rows = np.unique(np.concatenate([np.linspace(0, n - 1, 8 * threads - 2).round().astype(np.int64), big]))
    nrm = oracle.norm_inf(A) * oracle.norm_inf(B)
    t = time.perf_counter()
    ref = oracle.naive_rows(A, B, rows)
    cpu_t = time.perf_counter() - t
    if not args.no_cpu_baseline and cpu_t < args.cpu_seconds:
        more = int(len(rows) * (args.cpu_seconds / max(cpu_t, 1e-3) - 1.0))
        more = max(0, min(more, n - len(rows)))
        if more > 0:
            rest = np.setdiff1d(np.arange(n), rows)
            extra = np.sort(np.random.default_rng(2003).choice(rest, size=more, replace=False))
            t = time.perf_counter()
            ref2 = oracle.naive_rows(A, B, extra)
            cpu_t += time.perf_counter() - t
            rows = np.concatenate([rows, extra])
            ref = np.concatenate([ref, ref2])
    ridx = torch.from_numpy(rows).to(dev)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = {"value": 2.0 * len(rows) * n * n / cpu_t / 1e12, "unit": "TFLOP/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": "%d of the %d rows of C = AB at N = P = M = 8192 (wide-range workload) by the naive "
                         "definition in FP64 (k ascending, threads split rows), %.1f s wall"
                         % (len(rows), n, cpu_t),
               "cpu_model": _cpu_model(), "seconds": cpu_t}

    runs = {}
    for name, method, kw in todo:
        cfg = mmm.Config(**kw)
        ws = torch.empty(max(mmm.workspace_bytes(method, n, n, n, cfg), 1), dtype=torch.uint8, device=dev)
        for _ in range(args.warmup):
            mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        evs = []
        mmm.timer_start()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e0, e1 = _events(torch)
            e0.record(stream)
            mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws, stream=stream)
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern_ms, launches = mmm.timer_stop()
        ms = [a.elapsed_time(b) for a, b in evs]
        mean = float(np.mean(ms))
        err = _rel_err(oracle, C[ridx].cpu().numpy(), ref, nrm)
        ent = {"ms_mean": mean, "ms_p50": _pct(ms, 50), "ms_p99": _pct(ms, 99), "ms_min": float(np.min(ms)),
               "wall_s": wall, "tflops_fp64_grade": flop / (mean / 1e3) / 1e12,
               "dominant_kernel_ms_mean": kern_ms / max(launches, 1), "dominant_kernel_launches": launches,
               "rel_err_inf_sampled_rows": err, "fp64_grade": err <= FP64_GRADE}
        if method == "dgemm":
            ent["frac_fp64_mfma_peak"] = ent["tflops_fp64_grade"] / PEAK_FP64_MFMA_TFLOPS
        elif method == "split":
            s = kw["split_slices"]
            pairs = s * (s + 1) // 2
            peak = PEAK_INT8_MFMA_TOPS if kw["split_type"] == "int8" else PEAK_BF16_MFMA_TFLOPS
            ent["digit_pairs"] = pairs
            ent["digit_gemm_T_ops_per_s"] = pairs * flop / (ent["dominant_kernel_ms_mean"] / 1e3) / 1e12
            ent["digit_gemm_frac_peak"] = ent["digit_gemm_T_ops_per_s"] / peak
        elif method == "strassen_winograd":
            ent["leaf_flop_share"] = (7.0 / 8.0) ** kw["strassen_levels"]
        runs[name] = ent
        del ws

    out = {"workload": "C = AB, N = P = M = 8192, entries +-2^u (u ~ U[-20,20]) with rows scaled by 2^v "
                       "(v ~ U{-10..10}), seeds 2001/2002; one product per step, operands resident in HBM",
           "rows_checked": int(len(rows)),
           "error_note": "relative infinity-norm error on the sampled rows (including the two rows of A with "
                         "the largest row sums): a lower bound of the error over all rows",
           "configs": runs}
    # vendor-library ceilings measured on the same box (context for the peaks, never part of the path)
    ceil = {}
    for cname, X, Y, peak in (("vendor_fp64_gemm", Ad, Bd, PEAK_FP64_MFMA_TFLOPS),
                              ("vendor_bf16_gemm", Ad.to(torch.bfloat16).contiguous(),
                               Bd.to(torch.bfloat16).contiguous(), PEAK_BF16_MFMA_TFLOPS)):
        Z = torch.empty((n, n), dtype=X.dtype, device=dev)
        with torch.cuda.stream(stream):
            torch.matmul(X, Y, out=Z)
            ms = _time(torch, stream, lambda: torch.matmul(X, Y, out=Z), 5)
        tf = flop / (ms / 1e3) / 1e12
        ceil[cname] = {"ms_p50": ms, "tflops": tf, "frac_peak": tf / peak}
        del Z
    out["library_ceilings"] = ceil
    return out, cpu


# ---------------------------------------------------------------------------------------------------
# 256^3 latency (the small configuration) and the single-core oracle time

def latency_section(mmm, torch, synth, dev, stream):
    import oracle

    n = 256
    out = {"workload": "N = P = M = 256, U[-1,1] (seeds 1/2) and integers in {-8..8} (bitwise check)"}
    A = synth.uniform((n, n), synth.seed_a(0))
    B = synth.uniform((n, n), synth.seed_b(0))
    Ai = synth.integers((n, n), synth.seed_a(0))
    Bi = synth.integers((n, n), synth.seed_b(0))
    exact = (Ai.astype(np.int64) @ Bi.astype(np.int64)).astype(np.float64)
    Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    Aid, Bid = torch.from_numpy(Ai).to(dev), torch.from_numpy(Bi).to(dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    oracle.set_threads(1)
    t = time.perf_counter()
    ref = oracle.naive(A, B)
    out["oracle_single_core_ms"] = 1e3 * (time.perf_counter() - t)
    oracle.set_threads(_host_threads())
    nrm = oracle.norm_inf(A) * oracle.norm_inf(B)
    res = {}
    for name, method, kw in LATENCY_METHODS:
        cfg = mmm.Config(**kw)
        ws = torch.empty(max(mmm.workspace_bytes(method, n, n, n, cfg), 1), dtype=torch.uint8, device=dev)
        run = lambda: mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws, stream=stream)  # noqa: E731
        run()
        ms = []
        for _ in range(20):
            e0, e1 = _events(torch)
            e0.record(stream)
            run()
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        err = _rel_err(oracle, C.cpu().numpy(), ref, nrm)
        mmm.multiply(Aid, Bid, method, cfg, out=C, workspace=ws, stream=stream)
        ok = bool(np.array_equal(C.cpu().numpy().view(np.int64), exact.view(np.int64)))
        res[name] = {"us_p50": 1e3 * _pct(ms, 50), "us_p99": 1e3 * _pct(ms, 99), "rel_err_inf": err,
                     "integer_inputs_exact": ok}
    out["methods"] = res
    return out


# ---------------------------------------------------------------------------------------------------
# every method at N = M = 4096, P in {4096, 4097}

def allmethods_section(args, mmm, torch, synth, dev, stream):
    import oracle

    n = args.size
    shapes = [(n, n, n), (n, n + 1, n)]
    data = {}
    for (N, P, M) in shapes:
        A = synth.uniform((N, P), synth.seed_a(1))
        B = synth.uniform((P, M), synth.seed_b(1))
        data[P] = (A, B, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev),
                   torch.empty((N, M), dtype=torch.float64, device=dev))
    ws = {}
    for name, method, kw, _, _ in METHODS:
        cfg = mmm.Config(**kw)
        for (N, P, M) in shapes:
            ws[(name, P)] = torch.empty(max(mmm.workspace_bytes(method, N, P, M, cfg), 1), dtype=torch.uint8,
                                        device=dev)

    def one_step(timings):
        for name, method, kw, _, _ in METHODS:
            cfg = mmm.Config(**kw)
            for (N, P, M) in shapes:
                _, _, Ad, Bd, C = data[P]
                e0, e1 = _events(torch)
                e0.record(stream)
                mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws[(name, P)], stream=stream)
                e1.record(stream)
                if timings is not None:
                    timings.append((name, P, e0, e1))

    one_step(None)
    torch.cuda.synchronize()
    timings, steps = [], []
    steps_n = max(1, min(args.steps, 3))
    for _ in range(steps_n):
        s0, s1 = _events(torch)
        s0.record(stream)
        one_step(timings)
        s1.record(stream)
        steps.append((s0, s1))
    torch.cuda.synchronize()
    step_ms = [a.elapsed_time(b) for a, b in steps]
    per = {}
    for name, P, e0, e1 in timings:
        per.setdefault(name, []).append(e0.elapsed_time(e1))
    # the dominant kernel of each single-kernel method, timed with the library's event brackets
    kern = {}
    for name, method, kw, cost, _ in METHODS:
        if cost is None:
            continue
        cfg = mmm.Config(**kw)
        mmm.timer_start()
        for _ in range(steps_n):
            for (N, P, M) in shapes:
                _, _, Ad, Bd, C = data[P]
                mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws[(name, P)], stream=stream)
        tot, cnt = mmm.timer_stop()
        kern[name] = tot / max(cnt, 1)
    # errors on sampled rows against the oracle
    oracle.set_threads(_host_threads())
    rows = np.linspace(0, n - 1, 64).round().astype(np.int64)
    ridx = torch.from_numpy(rows).to(dev)
    ref = {P: oracle.naive_rows(data[P][0], data[P][1], rows) for (_, P, _) in shapes}
    nrm = {P: oracle.norm_inf(data[P][0]) * oracle.norm_inf(data[P][1]) for (_, P, _) in shapes}
    res = {}
    macs = np.mean([N * P * M for (N, P, M) in shapes])
    for name, method, kw, cost, bound in METHODS:
        cfg = mmm.Config(**kw)
        worst = 0.0
        for (N, P, M) in shapes:
            _, _, Ad, Bd, C = data[P]
            mmm.multiply(Ad, Bd, method, cfg, out=C, workspace=ws[(name, P)], stream=stream)
            worst = max(worst, _rel_err(oracle, C[ridx].cpu().numpy(), ref[P], nrm[P]))
        ms = np.array(per[name])
        ent = {"ms_mean": float(ms.mean()), "ms_p50": _pct(ms, 50), "ms_p99": _pct(ms, 99),
               "tflops_fp64_grade": 2.0 * macs / (ms.mean() / 1e3) / 1e12, "rel_err_inf_sampled_rows": worst}
        if cost is not None:
            km = kern[name]
            peak = PEAK_FP64_MFMA_TFLOPS if bound == "mfma" else PEAK_FP64_VALU_OPS_T
            ent["kernel_ms_mean"] = km
            ent["kernel_T_ops_per_s"] = cost * macs / (km / 1e3) / 1e12
            ent["kernel_frac_peak"] = ent["kernel_T_ops_per_s"] / peak
            ent["bound"] = bound
        res[name] = ent
    flop_step = sum(2.0 * N * P * M for (N, P, M) in shapes) * len(METHODS)
    dom = max((m for m in METHODS if m[3] is not None), key=lambda m: res[m[0]]["kernel_ms_mean"])
    return {"workload": "C = AB, N = M = %d, P in {%d, %d}, U[-1,1] (seeds 1001/1002); one step = every method "
                        "once on each shape" % (n, n, n + 1),
            "step_ms_mean": float(np.mean(step_ms)), "steps": steps_n,
            "tflops_fp64_grade_step": flop_step / (np.mean(step_ms) / 1e3) / 1e12,
            "fp64_grade_all": all(r["rel_err_inf_sampled_rows"] <= FP64_GRADE for r in res.values()),
            "dominant_kernel": {"kernel": dom[0], "bound": "alu" if dom[4] == "alu" else "mfma",
                                "achieved": res[dom[0]]["kernel_T_ops_per_s"],
                                "peak": PEAK_FP64_VALU_OPS_T if dom[4] == "alu" else PEAK_FP64_MFMA_TFLOPS,
                                "unit": "TFLOP/s", "frac": res[dom[0]]["kernel_frac_peak"],
                                "traffic": counted_traffic(dom[0])},
            "methods": res}


# ---------------------------------------------------------------------------------------------------

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


def batch_section(mmm, torch, synth, dev, stream, split_type="bf16", split_slices=6, tuner_path=None):
    """2048 independent products, N, P, M uniform on 16..512, entries
    U[-1,1]; even index FP64 DGEMM, odd index split: one graph launch
    (DGEMM tile shapes from the autotuner) against 2048 separate calls, then
    every result against the CPU oracle."""
    import oracle
    from paper_1106_1347_amd.tune import TileTuner

    shapes = synth.batch_shapes(2048, synth.seed_a(3), 16, 512)
    probs, host = [], []
    for g, (N, P, M) in enumerate(shapes):
        A = synth.uniform((N, P), synth.seed_item(3, g, "A"))
        B = synth.uniform((P, M), synth.seed_item(3, g, "B"))
        host.append((A, B))
        probs.append((torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev),
                      torch.empty((N, M), dtype=torch.float64, device=dev), "dgemm" if g % 2 == 0 else "split"))
    cfg = mmm.Config(split_type=split_type, split_slices=split_slices)
    t0 = time.perf_counter()
    if tuner_path is None:
        import tempfile

        # a fresh table for this run (tuned, persisted, then read back by the plan)
        tuner_path = os.path.join(tempfile.mkdtemp(prefix="mmm_tiles_"), "tiles.json")
    tuner = TileTuner(path=tuner_path)
    tuner.tune([s for g, s in enumerate(shapes) if g % 2 == 0], split=[s for g, s in enumerate(shapes) if g % 2 == 1],
               split_config=cfg)
    policy = tuner.tune_batch(probs, cfg)
    tune_s = time.perf_counter() - t0
    plan_probs = [(A, B, C, m, 0, t) for (A, B, C, m), t in zip(probs, tuner.tiles_for(probs, cfg))]
    t0 = time.perf_counter()
    plan = mmm.Batch(plan_probs, cfg, stream=stream)
    create_s = time.perf_counter() - t0
    plan.launch(stream)
    torch.cuda.synchronize()
    ms_graph = []
    for _ in range(10):
        e0, e1 = _events(torch)
        e0.record(stream)
        plan.launch(stream)
        e1.record(stream)
        e1.synchronize()
        ms_graph.append(e0.elapsed_time(e1))
    plan_auto = mmm.Batch(probs, cfg, stream=stream)
    plan_auto.launch(stream)
    ms_auto = _time(torch, stream, lambda: plan_auto.launch(stream), 5)
    plan_auto.close()
    plan.launch(stream)  # the results checked below come from the tuned graph

    torch.cuda.synchronize()
    outs = [C.cpu().numpy() for (_, _, C, _) in probs]

    def separate():
        for (A, B, C, m) in probs:
            mmm.multiply(A, B, m, cfg, out=C, stream=stream)

    separate()
    ms_sep = _time(torch, stream, separate, 3)
    plan.close()
    # extra: the same graph with the split half as int8 byte digits (6 digits of 8 bits), tiles tuned for it
    cfg8 = mmm.Config(split_type="int8", split_slices=6, split_bits=8)
    tuner.tune([s for g, s in enumerate(shapes) if g % 2 == 0], split=[s for g, s in enumerate(shapes) if g % 2 == 1],
               split_config=cfg8)
    policy8 = tuner.tune_batch(probs, cfg8)
    plan8 = mmm.Batch([(A, B, C, m, 0, t) for (A, B, C, m), t in zip(probs, tuner.tiles_for(probs, cfg8))], cfg8,
                      stream=stream)
    plan8.launch(stream)
    ms8 = _time(torch, stream, lambda: plan8.launch(stream), 10)
    plan8.launch(stream)
    torch.cuda.synchronize()
    outs8 = [C.cpu().numpy() for (_, _, C, m) in probs if m == "split"]
    plan8.close()
    # every result against the oracle (the naive definition, full products)
    oracle.set_threads(_host_threads())
    t0 = time.perf_counter()
    worst = {"dgemm": 0.0, "split": 0.0}
    worst8 = 0.0
    refs = {}
    for g, ((A, B), C) in enumerate(zip(host, outs)):
        ref = oracle.naive(A, B)
        e = _rel_err(oracle, C, ref, oracle.norm_inf(A) * oracle.norm_inf(B))
        k = "dgemm" if g % 2 == 0 else "split"
        worst[k] = max(worst[k], e)
        if k == "split":
            refs[g] = ref
    for g8, C in zip(sorted(refs), outs8):
        A, B = host[g8]
        worst8 = max(worst8, _rel_err(oracle, C, refs[g8], oracle.norm_inf(A) * oracle.norm_inf(B)))
    check_s = time.perf_counter() - t0
    flop = sum(2.0 * N * P * M for (N, P, M) in shapes)
    med = float(np.median(ms_graph))
    return {"workload": "2048 products, N,P,M ~ U{16..512}, U[-1,1] (item seeds 3010+2g / 3011+2g), even index "
                        "DGEMM, odd index split %s x%d, one HIP graph" % (split_type, split_slices),
            "tune_s": tune_s, "plan_create_s": create_s, "ms_graph_p50": med, "ms_graph_p99": _pct(ms_graph, 99),
            "ms_graph_untuned_p50": ms_auto, "ms_separate_calls_p50": ms_sep,
            "tflops_fp64_grade_graph": flop / (med / 1e3) / 1e12, "speedup_vs_separate": ms_sep / med,
            "flop": flop, "rel_err_inf_worst": worst, "all_within_1e-13": max(worst.values()) <= FP64_GRADE,
            "oracle_check": "every product in full against the naive definition, %.1f s" % check_s,
            "extra_int8_byte_digits": {"split": "int8 x6, 8-bit byte digits", "ms_graph_p50": ms8,
                                       "tflops_fp64_grade_graph": flop / (ms8 / 1e3) / 1e12,
                                       "rel_err_inf_worst_split": worst8, "tile_policy": {"dgemm": policy8[0], "split": policy8[1]}},
            "tile_policy": {"dgemm": policy[0], "split": policy[1]}, "tiles": tuner.summary()}


def serve_section(args, mmm, torch, synth, dev):
    """Poisson request stream, dims log-uniform on 32..4096 (half square),
    tolerance 1e-13 or 1e-10, methods routed by measured cost: capacity
    measured closed-loop, then p50/p99 latency (arrival to completion event)
    at a fixed rate (``--serve-rate``, the headline's) and at 50% and 80% of
    the capacity; afterwards every result of the 80% run against the CPU
    oracle on sampled rows."""
    import oracle
    from paper_1106_1347_amd.serve import Router, Server

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
    budget = int(args.serve_budget_gib * (1 << 30))
    t0 = time.perf_counter()
    router = Router()
    router.calibrate()
    cal_s = time.perf_counter() - t0
    # warm-up and closed-loop capacity
    srv = Server(budget, streams=4, router=router)
    for f in [srv.submit(A, B, tol) for (A, B, tol) in data[: min(40, n)]]:
        f.result()
    srv.close()
    srv = Server(budget, streams=4, router=router)
    for f in [srv.submit(A, B, tol) for (A, B, tol) in data]:
        f.result()
    cap = srv.stats()
    srv.close()
    out = {"workload": "%d requests, dims log-uniform 32..4096 (half square), U[-1,1], tol 1e-13 | 1e-10, HBM "
                       "budget %.0f GiB, 4 streams, methods routed by measured cost" % (n, args.serve_budget_gib),
           "router_calibration_s": cal_s, "router_ms": router.table, "router_sizes": router.sizes,
           "capacity_req_per_s": cap["req_per_s"], "closed_loop": cap}
    results = None
    for key, rate in (("fixed_rate", args.serve_rate), ("load_50", 0.5 * cap["req_per_s"]),
                      ("load_80", 0.8 * cap["req_per_s"])):
        arrivals = np.cumsum(np.random.default_rng(4004).exponential(1.0 / rate, size=n))
        srv = Server(budget, streams=4, router=router)
        t0 = time.perf_counter()
        futs = []
        for (A, B, tol), ta in zip(data, arrivals):
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            futs.append(srv.submit(A, B, tol))
        results = [f.result() for f in futs]
        st = srv.stats()
        srv.close()
        st["offered_req_per_s"] = rate
        out[key] = st
    # every result of the last run against the oracle: 4 rows each (the row of
    # A with the largest absolute row sum among them)
    oracle.set_threads(_host_threads())
    t0 = time.perf_counter()
    worst = {1e-13: 0.0, 1e-10: 0.0}
    fails = 0
    rng = np.random.default_rng(4005)
    for (A, B, tol), C in zip(data, results):
        An, Bn = A.cpu().numpy(), B.cpu().numpy()
        N = An.shape[0]
        rows = np.unique(np.concatenate([rng.choice(N, size=min(3, N), replace=False),
                                         [int(np.argmax(np.abs(An).sum(axis=1)))]])).astype(np.int64)
        ridx = torch.from_numpy(rows).to(dev)
        e = _rel_err(oracle, C[ridx].cpu().numpy(), oracle.naive_rows(An, Bn, rows),
                     oracle.norm_inf(An) * oracle.norm_inf(Bn))
        worst[tol] = max(worst[tol], e)
        fails += e > tol
    out["oracle_check"] = {"requests": n, "rows_per_request": "up to 4 (incl. the largest row sum of A)",
                           "worst_rel_err_tol_1e-13": worst[1e-13], "worst_rel_err_tol_1e-10": worst[1e-10],
                           "over_tolerance": int(fails), "seconds": time.perf_counter() - t0}
    return out


def paper_test_section():
    """The paper's test program at n = 800, R = 10 (C = A (8A), N := NaivKahan):
    per method the median time of one product and NormInf(N - C)."""
    from paper_1106_1347_amd import papertest

    res = papertest.run(n=800, repeats=10, seed=500)
    return {"workload": "C = A (8A), A 800 x 800 ~ U[0,1) (seed 500), N := NaivKahan, R = 10",
            "rows": {r["label"]: {"ms": 1e3 * r["seconds"], "norm_inf_n_minus_c": r["err"]} for r in res["rows"]}}


# ---------------------------------------------------------------------------------------------------

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
    only = set(args.only.split(",")) if args.only else set(SECTIONS)
    bad = only - set(SECTIONS)
    if bad:
        print("unknown sections %s; choose from %s" % (sorted(bad), SECTIONS), file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.copy_mib:
        src = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def log(msg):
        print("[bench] %s" % msg, file=sys.stderr, flush=True)

    head, cpu = (None, None)
    if "headline" in only:
        log("headline 8192^3")
        head, cpu = headline_section(args, mmm, torch, synth, dev, stream)
    extra = {}
    for key, sec, fn in (("latency_256", "latency", lambda: latency_section(mmm, torch, synth, dev, stream)),
                         ("allmethods_4096", "allmethods",
                          lambda: allmethods_section(args, mmm, torch, synth, dev, stream)),
                         ("aux_8192", "aux", lambda: aux_section(mmm, torch, dev, stream)),
                         ("batch_2048", "batch", lambda: batch_section(mmm, torch, synth, dev, stream)),
                         ("serving", "serve", lambda: serve_section(args, mmm, torch, synth, dev)),
                         ("paper_test_800", "paper", paper_test_section)):
        if sec in only:
            log(sec)
            extra[key] = fn()
            torch.cuda.empty_cache()

    out = {"metric": METRIC, "value": None, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": None, "data": "synthetic",
           "config": {"workload": "C = AB, N = P = M = 8192, FP64 wide-range entries (+-2^u, u ~ U[-20,20], rows "
                                  "x 2^v, v ~ U{-10..10}); split-precision product with 3-6 BF16 or FP16 slices "
                                  "and FP32 accumulation vs the plain FP64 matrix-core GEMM; one product per step "
                                  "(int8 digits beyond that under int8_extension)", "parallelism": "single GPU"}}
    if head is not None:
        cf = head["configs"]
        dg = cf.get("dgemm")

        def kw_of(name):
            return [h for h in HEADLINE if h[0] == name][0][2]

        def summary(name):
            b, kw = cf[name], kw_of(name)
            peak = PEAK_INT8_MFMA_TOPS if kw["split_type"] == "int8" else PEAK_BF16_MFMA_TFLOPS
            r = {"value": b["tflops_fp64_grade"], "ms_per_step": b["ms_mean"],
                 "dtype": {"int8": "i8 digits, i32 accumulation, f64 recombination",
                           "bf16": "bf16 digits, f32 accumulation, f64 recombination",
                           "fp16": "f16 digits, f32 accumulation, f64 recombination"}[kw["split_type"]],
                 "p50_ms": b["ms_p50"], "p99_ms": b["ms_p99"], "rel_err_inf": b["rel_err_inf_sampled_rows"],
                 "split": name, "digits": kw["split_slices"], "digit_type": kw["split_type"],
                 "digit_bits": kw.get("split_bits", 0) or {"int8": 7, "bf16": 8, "fp16": 9}[kw["split_type"]]}
            r["roofline"] = {"bound": "mfma", "kernel": "digit GEMM of %s" % name,
                             "achieved": b["digit_gemm_T_ops_per_s"], "peak": peak, "unit": "TFLOP/s",
                             "frac": b["digit_gemm_frac_peak"], "traffic": counted_traffic(name),
                             "note": "achieved = %d digit pairs x 2NPM / mean launch time of the digit GEMM "
                                     "kernel (HIP events on its stream, %d launches); peak = the published "
                                     "dense %s matrix-core rate (int8: operations)"
                                     % (b["digit_pairs"], b["dominant_kernel_launches"], kw["split_type"])}
            if dg is not None:
                r["vs_dgemm"] = b["tflops_fp64_grade"] / dg["tflops_fp64_grade"]
            return r

        ok = [k for k in cf if k.startswith("split") and cf[k]["fp64_grade"]]
        # the headline: the configuration the metric names (3-6 BF16 or FP16 slices, FP32 accumulation)
        named = [k for k in ok if kw_of(k)["split_type"] in ("bf16", "fp16") and 3 <= kw_of(k)["split_slices"] <= 6]
        best = max(named, key=lambda k: cf[k]["tflops_fp64_grade"]) if named else None
        if best is not None:
            h = summary(best)
            out.update({"value": h["value"], "ms_per_step": h["ms_per_step"], "dtype": h["dtype"],
                        "p50_ms": h["p50_ms"], "p99_ms": h["p99_ms"], "rel_err_inf": h["rel_err_inf"],
                        "best_split": best, "roofline": h["roofline"]})
            out["config"].update({"split": best, "digits": h["digits"], "digit_type": h["digit_type"],
                                  "digit_bits": h["digit_bits"]})
        # beyond the named configuration: INT8 digits (7-bit nearest digits or 8-bit byte digits)
        int8 = [k for k in ok if kw_of(k)["split_type"] == "int8"]
        if int8:
            out["int8_extension"] = summary(max(int8, key=lambda k: cf[k]["tflops_fp64_grade"]))
        if dg is not None:
            out["dgemm_tflops"] = dg["tflops_fp64_grade"]
            out["dgemm_ms"] = dg["ms_mean"]
            out["dgemm_rel_err_inf"] = dg["rel_err_inf_sampled_rows"]
            if out["value"] is not None:
                out["vs_dgemm"] = out["value"] / dg["tflops_fp64_grade"]
        out["precision_8192"] = head
    out["cpu_baseline"] = cpu
    if "serving" in extra:
        # at a fixed arrival rate, so that the figure does not move with the
        # capacity a box measures (the 50% / 80% runs are under "serving")
        out["serving_rate_req_per_s"] = extra["serving"]["fixed_rate"]["offered_req_per_s"]
        out["serving_p50_ms"] = extra["serving"]["fixed_rate"]["p50_ms"]
        out["serving_p99_ms"] = extra["serving"]["fixed_rate"]["p99_ms"]
    out.update(extra)
    out["device"] = torch.cuda.get_device_name(0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
