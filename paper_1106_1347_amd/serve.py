"""Continuous-batching request loop for C = AB on one GPU.

Requests (A, B, tolerance) arrive at any time.  A scheduler thread admits
waiting requests whenever their HBM footprint (operands, result and
workspace) fits the free part of the budget and a stream slot is free,
enqueues each admitted product on its own stream from a pool, and retires
products as their completion events fire, freeing their budget for the next
admissions.  Work of different requests therefore overlaps on the device
while new requests keep being admitted.

Admission order: arrival order, except that a later request that fits may
pass an earlier one that does not (no head-of-line blocking) -- until the
oldest waiting request has waited ``max_wait_s``: from then on nothing is
admitted ahead of it, so it is admitted as soon as the work already in
flight has freed enough budget (an aging bound: no request starves behind
a stream of smaller ones).

Each request is computed by a method chosen from its own shape and
tolerance only (``Router``: the fastest method whose error meets the
tolerance, by a table of measured times), with no cross-request reduction,
so its result is bit for bit the same alone and in any mix.

Latency of a request = completion time (its completion event observed by
the scheduler) - arrival time (``submit``), on the host clock.
"""
import bisect
import collections
import dataclasses
import json
import math
import os
import threading
import time
from concurrent.futures import Future
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import torch

from ._lib import Config, multiply, workspace_bytes

# Candidate methods per tolerance class, with the relative infinity-norm
# error each keeps on the serving workloads (uniform entries): the plain
# FP64 matrix-core GEMM, the int8 split with 7 digits, 6 byte digits (int8,
# 8 bits) and the bf16 split with 5 digits of 9 bits (about 3e-15) are
# FP64-grade (<= 1e-13); 5 int8 digits, 5 byte digits, 4 bf16 digits of 9
# bits (about 1e-12) and Strassen-Winograd with a DGEMM leaf are within
# 1e-10.  Each entry: (name, method, config kwargs).
CANDIDATES = {
    "fp64": [("dgemm", "dgemm", {}),
             ("split_int8_s7", "split", {"split_type": "int8", "split_slices": 7}),
             ("split_int8_b8_s6", "split", {"split_type": "int8", "split_slices": 6, "split_bits": 8}),
             ("split_bf16_b9_s5", "split", {"split_type": "bf16", "split_slices": 5, "split_bits": 9})],
    "relaxed": [("dgemm", "dgemm", {}),
                ("split_int8_s5", "split", {"split_type": "int8", "split_slices": 5}),
                ("split_int8_b8_s5", "split", {"split_type": "int8", "split_slices": 5, "split_bits": 8}),
                ("split_bf16_b9_s4", "split", {"split_type": "bf16", "split_slices": 4, "split_bits": 9}),
                ("strassen_winograd_L1", "strassen_winograd", {"strassen_levels": 1}),
                ("strassen_winograd_L2", "strassen_winograd", {"strassen_levels": 2})],
}
# square sizes at which Router.calibrate times every candidate
CAL_SIZES = (32, 64, 128, 256, 512, 1024, 2048, 4096)


def tol_class(tol: float) -> str:
    return "fp64" if tol < 1e-12 else "relaxed"


def _kw(name: str) -> dict:
    for cands in CANDIDATES.values():
        for n, m, kw in cands:
            if n == name:
                return kw
    raise KeyError(name)


def _method(name: str) -> str:
    for cands in CANDIDATES.values():
        for n, m, kw in cands:
            if n == name:
                return m
    raise KeyError(name)


class Router:
    """Method choice by measured cost.  ``table[name]`` holds the measured
    time (ms) of candidate ``name`` on square products of the sizes in
    ``sizes``; a request (N, P, M) is priced at the size d = (N P M)^(1/3)
    by interpolating the time per multiply-add (log-linear in d) and scaling
    by N P M.  The fastest candidate of the request's tolerance class wins.
    The choice depends on the request alone.  Without a table the rule of
    thumb is DGEMM below d = 1024 and the byte-digit int8 split above."""

    def __init__(self, table: Optional[Dict[str, List[float]]] = None, sizes: Sequence[int] = CAL_SIZES):
        self._sizes = list(sizes)
        self.table = dict(table or {})

    @property
    def table(self) -> Dict[str, List[float]]:
        return self._table

    @table.setter
    def table(self, table: Dict[str, List[float]]) -> None:
        self._table = table
        self._reprice()

    @property
    def sizes(self) -> List[int]:
        return self._sizes

    @sizes.setter
    def sizes(self, sizes: Sequence[int]) -> None:
        self._sizes = list(sizes)
        self._reprice()

    def _reprice(self) -> None:
        # the per-size terms of the pricing, formed once whenever the table or
        # the sizes are assigned (the same values cost_ms would form on every
        # call); a table changed in place must be assigned again
        self._xs = [math.log(s) for s in self._sizes]
        self._per = {n: [t / float(s) ** 3 for t, s in zip(ms, self._sizes)] for n, ms in self._table.items()}
        self._lper = {n: [math.log(v) for v in per] for n, per in self._per.items()}

    # -- pricing ---------------------------------------------------------------
    def cost_ms(self, name: str, N: int, P: int, M: int) -> float:
        ms = self._table[name]
        per = self._per[name]  # ms per multiply-add at each size
        xs = self._xs
        macs = float(N) * P * M
        d = macs ** (1.0 / 3.0)
        x = math.log(max(d, 1.0))
        if x <= xs[0]:
            # below the smallest size the time is launch-bound: no less than there
            return max(per[0] * macs, ms[0])
        if x >= xs[-1]:
            return per[-1] * macs
        k = bisect.bisect_right(xs, x) - 1
        w = (x - xs[k]) / (xs[k + 1] - xs[k])
        lper = self._lper[name]
        lp = (1 - w) * lper[k] + w * lper[k + 1]
        return math.exp(lp) * macs

    def choose(self, N: int, P: int, M: int, tol: float) -> Tuple[str, Config]:
        cands = CANDIDATES[tol_class(tol)]
        priced = [(self.cost_ms(n, N, P, M), n) for n, _, _ in cands if n in self.table]
        if priced:
            name = min(priced)[1]
        else:
            name = cands[0][0]
            if min(N, P, M) >= 1024:
                name = "split_int8_b8_s6" if tol_class(tol) == "fp64" else "split_int8_b8_s5"
        return _method(name), Config(**_kw(name))

    # -- measurement -----------------------------------------------------------
    def calibrate(self, device: int = 0, reps: int = 3) -> Dict[str, List[float]]:
        """Time every candidate on square products of the calibration sizes
        (median of ``reps`` launches, HIP events on one stream)."""
        dev = torch.device("cuda", device)
        stream = torch.cuda.current_stream(dev)
        names = sorted({n for cands in CANDIDATES.values() for n, _, _ in cands})
        table = {n: [] for n in names}
        for s in self.sizes:
            A = torch.rand((s, s), dtype=torch.float64, device=dev) * 2 - 1
            B = torch.rand((s, s), dtype=torch.float64, device=dev) * 2 - 1
            C = torch.empty((s, s), dtype=torch.float64, device=dev)
            for n in names:
                cfg = Config(**_kw(n))
                m = _method(n)
                ws = torch.empty(max(workspace_bytes(m, s, s, s, cfg), 1), dtype=torch.uint8, device=dev)
                multiply(A, B, m, cfg, out=C, workspace=ws, stream=stream)
                times = []
                for _ in range(reps):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    multiply(A, B, m, cfg, out=C, workspace=ws, stream=stream)
                    e1.record(stream)
                    e1.synchronize()
                    times.append(e0.elapsed_time(e1))
                table[n].append(sorted(times)[len(times) // 2])
                del ws
            del A, B, C
        self.table = table
        return table

    def save(self, path: str) -> None:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump({"sizes": self.sizes, "ms": self.table}, f, indent=1, sort_keys=True)

    @classmethod
    def load(cls, path: str) -> "Router":
        with open(path) as f:
            doc = json.load(f)
        return cls(doc["ms"], doc["sizes"])


_DEFAULT_ROUTER = Router()


def choose(N: int, P: int, M: int, tol: float):
    """Method and config for a request by the uncalibrated rule."""
    return _DEFAULT_ROUTER.choose(N, P, M, tol)


class Admission:
    """Admission bookkeeping (pure host logic).  Requests wait in arrival
    order; a request is admitted when a stream slot is free and its
    footprint fits the unused part of the budget.  A later request that fits
    may pass an earlier one that does not, unless the oldest waiting request
    has waited at least ``max_wait_s`` (on ``clock``): then admission stops
    at it until it fits, so its wait is bounded by ``max_wait_s`` plus the
    time the work in flight takes to free the budget it needs."""

    def __init__(self, budget: int, slots: int, max_wait_s: float = 0.05,
                 clock: Callable[[], float] = time.perf_counter):
        self.budget = int(budget)
        self.free_slots = collections.deque(range(slots))
        self.used = 0
        self.peak_used = 0
        self.waiting = collections.deque()
        self.max_wait_s = max_wait_s
        self.clock = clock

    def push(self, req) -> None:
        if req.footprint > self.budget:
            raise ValueError("request footprint %d exceeds the HBM budget %d" % (req.footprint, self.budget))
        self.waiting.append(req)

    def admit(self):
        if not self.free_slots:  # nothing can be admitted; skip the scan of the queue
            return []
        now = self.clock()
        out, keep = [], collections.deque()
        blocked = False
        while self.waiting:
            r = self.waiting.popleft()
            if not blocked and self.free_slots and self.used + r.footprint <= self.budget:
                self.used += r.footprint
                self.peak_used = max(self.peak_used, self.used)
                r.slot = self.free_slots.popleft()
                out.append(r)
            else:
                keep.append(r)
                # an aged request that cannot go yet holds back everything after it
                if not blocked and now - r.arrival >= self.max_wait_s:
                    blocked = True
        self.waiting = keep
        return out

    def release(self, req) -> None:
        self.used -= req.footprint
        self.free_slots.append(req.slot)


@dataclasses.dataclass
class Request:
    rid: int
    A: Optional[torch.Tensor]
    B: Optional[torch.Tensor]
    tol: float
    arrival: float
    future: Future
    method: str = ""
    cfg: Optional[Config] = None
    footprint: int = 0
    ws_bytes: int = 0  # workspace of the chosen method (part of the footprint)
    slot: int = -1
    C: Optional[torch.Tensor] = None
    ws: Optional[torch.Tensor] = None
    done_event: Optional[torch.cuda.Event] = None
    admitted: float = 0.0
    completed: float = 0.0
    shape: Tuple[int, int, int] = (0, 0, 0)


# What a finished request leaves behind for stats(): no tensors.
Record = collections.namedtuple("Record", "rid arrival admitted completed N P M method tol")


class _Done:
    """Completion marker of the host-only (device "cpu") test mode."""

    def query(self):
        return True


class Server:
    """The request loop.  ``launch`` is the function that enqueues one
    product (the library's ``multiply``).  ``device`` is a GPU index; the
    device "cpu" runs the same scheduler without streams or events, for host
    tests with a stub ``launch``."""

    def __init__(self, budget_bytes: int, streams: int = 4, device=0, poll_s: float = 20e-6,
                 router: Optional[Router] = None, max_wait_s: float = 0.05, launch: Callable = multiply):
        self.device = torch.device(device) if isinstance(device, (str, torch.device)) else torch.device("cuda", device)
        self.gpu = self.device.type == "cuda"
        self.streams = [torch.cuda.Stream(device=self.device) if self.gpu else None for _ in range(streams)]
        self.adm = Admission(budget_bytes, streams, max_wait_s=max_wait_s)
        self.router = router or _DEFAULT_ROUTER
        self.launch = launch
        self.poll_s = poll_s
        self.inflight = []
        self.done: List[Record] = []
        self.failed = 0
        self.lock = threading.Lock()
        self.wake = threading.Event()
        self.stopping = False
        self.next_id = 0
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    # -- client side ---------------------------------------------------------
    def submit(self, A: torch.Tensor, B: torch.Tensor, tol: float = 1e-13) -> Future:
        """Queue C = A B.  A and B are contiguous float64 matrices resident on
        this server's GPU, finished on the default stream (or synchronised)
        before the call.  Malformed operands raise here, before queueing."""
        for name, X in (("A", A), ("B", B)):
            if not isinstance(X, torch.Tensor) or X.dim() != 2:
                raise ValueError("%s must be a 2-D tensor" % name)
            if X.dtype != torch.float64:
                raise TypeError("%s must be float64, got %s" % (name, X.dtype))
            if X.device != self.device:
                raise ValueError("%s must live on %s, got %s" % (name, self.device, X.device))
            if not X.is_contiguous():
                raise ValueError("%s must be contiguous (row-major)" % name)
        N, P = A.shape
        if B.shape[0] != P:
            raise ValueError("inner dimensions differ: A is %dx%d, B is %dx%d" % (N, P, B.shape[0], B.shape[1]))
        M = B.shape[1]
        method, cfg = self.router.choose(N, P, M, tol)
        ws = workspace_bytes(method, N, P, M, cfg)
        fp = 8 * (N * P + P * M + N * M) + ws
        fut = Future()
        with self.lock:
            r = Request(self.next_id, A, B, tol, self.adm.clock(), fut, method, cfg, fp, ws, shape=(N, P, M))
            self.adm.push(r)
            self.next_id += 1
        self.wake.set()
        return fut

    def close(self):
        self.stopping = True
        self.wake.set()
        self.thread.join()

    # -- scheduler -----------------------------------------------------------
    def _fail(self, r, exc):
        with self.lock:
            self.adm.release(r)
        r.A = r.B = r.C = r.ws = None
        self.failed += 1
        r.future.set_exception(exc)

    def _admit(self):
        with self.lock:
            admitted = self.adm.admit()
        for r in admitted:
            s = self.streams[r.slot]
            try:
                with torch.cuda.stream(s):
                    N, P, M = r.shape
                    r.C = torch.empty((N, M), dtype=torch.float64, device=self.device)
                    r.ws = torch.empty(max(r.ws_bytes, 1), dtype=torch.uint8, device=self.device)
                    if self.gpu:
                        # the operands were produced on other streams: order this stream after them
                        s.wait_stream(torch.cuda.default_stream(self.device))
                    self.launch(r.A, r.B, r.method, r.cfg, out=r.C, workspace=r.ws, stream=s)
                    if self.gpu:
                        r.done_event = torch.cuda.Event()
                        r.done_event.record(s)
                    else:
                        r.done_event = _Done()
            except Exception as exc:  # keep serving the other requests
                self._fail(r, exc)
                continue
            r.admitted = self.adm.clock()
            self.inflight.append(r)

    def _retire(self):
        still = []
        for r in self.inflight:
            if r.done_event.query():
                r.completed = self.adm.clock()
                with self.lock:
                    self.adm.release(r)
                C = r.C
                N, P, M = r.shape
                self.done.append(Record(r.rid, r.arrival, r.admitted, r.completed, N, P, M, r.method, r.tol))
                r.A = r.B = r.C = r.ws = r.done_event = None
                r.future.set_result(C)
            else:
                still.append(r)
        self.inflight = still

    def _loop(self):
        if self.gpu:
            torch.cuda.set_device(self.device)
        while True:
            self.wake.clear()  # a submit after this point wakes the wait below
            try:
                self._retire()
                self._admit()
            except Exception as exc:  # a bookkeeping failure: fail what is pending, keep no future open
                with self.lock:
                    pending = list(self.adm.waiting)
                    self.adm.waiting.clear()
                for r in pending:
                    r.future.set_exception(exc)
            with self.lock:
                idle = not self.adm.waiting
            if self.stopping and not self.inflight and idle:
                break
            if not self.inflight and idle:
                self.wake.wait(0.01)
            else:
                time.sleep(self.poll_s)

    # -- report --------------------------------------------------------------
    def stats(self):
        recs = self.done
        lat = sorted(r.completed - r.arrival for r in recs)
        if not lat:
            return {}
        first = min(r.arrival for r in recs)
        last = max(r.completed for r in recs)
        flop = sum(2.0 * r.N * r.P * r.M for r in recs)

        def pct(p):
            return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]

        methods = collections.Counter(r.method for r in recs)
        return {"requests": len(lat), "failed": self.failed, "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99),
                "max_ms": 1e3 * lat[-1], "mean_ms": 1e3 * sum(lat) / len(lat), "req_per_s": len(lat) / (last - first),
                "tflops": flop / (last - first) / 1e12, "peak_budget_used": self.adm.peak_used,
                "methods": dict(methods)}
