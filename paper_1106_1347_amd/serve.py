"""Continuous-batching request loop for C = AB on one GPU.

Requests (A, B, tolerance) arrive at any time.  A scheduler thread admits
waiting requests in arrival order whenever their HBM footprint (operands,
result and workspace) fits the free part of the budget and a stream slot is
free, enqueues each admitted product on its own stream from a pool, and
retires products as their completion events fire, freeing their memory for
the next admissions.  Work of different requests therefore overlaps on the
device while new requests keep being admitted.

Each request is computed by a method chosen from its own tolerance and
shape only (``choose``), with no cross-request reduction, so its result is
bit for bit the same alone and in any mix.

Latency of a request = completion time (its completion event observed by
the scheduler) - arrival time (``submit``), on the host clock.
"""
import collections
import dataclasses
import threading
import time
from concurrent.futures import Future
from typing import Optional

import torch

from ._lib import Config, multiply, workspace_bytes


def choose(N: int, P: int, M: int, tol: float):
    """Method and config for a request.  The split product (int8 digits)
    beats FP64 DGEMM once the product is large enough to amortise digit
    extraction; 7 digits give FP64-grade results (<= 1e-13 relative
    infinity-norm error), 5 digits suffice for 1e-10."""
    big = min(N, P, M) >= 1024
    if tol < 1e-12:
        return ("split", Config(split_type="int8", split_slices=7)) if big else ("dgemm", Config())
    return ("split", Config(split_type="int8", split_slices=5)) if big else ("dgemm", Config())


class Admission:
    """Admission bookkeeping (pure host logic): requests wait in arrival
    order; a request is admitted when a stream slot is free and its
    footprint fits the unused part of the budget.  Later requests that fit
    may pass an earlier one that does not (no head-of-line blocking)."""

    def __init__(self, budget: int, slots: int):
        self.budget = int(budget)
        self.free_slots = collections.deque(range(slots))
        self.used = 0
        self.peak_used = 0
        self.waiting = collections.deque()

    def push(self, req) -> None:
        if req.footprint > self.budget:
            raise ValueError("request footprint %d exceeds the HBM budget %d" % (req.footprint, self.budget))
        self.waiting.append(req)

    def admit(self):
        out, keep = [], collections.deque()
        while self.waiting:
            r = self.waiting.popleft()
            if self.free_slots and self.used + r.footprint <= self.budget:
                self.used += r.footprint
                self.peak_used = max(self.peak_used, self.used)
                r.slot = self.free_slots.popleft()
                out.append(r)
            else:
                keep.append(r)
        self.waiting = keep
        return out

    def release(self, req) -> None:
        self.used -= req.footprint
        self.free_slots.append(req.slot)


@dataclasses.dataclass
class Request:
    rid: int
    A: torch.Tensor
    B: torch.Tensor
    tol: float
    arrival: float
    future: Future
    method: str = ""
    cfg: Optional[Config] = None
    footprint: int = 0
    slot: int = -1
    C: Optional[torch.Tensor] = None
    ws: Optional[torch.Tensor] = None
    done_event: Optional[torch.cuda.Event] = None
    admitted: float = 0.0
    completed: float = 0.0


class Server:
    def __init__(self, budget_bytes: int, streams: int = 4, device: int = 0, poll_s: float = 20e-6):
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.adm = Admission(budget_bytes, streams)
        self.poll_s = poll_s
        self.inflight = []
        self.done = []
        self.lock = threading.Lock()
        self.wake = threading.Event()
        self.stopping = False
        self.next_id = 0
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    # -- client side ---------------------------------------------------------
    def submit(self, A: torch.Tensor, B: torch.Tensor, tol: float = 1e-13) -> Future:
        """Queue C = A B.  A and B are float64 tensors resident on this GPU,
        finished on the default stream (or synchronised) before the call."""
        N, P = A.shape
        M = B.shape[1]
        method, cfg = choose(N, P, M, tol)
        fp = 8 * (N * P + P * M + N * M) + workspace_bytes(method, N, P, M, cfg)
        fut = Future()
        with self.lock:
            r = Request(self.next_id, A, B, tol, time.perf_counter(), fut, method, cfg, fp)
            self.adm.push(r)
            self.next_id += 1
        self.wake.set()
        return fut

    def close(self):
        self.stopping = True
        self.wake.set()
        self.thread.join()

    # -- scheduler -----------------------------------------------------------
    def _admit(self):
        with self.lock:
            admitted = self.adm.admit()
        for r in admitted:
            s = self.streams[r.slot]
            with torch.cuda.stream(s):
                N, P = r.A.shape
                M = r.B.shape[1]
                r.C = torch.empty((N, M), dtype=torch.float64, device=self.device)
                need = workspace_bytes(r.method, N, P, M, r.cfg)
                r.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)
                # the operands were produced on other streams: order this stream after them
                s.wait_stream(torch.cuda.default_stream(self.device))
                multiply(r.A, r.B, r.method, r.cfg, out=r.C, workspace=r.ws, stream=s)
                r.done_event = torch.cuda.Event()
                r.done_event.record(s)
            r.admitted = time.perf_counter()
            self.inflight.append(r)

    def _retire(self):
        still = []
        for r in self.inflight:
            if r.done_event.query():
                r.completed = time.perf_counter()
                with self.lock:
                    self.adm.release(r)
                r.ws = None
                self.done.append(r)
                r.future.set_result(r.C)
            else:
                still.append(r)
        self.inflight = still

    def _loop(self):
        torch.cuda.set_device(self.device)
        while True:
            self.wake.clear()  # a submit after this point wakes the wait below
            self._retire()
            self._admit()
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
        lat = sorted(r.completed - r.arrival for r in self.done)
        if not lat:
            return {}
        first = min(r.arrival for r in self.done)
        last = max(r.completed for r in self.done)
        flop = sum(2.0 * r.A.shape[0] * r.A.shape[1] * r.B.shape[1] for r in self.done)

        def pct(p):
            return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]

        return {"requests": len(lat), "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "max_ms": 1e3 * lat[-1],
                "mean_ms": 1e3 * sum(lat) / len(lat), "req_per_s": len(lat) / (last - first),
                "tflops": flop / (last - first) / 1e12, "peak_budget_used": self.adm.peak_used}
