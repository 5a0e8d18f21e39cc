"""Serving loop host logic: admission under a fake HBM budget and a fake
clock (the aging bound), method routing by a measured-cost table, and
failure handling with a stub launch (no GPU)."""
import types

import numpy as np
import pytest
import torch

from paper_1106_1347_amd.serve import CANDIDATES, Admission, Router, Server, choose


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def req(fp, rid, arrival=0.0):
    return types.SimpleNamespace(footprint=fp, rid=rid, slot=-1, arrival=arrival)


def test_admission_respects_budget_and_slots():
    a = Admission(budget=100, slots=2, max_wait_s=1e9)
    for i, fp in enumerate([60, 30, 50, 10]):
        a.push(req(fp, i))
    first = a.admit()
    # 60 and 30 fit (90 <= 100); slots are then exhausted
    assert [r.rid for r in first] == [0, 1] and a.used == 90
    assert [r.rid for r in a.waiting] == [2, 3]
    a.release(first[0])
    # 50 fits next to 30 (80 <= 100); 10 has no slot
    second = a.admit()
    assert [r.rid for r in second] == [2] and a.used == 80
    a.release(first[1])
    third = a.admit()
    assert [r.rid for r in third] == [3] and a.used == 60
    assert a.peak_used == 90


def test_no_head_of_line_blocking_before_the_bound():
    clk = FakeClock()
    a = Admission(budget=100, slots=4, max_wait_s=1.0, clock=clk)
    a.push(req(90, 0))
    a.admit()
    a.push(req(50, 1, arrival=0.0))  # does not fit yet
    a.push(req(10, 2, arrival=0.0))  # fits
    clk.t = 0.5
    got = a.admit()
    assert [r.rid for r in got] == [2]
    assert [r.rid for r in a.waiting] == [1]


def _small_stream_with_one_large(max_wait_s, steps=400):
    # Small requests (footprint 30 of 100) arrive every 0.25 time units and
    # each holds the budget for 1 unit after admission; they are started
    # 0.25 apart, so at most one finishes per step.  A large request (60)
    # arrives at t = 0.5 with 90 in use.  Returns (large request, admission
    # time or None, number of small requests admitted while it waited).
    clk = FakeClock()
    a = Admission(budget=100, slots=8, max_wait_s=max_wait_s, clock=clk)
    inflight = []  # (finish time, request)
    big = req(60, "big", arrival=0.5)
    admitted_big, passed, rid = None, 0, 0
    for step in range(steps):
        clk.t = step * 0.25
        for fin, r in list(inflight):
            if fin <= clk.t:
                a.release(r)
                inflight.remove((fin, r))
        a.push(req(30, rid, clk.t))
        rid += 1
        if step == 2:
            a.push(big)
        for r in a.admit():
            if r is big:
                admitted_big = clk.t
            elif step >= 2 and admitted_big is None:
                passed += 1
            inflight.append((clk.t + 1.0, r))
        assert a.used <= a.budget
        if admitted_big is not None:
            break
    return big, admitted_big, passed


def test_aging_bound_holds_under_a_stream_of_small_requests():
    # Without the bound the small requests pass the large one forever (the
    # budget never drops to 40); with max_wait_s = 2 it is admitted no later
    # than 2 + 1 (the longest time the work in flight holds the budget)
    # after its arrival, and smaller later requests still passed it before.
    big, t, passed = _small_stream_with_one_large(max_wait_s=1e9)
    assert t is None and passed > 100
    big, t, passed = _small_stream_with_one_large(max_wait_s=2.0)
    assert t is not None, "the large request starved"
    assert t <= big.arrival + 2.0 + 1.0
    assert passed >= 4


def test_oversized_request_rejected():
    a = Admission(budget=10, slots=1)
    with pytest.raises(ValueError):
        a.push(req(11, 0))


def test_method_choice_by_tolerance_uncalibrated():
    assert choose(4096, 4096, 4096, 1e-13)[0] == "split"
    assert (choose(4096, 4096, 4096, 1e-13)[1].split_slices, choose(4096, 4096, 4096, 1e-13)[1].split_bits) == (6, 8)
    assert (choose(4096, 4096, 4096, 1e-10)[1].split_slices, choose(4096, 4096, 4096, 1e-10)[1].split_bits) == (5, 8)
    assert choose(100, 4096, 4096, 1e-13)[0] == "dgemm"


def test_router_prices_by_measured_table():
    sizes = [32, 256, 2048]
    names = {n for c in CANDIDATES.values() for n, _, _ in c}
    # dgemm: 1 ms at 2048; split: cheaper only at the largest size; Strassen slowest
    table = {n: [0.01, 0.05, 10.0] for n in names}
    table["dgemm"] = [0.005, 0.02, 2.0]
    table["split_int8_s7"] = [0.05, 0.2, 1.5]
    table["split_int8_s5"] = [0.04, 0.15, 1.2]
    r = Router(table, sizes)
    assert r.choose(2048, 2048, 2048, 1e-13)[0] == "split"
    assert r.choose(256, 256, 256, 1e-13)[0] == "dgemm"
    assert r.choose(2048, 2048, 2048, 1e-10) == ("split", r.choose(4096, 4096, 4096, 1e-10)[1])
    assert r.choose(2048, 2048, 2048, 1e-10)[1].split_slices == 5
    # interpolation: the price grows with the work and is never below the smallest size's time
    assert r.cost_ms("dgemm", 16, 16, 16) == pytest.approx(0.005)
    assert r.cost_ms("dgemm", 512, 512, 512) < r.cost_ms("dgemm", 1024, 1024, 1024)
    assert r.cost_ms("dgemm", 2048, 2048, 2048) == pytest.approx(2.0)
    assert r.cost_ms("dgemm", 4096, 4096, 4096) == pytest.approx(16.0)
    # the choice depends on the request only: repeated calls agree
    assert all(r.choose(300, 700, 900, 1e-10) == r.choose(300, 700, 900, 1e-10) for _ in range(3))


def _price_by_definition(sizes, ms, N, P, M):
    # time per multiply-add interpolated linearly in log d between the measured
    # sizes (d = (N P M)^(1/3)), times N P M; below the smallest size no less than
    # its measured time, above the largest its time per multiply-add
    macs = float(N) * P * M
    d = max(macs ** (1.0 / 3.0), 1.0)
    per = np.array(ms) / np.array(sizes, dtype=np.float64) ** 3
    if d <= sizes[0]:
        return max(per[0] * macs, ms[0])
    if d >= sizes[-1]:
        return per[-1] * macs
    return float(np.exp(np.interp(np.log(d), np.log(sizes), np.log(per)))) * macs


def test_router_prices_follow_the_definition_after_any_assignment():
    rng = np.random.default_rng(7)
    names = sorted({n for c in CANDIDATES.values() for n, _, _ in c})
    sizes = [32, 128, 512, 2048, 8192]
    table = {n: sorted(rng.uniform(0.004, 40.0, len(sizes)).tolist()) for n in names}
    r = Router(table, sizes)
    shapes = [tuple(int(x) for x in rng.integers(1, 12000, 3)) for _ in range(400)] + [(1, 1, 1), (8192, 8192, 8192)]
    for stage in range(3):
        if stage == 1:
            # new sizes for the same table: every price follows them
            sizes = [64, 256, 1024, 4096, 16384]
            r.sizes = sizes
        if stage == 2:
            table = {n: sorted(rng.uniform(0.004, 40.0, len(sizes)).tolist()) for n in names}
            r.table = table
        for n in names:
            for (N, P, M) in shapes:
                assert r.cost_ms(n, N, P, M) == pytest.approx(_price_by_definition(sizes, table[n], N, P, M),
                                                              rel=1e-12), (stage, n, N, P, M)


def test_router_table_round_trip(tmp_path):
    r = Router({"dgemm": [1.0, 2.0]}, [64, 128])
    p = tmp_path / "router.json"
    r.save(str(p))
    q = Router.load(str(p))
    assert q.table == r.table and q.sizes == r.sizes


def _cpu_server(launch, budget=1 << 30):
    return Server(budget, streams=2, device="cpu", launch=launch, max_wait_s=1.0)


def test_failed_launch_resolves_its_future_and_frees_the_budget():
    calls = []

    def launch(A, B, method, cfg, out, workspace, stream):
        calls.append(A.shape)
        if A.shape[0] == 3:
            raise RuntimeError("planted launch failure")
        out.zero_()

    srv = _cpu_server(launch)
    ok1 = srv.submit(torch.ones(2, 4, dtype=torch.float64), torch.ones(4, 5, dtype=torch.float64))
    bad = srv.submit(torch.ones(3, 4, dtype=torch.float64), torch.ones(4, 5, dtype=torch.float64))
    ok2 = srv.submit(torch.ones(4, 4, dtype=torch.float64), torch.ones(4, 5, dtype=torch.float64))
    assert ok1.result(timeout=10).shape == (2, 5)
    with pytest.raises(RuntimeError, match="planted"):
        bad.result(timeout=10)
    assert ok2.result(timeout=10).shape == (4, 5)
    srv.close()
    st = srv.stats()
    assert st["requests"] == 2 and st["failed"] == 1
    assert srv.adm.used == 0 and sorted(srv.adm.free_slots) == [0, 1]
    # finished requests keep no tensors
    assert all(not any(isinstance(v, torch.Tensor) for v in rec) for rec in srv.done)


def test_submit_rejects_malformed_operands():
    srv = _cpu_server(lambda *a, **k: None)
    A = torch.ones(3, 4, dtype=torch.float64)
    with pytest.raises(TypeError):
        srv.submit(A.float(), torch.ones(4, 2, dtype=torch.float64))
    with pytest.raises(ValueError):
        srv.submit(A, torch.ones(5, 2, dtype=torch.float64))
    with pytest.raises(ValueError):
        srv.submit(A.t(), torch.ones(3, 2, dtype=torch.float64))
    with pytest.raises(ValueError):
        srv.submit(torch.ones(4, dtype=torch.float64), torch.ones(4, 2, dtype=torch.float64))
    srv.close()
    assert srv.adm.used == 0 and not srv.adm.waiting
