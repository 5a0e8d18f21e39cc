"""Admission logic of the serving loop with a fake HBM budget (host only)."""
import types

import pytest

from paper_1106_1347_amd.serve import Admission, choose


def req(fp, rid):
    return types.SimpleNamespace(footprint=fp, rid=rid, slot=-1)


def test_admission_respects_budget_and_slots():
    a = Admission(budget=100, slots=2)
    for i, fp in enumerate([60, 30, 50, 10]):
        a.push(req(fp, i))
    first = a.admit()
    # 60 and 30 fit (90 <= 100); slots are then exhausted
    assert [r.rid for r in first] == [0, 1] and a.used == 90
    assert [r.rid for r in a.waiting] == [2, 3]
    a.release(first[0])
    # 50 does not fit next to 30 (80 <= 100 does): admitted; 10 has no slot
    second = a.admit()
    assert [r.rid for r in second] == [2] and a.used == 80
    a.release(first[1])
    third = a.admit()
    assert [r.rid for r in third] == [3] and a.used == 60
    assert a.peak_used == 90


def test_no_head_of_line_blocking():
    a = Admission(budget=100, slots=4)
    a.push(req(90, 0))
    a.admit()
    a.push(req(50, 1))  # does not fit yet
    a.push(req(10, 2))  # fits
    got = a.admit()
    assert [r.rid for r in got] == [2]
    assert [r.rid for r in a.waiting] == [1]


def test_oversized_request_rejected():
    a = Admission(budget=10, slots=1)
    with pytest.raises(ValueError):
        a.push(req(11, 0))


def test_method_choice_by_tolerance():
    assert choose(4096, 4096, 4096, 1e-13)[0] == "split"
    assert choose(4096, 4096, 4096, 1e-13)[1].split_slices == 7
    assert choose(4096, 4096, 4096, 1e-10)[1].split_slices == 5
    assert choose(100, 4096, 4096, 1e-13)[0] == "dgemm"
