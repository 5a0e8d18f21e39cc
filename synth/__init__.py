"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws numbers: it holds none of the arithmetic of any
multiplication method, so both the GPU library's tests and the CPU oracle
can take their inputs from it without sharing code with each other.

Every generator uses numpy's PCG64 (``numpy.random.default_rng(seed)``).
Workload seeds: configuration ``c`` uses ``1000*c + 1`` for A and
``1000*c + 2`` for B; item ``g`` of a batch or request stream uses
``1000*c + 10 + 2*g`` and ``1000*c + 11 + 2*g``.
"""
import math

import numpy as np


def seed_a(cfg: int) -> int:
    return 1000 * cfg + 1


def seed_b(cfg: int) -> int:
    return 1000 * cfg + 2


def seed_item(cfg: int, g: int, which: str) -> int:
    return 1000 * cfg + (10 if which == "A" else 11) + 2 * g


def uniform(shape, seed, lo=-1.0, hi=1.0):
    """Entries i.i.d. uniform on [lo, hi) in float64."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def integers(shape, seed, lo=-8, hi=8):
    """Integer-valued float64 entries, uniform on {lo, ..., hi}."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=shape).astype(np.float64)


def wide_range(shape, seed, u_max=20.0, v_max=10):
    """Entries  (+-1) * 2^u  with u ~ U[-u_max, u_max] continuous (full 53-bit
    significands), every row then multiplied by 2^v with v ~ U{-v_max..v_max}
    (an exact scaling).  The distribution of the split-precision workload."""
    rng = np.random.default_rng(seed)
    rows, cols = shape
    sign = np.where(rng.random(size=shape) < 0.5, -1.0, 1.0)
    u = rng.uniform(-u_max, u_max, size=shape)
    v = rng.integers(-v_max, v_max + 1, size=(rows, 1))
    return np.ldexp(sign * np.exp2(u), v)


def paper_test_pair(n, seed):
    """The paper's test workload (Tests section): A an n x n random matrix and
    B = 8A.  The paper does not state the distribution; uniform [0, 1) is
    used."""
    A = np.random.default_rng(seed).random(size=(n, n))
    return A, 8.0 * A


def batch_shapes(count, seed, lo=16, hi=512):
    """(N, P, M) triples, each dimension uniform on {lo, ..., hi}."""
    rng = np.random.default_rng(seed)
    return [tuple(int(x) for x in rng.integers(lo, hi + 1, size=3)) for _ in range(count)]


def serving_requests(count, seed, rate_per_s, lo=32, hi=4096, tolerances=(1e-13, 1e-10)):
    """A Poisson request stream.  Half of the requests are square (one
    log-uniform draw on [lo, hi]), half rectangular (three independent
    draws); each carries an error tolerance drawn from ``tolerances`` with
    equal probability.  Returns a list of dicts with arrival time (s),
    shape and tolerance."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for g in range(count):
        t += rng.exponential(1.0 / rate_per_s)
        if rng.random() < 0.5:
            d = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            shape = (d, d, d)
        else:
            shape = tuple(int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(3))
        tol = tolerances[int(rng.integers(0, len(tolerances)))]
        out.append({"id": g, "arrival_s": t, "shape": shape, "tol": tol})
    return out
