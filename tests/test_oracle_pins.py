"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something the paper or mathematics
fixes: products of integer-valued matrices (exact in binary64), identity and
permutation matrices, brute force against exact rationals with textbook
rounding-error bounds, Brent's bound (Section 2.3.2), the embedding rule of
Section 2.4.1 worked by hand, the printed error tables of the Tests section,
and a brute-force search for the scaling exponent of Section 2.3.2.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53

SHAPES = [(1, 1, 1), (1, 7, 1), (3, 5, 7), (8, 8, 8), (16, 17, 18), (33, 64, 31), (40, 33, 50),
          (64, 65, 64), (2, 1, 3), (5, 2, 4)]


def _int_pair(shape, seed, lo=-8, hi=8):
    N, P, M = shape
    return synth.integers((N, P), seed, lo, hi), synth.integers((P, M), seed + 1, lo, hi)


def _exact(A, B):
    return (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)


def _methods(orc):
    out = {
        "naive": orc.naive,
        "kahan": orc.kahan,
        "winograd": orc.winograd,
        "winograd_scaled": orc.winograd_scaled,
        "naive_on_array": orc.naive_on_array,
        "dot2": orc.dot2,
        "unroll2": lambda A, B: orc.naive_unroll(A, B, 2),
        "unroll3": lambda A, B: orc.naive_unroll(A, B, 3),
        "unroll4": lambda A, B: orc.naive_unroll(A, B, 4),
        "split_bf16_s1": lambda A, B: orc.split_model(A, B, 1, 8),
        "split_bf16_s6": lambda A, B: orc.split_model(A, B, 6, 8),
        "split_fp16_s4": lambda A, B: orc.split_model(A, B, 4, 10),
        "split_int8_s7": lambda A, B: orc.split_model(A, B, 7, 7),
        "split_int8_bytes_s6": lambda A, B: orc.split_model(A, B, 6, 8, rule=1),
        "split_int8_bytes_s1": lambda A, B: orc.split_model(A, B, 1, 8, rule=1),
    }
    for v, name in ((0, "sn"), (1, "sw")):
        out[name + "_paper"] = (lambda v: lambda A, B: orc.strassen(A, B, v, orc.MODE_PAPER))(v)
        for L in (0, 1, 2, 3):
            out["%s_L%d" % (name, L)] = (lambda v, L: lambda A, B: orc.strassen(A, B, v, orc.MODE_LEVELS,
                                                                               L))(v, L)
    return out


@pytest.mark.parametrize("shape", SHAPES)
def test_integer_products_are_exact(orc, shape):
    """Integer entries in {-8..8}: every intermediate of every method is an
    integer far below 2^53 (split digits below 2^24), so each method must
    return the exact product bit for bit."""
    A, B = _int_pair(shape, 7 + sum(shape))
    ref = _exact(A, B)
    for name, f in _methods(orc).items():
        C = f(A, B)
        assert np.array_equal(C, ref), name


def test_integer_products_exact_wide_entries(orc):
    """Larger integers (|a| <= 1000) still give exact products; the split
    model then needs several digits, which exercises the digit recursion."""
    A, B = _int_pair((24, 37, 19), 99, -1000, 1000)
    ref = _exact(A, B)
    for name in ("naive", "kahan", "winograd", "winograd_scaled", "sn_L2", "sw_L2", "sw_paper"):
        assert np.array_equal(_methods(orc)[name](A, B), ref), name
    # two digits hold each entry exactly; the product of the two second
    # digits (t + u = 4) is kept only from s = 3 on
    assert np.array_equal(orc.split_model(A, B, 3, 8), ref)
    assert np.array_equal(orc.split_model(A, B, 3, 7), ref)
    assert not np.array_equal(orc.split_model(A, B, 2, 8), ref)
    assert not np.array_equal(orc.split_model(A, B, 1, 8), ref)


def test_identity_and_permutation(orc):
    rng = np.random.default_rng(5)
    A = synth.uniform((13, 21), 3)
    I = np.eye(21)
    perm = rng.permutation(21)
    Pm = np.eye(21)[:, perm]  # column permutation matrix
    for f in (orc.naive, orc.kahan):
        assert np.array_equal(f(A, I), A)
        assert np.array_equal(f(A, Pm), A[:, perm])
        assert np.array_equal(f(np.eye(13), A), A)


def test_bruteforce_tiny_against_rationals(orc):
    """All N, P, M in 1..5 with random doubles: NaivStandard obeys the
    textbook bound |C^ - C| <= gamma_P |A||B| elementwise (gamma_P =
    P u / (1 - P u)); Kahan obeys the compensated-sum bound
    (3u + 2 P u^2) sum_k |a_ik b_kj| + u|c_ij|."""
    rng = np.random.default_rng(11)
    for N in range(1, 6):
        for P in range(1, 6):
            for M in range(1, 6):
                A = rng.uniform(-1, 1, (N, P)) * 2.0 ** rng.integers(-3, 4, (N, P))
                B = rng.uniform(-1, 1, (P, M)) * 2.0 ** rng.integers(-3, 4, (P, M))
                Cn, Ck = orc.naive(A, B), orc.kahan(A, B)
                g = P * U / (1 - P * U)
                for i in range(N):
                    for j in range(M):
                        ex = sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(P))
                        ab = sum(abs(Fraction(A[i, k]) * Fraction(B[k, j])) for k in range(P))
                        assert abs(Fraction(Cn[i, j]) - ex) <= Fraction(g) * ab
                        kb = Fraction(3 * U + 2 * P * U * U) * ab + Fraction(U) * abs(ex)
                        assert abs(Fraction(Ck[i, j]) - ex) <= kb


def test_kahan_recovers_cancelled_digits(orc):
    """sum = 1 + 10 * 1e-16: naive accumulation loses every small term,
    Kahan's compensation returns the correctly rounded exact sum."""
    x = [1.0] + [1e-16] * 10
    A = np.array([x])
    B = np.ones((len(x), 1))
    exact = float(sum(Fraction(v) for v in x))
    assert orc.kahan(A, B)[0, 0] == exact
    assert orc.naive(A, B)[0, 0] == 1.0 != exact
    # four half-ulp terms: each naive step ties back to 1, Kahan carries them
    x = [1.0] + [2.0 ** -53] * 4
    A = np.array([x])
    B = np.ones((5, 1))
    assert orc.kahan(A, B)[0, 0] == 1.0 + 2.0 ** -51
    assert orc.naive(A, B)[0, 0] == 1.0


def test_kahan_random_long_sums_within_bound(orc):
    """Long random dot products (P = 3000): Kahan's error against the exact
    rational stays within (3u + 2Pu^2) sum|ab| + u|c|, a bound the naive sum
    exceeds for cancelling data."""
    rng = np.random.default_rng(3)
    P = 3000
    a = rng.uniform(-1, 1, P) * 1e3
    a[P // 2:] = -a[: P - P // 2] * (1 + 1e-12)
    b = np.ones(P)
    A, B = a[None, :], b[:, None]
    ex = sum(Fraction(v) for v in a)
    ab = sum(abs(Fraction(v)) for v in a)
    bound = Fraction(3 * U + 2 * P * U * U) * ab + Fraction(U) * abs(ex)
    assert abs(Fraction(orc.kahan(A, B)[0, 0]) - ex) <= bound


def test_winograd_small_cases(orc):
    """P = 1 (gamma = 0): the entry is the single product (odd-P tail only).
    P = 2: the printed pair identity with y and z; integer data makes both
    exact.  The y and z vectors equal their defining sums."""
    A = synth.uniform((4, 1), 1)
    B = synth.uniform((1, 5), 2)
    C = orc.winograd(A, B)
    for i in range(4):
        for k in range(5):
            assert C[i, k] == A[i, 0] * B[0, k]
    A, B = _int_pair((6, 9, 4), 17)
    C, y, z = orc.winograd(A, B, return_yz=True)
    assert np.array_equal(C, _exact(A, B))
    Ai, Bi = A.astype(np.int64), B.astype(np.int64)
    assert np.array_equal(y, np.array([sum(Ai[i, 2 * j] * Ai[i, 2 * j + 1] for j in range(4))
                                       for i in range(6)], dtype=float))
    assert np.array_equal(z, np.array([sum(Bi[2 * j, k] * Bi[2 * j + 1, k] for j in range(4))
                                       for k in range(4)], dtype=float))


def test_winograd_within_brent_bound(orc):
    """Section 2.3.2: ||E|| <= u (n^2 + 12n - 8)/4 (||A|| + ||B||)^2 for
    WinogradOriginal and u 9/8 (n^2 + 12n - 8) ||A|| ||B|| for the scaled
    variant, infinity norm, against exact rational products."""
    for n, P in ((12, 12), (12, 13), (20, 21)):
        A = synth.uniform((n, P), 40 + P) * 64.0
        B = synth.uniform((P, n), 41 + P) / 64.0
        ex = [[sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(P)) for j in range(n)]
              for i in range(n)]
        nA, nB = orc.norm_inf(A), orc.norm_inf(B)
        d = max(n, P)
        for C, bound in ((orc.winograd(A, B), U * (d * d + 12 * d - 8) / 4 * (nA + nB) ** 2),
                         (orc.winograd_scaled(A, B), U * 9 / 8 * (d * d + 12 * d - 8) * nA * nB)):
            err = max(float(sum(abs(Fraction(C[i, j]) - ex[i][j]) for j in range(n))) for i in range(n))
            assert err <= bound


def _lambda_bruteforce(nA, nB):
    """Largest integer lambda with 1/2 <= 2^(2 lambda) nA / nB <= 2, by
    exact rational search around the estimate."""
    r = Fraction(nA) / Fraction(nB)
    est = int(round(-math.log2(nA / nB) / 2)) if (nA / nB) > 0 else 0
    ok = []
    for lam in range(est - 4, est + 5):
        v = r * (Fraction(2) ** (2 * lam))
        if Fraction(1, 2) <= v <= 2:
            ok.append(lam)
    assert ok, (nA, nB)
    return max(ok)


def test_lambda_rule_against_bruteforce(orc):
    rng = np.random.default_rng(21)
    cases = []
    for _ in range(4000):
        cases.append((float(rng.uniform(0.5, 1) * 2.0 ** rng.integers(-60, 60)),
                      float(rng.uniform(0.5, 1) * 2.0 ** rng.integers(-60, 60))))
    for _ in range(500):  # exact powers of two apart: the two-solution ties
        a = float(rng.uniform(0.5, 1) * 2.0 ** rng.integers(-30, 30))
        cases.append((a, a * 2.0 ** int(rng.integers(-20, 21))))
    for _ in range(500):  # mantissas equal or adjacent
        a = float(rng.uniform(0.5, 1))
        b = float(np.nextafter(a, 2.0 if rng.random() < 0.5 else 0.0))
        cases.append((a * 2.0 ** int(rng.integers(-9, 9)), b * 2.0 ** int(rng.integers(-9, 9))))
    for nA, nB in cases:
        assert orc.winograd_lambda(nA, nB) == _lambda_bruteforce(nA, nB), (nA, nB)
    for bad in (0.0, float("inf"), float("nan")):
        assert orc.winograd_lambda(bad, 1.0) == 0
        assert orc.winograd_lambda(1.0, bad) == 0


def test_winograd_scaled_structure(orc):
    """The paper's test B = 8A puts ||B||/||A|| = 2^3 on a tie: lambda is 1
    or 2, the larger one is taken.  The scaled product equals
    WinogradOriginal on (2^lambda A, 2^-lambda B); lambda = 0 reproduces
    WinogradOriginal."""
    A, B = synth.paper_test_pair(40, 3)
    C, lam = orc.winograd_scaled(A, B, return_lambda=True)
    assert lam == 2
    assert np.array_equal(C, orc.winograd(A * 4.0, B / 4.0))
    A = synth.uniform((17, 23), 8)
    B = synth.uniform((23, 9), 9)
    C, lam = orc.winograd_scaled(A, B, return_lambda=True)
    nA, nB = orc.norm_inf(A), orc.norm_inf(B)
    assert Fraction(1, 2) <= Fraction(nA) * Fraction(2) ** (2 * lam) / Fraction(nB) <= 2
    if lam == 0:
        assert np.array_equal(C, orc.winograd(A, B))
    B2 = B * 2.0 ** 40
    C2, lam2 = orc.winograd_scaled(A, B2, return_lambda=True)
    assert lam2 != 0
    assert np.array_equal(C2, orc.winograd(A * 2.0 ** lam2, B2 * 2.0 ** -lam2))


def test_strassen_paper_plan_matches_hand_table(orc):
    with open(os.path.join(GOLDEN, "strassen_paper_plan.json")) as f:
        table = json.load(f)
    for c in table["cases"]:
        X = c["X"]
        for shape in ((X, 1, 1), (1, X, 3), (2, 2, X)):
            assert orc.strassen_paper_plan(*shape) == (c["k"], c["m"], c["Y"]), (X, shape)


def test_strassen_levels_zero_is_naive(orc):
    A = synth.uniform((21, 19, ), 1)
    B = synth.uniform((19, 23), 2)
    for v in (0, 1):
        assert np.array_equal(orc.strassen(A, B, v, orc.MODE_LEVELS, 0), orc.naive(A, B))
        # X = 23 < 32: the paper rule gives k = 0, a single naive product
        assert np.array_equal(orc.strassen(A, B, v, orc.MODE_PAPER), orc.naive(A, B))


def test_strassen_block_identities_noncommuting(orc):
    """4x4 integer matrices with 2x2 blocks: blocks do not commute, so an
    operand swapped inside any H term of Section 2.4 would break the exact
    product.  Many random draws, one level, both variants."""
    rng = np.random.default_rng(77)
    for _ in range(200):
        A = rng.integers(-9, 10, (4, 4)).astype(float)
        B = rng.integers(-9, 10, (4, 4)).astype(float)
        for v in (0, 1):
            assert np.array_equal(orc.strassen(A, B, v, orc.MODE_LEVELS, 1), _exact(A, B))


def test_strassen_rounding_level(orc):
    """Random data: both variants stay within a normwise error a few orders
    below the 1e-11 tolerance used for the GPU at 3 levels."""
    A = synth.uniform((128, 128), 1)
    B = synth.uniform((128, 128), 2)
    ref = orc.naive(A, B)
    nA, nB = orc.norm_inf(A), orc.norm_inf(B)
    for v in (0, 1):
        for L in (1, 2, 3):
            e = orc.rel_err_inf(orc.strassen(A, B, v, orc.MODE_LEVELS, L), ref, nA, nB)
            assert e < 1e-14, (v, L, e)


def test_paper_error_tables(orc):
    """Tests section: the printed NormInf(N - C) with N = NaivKahan and
    C = A (8A).  The distribution and seed are unstated, so this is a
    magnitude check (uniform [0,1) reading, mean over seeds): within 25% of
    every nonzero printed value at n = 800, and at n = 200 each entry rounds
    to the printed tenth decimal within a factor 1.5."""
    with open(os.path.join(GOLDEN, "paper_tables.json")) as f:
        tables = json.load(f)["tables"]
    names = {"NaivStandard": orc.naive, "NaivOnArray": orc.naive_on_array,
             "NaivLoopUnrollingTwo": lambda A, B: orc.naive_unroll(A, B, 2),
             "NaivLoopUnrollingThree": lambda A, B: orc.naive_unroll(A, B, 3),
             "NaivLoopUnrollingFour": lambda A, B: orc.naive_unroll(A, B, 4),
             "WinogradOriginal": orc.winograd,
             "WinogradScaled": orc.winograd_scaled,
             "StrassenNaiv": lambda A, B: orc.strassen(A, B, 0, orc.MODE_PAPER),
             "StrassenWinograd": lambda A, B: orc.strassen(A, B, 1, orc.MODE_PAPER)}
    for n, seeds in (("200", range(4)), ("800", range(2))):
        errs = {k: [] for k in names}
        for s in seeds:
            A, B = synth.paper_test_pair(int(n), 500 + s)
            Nk = orc.kahan(A, B)
            for k, f in names.items():
                errs[k].append(orc.norm_inf(orc.minus(Nk, f(A, B))))
        for k, printed in tables[n].items():
            mean = float(np.mean(errs[k]))
            if n == "800":
                assert abs(mean - printed) <= 0.25 * printed, (n, k, mean, printed)
            else:
                lo, hi = (0.0, 0.5e-10 * 1.5) if printed == 0.0 else (0.5e-10 / 1.5, 1.5e-10 * 1.5)
                assert lo <= mean < hi, (n, k, mean, printed)


def test_norm_inf_and_aux(orc):
    A = np.array([[1.0, -2.0, 3.0], [-4.0, 0.5, 0.25], [0.0, 0.0, -0.0]])
    assert orc.norm_inf(A) == 6.0
    assert orc.norm_inf(np.zeros((0, 3))) == 0.0
    assert orc.norm_inf(np.zeros((2, 0))) == 0.0
    # sums run left to right: 1 + 2^-53 + 2^-53 rounds to 1 twice
    t = 2.0 ** -53
    assert orc.norm_inf(np.array([[1.0, t, t]])) == 1.0
    assert orc.norm_inf(np.array([[t, t, 1.0]])) == 1.0 + 2.0 ** -52
    assert orc.max_int(3, -2) == 3 and orc.max_int(-5, -5) == -5
    assert orc.max_double(-0.5, 0.25) == 0.25


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.int64)


def _row(*v):
    return np.array([v], dtype=np.float64)


def test_plus_minus_scale_worked_by_hand(orc, aux_cases):
    # Sections 1.1, 1.2, 1.5: one rounding per entry.  Every expected value
    # is worked from the binary64 rounding rule; laying the cases out as a
    # matrix also checks that entries do not mix.
    PLUS_CASES, MINUS_CASES, SCALE_CASES = aux_cases
    for cases, f in ((PLUS_CASES, orc.plus), (MINUS_CASES, orc.minus)):
        X = np.array([c[0] for c in cases]).reshape(1, -1)
        Y = np.array([c[1] for c in cases]).reshape(1, -1)
        want = np.array([c[2] for c in cases]).reshape(1, -1)
        got = f(X, Y)
        assert np.array_equal(_bits(got), _bits(want)), (got, want)
        n = X.size
        got2 = f(np.tile(X, (3, 1)).reshape(3, n), np.tile(Y, (3, 1)).reshape(3, n))
        assert np.array_equal(_bits(got2), _bits(np.tile(want, (3, 1))))
    X = np.array([[c[1] for c in SCALE_CASES]])
    for idx, (alpha, x, w) in enumerate(SCALE_CASES):
        got = orc.scale(alpha, _row(x, x, -x))
        assert _bits(got[0, 0]) == _bits(w) and _bits(got[0, 1]) == _bits(w), (alpha, x, got, w)
        # (-x) alpha = -(x alpha) under round-to-nearest
        assert _bits(got[0, 2]) == _bits(-w), (alpha, x, got)
    got = orc.scale(0.5, np.tile(X, (2, 1)))
    assert np.array_equal(_bits(got), _bits(np.tile(X * 0.5, (2, 1))))  # entries stay in place
    # NaN operands give NaN
    assert np.isnan(orc.plus(_row(math.inf), _row(-math.inf))[0, 0])
    assert np.isnan(orc.minus(_row(math.inf), _row(math.inf))[0, 0])
    assert np.isnan(orc.scale(0.0, _row(math.inf))[0, 0])
    # empty matrices are accepted
    assert orc.plus(np.zeros((0, 4)), np.zeros((0, 4))).shape == (0, 4)


def test_norm_inf_nan_and_inf_reading(orc):
    # Section 1.4 with the Section 1.3 max, whose comparison does not order
    # NaN: a NaN anywhere makes the norm NaN (the reading), an infinity
    # makes it +inf; the position of the row does not matter.
    nan = float("nan")
    for r in range(4):
        A = np.ones((4, 3))
        A[r, 1] = nan
        got = orc.norm_inf(A)
        assert math.isnan(got), r
        assert _bits(got) == _bits(abs(nan)), r          # the NaN of the row sum, sign cleared by |.|
        A[r, 1] = -math.inf
        assert orc.norm_inf(A) == math.inf, r
    A = np.ones((5, 2))
    A[1, 0] = -math.inf
    A[3, 1] = nan
    assert math.isnan(orc.norm_inf(A))
    # lambda of WinogradScaled from a NaN or infinite norm is 0 (Section 2.3.2 reading)
    assert orc.winograd_lambda(nan, 2.0) == 0 and orc.winograd_lambda(2.0, math.inf) == 0


def test_rel_err_closed_form(orc):
    C = np.array([[1.0, 2.0], [3.0, 4.0]])
    R = np.array([[1.0, 2.5], [2.0, 4.0]])
    # NormInf(C - R) = max(0.5, 1.0) = 1.0
    assert orc.rel_err_inf(C, R, 2.0, 4.0) == 1.0 / 8.0
    assert orc.rel_err_inf(C, R, 0.0, 4.0) == 1.0


# -- split-precision model ----------------------------------------------------

def test_split_digits_reconstruct(orc):
    """Digits satisfy |d_t| <= 2^(beta-1) and sum_t d_t 2^(-beta t) is within
    2^(-beta s - 1) of the scaled entry, exactly (rational arithmetic); row
    exponents put every scaled entry in [-1/2, 1/2]."""
    X = synth.wide_range((6, 11), 4)
    for beta, s in ((8, 3), (7, 4), (10, 2)):
        for is_b in (False, True):
            d, e = orc.split_digits(X, s, beta, 0, is_b)
            assert np.abs(d).max() <= 2 ** (beta - 1)
            rows, cols = X.shape
            for i in range(rows):
                for j in range(cols):
                    ex = e[j] if is_b else e[i]
                    x = Fraction(X[i, j]) / Fraction(2) ** int(ex)
                    assert abs(x) <= Fraction(1, 2)
                    rec = sum(Fraction(int(d[t, i, j]), 2 ** (beta * (t + 1))) for t in range(s))
                    assert abs(rec - x) <= Fraction(1, 2 ** (beta * s + 1))


def test_split_lambda_invariance(orc):
    """Per-row and per-column exponents absorb the 2^(+-lambda) scaling
    exactly, so the model's result does not depend on it."""
    A = synth.wide_range((20, 33), 1)
    B = synth.wide_range((33, 17), 2) * 2.0 ** 30
    assert np.array_equal(orc.split_model(A, B, 5, 8, True), orc.split_model(A, B, 5, 8, False))


def test_split_truncation_bound(orc):
    """Against the exact rational product: dropping pairs with t+u > s+1 and
    the digit remainders costs at most (s+2) 2^(-beta s - 2) per term of the
    scaled dot product, plus FP64 rounding of the final s-term sum."""
    N, P, M = 6, 40, 5
    A = synth.wide_range((N, P), 11)
    B = synth.wide_range((P, M), 12)
    for s, beta in ((3, 8), (4, 8), (5, 7), (3, 10)):
        C = orc.split_model(A, B, s, beta, False)
        _, ea = orc.split_digits(A, 1, beta, 0, False)
        _, fb = orc.split_digits(B, 1, beta, 0, True)
        for i in range(N):
            for j in range(M):
                ex = sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(P))
                sc = Fraction(2) ** int(ea[i] + fb[j])
                trunc = P * (s + 2) * Fraction(1, 2 ** (beta * s + 2)) * Fraction(11, 10)
                rnd = (s + 1) * Fraction(U) * P * Fraction(1, 4) * 2
                err = abs(Fraction(C[i, j]) - ex)
                assert err <= (trunc + rnd) * sc, (s, beta, i, j)
        # one digit fewer must be visibly worse on this data
        C1 = orc.split_model(A, B, s - 1, beta, False)
        assert np.abs(C1 - C).max() > 0


def test_split_single_run_is_correctly_rounded(orc):
    """With s <= 2 digits the s groups form one run (L >= 2 for these sizes),
    so the model rounds once: every entry is the correctly rounded value of
    the exact truncated digit product (rational arithmetic from the
    digits), times 2^(e_i + f_j).  A wrong shift inside the run or a
    misplaced pair would change the exact value and fail."""
    N, P, M = 5, 37, 4
    A = synth.wide_range((N, P), 31)
    B = synth.wide_range((P, M), 32)
    for s, beta, rule in ((1, 8, 0), (2, 8, 0), (2, 9, 0), (2, 7, 0), (1, 8, 1), (2, 8, 1)):
        assert orc.split_run_length(s, beta, P) >= s
        C = orc.split_model(A, B, s, beta, False, rule=rule)
        dA, ea = orc.split_digits(A, s, beta, 0, False, rule=rule)
        dB, fb = orc.split_digits(B, s, beta, 0, True, rule=rule)
        for i in range(N):
            for j in range(M):
                v = Fraction(0)
                for t in range(s):
                    for u in range(s):
                        if t + u + 2 <= s + 1:
                            g = sum(int(dA[t, i, k]) * int(dB[u, k, j]) for k in range(P))
                            v += Fraction(g, 2 ** (beta * (t + u + 2)))
                want = np.ldexp(float(v), int(ea[i] + fb[j]))  # float(Fraction) rounds to nearest
                assert C[i, j] == want, (s, beta, i, j)


def _split_runs_reference(orc, A, B, s, beta, runs, rule=0):
    """The model's result with the given runs, from the oracle's digits by
    rational arithmetic: exact group sums, each run rounded once when it is
    added, finest run first."""
    N, P = A.shape
    M = B.shape[1]
    dA, ea = orc.split_digits(A, s, beta, 0, False, rule=rule)
    dB, fb = orc.split_digits(B, s, beta, 0, True, rule=rule)
    out = np.empty((N, M))
    for i in range(N):
        for j in range(M):
            G = {g: 0 for g in range(2, s + 2)}
            for t in range(s):
                for u in range(s):
                    if t + u + 2 <= s + 1:
                        G[t + u + 2] += int(np.dot(dA[t, i, :].astype(object), dB[u, :, j].astype(object)))
            c = 0.0
            for run in runs:
                c = float(Fraction(c) + sum(Fraction(G[g], 2 ** (beta * g)) for g in run))
            out[i, j] = np.ldexp(c, int(ea[i] + fb[j]))
    return out


def test_split_runs_of_three(orc):
    """Runs of three groups from the finest scale: with five 9-bit digits
    {6, 5, 4}, {3, 2}; with eight, {9, 8, 7}, {6, 5, 4}, {3, 2}; with seven
    7-bit digits {8, 7, 6}, {5, 4, 3}, {2}.  Every entry of the model equals
    the rational-arithmetic reference; on these 3600 entries a boundary in
    the wrong place (eight digits as two runs of four) changes about 1% of
    them, so the check sees where the roundings fall."""
    A = synth.wide_range((60, 6), 51)
    B = synth.wide_range((6, 60), 52)
    cases = ((5, 9, [(6, 5, 4), (3, 2)]), (8, 9, [(9, 8, 7), (6, 5, 4), (3, 2)]), (7, 7, [(8, 7, 6), (5, 4, 3), (2,)]))
    for s, beta, runs in cases:
        assert orc.split_run_length(s, beta, A.shape[1]) == 3
        C = orc.split_model(A, B, s, beta, False)
        assert np.array_equal(C, _split_runs_reference(orc, A, B, s, beta, runs)), (s, beta)
    wrong = _split_runs_reference(orc, A, B, 8, 9, [(9, 8, 7, 6), (5, 4, 3, 2)])
    assert (wrong != orc.split_model(A, B, 8, 9, False)).sum() >= 10
    # byte digits: the same runs over their own digits
    assert orc.split_run_length(7, 8, A.shape[1]) == 3
    assert np.array_equal(orc.split_model(A, B, 7, 8, False, rule=1),
                          _split_runs_reference(orc, A, B, 7, 8, [(8, 7, 6), (5, 4, 3), (2,)], rule=1))


def test_split_byte_digits(orc):
    """Byte digits (int8 with 8 bits): the exponent is one step larger than
    the nearest-digit rule's, so every scaled entry lies in [-1/4, 1/4); the
    digits lie in [-128, 127] and, read in base 256, equal the scaled entry
    rounded to nearest (ties to even) at 8 s fractional bits, exactly
    (rational arithmetic; Python's round on a Fraction rounds half to
    even).  Entries next to a tie and at the top of the range included."""
    X = synth.wide_range((7, 13), 61)
    X[0, :4] = [0.49999999999999994, -0.5, 0.25, -0.2490234375]
    X[1, :3] = [1.0 + 2.0 ** -40, -(1.0 + 2.0 ** -41), 2.0 ** -60]
    for s in (1, 2, 5, 6, 8):
        for is_b in (False, True):
            d, e = orc.split_digits(X, s, 8, 0, is_b, rule=1)
            _, e0 = orc.split_digits(X, s, 8, 0, is_b, rule=0)
            assert np.array_equal(e, e0 + 1)
            assert d.min() >= -128 and d.max() <= 127
            rows, cols = X.shape
            for i in range(rows):
                for j in range(cols):
                    ex = int(e[j] if is_b else e[i])
                    x = Fraction(X[i, j]) / Fraction(2) ** ex
                    assert abs(x) < Fraction(1, 4)
                    want = round(x * 2 ** (8 * s))
                    got = sum(int(d[t, i, j]) * 256 ** (s - 1 - t) for t in range(s))
                    assert got == want, (s, is_b, i, j)


def test_split_byte_digits_fp64_grade(orc):
    """Six byte digits (46 bits of each scaled entry) are FP64-grade on the
    wide-range distribution; four are not."""
    A = synth.wide_range((48, 256), 5)
    B = synth.wide_range((256, 40), 6)
    ref = orc.naive(A, B)
    e6 = orc.rel_err_inf(orc.split_model(A, B, 6, 8, rule=1), ref, orc.norm_inf(A), orc.norm_inf(B))
    assert e6 < 5e-14
    e4 = orc.rel_err_inf(orc.split_model(A, B, 4, 8, rule=1), ref, orc.norm_inf(A), orc.norm_inf(B))
    assert e4 > 1e-12


def test_split_run_length_rule(orc):
    """L is the largest of 3, 2, 1 for which every run's worst-case exact
    sum stays within 2^53, evaluated here with Python integers."""
    def rule(s, beta, P):
        for L in (3, 2):
            ok = True
            f = s + 1
            while f >= 2:
                bound = sum((g - 1) * P * 2 ** (2 * beta - 2 + beta * (f - g)) for g in range(f, max(f - L, 1), -1))
                ok = ok and bound <= 2 ** 53
                f -= L
            if ok:
                return L
        return 1
    rng = np.random.default_rng(5)
    cases = [(s, b, int(P)) for s in range(1, 9) for b in (7, 8, 9) for P in (1, 64, 8192, 70000, 2 ** 17, 2 ** 21 + 1, 2 ** 26, 2 ** 30)]
    cases += [(int(rng.integers(1, 9)), int(rng.integers(2, 10)), int(rng.integers(1, 2 ** 34))) for _ in range(300)]
    for s, b, P in cases:
        assert orc.split_run_length(s, b, P) == rule(s, b, P), (s, b, P)


def test_split_accuracy_fp64_grade(orc):
    """On the wide-range distribution (rows scaled by 2^v, entries 2^u),
    6 bf16-sized digits reach a relative infinity-norm error well below
    1e-13 against the naive product."""
    A = synth.wide_range((48, 256), 5)
    B = synth.wide_range((256, 40), 6)
    ref = orc.naive(A, B)
    e = orc.rel_err_inf(orc.split_model(A, B, 6, 8), ref, orc.norm_inf(A), orc.norm_inf(B))
    assert e < 5e-14
    e3 = orc.rel_err_inf(orc.split_model(A, B, 3, 8), ref, orc.norm_inf(A), orc.norm_inf(B))
    assert e3 > 1e-10


def test_thread_count_does_not_change_bits(orc):
    A = synth.uniform((70, 90), 1)
    B = synth.uniform((90, 60), 2)
    t0 = orc.get_threads()
    orc.set_threads(1)
    r1 = [orc.naive(A, B), orc.kahan(A, B), orc.winograd(A, B), orc.split_model(A, B, 4, 8)]
    orc.set_threads(4)
    r4 = [orc.naive(A, B), orc.kahan(A, B), orc.winograd(A, B), orc.split_model(A, B, 4, 8)]
    orc.set_threads(t0)
    for a, b in zip(r1, r4):
        assert np.array_equal(a, b)
    rows = np.array([0, 5, 69, 33])
    assert np.array_equal(orc.naive_rows(A, B, rows), orc.naive(A, B)[rows])
    assert np.array_equal(orc.kahan_rows(A, B, rows), orc.kahan(A, B)[rows])
    assert np.array_equal(orc.winograd_rows(A, B, rows), orc.winograd(A, B)[rows])
    B2 = B * 2.0 ** 9
    assert np.array_equal(orc.winograd_rows(A, B2, rows, scaled=True), orc.winograd_scaled(A, B2)[rows])
    Ao = synth.uniform((70, 91), 3)
    Bo = synth.uniform((91, 60), 4) * 64.0
    assert np.array_equal(orc.winograd_rows(Ao, Bo, rows, scaled=True), orc.winograd_scaled(Ao, Bo)[rows])
    assert np.array_equal(orc.split_model_rows(A, B, rows, 4, 8), orc.split_model(A, B, 4, 8)[rows])


def test_unrolled_sums_worked_examples(orc):
    """Section 2.2 groupings worked by hand with u = 2^-53 against a column
    of ones.  1 + u is a tie between 1 and 1 + 2u and rounds to 1 (even).
      Two,  a = [1,u,u,u]:        (1+u) -> 1;  (u+u) = 2u;  1 + 2u exact
                                   -> 1 + 2^-52   (NaivStandard: 1)
      Three, a = [1,u,u,u,u,u]:   ((1+u)+u) -> 1;  (u+u)+u = 3u;  1 + 3u is a
                                   tie between 1 + 2u and 1 + 4u -> 1 + 4u = 1 + 2^-51
      Four, a = [1,u,...,u] (P=8): 1;  4u;  1 + 4u exact -> 1 + 2^-51
    Leftover products go one at a time (reading of the correction terms):
      Four, a = [1,u,u,u,u,u] (P=6): group -> 1, then 1 + u -> 1 twice -> 1
      (a grouped tail would give 1 + (u+u) = 1 + 2^-52);
      Three, a = [1,u,u,u,u] (P=5): group -> 1, then 1 -> 1 -> 1.
    NaivOnArray rounds exactly like NaivStandard."""
    def run(f, row):
        a = np.array([row])
        return f(a, np.ones((a.shape[1], 1)))[0, 0]

    u = U
    one_u = [1.0] + [u] * 3
    assert run(orc.naive, one_u) == 1.0
    assert run(lambda A, B: orc.naive_unroll(A, B, 2), one_u) == 1.0 + 2.0 ** -52
    assert run(lambda A, B: orc.naive_unroll(A, B, 3), [1.0] + [u] * 5) == 1.0 + 2.0 ** -51
    assert run(lambda A, B: orc.naive_unroll(A, B, 4), [1.0] + [u] * 7) == 1.0 + 2.0 ** -51
    assert run(lambda A, B: orc.naive_unroll(A, B, 4), [1.0] + [u] * 5) == 1.0
    assert run(lambda A, B: orc.naive_unroll(A, B, 3), [1.0] + [u] * 4) == 1.0
    for row in (one_u, [u, u, 1.0], [1.0] + [u] * 7):
        assert run(orc.naive_on_array, row) == run(orc.naive, row)


def test_unrolled_sums_bounds_against_rationals(orc):
    """All N, P, M in 1..6, random doubles: every summation order of Section
    2.1/2.2 obeys |C^ - C| <= gamma_{P+1} |A||B| elementwise (no term passes
    through more than P + 1 roundings: its product, at most q - 1 group
    additions and at most ceil(P/q) + (P mod q) accumulations).  Where no
    full group exists (P < q) the grouped method is the plain sequential sum,
    and for P = q it is one group sum added to 0: both equal NaivStandard
    bit for bit; NaivOnArray always does."""
    rng = np.random.default_rng(12)
    for N in range(1, 4):
        for P in range(1, 7):
            for M in range(1, 4):
                A = rng.uniform(-1, 1, (N, P)) * 2.0 ** rng.integers(-3, 4, (N, P))
                B = rng.uniform(-1, 1, (P, M)) * 2.0 ** rng.integers(-3, 4, (P, M))
                Cn = orc.naive(A, B)
                assert np.array_equal(orc.naive_on_array(A, B), Cn)
                g = Fraction((P + 1) * U) / (1 - Fraction((P + 1) * U))
                for q in (2, 3, 4):
                    Cq = orc.naive_unroll(A, B, q)
                    if P <= q:
                        assert np.array_equal(Cq, Cn), (P, q)
                    for i in range(N):
                        for j in range(M):
                            ex = sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(P))
                            ab = sum(abs(Fraction(A[i, k]) * Fraction(B[k, j])) for k in range(P))
                            assert abs(Fraction(Cq[i, j]) - ex) <= g * ab, (P, q)


def test_dot2_cancellation_worked_by_hand(orc):
    """[1e16, 1, -1e16] . [1, 1, 1] = 1: the naive sum and the paper's Kahan
    loop both lose the 1 (1e16 + 1 rounds to 1e16; Kahan's err then absorbs
    -1e16 and rounds the 1 away), TwoSum keeps it exactly in the error term.
    [2^60, 1, -2^60, 1] = 2 likewise."""
    A = np.array([[1e16, 1.0, -1e16], [2.0 ** 60, 1.0, -(2.0 ** 60)]])
    B = np.ones((3, 1))
    assert orc.dot2(A, B)[:, 0].tolist() == [1.0, 1.0]
    assert orc.naive(A, B)[0, 0] == 0.0 and orc.kahan(A, B)[0, 0] == 0.0
    A4 = np.array([[2.0 ** 60, 1.0, -(2.0 ** 60), 1.0]])
    assert orc.dot2(A4, np.ones((4, 1)))[0, 0] == 2.0


def test_dot2_bound_against_rationals(orc):
    """Ogita-Rump-Oishi (2005), bound for Dot2:
    |res - x^T y| <= u |x^T y| + gamma_n^2 |x|^T |y|, gamma_n = n u / (1 - n u).
    Checked against exact rationals on random entries over 40 binades and on
    ill-conditioned rows (a random row followed by its negation plus a small
    remainder, so the exact result is tiny next to |x|^T|y|)."""
    rng = np.random.default_rng(21)
    u = Fraction(U)
    for trial in range(300):
        n = int(rng.integers(1, 24))
        a = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-20, 21, n)
        b = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-20, 21, n)
        if trial % 2 and n >= 3:
            h = n // 2
            a[h:2 * h] = -a[:h]
            b[h:2 * h] = b[:h]
            a[-1] = a[-1] * 2.0 ** -30
        res = orc.dot2(a[None, :], b[:, None])[0, 0]
        ex = sum(Fraction(x) * Fraction(y) for x, y in zip(a, b))
        ab = sum(abs(Fraction(x) * Fraction(y)) for x, y in zip(a, b))
        g = n * u / (1 - n * u)
        assert abs(Fraction(res) - ex) <= u * abs(ex) + g * g * ab, (trial, n)
