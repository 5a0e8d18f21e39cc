"""GPU parity of every method against the CPU oracle, through the C ABI.

Bar: methods whose rounding the paper fixes (NaivStandard, NaivKahan,
WinogradOriginal, WinogradScaled, both Strassen variants with the naive
leaf, the auxiliaries) must equal the oracle bit for bit; the FP64 matrix
core paths (DGEMM, Strassen with a DGEMM leaf) must stay within the
normwise tolerance ||C - C_oracle||inf / (||A||inf ||B||inf) <= 1e-13
(DGEMM) and <= 1e-11 (Strassen, up to 3 levels); integer-valued inputs
must give the exact product bit for bit for every method.
"""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

TOL_PLAIN = 1e-13
TOL_STRASSEN = 1e-11


@pytest.fixture(scope="module")
def mmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1106_1347_amd as m

    return m


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(mmm, A, B, method, cfg=None):
    C = mmm.multiply(dev(A), dev(B), method, cfg)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def relerr(orc, C, R, A, B):
    return orc.rel_err_inf(C, R, orc.norm_inf(A), orc.norm_inf(B))


def bits_equal(X, Y):
    return X.shape == Y.shape and np.array_equal(X.view(np.int64), Y.view(np.int64))


SHAPES = [(1, 1, 1), (3, 1, 2), (7, 5, 3), (1, 300, 1), (64, 1, 64), (33, 17, 65), (129, 130, 131),
          (200, 257, 190), (256, 256, 256), (130, 48, 40)]


def _strassen_cfgs(mmm):
    out = []
    for L in (1, 2, 3):
        out.append(("L%d_naive" % L, mmm.Config(strassen_levels=L, strassen_leaf="naive")))
    out.append(("paper", mmm.Config(pad_mode="paper")))
    return out


@pytest.mark.parametrize("shape", SHAPES)
def test_paper_rounded_methods_bitwise(mmm, orc, shape):
    N, P, M = shape
    print("case", shape, flush=True)
    A = synth.uniform((N, P), 101 + N)
    B = synth.uniform((P, M), 102 + M)
    assert bits_equal(run(mmm, A, B, "naive"), orc.naive(A, B))
    assert bits_equal(run(mmm, A, B, "kahan"), orc.kahan(A, B))
    assert bits_equal(run(mmm, A, B, "winograd"), orc.winograd(A, B))
    # an unbalanced pair so that lambda != 0
    Bs = B * 2.0 ** 13
    Cws, lam = orc.winograd_scaled(A, Bs, return_lambda=True)
    assert lam != 0
    assert bits_equal(run(mmm, A, Bs, "winograd_scaled"), Cws)
    for tag, cfg in _strassen_cfgs(mmm):
        for v, name in ((0, "strassen_naive"), (1, "strassen_winograd")):
            if cfg.pad_mode == "paper":
                ref = orc.strassen(A, B, v, orc.MODE_PAPER)
            else:
                ref = orc.strassen(A, B, v, orc.MODE_LEVELS, cfg.strassen_levels)
            assert bits_equal(run(mmm, A, B, name, cfg), ref), (name, tag)


@pytest.mark.parametrize("shape", SHAPES)
def test_matrix_core_paths_within_tolerance(mmm, orc, shape):
    N, P, M = shape
    print("case", shape, flush=True)
    A = synth.uniform((N, P), 201 + N)
    B = synth.uniform((P, M), 202 + M)
    ref = orc.naive(A, B)
    assert relerr(orc, run(mmm, A, B, "dgemm"), ref, A, B) <= TOL_PLAIN
    assert relerr(orc, run(mmm, A, B, "naive", mmm.Config(naive_fma=True)), ref, A, B) <= TOL_PLAIN
    for L in (1, 2, 3):
        cfg = mmm.Config(strassen_levels=L)
        for name in ("strassen_naive", "strassen_winograd"):
            assert relerr(orc, run(mmm, A, B, name, cfg), ref, A, B) <= TOL_STRASSEN, (name, L)


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 9, 5), (129, 130, 131), (256, 256, 256), (100, 257, 64)])
def test_integer_inputs_exact_every_method(mmm, shape):
    N, P, M = shape
    print("case", shape, flush=True)
    A = synth.integers((N, P), 301)
    B = synth.integers((P, M), 302)
    ref = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    cfgs = {"naive": [None, mmm.Config(naive_fma=True)], "kahan": [None], "winograd": [None],
            "naive_on_array": [None], "naive_unroll2": [None], "naive_unroll3": [None], "naive_unroll4": [None],
            "dot2": [None],
            "winograd_scaled": [None], "dgemm": [None],
            "strassen_naive": [mmm.Config(strassen_levels=L) for L in (1, 2, 3)] + [mmm.Config(pad_mode="paper")],
            "strassen_winograd": [mmm.Config(strassen_levels=L) for L in (1, 2, 3)] + [mmm.Config(pad_mode="paper")]}
    for method, cl in cfgs.items():
        for cfg in cl:
            assert np.array_equal(run(mmm, A, B, method, cfg), ref), (method, cfg)


def _sweep_shapes():
    """24 seeded shapes: dimensions from 1 to 600 (half of them near
    multiples of the 16 / 64 / 128 tile sizes, so interior and edge tiles,
    ragged K steps and odd P all occur)."""
    rng = np.random.default_rng(5150)
    out = []
    for k in range(24):
        if k % 2:
            N, P, M = (int(rng.integers(1, 5)) * 128 + int(rng.integers(-2, 3)) for _ in range(3))
        else:
            N, P, M = (int(x) for x in rng.integers(1, 601, size=3))
        out.append((max(N, 1), max(P, 1), max(M, 1)))
    return out


@pytest.mark.parametrize("shape", _sweep_shapes())
def test_random_shape_sweep(mmm, orc, shape):
    """Every method on a seeded sweep of shapes: the orders the paper fixes
    bit for bit against the oracle, the matrix-core paths and the split
    product within their tolerances."""
    N, P, M = shape
    print("case sweep", shape, flush=True)
    A = synth.uniform((N, P), 600 + N + P)
    B = synth.uniform((P, M), 700 + P + M)
    ref = orc.naive(A, B)
    assert bits_equal(run(mmm, A, B, "naive"), ref)
    assert bits_equal(run(mmm, A, B, "kahan"), orc.kahan(A, B))
    assert bits_equal(run(mmm, A, B, "winograd"), orc.winograd(A, B))
    assert bits_equal(run(mmm, A, B, "winograd_scaled"), orc.winograd_scaled(A, B))
    for name in VARIANTS:
        assert bits_equal(run(mmm, A, B, name), _variant_ref(orc, name, A, B)), name
    cfg2 = mmm.Config(strassen_levels=2, strassen_leaf="naive")
    assert bits_equal(run(mmm, A, B, "strassen_winograd", cfg2), orc.strassen(A, B, 1, orc.MODE_LEVELS, 2))
    assert relerr(orc, run(mmm, A, B, "dgemm"), ref, A, B) <= TOL_PLAIN
    assert relerr(orc, run(mmm, A, B, "strassen_winograd", mmm.Config(strassen_levels=2)), ref, A, B) <= TOL_STRASSEN
    cfg = mmm.Config(split_type="int8", split_slices=7)
    C = run(mmm, A, B, "split", cfg)
    assert relerr(orc, C, ref, A, B) <= TOL_PLAIN
    rows = np.unique(np.linspace(0, N - 1, 8).astype(np.int64))  # the model row by row
    assert bits_equal(C[rows], orc.split_model_rows(A, B, rows, 7, 7))


def test_auxiliaries_bitwise(mmm, orc):
    for rows, cols in ((1, 1), (7, 13), (255, 257), (1024, 1023)):
        print("case", rows, cols, flush=True)
        X = synth.uniform((rows, cols), 1)
        Y = synth.uniform((rows, cols), 2)
        Xd, Yd = dev(X), dev(Y)
        assert bits_equal(mmm.plus(Xd, Yd).cpu().numpy(), orc.plus(X, Y))
        assert bits_equal(mmm.minus(Xd, Yd).cpu().numpy(), orc.minus(X, Y))
        assert bits_equal(mmm.multiply_with_scalar(0.3, Xd).cpu().numpy(), orc.scale(0.3, X))
        assert mmm.norm_inf(Xd).item() == orc.norm_inf(X)
        # in place, and an operand that is not 16-byte aligned
        Z = Xd.clone()
        mmm.plus(Z, Yd, out=Z)
        assert bits_equal(Z.cpu().numpy(), orc.plus(X, Y))
        if rows * cols > 2:
            flat = dev(np.concatenate([[0.0], X.ravel()]))
            Xu = flat[1:].view(rows, cols)
            assert bits_equal(mmm.minus(Xu, Yd).cpu().numpy(), orc.minus(X, Y))
    # sums run left to right
    t = 2.0 ** -53
    assert mmm.norm_inf(dev(np.array([[1.0, t, t]]))).item() == 1.0
    assert mmm.norm_inf(dev(np.array([[t, t, 1.0]]))).item() == 1.0 + 2.0 ** -52


def test_auxiliaries_worked_values(mmm, orc, aux_cases):
    # Sections 1.1, 1.2, 1.5: the hand-worked roundings (ties, signed zeros,
    # overflow, subnormals), bitwise, through the C ABI; the oracle gives the
    # same bits (pinned on the CPU against the same cases).
    plus_c, minus_c, scale_c = aux_cases
    for cases, f, g in ((plus_c, mmm.plus, orc.plus), (minus_c, mmm.minus, orc.minus)):
        X = np.array([[c[0] for c in cases]] * 3)
        Y = np.array([[c[1] for c in cases]] * 3)
        want = np.array([[c[2] for c in cases]] * 3)
        got = f(dev(X), dev(Y)).cpu().numpy()
        assert bits_equal(got, want), (got, want)
        assert bits_equal(got, g(X, Y))
    for alpha, x, w in scale_c:
        got = mmm.multiply_with_scalar(alpha, dev(np.array([[x, -x, x]]))).cpu().numpy()
        assert bits_equal(got, np.array([[w, -w, w]])), (alpha, x, got, w)


def test_norm_inf_nan_and_inf(mmm, orc):
    # Section 1.4 with the NaN reading: a NaN anywhere gives a NaN norm (the
    # same bits as the oracle's), an infinity gives +inf, in a middle row and
    # in the last row, across row blocks; WinogradScaled's lambda from such a
    # norm is 0 on the device as in the oracle.
    nan = float("nan")
    for rows, cols in ((5, 3), (300, 257), (1024, 1030)):
        for r in (rows // 2, rows - 1):
            for bad in (nan, -math.inf):
                print("case", rows, cols, r, bad, flush=True)
                X = synth.uniform((rows, cols), 7)
                X[r, cols // 3] = bad
                got = mmm.norm_inf(dev(X))
                want = orc.norm_inf(X)
                assert bits_equal(got.cpu().numpy().reshape(1), np.array([want])), (got.item(), want)
                Y = synth.uniform((cols, 4), 8)
                lam = mmm.winograd_lambda(got, mmm.norm_inf(dev(Y)))
                assert lam.item() == orc.winograd_lambda(want, orc.norm_inf(Y)) == 0


def test_lambda_on_device(mmm, orc):
    rng = np.random.default_rng(4)
    vals = [(1.0, 8.0), (3.0, 3.0), (0.0, 1.0), (1.0, float("inf")), (2.5, 0.0001), (7.0, 7.0 * 2 ** 21)]
    vals += [(float(rng.uniform(0.5, 1)) * 2.0 ** int(rng.integers(-40, 40)),
              float(rng.uniform(0.5, 1)) * 2.0 ** int(rng.integers(-40, 40))) for _ in range(40)]
    for a, b in vals:
        na = torch.tensor(a, dtype=torch.float64, device="cuda")
        nb = torch.tensor(b, dtype=torch.float64, device="cuda")
        assert mmm.winograd_lambda(na, nb).item() == orc.winograd_lambda(a, b), (a, b)


VARIANTS = ("naive_on_array", "naive_unroll2", "naive_unroll3", "naive_unroll4", "dot2")


def _variant_ref(orc, name, A, B):
    if name == "naive_on_array":
        return orc.naive_on_array(A, B)
    if name == "dot2":
        return orc.dot2(A, B)
    return orc.naive_unroll(A, B, int(name[-1]))


@pytest.mark.parametrize("shape", SHAPES + [(70, 50, 90), (65, 97, 66), (130, 100, 129), (48, 47, 48)])
def test_naive_variants_bitwise(mmm, orc, shape):
    """NaivOnArray and NaivLoopUnrollingTwo/Three/Four (Sections 2.1.2, 2.2)
    and the compensated dot products (beyond the paper): bit for bit the
    oracle's evaluation order, including the leftover P mod q products and
    tiles that straddle the matrix edges."""
    N, P, M = shape
    print("case", shape, flush=True)
    A = synth.uniform((N, P), 111 + N)
    B = synth.uniform((P, M), 112 + M)
    for name in VARIANTS:
        assert bits_equal(run(mmm, A, B, name), _variant_ref(orc, name, A, B)), name


def test_zero_sizes(mmm):
    for method in ("naive", "kahan", "winograd", "winograd_scaled", "strassen_naive", "strassen_winograd", "dgemm",
                   *VARIANTS):
        A = torch.zeros((5, 0), dtype=torch.float64, device="cuda")
        B = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
        C = torch.full((5, 4), 7.0, dtype=torch.float64, device="cuda")
        mmm.multiply(A, B, method, out=C)
        assert torch.count_nonzero(C).item() == 0, method
        A = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
        B = torch.ones((3, 4), dtype=torch.float64, device="cuda")
        assert mmm.multiply(A, B, method).shape == (0, 4)


def test_deterministic_bits(mmm):
    A = dev(synth.uniform((300, 211), 5))
    B = dev(synth.uniform((211, 190), 6))
    for method in ("naive", "kahan", "winograd", "winograd_scaled", "dgemm", "strassen_winograd", "strassen_naive",
                   *VARIANTS):
        c1 = mmm.multiply(A, B, method).cpu().numpy()
        c2 = mmm.multiply(A, B, method).cpu().numpy()
        assert bits_equal(c1, c2), method


@pytest.mark.parametrize("P", [4096, 4097])
def test_full_size_sampled_rows(mmm, orc, P):
    """N = M = 4096, P = 4096 and 4097 (odd-P tail): every method run at full
    size in the launch configuration the benchmark times; checked on sampled
    rows that the oracle computes one by one."""
    N = M = 4096
    print("case full size P =", P, flush=True)
    A = synth.uniform((N, P), synth.seed_a(1))
    B = synth.uniform((P, M), synth.seed_b(1))
    rows = np.array([0, 1, 127, 128, 2047, 3000, 4094, 4095])
    ref = orc.naive_rows(A, B, rows)
    nA, nB = orc.norm_inf(A), orc.norm_inf(B)
    Ad, Bd = dev(A), dev(B)

    def rows_of(method, cfg=None):
        C = mmm.multiply(Ad, Bd, method, cfg)
        torch.cuda.synchronize()
        return C[torch.from_numpy(rows).cuda()].cpu().numpy()

    def err(X):
        return orc.norm_inf(orc.minus(X, ref)) / (nA * nB)

    assert bits_equal(rows_of("naive"), ref)
    assert bits_equal(rows_of("kahan"), orc.kahan_rows(A, B, rows))
    assert bits_equal(rows_of("winograd"), orc.winograd_rows(A, B, rows))
    assert bits_equal(rows_of("winograd_scaled"), orc.winograd_rows(A, B, rows, scaled=True))
    assert err(rows_of("dgemm")) <= TOL_PLAIN
    for name in VARIANTS:  # rows of C depend only on the same rows of A
        assert bits_equal(rows_of(name), _variant_ref(orc, name, A[rows], B)), name
    for L in (2, 3):
        for name in ("strassen_winograd", "strassen_naive"):
            assert err(rows_of(name, mmm.Config(strassen_levels=L))) <= TOL_STRASSEN, (name, L)


@pytest.mark.parametrize("P", [1025, 1030, 1040, 1047])
def test_padded_operand_copies_sampled_rows(mmm, orc, P):
    """N = M = 2048 with P whose rows of A are not 16-byte aligned (odd P)
    or whose K range ends in a partial step (P mod 16 or 32 != 0): large
    products run on zero-padded copies of A and B (whole padded steps for the
    naive sums and DGEMM, a partial last step for the other recurrences).
    Same bits as the oracle on sampled rows; DGEMM within tolerance."""
    N = M = 2048
    print("case padded copies P =", P, flush=True)
    A = synth.uniform((N, P), synth.seed_a(7))
    B = synth.uniform((P, M), synth.seed_b(7))
    rows = np.array([0, 1, 63, 64, 1023, 1500, 2046, 2047])
    Ad, Bd = dev(A), dev(B)
    padded = [m for m in ("naive", "kahan", "winograd", "winograd_scaled", "dgemm") + tuple(VARIANTS)
              if mmm.workspace_bytes(m, N, P, M) > (2 * 16384 + 3 * 256 if m.startswith("winograd") else 0)]
    # every residue here sends some method through the copies
    assert padded, P
    if P % 2:
        assert {"naive", "kahan", "winograd", "dgemm", "dot2"} <= set(padded)

    def rows_of(method):
        C = mmm.multiply(Ad, Bd, method)
        torch.cuda.synchronize()
        return C[torch.from_numpy(rows).cuda()].cpu().numpy()

    ref = orc.naive_rows(A, B, rows)
    assert bits_equal(rows_of("naive"), ref)
    assert bits_equal(rows_of("kahan"), orc.kahan_rows(A, B, rows))
    assert bits_equal(rows_of("winograd"), orc.winograd_rows(A, B, rows))
    assert bits_equal(rows_of("winograd_scaled"), orc.winograd_rows(A, B, rows, scaled=True))
    assert orc.norm_inf(orc.minus(rows_of("dgemm"), ref)) / (orc.norm_inf(A) * orc.norm_inf(B)) <= TOL_PLAIN
    for name in VARIANTS:
        assert bits_equal(rows_of(name), _variant_ref(orc, name, A[rows], B)), name


def test_padded_operand_copies_integer_inputs_exact(mmm):
    """2048 x 1031 x 2048 (odd, ragged P: every method takes zero-padded
    copies) on integer-valued inputs in [-8, 8]: every partial sum is an
    integer below 2^53, so every method, the fused naive variant included,
    must return the exact product."""
    N, P, M = 2048, 1031, 2048
    print("case padded integers", (N, P, M), flush=True)
    A = synth.integers((N, P), 411)
    B = synth.integers((P, M), 412)
    rows = np.array([0, 5, 64, 1000, 2047])
    ref = (A[rows].astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    Ad, Bd = dev(A), dev(B)
    cases = [("naive", None), ("naive", mmm.Config(naive_fma=True)), ("kahan", None), ("winograd", None),
             ("winograd_scaled", None), ("dgemm", None)] + [(v, None) for v in VARIANTS]
    for method, cfg in cases:
        assert mmm.workspace_bytes(method, N, P, M, cfg) > 0 or method == "naive_unroll3", method
        C = mmm.multiply(Ad, Bd, method, cfg)
        torch.cuda.synchronize()
        assert np.array_equal(C[torch.from_numpy(rows).cuda()].cpu().numpy(), ref), (method, cfg)


@pytest.mark.parametrize("shape", [(2048, 2048, 2048), (2048, 512, 4096), (4096, 16, 2048), (1024, 4096, 8192)])
def test_dgemm_direct_load_path_exact(mmm, shape):
    """Shapes whose every tile takes the direct global-to-LDS path (N, M
    multiples of 128 with at least 256 tiles, P a multiple of 16): integer
    data makes the product exact, so any layout or index error shows."""
    N, P, M = shape
    print("case", shape, flush=True)
    A = synth.integers((N, P), 401)
    B = synth.integers((P, M), 402)
    ref = A @ B  # integer-valued doubles below 2^53: exact in any order
    assert np.array_equal(run(mmm, A, B, "dgemm"), ref)
    cfg = mmm.Config(strassen_levels=1)
    assert np.array_equal(run(mmm, A, B, "strassen_winograd", cfg), ref)


def test_misaligned_views_take_the_staged_path(mmm, orc):
    """256^3 qualifies for the direct global-to-LDS paths; operands that are
    views 8 bytes into a buffer (rows no longer 16-byte aligned) must take
    the register-staged path and give the same bits."""
    N = P = M = 256
    A = synth.uniform((N, P), 21)
    B = synth.uniform((P, M), 22)

    def shifted(X):
        flat = dev(np.concatenate([[0.0], X.ravel()]))
        return flat[1:].view(*X.shape)

    Ad, Bd, Au, Bu = dev(A), dev(B), shifted(A), shifted(B)
    for method, ref in (("naive", orc.naive(A, B)), ("kahan", orc.kahan(A, B)), ("winograd", orc.winograd(A, B)),
                        ("naive_unroll4", orc.naive_unroll(A, B, 4)), ("dot2", orc.dot2(A, B))):
        for X, Y in ((Ad, Bd), (Au, Bd), (Ad, Bu), (Au, Bu)):
            C = mmm.multiply(X, Y, method)
            torch.cuda.synchronize()
            assert bits_equal(C.cpu().numpy(), ref), method
    base = mmm.multiply(Ad, Bd, "dgemm").cpu().numpy()
    assert relerr(orc, base, orc.naive(A, B), A, B) <= TOL_PLAIN
    for X, Y in ((Au, Bd), (Ad, Bu)):
        assert relerr(orc, mmm.multiply(X, Y, "dgemm").cpu().numpy(), orc.naive(A, B), A, B) <= TOL_PLAIN


def test_dot2_recovers_cancellation(mmm, orc):
    """Rows [1e16, 1, -1e16] against columns of ones: the compensated dot
    products return the exact 1 (the naive sum and Kahan's loop give 0), bit
    for bit the oracle, on a tile of 300 x 3 x 70."""
    A = np.tile(np.array([[1e16, 1.0, -1e16]]), (300, 1))
    A[::2] *= -1.0
    B = np.ones((3, 70))
    C = run(mmm, A, B, "dot2")
    assert bits_equal(C, orc.dot2(A, B))
    assert (C[1::2] == 1.0).all() and (C[::2] == -1.0).all()


@pytest.mark.parametrize("n", [384, 2048])
def test_nonfinite_inputs_stay_in_their_rows(mmm, orc, n):
    """Reading of non-finite inputs: nothing beyond IEEE propagation is
    promised, which for the plain sums (NaivStandard, DGEMM) means a NaN in
    row i of A makes row i of C NaN, an infinity makes it infinite (B has no
    zeros here), and every other row is the finite product.  n = 384 takes
    the register kernels, n = 2048 the direct-load ones."""
    A = synth.uniform((n, n), 41)
    B = synth.uniform((n, n), 42)
    B[B == 0.0] = 0.5
    i_nan, i_inf = 5, n - 3
    A[i_nan, n // 2] = np.nan
    A[i_inf, 7] = np.inf
    rows = np.array([0, i_nan, i_inf, n - 1], dtype=np.int64)
    ref = orc.naive_rows(A, B, rows)
    for method in ("naive", "dgemm"):
        print("case", method, n, flush=True)
        C = mmm.multiply(dev(A), dev(B), method)
        torch.cuda.synchronize()
        got = C.cpu().numpy()[rows]
        assert np.isnan(got[1]).all() and np.isnan(ref[1]).all(), method
        assert np.isinf(got[2]).all() and np.array_equal(np.sign(got[2]), np.sign(ref[2])), method
        fin = [0, 3]
        assert np.isfinite(got[fin]).all(), method
        if method == "naive":
            assert bits_equal(got[fin], ref[fin])
        else:
            err = orc.norm_inf(orc.minus(got[fin], ref[fin])) / (orc.norm_inf(A[[0, n - 1]]) * orc.norm_inf(B))
            assert err <= TOL_PLAIN


@pytest.mark.parametrize("shape,L", [((517, 1031, 263), 2), ((2048, 4097, 2048), 2), ((1030, 777, 1025), 3),
                                     ((300, 2049, 7), 1), ((3, 100, 9), 2)])
def test_strassen_dgemm_leaf_peeling(mmm, orc, shape, L):
    """The DGEMM leaf peels instead of padding (Section 2.4.1's embedding is
    the alternative): the recursion runs on the leading block whose sizes
    the block split divides, leftover rows, columns and inner terms are
    DGEMM products added afterwards.  Odd sizes on every side (and a core
    with no rows at all) stay within the Strassen tolerance and give the
    exact product on integer data, also with operands 8 bytes off
    alignment (leaf operands that would be views of the root are copied)."""
    N, P, M = shape
    print("case peel", shape, L, flush=True)
    cfg = mmm.Config(strassen_levels=L)
    A = synth.uniform((N, P), 61)
    B = synth.uniform((P, M), 62)
    ref = orc.naive(A, B)

    def shifted(X):
        flat = dev(np.concatenate([[0.0], X.ravel()]))
        return flat[1:].view(*X.shape)

    for name in ("strassen_winograd", "strassen_naive"):
        assert relerr(orc, run(mmm, A, B, name, cfg), ref, A, B) <= TOL_STRASSEN, name
        C = mmm.multiply(shifted(A), shifted(B), name, cfg)
        torch.cuda.synchronize()
        assert relerr(orc, C.cpu().numpy(), ref, A, B) <= TOL_STRASSEN, (name, "shifted")
    Ai = synth.integers((N, P), 63)
    Bi = synth.integers((P, M), 64)
    assert np.array_equal(run(mmm, Ai, Bi, "strassen_winograd", cfg), Ai @ Bi)
