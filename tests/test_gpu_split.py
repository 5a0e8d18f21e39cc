"""GPU parity of the split-precision product against the oracle's model.

The digit products are exact on the matrix cores, so the GPU result must
equal the oracle's split model bit for bit (same digits, same exact group
sums, same FP64 recombination order), for every digit type and digit count;
against the naive product it must reach FP64-grade accuracy (relative
infinity-norm error <= 1e-13) with the default digit counts.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

BETA = {"bf16": 8, "fp16": 9, "int8": 7}


@pytest.fixture(scope="module")
def mmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1106_1347_amd as m

    return m


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def split(mmm, A, B, typ, s, scale=True, bits=0):
    cfg = mmm.Config(split_type=typ, split_slices=s, split_scale_lambda=scale, split_bits=bits)
    C = mmm.multiply(dev(A), dev(B), "split", cfg)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def bits_equal(X, Y):
    return X.shape == Y.shape and np.array_equal(X.view(np.int64), Y.view(np.int64))


def model(orc, A, B, typ, s, bits, scale=True):
    """The oracle's model for a digit type and width (byte digits for int8 with 8 bits)."""
    beta = bits or BETA[typ]
    return orc.split_model(A, B, s, beta, scale, rule=orc.split_rule(typ, beta))


SHAPES = [(1, 1, 1), (5, 3, 7), (64, 64, 64), (65, 130, 63), (129, 257, 131), (200, 64, 300), (256, 300, 256)]
# (digit type, digit count, digit width; 0 = the type's default)
CASES = [("bf16", 6, 0), ("bf16", 3, 0), ("bf16", 8, 0), ("fp16", 4, 0), ("fp16", 6, 0), ("fp16", 5, 0),
         ("int8", 7, 0), ("int8", 4, 0), ("int8", 8, 0), ("int8", 1, 0),
         ("bf16", 5, 9), ("bf16", 8, 9), ("bf16", 4, 5), ("fp16", 3, 7), ("int8", 5, 6), ("int8", 8, 3),
         ("int8", 6, 8), ("int8", 1, 8), ("int8", 3, 8), ("int8", 8, 8)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("typ,s,bits", CASES)
def test_split_bitwise_vs_model(mmm, orc, shape, typ, s, bits):
    N, P, M = shape
    print("case", shape, typ, s, bits, flush=True)
    A = synth.wide_range((N, P), 11 + N)
    B = synth.wide_range((P, M), 12 + M) * 2.0 ** 17
    got = split(mmm, A, B, typ, s, bits=bits)
    assert bits_equal(got, model(orc, A, B, typ, s, bits))


@pytest.mark.parametrize("typ,s,bits", [("bf16", 5, 9), ("fp16", 5, 9), ("bf16", 6, 8), ("fp16", 8, 9)])
def test_split_flush_every_interval(mmm, orc, typ, s, bits):
    """K = 3000 runs every digit-pair group through several flushes at its
    own interval (with 9-bit digits the fullest groups flush every step):
    the result still equals the model bit for bit."""
    print("case flush", typ, s, bits, flush=True)
    A = synth.wide_range((70, 3000), 21)
    B = synth.wide_range((3000, 50), 22)
    assert bits_equal(split(mmm, A, B, typ, s, bits=bits), orc.split_model(A, B, s, bits, True))


@pytest.mark.parametrize("typ,s", [("bf16", 6), ("int8", 7), ("fp16", 5)])
def test_split_lambda_invariance_and_uniform(mmm, orc, typ, s):
    A = synth.uniform((130, 190), 1)
    B = synth.uniform((190, 70), 2) * 2.0 ** -40
    on = split(mmm, A, B, typ, s, True)
    off = split(mmm, A, B, typ, s, False)
    assert bits_equal(on, off)
    assert bits_equal(on, orc.split_model(A, B, s, BETA[typ], False))


@pytest.mark.parametrize("typ,s,bits", [("int8", 6, 8), ("int8", 7, 0), ("bf16", 6, 0), ("fp16", 5, 0)])
def test_split_zero_rows_and_columns(mmm, orc, typ, s, bits):
    """All-zero rows of A and columns of B (exponent of an empty maximum),
    and a zero operand, still give the model's bits (zeros where the row or
    column is zero)."""
    A = synth.wide_range((70, 130), 31)
    B = synth.wide_range((130, 50), 32)
    A[[0, 33, 69], :] = 0.0
    B[:, [0, 17, 49]] = 0.0
    got = split(mmm, A, B, typ, s, bits=bits)
    assert bits_equal(got, model(orc, A, B, typ, s, bits))
    assert not got[[0, 33, 69], :].any() and not got[:, [0, 17, 49]].any()
    Z = np.zeros_like(A)
    assert bits_equal(split(mmm, Z, B, typ, s, bits=bits), model(orc, Z, B, typ, s, bits))


@pytest.mark.parametrize("typ,s,bits", [("bf16", 5, 9), ("int8", 6, 8), ("fp16", 6, 0)])
def test_split_operands_at_odd_offsets(mmm, orc, typ, s, bits):
    """A, B and C as views one element (8 bytes) into larger buffers, so no
    row start is 16-byte aligned: the statistics and digit passes read them
    as they lie, and the result equals the model's bits (written into the
    view only)."""
    N, P, M = 97, 131, 75
    A = synth.wide_range((N, P), 41)
    B = synth.wide_range((P, M), 42)
    bufA = torch.zeros(N * P + 3, dtype=torch.float64, device="cuda")
    bufB = torch.zeros(P * M + 3, dtype=torch.float64, device="cuda")
    bufC = torch.full((N * M + 3,), float("nan"), dtype=torch.float64, device="cuda")
    bufA[1:1 + N * P] = dev(A).reshape(-1)
    bufB[1:1 + P * M] = dev(B).reshape(-1)
    Av, Bv, Cv = bufA[1:1 + N * P].view(N, P), bufB[1:1 + P * M].view(P, M), bufC[1:1 + N * M].view(N, M)
    assert Av.data_ptr() % 16 == 8 and Bv.data_ptr() % 16 == 8 and Cv.data_ptr() % 16 == 8
    cfg = mmm.Config(split_type=typ, split_slices=s, split_bits=bits)
    mmm.multiply(Av, Bv, "split", cfg, out=Cv)
    torch.cuda.synchronize()
    assert bits_equal(Cv.cpu().numpy(), model(orc, A, B, typ, s, bits))
    edge = bufC.cpu().numpy()
    assert np.isnan(edge[0]) and np.isnan(edge[1 + N * M:]).all()


def test_split_integer_inputs_exact(mmm):
    A = synth.integers((100, 257), 3)
    B = synth.integers((257, 90), 4)
    ref = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    for typ, s, bits in (("bf16", 1, 0), ("bf16", 6, 0), ("fp16", 2, 0), ("int8", 1, 0), ("int8", 7, 0),
                         ("int8", 1, 8), ("int8", 6, 8)):
        assert np.array_equal(split(mmm, A, B, typ, s, bits=bits), ref), (typ, s, bits)


@pytest.mark.parametrize("typ,s,bits", [("bf16", 8, 9), ("fp16", 5, 9)])
def test_split_run_length_edges(mmm, orc, typ, s, bits):
    """The recombination merges runs of three groups only while their exact
    sums fit binary64; K just below and just above the first K where that
    fails (two-group runs from there) still gives the model's bits."""
    lo, hi = 1, 1 << 20
    assert orc.split_run_length(s, bits, lo) == 3 and orc.split_run_length(s, bits, hi) < 3
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lo, hi = (mid, hi) if orc.split_run_length(s, bits, mid) == 3 else (lo, mid)
    for P in (lo, hi):
        print("case run edge", typ, s, bits, P, orc.split_run_length(s, bits, P), flush=True)
        A = synth.wide_range((5, P), 41)
        B = synth.wide_range((P, 3), 42)
        assert bits_equal(split(mmm, A, B, typ, s, bits=bits), orc.split_model(A, B, s, bits, True)), P


def test_split_fp64_grade(mmm, orc):
    A = synth.wide_range((256, 1024), 5)
    B = synth.wide_range((1024, 192), 6)
    ref = orc.naive(A, B)
    nA, nB = orc.norm_inf(A), orc.norm_inf(B)
    for typ, s, bits in (("bf16", 6, 0), ("int8", 7, 0), ("fp16", 6, 0), ("fp16", 5, 0), ("bf16", 5, 9), ("int8", 6, 8)):
        e = orc.rel_err_inf(split(mmm, A, B, typ, s, bits=bits), ref, nA, nB)
        print(typ, s, bits, e, flush=True)
        assert e <= 1e-13, (typ, s, bits, e)


def test_split_int8_flush_path(mmm, orc):
    """K = 70000 with 8 int8 digits exceeds the exact int32 range of one
    accumulation (65536 entries), so the kernel flushes to FP64 mid-loop."""
    A = synth.wide_range((32, 70000), 7)
    B = synth.wide_range((70000, 40), 8)
    assert bits_equal(split(mmm, A, B, "int8", 8), orc.split_model(A, B, 8, 7, True))
    # byte digits: 8 pairs of |d| <= 128 fill int32 after 16384 entries
    assert bits_equal(split(mmm, A, B, "int8", 8, bits=8), model(orc, A, B, "int8", 8, 8))


def test_split_full_size_sampled_rows(mmm, orc):
    """N = P = M = 8192 on the wide-range distribution (entries +-2^u,
    u ~ U[-20, 20], rows scaled by 2^v, v ~ U{-10..10}), in the launch
    configuration the benchmark uses; sampled rows checked bit for bit
    against the model, and FP64-grade against the naive product."""
    n = 8192
    A = synth.wide_range((n, n), synth.seed_a(2))
    B = synth.wide_range((n, n), synth.seed_b(2))
    # with the row of A of largest absolute sum: it sets the normwise error
    rows = np.unique(np.array([0, 4095, 8191, int(np.argmax(np.abs(A).sum(axis=1)))]))
    Ad, Bd = dev(A), dev(B)
    ref = orc.naive_rows(A, B, rows)
    nA, nB = orc.norm_inf(A), orc.norm_inf(B)
    for typ, s, bits in (("int8", 7, 0), ("bf16", 6, 0), ("bf16", 5, 9), ("int8", 6, 8)):
        print("case full size", typ, s, bits, flush=True)
        C = mmm.multiply(Ad, Bd, "split", mmm.Config(split_type=typ, split_slices=s, split_bits=bits))
        torch.cuda.synchronize()
        got = C[torch.from_numpy(rows).cuda()].cpu().numpy()
        del C
        beta = bits or BETA[typ]
        assert bits_equal(got, orc.split_model_rows(A, B, rows, s, beta, True, rule=orc.split_rule(typ, beta))), typ
        assert orc.norm_inf(orc.minus(got, ref)) / (nA * nB) <= 1e-13
