"""Host-side checks of the C ABI: the library loads, exports every function
include/mmm.h declares, and validates arguments on the host before any
device work (these calls never reach the GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmm.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1106_1347_amd import _lib

    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mmm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib._lib, n), n


def test_config_default_and_version(lib):
    c = lib._lib.mmm_config_default()
    assert (c.strassen_levels, c.pad_mode, c.strassen_leaf, c.split_slices, c.split_type, c.split_scale_lambda,
            c.naive_fma) == (2, 1, 0, 6, 0, 1, 0)
    assert c.split_bits == 0
    assert list(c.reserved) == [0] * 8
    assert lib.version() >= 100


def test_workspace_arithmetic(lib):
    ws = lib.workspace_bytes
    # dense-K shapes, small products and tiles that do not fit N or M run on
    # the caller's operands
    for m in ("naive", "kahan", "dgemm", "naive_unroll3", "dot2"):
        assert ws(m, 4096, 4096, 4096) == 0
        assert ws(m, 1024, 1025, 1024) == 0          # N P M < 2^32
        assert ws(m, 4000, 4097, 4096) == 0          # 4000 is no multiple of the tile rows
    assert ws("naive_unroll3", 4096, 4097, 4096) == 0  # no direct-load kernel for groups of three
    # P = 4097 on 4096 x 4096: zero-padded A (N x kp) and B (kp x M), kp the
    # next multiple of the K step (16; 32 for Kahan)
    assert ws("naive", 4096, 4097, 4096) == 2 * 4096 * 4112 * 8
    assert ws("dgemm", 4096, 4097, 4096) == 2 * 4096 * 4112 * 8
    assert ws("kahan", 4096, 4097, 4096) == 2 * 4096 * 4128 * 8
    assert ws("dot2", 4096, 4097, 4096) == 2 * 4096 * 4112 * 8
    # Winograd's pairs end at 4096 (a whole step): only A is copied, to an
    # even row length, after y and z
    assert ws("winograd", 4096, 4097, 4096) == 2 * 32768 + 4096 * 4098 * 8
    # (the two norms; 2^l A is scaled in place in A's copy; 2^-l B needs a buffer of its own)
    assert ws("winograd_scaled", 4096, 4097, 4096) == 2 * 32768 + 2 * 256 + 4096 * 4098 * 8 + 4097 * 4096 * 8
    # P even but not a multiple of the step: the same copies
    assert ws("naive", 4096, 4100, 4096) == 2 * 4096 * 4112 * 8
    assert ws("winograd", 100, 7, 300) == 1024 + 2560  # y: 800 B -> 1024, z: 2400 B -> 2560
    # WinogradScaled also holds 2^l A (5600 B -> 5632) and 2^-l B (16800 B -> 16896)
    assert ws("winograd_scaled", 100, 7, 300) == 1024 + 2560 + 2 * 256 + 5632 + 16896
    cfg = lib.Config(strassen_levels=2)
    # no padding at 4096^3: the deepest two levels run fused, so level 1 (the
    # fused level) holds nothing and level 2 holds 49 slots of A, B and products
    n1, n2 = 2048 * 2048 * 8, 1024 * 1024 * 8
    assert ws("strassen_winograd", 4096, 4096, 4096, cfg) == 3 * 49 * n2
    # three levels: level 2 is fused; levels 1 and 3 hold their slots
    n3 = 512 * 512 * 8
    assert ws("strassen_winograd", 4096, 4096, 4096, lib.Config(strassen_levels=3)) == 3 * (7 * n1 + 343 * n3)
    # one level: nothing fused
    assert ws("strassen_winograd", 4096, 4096, 4096, lib.Config(strassen_levels=1)) == 3 * 7 * n1
    assert ws("strassen_naive", 0, 5, 5) == 0
    # the naive leaf pads P = 4097 to a multiple of 2^L (4100), with padded
    # copies of A, B, C first; the DGEMM leaf peels instead: the recursion
    # runs on the leading 4096 (a multiple of 16 * 2^L) and the last column
    # of A / row of B is a DGEMM product added afterwards, so no copies
    def plan_bytes(Np, Pp, Mp, L, pad):
        al = lambda x: (x + 255) // 256 * 256
        tot = al(8 * Np * Pp) + al(8 * Pp * Mp) + al(8 * Np * Mp) if pad else 0
        for d in range(1, L + 1):
            if L >= 2 and d == L - 1:
                continue  # the fused level
            n, p_, m = Np >> d, Pp >> d, Mp >> d
            tot += al(8 * 7 ** d * n * p_) + al(8 * 7 ** d * p_ * m) + al(8 * 7 ** d * n * m)
        return tot
    assert ws("strassen_winograd", 4096, 4097, 4096, cfg) == plan_bytes(4096, 4096, 4096, 2, False) == 3 * 49 * n2
    assert ws("strassen_winograd", 4096, 4097, 4096, lib.Config(strassen_levels=2, strassen_leaf="naive")) == \
        plan_bytes(4096, 4100, 4096, 2, True)
    # small P: the 2^L granularity for both leaves (pad 33 -> 36, peel to 32)
    assert ws("strassen_winograd", 64, 33, 64, lib.Config(strassen_levels=2, strassen_leaf="naive")) == \
        plan_bytes(64, 36, 64, 2, True)
    assert ws("strassen_winograd", 64, 33, 64, lib.Config(strassen_levels=2)) == plan_bytes(64, 32, 64, 2, False)
    # a core with no rows left (N < 2^L): one DGEMM product, no workspace
    assert ws("strassen_winograd", 3, 5, 7, lib.Config(strassen_levels=2)) == 0
    with pytest.raises(ValueError):
        ws("dgemm", -1, 2, 2)
    # paper mode at X < 32 is a single naive product (no workspace)
    assert ws("strassen_naive", 20, 31, 3, lib.Config(pad_mode="paper")) == 0
    assert ws("strassen_naive", 20, 32, 3, lib.Config(pad_mode="paper")) > 0


def test_argument_errors_before_any_launch(lib):
    f = lib._lib.mmm_multiply
    c = lib._lib.mmm_config_default()
    r = ctypes.byref
    # negative size
    assert f(8, 8, 8, -1, 2, 2, 6, r(c), None, 0, None) == 1
    # unknown method
    assert f(8, 8, 8, 2, 2, 2, 99, r(c), None, 0, None) == 1
    # null C
    assert f(8, 8, None, 2, 2, 2, 6, r(c), None, 0, None) == 1
    # C overlapping A
    assert f(0x1000, 0x90000, 0x1008, 4, 4, 4, 6, r(c), None, 0, None) == 2
    # missing / small / misaligned workspace
    assert f(0x1000, 0x90000, 0x200000, 64, 64, 64, 2, r(c), None, 0, None) == 3
    assert f(0x1000, 0x90000, 0x200000, 64, 64, 64, 2, r(c), 0x400000, 16, None) == 3
    assert f(0x1000, 0x90000, 0x200000, 64, 64, 64, 2, r(c), 0x400008, 1 << 20, None) == 3
    # a large product with a ragged P needs its zero-padded copies (naive,
    # DGEMM), WinogradScaled its scaled operands: refused without them
    big = 1 << 40
    for method in (0, 6, 3):
        assert f(big, 2 * big, 3 * big, 4096, 4097, 4096, method, r(c), None, 0, None) == 3
    assert f(big, 2 * big, 3 * big, 4096, 4096, 4096, 3, r(c), None, 0, None) == 3
    # bad config fields
    bad = lib._lib.mmm_config_default()
    bad.strassen_levels = 40
    assert f(8, 8, 8, 2, 2, 2, 6, r(bad), None, 0, None) == 1
    bad = lib._lib.mmm_config_default()
    bad.reserved[3] = 1
    assert f(8, 8, 8, 2, 2, 2, 6, r(bad), None, 0, None) == 1
    # digit widths beyond what the digit type holds exactly
    for typ, bits in ((0, 10), (1, 10), (2, 9), (0, 1), (2, -1)):
        bad = lib._lib.mmm_config_default()
        bad.split_type, bad.split_bits = typ, bits
        assert f(8, 8, 8, 2, 2, 2, 7, r(bad), None, 0, None) == 1, (typ, bits)
    for typ, bits, s in (("bf16", 9, 8), ("fp16", 9, 8), ("int8", 7, 8), ("int8", 8, 8), ("bf16", 2, 1)):
        assert lib.workspace_bytes("split", 64, 3000, 64, lib.Config(split_type=typ, split_bits=bits, split_slices=s)) > 0
    # empty result: nothing to do, no device call
    assert f(None, None, None, 0, 5, 5, 6, r(c), None, 0, None) == 0
    assert lib._lib.mmm_last_error()  # message set by the failures above
    assert lib._lib.mmm_plus(8, 8, 8, -3, 1, None) == 1
    assert lib._lib.mmm_minus(0x1000, 0x9000, 0x1008, 4, 4, None) == 2
    assert lib._lib.mmm_norm_inf(8, 2, 2, None, None) == 1
    assert lib._lib.mmm_winograd_lambda(None, 8, 8, None) == 1
    assert lib._lib.mmm_status_string(2) == b"output overlaps an input"


def test_noalloc_refuses_before_any_launch(lib):
    """mmm_multiply_noalloc refuses a product whose workspace exceeds the
    static array, and bad arguments, on the host (no device call)."""
    f = lib._lib.mmm_multiply_noalloc
    c = lib._lib.mmm_config_default()
    r = ctypes.byref
    cap = lib.noalloc_scratch_bytes()
    assert cap == 64 << 20
    # the split digits of an 8192^3 product (1.5 GiB) do not fit
    assert lib.workspace_bytes("split", 8192, 8192, 8192) > cap
    assert f(0x1000, 0x90000, 0x200000, 8192, 8192, 8192, 7, r(c), None) == 3
    assert b"static scratch" in lib._lib.mmm_last_error()
    # argument errors are mmm_multiply's
    assert f(8, 8, 8, -1, 2, 2, 6, r(c), None) == 1
    assert f(8, 8, 8, 2, 2, 2, 99, r(c), None) == 1
    assert f(8, 8, None, 2, 2, 2, 6, r(c), None) == 1
    assert f(0x1000, 0x90000, 0x1008, 4, 4, 4, 6, r(c), None) == 2
    assert f(None, None, None, 0, 5, 5, 7, r(c), None) == 0


def test_batch_validation_before_any_allocation(lib):
    P = lib._CProblem
    f = lib._lib.mmm_batch_create
    c = lib._lib.mmm_config_default()
    h = ctypes.c_void_p()
    r = ctypes.byref

    def arr(*ps):
        a = (P * len(ps))()
        for i, p in enumerate(ps):
            a[i] = p
        return a

    ok = P(A=0x10000, B=0x20000, C=0x30000, N=4, P=4, M=4, method=6)
    assert f(arr(ok), 0, r(c), None, r(h)) == 1            # count 0
    assert f(arr(ok), 65536, r(c), None, r(h)) == 1        # count above 65535 (refused before reading the array)
    assert f(arr(P(A=8, B=8, C=8, N=-1, P=1, M=1, method=6)), 1, r(c), None, r(h)) == 1
    assert f(arr(P(A=8, B=8, C=8, N=1, P=1, M=1, method=2)), 1, r(c), None, r(h)) == 1  # not dgemm/split
    assert f(arr(P(A=8, B=8, C=8, N=1, P=1, M=1, method=6, tile=9)), 1, r(c), None, r(h)) == 1
    # C of one problem overlapping A of another
    bad = P(A=0x40000, B=0x50000, C=0x10008, N=2, P=2, M=2, method=6)
    assert f(arr(ok, bad), 2, r(c), None, r(h)) == 2
    # two outputs overlapping
    bad2 = P(A=0x40000, B=0x50000, C=0x30010, N=2, P=2, M=2, method=7)
    assert f(arr(ok, bad2), 2, r(c), None, r(h)) == 2
    assert h.value is None


def test_papertest_inputs_and_layout(lib):
    """Host side of the paper's test program: its inputs are the shared
    generator's (A ~ U[0,1), B = 8A exactly) and the table keeps the
    paper's columns and row order."""
    import synth
    from paper_1106_1347_amd import papertest

    A, B = papertest.paper_inputs(17, 3)
    A2, B2 = synth.paper_test_pair(17, 3)
    assert (A == A2).all() and (B == B2).all() and (B == 8.0 * A).all()
    assert [r[0] for r in papertest.PAPER_ROWS] == [
        "NaivStandard", "NaivOnArray", "NaivLoopUnrollingTwo", "NaivLoopUnrollingThree", "NaivLoopUnrollingFour",
        "StrassenNaiv", "StrassenWinograd", "WinogradOriginal", "WinogradScaled"]
    res = {"n": 5, "rows": [{"label": "N := NaivKahan", "seconds": 0.5, "err": None},
                            {"label": "NaivStandard", "seconds": 0.25, "err": 1e-10}]}
    lines = papertest.format_table(res).splitlines()
    assert len({len(l) for l in lines}) == 1  # a rectangular box
    assert "0.0000000001" in lines[-2] and lines[-3].split("|")[3].strip() == ""
