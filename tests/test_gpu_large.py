"""Operands with more than 2^31 entries (18.4 GB each), through the C ABI.

Every offset into such an operand beyond 2^31 elements (2^34 bytes) must be
formed in 64 bits: C = AB with A of 70016 x 32768 (then B of 32768 x 70016)
runs on the same direct-load and matrix-core kernels as the benchmark
shapes, and sampled entries on both sides of the 2^31-element boundary are
checked against the oracle: bit for bit for the methods whose rounding the
paper fixes and for the split model, within 1e-13 for DGEMM.  The inputs
are drawn on the device by torch's seeded generator; the rows and columns
the oracle needs are copied back from the very tensors the library reads.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

N_BIG, P_BIG, M_SMALL = 70016, 32768, 128  # 70016 x 32768 = 2.29e9 entries > 2^31
BITWISE = ("naive", "kahan", "winograd")


@pytest.fixture(scope="module")
def mmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1106_1347_amd as m

    return m


def _rand(shape, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return torch.rand(shape, generator=g, dtype=torch.float64, device="cuda") * 2 - 1


def _bits_equal(X, Y):
    return X.shape == Y.shape and np.array_equal(X.view(np.int64), Y.view(np.int64))


def _check(mmm, orc, Ad, Bd, rows, cols, A_sub, B_sub):
    """Run every method on the device operands; compare C[rows][:, cols]
    with the oracle on A_sub (the rows) and B_sub (the columns)."""
    r = np.arange(A_sub.shape[0])
    ref = orc.naive_rows(A_sub, B_sub, r)
    want = {"naive": ref, "kahan": orc.kahan_rows(A_sub, B_sub, r), "winograd": orc.winograd_rows(A_sub, B_sub, r)}
    ridx = torch.from_numpy(rows).cuda()
    cidx = torch.from_numpy(cols).cuda()
    for method in BITWISE + ("dgemm", "split"):
        print("method", method, tuple(Ad.shape), tuple(Bd.shape), flush=True)
        cfg = mmm.Config(split_type="int8", split_slices=7) if method == "split" else None
        C = mmm.multiply(Ad, Bd, method, cfg)
        got = C[ridx][:, cidx].cpu().numpy()
        del C
        torch.cuda.synchronize()
        if method in BITWISE:
            assert _bits_equal(got, want[method]), method
        elif method == "dgemm":
            err = orc.norm_inf(orc.minus(got, ref)) / (orc.norm_inf(A_sub) * orc.norm_inf(B_sub))
            assert err <= 1e-13, err
        else:
            assert _bits_equal(got, orc.split_model_rows(A_sub, B_sub, r, 7, 7)), method
        torch.cuda.empty_cache()


def test_a_beyond_int32_elements(mmm):
    import oracle as orc

    Ad = _rand((N_BIG, P_BIG), 9101)
    Bd = _rand((P_BIG, M_SMALL), 9102)
    assert Ad.numel() > 2 ** 31
    # row 65536 starts exactly 2^31 elements in; the last row ends at 2.29e9
    rows = np.array([0, 65535, 65536, N_BIG - 1], dtype=np.int64)
    cols = np.arange(M_SMALL, dtype=np.int64)
    A_sub = Ad[torch.from_numpy(rows).cuda()].cpu().numpy()
    B_all = Bd.cpu().numpy()
    _check(mmm, orc, Ad, Bd, rows, cols, A_sub, B_all)
    del Ad, Bd
    torch.cuda.empty_cache()


def test_b_beyond_int32_elements(mmm):
    import oracle as orc

    Ad = _rand((M_SMALL, P_BIG), 9103)
    Bd = _rand((P_BIG, N_BIG), 9104)
    assert Bd.numel() > 2 ** 31
    # entry (k, j) of B sits k * 70016 + j elements in: the last columns of
    # the last rows lie beyond 2^31
    rows = np.array([0, M_SMALL - 1], dtype=np.int64)
    cols = np.concatenate([np.arange(64), np.arange(N_BIG - 64, N_BIG)]).astype(np.int64)
    A_sub = Ad[torch.from_numpy(rows).cuda()].cpu().numpy()
    B_sub = Bd[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    _check(mmm, orc, Ad, Bd, rows, cols, A_sub, B_sub)
    del Ad, Bd
    torch.cuda.empty_cache()
