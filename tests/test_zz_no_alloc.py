"""mmm_multiply_noalloc (the library's static workspace array) against
mmm_multiply with a caller workspace: bitwise the same C, on two calls in a
row per method, the second smaller than the first, so whatever the first
call left in the shared array must not reach the second result."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1106_1347_amd as m

    return m


CASES = [
    # (method, config kwargs): every method whose workspace the array replaces
    ("winograd", {}),
    ("winograd_scaled", {}),
    ("strassen_winograd", {"strassen_levels": 2}),
    ("strassen_naive", {"strassen_levels": 1}),
    ("split", {"split_type": "bf16", "split_slices": 6}),
    ("split", {"split_type": "int8", "split_slices": 7}),
    ("split", {"split_type": "int8", "split_slices": 6, "split_bits": 8}),
    ("split", {"split_type": "fp16", "split_slices": 5}),
]
SHAPES = [(700, 613, 530), (257, 130, 91)]  # second call smaller


@pytest.mark.parametrize("method,kw", CASES, ids=["%s-%s" % (m, "-".join(map(str, k.values()))) for m, k in CASES])
def test_noalloc_equals_multiply(mmm, method, kw):
    cfg = mmm.Config(**kw)
    for g, (N, P, M) in enumerate(SHAPES):
        need = mmm.workspace_bytes(method, N, P, M, cfg)
        assert 0 < need <= mmm.noalloc_scratch_bytes(), (method, N, P, M, need)
        A = torch.from_numpy(synth.uniform((N, P), 900 + 2 * g)).cuda()
        B = torch.from_numpy(synth.uniform((P, M), 901 + 2 * g)).cuda()
        print("noalloc %s %s shape %s" % (method, kw, (N, P, M)), flush=True)
        want = mmm.multiply(A, B, method, cfg)
        got = torch.full((N, M), float("nan"), dtype=torch.float64, device="cuda")
        mmm.multiply_noalloc(A, B, got, method, cfg)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().view(np.int64), want.cpu().numpy().view(np.int64)), (method, g)


def test_noalloc_refuses_oversized_product(mmm):
    A = torch.zeros(2048, 2048, dtype=torch.float64, device="cuda")
    C = torch.zeros(2048, 2048, dtype=torch.float64, device="cuda")
    cfg = mmm.Config(split_type="bf16", split_slices=8)
    assert mmm.workspace_bytes("split", 2048, 2048, 2048, cfg) > mmm.noalloc_scratch_bytes()
    with pytest.raises(mmm.MmmError) as e:
        mmm.multiply_noalloc(A, A, C, "split", cfg)
    assert e.value.status == 3


def test_noalloc_at_the_array_limit(mmm):
    """The largest square split product (bf16, 6 digits) whose workspace fits
    the static array runs and equals mmm_multiply bitwise; the next size up
    is refused before anything is enqueued."""
    cfg = mmm.Config(split_type="bf16", split_slices=6)
    cap = mmm.noalloc_scratch_bytes()
    lo, hi = 1, 8192  # workspace_bytes grows with n: fits at lo, not at hi
    assert mmm.workspace_bytes("split", lo, lo, lo, cfg) <= cap < mmm.workspace_bytes("split", hi, hi, hi, cfg)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if mmm.workspace_bytes("split", mid, mid, mid, cfg) <= cap:
            lo = mid
        else:
            hi = mid
    n = lo
    print("noalloc limit: n = %d, %d of %d bytes" % (n, mmm.workspace_bytes("split", n, n, n, cfg), cap), flush=True)
    A = torch.from_numpy(synth.uniform((n, n), 960)).cuda()
    B = torch.from_numpy(synth.uniform((n, n), 961)).cuda()
    want = mmm.multiply(A, B, "split", cfg)
    got = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    mmm.multiply_noalloc(A, B, got, "split", cfg)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.int64), want.cpu().numpy().view(np.int64))
    A1 = torch.zeros(n + 1, n + 1, dtype=torch.float64, device="cuda")
    C1 = torch.zeros(n + 1, n + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(mmm.MmmError) as e:
        mmm.multiply_noalloc(A1, A1, C1, "split", cfg)
    assert e.value.status == 3
