"""Serving loop on the GPU: continuous admission under a tight HBM budget,
each result bitwise equal to the same request served alone."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1106_1347_amd.serve as s

    return s


def make_requests(n, seed, hi=1536):
    reqs = []
    for r in synth.serving_requests(n, seed, rate_per_s=1000.0, lo=32, hi=hi):
        N, P, M = r["shape"]
        g = torch.Generator(device="cuda").manual_seed(seed * 1000 + r["id"])
        A = torch.rand((N, P), generator=g, dtype=torch.float64, device="cuda") * 2 - 1
        B = torch.rand((P, M), generator=g, dtype=torch.float64, device="cuda") * 2 - 1
        reqs.append((A, B, r["tol"]))
    torch.cuda.synchronize()
    return reqs


def test_alone_equals_mix(serve, orc):
    reqs = make_requests(40, 5)
    # big enough for the split path too
    g = torch.Generator(device="cuda").manual_seed(9)
    A = torch.rand((1100, 1030), generator=g, dtype=torch.float64, device="cuda")
    B = torch.rand((1030, 1050), generator=g, dtype=torch.float64, device="cuda")
    reqs += [(A, B, 1e-13), (A, B, 1e-10)]
    torch.cuda.synchronize()
    alone = []
    srv = serve.Server(budget_bytes=8 << 30, streams=1)
    for (A, B, tol) in reqs:
        alone.append(srv.submit(A, B, tol).result(timeout=60).cpu())
    srv.close()
    foot = max(8 * (A.shape[0] * A.shape[1] + B.numel() + A.shape[0] * B.shape[1]) for (A, B, _) in reqs)
    srv = serve.Server(budget_bytes=3 * foot + (256 << 20), streams=4)
    futs = [srv.submit(A, B, tol) for (A, B, tol) in reqs]
    mix = [f.result(timeout=120).cpu() for f in futs]
    st = srv.stats()
    srv.close()
    assert st["requests"] == len(reqs)
    assert st["peak_budget_used"] <= 3 * foot + (256 << 20)
    for k, (a, m) in enumerate(zip(alone, mix)):
        assert torch.equal(a.view(torch.int64), m.view(torch.int64)), k
    # accuracy against the oracle for two of them, at their tolerance
    for k in (0, len(reqs) - 2, len(reqs) - 1):
        An, Bn = reqs[k][0].cpu().numpy(), reqs[k][1].cpu().numpy()
        e = orc.rel_err_inf(mix[k].numpy(), orc.naive(An, Bn), orc.norm_inf(An), orc.norm_inf(Bn))
        assert e <= reqs[k][2], (k, e)


def test_alone_equals_mix_up_to_4096_routed_by_measured_cost(serve, orc):
    # the serving shape range (dims log-uniform on 32..4096), the method of
    # each request picked by a router calibrated on this GPU; every result
    # bitwise equal alone and in the mix, and within its tolerance against
    # the oracle on sampled rows (the row of A with the largest row sum among
    # them)
    reqs = make_requests(24, 11, hi=4096)
    router = serve.Router()
    router.calibrate(reps=2)
    methods = set()
    alone = []
    srv = serve.Server(budget_bytes=32 << 30, streams=1, router=router)
    for (A, B, tol) in reqs:
        alone.append(srv.submit(A, B, tol).result(timeout=120))
    methods |= set(srv.stats()["methods"])
    srv.close()
    srv = serve.Server(budget_bytes=6 << 30, streams=4, router=router)
    futs = [srv.submit(A, B, tol) for (A, B, tol) in reqs]
    mix = [f.result(timeout=300) for f in futs]
    st = srv.stats()
    srv.close()
    assert st["requests"] == len(reqs) and st["failed"] == 0
    assert st["peak_budget_used"] <= 6 << 30
    rng = np.random.default_rng(12)
    for k, ((A, B, tol), a, m) in enumerate(zip(reqs, alone, mix)):
        print("request", k, tuple(A.shape), B.shape[1], tol, flush=True)
        assert torch.equal(a.view(torch.int64), m.view(torch.int64)), k
        An, Bn = A.cpu().numpy(), B.cpu().numpy()
        rows = np.unique(np.concatenate([rng.choice(An.shape[0], size=min(3, An.shape[0]), replace=False),
                                         [int(np.argmax(np.abs(An).sum(axis=1)))]])).astype(np.int64)
        got = m.cpu().numpy()[rows]
        e = orc.rel_err_inf(got, orc.naive_rows(An, Bn, rows), orc.norm_inf(An), orc.norm_inf(Bn))
        assert e <= tol, (k, e)
    print("methods used", sorted(methods), flush=True)


def test_degenerate_requests(serve):
    """Requests with an empty side (N = 0 or M = 0: an empty result) and with
    P = 0 (the empty sum: exact zeros), at both tolerance classes, mixed with
    an ordinary one; every future resolves with the right shape."""
    z = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")  # noqa: E731
    g = torch.Generator(device="cuda").manual_seed(21)
    A = torch.rand((70, 90), generator=g, dtype=torch.float64, device="cuda")
    B = torch.rand((90, 40), generator=g, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    cases = [(z(0, 5), z(5, 3), 1e-13), (z(4, 6), z(6, 0), 1e-10), (z(5, 0), z(0, 7), 1e-13), (z(3, 0), z(0, 4), 1e-10),
             (A, B, 1e-13)]
    srv = serve.Server(budget_bytes=1 << 30, streams=4)
    out = [f.result(timeout=60) for f in [srv.submit(a, b, tol) for (a, b, tol) in cases]]
    srv.close()
    assert [tuple(c.shape) for c in out] == [(0, 3), (4, 0), (5, 7), (3, 4), (70, 40)]
    assert torch.equal(out[2], z(5, 7)) and torch.equal(out[3], z(3, 4))
    m, cfg = srv.router.choose(70, 90, 40, 1e-13)
    from paper_1106_1347_amd import multiply

    assert torch.equal(out[4].view(torch.int64), multiply(A, B, m, cfg).view(torch.int64))
