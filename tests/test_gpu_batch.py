"""Batches: one HIP graph over many uneven products, FP64 and split mixed.

Every batched product must equal the single mmm_multiply result with the
same method and config bit for bit (the tile arithmetic does not depend on
the tile shape or on the workgroup that runs it), on every replay of the
graph, with unrelated eager work between replays.  The outputs are reset
to NaN before each replay, so a replay whose tile counters were not put
back to zero (its workgroups would claim nothing) fails.
"""
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


DGEMM_TILES = ["auto", "128x128", "64x64", "128x64"]
SPLIT_TILES = ["auto", "wide", "narrow"]


def make_problems(shapes, seed, methods, slices):
    # tile choices cycle per method: every DGEMM and every split tile shape
    # is exercised across the list
    out = []
    seen = {}
    for g, (N, P, M) in enumerate(shapes):
        A = torch.from_numpy(synth.uniform((N, P), seed + 2 * g)).cuda()
        B = torch.from_numpy(synth.uniform((P, M), seed + 2 * g + 1)).cuda()
        C = torch.full((N, M), float("nan"), dtype=torch.float64, device="cuda")
        m = methods[g % len(methods)]
        tiles = SPLIT_TILES if m == "split" else DGEMM_TILES
        n = seen.get(m, 0)
        seen[m] = n + 1
        out.append((A, B, C, m, slices[g % len(slices)], tiles[n % len(tiles)]))
    return out


def single(mmm, A, B, method, s, cfg):
    c = mmm.Config(**{**cfg.__dict__, "split_slices": s or cfg.split_slices})
    return mmm.multiply(A, B, method, c)


@pytest.mark.parametrize("typ,slices,bits", [("int8", [0, 4, 7], 0), ("bf16", [0, 3, 6], 0), ("fp16", [6], 0),
                                             ("int8", [0, 5, 6], 8), ("bf16", [5], 9)])
def test_batch_equals_single_calls_and_replays(mmm, typ, slices, bits):
    print("case batch", typ, slices, bits, flush=True)
    cfg = mmm.Config(split_type=typ, split_slices=7 if typ == "int8" else 6, split_bits=bits)
    shapes = synth.batch_shapes(48, 7, 1, 200) + [(16, 0, 9), (0, 5, 5), (300, 257, 3)]
    probs = make_problems(shapes, 100, ["dgemm", "split"], slices)
    want = [single(mmm, A, B, m, s, cfg).cpu() for (A, B, C, m, s, t) in probs]
    plan = mmm.Batch(probs, cfg)
    for rep in range(3):
        for p in probs:
            p[2].fill_(float("nan"))
        plan.launch()
        # unrelated eager work between replays
        X = torch.rand(300, 300, dtype=torch.float64, device="cuda")
        mmm.multiply(X, X, "winograd")
        torch.cuda.synchronize()
        for k, (p, w) in enumerate(zip(probs, want)):
            got = p[2].cpu()
            assert got.shape == w.shape
            assert np.array_equal(got.numpy().view(np.int64), w.numpy().view(np.int64)), (rep, k, shapes[k], p[3])
    plan.close()


@pytest.mark.parametrize("methods,slices", [(["dgemm"], [0]), (["split"], [3, 5, 6, 4])])
def test_batch_single_kind_plans(mmm, methods, slices):
    """Plans holding one kind of problem: only FP64 (no split branch; the FP64
    grids take their full occupancy) or only split products of several digit
    counts and tile variants (many split groups, several per graph branch,
    each with its own tile counters).  Bitwise equal to single calls on every
    replay."""
    print("case batch single kind", methods, slices, flush=True)
    cfg = mmm.Config(split_type="bf16", split_slices=6)
    shapes = synth.batch_shapes(36, 11, 1, 300) + [(257, 129, 300), (3, 700, 5)]
    probs = make_problems(shapes, 400, methods, slices)
    want = [single(mmm, A, B, m, s, cfg).cpu() for (A, B, C, m, s, t) in probs]
    plan = mmm.Batch(probs, cfg)
    for rep in range(3):
        for p in probs:
            p[2].fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        for k, (p, w) in enumerate(zip(probs, want)):
            got = p[2].cpu()
            assert np.array_equal(got.numpy().view(np.int64), w.numpy().view(np.int64)), (rep, k, shapes[k], p[3])
    plan.close()


def test_batch_at_the_count_limit(mmm):
    """65535 problems (the most one plan takes), half DGEMM and half split
    (int8 byte digits), dimensions 1..8, operands as views into one buffer:
    one graph launch, sampled results bitwise equal to single calls."""
    n = 65535
    rng = np.random.default_rng(5)
    dims = rng.integers(1, 9, size=(n, 3))
    na, nb, nc = (dims[:, 0] * dims[:, 1]), (dims[:, 1] * dims[:, 2]), (dims[:, 0] * dims[:, 2])
    oa = np.concatenate([[0], np.cumsum(na)])
    ob = oa[-1] + np.concatenate([[0], np.cumsum(nb)])
    oc = np.concatenate([[0], np.cumsum(nc)])
    gen = torch.Generator(device="cuda").manual_seed(5)
    buf = torch.rand(int(ob[-1]), dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
    cbuf = torch.full((int(oc[-1]),), float("nan"), dtype=torch.float64, device="cuda")
    probs = []
    for i, (N, P, M) in enumerate(dims.tolist()):
        probs.append((buf[oa[i]:oa[i + 1]].view(N, P), buf[ob[i]:ob[i + 1]].view(P, M), cbuf[oc[i]:oc[i + 1]].view(N, M),
                      "dgemm" if i % 2 == 0 else "split"))
    cfg = mmm.Config(split_type="int8", split_slices=6, split_bits=8)
    plan = mmm.Batch(probs, cfg)
    plan.launch()
    torch.cuda.synchronize()
    assert not torch.isnan(cbuf).any()
    for i in sorted(set(rng.integers(0, n, 300).tolist()) | {0, 1, n - 2, n - 1}):
        A, B, C, m = probs[i]
        w = mmm.multiply(A, B, m, cfg)
        assert torch.equal(C.view(torch.int64), w.view(torch.int64)), (i, dims[i], m)
    plan.close()


def test_batch_empty_and_zero_depth_problems(mmm):
    """Degenerate plans: problems with P = 0 (C is the empty sum, exact
    zeros, for both methods) beside empty ones (N = 0 or M = 0: nothing
    written), and a plan with no work at all, which still creates, launches
    and closes cleanly."""
    cfg = mmm.Config(split_type="int8", split_slices=6, split_bits=8)

    def mats(N, P, M):
        A = torch.rand(N, P, dtype=torch.float64, device="cuda")
        B = torch.rand(P, M, dtype=torch.float64, device="cuda")
        C = torch.full((N, M), float("nan"), dtype=torch.float64, device="cuda")
        return A, B, C

    probs = [(*mats(5, 0, 7), "dgemm"), (*mats(3, 0, 4), "split"), (*mats(0, 5, 5), "dgemm"), (*mats(4, 6, 0), "split"),
             (*mats(6, 9, 5), "split")]
    plan = mmm.Batch(probs, cfg)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(probs[0][2], torch.zeros(5, 7, dtype=torch.float64, device="cuda"))
        assert torch.equal(probs[1][2], torch.zeros(3, 4, dtype=torch.float64, device="cuda"))
        w = mmm.multiply(probs[4][0], probs[4][1], "split", cfg)
        assert torch.equal(probs[4][2].view(torch.int64), w.view(torch.int64))
    plan.close()
    empty = mmm.Batch([(*mats(0, 5, 5), "dgemm"), (*mats(4, 6, 0), "split")], cfg)
    empty.launch()
    torch.cuda.synchronize()
    empty.close()


def test_batch_full_workload(mmm, orc):
    """2048 problems, N, P, M uniform on 16..512, even index FP64 DGEMM, odd
    index split (bf16, 6 digits): one graph launch; sampled results checked
    against single calls bitwise and against the oracle."""
    shapes = synth.batch_shapes(2048, synth.seed_a(3), 16, 512)
    rng = np.random.default_rng(1)
    probs = []
    for g, (N, P, M) in enumerate(shapes):
        A = torch.rand(N, P, dtype=torch.float64, device="cuda") * 2 - 1
        B = torch.rand(P, M, dtype=torch.float64, device="cuda") * 2 - 1
        C = torch.empty(N, M, dtype=torch.float64, device="cuda")
        probs.append((A, B, C, "dgemm" if g % 2 == 0 else "split"))
    cfg = mmm.Config()
    plan = mmm.Batch(probs, cfg)
    plan.launch()
    torch.cuda.synchronize()
    sample = sorted(set(rng.integers(0, 2048, 40).tolist()) | {0, 1, 2046, 2047})
    for g in sample:
        A, B, C, m = probs[g]
        w = mmm.multiply(A, B, m, cfg)
        assert torch.equal(C.view(torch.int64), w.view(torch.int64)), g
    for g in sample[:6]:
        A, B, C, m = probs[g]
        An, Bn = A.cpu().numpy(), B.cpu().numpy()
        if m == "dgemm":
            e = orc.rel_err_inf(C.cpu().numpy(), orc.naive(An, Bn), orc.norm_inf(An), orc.norm_inf(Bn))
            assert e <= 1e-13
        else:
            assert np.array_equal(C.cpu().numpy().view(np.int64), orc.split_model(An, Bn, 6, 8).view(np.int64))
    plan.close()


def test_autotuner_batch_policy(mmm, tmp_path):
    """The whole-batch step: one of the policies is chosen, persisted per
    split configuration, and applied by tiles_for; the tuned plan still
    gives every product bitwise equal to its single call."""
    from paper_1106_1347_amd.tune import POLICIES, SPLIT_POLICIES, SPLIT_TILE_CODES, TileTuner

    cfg = mmm.Config(split_type="bf16", split_slices=6)
    shapes = synth.batch_shapes(24, 21, 16, 300)
    probs = [(p[0], p[1], p[2], p[3]) for p in make_problems(shapes, 700, ["dgemm", "split"], [0])]
    t = TileTuner(path=str(tmp_path / "tiles.json"))
    t.tune([s for g, s in enumerate(shapes) if g % 2 == 0], reps=2, split=[s for g, s in enumerate(shapes) if g % 2 == 1],
           split_config=cfg)
    pol, spol = t.tune_batch(probs, cfg, reps=2)
    assert pol in POLICIES and set(t.timings[t._policy_key(cfg, "dgemm")]) == set(POLICIES)
    assert spol in SPLIT_POLICIES and set(t.timings[t._policy_key(cfg, "split")]) == set(SPLIT_POLICIES)
    tiles = t.tiles_for(probs, cfg)
    for (A, B, C, m), tile in zip(probs, tiles):
        if m == "dgemm" and pol != "per-class":
            assert tile == pol
        if m == "split" and spol != "per-class":
            assert tile == SPLIT_TILE_CODES[spol]
    t2 = TileTuner(path=str(tmp_path / "tiles.json"))
    assert t2.tiles_for(probs, cfg) == tiles and t2.tune_batch(probs, cfg) == (pol, spol)
    plan = mmm.Batch([(A, B, C, m, 0, tile) for (A, B, C, m), tile in zip(probs, tiles)], cfg)
    plan.launch()
    torch.cuda.synchronize()
    for (A, B, C, m) in probs:
        w = single(mmm, A, B, m, 0, cfg)
        assert torch.equal(C.view(torch.int64), w.view(torch.int64))
    plan.close()


def test_autotuner_picks_and_persists(mmm, tmp_path):
    from paper_1106_1347_amd.tune import TileTuner

    t = TileTuner(path=str(tmp_path / "tiles.json"))
    shapes = [(64, 64, 64)] * 8 + [(512, 300, 512)] * 4
    table = t.tune(shapes, reps=3)
    assert len(table) == 2 and all(v in ("128x128", "64x64", "128x64") for v in table.values())
    t2 = TileTuner(path=str(tmp_path / "tiles.json"))
    assert t2.tile_for(64, 64, 64) == table[t.key((6, 6))]
