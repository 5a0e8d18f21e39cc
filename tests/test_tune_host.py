"""Host-side checks of the tile autotuner's shape classes and cache (no GPU
measurement: a cache written beforehand is read back)."""
import json

import torch

from paper_1106_1347_amd import tune
from paper_1106_1347_amd._lib import Config


def test_shape_classes():
    assert tune.shape_class(1, 1, 1) == (0, 0)
    assert tune.shape_class(16, 16, 16) == (4, 4)
    assert tune.shape_class(17, 16, 3) == (5, 4)  # max(N, M) rounds up to the next power of two
    assert tune.shape_class(300, 200, 400) == (9, 8)
    assert tune.shape_class(512, 513, 64) == (9, 10)
    assert tune.shape_class(0, 0, 0) == (0, 0)  # empty products share the smallest class


def test_cached_choices_are_read_back(tmp_path):
    path = tmp_path / "tiles.json"
    t0 = tune.TileTuner(path=str(path))
    key = t0.key((9, 8))
    assert key.endswith("/dgemm/f64/n9_p8")
    path.write_text(json.dumps({key: "64x64"}))
    t = tune.TileTuner(path=str(path))
    assert t.tile_for(300, 200, 400) == "64x64"
    assert t.tile_for(257, 129, 2) == "64x64"  # same class
    assert t.tile_for(2048, 200, 400) == "auto"  # class never measured
    # a class already in the cache is not measured again
    assert t.tune([(300, 200, 400)]) == t.table


def test_batch_policies_give_one_tile_per_problem(tmp_path):
    # CPU tensors stand in for the operands: only their shapes are read
    def prob(N, P, M, m):
        return (torch.empty(N, P), torch.empty(P, M), torch.empty(N, M), m)

    probs = [prob(300, 200, 400, "dgemm"), prob(40, 30, 20, "split"), prob(2048, 100, 64, "dgemm"),
             prob(300, 200, 400, "split")]
    cfg = Config(split_type="bf16", split_slices=6)
    path = tmp_path / "tiles.json"
    t = tune.TileTuner(path=str(path))
    t.table[t.key((9, 8))] = "64x64"
    t.table[t.key((9, 8), "split", cfg)] = "narrow"
    # no policy chosen yet: the per-class choices, "auto" for classes never measured
    assert t.tiles_for(probs, cfg) == ["64x64", 0, "auto", tune.SPLIT_TILE_CODES["narrow"]]
    kd, ks = t._policy_key(cfg, "dgemm"), t._policy_key(cfg, "split")
    assert kd != ks and kd.endswith("/batch/dgemm_policy/with_bf16_s6_b0")
    # a policy is kept per split configuration
    assert t._policy_key(Config(split_type="bf16", split_slices=5), "dgemm") != kd
    assert t._policy_key(Config(split_type="bf16", split_slices=6, split_bits=9), "dgemm") != kd
    t.table[kd] = "128x64"
    t.table[ks] = "wide"
    assert t.tiles_for(probs, cfg) == ["128x64", 1, "128x64", 1]
    t.table[kd] = "auto"
    t.table[ks] = "per-class"
    assert t.tiles_for(probs, cfg) == ["auto", 0, "auto", tune.SPLIT_TILE_CODES["narrow"]]
    # another split configuration has no policy: per-class for both kinds
    other = Config(split_type="int8", split_slices=7)
    assert t.tiles_for(probs, other) == ["64x64", 0, "auto", 0]
    # chosen policies are cached: a later process reads them back and does not measure again
    t.table[kd] = "64x64"
    t.save()
    t2 = tune.TileTuner(path=str(path))
    assert t2.tiles_for(probs, cfg) == ["64x64", 0, "64x64", tune.SPLIT_TILE_CODES["narrow"]]
    assert t2.tune_batch(probs, cfg) == ("64x64", "per-class")
    for pol in tune.POLICIES[1:]:
        assert pol == "auto" or pol in tune.CANDIDATES
    assert set(tune.SPLIT_POLICIES[1:]) == set(tune.SPLIT_TILE_CODES)
