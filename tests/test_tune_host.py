"""Host-side checks of the tile autotuner's shape classes and cache (no GPU
measurement: a cache written beforehand is read back)."""
import json

from paper_1106_1347_amd import tune


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
