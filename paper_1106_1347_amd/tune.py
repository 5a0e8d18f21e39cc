"""Autotuner for the DGEMM tile shape of batched products.

Problems are grouped into shape classes (powers of two of max(N, M) and of
P).  For each class the tuner builds a batch of that class's problems once
per candidate tile shape, times the graph launch with HIP events and keeps
the fastest.  Choices persist in a JSON cache keyed by device architecture,
method, shape class and data type, so a later process picks them up
without re-measuring.

    tuner = TileTuner()                      # loads the cache if present
    tuner.tune(shapes)                       # measures classes not cached
    tile = tuner.tile_for(N, P, M)           # "128x128", "64x64", ... or "auto"
"""
import json
import math
import os
from typing import Dict, Iterable, Optional, Tuple

import torch

from ._lib import Batch, Config

CANDIDATES = ("128x128", "64x64", "128x64")


def default_cache_path() -> str:
    return os.environ.get("MMM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mmm", "tiles.json"))


def shape_class(N: int, P: int, M: int) -> Tuple[int, int]:
    mx = max(N, M, 1)
    return (int(math.ceil(math.log2(mx))), int(math.ceil(math.log2(max(P, 1)))))


class TileTuner:
    def __init__(self, path: Optional[str] = None, device: int = 0):
        self.path = path or default_cache_path()
        self.device = device
        self.arch = self._arch()
        self.table: Dict[str, str] = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.table = json.load(f)

    def _arch(self) -> str:
        if torch.cuda.is_available():
            props = torch.cuda.get_device_properties(self.device)
            return getattr(props, "gcnArchName", "unknown").split(":")[0]
        return "unknown"

    def key(self, cls: Tuple[int, int]) -> str:
        return "%s/dgemm/f64/n%d_p%d" % (self.arch, cls[0], cls[1])

    def tile_for(self, N: int, P: int, M: int) -> str:
        return self.table.get(self.key(shape_class(N, P, M)), "auto")

    def tune(self, shapes: Iterable[Tuple[int, int, int]], reps: int = 5, max_per_class: int = 64) -> Dict[str, str]:
        by_cls: Dict[Tuple[int, int], list] = {}
        for s in shapes:
            by_cls.setdefault(shape_class(*s), []).append(s)
        dev = torch.device("cuda", self.device)
        for cls, group in sorted(by_cls.items()):
            k = self.key(cls)
            if k in self.table:
                continue
            group = group[:max_per_class]
            mats = [(torch.rand(N, P, dtype=torch.float64, device=dev), torch.rand(P, M, dtype=torch.float64, device=dev),
                     torch.empty(N, M, dtype=torch.float64, device=dev)) for (N, P, M) in group]
            best, best_ms = None, float("inf")
            for tile in CANDIDATES:
                b = Batch([(A, B, C, "dgemm", 0, tile) for (A, B, C) in mats], Config())
                b.launch()
                torch.cuda.synchronize()
                times = []
                for _ in range(reps):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    b.launch()
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                b.close()
                ms = sorted(times)[len(times) // 2]
                if ms < best_ms:
                    best, best_ms = tile, ms
            self.table[k] = best
        self.save()
        return self.table

    def save(self) -> None:
        os.makedirs(os.path.dirname(self.path), exist_ok=True)
        tmp = self.path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
