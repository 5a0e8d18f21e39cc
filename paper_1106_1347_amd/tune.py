"""Autotuner for the tile shapes of batched products.

Problems are grouped into shape classes (powers of two of max(N, M) and of
P).  For each class the tuner builds a batch of that class's problems once
per candidate tile shape, times the graph launch with HIP events and keeps
the fastest.  DGEMM problems choose among three tile shapes, split problems
(per digit type and count) between the wide tile and the narrow one (half
its rows).  A class timed alone has the chip to itself, while in a mixed
batch the FP64 groups share it with the split branch (their grids then leave
registers free for it), so a second step times the whole batch under a few
DGEMM tile policies -- the per-class choices, the library's own rule, and
each shape for every class -- and keeps the fastest for batches with that
split configuration, then does the same for the split tiles (per-class,
the library's rule, all wide, all narrow) under the chosen DGEMM policy.  Choices persist in a JSON cache keyed by device
architecture, method, shape class and data type (the policy by the split
configuration), so a later process picks them up without re-measuring.

    tuner = TileTuner()                          # loads the cache if present
    tuner.tune(dgemm_shapes, split=split_shapes, split_config=cfg)
    tuner.tune_batch(problems, cfg)              # (A, B, C, method) tuples of the batch
    tiles = tuner.tiles_for(problems, cfg)       # one tile per problem, for Batch
    tile = tuner.tile_for(N, P, M)               # "128x128", "64x64", ... or "auto"
    tile = tuner.tile_for(N, P, M, "split", cfg) # "wide", "narrow" or "auto"
"""
import json
import math
import os
from typing import Dict, Iterable, Optional, Sequence, Tuple

import torch

from ._lib import Batch, Config

CANDIDATES = ("128x128", "64x64", "128x64")
SPLIT_CANDIDATES = ("wide", "narrow")
SPLIT_TILE_CODES = {"auto": 0, "wide": 1, "narrow": 2}
# DGEMM tile policies of a whole batch: the per-class choices, the library's
# rule ("auto"), or one shape for every class
POLICIES = ("per-class", "auto") + CANDIDATES
# and of its split problems
SPLIT_POLICIES = ("per-class",) + tuple(SPLIT_TILE_CODES)


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
        self.timings: Dict[str, Dict[str, float]] = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.table = json.load(f)

    def _arch(self) -> str:
        if torch.cuda.is_available():
            props = torch.cuda.get_device_properties(self.device)
            return getattr(props, "gcnArchName", "unknown").split(":")[0]
        return "unknown"

    def key(self, cls: Tuple[int, int], method: str = "dgemm", config: Optional[Config] = None) -> str:
        if method == "dgemm":
            return "%s/dgemm/f64/n%d_p%d" % (self.arch, cls[0], cls[1])
        c = config or Config()
        return "%s/split/%s_s%d/n%d_p%d" % (self.arch, c.split_type, c.split_slices, cls[0], cls[1])

    def tile_for(self, N: int, P: int, M: int, method: str = "dgemm", config: Optional[Config] = None):
        """The tile a batch problem should request: a DGEMM tile name, or for
        split problems the integer code of the chosen variant."""
        t = self.table.get(self.key(shape_class(N, P, M), method, config), "auto")
        return t if method == "dgemm" else SPLIT_TILE_CODES[t]

    def _policy_key(self, config: Optional[Config], method: str = "dgemm") -> str:
        c = config or Config()
        return "%s/batch/%s_policy/with_%s_s%d_b%d" % (self.arch, method, c.split_type, c.split_slices, c.split_bits)

    def tiles_for(self, problems: Sequence[tuple], config: Optional[Config] = None) -> list:
        """One tile per problem of a batch ((A, B, C, method) tuples): DGEMM
        problems and split problems follow the policies ``tune_batch`` chose
        for batches with this split configuration (the per-class choices
        when none was chosen)."""
        pol = {m: self.table.get(self._policy_key(config, m), "per-class") for m in ("dgemm", "split")}
        out = []
        for p in problems:
            A, B, m = p[0], p[1], p[3]
            if pol[m] == "per-class":
                out.append(self.tile_for(A.shape[0], A.shape[1], B.shape[1], m, config))
            else:
                out.append(pol[m] if m == "dgemm" else SPLIT_TILE_CODES[pol[m]])
        return out

    def tune_batch(self, problems: Sequence[tuple], config: Optional[Config] = None, reps: int = 10) -> Tuple[str, str]:
        """Time the whole batch under each DGEMM tile policy and keep the
        fastest for batches with this split configuration, then likewise for
        the split tiles under that DGEMM policy (a policy the cache holds is
        kept).  Returns the (DGEMM, split) policies."""
        for method, pols in (("dgemm", POLICIES), ("split", SPLIT_POLICIES)):
            k = self._policy_key(config, method)
            if k in self.table:
                continue
            res = {}
            for pol in pols:
                self.table[k] = pol
                tiles = self.tiles_for(problems, config)
                res[pol] = self._time([(p[0], p[1], p[2], p[3], 0, t) for p, t in zip(problems, tiles)], config, reps)
            self.timings[k] = res
            self.table[k] = min(res, key=res.get)
        self.save()
        return self.table[self._policy_key(config, "dgemm")], self.table[self._policy_key(config, "split")]

    def _time(self, problems, config, reps):
        b = Batch(problems, config)
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
        return sorted(times)[len(times) // 2]

    def _tune_classes(self, shapes, method, config, candidates, reps, max_per_class):
        by_cls: Dict[Tuple[int, int], list] = {}
        for s in shapes:
            by_cls.setdefault(shape_class(*s), []).append(s)
        dev = torch.device("cuda", self.device)
        for cls, group in sorted(by_cls.items()):
            k = self.key(cls, method, config)
            if k in self.table:
                continue
            group = group[:max_per_class]
            mats = [(torch.rand(N, P, dtype=torch.float64, device=dev), torch.rand(P, M, dtype=torch.float64, device=dev),
                     torch.empty(N, M, dtype=torch.float64, device=dev)) for (N, P, M) in group]
            res = {}
            for tile in candidates:
                code = tile if method == "dgemm" else SPLIT_TILE_CODES[tile]
                res[tile] = self._time([(A, B, C, method, 0, code) for (A, B, C) in mats], config, reps)
            self.timings[k] = res
            self.table[k] = min(res, key=res.get)

    def tune(self, shapes: Iterable[Tuple[int, int, int]], reps: int = 5, max_per_class: int = 64,
             split: Optional[Sequence[Tuple[int, int, int]]] = None,
             split_config: Optional[Config] = None) -> Dict[str, str]:
        """Measure every class of ``shapes`` (DGEMM) and of ``split`` (split
        products with ``split_config``) that the cache does not hold yet."""
        self._tune_classes(list(shapes), "dgemm", Config(), CANDIDATES, reps, max_per_class)
        if split:
            self._tune_classes(list(split), "split", split_config or Config(), SPLIT_CANDIDATES, reps, max_per_class)
        self.save()
        return self.table

    def summary(self) -> Dict[str, object]:
        """Chosen tile per class (and the measured candidates of the classes
        tuned by this process)."""
        return {"choices": dict(sorted(self.table.items())), "measured_ms": dict(sorted(self.timings.items()))}

    def save(self) -> None:
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
