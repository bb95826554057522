"""Autotuner for batched contraction: picks the hash-table load factor, the
batch size (expected products per batch) and the tile size of the
single-entry (direct) class by timing candidates on a sample of the
workload, and caches the choice per device and shape class.

The load factor sizes every hashed key table (pow2 >= keys / load factor;
the paper's x1.3 rule is a load factor of 1/1.3).  The batch budget decides
how many contractions share one packed plan: larger batches amortise launches
and synchronisations, smaller ones keep tables and outputs cache-sized.  The
tile is the number of products a workgroup of the direct class takes (each
lane keeps tile / 256 loads in flight): larger tiles hide more latency,
smaller ones spread short classes over more of the GPU."""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Callable, Dict, Iterable, Optional, Sequence, Tuple

LOAD_FACTORS = (0.5, 0.625, 1 / 1.3, 0.9)
BATCH_BUDGETS = (2.5e8, 5e8, 1e9, 2e9)
TILES = (1024, 2048)


def choose(timings: Dict[Tuple, float]) -> Tuple:
    """The fastest candidate; ties go to the larger load factor (less memory),
    then the larger batch, then the larger tile."""
    return min(timings, key=lambda c: (timings[c],) + tuple(-x for x in c))


def signature(problems: Iterable, klass: Callable) -> str:
    """Shape class of a workload sample: its shape classes and order mix."""
    classes = sorted({klass(p) for p in problems})
    orders = sorted({(p.X.order, p.Y.order, len(p.cx)) for p in problems})
    return f"{'+'.join(classes)}|{len(orders)}-order-mixes"


class Autotuner:
    def __init__(self, cache_path: Optional[str] = None):
        self.cache_path = cache_path
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def save(self):
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    def tune(self, key: str, run: Callable[[float, float, int], float],
             load_factors: Sequence[float] = LOAD_FACTORS, budgets: Sequence[float] = BATCH_BUDGETS,
             tiles: Sequence[int] = TILES, reps: int = 1) -> dict:
        """run(load_factor, budget, tile) -> seconds for one pass of the
        sample.  Returns (and caches under key) the choice and every timing."""
        if key in self.cache:
            return self.cache[key]
        timings = {}
        t0 = time.perf_counter()
        for lf, bud, tile in itertools.product(load_factors, budgets, tiles):
            timings[(lf, bud, tile)] = min(run(lf, bud, tile) for _ in range(max(reps, 1)))
        lf, bud, tile = choose(timings)
        rec = {"load_factor": lf, "batch_products": bud, "tile": tile, "tuning_seconds": time.perf_counter() - t0,
               "timings": {f"{a:.4f}/{b:.3g}/{c}": round(t, 6) for (a, b, c), t in timings.items()}}
        self.cache[key] = rec
        self.save()
        return rec


def torch_batch_runner(draws, dev, klass):
    """run(load_factor, budget, tile) for sptc_batch_* on device tensors: one
    pass over the draws in batches cut by sched.make_batches (plan +
    execute)."""
    import torch

    import paper_2410_10094_amd as sptc
    from . import sched

    def run(lf: float, budget: float, tile: int = 0) -> float:
        cut = sched.make_batches(draws, sched.estimate_products, klass, budget)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for members in cut:
            opt = sptc.default_options(load_factor=lf, tile=tile)
            with sptc.batch([(dev[i][0], dev[i][1], draws[i].cx, draws[i].cy) for i in members],
                            options=opt) as bt:
                idx, val, nnz = bt.allocate_outputs()
                bt.execute_into(idx, val, nnz)
                torch.cuda.synchronize()
        return time.perf_counter() - t0

    return run
