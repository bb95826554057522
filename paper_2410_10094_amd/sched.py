"""Grouping of contractions into batches (host-side scheduling policy).

A batch runs as one packed contraction whose Y free key is as wide as the
widest member's, so a member whose own Y free key is narrow enough for the
dense LDS accumulator (at most 13 bits) loses it when batched with a wide
one.  Members are therefore bucketed by that shape class before they are cut
into batches under a budget of expected products."""
from __future__ import annotations

from typing import Callable, Dict, List, Sequence

DENSE_Y_BITS = 13  # widest Y free key the dense block accumulator takes
BATCH_MAX = 4096   # contractions per batch (sptc_batch_plan)


def bits_for(d: int) -> int:
    """Bits of a coordinate field for a mode of length d."""
    return 0 if d <= 1 else (int(d) - 1).bit_length()


def y_free_bits(y_dims: Sequence[int], cy: Sequence[int]) -> int:
    return sum(bits_for(d) for m, d in enumerate(y_dims) if m not in set(cy))


def shape_class(y_dims: Sequence[int], cy: Sequence[int]) -> str:
    return "dense" if y_free_bits(y_dims, cy) <= DENSE_Y_BITS else "hash"


def estimate_products(p) -> float:
    """Cost estimate of a contraction before pass 1: nnz_X * nnz_Y over the
    product of the contracted dims (exact in expectation for independent
    uniform coordinates)."""
    cells = 1
    for c in p.cx:
        cells *= int(p.X.dims[c])
    return p.X.nnz * p.Y.nnz / max(cells, 1)


def make_batches(items: Sequence, cost: Callable[[object], float], klass: Callable[[object], str],
                 budget: float, max_count: int = BATCH_MAX) -> List[List[int]]:
    """Indices of ``items`` cut into batches: same class within a batch,
    arrival order within a class, at most ``budget`` total cost (a single
    item above it forms its own batch) and ``max_count`` items."""
    buckets: Dict[str, List[int]] = {}
    for i, it in enumerate(items):
        buckets.setdefault(klass(it), []).append(i)
    out = []
    for idxs in buckets.values():
        cur, acc = [], 0.0
        for i in idxs:
            c = cost(items[i])
            if cur and (acc + c > budget or len(cur) >= max_count):
                out.append(cur)
                cur, acc = [], 0.0
            cur.append(i)
            acc += c
        if cur:
            out.append(cur)
    out.sort(key=lambda b: b[0])
    return out
