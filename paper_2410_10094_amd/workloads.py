"""Seeded synthetic sparse tensors shaped like the workloads the method targets.

This module only draws inputs: coordinates, values and the contracted-mode
pairs.  It holds none of the contraction's arithmetic, so the GPU path and the
CPU oracle can both be fed from it without sharing any computation.

Tensors are COO (paper section 2.1, Fig. 1): ``idx`` is a mode-major int32
array ``[order, nnz]`` of 0-based coordinates (``0 <= i_k < I_k``, section
2.1.1) and ``val`` a float64 array ``[nnz]``.  Values are never exactly zero:
COO omits zero entries, so the generators redraw an exact zero.

Every generator takes an integer ``seed`` and builds a numpy ``PCG64`` stream
from ``SeedSequence(seed)``; X and Y draw from independent child sequences.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

BASE_SEED = 241010094


@dataclasses.dataclass
class Coo:
    """A host COO tensor: ``dims`` (tuple of mode lengths), ``idx`` int32
    ``[order, nnz]`` (mode-major), ``val`` float64 ``[nnz]``."""

    dims: Tuple[int, ...]
    idx: np.ndarray
    val: np.ndarray

    def __post_init__(self):
        self.dims = tuple(int(d) for d in self.dims)
        self.idx = np.ascontiguousarray(self.idx, dtype=np.int32).reshape(len(self.dims), -1)
        self.val = np.ascontiguousarray(self.val, dtype=np.float64).reshape(-1)
        if self.idx.shape[1] != self.val.shape[0]:
            raise ValueError("idx and val disagree on nnz")

    @property
    def order(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])


@dataclasses.dataclass
class Problem:
    """One contraction: ``Z = X (x)_{cy}^{cx} Y`` (paper Eq. 1), modes 0-based."""

    name: str
    X: Coo
    Y: Coo
    cx: Tuple[int, ...]
    cy: Tuple[int, ...]

    def __post_init__(self):
        self.cx = tuple(int(c) for c in self.cx)
        self.cy = tuple(int(c) for c in self.cy)


def _streams(seed: int, n: int = 2):
    ss = np.random.SeedSequence(int(seed))
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def nonzero_uniform(rng: np.random.Generator, n: int, lo=-1.0, hi=1.0) -> np.ndarray:
    """U[lo, hi) values with exact zeros redrawn."""
    v = rng.uniform(lo, hi, size=n)
    bad = v == 0.0
    while bad.any():
        v[bad] = rng.uniform(lo, hi, size=int(bad.sum()))
        bad = v == 0.0
    return v


def _linear(coords: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    lin = np.zeros(coords.shape[1], dtype=np.int64)
    for m, d in enumerate(dims):
        lin = lin * int(d) + coords[m].astype(np.int64)
    return lin


def unique_coords(rng: np.random.Generator, dims: Sequence[int], nnz: int, draw_mode=None) -> np.ndarray:
    """``nnz`` distinct coordinates in random order.

    ``draw_mode(rng, n)`` may return an int64 ``[order, n]`` draw of candidate
    coordinates (default: each mode uniform).  Duplicates are dropped keeping
    the first occurrence, and the set is topped up until it holds ``nnz``.
    """
    dims = [int(d) for d in dims]
    total = math.prod(dims)
    if nnz > total:
        raise ValueError("nnz exceeds the number of cells")
    if draw_mode is None and total <= 4 * max(nnz, 1) and total <= 50_000_000:
        lin = rng.choice(total, size=nnz, replace=False)
        return np.stack(np.unravel_index(lin, dims)).astype(np.int32).reshape(len(dims), nnz)

    def draw(n):
        if draw_mode is not None:
            return np.asarray(draw_mode(rng, n), dtype=np.int64)
        return np.stack([rng.integers(0, d, size=n, dtype=np.int64) for d in dims])

    have = np.zeros((len(dims), 0), dtype=np.int64)
    have_lin = np.zeros(0, dtype=np.int64)
    while have.shape[1] < nnz:
        need = nnz - have.shape[1]
        cand = draw(int(need * 1.05) + 16)
        both = np.concatenate([have, cand], axis=1)
        lin = np.concatenate([have_lin, _linear(cand, dims)])
        _, first = np.unique(lin, return_index=True)
        first.sort()  # keep draw order: no sorting structure leaks into the input
        have, have_lin = both[:, first], lin[first]
    return have[:, :nnz].astype(np.int32)


# ----------------------------------------------------------------------------
# The workloads
# ----------------------------------------------------------------------------

def plain(seed: int = BASE_SEED + 1, n: int = 64, nnz: int = 2621) -> Problem:
    """Plain order-3 SpTC: X, Y on ``n^3`` with ``nnz`` distinct uniform
    coordinates each (2,621 of 64^3 is 1% density), values U[-1,1); X mode 2
    contracts with Y mode 0, so the output has order 4."""
    rx, ry = _streams(seed)
    dims = (n, n, n)
    X = Coo(dims, unique_coords(rx, dims, nnz), nonzero_uniform(rx, nnz))
    Y = Coo(dims, unique_coords(ry, dims, nnz), nonzero_uniform(ry, nnz))
    return Problem(f"plain-{n}^3-nnz{nnz}", X, Y, (2,), (0,))


def _block_sparse_tensor(rng, n, block, p_block, p_fill, decay):
    nb = n // block
    present = np.flatnonzero(rng.random(nb ** 4) < p_block)
    bcoords = np.stack(np.unravel_index(present, (nb,) * 4))  # [4, nblocks]
    cells = block ** 4
    inblock = np.stack(np.unravel_index(np.arange(cells), (block,) * 4))  # [4, cells]
    keep = rng.random((present.size, cells)) < p_fill
    bi, ci = np.nonzero(keep)
    coords = (bcoords[:, bi] * block + inblock[:, ci]).astype(np.int32)
    perm = rng.permutation(coords.shape[1])
    coords = coords[:, perm]
    g = rng.standard_normal(coords.shape[1])
    g[g == 0.0] = 1.0
    val = g * np.exp(-np.abs(coords[0].astype(np.float64) - coords[1]) / decay)
    return Coo((n,) * 4, coords, val)


def block_sparse(seed: int = BASE_SEED + 2, n: int = 48, block: int = 8, p_block: float = 0.1,
                 p_fill: float = 0.5, decay: float = 8.0) -> Problem:
    """Block-sparse order-4 x order-4 (electronic-structure-like): ``n^4`` dims
    cut into ``block^4`` blocks, each present with probability ``p_block``,
    each cell of a present block filled with probability ``p_fill``; values
    ``N(0,1) * exp(-|i-j|/decay)`` with i, j the coordinates of modes 0 and 1.
    X modes (2,3) contract with Y modes (0,1)."""
    rx, ry = _streams(seed)
    X = _block_sparse_tensor(rx, n, block, p_block, p_fill, decay)
    Y = _block_sparse_tensor(ry, n, block, p_block, p_fill, decay)
    return Problem(f"block-sparse-{n}^4-b{block}-p{p_block}-f{p_fill}", X, Y, (2, 3), (0, 1))


def zipf_ranks(rng, n: int, support: int, s: float) -> np.ndarray:
    """Ranks in 1..support with P(r) proportional to r^-s (inverse CDF)."""
    w = np.arange(1, support + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    r = np.searchsorted(cdf, rng.random(n), side="right") + 1
    return np.minimum(r, support)


def imbalanced(seed: int = BASE_SEED + 3, nnz_x: int = 10_000_000, nnz_y: int = 1_000_000,
               xdims=(1 << 17, 1 << 14, 1 << 15), ydims=(1 << 15, 1 << 12, 1 << 10),
               zipf_s: float = 1.2) -> Problem:
    """Imbalanced order-3 SpTC: X's contracting mode (2) is Zipf(s)
    distributed over its length, its other modes uniform; Y is uniform; X mode
    2 contracts with Y mode 0.  Coordinates are distinct, values U[-1,1)."""
    if xdims[2] != ydims[0]:
        raise ValueError("contracted modes must have equal length")
    rx, ry = _streams(seed)

    def draw_x(rng, n):
        return np.stack([rng.integers(0, xdims[0], size=n), rng.integers(0, xdims[1], size=n),
                         zipf_ranks(rng, n, xdims[2], zipf_s) - 1])

    X = Coo(xdims, unique_coords(rx, xdims, nnz_x, draw_x), nonzero_uniform(rx, nnz_x))
    Y = Coo(ydims, unique_coords(ry, ydims, nnz_y), nonzero_uniform(ry, nnz_y))
    return Problem(f"imbalanced-zipf{zipf_s}-{nnz_x}x{nnz_y}", X, Y, (2,), (0,))


def random_problem(seed: int, order_x: int, order_y: int, ncontract: int, dim_lo: int, dim_hi: int,
                   nnz_x: int, nnz_y: int, duplicates: bool = False) -> Problem:
    """A random contraction for tests: each dim uniform in [dim_lo, dim_hi],
    contracted modes drawn as distinct random choices, Y's contracted dims
    copied from X's.  With ``duplicates`` coordinates may repeat (COO with
    repeated coordinates)."""
    rng, rx, ry = _streams(seed, 3)
    xd = [int(d) for d in rng.integers(dim_lo, dim_hi + 1, size=order_x)]
    yd = [int(d) for d in rng.integers(dim_lo, dim_hi + 1, size=order_y)]
    cx = [int(c) for c in rng.permutation(order_x)[:ncontract]]
    cy = [int(c) for c in rng.permutation(order_y)[:ncontract]]
    for a, b in zip(cx, cy):
        yd[b] = xd[a]

    def make(r, dims, nnz):
        cells = math.prod(dims)
        if duplicates:
            coords = np.stack([r.integers(0, d, size=nnz) for d in dims]).astype(np.int32)
        else:
            coords = unique_coords(r, dims, min(nnz, cells))
        return Coo(dims, coords.reshape(len(dims), -1), nonzero_uniform(r, coords.reshape(len(dims), -1).shape[1]))

    return Problem(f"random-{seed}", make(rx, xd, nnz_x), make(ry, yd, nnz_y), cx, cy)


def batched_draw(seed: int, i: int, max_products: int = 1 << 28, nnz_lo: float = 1e3,
                 nnz_hi: float = 1e6) -> Problem:
    """Draw ``i`` of the batched workload: orders of X and Y uniform in
    {3,4,5}, 1-2 contracted pairs on distinct random modes, every dim uniform
    in [32, 4096] with Y's contracted dims copied from X's, nnz log-uniform in
    [nnz_lo, nnz_hi] clamped to 10% density, distinct coordinates, values
    U[-1,1).  A draw whose expected product count for uniform coordinates,
    nnz_X * nnz_Y / (product of the contracted dims), exceeds
    ``max_products`` is redrawn.  Draw i depends only on (seed, i)."""
    child = np.random.SeedSequence(int(seed), spawn_key=(int(i),))
    attempt = 0
    while True:
        ss = np.random.SeedSequence(child.entropy, spawn_key=child.spawn_key + (attempt,))
        rng, rx, ry = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
        ox, oy = int(rng.integers(3, 6)), int(rng.integers(3, 6))
        nc = int(rng.integers(1, 3))
        xd = [int(d) for d in rng.integers(32, 4097, size=ox)]
        yd = [int(d) for d in rng.integers(32, 4097, size=oy)]
        cx = [int(c) for c in rng.permutation(ox)[:nc]]
        cy = [int(c) for c in rng.permutation(oy)[:nc]]
        for a, b in zip(cx, cy):
            yd[b] = xd[a]
        nx = int(round(math.exp(rng.uniform(math.log(nnz_lo), math.log(nnz_hi)))))
        ny = int(round(math.exp(rng.uniform(math.log(nnz_lo), math.log(nnz_hi)))))
        nx = min(nx, max(1, math.prod(xd) // 10))
        ny = min(ny, max(1, math.prod(yd) // 10))
        expected = nx * ny / math.prod(xd[c] for c in cx)
        if expected <= max_products:
            X = Coo(xd, unique_coords(rx, xd, nx), nonzero_uniform(rx, nx))
            Y = Coo(yd, unique_coords(ry, yd, ny), nonzero_uniform(ry, ny))
            return Problem(f"batched-{i}", X, Y, cx, cy)
        attempt += 1


def batched_draws(seed: int = BASE_SEED + 4, count: int = 512, max_products: int = 1 << 28,
                  nnz_lo: float = 1e3, nnz_hi: float = 1e6) -> List[Problem]:
    """The first ``count`` draws of the batched workload (batched_draw)."""
    return [batched_draw(seed, i, max_products, nnz_lo, nnz_hi) for i in range(count)]


def expected_products(p: Problem) -> float:
    """nnz_X * nnz_Y / (product of the contracted dims): the product count
    for independent uniform coordinates."""
    return p.X.nnz * p.Y.nnz / math.prod(p.X.dims[c] for c in p.cx)


def paper_set(seed: int, mode_len: int, nnz: int, order_x: int = 5, order_y: int = 4) -> Problem:
    """Shapes of the paper's synthetic sets (Table 1, sets 1 and 2): an order-5
    tensor A and an order-4 tensor B with all modes of length ``mode_len``,
    random distinct coordinates and values, contracted along their second and
    third modes (modes 1 and 2, 0-based)."""
    rx, ry = _streams(seed)
    xd, yd = (mode_len,) * order_x, (mode_len,) * order_y
    X = Coo(xd, unique_coords(rx, xd, nnz), nonzero_uniform(rx, nnz))
    Y = Coo(yd, unique_coords(ry, yd, nnz), nonzero_uniform(ry, nnz))
    return Problem(f"paper-set-{mode_len}-o{order_x}x{order_y}-nnz{nnz}", X, Y, (1, 2), (1, 2))


# Named full-size workloads.
WORKLOADS = {
    "plain": lambda: plain(),
    "block-sparse": lambda: block_sparse(),
    "block-sparse-1.5M": lambda: block_sparse(p_block=0.565),
    "imbalanced": lambda: imbalanced(),
    # the largest shape of the synthetic sets' sweep (set 1, order 5 x 5)
    "paper-set-50-5x5-500K": lambda: paper_set(BASE_SEED + 10 + 5 + 5, 50, 500_000, 5, 5),
}
