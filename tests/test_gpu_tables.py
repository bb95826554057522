"""Grouping tables of the plan against the oracle: the compact 64-bit-slot X
table (hashed X free keys of 17..31 bits) with groups of one and of several
entries, repeated X coordinates, and inputs small enough that every scan is
a single tile."""
import numpy as np
import pytest

from paper_2410_10094_amd.workloads import Coo, Problem
from tests.gpu_common import assert_parity, run_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _wide_x(seed, a, b, c, nx, f, ny, duplicates=False):
    """X (a, b, c), Y (c, f); X mode 2 contracts with Y mode 0.  The X free
    key is log2(a) + log2(b) bits wide."""
    rng = np.random.default_rng(seed)
    xi = np.stack([rng.integers(0, a, nx), rng.integers(0, b, nx), rng.integers(0, c, nx)]).astype(np.int32)
    if not duplicates:
        xi = np.unique(xi, axis=1)
        xi = xi[:, rng.permutation(xi.shape[1])]
    yi = np.unique(np.stack([rng.integers(0, c, ny), rng.integers(0, f, ny)]).astype(np.int32), axis=1)
    X = Coo((a, b, c), xi, rng.uniform(-1, 1, xi.shape[1]))
    Y = Coo((c, f), yi, rng.uniform(-1, 1, yi.shape[1]))
    return Problem(f"wide-x-{seed}", X, Y, (2,), (0,))


@pytest.mark.parametrize("seed,a,b,nx,dup", [
    (61, 512, 512, 300_000, False),      # 18-bit key: about 30% of the keys hold several entries
    (62, 1 << 15, 1 << 16, 200_000, False),  # 31 bits, the widest the compact table takes: nearly all single
    (63, 600, 700, 150_000, True),       # repeated X coordinates (their products add up)
])
def test_compact_x_table(seed, a, b, nx, dup):
    p = _wide_x(seed, a, b, 64, nx, 100, 640, duplicates=dup)
    info, gidx, gval = run_gpu(p)
    assert info["x_groups"] > 0
    assert_parity(p, gidx, gval)


def test_single_tile_scans():
    """Fewer than 4,096 entries, keys and groups: every scan is one tile."""
    p = _wide_x(64, 40, 50, 30, 1_500, 20, 300)
    info, gidx, gval = run_gpu(p)
    assert_parity(p, gidx, gval)
