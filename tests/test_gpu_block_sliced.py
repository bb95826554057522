"""The dense block class (Y free key of at most 13 bits, large X groups),
walked as (group, slice of the Y free key space) tiles: runs short enough
to be sorted and runs cut slice by slice without sorting, every lanes-per-
entry variant, the smallest and the largest accumulator, repeated Y
coordinates and explicit zeros, tiles placed by an atomic each or by a
count pass and a scan, and small groups accumulated whole in a dense row.
Against the oracle, element by element."""
import numpy as np
import pytest

from paper_2410_10094_amd.workloads import Coo, Problem
from tests.gpu_common import assert_parity, log, run_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _tensor(rng, dims, nnz, duplicates=False, zeros=0.0):
    cells = int(np.prod(dims))
    if duplicates:
        lin = rng.integers(0, cells, size=nnz)
    else:
        lin = rng.choice(cells, size=min(nnz, cells), replace=False)
    idx = np.stack(np.unravel_index(lin, dims)).astype(np.int32)
    val = rng.uniform(-1.0, 1.0, size=idx.shape[1])
    val[val == 0.0] = 0.5
    if zeros:
        val[rng.random(idx.shape[1]) < zeros] = 0.0
    return Coo(tuple(dims), idx, val)


def _matrix_like(seed, rows, keys, cols, nnz_x, nnz_y, name, duplicates=False, zeros=0.0):
    """X [rows, keys] (free mode 0) times Y [keys, cols] (free mode 1)."""
    rng = np.random.default_rng(seed)
    X = _tensor(rng, (rows, keys), nnz_x, zeros=zeros)
    Y = _tensor(rng, (keys, cols), nnz_y, duplicates=duplicates, zeros=zeros)
    return Problem(name, X, Y, (1,), (0,))


CASES = [
    # runs of ~100 entries (sorted), ~12 per slice: 16 lanes per entry
    ("short-runs", lambda: _matrix_like(1, 300, 600, 4096, 60_000, 60_000, "short-runs")),
    # runs of ~400 (sorted): 32 lanes per entry
    ("mid-runs", lambda: _matrix_like(2, 200, 150, 4096, 20_000, 60_000, "mid-runs")),
    # runs of ~3,000 entries: longer than a workgroup sorts, cut slice by slice
    ("long-runs", lambda: _matrix_like(3, 64, 8, 4096, 400, 24_000, "long-runs")),
    # both kinds of run in one Y, repeated Y coordinates
    ("mixed-runs-repeats", lambda: _matrix_like(4, 128, 40, 2048, 3_000, 40_000, "mixed-runs-repeats",
                                                duplicates=True)),
    # smallest accumulator: a 6-bit Y free key (1024 cells, 128 per slice)
    ("six-bit-cells", lambda: _matrix_like(5, 100, 400, 64, 40_000, 20_000, "six-bit-cells")),
    # largest: a 13-bit Y free key (8192 cells, 1024 per slice)
    ("thirteen-bit-cells", lambda: _matrix_like(6, 150, 100, 8192, 9_000, 150_000, "thirteen-bit-cells")),
    # explicit zero values: zero products still make structural outputs
    ("explicit-zeros", lambda: _matrix_like(7, 200, 150, 4096, 20_000, 60_000, "explicit-zeros", zeros=0.3)),
    # 3,000 columns (a 12-bit key, 4,096 cells): the slices cut 0..2,999,
    # 384 cells each, not the packed key space's 512
    ("uneven-key-range", lambda: _matrix_like(12, 200, 150, 3000, 20_000, 60_000, "uneven-key-range")),
    # few large tiles (about 24,000 products each)
    ("few-large-tiles", lambda: _matrix_like(9, 16, 64, 4096, 1024, 192_000, "few-large-tiles")),
    # groups of about 680 products: each accumulated whole, its dense row in
    # one workgroup, instead of eight thin tiles
    ("small-groups-dense-rows", lambda: _matrix_like(10, 40_000, 2_000, 4096, 200_000, 200_000,
                                                     "small-groups-dense-rows")),
]
DENSE_ROWS = {c[0]: c[0] == "small-groups-dense-rows" for c in CASES}


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_sliced_block_class(name, make):
    p = make()
    log(f"[sliced] {p.name} nnz {p.X.nnz}x{p.Y.nnz}")
    info, gidx, gval = run_gpu(p)
    assert info["classes"]["block"] > 0 and not info["block_mfma"], info["classes"]
    assert info["block_dense_rows"] == DENSE_ROWS[name], (info["products"], info["classes"])
    assert not info["block_tiles_scanned"]
    assert_parity(p, gidx, gval)


def test_many_tiles_counted_then_placed_by_a_scan():
    """Over 131,072 tiles (16,400 groups x 8 slices) of 2,560 products
    (groups of 20,480: above the dense rows' 16,384): each tile's outputs are
    counted, a scan places them, and a second walk writes them (no atomic
    per tile).  336M products, against the oracle."""
    import oracle
    p = _matrix_like(11, 16_400, 64, 4096, 16_400 * 64, 64 * 320, "many-tiles")
    log(f"[sliced] {p.name} nnz {p.X.nnz}x{p.Y.nnz}")
    info, gidx, gval = run_gpu(p)
    assert info["block_tiles_scanned"] and not info["block_dense_rows"], (info["products"], info["classes"])
    assert_parity(p, gidx, gval, oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=16))


def test_sliced_block_class_order4():
    """Order-4 operands contracted on two modes, as the block-sparse
    workloads: rows and cells are packed keys of two modes each."""
    rng = np.random.default_rng(8)
    X = _tensor(rng, (12, 10, 20, 20), 30_000)
    Y = _tensor(rng, (20, 20, 30, 40), 120_000)
    p = Problem("order4-two-pairs", X, Y, (2, 3), (0, 1))
    log(f"[sliced] {p.name} nnz {p.X.nnz}x{p.Y.nnz}")
    info, gidx, gval = run_gpu(p)
    assert info["classes"]["block"] > 0, info["classes"]
    assert_parity(p, gidx, gval)


def test_sliced_block_class_two_uneven_free_modes():
    """A Y free key of two modes of 37 and 50 (6 bits each): the keys in use
    end at 36 * 64 + 49, so the slices are 320 cells wide, and the last
    slice holds the largest coordinates (every (y1, y2) pair occurs)."""
    rng = np.random.default_rng(13)
    X = _tensor(rng, (200, 40), 8_000)
    Y = _tensor(rng, (40, 37, 50), 37_000)
    assert Y.idx[1].max() == 36 and Y.idx[2].max() == 49
    p = Problem("two-uneven-free-modes", X, Y, (1,), (0,))
    log(f"[sliced] {p.name} nnz {p.X.nnz}x{p.Y.nnz}")
    info, gidx, gval = run_gpu(p)
    assert info["classes"]["block"] > 0 and not info["block_mfma"], info["classes"]
    assert not info["block_dense_rows"], (info["products"], info["classes"])
    assert_parity(p, gidx, gval)

