"""Block class on the matrix cores (dense Y free keys, one contraction):
the same outputs as the oracle, with the tile edges ragged in every
dimension, runs spread over many inner steps, long runs and large groups,
repeated X and Y coordinates (summed), explicit zero values (outputs all the
same), and the plan's choice and fallback."""
import numpy as np
import pytest

from paper_2410_10094_amd import workloads as W
from paper_2410_10094_amd.workloads import Coo, Problem
from tests.gpu_common import assert_parity, log, run_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _opts(v):
    import paper_2410_10094_amd as sptc
    return sptc.default_options(block_mfma=v)


def _dense_random(seed, groups_x, c, free_y, nx, ny, duplicates=False, zeros=False, name=""):
    """X (a, b, c) with groups_x = a * b X free keys, Y (c, f0, f1) with
    free_y = f0 * f1 cells; X mode 2 contracts with Y mode 0."""
    rng = np.random.default_rng(seed)
    a = int(np.sqrt(groups_x))
    b = groups_x // a
    f0 = int(np.sqrt(free_y))
    f1 = free_y // f0
    xi = np.stack([rng.integers(0, a, nx), rng.integers(0, b, nx), rng.integers(0, c, nx)]).astype(np.int32)
    yi = np.stack([rng.integers(0, c, ny), rng.integers(0, f0, ny), rng.integers(0, f1, ny)]).astype(np.int32)
    if not duplicates:
        xi = np.unique(xi, axis=1)
        yi = np.unique(yi, axis=1)
        xi = xi[:, rng.permutation(xi.shape[1])]
        yi = yi[:, rng.permutation(yi.shape[1])]
    xv = W.nonzero_uniform(rng, xi.shape[1])
    yv = W.nonzero_uniform(rng, yi.shape[1])
    if zeros:
        xv[::13] = 0.0
        yv[::17] = 0.0
    return Problem(name or f"dense-{seed}", Coo((a, b, c), xi, xv), Coo((c, f0, f1), yi, yv), (2,), (0,))


def _problems():
    return [
        W.block_sparse(seed=5, n=24, block=4, p_block=0.5, p_fill=0.7),  # 9 x 9 tiles, 18 steps: whole tiles
        W.block_sparse(seed=6, n=20, block=4, p_block=0.6, p_fill=0.6),  # 400 rows, columns, runs: ragged
        _dense_random(31, 1200, 200, 900, 60_000, 60_000, name="dense-1200x900-200-runs"),
        _dense_random(32, 700, 1000, 3000, 90_000, 150_000, name="dense-700x3000-1000-runs"),
        _dense_random(33, 500, 150, 600, 40_000, 40_000, duplicates=True, zeros=True, name="duplicates-and-zeros"),
    ]


@pytest.mark.parametrize("p", _problems(), ids=lambda p: p.name)
def test_matrix_core_block_class_matches_oracle(p):
    log(f"[mfma] {p.name} nnz {p.X.nnz}x{p.Y.nnz}")
    info, gidx, gval = run_gpu(p, options=_opts(1))
    assert info["classes"]["block"] > 0, info["classes"]
    assert info["block_mfma"], info
    assert_parity(p, gidx, gval)


def test_auto_takes_the_matrix_cores_when_dense():
    p = _dense_random(34, 1024, 256, 1024, 120_000, 120_000, name="dense-auto")
    info, gidx, gval = run_gpu(p, options=_opts(-1))  # the cost rule decides
    assert info["classes"]["block"] > 500 and info["block_mfma"], info
    assert_parity(p, gidx, gval)


def test_default_is_the_sparse_walk():
    p = _dense_random(36, 1024, 256, 1024, 120_000, 120_000, name="dense-default")
    info, gidx, gval = run_gpu(p)  # default options: the matrix cores are opt-in
    assert info["classes"]["block"] > 500 and not info["block_mfma"], info
    assert_parity(p, gidx, gval)


def test_never_means_the_sparse_walk():
    p = _dense_random(35, 1024, 256, 1024, 120_000, 120_000, name="dense-never")
    info, gidx, gval = run_gpu(p, options=_opts(0))
    assert not info["block_mfma"]
    assert_parity(p, gidx, gval)


def test_non_finite_value_falls_back():
    """An Inf anywhere in Y rules the class out (0 * Inf in the zero padding
    would be NaN); the Inf sits in a run no X entry reaches, so the outputs
    stay finite and comparable."""
    p = _dense_random(36, 400, 100, 400, 20_000, 20_000, name="inf")
    yi = np.concatenate([p.Y.idx, np.array([[100], [0], [0]], np.int32)], axis=1)
    Y = Coo((101,) + tuple(p.Y.dims[1:]), yi, np.concatenate([p.Y.val, [np.inf]]))
    X = Coo((p.X.dims[0], p.X.dims[1], 101), p.X.idx, p.X.val)
    q = Problem("inf", X, Y, (2,), (0,))
    info, gidx, gval = run_gpu(q, options=_opts(1))
    assert info["classes"]["block"] > 0 and not info["block_mfma"], info
    assert_parity(q, gidx, gval)


def test_non_finite_x_value_falls_back():
    """An Inf among the X values rules the class out as well; it sits on a
    contracting key no Y entry has, so no product takes it and the outputs
    stay finite and comparable."""
    p = _dense_random(38, 400, 100, 400, 20_000, 20_000, name="xinf")
    xi = np.concatenate([p.X.idx, np.array([[0], [0], [100]], np.int32)], axis=1)
    X = Coo((p.X.dims[0], p.X.dims[1], 101), xi, np.concatenate([p.X.val, [np.inf]]))
    Y = Coo((101,) + tuple(p.Y.dims[1:]), p.Y.idx, p.Y.val)
    q = Problem("xinf", X, Y, (2,), (0,))
    info, gidx, gval = run_gpu(q, options=_opts(1))
    assert info["classes"]["block"] > 0 and not info["block_mfma"], info
    assert_parity(q, gidx, gval)


def test_long_y_runs_and_large_groups():
    """Runs and groups far longer than a step or a tile: a run of 3000 Y
    entries and a group of 6000 X entries spread over many steps."""
    rng = np.random.default_rng(37)
    p = _dense_random(37, 400, 100, 4096, 20_000, 20_000, name="long")
    ey = np.stack([np.zeros(3000, int), rng.integers(0, 64, 3000), rng.integers(0, 64, 3000)]).astype(np.int32)
    yi = np.unique(np.concatenate([p.Y.idx, ey], axis=1), axis=1)
    ex = np.stack([np.zeros(6000, int), np.zeros(6000, int), rng.integers(0, 100, 6000)]).astype(np.int32)
    xi = np.concatenate([p.X.idx, ex], axis=1)  # repeated X coordinates too
    q = Problem("long", Coo(p.X.dims, xi, W.nonzero_uniform(rng, xi.shape[1])),
                Coo(p.Y.dims, yi, W.nonzero_uniform(rng, yi.shape[1])), (2,), (0,))
    assert np.count_nonzero(yi[0] == 0) > 1024
    info, gidx, gval = run_gpu(q, options=_opts(1))
    assert info["classes"]["block"] > 0 and info["block_mfma"], info
    assert_parity(q, gidx, gval)


def test_matrix_core_execute_is_graph_capturable():
    """Execute enqueues kernels only, so a plan on the matrix cores can be
    captured in a HIP graph; replays with eager work between them reproduce
    the oracle's result."""
    import paper_2410_10094_amd as sptc
    from tests.gpu_common import to_device
    import oracle
    p = _dense_random(38, 700, 300, 900, 50_000, 50_000, name="graph")
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy)
    X, Y = to_device(p)
    with sptc.plan(X, Y, p.cx, p.cy, options=_opts(1)) as pl:
        assert pl.block_mfma
        idx, val, nnz, cap = pl.allocate_outputs()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            pl.execute_into(idx, val, cap, nnz, stream=s)  # warm-up outside capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            pl.execute_into(idx, val, cap, nnz, stream=s)
        for rep in range(3):
            idx.fill_(-1)
            val.fill_(float("nan"))
            nnz.fill_(-99)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            n = int(nnz.item())
            log(f"[mfma graph] replay {rep} nnz {n}")
            assert n >= 0
            assert_parity(p, idx[:, :n].cpu().numpy(), val[:n].cpu().numpy(), ref=ref)
