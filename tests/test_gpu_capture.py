"""Plans that make no read-back (sptc_options.capture_out_cap): every count
stays on the device, so sptc_plan and sptc_execute can be captured together
into one HIP graph.  Parity in eager mode over every accumulation class and
both modes; plan + execute captured once and replayed with new values in
the inputs between replays, each replay against the oracle; an undersized
bound reported by the device.  Also the tile and lds_max_keys options."""
import numpy as np
import pytest

import oracle
from paper_2410_10094_amd import workloads as W
from paper_2410_10094_amd.workloads import Coo, Problem
from tests import helpers as H
from tests.gpu_common import assert_parity, log, to_device
from tests.test_gpu_parity import _class_problems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(p, options, allocator="torch"):
    import paper_2410_10094_amd as sptc
    X, Y = to_device(p)
    with sptc.plan(X, Y, p.cx, p.cy, options=options, allocator=allocator) as pl:
        idx, val = pl.execute()
        return pl, idx.cpu().numpy(), val.cpu().numpy()


CASES = [(name, p) for name, p in _class_problems()] + [("plain", W.plain(n=32, nnz=3000)),
                                                        ("block-sparse", W.block_sparse(n=24, block=4))]


@pytest.mark.parametrize("mode", ["grouped", "global"])
@pytest.mark.parametrize("name,p", CASES, ids=[f"{n}-{p.name}" for n, p in CASES])
def test_no_readback_plan_matches_oracle(name, p, mode):
    import paper_2410_10094_amd as sptc
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=8)
    cap = ref.nnz + 17
    opt = sptc.default_options(capture_out_cap=cap, mode={"grouped": 0, "global": 1}[mode])
    log(f"[capture] {p.name} {mode} nnz {p.X.nnz}x{p.Y.nnz} cap {cap}")
    pl, gidx, gval = _run(p, opt)
    # the bound is the cap, or the output's cell count when that is smaller
    cells = int(np.prod([d for m, d in enumerate(p.X.dims) if m not in p.cx], dtype=np.float64) *
                np.prod([d for m, d in enumerate(p.Y.dims) if m not in p.cy], dtype=np.float64))
    assert pl.products == -1 and pl.out_nnz_bound == min(cap, cells)
    assert_parity(p, gidx, gval, ref)


def test_no_readback_plan_reports_an_undersized_bound():
    import paper_2410_10094_amd as sptc
    p = W.plain(n=24, nnz=1500)
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy)
    opt = sptc.default_options(capture_out_cap=ref.nnz // 2)
    with pytest.raises(sptc.SptcError) as e:
        _run(p, opt)
    assert e.value.status == 5  # SPTC_ERR_CAPACITY, reported by the device through out_nnz


def _mixed_problem(seed):
    """Direct, wave and dense block groups in one contraction: X free key
    (i, j) with many single-entry groups, some of 2 entries (about 230
    products) and a few of 400, over a 12-bit Y free key."""
    rng = np.random.default_rng(seed)
    K = 512
    cols = []
    for g in range(3000):
        n = 400 if g % 300 == 0 else (2 if g % 10 == 0 else 1)
        cols.append(np.stack([np.full(n, g // 64), np.full(n, g % 64), rng.choice(K, n, replace=False)]))
    xi = np.concatenate(cols, axis=1).astype(np.int32)
    X = Coo((64, 64, K), xi, W.nonzero_uniform(rng, xi.shape[1]))
    Y = Coo((K, 64, 64), W.unique_coords(rng, (K, 64, 64), 60_000), W.nonzero_uniform(rng, 60_000))
    return Problem(f"mixed-{seed}", X, Y, (2,), (0,))


def test_plan_and_execute_captured_in_one_graph_and_replayed():
    import paper_2410_10094_amd as sptc
    p = _mixed_problem(5)
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=8)
    cap = ref.nnz + 100
    X, Y = to_device(p)
    order = ref.idx.shape[0]
    oi = torch.zeros((order, cap), dtype=torch.int32, device="cuda")
    ov = torch.zeros(cap, dtype=torch.float64, device="cuda")
    on = torch.zeros(1, dtype=torch.int64, device="cuda")
    opt = sptc.default_options(capture_out_cap=cap)
    # warm-up outside the capture (first-use set-up of the library and the allocator)
    _run(p, sptc.default_options(capture_out_cap=cap))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        pl = sptc.plan(X, Y, p.cx, p.cy, options=opt, allocator="torch")
        pl.execute_into(oi, ov, cap, on)
    info = (pl.products, pl.out_nnz_bound)
    assert info == (-1, cap)
    rng = np.random.default_rng(9)
    other = W.plain(n=16, nnz=500)
    for r in range(3):
        # new values in X and Y (same coordinates), written outside the graph
        xv = W.nonzero_uniform(rng, p.X.nnz)
        yv = W.nonzero_uniform(rng, p.Y.nnz)
        X.val.copy_(torch.from_numpy(xv))
        Y.val.copy_(torch.from_numpy(yv))
        q = Problem(p.name, Coo(p.X.dims, p.X.idx, xv), Coo(p.Y.dims, p.Y.idx, yv), p.cx, p.cy)
        on.fill_(-99)
        g.replay()
        torch.cuda.synchronize()
        n = int(on.item())
        log(f"[capture] replay {r}: nnz {n}")
        qref = oracle.contract(q.X, q.Y, q.cx, q.cy, nthreads=8)
        assert_parity(q, oi[:, :n].cpu().numpy(), ov[:n].cpu().numpy(), qref)
        # eager work of the library between replays
        _run(other, None, allocator="pool")
    pl.close()


def test_lds_max_keys_sends_large_hashed_groups_to_the_output_hash():
    import paper_2410_10094_amd as sptc
    p = [q for _, q in _class_problems() if q.name == "block-hash"][0]
    from tests.gpu_common import run_gpu
    info0, _, _ = run_gpu(p)
    info, gidx, gval = run_gpu(p, options=sptc.default_options(lds_max_keys=64))
    assert info["classes"]["global_"] > info0["classes"]["global_"], (info0["classes"], info["classes"])
    assert_parity(p, gidx, gval)


@pytest.mark.parametrize("tile", [1024, 2048])
def test_direct_class_tile_sizes(tile):
    import paper_2410_10094_amd as sptc
    from tests.gpu_common import run_gpu
    p = W.imbalanced(nnz_x=60_000, nnz_y=20_000, xdims=(1 << 12, 1 << 10, 1 << 10), ydims=(1 << 10, 1 << 8, 1 << 6))
    info, gidx, gval = run_gpu(p, options=sptc.default_options(tile=tile))
    assert info["classes"]["direct"] > 0
    assert_parity(p, gidx, gval)
