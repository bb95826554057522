"""GPU parity of batched contraction (sptc_batch_*): every contraction of a
batch against the oracle, to the same bar as single contractions
(coordinates and nnz bit-exact after sorting, values within
helpers.value_tolerance), and each result the same alone and in the mix."""
import numpy as np
import pytest

import oracle
from paper_2410_10094_amd import workloads as W
from paper_2410_10094_amd.workloads import Coo, Problem
from tests import helpers as H
from tests.gpu_common import assert_parity, log, run_gpu, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _batch(problems, **kw):
    import paper_2410_10094_amd as sptc
    dev = [to_device(p) for p in problems]
    return sptc.batch([(X, Y, p.cx, p.cy) for (X, Y), p in zip(dev, problems)], **kw)


def _check_batch(problems, results, b_obj=None):
    for b, (p, (idx, val)) in enumerate(zip(problems, results)):
        per_x, total = oracle.match_counts(p.X, p.Y, p.cx, p.cy)
        if b_obj is not None:
            assert b_obj.items[b]["products"] == total, (b, p.name)
        assert_parity(p, idx.cpu().numpy(), val.cpu().numpy())


def _mixed(seed, count):
    rng = np.random.default_rng(seed)
    ps = []
    for s in range(count):
        ox, oy = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        nc = int(rng.integers(0, min(ox, oy, 2) + 1))
        nx, ny = int(rng.integers(0, 4000)), int(rng.integers(0, 4000))
        lo, hi = (2, 9) if nc == 0 else (3, 60)
        ps.append(W.random_problem(seed * 1000 + s, ox, oy, nc, lo, hi, nx, ny, duplicates=s % 5 == 4))
    return ps


def test_batch_of_mixed_contractions():
    """Orders 1-5, 0-2 contracted pairs, empty inputs, repeated coordinates."""
    ps = _mixed(31, 40)
    log(f"[batch] mixed 40: nnz X {[p.X.nnz for p in ps]}")
    with _batch(ps) as bt:
        _check_batch(ps, bt.execute(), bt)


def test_batch_of_batched_workload_draws():
    """Draws of the batched workload (orders 3-5, dims 32..4096, 1-2 pairs),
    nnz scaled down so the oracle checks every output."""
    ps = W.batched_draws(seed=77, count=48, nnz_lo=1e2, nnz_hi=3e4)
    log(f"[batch] draws 48: products bound check")
    with _batch(ps) as bt:
        assert bt.count == 48
        _check_batch(ps, bt.execute(), bt)


def test_batch_with_block_sparse_and_imbalanced_members():
    """Members large enough to reach the block and global accumulation
    classes of the packed problem."""
    ps = [
        W.block_sparse(n=24, block=4),
        W.imbalanced(nnz_x=100_000, nnz_y=10_000, xdims=(1 << 12, 1 << 10, 1 << 11),
                     ydims=(1 << 11, 1 << 7, 1 << 6)),
        W.plain(),
        W.paper_set(23, 10, 2000),
    ]
    with _batch(ps) as bt:
        _check_batch(ps, bt.execute(), bt)


def test_batch_results_equal_single_plans():
    """Each contraction gives the same coordinates alone and in the batch,
    and values within the tolerance."""
    ps = _mixed(32, 12)
    with _batch(ps) as bt:
        res = bt.execute()
    for p, (idx, val) in zip(ps, res):
        _, sidx, sval = run_gpu(p)
        bi, bv = H.sort_coo(idx.cpu().numpy(), val.cpu().numpy())
        si, sv = H.sort_coo(sidx, sval)
        np.testing.assert_array_equal(bi, si)
        ref = assert_parity(p, sidx, sval)
        assert_parity(p, idx.cpu().numpy(), val.cpu().numpy(), ref=ref)
        # both within the tolerance of the oracle, hence within twice it of each other
        H.assert_values_close(bv, sv, ref.absval, ref.terms, rel=2e-12)


def test_batch_of_one_and_repeated_execute():
    p = W.plain(seed=12, n=32, nnz=3000)
    with _batch([p]) as bt:
        r1 = bt.execute()
        r2 = bt.execute()
    for idx, val in (r1[0], r2[0]):
        assert_parity(p, idx.cpu().numpy(), val.cpu().numpy())


def test_batch_torch_allocator():
    ps = _mixed(33, 6)
    with _batch(ps, allocator="torch") as bt:
        _check_batch(ps, bt.execute(), bt)


def test_batch_rejects_out_of_range_coordinate():
    import paper_2410_10094_amd as sptc
    good = W.plain(seed=13, n=16, nnz=200)
    bad_idx = good.X.idx.copy()
    bad_idx[1, 5] = 16  # mode length 16
    bad = Problem("bad", Coo(good.X.dims, bad_idx, good.X.val), good.Y, good.cx, good.cy)
    with pytest.raises(sptc.SptcError) as e:
        _batch([good, bad])
    assert e.value.status == 1


def test_batch_execute_is_graph_capturable():
    """Execute enqueues kernels only, so it can be captured in a HIP graph;
    replays with eager work between them reproduce the eager result."""
    ps = _mixed(34, 8)
    with _batch(ps) as bt:
        refs = [oracle.contract(p.X, p.Y, p.cx, p.cy) for p in ps]
        for p, r, (i, v) in zip(ps, refs, bt.execute()):
            assert_parity(p, i.cpu().numpy(), v.cpu().numpy(), ref=r)
        idx, val, nnz = bt.allocate_outputs()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            bt.execute_into(idx, val, nnz, stream=s)  # warm-up outside capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            bt.execute_into(idx, val, nnz, stream=s)
        for rep in range(3):
            idx.fill_(-1)
            val.fill_(float("nan"))
            nnz.fill_(-99)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            log(f"[batch graph] replay {rep}")
            for p, r, (gi, gv) in zip(ps, refs, bt.views(idx, val, nnz.cpu().tolist())):
                assert_parity(p, gi.cpu().numpy(), gv.cpu().numpy(), ref=r)
