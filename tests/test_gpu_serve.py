"""Serving loop on the GPU: requests arriving over time are batched
continuously under a memory budget, and each result is the same alone and in
the mix (coordinates bit-exact after sorting, values within the tolerance),
and matches the oracle."""
import numpy as np
import pytest

import oracle
from paper_2410_10094_amd import sched, serve
from paper_2410_10094_amd import workloads as W
from tests import helpers as H
from tests.gpu_common import assert_parity, log, run_gpu, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pool():
    ps = W.batched_draws(seed=91, count=24, nnz_lo=1e2, nnz_hi=2e4)
    ps += [W.plain(seed=92, n=32, nnz=3000), W.block_sparse(n=16, block=4, p_block=0.3),
           W.random_problem(93, 3, 3, 1, 3, 40, 3000, 3000, duplicates=True)]
    return ps


@pytest.mark.parametrize("arena_mb", [96, 24])
def test_served_results_match_alone_and_oracle(arena_mb):
    """At 24 MB the arena is tight, so that plans may be declined (the
    library's allocator returns NULL) and retried after a release."""
    pool = _pool()
    dev = [to_device(p) for p in pool]
    torch.cuda.synchronize()
    arrivals = serve.poisson_arrivals(4000.0, 0.05, 5)[:80]
    rng = np.random.default_rng(6)
    picks = rng.integers(0, len(pool), size=len(arrivals))
    reqs = []
    for i, (a, k) in enumerate(zip(arrivals, picks)):
        p = pool[k]
        reqs.append(serve.Request(i, dev[k][0], dev[k][1], p.cx, p.cy, float(a),
                                  expected_products=sched.estimate_products(p), klass=sched.shape_class(p.Y.dims, p.cy)))
    log(f"[serve] {len(reqs)} requests over {arrivals[-1]:.3f} s")
    be = serve.TorchBackend(arena_bytes=arena_mb << 20, keep_results=True)
    srv = serve.Server(be, budget_bytes=arena_mb << 20, batch_products=4e5)
    done = srv.run(reqs)
    log(f"[serve] arena {arena_mb} MB batches {srv.batches} peak {srv.peak_used} waits {srv.waits_for_memory}")
    assert len(done) == len(reqs)
    assert srv.batches > 1 and srv.peak_used <= arena_mb << 20
    assert not be.arena.chunks  # every batch gave its memory back
    refs, alone = {}, {}
    for r in sorted(done, key=lambda r: r.rid):
        k = int(picks[r.rid])
        p = pool[k]
        if k not in refs:
            refs[k] = oracle.contract(p.X, p.Y, p.cx, p.cy)
            _, ai, av = run_gpu(p)
            alone[k] = H.sort_coo(ai, av)
            assert_parity(p, ai, av, ref=refs[k])
        assert r.done >= r.arrival
        idx, val = r.result
        gi, gv = idx.cpu().numpy(), val.cpu().numpy()
        assert_parity(p, gi, gv, ref=refs[k])
        si, sv = H.sort_coo(gi, gv)
        np.testing.assert_array_equal(si, alone[k][0])
        H.assert_values_close(sv, alone[k][1], refs[k].absval, refs[k].terms, rel=2e-12)


def test_arena_allocator_out_of_room_then_same_result():
    """A batch planned through an ArenaAllocator: with too small an arena the
    library reports out-of-memory and every chunk is given back; with room,
    the result equals the one planned on the stream-ordered pool."""
    import paper_2410_10094_amd as sptc
    from paper_2410_10094_amd import binding as B
    pool = _pool()[:6]
    dev = [to_device(p) for p in pool]
    probs = [(X, Y, p.cx, p.cy) for (X, Y), p in zip(dev, pool)]
    buf = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    small = serve.RingArena(64 << 10)
    al = serve.ArenaAllocator(small, buf.data_ptr())
    with pytest.raises(sptc.SptcError) as e:
        sptc.batch(probs, allocator=al)
    assert e.value.status == B.ERR_OUT_OF_MEMORY
    al.undo()
    assert not small.chunks
    big = serve.RingArena(64 << 20)
    al = serve.ArenaAllocator(big, buf.data_ptr())
    with sptc.batch(probs, allocator=al) as bt, sptc.batch(probs) as ref:
        assert al.bytes >= bt.workspace_bytes
        i1, v1, n1 = bt.allocate_outputs()
        bt.execute_into(i1, v1, n1)
        i2, v2, n2 = ref.allocate_outputs()
        ref.execute_into(i2, v2, n2)
        torch.cuda.synchronize()
        h1, h2 = n1.cpu().tolist(), n2.cpu().tolist()
        assert h1 == h2
        for p, (a, b) in zip(pool, zip(bt.views(i1, v1, h1), ref.views(i2, v2, h2))):
            gi, gv = a[0].cpu().numpy(), a[1].cpu().numpy()
            assert_parity(p, gi, gv)
            np.testing.assert_array_equal(H.sort_coo(gi, gv)[0], H.sort_coo(b[0].cpu().numpy(), b[1].cpu().numpy())[0])
    al.give_back()
    assert not big.chunks
