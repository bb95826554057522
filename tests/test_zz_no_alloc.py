"""sptc_contract_noalloc (the entry point that allocates nothing) against
sptc_plan + sptc_execute: two calls in a row on one stream, the second on a
smaller input, and a contraction too large for the static scratch."""
import numpy as np
import pytest

from paper_2410_10094_amd import workloads as W
from tests import helpers as H
from tests.gpu_common import assert_parity, log, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _existing(p, X, Y):
    import paper_2410_10094_amd as sptc
    with sptc.plan(X, Y, p.cx, p.cy) as pl:
        idx, val = pl.execute()
        return pl.out_nnz_bound, pl.out_order, idx.cpu().numpy(), val.cpu().numpy()


def test_noalloc_matches_plan_and_execute_twice():
    import paper_2410_10094_amd as sptc
    big = W.block_sparse(n=32, block=4, p_block=0.3)
    small = W.plain(n=24, nnz=1500)
    cases = []
    for p in (big, small):
        X, Y = to_device(p)
        bound, order, ridx, rval = _existing(p, X, Y)
        cases.append((p, X, Y, bound, order, ridx, rval))
    # outputs allocated before either call; the calls themselves allocate nothing
    outs = [(torch.full((max(order, 1), max(bound, 1)), -1, dtype=torch.int32, device="cuda"),
             torch.full((max(bound, 1),), np.nan, dtype=torch.float64, device="cuda"),
             torch.zeros(1, dtype=torch.int64, device="cuda")) for (_, _, _, bound, order, _, _) in cases]
    torch.cuda.synchronize()
    for (p, X, Y, bound, order, _, _), (oi, ov, on) in zip(cases, outs):
        log(f"[noalloc] {p.name} nnz {p.X.nnz}x{p.Y.nnz}, out_cap {bound}")
        sptc.contract_noalloc(X, Y, p.cx, p.cy, oi, ov, bound, on)
    torch.cuda.synchronize()
    for (p, X, Y, bound, order, ridx, rval), (oi, ov, on) in zip(cases, outs):
        n = int(on.item())
        assert n == rval.shape[0], (p.name, n, rval.shape[0])
        gi, gv = oi[:order, :n].cpu().numpy(), ov[:n].cpu().numpy()
        ref = assert_parity(p, gi, gv)
        # against the existing entry point's result: same coordinates, values
        # within the tolerance of two GPU results of the same oracle value
        si, sv = H.sort_coo(gi, gv)
        ri, rv = H.sort_coo(ridx, rval)
        np.testing.assert_array_equal(si, ri)
        H.assert_values_close(sv, rv, ref.absval, ref.terms, rel=2e-12)
        log(f"[noalloc] {p.name}: {n} outputs match")


def test_noalloc_rejects_workspace_beyond_the_scratch():
    import paper_2410_10094_amd as sptc
    from paper_2410_10094_amd import binding as B
    # 2^24 X entries: the grouped X records alone (16 B each) exceed 256 MiB
    n = 1 << 24
    g = torch.Generator(device="cuda").manual_seed(7)
    xi = torch.randint(0, 1 << 12, (2, n), dtype=torch.int32, device="cuda", generator=g)
    xv = torch.ones(n, dtype=torch.float64, device="cuda")
    yi = torch.randint(0, 1 << 12, (2, 64), dtype=torch.int32, device="cuda", generator=g)
    yv = torch.ones(64, dtype=torch.float64, device="cuda")
    X = sptc.DeviceCoo((1 << 12, 1 << 12), xi, xv)
    Y = sptc.DeviceCoo((1 << 12, 1 << 12), yi, yv)
    oi = torch.empty((2, 16), dtype=torch.int32, device="cuda")
    ov = torch.empty(16, dtype=torch.float64, device="cuda")
    on = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(B.SptcError) as e:
        sptc.contract_noalloc(X, Y, [1], [0], oi, ov, 16, on)
    assert e.value.status == B.ERR_CAPACITY
    assert "static scratch" in str(e.value)
    # the entry point still works after the rejection
    p = W.plain(n=16, nnz=600)
    Xs, Ys = to_device(p)
    bound, order, ridx, rval = _existing(p, Xs, Ys)
    oi = torch.empty((order, bound), dtype=torch.int32, device="cuda")
    ov = torch.empty(bound, dtype=torch.float64, device="cuda")
    sptc.contract_noalloc(Xs, Ys, p.cx, p.cy, oi, ov, bound, on)
    n = int(on.item())
    assert n == rval.shape[0]
    assert_parity(p, oi[:, :n].cpu().numpy(), ov[:n].cpu().numpy())
