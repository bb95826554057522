"""Parity at the full workload sizes, in the launch configurations the
benchmark times.

* block-sparse 48^4 (literal parameters): complete element-wise parity.
* block-sparse 48^4 at ~1.5M nnz: complete element-wise parity of all
  5,308,416 outputs against the oracle (16 threads), for the walk (the
  default), the matrix-core block class and the global output hash.
* imbalanced 1e7 x 1e6: nnz equal to the oracle's count of the output
  coordinate set; outputs sampled by the oracle and evaluated one by one;
  properties that hold at any size: P equals the oracle's pair count,
  coordinates are distinct and inside the output shape, the sum of all
  outputs equals sum_k (sum X_k)(sum Y_k), nnz is bounded by P.  Both
  accumulation modes.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2410_10094_amd import workloads as W
from tests import helpers as H
from tests.gpu_common import MODES, assert_parity, log, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _linear(idx, dims):
    lin = torch.zeros(idx.shape[1], dtype=torch.int64, device=idx.device)
    for m, d in enumerate(dims):
        lin = lin * int(d) + idx[m].to(torch.int64)
    return lin


def _key_sum_identity(p):
    """(sum over contracting keys of (sum X_k)(sum Y_k), same with |.|)."""
    def keyed(T, modes):
        dims = [T.dims[c] for c in modes]
        lin = np.zeros(T.nnz, dtype=np.int64)
        for c, d in zip(modes, dims):
            lin = lin * d + T.idx[c].astype(np.int64)
        u, inv = np.unique(lin, return_inverse=True)
        return u, np.bincount(inv, weights=T.val), np.bincount(inv, weights=np.abs(T.val))
    ux, sx, ax = keyed(p.X, p.cx)
    uy, sy, ay = keyed(p.Y, p.cy)
    _, ix, iy = np.intersect1d(ux, uy, assume_unique=True, return_indices=True)
    return math.fsum(sx[ix] * sy[iy]), math.fsum(ax[ix] * ay[iy])


def _check_output(p, idx, val, P, bound, dims, nsamples, seed=20241010):
    """Properties that hold at any size, then sampled outputs evaluated one
    by one by the oracle."""
    nnz = val.shape[0]
    _, total = oracle.match_counts(p.X, p.Y, p.cx, p.cy)
    assert P == total
    assert nnz <= min(P, bound)
    if total == 0:
        assert nnz == 0
        return
    assert nnz > 0
    for m, d in enumerate(dims):
        assert int(idx[m].min()) >= 0 and int(idx[m].max()) < d
    lin = _linear(idx, dims)
    slin, order = torch.sort(lin)
    assert bool((slin[1:] > slin[:-1]).all()), "duplicate output coordinates"
    ident, scale = _key_sum_identity(p)
    assert abs(float(val.sum()) - ident) <= 1e-10 * scale
    q = oracle.sample_outputs(p.X, p.Y, p.cx, p.cy, nsamples, seed=seed)
    ref_val, ref_abs, ref_terms = oracle.values_at(p.X, p.Y, p.cx, p.cy, q)
    qlin = _linear(torch.from_numpy(q).to(idx.device), dims)
    pos = torch.searchsorted(slin, qlin).clamp(max=nnz - 1)
    assert bool((slin[pos] == qlin).all()), "a sampled output coordinate is missing"
    got = val[order[pos]].cpu().numpy()
    H.assert_values_close(got, ref_val, ref_abs, ref_terms)


ORACLE_THREADS = 16


def _run(p, mode="grouped", block_mfma=0):
    import paper_2410_10094_amd as sptc
    X, Y = to_device(p)
    opt = sptc.default_options(mode=MODES[mode], block_mfma=block_mfma)
    log(f"[full] {p.name} {mode} block_mfma={block_mfma}: planning")
    with sptc.plan(X, Y, p.cx, p.cy, options=opt) as pl:
        idx, val = pl.execute()
        info = dict(products=pl.products, bound=pl.out_nnz_bound, dims=pl.out_dims, block_mfma=pl.block_mfma)
    log(f"[full] {p.name}: P={info['products']} nnz={val.shape[0]}")
    return info, idx, val


@pytest.fixture(scope="module")
def c2_1p5m():
    p = W.block_sparse(p_block=0.565)
    log(f"[full] {p.name} nnz {p.X.nnz}x{p.Y.nnz}: oracle on {ORACLE_THREADS} threads")
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=ORACLE_THREADS)
    log(f"[full] {p.name}: oracle nnz {ref.nnz}, P {int(ref.terms.sum())}")
    return p, ref


@pytest.mark.parametrize("mode,block_mfma", [("grouped", 0), ("grouped", 1), ("global", 0)])
def test_block_sparse_1p5m_full_parity(c2_1p5m, mode, block_mfma):
    p, ref = c2_1p5m
    info, idx, val = _run(p, mode, block_mfma)
    if mode == "grouped":
        assert info["block_mfma"] == block_mfma
    assert info["products"] == int(ref.terms.sum())
    assert_parity(p, idx.cpu().numpy(), val.cpu().numpy(), ref)
    log(f"[full] {p.name} {mode} block_mfma={block_mfma}: all {ref.nnz} outputs match")


@pytest.fixture(scope="module")
def c3():
    p = W.imbalanced()
    log(f"[full] {p.name} nnz {p.X.nnz}x{p.Y.nnz}: oracle output count on {ORACLE_THREADS} threads")
    n = oracle.count_outputs(p.X, p.Y, p.cx, p.cy, nthreads=ORACLE_THREADS)
    log(f"[full] {p.name}: oracle nnz {n}")
    return p, n


@pytest.mark.parametrize("mode", ["grouped", "global"])
def test_imbalanced_full_size(c3, mode):
    p, n = c3
    info, idx, val = _run(p, mode)
    assert val.shape[0] == n, f"nnz {val.shape[0]} != oracle {n}"
    _check_output(p, idx, val, info["products"], info["bound"], info["dims"], 3000)
    log(f"[full] {p.name} {mode}: ok")


def test_block_sparse_full_parity():
    p = W.block_sparse()
    log(f"[full] {p.name} nnz {p.X.nnz}x{p.Y.nnz}")
    from tests.gpu_common import run_gpu
    info, gidx, gval = run_gpu(p)
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=16)
    assert info["products"] == int(ref.terms.sum())
    assert_parity(p, gidx, gval, ref)


def test_batched_workload_full_size_draws():
    """The first 64 full-size draws of the batched workload, cut into batches
    as the benchmark cuts them (by Y free key class, at most 1e9 expected
    products each) and executed with sptc_batch_*; every member is checked by
    the properties above and sampled outputs."""
    import paper_2410_10094_amd as sptc
    from paper_2410_10094_amd import sched
    draws = [W.batched_draw(W.BASE_SEED + 4, i) for i in range(64)]
    cut = sched.make_batches(draws, sched.estimate_products, lambda p: sched.shape_class(p.Y.dims, p.cy), 1e9)
    dev = [to_device(p) for p in draws]
    checked = 0
    for members in cut:
        log(f"[full] batch of {len(members)}: planning")
        with sptc.batch([(dev[i][0], dev[i][1], draws[i].cx, draws[i].cy) for i in members]) as bt:
            res = bt.execute()
            for i, it, (idx, val) in zip(members, bt.items, res):
                _check_output(draws[i], idx, val, it["products"], it["out_nnz_bound"], it["out_dims"], 200,
                              seed=1000 + i)
                checked += 1
        log(f"[full] batch of {len(members)}: ok")
    assert checked == 64
