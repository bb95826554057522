"""Parity at the full workload sizes, with the default launch configuration
the benchmark times.

* block-sparse 48^4 (literal parameters): complete element-wise parity.
* block-sparse 48^4 at ~1.5M nnz and the imbalanced 1e7 x 1e6 workload:
  outputs sampled by the oracle and evaluated one by one, plus properties
  that hold at any size: P equals the oracle's pair count, coordinates are
  distinct and inside the output shape, the sum of all outputs equals
  sum_k (sum X_k)(sum Y_k), and nnz is bounded by P.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2410_10094_amd import workloads as W
from tests import helpers as H
from tests.gpu_common import assert_parity, log, to_device

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


def _check_large(p, nsamples=3000):
    import paper_2410_10094_amd as sptc
    X, Y = to_device(p)
    log(f"[full] {p.name}: planning")
    with sptc.plan(X, Y, p.cx, p.cy) as pl:
        idx, val = pl.execute()
        P, bound, dims = pl.products, pl.out_nnz_bound, pl.out_dims
    nnz = val.shape[0]
    log(f"[full] {p.name}: P={P} nnz={nnz}")
    _, total = oracle.match_counts(p.X, p.Y, p.cx, p.cy)
    assert P == total
    assert 0 < nnz <= min(P, bound)
    for m, d in enumerate(dims):
        assert int(idx[m].min()) >= 0 and int(idx[m].max()) < d
    lin = _linear(idx, dims)
    slin, order = torch.sort(lin)
    assert bool((slin[1:] > slin[:-1]).all()), "duplicate output coordinates"
    ident, scale = _key_sum_identity(p)
    assert abs(float(val.sum()) - ident) <= 1e-10 * scale
    # sampled outputs, evaluated one by one by the oracle
    q = oracle.sample_outputs(p.X, p.Y, p.cx, p.cy, nsamples, seed=20241010)
    ref_val, ref_abs, ref_terms = oracle.values_at(p.X, p.Y, p.cx, p.cy, q)
    qlin = _linear(torch.from_numpy(q).to(idx.device), dims)
    pos = torch.searchsorted(slin, qlin).clamp(max=nnz - 1)
    assert bool((slin[pos] == qlin).all()), "a sampled output coordinate is missing"
    got = val[order[pos]].cpu().numpy()
    H.assert_values_close(got, ref_val, ref_abs, ref_terms)
    log(f"[full] {p.name}: ok")


def test_block_sparse_full_parity():
    p = W.block_sparse()
    log(f"[full] {p.name} nnz {p.X.nnz}x{p.Y.nnz}")
    from tests.gpu_common import run_gpu
    info, gidx, gval = run_gpu(p)
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=16)
    assert info["products"] == int(ref.terms.sum())
    assert_parity(p, gidx, gval, ref)


def test_block_sparse_1p5m_sampled():
    _check_large(W.block_sparse(p_block=0.565))


def test_imbalanced_full_size_sampled():
    _check_large(W.imbalanced())
