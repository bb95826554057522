"""Helpers for the GPU tests: run the HIP path through the C ABI and compare
with the oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from tests import helpers as H


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_device(p):
    import paper_2410_10094_amd as sptc
    return sptc.DeviceCoo.from_host(p.X), sptc.DeviceCoo.from_host(p.Y)


MODES = {"grouped": 0, "global": 1}


def run_gpu(p, options=None, allocator="pool", mode=None, order=1):
    """Plan + execute on cuda:0; returns (plan info dict, idx numpy, val numpy).
    order: sptc_options.operand_order, pinned to 1 (X grouped, as given) by
    default so that a test's class and kernel assertions hold for the
    operands it built; 0 lets the plan pick the operand to group."""
    import paper_2410_10094_amd as sptc
    X, Y = to_device(p)
    options = options or sptc.default_options()
    options.operand_order = order
    if mode is not None:
        options.mode = MODES[mode]
    with sptc.plan(X, Y, p.cx, p.cy, options=options, allocator=allocator) as pl:
        idx, val = pl.execute()
        info = dict(products=pl.products, out_nnz_bound=pl.out_nnz_bound, y_groups=pl.y_groups,
                    out_order=pl.out_order, out_dims=pl.out_dims, out_table_slots=pl.out_table_slots,
                    mode=pl.mode, x_groups=pl.x_groups, classes=pl.group_classes, block_mfma=pl.block_mfma,
                    block_tiles_scanned=pl.block_tiles_scanned, operands_swapped=pl.operands_swapped,
                    block_dense_rows=pl.block_dense_rows)
        return info, idx.cpu().numpy(), val.cpu().numpy()


def assert_parity(p, gidx, gval, ref=None, nthreads=8):
    """Coordinates and nnz bit-exact after sorting; values within the
    tolerance of helpers.value_tolerance."""
    if ref is None:
        ref = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=nthreads)
    assert gval.shape[0] == ref.nnz, f"nnz {gval.shape[0]} != oracle {ref.nnz}"
    gi, gv = H.sort_coo(gidx, gval)
    np.testing.assert_array_equal(gi, ref.idx)
    stats = H.assert_values_close(gv, ref.val, ref.absval, ref.terms)
    if stats["multi_term_outputs"]:
        log(f"[values] {getattr(p, 'name', '?')}: nnz {ref.nnz}, worst error "
            f"{stats['worst_ratio_to_1e-12_sum_abs']:.3g} x 1e-12*sum|xy|, "
            f"{stats['second_clause']} of {stats['multi_term_outputs']} multi-term outputs past 1e-12*|z|")
    return ref
