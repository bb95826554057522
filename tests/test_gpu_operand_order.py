"""Operand order (sptc_options.operand_order, paper section 5.4): by
default the grouped mode groups whichever operand has the larger free key
space and indexes the per-group tables by the other's free key, trading X
and Y when Y's space is the larger; Z keeps X's free modes first.  Each
problem runs with the plan's choice and with the order pinned, both
against the oracle element by element, and the choice is checked against
the rule."""
import numpy as np
import pytest

import oracle
from paper_2410_10094_amd import workloads as W
from paper_2410_10094_amd.workloads import Problem
from tests.gpu_common import assert_parity, log, run_gpu
from tests.test_gpu_parity import _class_problems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _free_cells(T, c):
    return int(np.prod([d for m, d in enumerate(T.dims) if m not in c], dtype=np.float64))


def _problems():
    out = []
    for ox, oy in ((4, 5), (5, 4)):
        out.append(W.paper_set(W.BASE_SEED + 70 + ox, 9, 4000, ox, oy))
    for cls, p in _class_problems():  # every accumulation class, with X and Y traded
        out.append(Problem(f"{p.name}-traded", p.Y, p.X, p.cy, p.cx))
    out.append(W.random_problem(71, 3, 4, 1, 3, 12, 3000, 4000))
    out.append(W.random_problem(72, 2, 4, 1, 4, 40, 500, 6000, duplicates=True))
    return out


@pytest.mark.parametrize("p", _problems(), ids=lambda p: p.name)
def test_operand_order_matches_oracle(p):
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=8)
    want_swap = _free_cells(p.Y, p.cy) > _free_cells(p.X, p.cx)
    log(f"[order] {p.name} nnz {p.X.nnz}x{p.Y.nnz} swap expected {want_swap}")
    info, gidx, gval = run_gpu(p, mode="grouped", order=0)
    assert info["operands_swapped"] == want_swap
    dims = [d for m, d in enumerate(p.X.dims) if m not in p.cx] + [d for m, d in enumerate(p.Y.dims) if m not in p.cy]
    assert list(info["out_dims"]) == dims
    assert_parity(p, gidx, gval, ref)
    info1, gidx1, gval1 = run_gpu(p, mode="grouped", order=1)
    assert not info1["operands_swapped"]
    assert_parity(p, gidx1, gval1, ref)


def test_global_mode_keeps_the_order():
    p = W.paper_set(W.BASE_SEED + 74, 9, 4000, 4, 5)
    info, gidx, gval = run_gpu(p, mode="global", order=0)
    assert not info["operands_swapped"]
    assert_parity(p, gidx, gval)
