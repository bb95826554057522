"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Coordinates and nnz must match the oracle bit for bit after sorting; values
must agree within helpers.value_tolerance (1e-12 relative, or the
summation-reordering bound for sums that cancel; bit-exact for single-term
outputs)."""
import numpy as np
import pytest

import oracle
from paper_2410_10094_amd import workloads as W
from paper_2410_10094_amd.workloads import Coo, Problem
from tests import helpers as H
from tests.gpu_common import assert_parity, log, run_gpu, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _problems():
    ps = [
        W.plain(),  # the plain order-3 workload at full size
        W.plain(seed=11, n=32, nnz=3000),
        W.block_sparse(n=24, block=4),
        W.block_sparse(seed=5, n=16, block=4, p_block=0.5, p_fill=0.7),
        W.imbalanced(nnz_x=200_000, nnz_y=20_000, xdims=(1 << 13, 1 << 10, 1 << 11),
                     ydims=(1 << 11, 1 << 8, 1 << 6)),
        W.paper_set(21, 12, 3000),
        W.paper_set(22, 10, 2000, order_x=4, order_y=4),
    ]
    rng = np.random.default_rng(42)
    for s in range(14):
        ox, oy = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        nc = int(rng.integers(0, min(ox, oy, 3) + 1))
        dup = s % 4 == 3
        nx, ny = int(rng.integers(1, 6000)), int(rng.integers(1, 6000))
        lo, hi = (2, 9) if nc == 0 else (3, 40)
        ps.append(W.random_problem(7000 + s, ox, oy, nc, lo, hi, nx, ny, duplicates=dup))
    return ps


PROBLEMS = _problems()


@pytest.mark.parametrize("mode", ["grouped", "global"])
@pytest.mark.parametrize("p", PROBLEMS, ids=lambda p: p.name)
def test_parity_against_oracle(p, mode):
    log(f"[parity] {p.name} {mode} nnz {p.X.nnz}x{p.Y.nnz} cx={p.cx} cy={p.cy}")
    info, gidx, gval = run_gpu(p, mode=mode, order=0)  # the plan picks the operand to group
    per_x, total = oracle.match_counts(p.X, p.Y, p.cx, p.cy)
    assert info["products"] == total
    ref = assert_parity(p, gidx, gval)
    assert ref.nnz <= info["out_nnz_bound"]


def test_stage_y_groups_and_grouped_array():
    """Y grouping (counting sort by contracting key): group counts equal the
    oracle's per-tuple counts; each group's run in the grouped array is a
    permutation of Y's entries with that key."""
    import paper_2410_10094_amd as sptc
    for p in [W.block_sparse(n=24, block=4), W.random_problem(91, 4, 3, 2, 2, 9, 4000, 3000, duplicates=True),
              W.plain()]:
        log(f"[stage-A] {p.name}")
        X, Y = to_device(p)
        with sptc.plan(X, Y, p.cx, p.cy, options=sptc.default_options(operand_order=1)) as pl:
            kc, counts, starts = (t.cpu().numpy() for t in pl.y_groups_table())
            free, vals = (t.cpu().numpy() for t in pl.y_grouped())
        tuples, ocounts = oracle.group_counts(p.Y, p.cy)
        assert pl.y_groups == ocounts.shape[0]
        gi, gc, gs = H.sort_coo(kc, counts, starts)
        np.testing.assert_array_equal(gi, tuples)
        np.testing.assert_array_equal(gc, ocounts)
        # runs tile the grouped array exactly
        order = np.argsort(gs)
        assert gs[order][0] == 0 and np.all(gs[order][1:] == (gs[order] + gc[order])[:-1])
        assert (gs + gc).max() == p.Y.nnz
        fy = [m for m in range(p.Y.order) if m not in p.cy]
        for g in range(0, gi.shape[1], max(1, gi.shape[1] // 50)):
            sel = np.all(p.Y.idx[list(p.cy)] == gi[:, g:g + 1], axis=0)
            want = sorted(zip(*[p.Y.idx[m, sel].tolist() for m in fy], p.Y.val[sel].tolist()))
            run = slice(gs[g], gs[g] + gc[g])
            got = sorted(zip(*[free[k, run].tolist() for k in range(len(fy))], vals[run].tolist()))
            assert got == want


def test_stage_x_probe_counts():
    """Pass 1 (global mode): per-X product counts equal the oracle's match
    counts exactly, and P is their sum."""
    import paper_2410_10094_amd as sptc
    for p in [W.plain(), W.imbalanced(nnz_x=100_000, nnz_y=10_000, xdims=(1 << 12, 1 << 10, 1 << 10),
                                      ydims=(1 << 10, 1 << 8, 1 << 6))]:
        log(f"[stage-B] {p.name}")
        X, Y = to_device(p)
        with sptc.plan(X, Y, p.cx, p.cy, options=sptc.default_options(mode=1)) as pl:
            counts = pl.x_counts().cpu().numpy()
            P = pl.products
        per_x, total = oracle.match_counts(p.X, p.Y, p.cx, p.cy)
        np.testing.assert_array_equal(counts, per_x)
        assert P == total


def test_stage_x_groups():
    """X grouped by free key (section 4.1): one group per distinct X free
    tuple, with the number of X entries carrying it and the sum of their
    product counts (the bound of section 4.3), all exact."""
    import paper_2410_10094_amd as sptc
    for p in [W.block_sparse(n=24, block=4), W.plain(),
              W.random_problem(92, 4, 3, 1, 2, 7, 5000, 3000, duplicates=True),
              # X free keys of 22 and 24 bits, hashed: grouped by partition
              # into 16 and 8 buckets (the second with repeated coordinates)
              W.imbalanced(nnz_x=50_000, nnz_y=20_000, xdims=(1 << 12, 1 << 10, 1 << 10),
                           ydims=(1 << 10, 1 << 8, 1 << 6)),
              W.random_problem(93, 3, 3, 1, 2000, 3000, 30_000, 5_000, duplicates=True),
              # 1.2M X entries: 512 buckets of the partition
              W.imbalanced(nnz_x=1_200_000, nnz_y=20_000, xdims=(1 << 12, 1 << 10, 1 << 10),
                           ydims=(1 << 10, 1 << 8, 1 << 6))]:
        log(f"[stage-X] {p.name}")
        X, Y = to_device(p)
        with sptc.plan(X, Y, p.cx, p.cy, options=sptc.default_options(operand_order=1)) as pl:
            coords, counts, prods = (t.cpu().numpy() for t in pl.x_groups_table())
            ng, P = pl.x_groups, pl.products
        fx = [m for m in range(p.X.order) if m not in p.cx]
        per_x, total = oracle.match_counts(p.X, p.Y, p.cx, p.cy)
        keys = [tuple(p.X.idx[fx, e].tolist()) for e in range(p.X.nnz)]
        want = {}
        for k, c in zip(keys, per_x.tolist()):
            n, s_ = want.get(k, (0, 0))
            want[k] = (n + 1, s_ + c)
        got = {tuple(coords[:, g].tolist()): (int(counts[g]), int(prods[g])) for g in range(ng)}
        assert ng == len(want) and got == want
        assert P == total == int(prods.sum())


def _class_problems():
    """One problem per accumulation class of the grouped path."""
    rng = np.random.default_rng(33)
    out = []
    # direct: single-entry X groups, Y without repeated coordinates
    out.append(("direct", W.imbalanced(nnz_x=50_000, nnz_y=20_000, xdims=(1 << 12, 1 << 10, 1 << 10),
                                       ydims=(1 << 10, 1 << 8, 1 << 6))))
    # wave: groups of ~20 X entries with a few hundred products each
    out.append(("wave", W.random_problem(34, 3, 3, 1, 1, 1, 1, 1)))
    X = Coo((16, 8, 32), W.unique_coords(rng, (16, 8, 32), 3000), W.nonzero_uniform(rng, 3000))
    Y = Coo((32, 20, 20), W.unique_coords(rng, (32, 20, 20), 400), W.nonzero_uniform(rng, 400))
    out[-1] = ("wave", Problem("wave-groups", X, Y, (2,), (0,)))
    # block, dense: Y free key of 12 bits, large groups
    out.append(("block", W.block_sparse(n=16, block=4, p_block=0.6, p_fill=0.8)))
    # block, hash: Y free key wider than 13 bits, <= 5734 distinct outputs per group
    X = Coo((200, 40), np.stack([rng.integers(0, 200, 3000), rng.integers(0, 40, 3000)]).astype(np.int32),
            W.nonzero_uniform(rng, 3000))
    Y = Coo((40, 1 << 16), np.stack([rng.integers(0, 40, 2000), rng.integers(0, 1 << 16, 2000)]).astype(np.int32),
            W.nonzero_uniform(rng, 2000))
    out.append(("block", Problem("block-hash", X, Y, (1,), (0,))))
    # block, hash, all three table sizes: rows 0-49 with ~15 entries (bounds
    # below 1,433: the 2,048-slot table), rows 50-99 with 40 (bounds ~2,000:
    # 4,096), rows 100-119 with every contracting key twice or three times
    # (repeated X coordinates; bounds ~5,000: 8,192)
    xl = np.concatenate([np.tile(np.arange(40), 2), rng.integers(0, 40, 20)])
    xs = np.concatenate([np.stack([rng.integers(0, 50, 750), rng.integers(0, 40, 750)]),
                         np.stack([np.repeat(np.arange(50, 100), 40), np.tile(np.arange(40), 50)]),
                         np.stack([np.repeat(np.arange(100, 120), xl.size), np.tile(xl, 20)])], axis=1)
    X = Coo((120, 40), xs.astype(np.int32), W.nonzero_uniform(rng, xs.shape[1]))
    out.append(("block", Problem("block-hash-three-sizes", X, Y, (1,), (0,))))
    # global: groups with more distinct outputs than a workgroup's LDS holds
    X = Coo((3, 8), np.stack([rng.integers(0, 3, 200), rng.integers(0, 8, 200)]).astype(np.int32),
            W.nonzero_uniform(rng, 200))
    Y = Coo((8, 1 << 20), np.stack([rng.integers(0, 8, 40_000), rng.integers(0, 1 << 20, 40_000)]).astype(np.int32),
            W.nonzero_uniform(rng, 40_000))
    out.append(("global_", Problem("global-class", X, Y, (1,), (0,))))
    # heavy accumulation: tiny Y free space, many products per output
    X = Coo((4, 64), np.stack([rng.integers(0, 4, 5000), rng.integers(0, 64, 5000)]).astype(np.int32),
            W.nonzero_uniform(rng, 5000))
    Y = Coo((64, 3), np.stack([rng.integers(0, 64, 4000), rng.integers(0, 3, 4000)]).astype(np.int32),
            W.nonzero_uniform(rng, 4000))
    out.append(("block", Problem("heavy-accumulation", X, Y, (1,), (0,))))
    # many small entries per group in a block group: product-parallel walk
    X = Coo((2, 20_000), np.stack([rng.integers(0, 2, 40_000), rng.integers(0, 20_000, 40_000)]).astype(np.int32),
            W.nonzero_uniform(rng, 40_000))
    Y = Coo((20_000, 64), np.stack([rng.integers(0, 20_000, 24_000), rng.integers(0, 64, 24_000)]).astype(np.int32),
            W.nonzero_uniform(rng, 24_000))
    out.append(("block", Problem("block-product-parallel", X, Y, (1,), (0,))))
    return out


def _wide_key_problems():
    """Output keys wider than 63 bits: X free and Y free keys each fit, their
    concatenation does not."""
    rng = np.random.default_rng(36)
    out = []
    # direct and wave classes: 60-bit X free key, 40-bit Y free key
    X = Coo((1 << 30, 1 << 30, 6), np.stack([rng.integers(0, 1 << 30, 3000), rng.integers(0, 1 << 30, 3000),
                                             rng.integers(0, 6, 3000)]).astype(np.int32), W.nonzero_uniform(rng, 3000))
    X.idx[:, 2000:] = X.idx[:, :1000]  # 1000 two-entry groups (wave class), 1000 single-entry (direct)
    X.idx[2, 2000:] = (X.idx[2, :1000] + 1) % 6
    Y = Coo((6, 1 << 20, 1 << 20), np.stack([rng.integers(0, 6, 500), rng.integers(0, 1 << 20, 500),
                                             rng.integers(0, 1 << 20, 500)]).astype(np.int32),
            W.nonzero_uniform(rng, 500))
    out.append(Problem("wide-100-bits", X, Y, (2,), (0,)))
    # global class: one X group reaching 40000 distinct Y free keys
    X = Coo((1 << 31, 1 << 31, 4), np.array([[7] * 4, [9] * 4, [0, 1, 2, 3]], np.int32), W.nonzero_uniform(rng, 4))
    Y = Coo((4, 1 << 20), np.stack([rng.integers(0, 4, 40_000), rng.integers(0, 1 << 20, 40_000)]).astype(np.int32),
            W.nonzero_uniform(rng, 40_000))
    out.append(Problem("wide-global-class", X, Y, (2,), (0,)))
    # global class among 70000 X groups with a 48-bit Y free key: 17 bits of
    # group id plus 48 would not fit a 63-bit table key; the place in the
    # global class's list (one group) does.  Most X entries meet no Y entry.
    nx = 70_000
    lin = rng.choice(1 << 24, nx, replace=False)
    X = Coo((1 << 12, 1 << 12, 8), np.stack([lin >> 12, lin & 4095, rng.integers(4, 8, nx)]).astype(np.int32),
            W.nonzero_uniform(rng, nx))
    X.idx[:, :4] = np.array([[lin[0] >> 12] * 4, [lin[0] & 4095] * 4, [0, 1, 2, 3]], np.int32)
    ny = 6400  # the one group's 6,400 products: more than the largest LDS table takes (5,734)
    Y = Coo((8,) + (1 << 12,) * 4, np.stack([np.arange(ny) % 4] + [rng.integers(0, 1 << 12, ny) for _ in range(4)])
            .astype(np.int32), W.nonzero_uniform(rng, ny))
    out.append(Problem("wide-global-class-many-groups", X, Y, (2,), (0,)))
    return out


@pytest.mark.parametrize("p", _wide_key_problems(), ids=lambda p: p.name)
def test_output_keys_wider_than_63_bits(p):
    log(f"[wide] {p.name}")
    info, gidx, gval = run_gpu(p, mode="grouped")
    assert_parity(p, gidx, gval)
    if p.name.startswith("wide-global-class"):
        assert info["classes"]["global_"] > 0
    else:
        assert info["classes"]["direct"] > 0 and info["classes"]["wave"] > 0


@pytest.mark.parametrize("kind", ["dense", "dense-long-runs", "hashed"])
def test_repeated_y_coordinates_disable_direct_class(kind):
    """With a repeated Y coordinate a single-entry X group can have two
    products on one output, so the direct class must not be used.  Dense Y
    free keys find repeats in the run sort (runs up to 1024 entries sorted,
    longer ones copied), others in a device set."""
    rng = np.random.default_rng(35)
    nc, ny_free, ny = {"dense": (50, 100, 800), "dense-long-runs": (4, 5000, 6000),
                       "hashed": (50, 1 << 20, 800)}[kind]
    X = Coo((1000, nc), W.unique_coords(rng, (1000, nc), 2000), W.nonzero_uniform(rng, 2000))
    yc = W.unique_coords(rng, (nc, ny_free), ny)
    yc = np.concatenate([yc, yc[:, :5]], axis=1)  # five coordinates appear twice
    Y = Coo((nc, ny_free), yc, W.nonzero_uniform(rng, yc.shape[1]))
    p = Problem(f"y-repeats-{kind}", X, Y, (1,), (0,))
    log(f"[ydup] {kind}")
    info, gidx, gval = run_gpu(p, mode="grouped")
    assert info["classes"]["direct"] == 0
    assert_parity(p, gidx, gval)
    q = Problem(f"y-unique-{kind}", X, Coo((nc, ny_free), yc[:, :ny], W.nonzero_uniform(rng, ny)), (1,), (0,))
    info, gidx, gval = run_gpu(q, mode="grouped")
    assert info["classes"]["direct"] > 0
    assert_parity(q, gidx, gval)


@pytest.mark.parametrize("where", ["short-run", "long-run"])
def test_repeated_y_coordinates_in_a_large_y_table(where):
    """A dense Y free key with 20,000 contracting keys: a Y table of more than
    8,192 slots, whose repeat check reads the slots by waves and hands runs
    of more than 512 entries to a workgroup each.  One repeated coordinate,
    in a run of two entries or in a run of 700, disables the direct class;
    without it the class is used; both match the oracle."""
    rng = np.random.default_rng(37)
    nc, nf = 20_000, 4096
    xc = W.unique_coords(rng, (1000, nc), 2000)
    xc[1, :50] = 7  # X entries that meet the long run
    xc = np.unique(xc, axis=1).astype(np.int32)
    X = Coo((1000, nc), xc, W.nonzero_uniform(rng, xc.shape[1]))
    base = W.unique_coords(rng, (nc, nf), 30_000)
    base = base[:, base[0] != 7]
    long_run = np.stack([np.full(700, 7), np.arange(700)]).astype(np.int32)
    yc = np.concatenate([base, long_run], axis=1)
    rep = yc[:, :1] if where == "short-run" else long_run[:, 3:4]
    for name, coords, want_direct in ((f"y-repeat-{where}", np.concatenate([yc, rep], axis=1), False),
                                      (f"y-unique-{where}", yc, True)):
        Y = Coo((nc, nf), coords, W.nonzero_uniform(rng, coords.shape[1]))
        p = Problem(name, X, Y, (1,), (0,))
        log(f"[ydup-large] {name}")
        info, gidx, gval = run_gpu(p, mode="grouped")
        assert (info["classes"]["direct"] > 0) == want_direct, info["classes"]
        assert_parity(p, gidx, gval)


@pytest.mark.parametrize("cls,p", _class_problems(), ids=lambda v: v if isinstance(v, str) else v.name)
def test_grouped_accumulation_classes(cls, p):
    log(f"[class] {cls} {p.name}")
    info, gidx, gval = run_gpu(p, mode="grouped")
    assert info["classes"][cls] > 0, info["classes"]
    assert sum(info["classes"].values()) == info["x_groups"]
    assert_parity(p, gidx, gval)


def _edge_problems():
    out = []
    e = np.zeros((3, 0), np.int32)
    some = W.random_problem(1, 3, 3, 1, 4, 4, 50, 50)
    out.append(Problem("empty-x", Coo((4, 4, 4), e, np.zeros(0)), some.Y, (2,), (0,)))
    out.append(Problem("empty-y", some.X, Coo((4, 4, 4), e, np.zeros(0)), (2,), (0,)))
    out.append(Problem("empty-both", Coo((4, 4, 4), e, np.zeros(0)), Coo((4, 4, 4), e, np.zeros(0)), (2,), (0,)))
    out.append(W.random_problem(2, 2, 3, 0, 2, 6, 40, 30))  # outer product
    out.append(W.random_problem(3, 2, 2, 2, 3, 5, 20, 20))  # full contraction: order-0 output
    out.append(W.random_problem(4, 1, 1, 1, 7, 7, 5, 6))    # order-1 dot product
    out.append(W.random_problem(5, 3, 3, 1, 1, 1, 1, 1))    # all dims 1
    # explicit zeros and exact cancellation still give structural entries
    out.append(Problem("zeros", Coo((2, 3), np.array([[0, 0], [1, 2]], np.int32), np.array([0.0, 1.0])),
                       Coo((3, 2), np.array([[1, 2], [1, 1]], np.int32), np.array([5.0, -5.0])), (1,), (0,)))
    out.append(Problem("cancel", Coo((1, 2), np.array([[0, 0], [0, 1]], np.int32), np.array([1.0, 1.0])),
                       Coo((2, 1), np.array([[0, 1], [0, 0]], np.int32), np.array([2.5, -2.5])), (1,), (0,)))
    # a 63-bit output key (40 + 23 bits)
    rng = np.random.default_rng(9)
    X = Coo((1 << 20, 1 << 20, 8), np.stack([rng.integers(0, 1 << 20, 500), rng.integers(0, 1 << 20, 500),
                                             rng.integers(0, 8, 500)]).astype(np.int32), W.nonzero_uniform(rng, 500))
    Y = Coo((8, 1 << 23), np.stack([rng.integers(0, 8, 400), rng.integers(0, 1 << 23, 400)]).astype(np.int32),
            W.nonzero_uniform(rng, 400))
    out.append(Problem("key-63-bits", X, Y, (2,), (0,)))
    # huge groups: every X entry expands thousands of products
    out.append(W.random_problem(6, 3, 3, 1, 2, 2, 300, 20000))
    # most X entries match nothing: one tile spans many X entries
    rng = np.random.default_rng(10)
    X = Coo((200, 5000), np.stack([rng.integers(0, 200, 120_000), rng.integers(0, 5000, 120_000)]).astype(np.int32),
            W.nonzero_uniform(rng, 120_000))
    Y = Coo((5000, 30), np.array([[7, 7, 4000], [1, 2, 3]], np.int32), np.array([1.0, -2.0, 0.5]))
    out.append(Problem("sparse-matches", X, Y, (1,), (0,)))
    # many duplicates of the same coordinates
    out.append(Problem("duplicates", Coo((3, 3), np.array([[1] * 50 + [2] * 50, [0] * 100], np.int32),
                                         W.nonzero_uniform(np.random.default_rng(1), 100)),
                       Coo((3, 2), np.array([[0] * 30, [1] * 30], np.int32),
                           W.nonzero_uniform(np.random.default_rng(2), 30)), (1,), (0,)))
    return out


@pytest.mark.parametrize("mode", ["grouped", "global"])
@pytest.mark.parametrize("p", _edge_problems(), ids=lambda p: p.name)
def test_edge_cases(p, mode):
    log(f"[edge] {p.name} {mode}")
    info, gidx, gval = run_gpu(p, mode=mode)
    assert_parity(p, gidx, gval)


def test_operand_swap():
    p = W.random_problem(123, 3, 4, 2, 3, 12, 5000, 4000)
    log("[swap]")
    _, ai, av = run_gpu(p)
    q = Problem("swapped", p.Y, p.X, p.cy, p.cx)
    _, bi, bv = run_gpu(q)
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy)
    nfx, nfy = p.X.order - 2, p.Y.order - 2
    perm = list(range(nfy, nfy + nfx)) + list(range(nfy))
    assert_parity(p, ai, av, ref)
    assert_parity(p, bi[perm], bv, ref)


def test_repeated_execute_and_determinism():
    import paper_2410_10094_amd as sptc
    p = W.block_sparse(n=24, block=4)
    log("[repeat]")
    X, Y = to_device(p)
    ref = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=8)
    with sptc.plan(X, Y, p.cx, p.cy) as pl:
        for _ in range(4):
            idx, val = pl.execute()
            assert_parity(p, idx.cpu().numpy(), val.cpu().numpy(), ref)


def test_torch_allocator_matches_pool():
    p = W.plain(seed=77, n=40, nnz=4000)
    log("[torch-allocator]")
    _, ai, av = run_gpu(p, allocator="torch")
    assert_parity(p, ai, av)


def test_small_out_cap_reports_capacity_and_plan_recovers():
    import paper_2410_10094_amd as sptc
    p = W.plain(seed=5, n=16, nnz=400)
    log("[out-cap]")
    X, Y = to_device(p)
    with sptc.plan(X, Y, p.cx, p.cy) as pl:
        with pytest.raises(sptc.SptcError) as e:
            pl.execute(out_cap=10)
        assert e.value.status == 5
        idx, val = pl.execute()
        assert_parity(p, idx.cpu().numpy(), val.cpu().numpy())


def test_undersized_output_table_reports_capacity():
    import paper_2410_10094_amd as sptc
    p = W.plain(seed=6, n=16, nnz=400)
    log("[tiny-table]")
    X, Y = to_device(p)
    opt = sptc.default_options(out_table_slots=64, mode=1)
    with sptc.plan(X, Y, p.cx, p.cy, options=opt) as pl:
        with pytest.raises(sptc.SptcError) as e:
            pl.execute()
        assert e.value.status == 5


def test_out_of_range_coordinate_is_rejected():
    import paper_2410_10094_amd as sptc
    p = W.plain(seed=7, n=16, nnz=100)
    p.X.idx[0, 17] = 16  # one past the end of mode 0
    log("[validate]")
    X, Y = to_device(p)
    with pytest.raises(sptc.SptcError) as e:
        sptc.plan(X, Y, p.cx, p.cy)
    assert e.value.status == 1


def _co_problems():
    """Many dense block-class groups of uneven sizes (many more tiles than
    waves in flight), explicit zero values, repeated X coordinates, and one
    group far larger than the rest."""
    rng = np.random.default_rng(71)
    out = []

    def y_dense(C, per):
        ny = C * per
        yi = np.stack([np.repeat(np.arange(C), per), rng.integers(0, 64, ny), rng.integers(0, 64, ny)])
        return Coo((C, 64, 64), yi.astype(np.int32), W.nonzero_uniform(rng, ny))

    # ~2000 groups, most with ~20 entries, every 50th with ~700
    C = 1024
    cols = []
    for g in range(2000):
        n = 700 if g % 50 == 0 else int(rng.integers(8, 32))
        ks = rng.choice(C, n, replace=False)
        cols.append(np.stack([np.full(n, g // 40), np.full(n, g % 40), ks]))
    xi = np.concatenate(cols, axis=1).astype(np.int32)
    xv = W.nonzero_uniform(rng, xi.shape[1])
    xv[::97] = 0.0  # zero products still make outputs
    dup = xi[:, :300:7]  # repeated X coordinates (additive)
    xi = np.concatenate([xi, dup], axis=1)
    xv = np.concatenate([xv, W.nonzero_uniform(rng, dup.shape[1])])
    out.append(Problem("co-2000-groups", Coo((50, 40, C), xi, xv), y_dense(C, 30), (2,), (0,)))
    # ~300 groups of 40-400 entries
    cols = []
    for g in range(300):
        n = int(rng.integers(40, 400))
        cols.append(np.stack([np.full(n, g // 20), np.full(n, g % 20), rng.choice(C, n, replace=False)]))
    xi = np.concatenate(cols, axis=1).astype(np.int32)
    out.append(Problem("co-300-groups", Coo((15, 20, C), xi, W.nonzero_uniform(rng, xi.shape[1])),
                       y_dense(C, 20), (2,), (0,)))
    # a group of 5000 entries among 2000 small ones (13-bit Y free key)
    C2 = 8192
    cols = [np.stack([np.zeros(5000, int), np.zeros(5000, int), rng.choice(C2, 5000, replace=False)])]
    for g in range(1, 2000):
        n = int(rng.integers(10, 20))
        cols.append(np.stack([np.full(n, g // 40), np.full(n, g % 40), rng.choice(C2, n, replace=False)]))
    xi = np.concatenate(cols, axis=1).astype(np.int32)
    out.append(Problem("co-fallback", Coo((50, 40, C2), xi, W.nonzero_uniform(rng, xi.shape[1])),
                       y_dense(C2, 40), (2,), (0,)))
    return out


@pytest.mark.parametrize("mfma", [0, 1], ids=["walk", "mfma"])
@pytest.mark.parametrize("p", _co_problems(), ids=lambda p: p.name)
def test_dense_block_many_groups(p, mfma):
    """Both dense block-class kernels: the sliced walk and the matrix-core
    product."""
    import paper_2410_10094_amd as sptc
    log(f"[co] {p.name} nnz {p.X.nnz}x{p.Y.nnz} block_mfma {mfma}")
    info, gidx, gval = run_gpu(p, options=sptc.default_options(block_mfma=mfma))
    assert info["classes"]["block"] > 100, info["classes"]
    assert info["block_mfma"] == (mfma == 1)
    assert_parity(p, gidx, gval)
