"""Pins the CPU oracle to things other than itself: dense einsum and matmul,
a brute-force pair loop, the worked examples printed in the paper, and
invariants of Eq. 2.  Runs on the CPU."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2410_10094_amd import workloads as W
from paper_2410_10094_amd.workloads import Coo, Problem
from tests import helpers as H


def _dense_of_result(r, out_dims):
    D = np.zeros(out_dims)
    T = np.zeros(out_dims)
    A = np.zeros(out_dims)
    if r.nnz:
        np.add.at(D, tuple(r.idx.astype(np.int64)), r.val)
        np.add.at(T, tuple(r.idx.astype(np.int64)), r.terms)
        np.add.at(A, tuple(r.idx.astype(np.int64)), r.absval)
    elif len(out_dims) == 0 and r.val.size:
        D, T, A = r.val[0], r.terms[0], r.absval[0]
    return D, T, A


def _out_dims(p):
    return tuple(p.X.dims[m] for m in range(p.X.order) if m not in p.cx) + \
        tuple(p.Y.dims[m] for m in range(p.Y.order) if m not in p.cy)


@pytest.mark.parametrize("p", H.tiny_problems(60), ids=lambda p: p.name)
def test_oracle_matches_dense_einsum(p):
    """Eq. 2 on densified tensors: values, term counts (einsum of indicator
    tensors) and |term| sums must agree; the emitted coordinates are exactly
    the cells with at least one term."""
    r = oracle.contract(p.X, p.Y, p.cx, p.cy)
    ref_val, ref_terms, ref_abs = H.dense_reference(p)
    out_dims = _out_dims(p)
    if len(out_dims) == 0:
        assert r.idx.shape == (0, r.nnz)
        assert r.nnz == (1 if ref_terms > 0 else 0)
        if r.nnz:
            assert r.terms[0] == ref_terms
            assert abs(r.val[0] - ref_val) <= 1e-12 * max(abs(ref_val), ref_abs)
        return
    # sorted, distinct coordinates
    if r.nnz > 1:
        lin = np.ravel_multi_index(tuple(r.idx.astype(np.int64)), out_dims)
        assert np.all(np.diff(lin) > 0)
    got_val, got_terms, got_abs = _dense_of_result(r, out_dims)
    np.testing.assert_array_equal(got_terms, ref_terms)
    assert set(map(tuple, np.argwhere(ref_terms > 0))) == set(map(tuple, r.idx.T.tolist()))
    np.testing.assert_allclose(got_val, ref_val, rtol=0, atol=1e-12 * max(1.0, float(np.max(np.abs(ref_abs), initial=0))))
    np.testing.assert_allclose(got_abs, ref_abs, rtol=1e-13, atol=0)


@pytest.mark.parametrize("seed", range(6))
def test_oracle_matrix_multiply_special_case(seed):
    """Section 2.2, Fig. 2: an order-2 contraction of X's mode 1 with Y's mode
    0 is the matrix product."""
    rng = np.random.default_rng(seed)
    m, k, n = rng.integers(1, 12, size=3)
    A = np.where(rng.random((m, k)) < 0.4, rng.uniform(-1, 1, (m, k)), 0.0)
    B = np.where(rng.random((k, n)) < 0.4, rng.uniform(-1, 1, (k, n)), 0.0)
    ai, bi = np.nonzero(A), np.nonzero(B)
    X = Coo((m, k), np.stack(ai), A[ai])
    Y = Coo((k, n), np.stack(bi), B[bi])
    r = oracle.contract(X, Y, [1], [0])
    C = np.zeros((m, n))
    if r.nnz:
        C[tuple(r.idx)] = r.val
    np.testing.assert_allclose(C, A @ B, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("p", H.tiny_problems(25, seed0=5000), ids=lambda p: p.name)
def test_oracle_bit_exact_with_brute_force(p):
    """A Python loop over all pairs in the same order (x, then y) must give
    the same coordinates and bit-identical values."""
    ref = H.brute_force(p)
    r = oracle.contract(p.X, p.Y, p.cx, p.cy)
    got = {tuple(int(c) for c in r.idx[:, e]): r.val[e] for e in range(r.nnz)}
    assert got.keys() == ref.keys()
    for k, v in ref.items():
        assert got[k] == v, (k, got[k], v)


def test_oracle_nested_and_index_join_agree():
    """Above ~2e6 pairs the oracle switches from the nested loop to the Y
    index; both sides of the switch must agree with brute force."""
    for nx, ny in [(1400, 1400), (1500, 1500)]:
        p = W.random_problem(77, 3, 3, 1, 8, 20, nx, ny)
        ref = H.brute_force(p)
        r = oracle.contract(p.X, p.Y, p.cx, p.cy)
        got = {tuple(int(c) for c in r.idx[:, e]): r.val[e] for e in range(r.nnz)}
        assert got == ref


def test_golden_accumulation_example():
    g = H.load_golden("accumulation_example.json")
    X, Y = H.coo_from(g["X"]), H.coo_from(g["Y"])
    r = oracle.contract(X, Y, g["cx"], g["cy"])
    np.testing.assert_array_equal(r.idx, np.array(g["expected"]["idx"]))
    assert r.val.tolist() == g["expected"]["val"]
    assert r.terms.tolist() == [2]


def test_golden_signature_example():
    g = H.load_golden("signature_example.json")
    X, Y = H.coo_from(g["X"]), H.coo_from(g["Y"])
    r = oracle.contract(X, Y, g["cx"], g["cy"])
    np.testing.assert_array_equal(r.idx, np.array(g["expected"]["idx"]))
    assert r.val.tolist() == g["expected"]["val"]


def test_golden_bound_example():
    g = H.load_golden("bound_example.json")
    X, Y = H.coo_from(g["X"]), H.coo_from(g["Y"])
    per_x, total = oracle.match_counts(X, Y, g["cx"], g["cy"])
    assert per_x.tolist() == g["expected"]["per_x"]
    assert total == g["expected"]["total"]
    # the number of products equals the number of terms the contraction sums
    r = oracle.contract(X, Y, g["cx"], g["cy"])
    assert int(r.terms.sum()) == g["expected"]["total"]


def test_golden_counting_sort_example():
    g = H.load_golden("counting_sort_example.json")
    Y = H.coo_from(g["Y"])
    tuples, counts = oracle.group_counts(Y, g["cy"])
    got = {int(t): int(c) for t, c in zip(tuples[0], counts)}
    for k, v in g["expected"]["counts"].items():
        assert got[int(k)] == v
    for k in g["expected"]["absent"]:
        assert k not in got
    # cumulative count up to value 3 is where the first 3 lands (1-based)
    assert sum(c for t, c in got.items() if t <= 3) == g["expected"]["end_position_of_3"]
    assert counts.sum() == Y.nnz and np.all(np.diff(tuples[0]) > 0)


@pytest.mark.parametrize("p", H.tiny_problems(15, seed0=9000) + [W.plain(n=12, nnz=150)], ids=lambda p: p.name)
def test_value_sum_identity(p):
    """By bilinearity of Eq. 2, the sum of all outputs equals the sum over
    contracting tuples k of (sum X_k)(sum Y_k).  The oracle's outputs are each
    within k*u*sum|terms| of their exact value."""
    r = oracle.contract(p.X, p.Y, p.cx, p.cy)
    exact = H.exact_key_sum_identity(p)
    got = sum((Fraction(float(v)) for v in r.val), Fraction(0))
    bound = float(sum(1.0001 * t * H.U * a for t, a in zip(r.terms, r.absval)))
    assert abs(float(got - exact)) <= bound + 1e-300


@pytest.mark.parametrize("p", H.tiny_problems(15, seed0=9100) + [W.plain(n=10, nnz=120)], ids=lambda p: p.name)
def test_coordinate_set_identity(p):
    """The output coordinates are exactly the free-coordinate pairs that share
    a contracting tuple."""
    r = oracle.contract(p.X, p.Y, p.cx, p.cy)
    assert set(map(tuple, r.idx.T.tolist())) == H.free_pair_set(p) if r.idx.shape[0] else \
        (r.nnz == (1 if H.free_pair_set(p) else 0))


@pytest.mark.parametrize("seed", range(8))
def test_operand_swap_symmetry(seed):
    """Section 5.4: swapping operands gives the same tensor with X's and Y's
    free modes exchanged; coordinates and term counts exact, values within the
    reordering bound."""
    p = W.random_problem(300 + seed, 3, 4, 1 + seed % 2, 2, 7, 80, 90)
    a = oracle.contract(p.X, p.Y, p.cx, p.cy)
    b = oracle.contract(p.Y, p.X, p.cy, p.cx)
    nfx = p.X.order - len(p.cx)
    nfy = p.Y.order - len(p.cy)
    perm = list(range(nfy, nfy + nfx)) + list(range(nfy))
    bi, bv, bt, ba = H.sort_coo(b.idx[perm], b.val, b.terms, b.absval)
    np.testing.assert_array_equal(a.idx, bi)
    np.testing.assert_array_equal(a.terms, bt)
    H.assert_values_close(bv, a.val, a.absval, a.terms)


@pytest.mark.parametrize("k", [-3, 1, 7])
def test_power_of_two_scaling_is_exact(k):
    p = W.random_problem(400 + k, 3, 3, 1, 3, 9, 150, 150)
    a = oracle.contract(p.X, p.Y, p.cx, p.cy)
    X2 = Coo(p.X.dims, p.X.idx, p.X.val * 2.0 ** k)
    b = oracle.contract(X2, p.Y, p.cx, p.cy)
    np.testing.assert_array_equal(a.idx, b.idx)
    assert np.array_equal(a.val * 2.0 ** k, b.val)


def test_thread_count_does_not_change_results():
    p = W.random_problem(501, 3, 3, 1, 20, 40, 3000, 3000)
    a = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=1)
    for t in (2, 3, 8):
        b = oracle.contract(p.X, p.Y, p.cx, p.cy, nthreads=t)
        np.testing.assert_array_equal(a.idx, b.idx)
        assert np.array_equal(a.val, b.val)
    # leading output coordinate from Y when X has no free mode
    q = W.random_problem(502, 1, 3, 1, 20, 40, 15, 3000)
    a = oracle.contract(q.X, q.Y, q.cx, q.cy, nthreads=1)
    b = oracle.contract(q.X, q.Y, q.cx, q.cy, nthreads=5)
    np.testing.assert_array_equal(a.idx, b.idx)
    assert np.array_equal(a.val, b.val)


def test_edge_outer_product_and_full_contraction():
    p = W.random_problem(601, 2, 2, 0, 2, 5, 7, 9)
    r = oracle.contract(p.X, p.Y, [], [])
    assert r.nnz == p.X.nnz * p.Y.nnz  # distinct coords on both sides
    assert int(r.terms.sum()) == p.X.nnz * p.Y.nnz
    q = W.random_problem(602, 2, 2, 2, 3, 3, 6, 6)
    r = oracle.contract(q.X, q.Y, q.cx, q.cy)
    ref, terms, _ = H.dense_reference(q)
    assert r.idx.shape[0] == 0 and r.nnz == (1 if terms > 0 else 0)


def test_edge_empty_and_explicit_zero():
    X = Coo((4, 4), np.zeros((2, 0), np.int32), np.zeros(0))
    Y = Coo((4, 4), np.array([[1], [2]], np.int32), np.array([3.0]))
    assert oracle.contract(X, Y, [1], [0]).nnz == 0
    assert oracle.contract(Y, X, [1], [0]).nnz == 0
    # explicit zero values still produce structural outputs, and a sum that
    # cancels exactly is still emitted
    X = Coo((2, 3), np.array([[0, 0], [1, 2]], np.int32), np.array([0.0, 1.0]))
    Y = Coo((3, 2), np.array([[1, 2], [1, 1]], np.int32), np.array([5.0, -5.0]))
    r = oracle.contract(X, Y, [1], [0])
    assert r.idx.tolist() == [[0], [1]] and r.val.tolist() == [-5.0] and r.terms.tolist() == [2]
    X = Coo((1, 2), np.array([[0, 0], [0, 1]], np.int32), np.array([1.0, 1.0]))
    Y = Coo((2, 1), np.array([[0, 1], [0, 0]], np.int32), np.array([2.5, -2.5]))
    r = oracle.contract(X, Y, [1], [0])
    assert r.nnz == 1 and r.val[0] == 0.0 and r.terms[0] == 2


def test_oracle_rejects_bad_arguments():
    X = Coo((4, 5), np.array([[1], [2]], np.int32), np.array([1.0]))
    Y = Coo((6, 4), np.array([[1], [2]], np.int32), np.array([1.0]))
    with pytest.raises(ValueError, match="unequal"):
        oracle.contract(X, Y, [1], [0])
    with pytest.raises(ValueError):
        oracle.contract(X, Y, [0, 0], [1, 1])
    with pytest.raises(ValueError):
        oracle.contract(X, Y, [2], [0])
    bad = Coo((4, 5), np.array([[1], [5]], np.int32), np.array([1.0]))
    with pytest.raises(ValueError):
        oracle.contract(bad, Y, [0], [1])


def test_sampled_values_match_full_result():
    p = W.block_sparse(n=16, block=4, p_block=0.3)
    r = oracle.contract(p.X, p.Y, p.cx, p.cy)
    coords = oracle.sample_outputs(p.X, p.Y, p.cx, p.cy, 500, seed=3)
    val, absval, terms = oracle.values_at(p.X, p.Y, p.cx, p.cy, coords)
    lin_r = np.ravel_multi_index(tuple(r.idx.astype(np.int64)), (16,) * 4)
    lin_q = np.ravel_multi_index(tuple(coords.astype(np.int64)), (16,) * 4)
    pos = np.searchsorted(lin_r, lin_q)
    assert np.array_equal(lin_r[pos], lin_q)
    assert np.array_equal(val, r.val[pos]) and np.array_equal(terms, r.terms[pos])
    assert np.array_equal(absval, r.absval[pos])
    # a coordinate no pair reaches has no terms
    v, a, t = oracle.values_at(p.X, p.Y, p.cx, p.cy, np.zeros((4, 1), np.int32) + 15)
    assert t[0] == 0 or (r.idx[:, -1] == 15).all()


@pytest.mark.parametrize("p", H.tiny_problems(40, seed0=9300) + [W.plain(n=10, nnz=120)], ids=lambda p: p.name)
def test_output_count_is_the_coordinate_set_size(p):
    """nnz(Z) counted without values equals the size of the set of
    free-coordinate pairs that share a contracting tuple (a Python set built
    per key), and the number of cells einsum reaches with indicator
    tensors."""
    n = oracle.count_outputs(p.X, p.Y, p.cx, p.cy)
    assert n == len(H.free_pair_set(p))
    _, terms, _ = H.dense_reference(p)
    assert n == int(np.count_nonzero(terms))
    assert n == oracle.contract(p.X, p.Y, p.cx, p.cy).nnz


def test_output_count_takes_the_union_over_keys():
    """An X free tuple whose entries carry several contracting tuples reaches
    the union of their Y free tuples: here 2 keys, each with Y free tuples
    {0, 1} and {1, 2}, give 3 outputs, not 4.  Repeated entries count once."""
    X = Coo((1, 2), np.array([[0, 0, 0], [0, 1, 1]], np.int32), np.array([1.0, 2.0, 3.0]))
    Y = Coo((2, 3), np.array([[0, 0, 1, 1, 1], [0, 1, 1, 2, 2]], np.int32), np.ones(5))
    assert oracle.count_outputs(X, Y, [1], [0]) == 3
    assert oracle.contract(X, Y, [1], [0]).nnz == 3


def test_output_count_threads_and_sizes():
    p = W.random_problem(701, 3, 3, 1, 20, 40, 3000, 3000)
    n = oracle.count_outputs(p.X, p.Y, p.cx, p.cy)
    assert n == oracle.contract(p.X, p.Y, p.cx, p.cy).nnz
    for t in (2, 7):
        assert oracle.count_outputs(p.X, p.Y, p.cx, p.cy, nthreads=t) == n
    q = W.block_sparse(n=16, block=4, p_block=0.3)
    assert oracle.count_outputs(q.X, q.Y, q.cx, q.cy, nthreads=4) == oracle.contract(q.X, q.Y, q.cx, q.cy).nnz
