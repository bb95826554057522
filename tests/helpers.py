"""Shared test helpers: dense references, brute force and the value tolerance.

Nothing here is used by the GPU library; the GPU tests call the library
through its C ABI and compare against ``oracle``.
"""
from __future__ import annotations

import json
import math
import os
import string
from typing import Sequence

import numpy as np

from paper_2410_10094_amd.workloads import Coo, Problem

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U = 2.0 ** -53  # unit roundoff of IEEE double, round to nearest


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def coo_from(d) -> Coo:
    return Coo(tuple(d["dims"]), np.array(d["idx"], dtype=np.int32).reshape(len(d["dims"]), -1),
               np.array(d["val"], dtype=np.float64))


def densify(T: Coo, values=None) -> np.ndarray:
    """Dense array of a COO tensor; repeated coordinates add up."""
    D = np.zeros(T.dims, dtype=np.float64)
    v = T.val if values is None else values
    np.add.at(D, tuple(T.idx.astype(np.int64)), v)
    return D


def einsum_spec(order_x, order_y, cx, cy):
    """einsum subscripts for Eq. 2: paired modes share a letter; the output is
    X's free letters ascending, then Y's free letters ascending."""
    letters = iter(string.ascii_letters)
    xs = [next(letters) for _ in range(order_x)]
    ys = [next(letters) for _ in range(order_y)]
    for a, b in zip(cx, cy):
        ys[b] = xs[a]
    out = [xs[m] for m in range(order_x) if m not in cx] + [ys[m] for m in range(order_y) if m not in cy]
    return "".join(xs) + "," + "".join(ys) + "->" + "".join(out)


def dense_reference(p: Problem):
    """(values, term counts, |term| sums) of Eq. 2 on dense arrays via einsum."""
    spec = einsum_spec(p.X.order, p.Y.order, p.cx, p.cy)
    val = np.einsum(spec, densify(p.X), densify(p.Y))
    terms = np.einsum(spec, densify(p.X, np.ones(p.X.nnz)), densify(p.Y, np.ones(p.Y.nnz)))
    absv = np.einsum(spec, densify(p.X, np.abs(p.X.val)), densify(p.Y, np.abs(p.Y.val)))
    return val, terms, absv


def brute_force(p: Problem):
    """All pairs, in input order of x then y, summed into a dict in Python
    floats.  Returns {coordinate tuple: value}."""
    X, Y = p.X, p.Y
    fx = [m for m in range(X.order) if m not in p.cx]
    fy = [m for m in range(Y.order) if m not in p.cy]
    acc = {}
    for i in range(X.nnz):
        for j in range(Y.nnz):
            if all(X.idx[a, i] == Y.idx[b, j] for a, b in zip(p.cx, p.cy)):
                key = tuple(int(X.idx[m, i]) for m in fx) + tuple(int(Y.idx[m, j]) for m in fy)
                acc[key] = acc.get(key, 0.0) + float(X.val[i]) * float(Y.val[j])
    return acc


def sort_coo(idx: np.ndarray, *vals):
    """Sort COO columns lexicographically (first mode most significant)."""
    idx = np.asarray(idx)
    if idx.shape[0] == 0 or idx.shape[1] == 0:
        return (idx,) + tuple(vals)
    order = np.lexsort(idx[::-1])
    return (idx[:, order],) + tuple(np.asarray(v)[order] for v in vals)


def value_tolerance(ref_val, absval, terms, rel=1e-12):
    """Allowed |gpu - oracle| per output: the larger of rel*|z| and
    min(2.0002*k*u*S, rel*S), where k is the output's number of terms and S
    their sum of |x*y|; a single-term output must match bit for bit.

    Where a sum cancels, rel*|z| alone would ask for more than either side's
    rounding can give, so the bar falls back to rel*S (1e-12 of the summation
    error scale).  Below about 4,500 terms the rounding-error bound is the
    tighter of the two.  With fl(a op b) = (a op b)(1 + d), |d| <= u, and
    gamma_n = n*u/(1 - n*u): a sum of the k rounded products in any order
    (the oracle, the LDS classes) is within u*S + gamma_(k-1)*(1+u)*S <=
    gamma_k*S of the exact sum; a chain of k fused multiply-adds from zero
    (the matrix cores: each exact product added with one rounding) is within
    gamma_k*S too, and so is that chain when r repeated X coordinates are
    summed before their multiply (r - 1 more roundings on those terms, r - 1
    fewer steps in the chain: no term is rounded more than k times).  Two
    results within gamma_k*S of the same exact sum differ by at most
    2*gamma_k*S <= 2.0002*k*u*S (k*u <= 1e-4).  Above about 4,500 terms the
    bar stays at rel*S: a statistical bar there, not a worst case (rounding
    errors of many terms behave like a random walk, of order sqrt(k)*u*S)."""
    k = np.asarray(terms, dtype=np.float64)
    S = np.asarray(absval)
    bound = np.minimum(2.0002 * k * U * S, rel * S)
    return np.maximum(rel * np.abs(ref_val), bound) * (k > 1)


def value_error_stats(got, ref_val, absval, terms):
    """Worst |gpu - oracle| as a fraction of 1e-12 * sum|x*y| over the
    multi-term outputs, and how many outputs needed the second clause of the
    tolerance (their error exceeds 1e-12 * |z|)."""
    got = np.asarray(got)
    err = np.abs(got - ref_val)
    multi = np.asarray(terms) > 1
    scale = 1e-12 * np.asarray(absval)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(multi & (scale > 0), err / scale, 0.0)
    second = int(np.count_nonzero(multi & (err > 1e-12 * np.abs(ref_val))))
    return {"worst_ratio_to_1e-12_sum_abs": float(ratio.max(initial=0.0)), "second_clause": second,
            "multi_term_outputs": int(np.count_nonzero(multi))}


def assert_values_close(got, ref_val, absval, terms, rel=1e-12):
    """Checks every value against value_tolerance; returns value_error_stats."""
    got = np.asarray(got)
    tol = value_tolerance(ref_val, absval, terms, rel)
    err = np.abs(got - ref_val)
    bad = np.flatnonzero(~(err <= tol))
    if bad.size:
        i = bad[0]
        raise AssertionError(f"{bad.size} values out of tolerance; first at {i}: got {got[i]!r} "
                             f"want {ref_val[i]!r} (terms {terms[i]}, |sum| {absval[i]!r}, tol {tol[i]!r})")
    return value_error_stats(got, ref_val, absval, terms)


def exact_key_sum_identity(p: Problem):
    """Sum over contracting tuples k of (sum of X values with key k) * (sum of
    Y values with key k), evaluated exactly in rationals (float result)."""
    from fractions import Fraction
    kx = {}
    for i in range(p.X.nnz):
        k = tuple(int(p.X.idx[c, i]) for c in p.cx)
        kx[k] = kx.get(k, Fraction(0)) + Fraction(float(p.X.val[i]))
    ky = {}
    for j in range(p.Y.nnz):
        k = tuple(int(p.Y.idx[c, j]) for c in p.cy)
        ky[k] = ky.get(k, Fraction(0)) + Fraction(float(p.Y.val[j]))
    return sum((kx[k] * ky[k] for k in kx if k in ky), Fraction(0))


def free_pair_set(p: Problem):
    """Set of (X free coords + Y free coords) over pairs that share a
    contracting tuple, built per key as a Cartesian product."""
    fx = [m for m in range(p.X.order) if m not in p.cx]
    fy = [m for m in range(p.Y.order) if m not in p.cy]
    xs, ys = {}, {}
    for i in range(p.X.nnz):
        xs.setdefault(tuple(int(p.X.idx[c, i]) for c in p.cx), set()).add(tuple(int(p.X.idx[m, i]) for m in fx))
    for j in range(p.Y.nnz):
        ys.setdefault(tuple(int(p.Y.idx[c, j]) for c in p.cy), set()).add(tuple(int(p.Y.idx[m, j]) for m in fy))
    out = set()
    for k, a in xs.items():
        for b in ys.get(k, ()):
            for f in a:
                out.add(f + b)
    return out


def tiny_problems(count: int, seed0: int = 1000):
    """Random tiny contractions: orders 1-4, 0-2 pairs, dims <= 6."""
    from paper_2410_10094_amd.workloads import random_problem
    rng = np.random.default_rng(seed0)
    out = []
    for s in range(count):
        ox, oy = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        nc = int(rng.integers(0, min(ox, oy, 2) + 1))
        dup = bool(s % 5 == 4)
        nx, ny = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        out.append(random_problem(seed0 + s, ox, oy, nc, 1, 6, nx, ny, duplicates=dup))
    return out
