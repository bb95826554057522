"""CPU oracle for sparse tensor contraction -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It computes the contraction by its
definition (paper section 2.2, Eq. 2) with a nested-loop / index join and a
``std::map`` accumulator in ``oracle.cpp``, and shares no code with the GPU
library.  Inputs are host numpy arrays (``workloads.Coo``-like objects with
``dims``, ``idx`` int32 ``[order, nnz]`` and ``val`` float64 ``[nnz]``).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCE = os.path.join(_HERE, "oracle.cpp")

_ERRORS = {1: "invalid argument", 2: "contracted modes of unequal length", 3: "out of memory"}


def build(force: bool = True) -> str:
    """Compile ``oracle.cpp`` with g++ (no fused multiply-add) into liboracle.so."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-pthread", SOURCE, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        tens = [i32, P, i64, P, P]
        lib.oracle_contract.argtypes = tens + tens + [i32, P, P, i32, ctypes.POINTER(ctypes.c_void_p)]
        lib.oracle_contract.restype = ctypes.c_int
        lib.oracle_result_nnz.argtypes = [P]
        lib.oracle_result_nnz.restype = i64
        lib.oracle_result_order.argtypes = [P]
        lib.oracle_result_order.restype = i32
        lib.oracle_result_copy.argtypes = [P, P, P, P, P]
        lib.oracle_result_free.argtypes = [P]
        lib.oracle_group_counts.argtypes = [i32, P, i64, P, i32, P, i64, P, P, P]
        lib.oracle_group_counts.restype = ctypes.c_int
        lib.oracle_match_counts.argtypes = tens + tens + [i32, P, P, P, P]
        lib.oracle_match_counts.restype = ctypes.c_int
        lib.oracle_sample_outputs.argtypes = tens + tens + [i32, P, P, i64, ctypes.c_uint64, P]
        lib.oracle_sample_outputs.restype = ctypes.c_int
        lib.oracle_values_at.argtypes = tens + tens + [i32, P, P, i64, P, P, P, P]
        lib.oracle_values_at.restype = ctypes.c_int
        lib.oracle_count_outputs.argtypes = tens + tens + [i32, P, P, i32, P]
        lib.oracle_count_outputs.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


class _Keep:
    """Holds contiguous copies alive for the duration of a call."""

    def __init__(self, T):
        self.dims = np.ascontiguousarray(np.asarray(T.dims, dtype=np.int64))
        self.idx = np.ascontiguousarray(np.asarray(T.idx, dtype=np.int32)).reshape(len(T.dims), -1)
        self.val = np.ascontiguousarray(np.asarray(T.val, dtype=np.float64)).reshape(-1)
        self.args = [len(T.dims), _ptr(self.dims), self.val.shape[0], _ptr(self.idx), _ptr(self.val)]


def _modes(c: Sequence[int]):
    a = np.ascontiguousarray(np.asarray(list(c), dtype=np.int32))
    return a, _ptr(a)


def _check(rc: int):
    if rc != 0:
        raise ValueError(f"oracle: {_ERRORS.get(rc, rc)}")


@dataclasses.dataclass
class OracleResult:
    """Output of the oracle, sorted lexicographically by coordinate."""

    idx: np.ndarray      # int32 [order, nnz]
    val: np.ndarray      # float64 [nnz]
    absval: np.ndarray   # float64 [nnz]: sum of |x*y| over each output's terms
    terms: np.ndarray    # int64 [nnz]: number of products summed into each output

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])


def contract(X, Y, cx: Sequence[int], cy: Sequence[int], nthreads: int = 1) -> OracleResult:
    """Z = X contracted with Y over the paired modes cx[t] <-> cy[t]."""
    lib = _load()
    kx, ky = _Keep(X), _Keep(Y)
    ax, px = _modes(cx)
    ay, py = _modes(cy)
    h = ctypes.c_void_p()
    _check(lib.oracle_contract(*kx.args, *ky.args, len(cx), px, py, int(nthreads), ctypes.byref(h)))
    try:
        n = lib.oracle_result_nnz(h)
        order = lib.oracle_result_order(h)
        idx = np.zeros((order, n), dtype=np.int32)
        val = np.zeros(n, dtype=np.float64)
        absval = np.zeros(n, dtype=np.float64)
        terms = np.zeros(n, dtype=np.int64)
        lib.oracle_result_copy(h, _ptr(idx), _ptr(val), _ptr(absval), _ptr(terms))
    finally:
        lib.oracle_result_free(h)
    return OracleResult(idx, val, absval, terms)


def group_counts(Y, cy: Sequence[int]):
    """Distinct contracting tuples of Y (ascending) and their entry counts:
    returns (tuples int32 [nc, k], counts int64 [k])."""
    lib = _load()
    ky = _Keep(Y)
    ay, py = _modes(cy)
    cap = max(1, ky.val.shape[0])
    tuples = np.zeros((len(cy), cap), dtype=np.int32)
    counts = np.zeros(cap, dtype=np.int64)
    ng = ctypes.c_int64()
    _check(lib.oracle_group_counts(ky.args[0], ky.args[1], ky.args[2], ky.args[3], len(cy), py, cap,
                                   _ptr(tuples), _ptr(counts), ctypes.byref(ng)))
    k = ng.value
    return np.ascontiguousarray(tuples[:, :k]), counts[:k]


def match_counts(X, Y, cx, cy):
    """Per X entry, how many Y entries share its contracting tuple; and the
    total number of matching (x, y) pairs."""
    lib = _load()
    kx, ky = _Keep(X), _Keep(Y)
    ax, px = _modes(cx)
    ay, py = _modes(cy)
    per_x = np.zeros(max(1, kx.val.shape[0]), dtype=np.int64)
    total = ctypes.c_int64()
    _check(lib.oracle_match_counts(*kx.args, *ky.args, len(cx), px, py, _ptr(per_x), ctypes.byref(total)))
    return per_x[: kx.val.shape[0]], total.value


def sample_outputs(X, Y, cx, cy, n: int, seed: int) -> np.ndarray:
    """``n`` output coordinates drawn from matching pairs (int32 [order, n])."""
    lib = _load()
    kx, ky = _Keep(X), _Keep(Y)
    ax, px = _modes(cx)
    ay, py = _modes(cy)
    order = len(X.dims) + len(Y.dims) - 2 * len(cx)
    coords = np.zeros((max(order, 1), n), dtype=np.int32)
    _check(lib.oracle_sample_outputs(*kx.args, *ky.args, len(cx), px, py, n, seed, _ptr(coords)))
    return coords[:order]


def values_at(X, Y, cx, cy, coords: np.ndarray):
    """Evaluate the contraction at the given output coordinates (int32
    [order, n]); returns (val, absval, terms)."""
    lib = _load()
    kx, ky = _Keep(X), _Keep(Y)
    ax, px = _modes(cx)
    ay, py = _modes(cy)
    coords = np.ascontiguousarray(coords, dtype=np.int32)
    n = coords.shape[1]
    val = np.zeros(max(n, 1))
    absval = np.zeros(max(n, 1))
    terms = np.zeros(max(n, 1), dtype=np.int64)
    _check(lib.oracle_values_at(*kx.args, *ky.args, len(cx), px, py, n, _ptr(coords) if coords.size else None,
                                _ptr(val), _ptr(absval), _ptr(terms)))
    return val[:n], absval[:n], terms[:n]


def count_outputs(X, Y, cx, cy, nthreads: int = 1) -> int:
    """nnz of the contraction: the size of the output coordinate set of Eq. 2
    (every coordinate reached by a matching pair, zero sums included),
    counted without forming any value."""
    lib = _load()
    kx, ky = _Keep(X), _Keep(Y)
    ax, px = _modes(cx)
    ay, py = _modes(cy)
    n = ctypes.c_int64()
    _check(lib.oracle_count_outputs(*kx.args, *ky.args, len(cx), px, py, int(nthreads), ctypes.byref(n)))
    return n.value
