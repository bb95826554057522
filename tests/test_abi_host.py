"""The C-ABI library loads and exports every declared symbol, and argument
validation (which runs before any HIP call) reports the right status.  CPU
only: no call here reaches the GPU."""
import ctypes
import os
import re

import pytest

from paper_2410_10094_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "sptc.h")) as f:
        text = f.read()
    return re.findall(r"SPTC_API\s+[\w\s\*]+?\b(sptc_\w+)\s*\(", text)


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = declared_functions()
    assert len(names) >= 11
    assert set(names) == set(B.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    for s in range(8):
        assert B.status_string(s)
    assert B.status_string(0) == "success"


def test_default_options():
    o = B.default_options()
    assert abs(o.load_factor - 1 / 1.3) < 1e-15
    assert o.validate == 1 and o.max_probe == 0 and o.out_table_slots == 0
    assert o.block_mfma == 0  # the matrix-core block class is opt-in
    assert o.tile == 0 and o.lds_max_keys == 0 and o.capture_out_cap == 0
    assert o.operand_order == 0  # the grouped mode picks the operand to group


def _plan(X, Y, cx, cy, opt=None):
    lib = B.load()
    h = ctypes.c_void_p(12345)
    acx, acy = B.int_array(cx), B.int_array(cy)
    st = lib.sptc_plan(ctypes.byref(h), ctypes.byref(X) if X is not None else None,
                       ctypes.byref(Y) if Y is not None else None, len(cx), acx, acy,
                       ctypes.byref(opt) if opt is not None else None, None, None)
    return st, h.value


# Non-null fake device pointers: validation never dereferences them.
FAKE = 0x1000


def coo(dims, nnz=4, idx=FAKE, val=FAKE):
    c, keep = B.make_coo(len(dims), dims, nnz, idx, val)
    coo.keep.append(keep)
    return c


coo.keep = []


@pytest.mark.parametrize("case,status", [
    ("dim_mismatch", B.ERR_DIM_MISMATCH),
    ("repeated_mode", B.ERR_INVALID_ARG),
    ("mode_out_of_range", B.ERR_INVALID_ARG),
    ("order_too_big", B.ERR_INVALID_ARG),
    ("zero_dim", B.ERR_INVALID_ARG),
    ("negative_nnz", B.ERR_INVALID_ARG),
    ("null_idx", B.ERR_INVALID_ARG),
    ("null_tensor", B.ERR_INVALID_ARG),
    ("too_many_pairs", B.ERR_INVALID_ARG),
    ("output_key_overflow_global_mode", B.ERR_KEY_OVERFLOW),
    ("free_key_overflow", B.ERR_KEY_OVERFLOW),
    ("bad_mode", B.ERR_INVALID_ARG),
    ("bad_load_factor", B.ERR_INVALID_ARG),
    ("bad_table_slots", B.ERR_INVALID_ARG),
    ("bad_tile", B.ERR_INVALID_ARG),
    ("bad_lds_max_keys", B.ERR_INVALID_ARG),
    ("negative_capture_out_cap", B.ERR_INVALID_ARG),
    ("capture_without_allocator", B.ERR_INVALID_ARG),
    ("bad_operand_order", B.ERR_INVALID_ARG),
])
def test_plan_validation(case, status):
    X, Y, cx, cy, opt = coo((8, 9, 10)), coo((10, 9, 7)), [2], [0], None
    if case == "dim_mismatch":
        cx, cy = [1], [0]
    elif case == "repeated_mode":
        cx, cy = [2, 2], [0, 1]
    elif case == "mode_out_of_range":
        cx, cy = [3], [0]
    elif case == "order_too_big":
        X = coo((2,) * 17)
        cx, cy = [0], [1]
        Y = coo((10, 2, 7))
    elif case == "zero_dim":
        X = coo((8, 0, 10))
    elif case == "negative_nnz":
        X = coo((8, 9, 10), nnz=-1)
    elif case == "null_idx":
        X = coo((8, 9, 10), idx=None)
    elif case == "null_tensor":
        X = None
    elif case == "too_many_pairs":
        cx, cy = [0, 1, 2, 0], [0, 1, 2, 1]
    elif case == "output_key_overflow_global_mode":
        # X free 60 bits + Y free 23 bits: only the grouped mode can take it
        X = coo((1 << 30, 1 << 30, 10))
        Y = coo((10, 1 << 20, 7))
        opt = B.default_options()
        opt.mode = B.MODE_GLOBAL
    elif case == "free_key_overflow":
        X = coo((1 << 30, 1 << 30, 1 << 30, 10))  # 90-bit X free key
        cx = [3]
    elif case == "bad_mode":
        opt = B.default_options()
        opt.mode = 7
    elif case == "bad_load_factor":
        opt = B.default_options()
        opt.load_factor = 1.5
    elif case == "bad_table_slots":
        opt = B.default_options()
        opt.out_table_slots = 100
    elif case == "bad_tile":
        opt = B.default_options()
        opt.tile = 512
    elif case == "bad_lds_max_keys":
        opt = B.default_options()
        opt.lds_max_keys = 6000
    elif case == "negative_capture_out_cap":
        opt = B.default_options()
        opt.capture_out_cap = -1
    elif case == "capture_without_allocator":
        opt = B.default_options()
        opt.capture_out_cap = 1000  # a plan without read-backs must not allocate from the stream's pool
    elif case == "bad_operand_order":
        opt = B.default_options()
        opt.operand_order = 2
    st, h = _plan(X, Y, cx, cy, opt)
    assert st == status, (st, B.last_error())
    assert h is None  # *plan is reset to NULL on failure
    assert B.last_error()


def test_execute_and_free_reject_null_plan():
    lib = B.load()
    assert lib.sptc_execute(None, None, None, 0, None, None) == B.ERR_INVALID_ARG
    lib.sptc_free(None)  # no-op
    info = B.Info()
    assert lib.sptc_plan_info(None, ctypes.byref(info)) == B.ERR_INVALID_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        B.load()


def _batch_plan(problems, opt=None, count=None):
    """problems: list of (X, Y, cx, cy) sptc_coo structs and mode lists."""
    lib = B.load()
    n = len(problems)
    xs = (B.Coo * max(n, 1))(*[p[0] for p in problems])
    ys = (B.Coo * max(n, 1))(*[p[1] for p in problems])
    nc = (ctypes.c_int32 * max(n, 1))(*[len(p[2]) for p in problems])
    arrs = [(B.int_array(p[2]), B.int_array(p[3])) for p in problems]
    cxp = (ctypes.c_void_p * max(n, 1))(*[ctypes.cast(a, ctypes.c_void_p).value for a, _ in arrs])
    cyp = (ctypes.c_void_p * max(n, 1))(*[ctypes.cast(b, ctypes.c_void_p).value for _, b in arrs])
    h = ctypes.c_void_p(12345)
    st = lib.sptc_batch_plan(ctypes.byref(h), n if count is None else count, xs, ys, nc, cxp, cyp,
                             ctypes.byref(opt) if opt is not None else None, None, None)
    return st, h.value


@pytest.mark.parametrize("case,status", [
    ("zero_count", B.ERR_INVALID_ARG),
    ("count_too_big", B.ERR_INVALID_ARG),
    ("global_mode", B.ERR_INVALID_ARG),
    ("bad_member", B.ERR_DIM_MISMATCH),
    ("member_key_overflow", B.ERR_KEY_OVERFLOW),
    ("batch_key_overflow", B.ERR_KEY_OVERFLOW),
])
def test_batch_plan_validation(case, status):
    good = (coo((8, 9, 10)), coo((10, 9, 7)), [2], [0])
    probs, opt, count = [good, good], None, None
    if case == "zero_count":
        count = 0
    elif case == "count_too_big":
        count = B.BATCH_MAX + 1
    elif case == "global_mode":
        opt = B.default_options()
        opt.mode = B.MODE_GLOBAL
    elif case == "bad_member":
        probs = [good, (coo((8, 9, 10)), coo((10, 9, 7)), [1], [0])]
    elif case == "member_key_overflow":
        probs = [good, (coo((1 << 30, 1 << 30, 1 << 30, 10)), coo((10, 9, 7)), [3], [0])]
    elif case == "batch_key_overflow":
        # a 62-bit X free key leaves no room for the contraction index
        probs = [good, (coo((1 << 31, 1 << 31, 10)), coo((10, 9, 7)), [2], [0])]
    st, h = _batch_plan(probs, opt, count)
    assert st == status, (st, B.last_error())
    assert h is None
    if case == "bad_member":
        assert B.last_error().startswith("contraction 1:")


def test_batch_functions_reject_null():
    lib = B.load()
    assert lib.sptc_batch_execute(None, None, None, None, None) == B.ERR_INVALID_ARG
    assert lib.sptc_batch_sizes(None, None, None, None) == B.ERR_INVALID_ARG
    assert lib.sptc_batch_info(None, 0, None, None, None) == B.ERR_INVALID_ARG
    lib.sptc_batch_free(None)
    assert lib.sptc_batch_plan(None, 1, None, None, None, None, None, None, None, None) == B.ERR_INVALID_ARG
