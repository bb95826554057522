"""Sparse-sparse tensor contraction on AMD Instinct MI355X (gfx950).

    import paper_2410_10094_amd as sptc
    X = sptc.DeviceCoo.from_host(x_host)         # COO on the GPU
    plan = sptc.plan(X, Y, cx=[2], cy=[0])        # group Y, probe X, count products
    idx, val = plan.execute()                     # expand, accumulate, compact

Z = X contracted with Y over the paired modes cx[t] <-> cy[t] (paper section
2.2, Eq. 2); the output coordinate is X's free coordinates then Y's, each in
ascending mode order; output order is unspecified.  All work runs in the HIP
library ``libsptc.so`` through its C ABI (``include/sptc.h``); this module only
marshals arguments, and fails if the library is not built.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import binding as _b
from .binding import SptcError

__all__ = ["DeviceCoo", "Plan", "plan", "contract", "Batch", "batch", "SptcError", "default_options", "pool_trim"]


def _torch():
    import torch
    return torch


def default_options(**overrides):
    o = _b.default_options()
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


class DeviceCoo:
    """A COO tensor in device memory: ``idx`` int32 ``[order, nnz]``
    (contiguous, mode-major), ``val`` float64 ``[nnz]``, ``dims`` tuple."""

    def __init__(self, dims: Sequence[int], idx, val):
        torch = _torch()
        self.dims = tuple(int(d) for d in dims)
        if idx.dtype != torch.int32 or val.dtype != torch.float64:
            raise TypeError("idx must be int32 and val float64")
        if not (idx.is_cuda and val.is_cuda):
            raise ValueError("idx and val must be device tensors")
        self.idx = idx.contiguous().reshape(len(self.dims), -1)
        self.val = val.contiguous().reshape(-1)
        if self.idx.shape[1] != self.val.shape[0]:
            raise ValueError("idx and val disagree on nnz")

    @classmethod
    def from_host(cls, coo, device="cuda"):
        """From any object with ``dims``, ``idx`` (numpy int32 [order, nnz])
        and ``val`` (numpy float64 [nnz])."""
        torch = _torch()
        idx = torch.from_numpy(coo.idx).to(device=device, dtype=torch.int32)
        val = torch.from_numpy(coo.val).to(device=device, dtype=torch.float64)
        return cls(coo.dims, idx.reshape(len(coo.dims), -1), val)

    @property
    def order(self):
        return len(self.dims)

    @property
    def nnz(self):
        return int(self.val.shape[0])

    def as_c(self):
        return _b.make_coo(self.order, self.dims, self.nnz,
                           self.idx.data_ptr() if self.nnz and self.order else None,
                           self.val.data_ptr() if self.nnz else None)


def _stream_handle(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class _TorchAllocator:
    """Routes the library's workspace through torch's caching allocator."""

    def __init__(self, device_index: int):
        torch = _torch()
        self._sizes = {}

        def alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device_index, stream)
            except Exception:  # out of memory: the library reports SPTC_ERR_OUT_OF_MEMORY
                return None

        def release(ptr, nbytes, stream, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc = _b.ALLOC_FN(alloc)
        self._release = _b.RELEASE_FN(release)
        self.struct = _b.Allocator(self._alloc, self._release, None)


def _resolve_allocator(allocator, device):
    """(keep-alive object, sptc_allocator pointer or None) for an allocator
    argument: "pool" (the device's stream-ordered pool), "torch" (torch's
    caching allocator) or any object whose ``struct`` is a binding.Allocator
    (kept alive as long as the plan or batch)."""
    if isinstance(allocator, str):
        if allocator == "pool":
            return None, None
        if allocator == "torch":
            a = _TorchAllocator(device.index if device.index is not None else _torch().cuda.current_device())
            return a, ctypes.byref(a.struct)
        raise ValueError("allocator must be 'pool', 'torch' or an object with an Allocator struct")
    if not isinstance(getattr(allocator, "struct", None), _b.Allocator):
        raise ValueError("allocator must be 'pool', 'torch' or an object with an Allocator struct")
    return allocator, ctypes.byref(allocator.struct)


def contract_noalloc(X: DeviceCoo, Y: DeviceCoo, cx: Sequence[int], cy: Sequence[int], out_idx, out_val,
                     out_cap: int, out_nnz, options=None, stream=None):
    """``sptc_contract_noalloc``: plan, execute and release one contraction
    with no device allocation (workspace from the library's static device
    array).  The caller's output tensors are written as by
    ``Plan.execute_into``; nnz lands in ``out_nnz`` (not synchronised)."""
    if len(cx) != len(cy):
        raise ValueError("cx and cy must have the same length")
    lib = _b.load()
    cX, kx = X.as_c()
    cY, ky = Y.as_c()
    acx, acy = _b.int_array(cx), _b.int_array(cy)
    opt = options if options is not None else _b.default_options()
    _b.check(lib.sptc_contract_noalloc(ctypes.byref(cX), ctypes.byref(cY), len(cx), acx, acy, ctypes.byref(opt),
                                       out_idx.data_ptr() if out_idx is not None and out_idx.numel() else None,
                                       out_val.data_ptr(), int(out_cap), out_nnz.data_ptr(), _stream_handle(stream)))


class Plan:
    """A contraction plan (``sptc_plan``): Y grouped, X probed, products
    counted and the output hash sized.  ``execute`` may run any number of
    times; X's and Y's device arrays are read only while the plan is built."""

    def __init__(self, X: DeviceCoo, Y: DeviceCoo, cx: Sequence[int], cy: Sequence[int], options=None,
                 allocator: str = "pool", stream=None):
        torch = _torch()
        lib = _b.load()
        if len(cx) != len(cy):
            raise ValueError("cx and cy must have the same length")
        self.X, self.Y = X, Y
        self.cx, self.cy = tuple(int(c) for c in cx), tuple(int(c) for c in cy)
        self._stream = _stream_handle(stream)
        cX, kx = X.as_c()
        cY, ky = Y.as_c()
        acx, acy = _b.int_array(self.cx), _b.int_array(self.cy)
        opt = options if options is not None else _b.default_options()
        self._allocator, alloc_ptr = _resolve_allocator(allocator, X.val.device)
        h = ctypes.c_void_p()
        self._h = None
        _b.check(lib.sptc_plan(ctypes.byref(h), ctypes.byref(cX), ctypes.byref(cY), len(self.cx), acx, acy,
                               ctypes.byref(opt), alloc_ptr, self._stream))
        self._h = h
        info = _b.Info()
        _b.check(lib.sptc_plan_info(self._h, ctypes.byref(info)))
        self.out_order = info.out_order
        self.out_dims = tuple(info.out_dims[m] for m in range(info.out_order))
        self.products = info.products
        self.out_nnz_bound = info.out_nnz_bound
        self.y_groups = info.y_groups
        self.y_table_slots = info.y_table_slots
        self.out_table_slots = info.out_table_slots
        self.workspace_bytes = info.workspace_bytes
        self.key_bits = (info.key_bits_contract, info.key_bits_x_free, info.key_bits_y_free)
        self.mode = info.mode
        self.x_groups = info.x_groups
        self.group_classes = dict(direct=info.direct_groups, wave=info.wave_groups, block=info.block_groups,
                                  global_=info.global_groups)
        self.direct_products = info.direct_products
        self.block_mfma = bool(info.block_mfma)
        self.block_mfma_work = info.block_mfma_work
        self.block_tiles_scanned = bool(info.block_tiles_scanned)
        self.operands_swapped = bool(info.operands_swapped)
        self.block_dense_rows = bool(info.block_dense_rows)

    def close(self):
        if getattr(self, "_h", None):
            _b.load().sptc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def allocate_outputs(self, out_cap: Optional[int] = None):
        torch = _torch()
        cap = self.out_nnz_bound if out_cap is None else int(out_cap)
        dev = self.X.val.device
        idx = torch.empty((self.out_order, max(cap, 1)), dtype=torch.int32, device=dev)
        val = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        nnz = torch.empty(1, dtype=torch.int64, device=dev)
        return idx, val, nnz, cap

    def execute_into(self, out_idx, out_val, out_cap: int, out_nnz, stream=None):
        """Enqueue ``sptc_execute`` (no synchronisation)."""
        _b.check(_b.load().sptc_execute(self._h, out_idx.data_ptr() if self.out_order else None,
                                        out_val.data_ptr(), int(out_cap), out_nnz.data_ptr(),
                                        _stream_handle(stream)))

    def execute(self, out_cap: Optional[int] = None, stream=None):
        """Run the contraction and return ``(idx [out_order, nnz] int32,
        val [nnz] float64)`` as device tensors (synchronises to read nnz)."""
        idx, val, nnz, cap = self.allocate_outputs(out_cap)
        self.execute_into(idx, val, cap, nnz, stream)
        n = int(nnz.item())
        if n < 0:
            raise SptcError(-n, "reported by the device during execute")
        return idx[:, :n], val[:n]

    def status(self, stream=None):
        _b.check(_b.load().sptc_plan_status(self._h, _stream_handle(stream)))

    # ---- inspection of intermediate structures ----
    def y_groups_table(self):
        """(key coordinates int32 [ncontract, g], counts int64 [g], starts
        int64 [g]) of Y's contracting-key groups, on the device."""
        torch = _torch()
        dev = self.X.val.device
        g = self.y_groups
        kc = torch.empty((len(self.cy), max(g, 1)), dtype=torch.int32, device=dev)
        counts = torch.empty(max(g, 1), dtype=torch.int64, device=dev)
        starts = torch.empty(max(g, 1), dtype=torch.int64, device=dev)
        ng = ctypes.c_int64()
        _b.check(_b.load().sptc_plan_y_groups(self._h, kc.data_ptr(), counts.data_ptr(), starts.data_ptr(),
                                              max(g, 1), ctypes.byref(ng), _stream_handle(None)))
        return kc[:, :g], counts[:g], starts[:g]

    def y_grouped(self):
        """(Y free coordinates int32 [nfree_Y, nnz_Y], values [nnz_Y]) in
        grouped order."""
        torch = _torch()
        dev = self.X.val.device
        nfy = self.Y.order - len(self.cy)
        coords = torch.empty((nfy, max(self.Y.nnz, 1)), dtype=torch.int32, device=dev)
        vals = torch.empty(max(self.Y.nnz, 1), dtype=torch.float64, device=dev)
        _b.check(_b.load().sptc_plan_y_grouped(self._h, coords.data_ptr() if nfy else None, vals.data_ptr(),
                                               _stream_handle(None)))
        return coords[:, : self.Y.nnz], vals[: self.Y.nnz]

    def x_groups_table(self):
        """Grouped mode: (X free coordinates int32 [nfree_X, g], entry counts
        int64 [g], product counts int64 [g]) of X's free-key groups."""
        torch = _torch()
        dev = self.X.val.device
        g = self.x_groups
        nfx = self.X.order - len(self.cx)
        coords = torch.empty((nfx, max(g, 1)), dtype=torch.int32, device=dev)
        counts = torch.empty(max(g, 1), dtype=torch.int64, device=dev)
        prods = torch.empty(max(g, 1), dtype=torch.int64, device=dev)
        ng = ctypes.c_int64()
        _b.check(_b.load().sptc_plan_x_groups(self._h, coords.data_ptr() if nfx else None, counts.data_ptr(),
                                              prods.data_ptr(), max(g, 1), ctypes.byref(ng), _stream_handle(None)))
        return coords[:, :g], counts[:g], prods[:g]

    def x_counts(self):
        torch = _torch()
        counts = torch.empty(max(self.X.nnz, 1), dtype=torch.int64, device=self.X.val.device)
        _b.check(_b.load().sptc_plan_x_counts(self._h, counts.data_ptr(), _stream_handle(None)))
        return counts[: self.X.nnz]


class Batch:
    """Many independent contractions planned and executed together
    (``sptc_batch_plan``): one pass of the grouped pipeline serves all of
    them, and each gets its own COO output."""

    def __init__(self, problems: Sequence[tuple], options=None, allocator: str = "pool", stream=None):
        """problems: sequence of ``(X, Y, cx, cy)`` with DeviceCoo X and Y."""
        torch = _torch()
        lib = _b.load()
        n = len(problems)
        if not 1 <= n <= _b.BATCH_MAX:
            raise ValueError(f"a batch holds 1..{_b.BATCH_MAX} contractions")
        self.count = n
        self._stream = _stream_handle(stream)
        self.device = problems[0][0].val.device
        xs = (_b.Coo * n)()
        ys = (_b.Coo * n)()
        nc = (ctypes.c_int32 * n)()
        cxp = (ctypes.c_void_p * n)()
        cyp = (ctypes.c_void_p * n)()
        keep = []
        for b, (X, Y, cx, cy) in enumerate(problems):
            if len(cx) != len(cy):
                raise ValueError("cx and cy must have the same length")
            xs[b], kx = X.as_c()
            ys[b], ky = Y.as_c()
            acx, acy = _b.int_array(cx), _b.int_array(cy)
            keep += [kx, ky, acx, acy]
            nc[b] = len(cx)
            cxp[b] = ctypes.cast(acx, ctypes.c_void_p)
            cyp[b] = ctypes.cast(acy, ctypes.c_void_p)
        opt = options if options is not None else _b.default_options()
        self._allocator, alloc_ptr = _resolve_allocator(allocator, self.device)
        h = ctypes.c_void_p()
        self._h = None
        _b.check(lib.sptc_batch_plan(ctypes.byref(h), n, xs, ys, nc, cxp, cyp, ctypes.byref(opt), alloc_ptr,
                                     self._stream))
        self._h = h
        ie, ve, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _b.check(lib.sptc_batch_sizes(self._h, ctypes.byref(ie), ctypes.byref(ve), ctypes.byref(ws)))
        self.idx_elems, self.val_elems, self.workspace_bytes = ie.value, ve.value, ws.value
        self.items = []
        for b in range(n):
            info = _b.Info()
            io, vo = ctypes.c_int64(), ctypes.c_int64()
            _b.check(lib.sptc_batch_info(self._h, b, ctypes.byref(info), ctypes.byref(io), ctypes.byref(vo)))
            self.items.append(dict(out_order=info.out_order,
                                   out_dims=tuple(info.out_dims[m] for m in range(info.out_order)),
                                   products=info.products, out_nnz_bound=info.out_nnz_bound,
                                   idx_offset=io.value, val_offset=vo.value))
        self.products = sum(it["products"] for it in self.items)

    def close(self):
        if getattr(self, "_h", None):
            _b.load().sptc_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def output_bytes(self):
        """Device bytes of the outputs: what pass 1's product counts say one
        execute needs beyond the batch itself."""
        return 4 * self.idx_elems + 8 * self.val_elems + 8 * self.count

    def allocate_outputs(self):
        """(idx, val, nnz) device tensors for execute_into."""
        torch = _torch()
        idx = torch.empty(max(self.idx_elems, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(self.val_elems, 1), dtype=torch.float64, device=self.device)
        nnz = torch.empty(self.count, dtype=torch.int64, device=self.device)
        return idx, val, nnz

    def execute_into(self, out_idx, out_val, out_nnz, stream=None):
        """Enqueue ``sptc_batch_execute`` (no synchronisation)."""
        _b.check(_b.load().sptc_batch_execute(self._h, out_idx.data_ptr(), out_val.data_ptr(), out_nnz.data_ptr(),
                                              _stream_handle(stream)))

    def views(self, out_idx, out_val, nnz_host):
        """Per-contraction ``(idx [out_order, nnz], val [nnz])`` views of the
        shared output buffers, given the nnz array on the host."""
        res = []
        for it, n in zip(self.items, nnz_host):
            n = int(n)
            if n < 0:
                raise SptcError(-n, "reported by the device during batch execute")
            cap, k = it["out_nnz_bound"], it["out_order"]
            idx = out_idx[it["idx_offset"]: it["idx_offset"] + k * cap].view(k, cap)[:, :n]
            val = out_val[it["val_offset"]: it["val_offset"] + n]
            res.append((idx, val))
        return res

    def execute(self, stream=None):
        """Run every contraction; returns a list of ``(idx, val)`` device
        tensors (synchronises to read the nnz)."""
        idx, val, nnz = self.allocate_outputs()
        self.execute_into(idx, val, nnz, stream)
        return self.views(idx, val, nnz.cpu().tolist())


def pool_trim(keep_bytes: int = 0):
    """Return workspace memory cached in the device's stream-ordered pool
    (above keep_bytes) to the device (sptc_pool_trim)."""
    _b.check(_b.load().sptc_pool_trim(int(keep_bytes)))


def batch(problems: Sequence[tuple], options=None, allocator: str = "pool", stream=None) -> Batch:
    return Batch(problems, options=options, allocator=allocator, stream=stream)


def plan(X: DeviceCoo, Y: DeviceCoo, cx: Sequence[int], cy: Sequence[int], options=None, allocator: str = "pool",
         stream=None) -> Plan:
    return Plan(X, Y, cx, cy, options=options, allocator=allocator, stream=stream)


def contract(X: DeviceCoo, Y: DeviceCoo, cx: Sequence[int], cy: Sequence[int], options=None, stream=None):
    """Plan and execute in one call; returns (idx, val) device tensors."""
    with Plan(X, Y, cx, cy, options=options, stream=stream) as p:
        return p.execute(stream=stream)
