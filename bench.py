#!/usr/bin/env python3
"""Throughput of the sparse tensor contraction hot path on one MI355X.

A step is one pass of the whole path over one synthetic input already resident
in HBM: plan (group Y by contracting key, probe X, count products, size the
output hash) then execute (expand and accumulate products, compact to COO).
Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--also a,b]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "products/s + output nnz/s vs HBM roofline; batched/served p50/p99 vs per-call"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix, published

DESCRIPTIONS = {
    "plain": "plain order-3 SpTC: 64^3 x 64^3, 2,621 nnz each (1%), X mode 2 with Y mode 0",
    "block-sparse": "block-sparse order-4 x order-4: 48^4, 8^4 blocks p=0.1, 50% fill, values N(0,1)exp(-|i-j|/8), "
                    "X modes (2,3) with Y modes (0,1)",
    "block-sparse-1.5M": "block-sparse order-4 x order-4: 48^4, 8^4 blocks p=0.565 (~1.5M nnz), 50% fill, "
                         "X modes (2,3) with Y modes (0,1)",
    "imbalanced": "imbalanced order-3 SpTC: X 1e7 nnz on 2^17x2^14x2^15 (contracting mode Zipf 1.2), "
                  "Y 1e6 nnz on 2^15x2^12x2^10, X mode 2 with Y mode 0",
    "paper-set-50-5x5-500K": "synthetic set 1 (Table 1): order-5 x order-5, all modes 50, 500K random nnz each, "
                             "modes (1,2) contracted",
}


def algorithmic_bytes(stage, p, products, nnz_z, x_groups=0, mode="grouped", info=None):
    """Bytes a stage must move through HBM at minimum (each datum once; on the
    global-hash path the output hash is read-modify-written once per
    product), per launch."""
    nx, ny = p.X.nnz, p.Y.nnz
    ox, oy = p.X.order, p.Y.order
    nz_order = ox + oy - 2 * len(p.cx)
    nc = len(p.cx)
    info = info or {}
    if stage == "direct":
        # per direct group: group record 16 B, its X record 16 B, list id 4 B and
        # offset 8 B; grouped-Y entries read once; one COO entry per product
        nd, pd = info.get("direct_groups", 0), info.get("direct_products", 0)
        return nd * (16 + 16 + 4 + 8) + 16 * ny + pd * (4 * nz_order + 8)
    if stage == "block":
        # grouped X records and grouped-Y entries read once, COO written once
        return 16 * nx + 16 * ny + nnz_z * (4 * nz_order + 8)
    if stage == "x_probe" and mode == "grouped":
        # X COO read once, grouped X records (16 B) written once
        return nx * (4 * ox + 8) + 16 * nx
    if stage == "expand":
        # per product: output-hash key read 8 B + value read 8 B + value write 8 B;
        # X records (poff 8 B, group start 4 B, packed free key + value 16 B) and
        # grouped Y entries (16 B) read once.
        return 24 * products + 28 * nx + 16 * ny
    if stage == "compact":
        # occupied slot read once (16 B), COO written once (4 B per mode + 8 B value)
        return nnz_z * (16 + 4 * nz_order + 8)
    if stage == "x_probe":
        return nx * (4 * ox + 8) + nx * (16 + 4 + 4)
    if stage == "y_count":
        return ny * 4 * nc
    if stage == "y_scatter":
        return ny * (4 * oy + 8) + 16 * ny
    if stage == "p_scan":
        return 4 * nx + 8 * (nx + 1)
    return 0


def survey_byte_model(p, products, nnz_z):
    """Whole-step algorithmic bytes of the method as a global-hash design
    prices them: COO inputs read once, grouped Y written and read once (32 B
    per Y entry), a pass-1 record per X entry (16 B), 24 B of output-hash
    traffic per product (key read, value read, value written) and the
    compaction (occupied slot read, COO written).  The global mode moves at
    least this much.  The grouped path keeps the per-product traffic in LDS,
    so its fraction of this model can exceed 1: the model then says how much
    HBM traffic the per-group tables saved, not how close a kernel is to the
    HBM peak."""
    nx, ny = p.X.nnz, p.Y.nnz
    nz_order = p.X.order + p.Y.order - 2 * len(p.cx)
    return (nx * (4 * p.X.order + 8) + ny * (4 * p.Y.order + 8) + 32 * ny + 16 * nx + 24 * products
            + nnz_z * (16 + 4 * nz_order + 8))


def survey_roofline(p, products, nnz_z, sec):
    b = survey_byte_model(p, products, nnz_z)
    return {"bytes_per_step": b, "achieved_GBps": round(b / sec / 1e9, 1),
            "frac_of_8TBps": round(b / sec / (HBM_PEAK_GBS * 1e9), 4)}


def _oracle_sample(p, max_seconds, threads):
    """The oracle on a prefix of X (against all of Y) sized so one run takes
    about max_seconds at most.  Returns (products, outputs, seconds, n, nx)."""
    import oracle
    from paper_2410_10094_amd.workloads import Coo
    nx = p.X.nnz
    probe_n = max(1, min(nx, 20_000 if threads > 1 else 4_000))
    Xs = Coo(p.X.dims, p.X.idx[:, :probe_n], p.X.val[:probe_n])
    _, pairs = oracle.match_counts(Xs, p.Y, p.cx, p.cy)
    t0 = time.perf_counter()
    oracle.contract(Xs, p.Y, p.cx, p.cy, nthreads=threads)
    per_x = max(time.perf_counter() - t0, 1e-6) / probe_n
    n = max(1, min(nx, int(max_seconds / per_x)))
    Xs = Coo(p.X.dims, p.X.idx[:, :n], p.X.val[:n])
    _, pairs = oracle.match_counts(Xs, p.Y, p.cx, p.cy)
    t0 = time.perf_counter()
    r = oracle.contract(Xs, p.Y, p.cx, p.cy, nthreads=threads)
    return pairs, r.nnz, time.perf_counter() - t0, n, nx


def time_oracle(p, max_seconds=12.0):
    """The CPU oracle as it stands, on bounded samples of the workload: on
    the host cores this process may use (at most 16, the host share of one
    GPU), and single-threaded.  Returns the cpu_baseline record."""
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    pairs, nnz, dt, n, nx = _oracle_sample(p, max_seconds, threads)
    pairs1, nnz1, dt1, n1, _ = _oracle_sample(p, max_seconds, 1)
    what = lambda k: "full workload" if k == nx else f"first {k} of {nx} X nonzeros against all of Y"
    return {"value": pairs / dt, "unit": "products/s", "cores": threads, "kind": "oracle",
            "sample": f"{what(n)}: {pairs} products, {nnz} outputs, {dt:.2f} s, std::map join, "
                      f"{threads} threads partitioned by leading output coordinate",
            "output_nnz_per_s": nnz / dt,
            "single_thread": {"value": pairs1 / dt1, "unit": "products/s", "cores": 1,
                              "sample": f"{what(n1)}: {pairs1} products, {nnz1} outputs, {dt1:.2f} s",
                              "output_nnz_per_s": nnz1 / dt1},
            "host_cpus_visible": len(os.sched_getaffinity(0))}


def run_workload(name, steps, warmup, with_events=True, mode="grouped", block_mfma=0):
    import torch

    import paper_2410_10094_amd as sptc
    from paper_2410_10094_amd import binding as B
    from paper_2410_10094_amd import workloads as W

    p = W.WORKLOADS[name]()
    X = sptc.DeviceCoo.from_host(p.X)
    Y = sptc.DeviceCoo.from_host(p.Y)
    stream = torch.cuda.current_stream()

    mode_id = {"grouped": B.MODE_GROUPED, "global": B.MODE_GLOBAL}[mode]
    # Output buffers are sized once (the bound is the same every step).
    with sptc.plan(X, Y, p.cx, p.cy, options=sptc.default_options(mode=mode_id, block_mfma=block_mfma)) as pl0:
        out_idx, out_val, out_nnz, cap = pl0.allocate_outputs()
        products = pl0.products
        out_slots = pl0.out_table_slots
        info = dict(mode=mode, y_groups=pl0.y_groups, y_table_slots=pl0.y_table_slots, out_table_slots=out_slots,
                    workspace_bytes=pl0.workspace_bytes, key_bits=pl0.key_bits, x_groups=pl0.x_groups,
                    group_classes=pl0.group_classes, direct_groups=pl0.group_classes["direct"],
                    direct_products=pl0.direct_products, block_mfma=pl0.block_mfma,
                    block_mfma_work=pl0.block_mfma_work, block_dense_rows=pl0.block_dense_rows,
                    block_tiles_scanned=pl0.block_tiles_scanned, operands_swapped=pl0.operands_swapped)

    nst = len(B.STAGES)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * nst)] for _ in range(steps)]
    for row in evs:
        for e in row:
            e.record(stream)  # torch creates the hipEvent_t lazily, at the first record
    ev_arrays = [(ctypes.c_void_p * (2 * nst))(*[e.cuda_event for e in row]) for row in evs]
    assert all(e.cuda_event for row in evs for e in row)

    def step(arrays=None):
        opt = sptc.default_options(mode=mode_id, block_mfma=block_mfma)
        if arrays is not None:
            opt.stage_events = ctypes.cast(arrays, ctypes.POINTER(ctypes.c_void_p))
        pl = sptc.plan(X, Y, p.cx, p.cy, options=opt)
        pl.execute_into(out_idx, out_val, cap, out_nnz)
        pl.close()

    for _ in range(warmup):
        step()
    stage_ms = {}
    dominant = None
    if with_events:
        # stage breakdown from a few untimed steps with every stage marked
        # (each marker is a packet of its own on the stream)
        nbreak = max(1, min(steps, 3))
        for k in range(nbreak):
            step(ev_arrays[k])
        torch.cuda.synchronize()
        for s, sname in enumerate(B.STAGES):
            stage_ms[sname] = sum(evs[k][2 * s].elapsed_time(evs[k][2 * s + 1]) for k in range(nbreak)) / nbreak
        dominant = max(range(nst), key=lambda s: stage_ms[B.STAGES[s]])
        # the timed steps mark the dominant stage only; its time per launch
        # is measured live over them
        ev_arrays = [(ctypes.c_void_p * (2 * nst))(*[e.cuda_event if j // 2 == dominant else None
                                                       for j, e in enumerate(row)]) for row in evs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(ev_arrays[k] if with_events else None)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nnz_z = int(out_nnz.item())
    if nnz_z < 0:
        raise RuntimeError(f"device reported status {-nnz_z}")
    sec = (t1 - t0) / steps
    if dominant is not None:
        stage_ms[B.STAGES[dominant]] = sum(evs[k][2 * dominant].elapsed_time(evs[k][2 * dominant + 1])
                                           for k in range(steps)) / steps
    return dict(problem=p, products=products, nnz_z=nnz_z, sec=sec, stage_ms=stage_ms, info=info, mode=mode, name=name)


def generate_draws(count, seed, workers):
    """Draws of the batched workload, generated in worker processes (before
    the GPU is touched)."""
    import multiprocessing as mp

    from paper_2410_10094_amd import workloads as W
    if workers <= 1 or count <= 4:
        return [W.batched_draw(seed, i) for i in range(count)]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.starmap(W.batched_draw, [(seed, i) for i in range(count)], chunksize=2)


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if xs else None


def klass(p):
    from paper_2410_10094_amd import sched
    return sched.shape_class(p.Y.dims, p.cy)


def sub_batches(draws, budget):
    """Batches of draws: bucketed by Y free key class, cut at `budget`
    expected products."""
    from paper_2410_10094_amd import sched
    return sched.make_batches(draws, sched.estimate_products, klass, budget)


def release_cached_memory():
    """Give memory cached by torch and by the library's pool back to the
    device between legs, so that each leg starts from the same state."""
    import torch

    import paper_2410_10094_amd as sptc
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    sptc.pool_trim(0)


def upload(draws):
    import torch

    import paper_2410_10094_amd as sptc
    dev = [(sptc.DeviceCoo.from_host(p.X), sptc.DeviceCoo.from_host(p.Y)) for p in draws]
    torch.cuda.synchronize()
    return dev


def run_served(draws, dev, seconds, rate, budget_bytes, batch_products, max_batch, seed, load_factor=1 / 1.3,
               label="served"):
    """Poisson arrivals at `rate` per second for `seconds`; each request is a
    draw picked uniformly from the pool (inputs resident in HBM).  Served
    with continuous batching under the memory budget (max_batch 1: one
    request per launch).  Every request is served to completion; the wall
    time therefore exceeds the arrival window when the server falls
    behind."""
    import numpy as np

    from paper_2410_10094_amd import sched, serve
    arrivals = serve.poisson_arrivals(rate, seconds, seed)
    picks = np.random.default_rng(seed + 1).integers(0, len(draws), size=len(arrivals))
    reqs = [serve.Request(i, dev[k][0], dev[k][1], draws[k].cx, draws[k].cy, float(a),
                          expected_products=sched.estimate_products(draws[k]),
                          klass=sched.shape_class(draws[k].Y.dims, draws[k].cy))
            for i, (a, k) in enumerate(zip(arrivals, picks))]
    import paper_2410_10094_amd as sptc
    backend = serve.TorchBackend(arena_bytes=budget_bytes, options=sptc.default_options(load_factor=load_factor))
    srv = serve.Server(backend, budget_bytes=budget_bytes, batch_products=batch_products, max_batch=max_batch)
    progress(f"{label}: {len(reqs)} requests over {seconds:.0f} s")
    t0 = time.perf_counter()
    done = srv.run(reqs, progress=lambda m: progress(f"{label}: {m}"))
    wall = time.perf_counter() - t0
    out = serve.latency_summary(done)
    products = sum(r.products for r in done)
    in_window = [r for r in done if r.done <= seconds]
    out.update({"offered_requests_per_s": rate, "arrival_seconds": seconds, "wall_seconds": round(wall, 3),
                "requests_per_s": len(done) / wall, "products": products, "products_per_s": products / wall,
                "served_within_arrival_window": len(in_window),
                "batches": srv.batches, "mean_batch": round(len(done) / max(srv.batches, 1), 2),
                "peak_bytes": srv.peak_used, "budget_bytes": budget_bytes, "waits_for_memory": srv.waits_for_memory,
                "deferred_requests": srv.deferred_requests, "admitted_requests": len(done),
                "batch_products": batch_products, "max_batch": max_batch})
    for k in ("latency_ms_p50", "latency_ms_p99", "latency_ms_max", "latency_ms_mean"):
        if k in out:
            out[k] = round(out[k], 3)
    progress(f"{label}: {len(done)} requests in {wall:.1f} s, p50 {out.get('latency_ms_p50')} ms, "
             f"p99 {out.get('latency_ms_p99')} ms")
    return out


def autotune_batched(draws, dev, sample):
    """Load factor and batch budget for the batched legs, tuned on the first
    `sample` draws (outside every timed region)."""
    from paper_2410_10094_amd import autotune
    sub = draws[:sample]
    tuner = autotune.Autotuner()
    run = autotune.torch_batch_runner(sub, dev[:sample], klass)
    run(1 / 1.3, 1e9, 0)  # warm the pools before timing candidates
    return tuner.tune(autotune.signature(sub, klass), run)


def run_batched(draws, dev, steps, warmup, budget, load_factor=1 / 1.3, tile=0):
    """The batched workload two ways, each step covering every draw:
    per-call (sptc_plan + sptc_execute per contraction) and batched
    (sptc_batch_plan + sptc_batch_execute per sub-batch of at most `budget`
    expected products).  Latency of a contraction: per-call, its own plan +
    execute; batched, its sub-batch's plan + execute (all members complete
    together)."""
    import torch

    import paper_2410_10094_amd as sptc
    groups = sub_batches(draws, budget)

    # per-call: one output buffer sized for the largest bound
    bounds, orders, products = [], [], []
    opts = lambda: sptc.default_options(load_factor=load_factor, tile=tile)
    for (X, Y), p in zip(dev, draws):
        with sptc.plan(X, Y, p.cx, p.cy, options=opts()) as pl:
            bounds.append(pl.out_nnz_bound)
            orders.append(pl.out_order)
            products.append(pl.products)
    total_products = sum(products)
    cap = max(bounds)
    oidx = torch.empty((max(orders) * max(cap, 1),), dtype=torch.int32, device="cuda")
    oval = torch.empty(max(cap, 1), dtype=torch.float64, device="cuda")
    onnz = torch.empty(len(draws), dtype=torch.int64, device="cuda")

    def per_call(lat):
        for i, ((X, Y), p) in enumerate(zip(dev, draws)):
            t0 = time.perf_counter()
            pl = sptc.plan(X, Y, p.cx, p.cy, options=opts())
            k = pl.out_order
            pl.execute_into(oidx[: max(k, 1) * max(cap, 1)].view(max(k, 1), max(cap, 1)), oval, cap, onnz[i:i + 1])
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            pl.close()

    # batched: buffers sized for the largest sub-batch
    need_i = need_v = 0
    for g in groups:
        with sptc.batch([(dev[i][0], dev[i][1], draws[i].cx, draws[i].cy) for i in g], options=opts()) as bt:
            need_i, need_v = max(need_i, bt.idx_elems), max(need_v, bt.val_elems)
    bidx = torch.empty(max(need_i, 1), dtype=torch.int32, device="cuda")
    bval = torch.empty(max(need_v, 1), dtype=torch.float64, device="cuda")
    bnnz = torch.empty(len(draws), dtype=torch.int64, device="cuda")
    # batch k's members' nnz land at bnnz[first[k] : first[k] + len(groups[k])]
    first = [0]
    for g in groups:
        first.append(first[-1] + len(g))

    from paper_2410_10094_amd import binding as B
    nst = len(B.STAGES)
    stream = torch.cuda.current_stream()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * nst)] for _ in groups]
    for row in evs:
        for e in row:
            e.record(stream)
    ev_arrays = [(ctypes.c_void_p * (2 * nst))(*[e.cuda_event for e in row]) for row in evs]
    stage_ms = {s: 0.0 for s in B.STAGES}

    def batched(lat, timed=False):
        for k, g in enumerate(groups):
            opt = opts()
            if timed:
                opt.stage_events = ctypes.cast(ev_arrays[k], ctypes.POINTER(ctypes.c_void_p))
            t0 = time.perf_counter()
            bt = sptc.batch([(dev[i][0], dev[i][1], draws[i].cx, draws[i].cy) for i in g], options=opt)
            bt.execute_into(bidx, bval, bnnz[first[k]:first[k] + len(g)])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            lat.extend([dt] * len(g))
            bt.close()
            if timed:
                for j, sname in enumerate(B.STAGES):
                    stage_ms[sname] += evs[k][2 * j].elapsed_time(evs[k][2 * j + 1])

    res = {}
    for name, fn, nnz in (("per_call", per_call, onnz), ("batched", batched, bnnz)):
        for _ in range(warmup):
            fn([])
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(lat) if fn is per_call else fn(lat, timed=True)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        bad = int((nnz < 0).sum().item())
        if bad:
            raise RuntimeError(f"{name}: {bad} contractions reported an error")
        res[name] = {"sec_per_step": round(sec, 5), "products_per_s": total_products / sec,
                     "latency_ms_p50": round(percentile(lat, 50) * 1e3, 4),
                     "latency_ms_p99": round(percentile(lat, 99) * 1e3, 4)}
    res["batched"]["stage_ms_per_step"] = {k: round(v / steps, 3) for k, v in stage_ms.items() if v > 0.01 * steps}
    res["load_factor"] = load_factor
    res["batched"]["sub_batches"] = len(groups)
    res["batched"]["sub_batch_sizes"] = [len(g) for g in groups]
    res["batched"]["sub_batch_budget_expected_products"] = budget
    res["speedup_batched_vs_per_call"] = round(res["per_call"]["sec_per_step"] / res["batched"]["sec_per_step"], 3)
    res["contractions"] = len(draws)
    res["products"] = total_products
    res["nnz_x_total"] = sum(p.X.nnz for p in draws)
    res["nnz_y_total"] = sum(p.Y.nnz for p in draws)
    # nnz(Z) of every draw, from the per-call leg, and the same total from the batched leg
    per_nnz = onnz.cpu().tolist()
    bat = bnnz.cpu().tolist()
    batched_nnz = [0] * len(draws)
    for k, g in enumerate(groups):
        for j, i in enumerate(g):
            batched_nnz[i] = bat[first[k] + j]
    if batched_nnz != per_nnz:
        raise RuntimeError("batched and per-call legs disagree on nnz(Z)")
    res["nnz_z_total"] = sum(per_nnz)
    b_alg = sum(survey_byte_model(p, P, n) for p, P, n in zip(draws, products, per_nnz))
    res["survey_roofline"] = {"bytes_per_pass": b_alg}
    for name in ("per_call", "batched"):
        sec = res[name]["sec_per_step"]
        res[name]["output_nnz_per_s"] = res["nnz_z_total"] / sec
        res[name]["survey_frac_of_8TBps"] = round(b_alg / sec / (HBM_PEAK_GBS * 1e9), 4)
    res["steps"] = steps
    return res


# HBM traffic of a dominant kernel, from two committed rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE), keyed by (workload, kernel).  A figure only
# holds while the kernel's sources are the ones profiled.
TRAFFIC_PROFILES = {
    ("block-sparse-1.5M", "k_lds_queue"): "lds_queue_block-sparse-1.5M_counters.md",
    ("block-sparse-1.5M", "k_group_block_mfma"): "block_mfma_block-sparse-1.5M_counters.md",
    ("imbalanced", "k_group_direct"): "direct_imbalanced_counters.md",
    ("block-sparse-1.5M", "k_expand_acc"): "expand_global_block-sparse-1.5M_counters.md",
    ("imbalanced", "k_expand_acc"): "expand_global_imbalanced_counters.md",
    ("paper-set-50-5x5-500K", "k_group_block"): "group_block_paper-set-50-5x5-500K_counters.md",
}
_CSRC = "paper_2410_10094_amd/csrc/"
_COMMON = (_CSRC + "prim.hpp", _CSRC + "sptc_internal.hpp")
# the sources each kernel is compiled from
KERNEL_SOURCES = {
    "k_lds_queue": (_CSRC + "queue.hip", _CSRC + "lds_items.hpp") + _COMMON,
    "k_group_block": (_CSRC + "grouped.hip", _CSRC + "lds_items.hpp") + _COMMON,
    "k_group_direct": (_CSRC + "grouped.hip", _CSRC + "lds_items.hpp") + _COMMON,
    "k_expand_acc": (_CSRC + "kernels.hip",) + _COMMON,
    "k_group_block_mfma": (_CSRC + "block_mfma.hip",) + _COMMON,
}


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """Bytes per launch from the committed counter summary, or None when
    there is none or the kernel changed since it was taken."""
    name = TRAFFIC_PROFILES.get((workload, kernel))
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if kernel not in KERNEL_SOURCES or fields.get("source_sha256") != kernel_source_hash(kernel):
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_problem(p, steps, warmup):
    """Seconds per plan + execute of one problem (inputs resident)."""
    import torch

    import paper_2410_10094_amd as sptc
    X, Y = sptc.DeviceCoo.from_host(p.X), sptc.DeviceCoo.from_host(p.Y)
    with sptc.plan(X, Y, p.cx, p.cy) as pl0:
        idx, val, nnz, cap = pl0.allocate_outputs()
        products = pl0.products

    def step():
        with sptc.plan(X, Y, p.cx, p.cy) as pl:
            pl.execute_into(idx, val, cap, nnz)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    n = int(nnz.item())
    if n < 0:
        raise RuntimeError(f"{p.name}: device reported status {-n}")
    return sec, products, n


def run_sweep(steps):
    """The shapes of the paper's synthetic sets (Table 1, sets 1 and 2): all
    modes of length 50 or 100, order-5 (A) and order-4 (B) tensors of
    50K-500K random entries, contracted on modes 1 and 2; A x A, A x B, B x B,
    and B x A (operand swap, section 5.4)."""
    from paper_2410_10094_amd import workloads as W
    rows = []
    for set_no, mode_len in ((1, 50), (2, 100)):
        for nnz in (50_000, 100_000, 200_000, 300_000, 500_000):
            for ox, oy in ((5, 5), (5, 4), (4, 4)):
                p = W.paper_set(W.BASE_SEED + 10 * set_no + ox + oy, mode_len, nnz, ox, oy)
                sec, P, n = time_problem(p, steps, 1)
                row = {"set": set_no, "nnz": nnz, "orders": f"{ox}x{oy}", "products": P, "out_nnz": n,
                       "ms": round(sec * 1e3, 4)}
                if ox != oy:  # operand swap: Y x X on the same data
                    from paper_2410_10094_amd.workloads import Problem
                    q = Problem(p.name + "-swap", p.Y, p.X, p.cy, p.cx)
                    sec2, P2, n2 = time_problem(q, steps, 1)
                    assert P2 == P and n2 == n
                    row["swap_ms"] = round(sec2 * 1e3, 4)
                rows.append(row)
    return rows


def kernel_of(stage, info):
    """The kernel that does a stage's work (for the dominant stage)."""
    if stage == "block":
        if info.get("block_mfma"):
            return "k_group_block_mfma"
        if info.get("block_dense_rows"):
            return "k_group_block"
        return "k_lds_queue" if info["key_bits"][2] <= 13 else "k_group_block"
    return {"direct": "k_group_direct", "expand": "k_expand_acc", "compact": "occupancy scan", "x_probe": "X grouping",
            "x_sort": "block entry sort"}.get(stage, stage)


def roofline_of(r):
    """Roofline of the dominant stage's kernel: its algorithmic bytes per
    launch (bench.algorithmic_bytes: each datum it must move through HBM,
    once; on the global path that includes 24 B of output-hash traffic per
    product) over its event-measured time per launch, against 8 TB/s."""
    p = r["problem"]
    stage = max(r["stage_ms"], key=lambda s: r["stage_ms"][s])
    ms = r["stage_ms"][stage]
    bytes_alg = algorithmic_bytes(stage, p, r["products"], r["nnz_z"], r["info"]["x_groups"], r["mode"], r["info"])
    achieved = bytes_alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    kernel = kernel_of(stage, r["info"])
    out = {"kernel": kernel, "stage": stage, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(r["name"], kernel),
           "ms_per_launch": round(ms, 4), "algorithmic_bytes_per_launch": bytes_alg,
           "byte_model": "per-kernel" if stage != "expand" else "survey (24 B per product in the output hash)",
           "products_per_s_in_kernel": round(r["products"] / (ms * 1e-3)) if ms > 0 else None}
    work = r["info"].get("block_mfma_work", 0)
    if stage == "block" and r["info"].get("block_mfma") and work and ms > 0:
        # the block class ran as a dense FP64 product: the method's useful
        # flops (one multiply and one add per product) against the matrix
        # cores' FP64 peak; the padded dense work it spent them in is context
        useful = 2.0 * r["products"] / (ms * 1e-3) / 1e12
        dense = 2.0 * work / (ms * 1e-3) / 1e12
        out["matrix_cores"] = {"kernel": "k_group_block_mfma", "useful_flops_per_launch": 2 * r["products"],
                               "achieved_tflops": round(useful, 2), "peak_tflops": FP64_MFMA_PEAK_TFLOPS,
                               "frac": round(useful / FP64_MFMA_PEAK_TFLOPS, 4),
                               "padded_flops_per_launch": 2 * work, "padded_tflops": round(dense, 2),
                               "padding_ratio": round(work / max(r["products"], 1), 2)}
    return out


def summary(name, r, variant=None):
    out = {"workload": name, "mode": r["mode"], "products": r["products"], "out_nnz": r["nnz_z"],
           "ms_per_step": round(r["sec"] * 1e3, 4), "products_per_s": r["products"] / r["sec"],
           "output_nnz_per_s": r["nnz_z"] / r["sec"],
           "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items() if not k.startswith("batch_")},
           "roofline": roofline_of(r),
           "survey_roofline": survey_roofline(r["problem"], r["products"], r["nnz_z"], r["sec"])}
    if variant:
        out["variant"] = variant
    return out


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def compact_batched(res):
    if not res:
        return res
    keep = ("contractions", "products", "nnz_z_total", "load_factor", "speedup_batched_vs_per_call", "steps",
            "survey_roofline")
    out = {k: res[k] for k in keep if k in res}
    for name in ("per_call", "batched"):
        out[name] = {k: v for k, v in res[name].items() if k != "stage_ms_per_step"}
    out["batched"]["top_stages_ms"] = dict(sorted(res["batched"].get("stage_ms_per_step", {}).items(),
                                                  key=lambda kv: -kv[1])[:5])
    if res.get("autotune"):
        out["autotune"] = {k: res["autotune"][k] for k in ("load_factor", "batch_products", "tile", "tuning_seconds")
                           if k in res["autotune"]}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="block-sparse-1.5M", choices=sorted(DESCRIPTIONS))
    ap.add_argument("--also", default="block-sparse,imbalanced,plain",
                    help="comma-separated extra workloads reported under 'also' ('' for none)")
    ap.add_argument("--global-legs", default="block-sparse-1.5M,imbalanced",
                    help="workloads also timed in the global mode (every product in the device output hash)")
    ap.add_argument("--mfma-leg", type=int, default=1,
                    help="1: also time the headline workload with the opt-in matrix-core block class")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (known bytes for scaling HBM counters) and exit")
    ap.add_argument("--mode", default="grouped", choices=["grouped", "global"],
                    help="accumulation strategy: per-X-group LDS tables (default) or one global hash")
    ap.add_argument("--block-mfma", type=int, default=0, choices=[-1, 0, 1],
                    help="dense block class on the FP64 matrix cores: 0 never (default), 1 when eligible, "
                         "-1 the plan's cost rule")
    ap.add_argument("--batched", type=int, default=512, metavar="COUNT",
                    help="draws of the batched workload timed per-call and batched (0: skip)")
    ap.add_argument("--batch-budget", type=float, default=1.0e9,
                    help="expected products per sub-batch of the batched leg (without --autotune)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: tune load factor and batch budget on the first 128 draws before the batched legs")
    ap.add_argument("--sweep", type=int, default=1, help="1: time the paper's synthetic-set shapes (Table 1, sets 1-2)")
    ap.add_argument("--serve", type=float, default=60.0, metavar="SECONDS",
                    help="seconds of Poisson arrivals for the served legs (0: skip); the pool is the batched draws")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="arrivals per second of the served leg")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0, help="device-memory budget of the served leg")
    ap.add_argument("--serve-batch-products", type=float, default=1e9,
                    help="expected products per served batch")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the contraction would shard X by free key; see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        sys.exit("--steps must be >= 1")

    from paper_2410_10094_amd.workloads import BASE_SEED
    draws = None
    if args.batched and not args.calibrate_copy:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
        draws = generate_draws(args.batched, BASE_SEED + 4, workers)

    import torch
    torch.cuda.set_device(0)

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.randn(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 8, "calibrate_copy_bytes_written": n * 8, "launches": 3}))
        return

    progress(f"headline: {args.workload}, {args.mode} mode, block_mfma={args.block_mfma}")
    r = run_workload(args.workload, args.steps, args.warmup, mode=args.mode, block_mfma=args.block_mfma)
    p = r["problem"]
    progress(f"headline: {r['sec'] * 1e3:.3f} ms per step")
    also = []
    for name in [a for a in args.also.split(",") if a and a != args.workload]:
        also.append(summary(name, run_workload(name, max(3, args.steps // 2), max(1, args.warmup), mode=args.mode,
                                               block_mfma=args.block_mfma)))
    if args.mfma_leg and args.mode == "grouped" and args.block_mfma != 1:
        also.append(summary(args.workload, run_workload(args.workload, max(3, args.steps // 2), max(1, args.warmup),
                                                        block_mfma=1),
                            variant="opt-in matrix-core block class (dense FP64 product of padded panels)"))
    glob = []
    for name in [a for a in args.global_legs.split(",") if a]:
        progress(f"global mode: {name}")
        glob.append(summary(name, run_workload(name, 3, 1, mode="global")))
    progress("single-workload legs done")

    batched = served = None
    if draws:
        dev = upload(draws)
        tuned = autotune_batched(draws, dev, min(len(draws), 128)) if args.autotune else None
        budget = tuned["batch_products"] if tuned else args.batch_budget
        lf = tuned["load_factor"] if tuned else 1 / 1.3
        tile = tuned["tile"] if tuned else 0
        progress("batched workload: per-call and batched legs")
        batched = run_batched(draws, dev, max(1, args.steps // 5), 1, budget, lf, tile)
        batched["autotune"] = tuned
        release_cached_memory()
        batched["workload"] = (f"{len(draws)} draws: orders 3-5, dims U[32,4096], nnz log-U[1e3,1e6], "
                               "1-2 contracted pairs, FP64 U[-1,1)")
        if args.serve > 0:
            budget = int(args.serve_budget_gb * (1 << 30))
            served = {"workload": f"Poisson arrivals at {args.serve_rate:.0f}/s for {args.serve:.0f} s, each request "
                                  f"one of the {len(draws)} batched draws picked uniformly, inputs resident in HBM; "
                                  "both legs serve the same arrival trace to completion"}
            served["batched"] = run_served(draws, dev, args.serve, args.serve_rate, budget,
                                           args.serve_batch_products, 4096, BASE_SEED + 5, lf, label="served batched")
            release_cached_memory()
            served["per_call"] = run_served(draws, dev, args.serve, args.serve_rate, budget,
                                            args.serve_batch_products, 1, BASE_SEED + 5, lf,
                                            label="served per call")

    sweep = None
    if args.sweep:
        progress("paper-set sweep")
        sweep = run_sweep(2)

    cpu = None
    if not args.no_cpu_baseline:
        progress("cpu baseline: the oracle on the host")
        cpu = time_oracle(p)

    # The driver keeps the tail of this line: the extras that matter most come last.
    line = {
        "metric": METRIC,
        "value": r["products"] / r["sec"],
        "unit": "products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[args.workload], "nnz_x": p.X.nnz, "nnz_y": p.Y.nnz,
                   "products": r["products"], "out_nnz": r["nnz_z"], "step": "plan + execute",
                   "mode": args.mode, "block_mfma": args.block_mfma, "parallelism": "single GPU"},
        "paper_set_sweep": sweep,
        "also": also,
        "batched": compact_batched(batched),
        "served": served,
        "global_mode": glob,
        "plan": {k: v for k, v in r["info"].items() if k not in ("mode",)},
        "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items() if v >= 0.01 and not k.startswith("batch_")},
        "output_nnz_per_s": r["nnz_z"] / r["sec"],
        "cpu_baseline": cpu,
        "survey_roofline": survey_roofline(p, r["products"], r["nnz_z"], r["sec"]),
        "roofline": roofline_of(r),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
