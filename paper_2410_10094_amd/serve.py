"""Serving loop: contractions arrive over time and are admitted, batched and
executed continuously under a device-memory budget.

One host thread runs the loop.  Arrived requests wait in a FIFO queue.  When
fewer than ``max_inflight`` batches are on the device, the loop takes the
queued requests of the head request's shape class (sched.shape_class), up to
``batch_products`` expected products, and plans them as one batch on the
plan stream: this is pass 1, which counts every member's products and so
fixes the output bytes its execution needs.  The batch is
admitted to the execute stream once its workspace plus those bytes fit in
what the budget has left; until then it waits, and the loop keeps retiring
finished batches.  Planning the next batch overlaps on the device with the
batches executing on the other stream, and requests that arrive meanwhile
join the next batch.  A request's latency runs from its arrival to the end
of its batch's execution on the device clock.

Before planning, the loop also checks that an estimate of the batch's own
workspace (from its nonzero counts) fits, so that a batch waiting for memory
does not hold more than the budget allows.  A backend may also decline to
plan a batch for lack of room (its plan returns None): the members go back
to the queue in arrival order and planning resumes after the next batch in
flight is released.

The device work goes through a backend (TorchBackend: the HIP library on a
GPU, all of its memory in one preallocated arena); the policy itself is
plain host code."""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Deque, List, Optional, Sequence

from . import sched


@dataclasses.dataclass
class Request:
    rid: int
    X: Any
    Y: Any
    cx: Sequence[int]
    cy: Sequence[int]
    arrival: float                    # seconds after the server starts
    expected_products: float = 0.0    # admission hint before pass 1
    klass: str = ""
    products: int = 0                 # pass 1 count
    done: float = -1.0                # device-clock completion, seconds after start
    result: Any = None                # (idx, val) device views, when kept

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class _Batch:
    members: List[Request]
    handle: Any
    need: int          # workspace + output bytes
    token: Any = None


class RingArena:
    """First-in first-out suballocator over one device buffer.  Batches
    execute on one stream, so they finish, and give their chunk back, in the
    order they took it."""

    ALIGN = 256

    def __init__(self, nbytes: int):
        self.size = int(nbytes)
        self.chunks: Deque = collections.deque()  # (start, end), oldest first

    def alloc(self, n: int) -> Optional[int]:
        """Start offset of a free chunk of n bytes, or None."""
        n = (int(n) + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        if not self.chunks:
            start = 0 if n <= self.size else None
        else:
            tail, head = self.chunks[0][0], self.chunks[-1][1]
            if head > tail:  # used: [tail, head)
                start = head if head + n <= self.size else (0 if n <= tail else None)
            else:            # wrapped; free: [head, tail)
                start = head if head + n <= tail else None
        if start is not None:
            self.chunks.append((start, start + n))
        return start

    def release(self, start: int):
        if not self.chunks or self.chunks[0][0] != start:
            raise RuntimeError("arena chunks must be released oldest first")
        self.chunks.popleft()

    def release_last(self, start: int):
        """Gives back the newest chunk (undoing an allocation that failed
        part-way)."""
        if not self.chunks or self.chunks[-1][0] != start:
            raise RuntimeError("only the newest arena chunk can be released last")
        self.chunks.pop()

    @staticmethod
    def rounded(n: int) -> int:
        return (int(n) + RingArena.ALIGN - 1) // RingArena.ALIGN * RingArena.ALIGN


class ArenaAllocator:
    """sptc_allocator over a RingArena for one batch: every buffer the
    library asks for while planning comes from the arena, in order.  The
    library's per-buffer releases are ignored (a buffer it frees early stays
    reserved); the owner gives all chunks back together, oldest first, when
    the batch is released, or newest first when planning failed."""

    def __init__(self, arena: RingArena, base_ptr: int):
        from . import binding as B
        self.arena = arena
        self.chunks: List[int] = []
        self.bytes = 0

        def alloc(nbytes, stream, ctx):
            start = arena.alloc(nbytes)
            if start is None:
                return None  # the library reports SPTC_ERR_OUT_OF_MEMORY
            self.chunks.append(start)
            self.bytes += RingArena.rounded(nbytes)
            return base_ptr + start

        def release(ptr, nbytes, stream, ctx):
            pass

        self._alloc = B.ALLOC_FN(alloc)
        self._release = B.RELEASE_FN(release)
        self.struct = B.Allocator(self._alloc, self._release, None)

    def take(self, nbytes: int) -> Optional[int]:
        """An extra chunk (the outputs) after the library's buffers."""
        start = self.arena.alloc(nbytes)
        if start is not None:
            self.chunks.append(start)
            self.bytes += RingArena.rounded(nbytes)
        return start

    def give_back(self):
        for start in self.chunks:
            self.arena.release(start)
        self.chunks = []

    def undo(self):
        for start in reversed(self.chunks):
            self.arena.release_last(start)
        self.chunks = []


class TorchBackend:
    """Runs batches with sptc_batch_* on one GPU: a plan stream and an
    execute stream (both at the default priority).  One preallocated ring
    arena holds every batch's memory: the library's workspace (through an
    ArenaAllocator) and then the outputs, both taken when the batch is
    planned, so that serving makes no device allocation at all and a batch
    that has been planned can always launch."""

    def __init__(self, arena_bytes: int, keep_results: bool = False, options=None):
        import torch
        self.torch = torch
        self.plan_stream = torch.cuda.Stream()
        self.exec_stream = torch.cuda.Stream()
        self.keep_results = keep_results
        self.options = options
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_host = 0.0
        self.arena = RingArena(arena_bytes)
        self.buf = torch.empty(max(int(arena_bytes), 1), dtype=torch.uint8, device="cuda")

    def start(self) -> float:
        """Marks time zero on both clocks; returns the host time of it."""
        torch = self.torch
        torch.cuda.synchronize()
        self.t0_event.record(self.exec_stream)
        self.t0_event.synchronize()
        self.t0_host = time.perf_counter()
        return self.t0_host

    def estimate(self, members: List[Request]) -> int:
        """Workspace bytes a batch of these members holds (before pass 1):
        about 96 bytes per nonzero of X and Y plus a fixed part."""
        return 96 * sum(r.X.nnz + r.Y.nnz for r in members) + (1 << 20)

    def plan(self, members: List[Request]):
        """(handle, bytes held) or None when the arena has no room for the
        batch until an earlier batch is released."""
        from . import Batch, SptcError
        from . import binding as B
        al = ArenaAllocator(self.arena, self.buf.data_ptr())
        try:
            b = Batch([(r.X, r.Y, r.cx, r.cy) for r in members], options=self.options, allocator=al,
                      stream=self.plan_stream)
        except SptcError as e:
            al.undo()  # the library synchronised its stream before reporting
            if e.status == B.ERR_OUT_OF_MEMORY:
                return None
            raise
        a = RingArena.ALIGN
        rnd = lambda n: (n + a - 1) // a * a
        parts = [rnd(4 * max(b.idx_elems, 1)), rnd(8 * max(b.val_elems, 1)), rnd(8 * b.count)]
        start = al.take(sum(parts))
        if start is None:
            b.close()
            al.undo()
            return None
        offs = [start]
        for n in parts[:-1]:
            offs.append(offs[-1] + n)
        torch = self.torch
        b.serve_out = (self.buf[offs[0]:offs[0] + 4 * max(b.idx_elems, 1)].view(torch.int32),
                       self.buf[offs[1]:offs[1] + 8 * max(b.val_elems, 1)].view(torch.float64),
                       self.buf[offs[2]:offs[2] + 8 * b.count].view(torch.int64))
        b.serve_alloc = al
        for r, it in zip(members, b.items):
            r.products = it["products"]
        return b, al.bytes

    def launch(self, b):
        """Enqueues the batch (its memory is already held)."""
        torch = self.torch
        idx, val, nnz = b.serve_out
        b.execute_into(idx, val, nnz, stream=self.exec_stream)
        # the counts travel to pinned host memory behind the batch, so that a
        # finished batch is checked without waiting on the execute stream
        # (which by then may hold the next batch)
        nnz_host = torch.empty(b.count, dtype=torch.int64, pin_memory=True)
        with torch.cuda.stream(self.exec_stream):
            nnz_host.copy_(nnz, non_blocking=True)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.exec_stream)
        return ((idx, val, nnz, nnz_host), ev)

    def done(self, token) -> bool:
        return token[1].query()

    def finish_time(self, token) -> float:
        return self.t0_event.elapsed_time(token[1]) * 1e-3

    def results(self, b, token, members: List[Request]):
        """Kept results are copied out of the arena, which is reused."""
        if not self.keep_results:
            return
        torch = self.torch
        idx, val, _, nnz_host = token[0]
        with torch.cuda.stream(self.exec_stream):
            for r, (i, v) in zip(members, b.views(idx, val, nnz_host.tolist())):
                r.result = (i.clone(), v.clone())
        # the next plan may reuse this part of the arena on the plan stream
        ev = torch.cuda.Event()
        ev.record(self.exec_stream)
        self.plan_stream.wait_event(ev)

    def check(self, b, token):
        """Raises if any member reported an error status (host copy, no wait)."""
        bad = sum(1 for n in token[0][3].tolist() if n < 0)
        if bad:
            raise RuntimeError(f"{bad} contractions of a batch reported an error")

    def release(self, b, token):
        b.close()
        b.serve_alloc.give_back()


class Server:
    def __init__(self, backend, budget_bytes: int = 64 << 30, max_inflight: int = 2,
                 batch_products: float = 5e8, max_batch: int = sched.BATCH_MAX,
                 clock: Callable[[], float] = time.perf_counter, idle_wait: float = 50e-6,
                 bytes_per_product: Optional[float] = 40.0):
        """bytes_per_product: rough device bytes a batch needs per product
        (its output COO entry, 4 B per output mode + 8 B value, plus
        workspace); batches are kept to budget / (max_inflight *
        bytes_per_product) expected products so that max_inflight of them fit
        at once.  None: no such cap."""
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.batch_products = batch_products
        if bytes_per_product:
            self.batch_products = min(batch_products, budget_bytes / (max_inflight * bytes_per_product))
        self.max_batch = max_batch
        self.clock = clock
        self.idle_wait = idle_wait
        self.used = 0
        self.peak_used = 0
        self.batches = 0
        self.waits_for_memory = 0
        self.deferred_requests = 0  # members of plans declined for lack of room, each time

    def _select(self, queue: Deque[Request]) -> List[int]:
        """Positions in the queue of the next batch: the head request's shape
        class, FIFO within it, up to the product and count caps (the head
        always goes)."""
        head = queue[0]
        picked, acc = [], 0.0
        for k, r in enumerate(queue):
            if len(picked) >= self.max_batch:
                break
            if r.klass != head.klass:
                continue
            if picked and acc + r.expected_products > self.batch_products:
                break
            picked.append(k)
            acc += r.expected_products
        return picked

    @staticmethod
    def _remove(queue: Deque[Request], picked: List[int]) -> List[Request]:
        if picked[-1] == len(picked) - 1:  # a prefix of the queue (always, with one shape class)
            return [queue.popleft() for _ in picked]
        chosen = set(picked)
        members = [r for k, r in enumerate(queue) if k in chosen]
        rest = [r for k, r in enumerate(queue) if k not in chosen]
        queue.clear()
        queue.extend(rest)
        return members

    def run(self, requests: Sequence[Request], progress: Optional[Callable[[str], None]] = None,
            progress_every: float = 10.0) -> List[Request]:
        """Serves requests (sorted by arrival) to completion; returns them.
        progress, if given, receives a status line every progress_every
        seconds."""
        be = self.backend
        next_report = progress_every
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: Deque[Request] = collections.deque()
        inflight: List[_Batch] = []
        staged: Optional[_Batch] = None
        plan_blocked = False
        done: List[Request] = []
        t0 = be.start()
        while pending or queue or inflight or staged:
            now = self.clock() - t0
            if progress and now >= next_report:
                progress(f"{now:.0f} s: {len(done)} served, {len(queue)} queued, {len(pending)} yet to arrive, "
                         f"{self.batches} batches")
                next_report += progress_every
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            for b in [b for b in inflight if be.done(b.token)]:
                be.check(b.handle, b.token)
                t = be.finish_time(b.token)
                for r in b.members:
                    r.done = t
                be.results(b.handle, b.token, b.members)
                be.release(b.handle, b.token)
                self.used -= b.need
                inflight.remove(b)
                done.extend(b.members)
                progressed = True
                plan_blocked = False
            if staged is None and queue and len(inflight) < self.max_inflight and not plan_blocked:
                picked = self._select(queue)
                if self.used + be.estimate([queue[k] for k in picked]) <= self.budget or not inflight:
                    members = self._remove(queue, picked)
                    planned = be.plan(members)
                    if planned is None:
                        # no room until a batch in flight is released
                        if not inflight:
                            raise RuntimeError(f"a batch of {len(members)} does not fit the device memory of "
                                               f"{self.budget} bytes even alone; lower batch_products")
                        queue.extend(members)
                        queue = collections.deque(sorted(queue, key=lambda r: (r.arrival, r.rid)))
                        plan_blocked = True
                        self.waits_for_memory += 1
                        self.deferred_requests += len(members)
                    else:
                        handle, need = planned
                        if need > self.budget:
                            raise RuntimeError(f"a batch of {len(members)} needs {need} bytes, above the budget "
                                               f"{self.budget}; lower batch_products")
                        staged = _Batch(members, handle, need)
                        progressed = True
                else:
                    self.waits_for_memory += 1
            if staged is not None and len(inflight) < self.max_inflight:
                token = be.launch(staged.handle) if self.used + staged.need <= self.budget else None
                if token is not None:
                    staged.token = token
                    self.used += staged.need
                    self.peak_used = max(self.peak_used, self.used)
                    self.batches += 1
                    inflight.append(staged)
                    staged = None
                    progressed = True
                elif not progressed:
                    self.waits_for_memory += 1
            if not progressed:
                if pending and not queue and not inflight and staged is None:
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                elif self.idle_wait > 0:
                    time.sleep(self.idle_wait)
        return done


def poisson_arrivals(rate: float, seconds: float, seed: int):
    """Arrival times of a Poisson process of ``rate`` per second over
    ``seconds``, seeded."""
    import numpy as np
    rng = np.random.default_rng(seed)
    n_max = int(rate * seconds * 1.5 + 100)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_max))
    while t[-1] < seconds:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, size=n_max))])
    return t[t < seconds]


def latency_summary(done: Sequence[Request]):
    import numpy as np
    lat = np.array([r.latency for r in done], dtype=np.float64)
    if lat.size == 0:
        return {"requests": 0}
    return {"requests": int(lat.size), "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "latency_ms_p99": float(np.percentile(lat, 99) * 1e3), "latency_ms_max": float(lat.max() * 1e3),
            "latency_ms_mean": float(lat.mean() * 1e3)}
