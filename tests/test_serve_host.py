"""Host-side policy of the serving loop, on the CPU: a fake backend stands in
for the device (one execution queue, durations from the product counts), so
the admission, batching and memory accounting are checked without a GPU."""
import time

import numpy as np
import pytest

from paper_2410_10094_amd import serve


class _T:
    def __init__(self, nnz):
        self.nnz = nnz


class FakeBackend:
    """Batches run one after another; a batch of P products takes
    P * sec_per_product + overhead seconds.  Each request carries
    `need_bytes` (output bytes after pass 1)."""

    def __init__(self, sec_per_product=1e-9, overhead=2e-4):
        self.spp = sec_per_product
        self.overhead = overhead
        self.free_at = 0.0
        self.t0 = 0.0
        self.planned = []
        self.launched = []
        self.unfinished_at_launch = []

    def start(self):
        self.t0 = time.perf_counter()
        return self.t0

    def estimate(self, members):
        return sum(r.X.nnz + r.Y.nnz for r in members)

    def plan(self, members):
        for r in members:
            r.products = int(r.expected_products)
        self.planned.append([r.rid for r in members])
        return list(members), self.estimate(members) + sum(r.need_bytes for r in members)

    def launch(self, handle):
        now = time.perf_counter() - self.t0
        self.unfinished_at_launch.append(sum(1 for (_, e, _) in self.launched if e > now))
        start = max(now, self.free_at)
        end = start + self.overhead + self.spp * sum(r.products for r in handle)
        self.free_at = end
        self.launched.append((start, end, [r.rid for r in handle]))
        return end

    def done(self, token):
        return time.perf_counter() - self.t0 >= token

    def finish_time(self, token):
        return token

    def results(self, b, token, members):
        for r in members:
            r.result = ("ok", r.rid)

    def check(self, b, token):
        pass

    def release(self, b, token):
        pass


def _requests(n, rate, seed, classes=("dense", "hash")):
    rng = np.random.default_rng(seed)
    t = serve.poisson_arrivals(rate, n / rate * 2, seed)[:n]
    out = []
    for i, a in enumerate(t):
        r = serve.Request(i, _T(int(rng.integers(10, 1000))), _T(int(rng.integers(10, 1000))), (0,), (0,), float(a),
                          expected_products=float(rng.integers(1e4, 1e6)), klass=str(rng.choice(classes)))
        r.need_bytes = int(rng.integers(1000, 100_000))
        out.append(r)
    return out


def test_every_request_completes_after_it_arrives():
    reqs = _requests(300, 20_000, 1)
    be = FakeBackend()
    srv = serve.Server(be, budget_bytes=10 << 20, batch_products=3e6)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(300))
    for r in done:
        assert r.done >= r.arrival
        assert r.result == ("ok", r.rid)
    assert srv.used == 0
    assert srv.peak_used <= srv.budget


def test_batches_hold_one_shape_class_in_arrival_order():
    reqs = _requests(400, 50_000, 2)
    by_id = {r.rid: r for r in reqs}
    be = FakeBackend()
    srv = serve.Server(be, budget_bytes=1 << 30, batch_products=5e6, max_batch=64)
    srv.run(reqs)
    for ids in be.planned:
        assert len({by_id[i].klass for i in ids}) == 1
        assert ids == sorted(ids)  # FIFO within the class
        assert len(ids) <= 64
        assert len(ids) == 1 or sum(by_id[i].expected_products for i in ids) <= 5e6
    # continuous batching: later batches take requests that arrived while others ran
    assert max(len(ids) for ids in be.planned) > 1


def test_memory_budget_holds_back_batches():
    reqs = _requests(120, 100_000, 3)
    be = FakeBackend(sec_per_product=2e-9)
    budget = 400_000
    srv = serve.Server(be, budget_bytes=budget, batch_products=2e6, max_inflight=3, bytes_per_product=None)
    done = srv.run(reqs)
    assert len(done) == 120
    assert srv.peak_used <= budget
    assert srv.waits_for_memory > 0


def test_in_flight_batches_never_exceed_the_limit():
    reqs = _requests(200, 100_000, 4)
    be = FakeBackend()
    srv = serve.Server(be, budget_bytes=1 << 30, batch_products=1e6, max_inflight=2)
    srv.run(reqs)
    # a launch happens only while fewer than max_inflight batches are unfinished
    assert max(be.unfinished_at_launch) <= 1
    assert len(be.launched) == srv.batches


class DecliningBackend(FakeBackend):
    """Holds each batch's bytes from plan to release in a ring arena of
    `capacity` bytes, as the GPU backend does; plan returns None when the
    arena has no room."""

    def __init__(self, capacity, **kw):
        super().__init__(**kw)
        self.arena = serve.RingArena(capacity)
        self.declined = 0

    def plan(self, members):
        need = sum(r.need_bytes for r in members)
        start = self.arena.alloc(need)
        if start is None:
            self.declined += 1
            return None
        handle, _ = super().plan(members)
        return (handle, start), serve.RingArena.rounded(need)

    def launch(self, handle):
        return super().launch(handle[0])

    def release(self, b, token):
        self.arena.release(b[1])


def test_declined_plans_are_retried_in_arrival_order():
    reqs = _requests(300, 200_000, 11)
    by_id = {r.rid: r for r in reqs}
    be = DecliningBackend(capacity=2 << 20, sec_per_product=1e-9)
    # at most 16 members of at most 100 KB: every batch fits the arena alone
    srv = serve.Server(be, budget_bytes=1 << 30, batch_products=1e7, max_batch=16, max_inflight=3,
                       bytes_per_product=None)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(300))
    assert be.declined > 0 and srv.waits_for_memory >= be.declined
    assert not be.arena.chunks
    for ids in be.planned:
        assert ids == sorted(ids) and len({by_id[i].klass for i in ids}) == 1
    # FIFO within a class survives the requeueing: each class is planned in arrival order
    for k in ("dense", "hash"):
        seq = [i for ids in be.planned for i in ids if by_id[i].klass == k]
        assert seq == sorted(seq)


def test_declined_plan_with_nothing_in_flight_is_an_error():
    reqs = _requests(3, 1000, 12)
    for r in reqs:
        r.need_bytes = 10 << 20
    with pytest.raises(RuntimeError, match="even alone"):
        serve.Server(DecliningBackend(capacity=1 << 20), budget_bytes=1 << 30).run(reqs)


def test_arena_allocator_undo_and_give_back():
    a = serve.RingArena(1 << 16)
    first = a.alloc(1000)
    s1, s2 = a.alloc(300), a.alloc(5000)
    a.release_last(s2)
    a.release_last(s1)
    with pytest.raises(RuntimeError):
        a.release_last(s1)
    assert a.alloc(256) == serve.RingArena.rounded(1000)
    a.release(first)


def test_batch_above_the_budget_is_an_error():
    reqs = _requests(5, 1000, 5)
    for r in reqs:
        r.need_bytes = 10 << 20
    srv = serve.Server(FakeBackend(), budget_bytes=1 << 20)
    with pytest.raises(RuntimeError, match="above the budget"):
        srv.run(reqs)


def test_poisson_arrivals_rate_and_order():
    t = serve.poisson_arrivals(2000.0, 5.0, 7)
    assert np.all(np.diff(t) > 0) and t[-1] < 5.0
    assert abs(len(t) - 10_000) < 5 * np.sqrt(10_000)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 2000) < 0.05 / 2000
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05  # exponential: coefficient of variation 1


def test_latency_summary():
    rs = [serve.Request(i, None, None, (), (), 0.0) for i in range(100)]
    for i, r in enumerate(rs):
        r.done = (i + 1) * 1e-3
    s = serve.latency_summary(rs)
    assert s["requests"] == 100
    assert abs(s["latency_ms_p50"] - 50.5) < 1e-9
    assert abs(s["latency_ms_p99"] - 99.01) < 1e-9


def test_ring_arena_first_in_first_out():
    a = serve.RingArena(1000 * 256)
    s0 = a.alloc(400 * 256)
    s1 = a.alloc(400 * 256)
    assert (s0, s1) == (0, 400 * 256)
    assert a.alloc(300 * 256) is None  # 200 free at the end, 0 at the front
    a.release(s0)
    s2 = a.alloc(300 * 256)  # wraps to the front
    assert s2 == 0
    assert a.alloc(101 * 256) is None  # free: [300, 400) only
    s3 = a.alloc(100 * 256)
    assert s3 == 300 * 256
    with pytest.raises(RuntimeError):
        a.release(s2)  # s1 is older
    a.release(s1)
    a.release(s2)
    a.release(s3)
    assert a.alloc(1000 * 256) == 0
    assert a.alloc(1) is None


def test_ring_arena_never_overlaps():
    rng = np.random.default_rng(9)
    a = serve.RingArena(1 << 20)
    live = []
    for _ in range(2000):
        if live and (rng.random() < 0.45 or len(live) > 20):
            a.release(live.pop(0)[0])
        else:
            n = int(rng.integers(1, 200_000))
            s = a.alloc(n)
            if s is not None:
                e = s + n
                assert 0 <= s and e <= a.size
                for (s2, e2) in live:
                    assert e <= s2 or s >= e2
                live.append((s, e))


def test_autotuner_picks_fastest_and_caches(tmp_path):
    from paper_2410_10094_amd import autotune
    calls = []

    def run(lf, bud, tile):
        calls.append((lf, bud, tile))
        return abs(lf - 0.625) + abs(bud - 5e8) / 1e9 + (tile == 2048) * 0.01  # fastest at (0.625, 5e8, 1024)

    path = str(tmp_path / "tune.json")
    t = autotune.Autotuner(path)
    rec = t.tune("k", run)
    assert (rec["load_factor"], rec["batch_products"], rec["tile"]) == (0.625, 5e8, 1024)
    n = len(autotune.LOAD_FACTORS) * len(autotune.BATCH_BUDGETS) * len(autotune.TILES)
    assert len(calls) == n
    again = autotune.Autotuner(path).tune("k", run)  # from the cache: no new timings
    assert again["load_factor"] == 0.625 and again["tile"] == 1024 and len(calls) == n


def test_autotuner_tie_prefers_larger_load_factor_and_batch():
    from paper_2410_10094_amd import autotune
    assert autotune.choose({(0.5, 1e9, 1024): 1.0, (0.9, 1e9, 1024): 1.0, (0.9, 2e9, 1024): 1.0,
                            (0.9, 2e9, 2048): 1.0, (0.5, 2e8, 2048): 2.0}) == (0.9, 2e9, 2048)


def test_scheduler_cost_estimate_and_classes():
    from paper_2410_10094_amd import sched

    class C:
        def __init__(self, dims, nnz):
            self.dims, self.nnz = dims, nnz

    class Prob:
        X = C((10, 20, 30), 600)
        Y = C((30, 8, 8), 90)
        cx, cy = (2,), (0,)

    assert sched.estimate_products(Prob) == 600 * 90 / 30
    assert sched.shape_class((30, 8, 8), (0,)) == "dense"  # 6 bits of Y free key
    assert sched.shape_class((30, 4096, 4096), (0,)) == "hash"  # 24 bits
    b = sched.make_batches([1, 2, 3, 4, 5], lambda x: x, lambda x: "odd" if x % 2 else "even", 4)
    assert b == [[0, 2], [1], [3], [4]]  # one class per batch, arrival order, cost within 4


def test_batches_sized_so_in_flight_batches_fit():
    srv = serve.Server(FakeBackend(), budget_bytes=64 << 30, batch_products=1e9, max_inflight=2)
    assert srv.batch_products == (64 << 30) / (2 * 40.0)
    srv = serve.Server(FakeBackend(), budget_bytes=1 << 40, batch_products=1e9, max_inflight=2)
    assert srv.batch_products == 1e9
