"""Scheduling logic of the serving loop on the CPU, with a stand-in executor (a test double:
it never computes a likelihood, it returns a deterministic function of the request so that
batching, chunking, admission and error isolation can be checked exactly)."""
import threading
import time

import numpy as np
import pytest

from paper_2606_27607_amd import _lib
from paper_2606_27607_amd.serve import Arena, Dataset, Server


class FakeExecutor:
    def __init__(self, service_s=0.002, fail_clients=(), raise_on_launch=(), raise_on_load=(),
                 raise_on_poll=0, arena_bytes=None, cost_per_pattern=None):
        self.service_s = service_s
        # with cost_per_pattern, a session's estimated cost (and a batch's service time, that
        # of its slowest member) is proportional to its pattern count
        self.cost_per_pattern = cost_per_pattern
        self.fail_clients = set(fail_clients)
        self.raise_on_launch = set(raise_on_launch)
        self.raise_on_load = set(raise_on_load)
        self.raise_on_poll = raise_on_poll            # polls that raise, counted down
        self.arena = Arena(1 << 40, arena_bytes) if arena_bytes else None
        self.resident = set()
        self.used = 0
        self.budget = None
        self.max_used = 0
        self.launches = []
        self.lock = threading.Lock()

    def free_memory(self):
        return 1 << 40

    def footprint(self, data, precision):
        return data.n_tips * data.n_patterns * 8

    def cost(self, data, precision):
        return (self.cost_per_pattern or 1e-9) * data.n_patterns

    def load(self, s):
        if s.client in self.raise_on_load:
            raise RuntimeError("device allocation failed")
        ptr = self.arena.alloc(s.footprint) if self.arena else None
        with self.lock:
            assert s not in self.resident
            self.resident.add(s)
            self.used += s.footprint
            self.max_used = max(self.max_used, self.used)
        s.state = {"loaded": True, "ptr": ptr}
        return (s.precision, 4 if s.data.n_states <= 4 else 64, len(s.data.rates))

    def evict(self, s):
        if self.arena:
            self.arena.release(s.state["ptr"], s.footprint)
        with self.lock:
            self.resident.discard(s)
            self.used -= s.footprint
        s.state = None

    def launch(self, key, items):
        clients = {s.client for s, _ in items}
        if clients & self.raise_on_launch:
            raise RuntimeError("launch failed")
        for s, _ in items:
            assert s in self.resident
        self.launches.append([s.client for s, _ in items])
        if self.cost_per_pattern:
            return (time.perf_counter() + max(s.cost for s, _ in items), items)
        return (time.perf_counter() + self.service_s, items)

    def poll(self, token):
        if self.raise_on_poll > 0:
            self.raise_on_poll -= 1
            raise RuntimeError("device lost")
        t_done, items = token
        if time.perf_counter() < t_done:
            return None
        res = []
        for s, t in items:
            if s.client in self.fail_clients:
                res.append((False, _lib.HPError(_lib.HP_ERR_NUMERIC, "injected")))
            else:
                npat = s.data.n_patterns
                res.append((True, np.concatenate([[t.sum() * npat], t * npat])))
        return res


def dataset(n_tips, n_patterns, n_states=4):
    return Dataset(tips=np.zeros((n_tips, n_patterns), np.uint8), weights=np.ones(n_patterns),
                   V=np.eye(n_states), Vinv=np.eye(n_states), lam=np.zeros(n_states),
                   pi=np.full(n_states, 1.0 / n_states), rates=np.ones(4), cat_weights=np.full(4, 0.25),
                   children=np.zeros((2 * n_tips - 1, 2), np.int64))


def expected(t, n_patterns):
    return t.sum() * n_patterns, t * n_patterns


def test_results_and_batching():
    ex = FakeExecutor(service_s=0.005)
    with Server(memory_budget=10 ** 9, executor=ex, max_inflight_per_class=2) as srv:
        for c in range(12):
            srv.register(c, dataset(5 + c, 100 + 10 * c, 4 if c % 2 else 61))
        futs = []
        rng = np.random.default_rng(0)
        for rep in range(4):
            for c in range(12):
                t = rng.random(2 * (5 + c) - 2)
                futs.append((c, t, srv.submit(c, t)))
        for c, t, f in futs:
            lnl, g = f.result(timeout=10)
            e_l, e_g = expected(t, 100 + 10 * c)
            assert lnl == e_l and np.array_equal(g, e_g)
        st = srv.stats()
    assert st["completed"] == 48 and st["errors"] == 0
    assert st["mean_batch"] > 1.0                      # same-class requests shared launches
    assert st["max_concurrent_batches"] >= 2           # batches overlapped (in flight together)
    # one request per session per batch, and a session's requests are served in order
    for b in ex.launches:
        assert len(b) == len(set(b))


def test_continuous_admission_while_busy():
    """Requests arriving while a batch is in flight join the next batch, not a queue behind it."""
    ex = FakeExecutor(service_s=0.05)
    with Server(memory_budget=10 ** 9, executor=ex, max_inflight_per_class=1) as srv:
        for c in range(6):
            srv.register(c, dataset(6, 50))
        f0 = srv.submit(0, np.ones(10))
        time.sleep(0.01)                               # batch [0] is running
        fs = [srv.submit(c, np.ones(10)) for c in range(1, 6)]
        for f in [f0] + fs:
            f.result(timeout=10)
    assert ex.launches[0] == [0]
    assert sorted(ex.launches[1]) == [1, 2, 3, 4, 5]  # all late arrivals in one launch


def test_memory_admission_and_eviction():
    ex = FakeExecutor(service_s=0.001)
    fp = 10 * 100 * 8
    with Server(memory_budget=3 * fp, executor=ex) as srv:   # three sessions fit at once
        for c in range(8):
            srv.register(c, dataset(10, 100))
        futs = [srv.submit(c % 8, np.full(18, 0.1)) for c in range(40)]
        for f in futs:
            f.result(timeout=20)
        st = srv.stats()
    assert ex.max_used <= 3 * fp
    assert st["evictions"] > 0 and st["completed"] == 40


def test_pattern_chunking_sums_chunks():
    ex = FakeExecutor()
    with Server(memory_budget=10 ** 6, max_session_bytes=20 * 1000 * 8 // 3 + 8, executor=ex) as srv:
        n = srv.register(7, dataset(20, 1000))
        assert n == 3
        t = np.linspace(0.01, 0.2, 38)
        lnl, g = srv.evaluate(7, t)
    e_l, e_g = expected(t, 1000)
    assert np.isclose(lnl, e_l, rtol=1e-15) and np.allclose(g, e_g, rtol=1e-15)
    assert sorted(sum(ex.launches, [])) == [7, 7, 7]


def test_error_isolation():
    ex = FakeExecutor(fail_clients={3}, raise_on_launch={5})
    with Server(memory_budget=10 ** 9, executor=ex, precision={4: "f32", 61: "bf16"}) as srv:
        for c in range(6):
            srv.register(c, dataset(4, 20, 61 if c == 5 else 4))
        bad_len = srv.submit(0, np.ones(3))
        bad_val = srv.submit(1, np.array([0.1, np.nan, 0.1, 0.1, 0.1, 0.1]))
        bad_neg = srv.submit(2, np.array([0.1, -0.2, 0.1, 0.1, 0.1, 0.1]))
        dev_err = srv.submit(3, np.full(6, 0.1))
        launch_err = srv.submit(5, np.full(6, 0.1))
        good = [srv.submit(c, np.full(6, 0.1 * (c + 1))) for c in (0, 1, 2, 4)]
        for f in (bad_len, bad_val, bad_neg):
            with pytest.raises(_lib.HPError) as e:
                f.result(timeout=10)
            assert e.value.code == _lib.HP_ERR_VALUE
        with pytest.raises(_lib.HPError):
            dev_err.result(timeout=10)
        with pytest.raises(RuntimeError):
            launch_err.result(timeout=10)
        for c, f in zip((0, 1, 2, 4), good):
            lnl, g = f.result(timeout=10)
            assert lnl == pytest.approx(0.6 * (c + 1) * 20)
        # the server still serves the failing clients' next valid requests (client 3 keeps
        # failing by construction, client 5's launches keep raising)
        assert srv.evaluate(0, np.full(6, 0.2))[0] == pytest.approx(1.2 * 20)
        st = srv.stats()
    assert st["errors"] == 5


def test_unknown_client_and_budget_checks():
    ex = FakeExecutor()
    srv = Server(memory_budget=1000, max_session_bytes=1000, executor=ex)
    with pytest.raises(KeyError):
        srv.submit(99, np.ones(4))
    with pytest.raises(ValueError):
        srv.register(1, dataset(500, 2))                  # cannot be chunked below the cap
    srv.close()


def test_load_failure_fails_only_that_session():
    ex = FakeExecutor(raise_on_load={2})
    with Server(memory_budget=10 ** 9, executor=ex) as srv:
        for c in range(4):
            srv.register(c, dataset(5, 30))
        futs = {c: srv.submit(c, np.full(8, 0.1)) for c in range(4)}
        with pytest.raises(RuntimeError):
            futs[2].result(timeout=10)
        for c in (0, 1, 3):
            assert futs[c].result(timeout=10)[0] == pytest.approx(0.8 * 30)
        with pytest.raises(RuntimeError):                # still failing, still isolated
            srv.evaluate(2, np.full(8, 0.1))
        assert srv.evaluate(1, np.full(8, 0.2))[0] == pytest.approx(1.6 * 30)


def test_loop_survives_unexpected_errors():
    """An error outside any request (here: the completion poll raising) fails what is queued
    and in flight, and the loop keeps serving new requests."""
    ex = FakeExecutor(service_s=0.01, raise_on_poll=1)
    with Server(memory_budget=10 ** 9, executor=ex) as srv:
        for c in range(3):
            srv.register(c, dataset(5, 30))
        first = [srv.submit(c, np.full(8, 0.1)) for c in range(3)]
        for f in first:
            with pytest.raises(RuntimeError):
                f.result(timeout=10)
        assert srv.evaluate(0, np.full(8, 0.1))[0] == pytest.approx(0.8 * 30)


def test_arena_first_fit_and_coalescing():
    a = Arena(4096, 256 * 100)
    p = [a.alloc(256 * n) for n in (10, 20, 30, 40)]
    assert p == [4096, 4096 + 2560, 4096 + 7680, 4096 + 15360]
    with pytest.raises(MemoryError):
        a.alloc(256 * 1)                                  # full
    a.release(p[1], 256 * 20)
    a.release(p[2], 256 * 30)                             # coalesces with p[1]'s range
    assert a.largest() == 256 * 50
    assert a.alloc(256 * 45) == p[1]
    a.release(p[0], 256 * 10)
    a.release(p[1], 256 * 45)
    a.release(p[3], 256 * 40)
    assert a.free == [(0, 256 * 100)]
    assert a.alloc(100) == 4096                           # rounded up to a granule
    assert a.largest() == 256 * 99


def test_fragmented_memory_evicts_until_a_range_fits():
    """Sessions sized 3, 3, 3 (budget 10): a size-4 session fits the budget after one
    eviction but needs two neighbouring ranges free, so admission evicts more."""
    unit = 5 * 100 * 8
    ex = FakeExecutor(service_s=0.001, arena_bytes=10 * unit)
    with Server(memory_budget=10 * unit, executor=ex) as srv:
        for c in range(3):
            srv.register(c, dataset(5, 300))              # footprint 3 units each
        srv.register(3, dataset(5, 400))                  # 4 units
        for c in range(3):
            srv.evaluate(c, np.full(8, 0.1))
        srv.evaluate(1, np.full(8, 0.1))                  # client 0 is now least recently used
        assert srv.evaluate(3, np.full(8, 0.1))[0] == pytest.approx(0.8 * 400)
        st = srv.stats()
    assert st["evictions"] >= 2 and ex.max_used <= 10 * unit


def test_small_requests_never_wait_behind_a_large_one():
    """One large evaluation of a class in flight (its only large slot taken) and small
    requests of the same class arriving after it: they run in their own tier and finish
    long before it, batched with each other."""
    ex = FakeExecutor(cost_per_pattern=2e-6)                  # 100,000 patterns: 0.2 s
    with Server(memory_budget=10 ** 9, executor=ex, max_inflight_per_class=1,
                small_seconds=2e-3, max_inflight_small=2, max_chunk_seconds=10.0) as srv:
        srv.register(0, dataset(8, 100_000))
        for c in range(1, 9):
            srv.register(c, dataset(6, 200))                  # 0.4 ms each
        big = srv.submit(0, np.ones(14))
        time.sleep(0.01)
        smalls = [srv.submit(c, np.ones(10)) for c in range(1, 9)]
        for f in smalls:
            f.result(timeout=5)
        assert not big.done()
        big.result(timeout=5)
        st = srv.stats()
    assert st["small_completed"] == 8 and st["small_p99_ms"] < 100
    small_batches = [b for b in ex.launches if 0 not in b]
    assert len(small_batches) < 8                             # they shared launches


def test_large_sessions_batch_only_with_similar_costs():
    """Large sessions whose costs differ by more than large_ratio never share a batch (a batch
    runs as long as its slowest member); similar ones do."""
    ex = FakeExecutor(cost_per_pattern=1e-7)
    with Server(memory_budget=10 ** 10, executor=ex, small_seconds=1e-3, large_ratio=2.0,
                max_inflight_per_class=1, max_chunk_seconds=10.0) as srv:
        sizes = {0: 50_000, 1: 60_000, 2: 400_000, 3: 450_000}   # 5, 6, 40 and 45 ms
        for c, n in sizes.items():
            srv.register(c, dataset(6, n))
        for rep in range(3):
            futs = [srv.submit(c, np.full(10, 0.1 * (rep + 1))) for c in sizes]
            for f in futs:
                f.result(timeout=10)
    for b in ex.launches:
        costs = [sizes[c] for c in b]
        assert max(costs) <= 2.0 * min(costs), b
    assert any(len(b) > 1 for b in ex.launches)


def test_long_evaluations_are_cut_into_time_chunks():
    """A data set estimated at 0.2 s per evaluation becomes 20 pattern chunks of ~10 ms (each at
    least min_chunk_patterns patterns); one whose chunks would fall below that minimum stays
    whole.  Results are the chunk sums, as for memory chunking."""
    ex = FakeExecutor(cost_per_pattern=2e-6)
    with Server(memory_budget=10 ** 12, executor=ex, max_chunk_seconds=10e-3, min_chunk_patterns=4096) as srv:
        assert srv.register(0, dataset(8, 100_000)) == 20
        assert srv.register(1, dataset(8, 6_000)) == 1            # 12 ms, but 6,000 < 2 x 4,096
        assert srv.register(2, dataset(8, 9_000)) == 2
        for c, n in ((0, 100_000), (1, 6_000), (2, 9_000)):
            t = np.linspace(0.01, 0.1, 14)
            lnl, g = srv.evaluate(c, t)
            e_l, e_g = expected(t, n)
            assert np.isclose(lnl, e_l, rtol=1e-12) and np.allclose(g, e_g, rtol=1e-12)
