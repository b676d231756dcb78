"""Serving: continuous batching of lnL + gradient requests from many MCMC / optimiser clients.

Each client registers a data set (tips, pattern weights, model, tree) once and then submits
branch-length vectors; every request returns lnL and all 2N-2 branch gradients.

* Sessions keep their instance (partial buffers, matrices, tip states) resident on the
  device between requests.  A session is admitted only if its workspace fits the device
  memory budget; idle sessions are evicted least-recently-used to make room, and a request
  whose session cannot be admitted waits.
* A data set larger than the per-session cap is split into pattern chunks (patterns are
  conditionally independent given the tree and model); each chunk is its own sub-session
  and the request's result is the sum over chunks, taken in chunk order.  So is a data set
  whose evaluation is estimated to take longer than `max_chunk_seconds` (chunks of at least
  `min_chunk_patterns`): a long evaluation then reaches the device as several shorter
  launches, between which other clients' work gets the compute units it would otherwise
  wait for behind one long kernel.
* A scheduler thread forms batches continuously: requests that arrive while earlier batches
  run are admitted as soon as memory and their session are free, and up to HP_MAX_BATCH
  sessions of one class (precision, state padding, categories) are evaluated by a single
  launch per kernel (hp_batch_evaluate_device) on that class's stream; several batches per
  class may be in flight and different classes overlap on the device.
* Batching is size-aware.  A batch finishes with its slowest member, so each session's
  evaluation time is estimated from its algorithmic bytes and flops, and sessions below
  `small_seconds` form their own tier: small requests are batched with small requests, on
  streams and in-flight slots of their own, and never wait behind a large evaluation of their
  class.  Large sessions are batched only with sessions of similar cost.
* Latency is measured from submission to result (p50 / p99), beside throughput.
* A malformed request (wrong length, negative or non-finite branch length) fails with
  HP_ERR_VALUE on its own future; an error reported by the device for one session fails
  only that session's request; the loop keeps serving everyone else.

Results do not depend on what else is batched or running: the batched kernels run the same
per-instance arithmetic with fixed-order reductions, so a result is bitwise the same alone
and in the mix.

All device work goes through an executor (`HipExecutor`); the scheduling logic itself is
plain Python and is tested on the CPU with a stand-in executor.
"""
from __future__ import annotations

import collections
import ctypes
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import _lib

DEFAULT_PRECISION = {4: "f32"}   # larger state spaces default to "bf16"
MAX_BATCH = 32                   # HP_MAX_BATCH


@dataclass
class Dataset:
    tips: np.ndarray          # uint8 [N, P]
    weights: np.ndarray       # float64 [P]
    V: np.ndarray
    Vinv: np.ndarray
    lam: np.ndarray
    pi: np.ndarray
    rates: np.ndarray
    cat_weights: np.ndarray
    children: np.ndarray      # int [2N-1, 2]

    @property
    def n_tips(self):
        return self.tips.shape[0]

    @property
    def n_patterns(self):
        return self.tips.shape[1]

    @property
    def n_states(self):
        return self.pi.shape[0]

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights,
                   wl.tree.children)

    def chunk(self, lo, hi):
        return Dataset(np.ascontiguousarray(self.tips[:, lo:hi]), self.weights[lo:hi], self.V,
                       self.Vinv, self.lam, self.pi, self.rates, self.cat_weights, self.children)


def scaling_for(n_states, precision):
    return _lib.default_scaling(n_states, precision)


ELEM_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "bf16x3": 4}


def work_seconds(data: Dataset, precision: str, hbm_bytes_per_s: float = 5e12,
                 flops_per_s: float = 100e12, fixed_s: float = 30e-6) -> float:
    """Estimated device time of one evaluation with gradients: the algorithmic bytes of the
    per-operation accounting (5 (N-2) partial-sized transfers) over a sustained bandwidth,
    or the matrix products (4 per internal node, 2 S^2 flops per pattern and category) over a
    sustained throughput, whichever is longer, plus a fixed launch cost.  Used only to order
    and group work, never for results."""
    N, P, S, K = data.n_tips, data.n_patterns, data.n_states, len(data.rates)
    S_pad = 4 if S <= 4 else (32 if S <= 32 else 64)
    nbytes = 5.0 * max(N - 2, 1) * P * K * S_pad * ELEM_BYTES.get(precision, 4) + 2.0 * N * P
    flops = 0.0 if S <= 4 else 4.0 * max(N - 2, 1) * P * K * 2.0 * S * S
    return max(nbytes / hbm_bytes_per_s, flops / flops_per_s) + fixed_s


class DeviceMemory:
    """Session workspaces straight from hipMalloc / hipFree.  An evicted session's memory goes
    back to the device at once; a caching allocator would keep it for its own reuse, and
    sessions of very different sizes then fragment it until a large one no longer fits."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = device
        _lib.load()                                   # torch first, then the runtime it loaded
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.hip.hipMalloc.restype = ctypes.c_int
        self.hip.hipFree.argtypes = [ctypes.c_void_p]
        self.hip.hipFree.restype = ctypes.c_int

    def alloc(self, nbytes: int) -> int:
        p = ctypes.c_void_p()
        with self.torch.cuda.device(self.device):
            rc = self.hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(nbytes))
        if rc != 0 or not p.value:
            raise MemoryError(f"hipMalloc of {nbytes} bytes failed (hipError {rc})")
        return p.value

    def free(self, ptr: int) -> None:
        with self.torch.cuda.device(self.device):
            self.hip.hipFree(ctypes.c_void_p(ptr))


class Arena:
    """Session workspaces carved out of one device allocation (first fit over a sorted free
    list, neighbours coalesced, 256-byte granules).  Evicting a session returns its range
    here and never to the runtime: freeing device memory synchronises the whole device,
    which would stall every batch in flight.  alloc raises MemoryError when no free range
    is large enough; the server then evicts more idle sessions."""

    GRAIN = 256

    def __init__(self, base: int, nbytes: int):
        self.base = base
        self.size = nbytes // self.GRAIN * self.GRAIN
        self.free = [(0, self.size)]                # (offset, length), sorted by offset

    def alloc(self, nbytes: int) -> int:
        n = -(-nbytes // self.GRAIN) * self.GRAIN
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[i]
                else:
                    self.free[i] = (off + n, ln - n)
                return self.base + off
        raise MemoryError(f"no free range of {n} bytes (largest {self.largest()})")

    def release(self, ptr: int, nbytes: int) -> None:
        off = ptr - self.base
        n = -(-nbytes // self.GRAIN) * self.GRAIN
        import bisect
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, n))
        # coalesce with the right, then the left neighbour
        if i + 1 < len(self.free) and off + n == self.free[i + 1][0]:
            self.free[i] = (off, n + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    def largest(self) -> int:
        return max((ln for _, ln in self.free), default=0)


class HipExecutor:
    """Device side of the server: instances, batched launches on a few streams per size tier.

    The runtime maps streams onto a handful of hardware queues (four by default), and work on
    one queue runs in order: a small batch placed behind a long evaluation on the same queue
    waits for all of it.  So there are few streams, created together at start-up: two for
    small batches and one for large ones, shared by every class, which keeps small work on
    queues of its own."""

    STREAMS = {0: 2, 1: 1}          # size tier -> streams

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = _lib.load()
        self.device_index = device
        self.device = torch.device("cuda", device)
        self.streams = {tier: [torch.cuda.Stream(device=self.device) for _ in range(n)]
                        for tier, n in self.STREAMS.items()}
        self.turn = collections.Counter()
        self.memory = DeviceMemory(device)
        self.arena = None

    def reserve(self, nbytes: int) -> None:
        """Take the sessions' device memory once, up front."""
        if self.arena is None:
            self.arena = Arena(self.memory.alloc(nbytes), nbytes)

    def close(self) -> None:
        """Give the arena back to the device (every session must have been evicted)."""
        if self.arena is not None:
            self.torch.cuda.synchronize(self.device)
            self.memory.free(self.arena.base)
            self.arena = None

    def free_memory(self):
        free, _ = self.torch.cuda.mem_get_info(self.device)
        return free

    @staticmethod
    def pre_buffers(data: Dataset) -> int:
        """Pre-order buffers the session's tree needs (the walk reuses them: ~ tree height)."""
        if getattr(data, "_n_pre", None) is None:
            data._n_pre = _lib.plan_pre_buffers(data.children)
        return data._n_pre

    def footprint(self, data: Dataset, precision: str) -> int:
        sc = scaling_for(data.n_states, precision)
        d = _lib.hp_desc(n_tips=data.n_tips, n_patterns=data.n_patterns, n_states=data.n_states,
                         n_categories=len(data.rates), n_partials=data.n_tips - 1,
                         n_matrices=2 * data.n_tips - 2, n_eigen=1,
                         precision=_lib.PRECISIONS[precision], scaling=_lib.SCALINGS[sc[0]],
                         scale_period=sc[1], device=self.device_index,
                         n_pre_partials=self.pre_buffers(data))
        n = ctypes.c_size_t()
        _lib.check(self.lib, self.lib.hp_workspace_bytes(ctypes.byref(d), ctypes.byref(n)))
        return n.value

    def load(self, s):
        torch = self.torch
        from .instance import Instance
        d = s.data
        sc = scaling_for(d.n_states, s.precision)
        if self.arena is None:
            raise RuntimeError("HipExecutor.reserve was not called")
        ptr = self.arena.alloc(s.footprint)
        try:
            inst = Instance(d.n_tips, d.n_patterns, d.n_states, len(d.rates), precision=s.precision,
                            scaling=sc[0], scale_period=sc[1], device=self.device_index,
                            workspace_ptr=ptr, n_pre_partials=self.pre_buffers(d))
            inst.load(d.tips, d.weights, d.V, d.Vinv, d.lam, d.pi, d.rates, d.cat_weights,
                      children=d.children)
        except BaseException:
            torch.cuda.synchronize(self.device)
            self.arena.release(ptr, s.footprint)
            raise
        nb = 2 * d.n_tips - 2
        s.state = {"inst": inst, "ptr": ptr,
                   "t_dev": torch.empty(nb, dtype=torch.float64, device=self.device),
                   "out_dev": torch.empty(1 + nb, dtype=torch.float64, device=self.device),
                   "t_host": torch.empty(nb, dtype=torch.float64, pin_memory=True),
                   "out_host": torch.empty(1 + nb, dtype=torch.float64, pin_memory=True)}
        return (s.precision, inst.query(_lib.HP_Q_STATE_PAD), len(d.rates), inst.query(_lib.HP_Q_TILE))

    def evict(self, s):
        if s.state is not None:
            # the session is idle: its last batch has completed and its uploads were
            # synchronous, so nothing in flight reads this range any more
            s.state["inst"].close()
            self.arena.release(s.state["ptr"], s.footprint)
        s.state = None

    def launch(self, key, items):
        """items: [(session, t)].  Enqueue one batched evaluation; return a completion token."""
        torch = self.torch
        # the streams of the batch's size tier (key: (class, tier)), in turn
        tier = key[1] if isinstance(key, tuple) and len(key) == 2 and key[1] in self.streams else 1
        pool = self.streams[tier]
        stream = pool[self.turn[tier] % len(pool)]
        self.turn[tier] += 1
        with torch.cuda.stream(stream):
            for s, t in items:
                st = s.state
                st["t_host"].numpy()[:] = t
                st["t_dev"].copy_(st["t_host"], non_blocking=True)
            n = len(items)
            insts = (ctypes.c_void_p * n)(*[s.state["inst"]._inst.value for s, _ in items])
            tp = (ctypes.c_void_p * n)(*[s.state["t_dev"].data_ptr() for s, _ in items])
            op = (ctypes.c_void_p * n)(*[s.state["out_dev"].data_ptr() for s, _ in items])
            rc = self.lib.hp_batch_evaluate_device(insts, tp, op, n, 1, ctypes.c_void_p(stream.cuda_stream))
            if rc != _lib.HP_OK:
                raise _lib.HPError(rc, _lib.last_error(self.lib, None))
            for s, _ in items:
                s.state["out_host"].copy_(s.state["out_dev"], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return (ev, items)

    def poll(self, token):
        """None while running; then [(ok, result or exception)] per item.  Branch lengths
        were validated on submission, so the only device-side error left is a zero or
        non-finite site likelihood, which makes lnL -inf or NaN: the instance's status word
        (read and cleared with a wait on its stream) is consulted only for such a result,
        and a completed batch never waits on other work."""
        ev, items = token
        if not ev.query():
            return None
        res = []
        for s, _ in items:
            out = s.state["out_host"].numpy().copy()
            if np.all(np.isfinite(out)):
                res.append((True, out))
                continue
            try:
                s.state["inst"].status()
                res.append((False, _lib.HPError(_lib.HP_ERR_NUMERIC, "a site likelihood was zero or not finite")))
            except Exception as e:  # noqa: BLE001 - reported on that request only
                res.append((False, e))
        return res


class _Session:
    """One admitted-or-evictable unit: a client's data set or one pattern chunk of it."""

    def __init__(self, client, chunk, data: Dataset, precision, footprint, cost=0.0, tier=0):
        self.client = client
        self.chunk = chunk
        self.data = data
        self.precision = precision
        self.footprint = footprint
        self.cost = cost           # estimated seconds per evaluation
        self.tier = tier           # 0: small (its own batches, streams and slots), 1: large
        self.state = None          # executor's resident state (None: not on the device)
        self.key = None
        self.busy = False
        self.last_used = 0.0

    @property
    def resident(self):
        return self.state is not None


@dataclass
class _Request:
    client: int
    t: np.ndarray
    arrival: float
    future: Future
    parts: dict = field(default_factory=dict)     # chunk -> out (lnL, grads)
    remaining: int = 0


class Server:
    """Continuous-batching request loop on one device.

    memory_budget: bytes of device memory the sessions' workspaces may occupy (default: 85 %
    of the device's free memory at start-up); max_session_bytes: data sets whose workspace
    exceeds this are split into pattern chunks (default: a quarter of the budget).
    small_seconds: sessions whose estimated evaluation time is below this are small (their
    own tier); max_inflight_per_class / max_inflight_small: batches in flight per class and
    tier (large / small); large_ratio: large sessions are batched only with sessions within
    this factor of the oldest request's cost.
    """

    def __init__(self, device: int = 0, memory_budget: int | None = None,
                 max_session_bytes: int | None = None, max_batch: int = MAX_BATCH,
                 max_inflight_per_class: int = 2, precision: dict | None = None, executor=None,
                 small_seconds: float = 2e-3, max_inflight_small: int = 4, large_ratio: float = 2.0,
                 max_chunk_seconds: float = 10e-3, min_chunk_patterns: int = 4096):
        self.ex = executor if executor is not None else HipExecutor(device)
        if memory_budget is None:
            memory_budget = int(0.85 * self.ex.free_memory())
        self.memory_budget = int(memory_budget)
        if hasattr(self.ex, "reserve"):
            self.ex.reserve(self.memory_budget)
        self.max_session_bytes = int(max_session_bytes or self.memory_budget // 4)
        self.max_batch = max(1, min(int(max_batch), MAX_BATCH))
        self.max_inflight = max(1, int(max_inflight_per_class))
        self.max_inflight_small = max(1, int(max_inflight_small))
        self.small_seconds = float(small_seconds)
        self.large_ratio = max(1.0, float(large_ratio))
        self.max_chunk_seconds = float(max_chunk_seconds)
        self.min_chunk_patterns = max(1, int(min_chunk_patterns))
        self.precision = dict(DEFAULT_PRECISION)
        self.precision.update(precision or {})
        self.sessions = {}                          # client -> [chunk sessions]
        self.used = 0
        self.pending = collections.OrderedDict()    # session -> deque of requests
        self.inflight = []                          # (token, key, [(session, request)])
        self.cv = threading.Condition()
        self.incoming = collections.deque()
        self.running = False
        self.thread = None
        self.latencies = []
        self.latencies_small = []                   # requests whose every session is small
        self.completed = 0
        self.errors = 0
        self.batches = 0
        self.batch_sizes = []
        self.evictions = 0
        self.loads = 0
        self.load_seconds = 0.0
        self.evict_seconds = 0.0
        self.max_concurrent_batches = 0
        self.t_first = None
        self.t_last = None

    # ------------------------------------------------------------------ clients
    def register(self, client, data: Dataset, precision: str | None = None) -> int:
        prec = precision or self.precision.get(data.n_states, "bf16")
        full = self.ex.footprint(data, prec)
        n_chunks = max(1, -(-full // self.max_session_bytes))
        # long evaluations are cut into chunks of about max_chunk_seconds, never below
        # min_chunk_patterns patterns each
        cost_full = self.ex.cost(data, prec) if hasattr(self.ex, "cost") else work_seconds(data, prec)
        n_time = min(int(np.ceil(cost_full / self.max_chunk_seconds)), data.n_patterns // self.min_chunk_patterns)
        n_chunks = max(n_chunks, n_time)
        if n_chunks > data.n_patterns:
            raise ValueError(f"client {client}: cannot chunk {data.n_patterns} patterns into {n_chunks}")
        bounds = np.linspace(0, data.n_patterns, n_chunks + 1).astype(int)
        sess = []
        for c in range(n_chunks):
            d = data if n_chunks == 1 else data.chunk(bounds[c], bounds[c + 1])
            fp = full if n_chunks == 1 else self.ex.footprint(d, prec)
            if fp > self.memory_budget:
                raise ValueError(f"client {client}: a pattern chunk does not fit the memory budget")
            cost = self.ex.cost(d, prec) if hasattr(self.ex, "cost") else work_seconds(d, prec)
            sess.append(_Session(client, c, d, prec, fp, cost, 0 if cost < self.small_seconds else 1))
        with self.cv:
            self.sessions[client] = sess
        return n_chunks

    def submit(self, client, t) -> Future:
        fut = Future()
        with self.cv:
            if client not in self.sessions:
                raise KeyError(f"client {client} is not registered")
            nb = 2 * self.sessions[client][0].data.n_tips - 2
        t = np.asarray(t, dtype=np.float64).ravel()
        if t.size != nb or not np.all(np.isfinite(t)) or np.any(t < 0):
            fut.set_exception(_lib.HPError(_lib.HP_ERR_VALUE,
                                           f"client {client}: need {nb} finite non-negative branch lengths"))
            with self.cv:
                self.errors += 1
            return fut
        req = _Request(client, np.ascontiguousarray(t), time.perf_counter(), fut)
        with self.cv:
            self.incoming.append(req)
            self.cv.notify()
        return fut

    def evaluate(self, client, t):
        """Synchronous convenience: submit and wait for (lnL, gradients)."""
        return self.submit(client, t).result()

    # ------------------------------------------------------------------ lifecycle
    def start(self):
        if not self.running:
            self.running = True
            self.thread = threading.Thread(target=self._loop, name="hipphylo-serve", daemon=True)
            self.thread.start()
        return self

    def stop(self):
        """Finish every submitted request, then stop the scheduler thread."""
        with self.cv:
            self.running = False
            self.cv.notify()
        if self.thread is not None:
            self.thread.join()
        self.thread = None

    def close(self):
        self.stop()
        for sess in self.sessions.values():
            for s in sess:
                if s.resident:
                    self.ex.evict(s)
        self.used = 0
        if hasattr(self.ex, "close"):
            self.ex.close()

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.close()

    def reset_stats(self):
        """Start a new measurement window (counters, latencies, throughput span)."""
        with self.cv:
            self.latencies = []
            self.latencies_small = []
            self.completed = self.errors = self.batches = self.evictions = self.loads = 0
            self.load_seconds = self.evict_seconds = 0.0
            self.batch_sizes = []
            self.max_concurrent_batches = 0
            self.t_first = self.t_last = None

    def stats(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        lat_s = np.array(self.latencies_small) if self.latencies_small else np.zeros(1)
        span = (self.t_last - self.t_first) if self.completed else 0.0
        return {"completed": self.completed, "errors": self.errors, "batches": self.batches,
                "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
                "max_concurrent_batches": self.max_concurrent_batches,
                "evictions": self.evictions, "loads": self.loads,
                "load_seconds": self.load_seconds, "evict_seconds": self.evict_seconds,
                "p50_ms": 1000 * float(np.percentile(lat, 50)),
                "p99_ms": 1000 * float(np.percentile(lat, 99)),
                "mean_ms": 1000 * float(np.mean(lat)),
                "small_completed": len(self.latencies_small),
                "small_p50_ms": 1000 * float(np.percentile(lat_s, 50)),
                "small_p99_ms": 1000 * float(np.percentile(lat_s, 99)),
                "requests_per_s": self.completed / span if span > 0 else float("nan"),
                "memory_used": self.used, "memory_budget": self.memory_budget}

    # ------------------------------------------------------------------ scheduler (one thread)
    def _loop(self):
        while True:
            with self.cv:
                while self.incoming:
                    req = self.incoming.popleft()
                    sess = self.sessions[req.client]
                    req.remaining = len(sess)
                    for s in sess:
                        self.pending.setdefault(s, collections.deque()).append(req)
                if not self.running and not self.pending and not self.inflight:
                    return
                if not self.pending and not self.inflight:
                    self.cv.wait(timeout=0.01)
                    continue
            try:
                progressed = self._complete()
                progressed |= self._dispatch()
            except Exception as e:  # noqa: BLE001 - the loop must outlive any one failure
                self._fail_everything(e)
                progressed = True
            if not progressed:
                time.sleep(50e-6)

    def _fail_everything(self, err):
        """An error outside any one request's scope: fail what is queued and in flight, free
        the sessions' busy marks, and keep serving new requests."""
        with self.cv:
            for q in self.pending.values():
                for req in q:
                    self._fail(req, err)
            self.pending.clear()
            for _, _, items in self.inflight:
                for s, req in items:
                    s.busy = False
                    self._fail(req, err)
            self.inflight = []

    def _idle_lru(self):
        idle = [x for sess in self.sessions.values() for x in sess
                if x.resident and not x.busy and not self.pending.get(x)]
        return min(idle, key=lambda x: x.last_used) if idle else None

    def _evict(self, x):
        t0 = time.perf_counter()
        self.ex.evict(x)
        self.used -= x.footprint
        self.evictions += 1
        self.evict_seconds += time.perf_counter() - t0

    def _admit(self, s: _Session) -> bool:
        """Make s resident: evict idle sessions, least recently used first, until its
        footprint fits the budget and the executor finds room for it (a fragmented arena
        can refuse a fitting total); False if that cannot be done now."""
        if s.resident:
            return True
        while True:
            if self.used + s.footprint <= self.memory_budget:
                t0 = time.perf_counter()
                try:
                    s.key = self.ex.load(s)
                except MemoryError:
                    pass                              # no contiguous room: evict more
                except Exception as e:  # noqa: BLE001 - fail this session's requests only
                    for req in self.pending.get(s, ()):
                        self._fail(req, e)
                    self.pending[s] = collections.deque()
                    return False
                else:
                    self.used += s.footprint
                    self.loads += 1
                    self.load_seconds += time.perf_counter() - t0
                    return True
            victim = self._idle_lru()
            if victim is None:
                return False
            self._evict(victim)

    def _dispatch(self) -> bool:
        launched = False
        by_class = collections.defaultdict(list)
        for s in [s for s, q in self.pending.items() if q and not s.busy]:
            if self._admit(s):
                by_class[(s.key, s.tier)].append(s)
        for key, group in by_class.items():
            tier = key[1]
            limit = self.max_inflight if tier else self.max_inflight_small
            if sum(1 for b in self.inflight if b[1] == key) >= limit:
                continue
            group.sort(key=lambda s: self.pending[s][0].arrival)
            if tier:
                # a batch of large sessions runs as long as its slowest member: only sessions
                # within large_ratio of the oldest request's cost join it
                c0 = group[0].cost
                group = [s for s in group if c0 / self.large_ratio <= s.cost <= c0 * self.large_ratio]
            items = []
            for s in group[: self.max_batch]:
                req = self.pending[s].popleft()
                s.busy = True
                items.append((s, req))
            try:
                token = self.ex.launch(key, [(s, req.t) for s, req in items])
            except Exception as e:  # noqa: BLE001 - fail this batch's requests only
                for s, req in items:
                    s.busy = False
                    self._fail(req, e)
                continue
            self.inflight.append((token, key, items))
            self.max_concurrent_batches = max(self.max_concurrent_batches, len(self.inflight))
            self.batches += 1
            self.batch_sizes.append(len(items))
            launched = True
        for s in [s for s, q in self.pending.items() if not q]:
            del self.pending[s]
        return launched

    def _fail(self, req, err):
        if not req.future.done():
            req.future.set_exception(err)
            self.errors += 1

    def _complete(self) -> bool:
        done_any = False
        still = []
        for token, key, items in self.inflight:
            res = self.ex.poll(token)
            if res is None:
                still.append((token, key, items))
                continue
            done_any = True
            now = time.perf_counter()
            for (s, req), (ok, val) in zip(items, res):
                s.busy = False
                s.last_used = now
                if not ok:
                    self._fail(req, val)
                    continue
                req.parts[s.chunk] = val
                req.remaining -= 1
                if req.remaining == 0 and not req.future.done():
                    out = req.parts[0].copy()
                    for c in range(1, len(req.parts)):
                        out += req.parts[c]
                    req.future.set_result((float(out[0]), out[1:]))
                    self.latencies.append(now - req.arrival)
                    if all(x.tier == 0 for x in self.sessions[req.client]):
                        self.latencies_small.append(now - req.arrival)
                    self.completed += 1
                    self.t_first = req.arrival if self.t_first is None else min(self.t_first, req.arrival)
                    self.t_last = now
        self.inflight = still
        return done_any


__all__ = ["Server", "Dataset", "HipExecutor", "Arena"]
