"""Serving ad hoc layer-pricing queries against a device-resident YET.

A query is a new layer: some ELTs of a pool already resident on the GPU,
with its own occurrence and aggregate terms.  Its answer is the layer's YLT
and PML/TVaR at the requested return periods.  The paper motivates this use
(ad hoc, real-time pricing on a portfolio, Sections I and III); the
scheduling here is this library's own.

Two servers with the same clock and the same device work per query:

* ``serve_batched`` -- continuous batching.  Arrivals are admitted while the
  pool has a free layer slot (the pool's fixed table memory is the admission
  budget; a query that does not fit waits in the queue), and their fused
  tables are built on the GPU on a build stream while the previous group runs
  on the run stream.  Whenever the run stream can take more work, everything
  admitted and built so far (up to ARA_MAX_BATCH layers) leaves as one group:
  one batched pass (dense records for up to 16 layers, sparse records above)
  followed on the same stream by PML/TVaR of the whole group into device
  memory (the entry point that allocates nothing) and a copy of the results
  into pinned host memory.  A group smaller than the measured crossover runs
  as single-layer passes instead, each followed by its own PML/TVaR and copy,
  so that each of its queries is answered when its own pass is done.  The
  host loop never waits for the device: it keeps admitting and building
  arrivals and answers a query when its event has fired.
* ``serve_one_at_a_time`` -- the baseline: each query in arrival order is
  built, run with the single-layer pass and reduced to PML/TVaR before the
  next one starts.

Latency of a query = time its answer is on the host - its scheduled arrival.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from . import ara as A


@dataclass
class Query:
    qid: int
    arrival: float          # seconds after the start of the run
    elt_index: np.ndarray   # pool ELT indices, layer order
    ret: np.ndarray
    lim: np.ndarray
    occ_ret: float
    occ_lim: float
    agg_ret: float
    agg_lim: float
    # filled by the server
    admitted: float = -1.0
    done: float = -1.0
    batch_size: int = 0
    pml: Optional[np.ndarray] = None
    tvar: Optional[np.ndarray] = None
    ylt: Optional[torch.Tensor] = None
    layer: object = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_queries(items) -> List[Query]:
    """Queries from (arrival, LayerSpec, pool indices) triples."""
    out = []
    for i, (t, spec, pick) in enumerate(items):
        out.append(Query(i, float(t), np.asarray(pick, np.int32), np.asarray(spec.ret, np.float64),
                         np.asarray(spec.lim, np.float64), spec.occ_ret, spec.occ_lim, spec.agg_ret, spec.agg_lim))
    return out


def _build(pool: A.Pool, q: Query, stream) -> A.Layer:
    return pool.layer(q.elt_index, q.ret, q.lim, q.occ_ret, q.occ_lim, q.agg_ret, q.agg_lim, stream=stream)


@dataclass
class _InFlight:
    """A group on the run stream: its queries, YLT buffers, one completion
    event per query (the same event for every query of a batched pass),
    the result slot, and how many of its queries have been answered."""
    group: List[Query]
    outs: List[torch.Tensor]
    evs: List[torch.cuda.Event]
    slot: int
    per_query: bool
    next: int = 0


def _wait_until(clock, t):
    while True:
        d = t - clock()
        if d <= 0:
            return
        time.sleep(min(d, 0.0005) if d > 0.0002 else 0)


class BatchingServer:
    """Continuous-batching server over one YET and one ELT pool.  Its streams,
    batch objects and result buffers live as long as the server, so repeated
    runs pay no set-up.  A group of fewer than ``min_batch`` queries runs as
    single-layer passes, each query answered when its own pass is done
    (below the crossover that ``warm_up`` measures, a batched pass loses to
    separate ones)."""

    def __init__(self, yet: A.Yet, pool: A.Pool, return_periods=(100.0, 250.0), max_batch: int = L.ARA_MAX_BATCH,
                 min_batch: int = 2):
        self.yet, self.pool = yet, pool
        self.return_periods = tuple(return_periods)
        self.max_batch = int(max_batch)
        self.min_batch = int(min_batch)
        self.run_s = torch.cuda.Stream()
        self.build_s = torch.cuda.Stream()
        # two groups in flight at most; each holds a slot: a batch object and
        # the device and pinned host buffers of its PML/TVaR
        self.n_slots = 2
        n_rp = len(self.return_periods)
        self.batches = [None] * self.n_slots
        self.dev_risk = [torch.empty(2 * self.max_batch * n_rp, dtype=torch.float64, device="cuda")
                         for _ in range(self.n_slots)]
        self.host_risk = [torch.empty(2 * self.max_batch * n_rp, dtype=torch.float64, pin_memory=True)
                          for _ in range(self.n_slots)]
        self.ylt_bufs = [[] for _ in range(self.n_slots)]

    def warm_up(self, items, sizes=(2, 4, 8, 16, 32, 64)) -> int:
        """First-use work outside any timed run, and the crossover.

        Every group size from 2 to ``max_batch`` runs once on the first
        slot's batch, with the layers in arrival order and with the layers
        of most ELTs (so that both record forms occur), and the largest
        groups of each form run on every slot: the launch shapes of every
        layer count are tuned and each slot's device buffers have grown to
        their largest use before a query is timed.  The crossover -- the
        smallest group size for which one batched pass beats the
        single-layer passes of the same layers, measured at ``sizes`` --
        becomes ``min_batch`` and is returned.  ``items`` must hold at least
        ``max_batch`` queries."""
        yet, T = self.yet, self.yet.n_trials
        qs = make_queries(items)
        if len(qs) < self.max_batch:
            raise ValueError("warm-up needs at least max_batch queries")
        layers = [_build(self.pool, q, None) for q in qs[:self.max_batch]]
        torch.cuda.synchronize()
        most = sorted(range(len(layers)), key=lambda i: -len(qs[i].elt_index))
        outs = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in range(self.max_batch)]

        def run(slot, group):
            if self.batches[slot] is None:
                self.batches[slot] = A.Batch(yet, group)
            else:
                self.batches[slot].rebuild(group)
            self.batches[slot].run(outs[:len(group)])

        def timed(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / reps

        for n in range(2, self.max_batch + 1):
            run(0, layers[:n])
            run(0, [layers[i] for i in most[:n]])
        for slot in range(self.n_slots):
            for n in (min(16, self.max_batch), self.max_batch):
                run(slot, [layers[i] for i in most[:n]])
        # each layer's own single-layer pass: a group is compared with the
        # passes of the same layers, whose cost grows with their ELT counts
        t_single = [timed(lambda l=l: A.run_layer(yet, l, out=outs[0])) for l in layers]
        t_batch = {n: timed(lambda n=n: run(0, layers[:n])) for n in sizes if n <= self.max_batch}
        A.pml_tvar_many(outs, self.return_periods)
        torch.cuda.synchronize()
        for l in layers:
            l.close()
        cross = self.max_batch + 1
        for n in sorted(t_batch):
            if t_batch[n] < sum(t_single[:n]):
                cross = n  # the first measured size that wins
                break
        self.min_batch = min(cross, L.ARA_MAX_BATCH)
        return self.min_batch

    def close(self):
        for b in self.batches:
            if b is not None:
                b.close()
        self.batches = [None] * self.n_slots
        self.ylt_bufs = [[] for _ in range(self.n_slots)]

    def serve(self, queries: Sequence[Query], keep_ylt: bool = False, progress=None) -> dict:
        """Serve the queries at their arrival times; ``progress(n_done)`` (if
        given) is called each time another 200 answers are out."""
        yet, pool = self.yet, self.pool
        run_s, build_s = self.run_s, self.build_s
        rps = self.return_periods
        T = yet.n_trials
        pending = collections.deque(sorted(queries, key=lambda q: q.arrival))
        waiting: collections.deque = collections.deque()   # arrived, not admitted
        built: List[Query] = []                           # admitted, table being built / ready
        inflight: collections.deque = collections.deque()  # _InFlight, in launch order
        free_slots = list(range(self.n_slots))
        n_done = 0
        n_launches = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        reported = 0
        while n_done < len(queries):
            if progress is not None and n_done - reported >= 200:
                reported = n_done - n_done % 200
                progress(n_done)
            now = clock()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission: a query enters when a layer slot (its table memory) is free
            while waiting:
                q = waiting[0]
                try:
                    # with nothing on the run stream, build there (the pass
                    # then needs no wait on another stream's event)
                    q.layer = _build(pool, q, run_s if not inflight else build_s)
                except L.AraError as e:
                    if e.name == "ARA_ERR_OOM":
                        break
                    raise
                waiting.popleft()
                q.admitted = clock()
                built.append(q)
            # launch when the run stream has at most one group queued behind the running one
            if built and free_slots:
                group = built[:self.max_batch]
                del built[:self.max_batch]
                slot = free_slots.pop()
                n = len(group)
                if keep_ylt:
                    with torch.cuda.stream(run_s):
                        outs = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in group]
                else:
                    # the slot's own YLT buffers (a slot is reused only after
                    # its group has been answered)
                    bufs = self.ylt_bufs[slot]
                    while len(bufs) < n:
                        bufs.append(torch.empty(T, dtype=torch.float64, device="cuda"))
                    outs = bufs[:n]
                r = len(rps)
                dev, host = self.dev_risk[slot], self.host_risk[slot]
                if n < max(2, self.min_batch):
                    # below the crossover: single-layer passes, each query
                    # answered as soon as its own PML/TVaR is on the host
                    # (query i's [PML, TVaR] at [2 r i, 2 r (i + 1)))
                    evs = []
                    for i, (q, o) in enumerate(zip(group, outs)):
                        A.run_layer(yet, q.layer, out=o, stream=run_s)
                        a = 2 * r * i
                        A.pml_tvar_many_noalloc([o], rps, dev[a:a + r], dev[a + r:a + 2 * r], stream=run_s)
                        with torch.cuda.stream(run_s):
                            host[a:a + 2 * r].copy_(dev[a:a + 2 * r], non_blocking=True)
                            ev = torch.cuda.Event()
                            ev.record(run_s)
                        evs.append(ev)
                    per_query = True
                else:
                    layers = [q.layer for q in group]
                    if self.batches[slot] is None:
                        self.batches[slot] = A.Batch(yet, layers)
                    else:
                        self.batches[slot].rebuild(layers)
                    self.batches[slot].run(outs, stream=run_s)
                    # PML of the group, then its TVaR, in one piece of device
                    # memory: one copy brings both to the host
                    m = n * r
                    A.pml_tvar_many_noalloc(outs, rps, dev[:m], dev[m:2 * m], stream=run_s)
                    with torch.cuda.stream(run_s):
                        host[:2 * m].copy_(dev[:2 * m], non_blocking=True)
                        ev = torch.cuda.Event()
                        ev.record(run_s)
                    evs = [ev] * n
                    per_query = False
                inflight.append(_InFlight(group, outs, evs, slot, per_query))
                n_launches += n if per_query else 1
            # completion, in launch order
            if inflight and inflight[0].evs[inflight[0].next].query():
                g = inflight[0]
                t = clock()
                n, r = len(g.group), len(rps)
                host = self.host_risk[g.slot]
                while g.next < n and g.evs[g.next].query():
                    i = g.next
                    q = g.group[i]
                    if g.per_query:
                        res = host[2 * r * i:2 * r * (i + 1)].numpy().copy()
                        q.pml, q.tvar = res[:r], res[r:]
                    else:
                        q.pml = host[r * i:r * (i + 1)].numpy().copy()
                        q.tvar = host[n * r + r * i:n * r + r * (i + 1)].numpy().copy()
                    q.done = t
                    q.batch_size = 1 if g.per_query else n
                    q.ylt = g.outs[i] if keep_ylt else None
                    q.layer.close()
                    q.layer = None
                    g.next += 1
                    n_done += 1
                if g.next == n:
                    inflight.popleft()
                    free_slots.append(g.slot)
                continue
            if not inflight and not built and not waiting and pending:
                _wait_until(clock, pending[0].arrival)
        return _summary(queries, n_launches)


def serve_batched(yet: A.Yet, pool: A.Pool, queries: Sequence[Query], return_periods=(100.0, 250.0),
                  max_batch: int = L.ARA_MAX_BATCH, min_batch: int = 2, keep_ylt: bool = False,
                  progress=None) -> dict:
    """One run of a fresh BatchingServer."""
    srv = BatchingServer(yet, pool, return_periods, max_batch, min_batch)
    try:
        return srv.serve(queries, keep_ylt, progress)
    finally:
        srv.close()


def serve_one_at_a_time(yet: A.Yet, pool: A.Pool, queries: Sequence[Query], return_periods=(100.0, 250.0),
                        keep_ylt: bool = False, progress=None) -> dict:
    s = torch.cuda.Stream()
    T = yet.n_trials
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    for i, q in enumerate(sorted(queries, key=lambda q: q.arrival)):
        if progress is not None and i and i % 200 == 0:
            progress(i)
        _wait_until(clock, q.arrival)
        q.admitted = clock()
        lay = _build(pool, q, s)
        out = torch.empty(T, dtype=torch.float64, device="cuda")
        A.run_layer(yet, lay, out=out, stream=s)
        q.pml, q.tvar = (x[0] for x in A.pml_tvar_many([out], return_periods, stream=s))
        q.done = clock()
        q.batch_size = 1
        q.ylt = out if keep_ylt else None
        lay.close()
    return _summary(queries, len(queries))


def _pct(x: np.ndarray, p: float) -> float:
    """Nearest-rank percentile."""
    xs = np.sort(x)
    k = max(1, int(np.ceil(p / 100.0 * len(xs))))
    return float(xs[k - 1])


def _summary(queries: Sequence[Query], n_launches: int) -> dict:
    lat = np.array([q.latency for q in queries])
    span = max(q.done for q in queries) - min(q.arrival for q in queries)
    sizes = np.array([q.batch_size for q in queries])
    return {"n_queries": len(queries), "p50_ms": _pct(lat, 50) * 1e3, "p99_ms": _pct(lat, 99) * 1e3,
            "max_ms": float(lat.max()) * 1e3, "mean_ms": float(lat.mean()) * 1e3,
            "layers_per_s": len(queries) / span if span > 0 else float("inf"), "launches": n_launches,
            "mean_batch": float(sizes.mean())}
