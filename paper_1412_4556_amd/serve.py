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
  one batched pass (dense records for up to 16 layers, sparse records above),
  or a single-layer pass for a group of one, followed on the same stream by
  PML/TVaR of the whole group into device memory (the entry point that
  allocates nothing) and a copy of the results into pinned host memory.  The
  host loop never waits for the device: it keeps admitting and building
  arrivals and answers a group when its event has fired.
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
    back-to-back single-layer passes (below the crossover that ``warm_up``
    measures, a batched pass loses to separate ones)."""

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
        inflight: collections.deque = collections.deque()  # (queries, outs, event, slot)
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
                if n < max(2, self.min_batch):
                    for q, o in zip(group, outs):
                        A.run_layer(yet, q.layer, out=o, stream=run_s)
                else:
                    layers = [q.layer for q in group]
                    if self.batches[slot] is None:
                        self.batches[slot] = A.Batch(yet, layers)
                    else:
                        self.batches[slot].rebuild(layers)
                    self.batches[slot].run(outs, stream=run_s)
                # PML of the group, then its TVaR, in one piece of device
                # memory: one copy brings both to the host
                m = n * len(rps)
                dev, host = self.dev_risk[slot], self.host_risk[slot]
                A.pml_tvar_many_noalloc(outs, rps, dev[:m], dev[m:2 * m], stream=run_s)
                with torch.cuda.stream(run_s):
                    host[:2 * m].copy_(dev[:2 * m], non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(run_s)
                inflight.append((group, outs, ev, slot))
                n_launches += 1
            # completion, in launch order
            if inflight and inflight[0][2].query():
                group, outs, ev, slot = inflight.popleft()
                t = clock()
                n, r = len(group), len(rps)
                res = self.host_risk[slot][:2 * n * r].numpy().reshape(2, n, r).copy()
                for i, q in enumerate(group):
                    q.done = t
                    q.batch_size = len(group)
                    q.pml, q.tvar = res[0, i], res[1, i]
                    q.ylt = outs[i] if keep_ylt else None
                    q.layer.close()
                    q.layer = None
                free_slots.append(slot)
                n_done += len(group)
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


def warm_up(yet: A.Yet, pool: A.Pool, items, sizes=(2, 4, 8, 16, 32, 64)) -> int:
    """First-use work outside any timed run (the batch launch shape of every
    power-of-two batch size, tuned once per process; allocator growth), and
    the crossover: the smallest group for which one record pass beats the
    same number of single-layer passes.  Returns that group size."""
    qs = make_queries(items[:max(sizes)])
    layers = [_build(pool, q, None) for q in qs]
    torch.cuda.synchronize()
    T = yet.n_trials

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

    one = torch.empty(T, dtype=torch.float64, device="cuda")
    t_single = timed(lambda: A.run_layer(yet, layers[0], out=one))
    b = None
    t_batch = {}
    for n in sizes:
        if n > len(layers):
            break
        outs = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in range(n)]
        if b is None:
            b = A.Batch(yet, layers[:n])
        else:
            b.rebuild(layers[:n])
        t_batch[n] = timed(lambda: b.run(outs))
        A.pml_tvar_many(outs, (100.0, 250.0))
    torch.cuda.synchronize()
    if b is not None:
        b.close()
    for l in layers:
        l.close()
    cross = max(sizes) + 1
    for n in sorted(t_batch):
        if t_batch[n] < n * t_single:
            # first measured size that wins; interpolate down to the exact crossover
            cross = max(2, min(n, int(np.ceil(t_batch[n] / t_single))))
            break
    return min(cross, L.ARA_MAX_BATCH)


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
