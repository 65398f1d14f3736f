"""Seeded synthetic inputs for the Aggregate Risk Analysis trial pass.

This module only draws random inputs: Year Event Tables (YET), Event Loss
Tables (ELT) and financial terms. It holds none of the analysis arithmetic,
so that both the GPU path and the CPU oracle can be fed the very same inputs.

Shapes follow the paper's data model (Section III, the YET / ELT / Layer
definitions) and its experimental workload (Section IV: one million trials of
about one thousand events, one layer of sixteen ELTs of 10,000-30,000 event
losses).  The paper's own data are industry data that are not public; these
generators stand in for them.

Every stream is a ``numpy.random.PCG64`` seeded from
``SeedSequence(ROOT_SEED, spawn_key=(workload, component, ...))``.  YET event
IDs are drawn in blocks of ``TRIAL_BLOCK`` trials, each block from its own
stream, so any subset of trials of a full-size YET can be regenerated on the
host without materialising the whole table.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

ROOT_SEED = 14124556
TRIAL_BLOCK = 1 << 16

# component tags of the spawn keys
_C_YET_IDS, _C_YET_LEN, _C_ELTS, _C_TERMS, _C_QUERIES, _C_ARRIVALS = range(6)

# workload indices (first element of every spawn key)
W_PLAIN_TINY = 0
W_PLAIN_PAPER = 1
W_PRECISION = 2
W_BATCH = 3
W_SERVING = 4


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=tuple(key))))


# --------------------------------------------------------------------------- YET
@dataclass(frozen=True)
class YetSpec:
    """A synthetic YET: ``n_trials`` trials of event IDs uniform over the catalogue.

    ``fixed_len`` gives every trial the same number of events (no offsets
    array); otherwise trial lengths are Poisson(``poisson_mean``) and the YET
    carries an int64 offsets array of ``n_trials + 1`` entries.
    """

    workload: int
    n_trials: int
    catalog_size: int
    fixed_len: Optional[int] = None
    poisson_mean: Optional[float] = None

    @property
    def n_blocks(self) -> int:
        return (self.n_trials + TRIAL_BLOCK - 1) // TRIAL_BLOCK


def yet_lengths(spec: YetSpec) -> np.ndarray:
    """Events per trial (int64 [n_trials])."""
    if spec.fixed_len is not None:
        return np.full(spec.n_trials, spec.fixed_len, dtype=np.int64)
    rng = _rng(spec.workload, _C_YET_LEN)
    return rng.poisson(spec.poisson_mean, size=spec.n_trials).astype(np.int64)


def yet_offsets(spec: YetSpec) -> np.ndarray:
    """int64 [n_trials + 1] offsets of each trial into the flat event-ID array."""
    off = np.zeros(spec.n_trials + 1, dtype=np.int64)
    np.cumsum(yet_lengths(spec), out=off[1:])
    return off


def _block_ids(spec: YetSpec, b: int, n_events: int) -> np.ndarray:
    rng = _rng(spec.workload, _C_YET_IDS, b)
    return rng.integers(0, spec.catalog_size, size=n_events, dtype=np.int32)


def yet_full(spec: YetSpec, offsets: Optional[np.ndarray] = None):
    """Whole YET: (int32 ids [n_events], int64 offsets [T+1] or None)."""
    off = yet_offsets(spec) if offsets is None else offsets
    ids = np.empty(int(off[-1]), dtype=np.int32)
    for b in range(spec.n_blocks):
        t0, t1 = b * TRIAL_BLOCK, min((b + 1) * TRIAL_BLOCK, spec.n_trials)
        lo, hi = int(off[t0]), int(off[t1])
        ids[lo:hi] = _block_ids(spec, b, hi - lo)
    return ids, (None if spec.fixed_len is not None else off)


def yet_subset(spec: YetSpec, trials: Sequence[int], offsets: Optional[np.ndarray] = None):
    """Regenerate only the given trials: (ids, offsets [len(trials)+1]).

    The result is the sub-YET made of those trials, in the order given.
    """
    off = yet_offsets(spec) if offsets is None else offsets
    trials = np.asarray(trials, dtype=np.int64)
    pieces = []
    cache = {}
    for t in trials:
        b = int(t) // TRIAL_BLOCK
        if b not in cache:
            t0, t1 = b * TRIAL_BLOCK, min((b + 1) * TRIAL_BLOCK, spec.n_trials)
            lo, hi = int(off[t0]), int(off[t1])
            cache[b] = (lo, _block_ids(spec, b, hi - lo))
        lo, blk = cache[b]
        pieces.append(blk[int(off[t]) - lo:int(off[t + 1]) - lo])
    sub_off = np.zeros(len(trials) + 1, dtype=np.int64)
    np.cumsum([len(p) for p in pieces], out=sub_off[1:])
    ids = np.concatenate(pieces) if pieces else np.zeros(0, dtype=np.int32)
    return ids.astype(np.int32, copy=False), sub_off


# --------------------------------------------------------------------------- layers
@dataclass
class LayerSpec:
    """One layer: ELTs (event IDs + losses) with per-ELT terms, plus the
    occurrence and aggregate terms of the layer (Section III)."""

    elt_ids: List[np.ndarray]
    elt_losses: List[np.ndarray]
    ret: np.ndarray  # per-ELT retention (float64 [J])
    lim: np.ndarray  # per-ELT limit (float64 [J]; +inf allowed)
    occ_ret: float
    occ_lim: float
    agg_ret: float
    agg_lim: float
    name: str = ""

    @property
    def n_elts(self) -> int:
        return len(self.elt_ids)

    def concat(self):
        """Flat (ids int32, losses float64, sizes int64) over the ELTs in layer order."""
        sizes = np.array([len(a) for a in self.elt_ids], dtype=np.int64)
        ids = np.concatenate(self.elt_ids).astype(np.int32) if len(self.elt_ids) else np.zeros(0, np.int32)
        loss = np.concatenate(self.elt_losses).astype(np.float64) if len(self.elt_ids) else np.zeros(0)
        return ids, loss, sizes

    def with_terms(self, **kw) -> "LayerSpec":
        d = dict(ret=self.ret.copy(), lim=self.lim.copy(), occ_ret=self.occ_ret, occ_lim=self.occ_lim,
                 agg_ret=self.agg_ret, agg_lim=self.agg_lim)
        d.update(kw)
        return LayerSpec(list(self.elt_ids), list(self.elt_losses), np.asarray(d["ret"], np.float64),
                         np.asarray(d["lim"], np.float64), float(d["occ_ret"]), float(d["occ_lim"]),
                         float(d["agg_ret"]), float(d["agg_lim"]), self.name)

    def open_terms(self) -> "LayerSpec":
        """Zero retentions, infinite limits everywhere."""
        J = self.n_elts
        return self.with_terms(ret=np.zeros(J), lim=np.full(J, np.inf), occ_ret=0.0, occ_lim=np.inf,
                               agg_ret=0.0, agg_lim=np.inf)


def _elt(rng: np.random.Generator, catalog: int, size: int, loss: str):
    ids = rng.choice(catalog, size=size, replace=False).astype(np.int32)
    if loss == "lognormal":
        losses = rng.lognormal(10.0, 2.0, size=size)
    elif loss == "pareto":  # classic Pareto(alpha=1.5, x_m=1e4); numpy's pareto() is the Lomax form
        losses = 1e4 * (1.0 + rng.pareto(1.5, size=size))
    else:
        raise ValueError(loss)
    return ids, losses


def _pct_terms(losses: np.ndarray):
    r, u = np.percentile(losses, [10, 90])
    return float(r), float(u)


def layer_percentile_rule(workload: int, catalog: int, n_elts: int, elt_size: int, loss: str = "lognormal",
                          occ=(1e5, 1e7), agg=(1e6, 5e7), name: str = "") -> LayerSpec:
    """Layer whose per-ELT retention/limit are the 10th/90th percentiles of that
    ELT's losses, with fixed occurrence and aggregate terms."""
    rng = _rng(workload, _C_ELTS)
    ids, losses, ret, lim = [], [], [], []
    for _ in range(n_elts):
        i, l = _elt(rng, catalog, elt_size, loss)
        r, u = _pct_terms(l)
        ids.append(i); losses.append(l); ret.append(r); lim.append(u)
    return LayerSpec(ids, losses, np.array(ret), np.array(lim), occ[0], occ[1], agg[0], agg[1], name)


def _logu(rng, lo, hi):
    return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))


def random_layer_terms(rng: np.random.Generator, losses: Sequence[np.ndarray]):
    """Per-layer random terms: per-ELT retention/limit at U(0,0.2) / U(0.8,1.0)
    quantiles of the ELT's losses (limit infinite with probability 1/4);
    occurrence retention/limit log-uniform on [1e4,1e6] / [1e6,1e8]; aggregate
    retention/limit log-uniform on [1e5,1e7] / [1e7,1e9]."""
    ret, lim = [], []
    for l in losses:
        ret.append(float(np.quantile(l, rng.uniform(0.0, 0.2))))
        u = float(np.quantile(l, rng.uniform(0.8, 1.0)))
        lim.append(np.inf if rng.uniform() < 0.25 else u)
    return (np.array(ret), np.array(lim), _logu(rng, 1e4, 1e6), _logu(rng, 1e6, 1e8),
            _logu(rng, 1e5, 1e7), _logu(rng, 1e7, 1e9))


# --------------------------------------------------------------------------- named workloads
@dataclass
class Workload:
    name: str
    yet: YetSpec
    layers: List[LayerSpec] = field(default_factory=list)
    return_periods: tuple = (100.0, 250.0)


def plain_tiny() -> Workload:
    """10,000 trials x 1,000 events over a 100,000-event catalogue; one layer of
    4 ELTs x 10,000 events, lognormal(10, 2) losses."""
    y = YetSpec(W_PLAIN_TINY, 10_000, 100_000, fixed_len=1000)
    return Workload("plain_fp64_10k_trials_4_elts", y,
                    [layer_percentile_rule(W_PLAIN_TINY, 100_000, 4, 10_000, name="tiny_4elt")])


def plain_paper(n_trials: int = 1_000_000) -> Workload:
    """The paper's workload shape: 1,000,000 trials x 1,000 events over a
    2,000,000-event catalogue; one layer of 16 ELTs x 20,000 events."""
    y = YetSpec(W_PLAIN_PAPER, n_trials, 2_000_000, fixed_len=1000)
    return Workload("plain_1M_trials_x_1000_events_16_elts", y,
                    [layer_percentile_rule(W_PLAIN_PAPER, 2_000_000, 16, 20_000, name="paper_16elt")])


def precision_poisson() -> Workload:
    """10,000 trials with Poisson(1000) events over 100,000 events; 4 ELTs x
    10,000 of Pareto(1.5, 1e4) losses.  Two term sets: per-ELT limits removed
    (the 90th-percentile cap would keep every trial under the aggregate
    retention) and all terms open."""
    y = YetSpec(W_PRECISION, 10_000, 100_000, poisson_mean=1000.0)
    base = layer_percentile_rule(W_PRECISION, 100_000, 4, 10_000, loss="pareto", name="pareto_4elt")
    capped = base.with_terms(lim=np.full(4, np.inf))
    capped.name = "pareto_uncapped_elt"
    opened = base.open_terms()
    opened.name = "pareto_open_terms"
    return Workload("precision_poisson_pareto_10k_trials", y, [capped, opened])


def batch_layers(n_trials: int = 1_000_000, n_layers: int = 64) -> Workload:
    """One YET of Poisson(1000)-length trials over 2,000,000 events and
    ``n_layers`` layers with 1..32 ELTs each (5,000-50,000 events per ELT,
    lognormal losses, random terms)."""
    y = YetSpec(W_BATCH, n_trials, 2_000_000, poisson_mean=1000.0)
    rng = _rng(W_BATCH, _C_ELTS)
    trng = _rng(W_BATCH, _C_TERMS)
    layers = []
    for li in range(n_layers):
        J = int(rng.integers(1, 33))
        ids, losses = [], []
        for _ in range(J):
            i, l = _elt(rng, y.catalog_size, int(rng.integers(5_000, 50_001)), "lognormal")
            ids.append(i); losses.append(l)
        r, u, r2, l2, r3, l3 = random_layer_terms(trng, losses)
        layers.append(LayerSpec(ids, losses, r, u, r2, l2, r3, l3, name=f"batch_{li}"))
    return Workload(f"batch_{n_layers}_layers_{n_trials}_trials", y, layers)


@dataclass
class ElTPool:
    ids: List[np.ndarray]
    losses: List[np.ndarray]
    ret: np.ndarray
    lim: np.ndarray


def serving_pool(n_trials: int = 500_000, pool_size: int = 256):
    """Serving workload: a YET of Poisson(1000)-length trials over 2,000,000
    events and a pool of pre-loaded ELTs (5,000-50,000 events, lognormal
    losses, 10th/90th-percentile per-ELT terms)."""
    y = YetSpec(W_SERVING, n_trials, 2_000_000, poisson_mean=1000.0)
    rng = _rng(W_SERVING, _C_ELTS)
    ids, losses, ret, lim = [], [], [], []
    for _ in range(pool_size):
        i, l = _elt(rng, y.catalog_size, int(rng.integers(5_000, 50_001)), "lognormal")
        r, u = _pct_terms(l)
        ids.append(i); losses.append(l); ret.append(r); lim.append(u)
    return y, ElTPool(ids, losses, np.array(ret), np.array(lim))


def serving_queries(pool: ElTPool, n_queries: int, rate_per_s: float, stream: int = 0):
    """Open-loop Poisson arrivals of ad hoc layer queries.

    Returns a list of (arrival_time_s, LayerSpec, pool indices); each query covers 1..16 ELTs
    drawn without replacement from the pool, with random occurrence and
    aggregate terms drawn as in the batching workload.
    """
    qrng = _rng(W_SERVING, _C_QUERIES, stream)
    arng = _rng(W_SERVING, _C_ARRIVALS, stream, int(rate_per_s * 1000))
    t = np.cumsum(arng.exponential(1.0 / rate_per_s, size=n_queries))
    out = []
    P = len(pool.ids)
    for q in range(n_queries):
        J = int(qrng.integers(1, 17))
        pick = qrng.choice(P, size=J, replace=False)
        _, _, r2, l2, r3, l3 = random_layer_terms(qrng, [pool.losses[p] for p in pick])
        out.append((float(t[q]), LayerSpec([pool.ids[p] for p in pick], [pool.losses[p] for p in pick],
                                           pool.ret[pick].copy(), pool.lim[pick].copy(), r2, l2, r3, l3,
                                           name=f"query_{q}"), pick.astype(np.int32)))
    return out


# --------------------------------------------------------------------------- small random cases for tests
def random_case(seed: int, n_trials: int, mean_len: float, catalog: int, n_elts: int, elt_size: int,
                integer_losses: bool = False, max_int_loss: int = 100, terms: str = "random",
                fixed_len: bool = False, empty_frac: float = 0.0):
    """A small seeded random case: (ids, offsets, LayerSpec).

    ``terms``: "random" (quantile-based per-ELT terms and moderate layer
    terms), "open" (no retentions, infinite limits) or "counting" (open
    per-ELT terms and occurrence limit 1).
    With ``integer_losses`` every loss and term is a small integer, so every
    sum in the pass is exact in both float32 and float64.
    """
    rng = np.random.default_rng(seed)
    if fixed_len:
        lens = np.full(n_trials, int(mean_len), dtype=np.int64)
    else:
        lens = rng.poisson(mean_len, size=n_trials).astype(np.int64)
    if empty_frac > 0:
        lens[rng.uniform(size=n_trials) < empty_frac] = 0
    off = np.zeros(n_trials + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    ids = rng.integers(0, catalog, size=int(off[-1]), dtype=np.int32)
    eids, elos = [], []
    for _ in range(n_elts):
        sz = min(elt_size, catalog)
        eids.append(rng.choice(catalog, size=sz, replace=False).astype(np.int32))
        if integer_losses:
            elos.append(rng.integers(1, max_int_loss + 1, size=sz).astype(np.float64))
        else:
            elos.append(rng.lognormal(8.0, 2.0, size=sz))
    J = n_elts
    if terms == "open":
        lay = LayerSpec(eids, elos, np.zeros(J), np.full(J, np.inf), 0.0, np.inf, 0.0, np.inf)
    elif terms == "counting":
        lay = LayerSpec(eids, elos, np.zeros(J), np.full(J, np.inf), 0.0, 1.0, 0.0, np.inf)
    elif integer_losses:
        ret = rng.integers(0, max_int_loss // 4 + 1, size=J).astype(np.float64)
        lim = rng.integers(max_int_loss // 2, max_int_loss + 1, size=J).astype(np.float64)
        m = float(max_int_loss)
        lay = LayerSpec(eids, elos, ret, lim, float(rng.integers(0, int(m) + 1)), float(rng.integers(int(m), int(3 * m) + 1)),
                        float(rng.integers(0, int(mean_len * m / 4) + 1)), float(rng.integers(int(mean_len * m / 4) + 1, int(mean_len * m) + 2)))
    else:
        ret = np.array([np.quantile(l, rng.uniform(0, 0.3)) for l in elos])
        lim = np.array([np.quantile(l, rng.uniform(0.7, 1.0)) for l in elos])
        scale = float(np.median(np.concatenate(elos))) if elos else 1.0
        lay = LayerSpec(eids, elos, ret, lim, scale * rng.uniform(0, 2), scale * rng.uniform(5, 50),
                        scale * mean_len * rng.uniform(0.0, 0.2), scale * mean_len * rng.uniform(0.5, 3.0))
    return ids, off, lay
