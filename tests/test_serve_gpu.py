"""Serving: layers built on the GPU from a resident ELT pool, continuous
batching with admission by table memory, and answers that are the same alone
and in the mix."""
import numpy as np
import pytest
import torch

from gpu_cases import assert_close_to_oracle, assert_risk_close, oracle_run
from oracle import oracle
from paper_1412_4556_amd import _lib as L
from paper_1412_4556_amd import ara as A
from paper_1412_4556_amd import serve as S
from paper_1412_4556_amd import workloads as W

pytestmark = pytest.mark.gpu

RPS = (10.0, 25.0)


def _setup(T=4000, mean_len=150.0, C=30000, n_pool=40, seed=3):
    ids, off, _ = W.random_case(seed, T, mean_len, C, 1, 1, empty_frac=0.05)
    rng = np.random.default_rng(seed)
    pool = W.ElTPool([], [], None, None)
    rets, lims = [], []
    for j in range(n_pool):
        _, _, spec = W.random_case(seed * 100 + j, 1, 1.0, C, 1, int(rng.integers(500, 4000)))
        pool.ids.append(spec.elt_ids[0])
        pool.losses.append(spec.elt_losses[0])
        rets.append(spec.ret[0])
        lims.append(spec.lim[0])
    pool.ret, pool.lim = np.array(rets), np.array(lims)
    return ids, off, pool


def _queries(pool, n, rate, seed=0):
    rng = np.random.default_rng(seed)
    items, t = [], 0.0
    for q in range(n):
        t += rng.exponential(1.0 / rate)
        J = int(rng.integers(1, 9))
        pick = rng.choice(len(pool.ids), size=J, replace=False).astype(np.int32)
        _, _, r2, l2, r3, l3 = W.random_layer_terms(rng, [pool.losses[p] for p in pick])
        spec = W.LayerSpec([pool.ids[p] for p in pick], [pool.losses[p] for p in pick], pool.ret[pick].copy(),
                           pool.lim[pick].copy(), r2 * 0.01, l2 * 0.01, r3 * 0.01, l3 * 0.01)
        items.append((t, spec, pick))
    return items


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_pool_layer_equals_host_layer(prec):
    ids, off, pool = _setup()
    T, C = len(off) - 1, 30000
    yet = A.yet_from_numpy(ids, off, T, C)
    P = A.Pool(yet, pool.ids, pool.losses, prec, max_layers=4)
    s = torch.cuda.Stream()
    for t, spec, pick in _queries(pool, 6, 100.0, seed=1):
        lay_p = P.layer(pick, spec.ret, spec.lim, spec.occ_ret, spec.occ_lim, spec.agg_ret, spec.agg_lim, stream=s)
        lay_h = A.Layer(yet, spec, prec, "fused")
        y_p = A.run_layer(yet, lay_p).cpu().numpy()  # waits for the build on s
        y_h = A.run_layer(yet, lay_h).cpu().numpy()
        assert np.array_equal(y_p, y_h)
        lay_p.close()
        lay_h.close()
    assert P.free_slots == 4


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_pool_layer_repeated_and_empty_elts(prec):
    """A pool layer may name one pool ELT several times and may hold an
    empty ELT: its table gives bitwise the YLT of the host-built layer with
    the same ELT list, within tolerance of the oracle."""
    ids, off, pool = _setup(T=1500)
    T, C = len(off) - 1, 30000
    e_ids = list(pool.ids) + [np.zeros(0, np.int32)]
    e_loss = list(pool.losses) + [np.zeros(0)]
    empty = len(e_ids) - 1
    yet = A.yet_from_numpy(ids, off, T, C)
    P = A.Pool(yet, e_ids, e_loss, prec, max_layers=2)
    pick = np.array([3, 7, 3, empty, 7, 0], np.int32)
    ret = np.array([pool.ret[i] if i != empty else 0.0 for i in pick])
    lim = np.array([pool.lim[i] if i != empty else np.inf for i in pick])
    terms = (50.0, 1e6, 100.0, 1e8)
    spec = W.LayerSpec([e_ids[i] for i in pick], [e_loss[i] for i in pick], ret, lim, *terms)
    lp = P.layer(pick, ret, lim, *terms)
    y_p = A.run_layer(yet, lp).cpu().numpy()
    lh = A.Layer(yet, spec, prec, "fused")
    y_h = A.run_layer(yet, lh).cpu().numpy()
    assert np.array_equal(y_p, y_h)
    assert (y_p > 0).mean() > 0.05
    assert_close_to_oracle(y_p, oracle_run(ids, off, T, C, 0, spec), prec)
    lp.close()
    lh.close()
    assert P.free_slots == 2


def test_pool_admission_limit():
    ids, off, pool = _setup(T=500)
    yet = A.yet_from_numpy(ids, off, 500, 30000)
    P = A.Pool(yet, pool.ids, pool.losses, "fp64", max_layers=2)
    a = P.layer([0, 1], pool.ret[:2], pool.lim[:2], 0, np.inf, 0, np.inf)
    b = P.layer([2], pool.ret[2:3], pool.lim[2:3], 0, np.inf, 0, np.inf)
    with pytest.raises(L.AraError) as ei:
        P.layer([3], pool.ret[3:4], pool.lim[3:4], 0, np.inf, 0, np.inf)
    assert ei.value.name == "ARA_ERR_OOM"
    assert P.free_slots == 0
    a.close()
    c = P.layer([3], pool.ret[3:4], pool.lim[3:4], 0, np.inf, 0, np.inf)
    assert P.free_slots == 0
    with pytest.raises(L.AraError):
        P.layer([99], pool.ret[:1], pool.lim[:1], 0, np.inf, 0, np.inf)  # index outside the pool
    b.close()
    c.close()
    assert P.free_slots == 2


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("max_layers", [3, 64])
def test_served_answers_same_alone_and_in_mix(prec, max_layers):
    ids, off, pool = _setup()
    T, C = len(off) - 1, 30000
    yet = A.yet_from_numpy(ids, off, T, C)
    P = A.Pool(yet, pool.ids, pool.losses, prec, max_layers=max_layers)
    items = _queries(pool, 80, 5000.0, seed=2)  # fast arrivals: batches form
    qs = S.make_queries(items)
    summ = S.serve_batched(yet, P, qs, RPS, keep_ylt=True, min_batch=2 if max_layers == 64 else 3)
    torch.cuda.synchronize()
    assert summ["n_queries"] == 80 and all(q.done >= q.arrival for q in qs)
    assert max(q.batch_size for q in qs) <= max_layers
    if max_layers == 64:
        assert summ["mean_batch"] > 1.5  # queries really were batched
    alone = S.make_queries(items)
    S.serve_one_at_a_time(yet, P, alone, RPS, keep_ylt=True)
    torch.cuda.synchronize()
    for q, a in zip(qs, alone):
        assert torch.equal(q.ylt, a.ylt), q.qid
        assert np.array_equal(q.pml, a.pml) and np.array_equal(q.tvar, a.tvar)
    assert P.free_slots == max_layers
    # the answers are those of the oracle
    for q in qs[:3]:
        spec = items[q.qid][1]
        ref = oracle_run(ids, off, T, C, 0, spec)
        assert_close_to_oracle(q.ylt.cpu().numpy(), ref, prec)
        rp, rt = oracle.pml_tvar(ref["ylt"], RPS)
        assert_risk_close(q.pml, q.tvar, rp, rt, prec, ref)


def test_warmed_server_answers_same_alone_and_in_mix():
    """A server whose warm-up ran every group size (growing its batches'
    buffers, tuning their launch shapes) and chose its crossover still
    answers each query as the one-at-a-time server does."""
    ids, off, pool = _setup()
    T, C = len(off) - 1, 30000
    yet = A.yet_from_numpy(ids, off, T, C)
    P = A.Pool(yet, pool.ids, pool.losses, "fp64", max_layers=24)
    srv = S.BatchingServer(yet, P, RPS, max_batch=8)
    warm = _queries(pool, 8, 1e6, seed=5)
    mb = srv.warm_up(warm, sizes=(2, 4, 8))
    assert mb == srv.min_batch and 2 <= mb <= 9
    assert P.free_slots == 24
    items = _queries(pool, 60, 3000.0, seed=6)
    qs = S.make_queries(items)
    srv.serve(qs, keep_ylt=True)
    torch.cuda.synchronize()
    srv.close()
    alone = S.make_queries(items)
    S.serve_one_at_a_time(yet, P, alone, RPS, keep_ylt=True)
    torch.cuda.synchronize()
    for q, a in zip(qs, alone):
        assert torch.equal(q.ylt, a.ylt), q.qid
        assert np.array_equal(q.pml, a.pml) and np.array_equal(q.tvar, a.tvar)
    assert P.free_slots == 24


def test_pml_tvar_many_matches_single():
    rng = np.random.default_rng(0)
    ys = [torch.from_numpy(rng.lognormal(5, 2, 5000) * (rng.uniform(size=5000) < 0.5)).cuda() for _ in range(20)]
    pm, tv = A.pml_tvar_many(ys, [2, 10, 100])
    for i, y in enumerate(ys):
        p1, t1 = A.pml_tvar(y, [2, 10, 100])
        assert np.array_equal(pm[i], p1) and np.array_equal(tv[i], t1)
        op, ot = oracle.pml_tvar(y.cpu().numpy(), [2, 10, 100])
        assert np.array_equal(p1, op) and np.allclose(t1, ot, rtol=1e-12, atol=0)
