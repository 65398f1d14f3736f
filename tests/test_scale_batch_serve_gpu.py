"""The batching and serving workloads at full size, in the configurations the
benchmark times, checked against the oracle on sampled trials (regenerated on
the host from the same seeded blocks) and against single-layer passes."""
import numpy as np
import pytest
import torch

from gpu_cases import TOL, assert_close_to_oracle, oracle_run
from oracle import oracle
from paper_1412_4556_amd import ara as A
from paper_1412_4556_amd import serve as S
from paper_1412_4556_amd import workloads as W

pytestmark = pytest.mark.gpu

N_SAMPLE = 120


def _sample(spec, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, spec.n_trials - 1], rng.choice(spec.n_trials, N_SAMPLE, replace=False)]))


def test_batch_workload_full_size():
    wl = W.batch_layers()
    ids, off = W.yet_full(wl.yet)
    yet = A.Yet(torch.from_numpy(ids).cuda(), torch.from_numpy(off).cuda(), wl.yet.n_trials, wl.yet.catalog_size)
    del ids
    layers = [A.Layer(yet, s, "fp64", "fused") for s in wl.layers]
    batch = A.Batch(yet, layers)
    outs = batch.run()
    torch.cuda.synchronize()
    for l, lay in enumerate(layers):
        assert torch.equal(outs[l], A.run_layer(yet, lay)), l
    sample = _sample(wl.yet, 7)
    sub_ids, sub_off = W.yet_subset(wl.yet, sample, off)
    for l, spec in enumerate(wl.layers):
        ref = oracle_run(sub_ids, sub_off, len(sample), wl.yet.catalog_size, 0, spec)
        assert_close_to_oracle(outs[l][torch.from_numpy(sample).cuda()].cpu().numpy(), ref, "fp64")
    pml, tvar = A.pml_tvar_many(outs, wl.return_periods)
    for l in (0, 31, 63):
        op, ot = oracle.pml_tvar(outs[l].cpu().numpy(), wl.return_periods)
        assert np.array_equal(pml[l], op) and np.allclose(tvar[l], ot, rtol=1e-12, atol=0)


def test_serving_workload_full_size():
    y, pool = W.serving_pool()
    ids, off = W.yet_full(y)
    yet = A.Yet(torch.from_numpy(ids).cuda(), torch.from_numpy(off).cuda(), y.n_trials, y.catalog_size)
    del ids
    P = A.Pool(yet, pool.ids, pool.losses, "fp64", max_layers=64)
    items = W.serving_queries(pool, 40, 3000.0, stream=17)
    qs = S.make_queries(items)
    srv = S.BatchingServer(yet, P, min_batch=4)
    summ = srv.serve(qs, keep_ylt=True)
    torch.cuda.synchronize()
    srv.close()
    assert summ["n_queries"] == 40
    sample = _sample(y, 11)
    sub_ids, sub_off = W.yet_subset(y, sample, off)
    idx = torch.from_numpy(sample).cuda()
    for q, (t, spec, pick) in zip(qs, items):
        ref = oracle_run(sub_ids, sub_off, len(sample), y.catalog_size, 0, spec)
        assert_close_to_oracle(q.ylt[idx].cpu().numpy(), ref, "fp64")
        op, ot = oracle.pml_tvar(q.ylt.cpu().numpy(), (100.0, 250.0))
        assert np.array_equal(q.pml, op) and np.allclose(q.tvar, ot, rtol=1e-12, atol=0)
