"""Calls from several host threads at once (the library's calls release the
interpreter lock, so they really overlap): layers built from host ELTs in
every layout and precision and from one shared pool, passes on each thread's
own stream, a batch per thread, and PML/TVaR give bitwise the results of the
same calls made one after another."""
import threading

import numpy as np
import pytest
import torch

from paper_1412_4556_amd import ara as A
from paper_1412_4556_amd import workloads as W

pytestmark = pytest.mark.gpu

RPS = (10.0, 50.0)
N_THREADS = 6
C = 40000


def _yet():
    ids, off, _ = W.random_case(11, 6000, 200.0, C, 1, 1, empty_frac=0.02)
    return A.yet_from_numpy(ids, off, len(off) - 1, C), len(off) - 1


def _run_all(jobs, n_jobs):
    """Results of job(k) for every k, from N_THREADS threads."""
    res, errs = [None] * n_jobs, []

    def worker(t):
        try:
            for k in range(t, n_jobs, N_THREADS):
                res[k] = jobs(k)
        except Exception as e:  # reported by the test thread
            errs.append(e)

    ths = [threading.Thread(target=worker, args=(t,)) for t in range(N_THREADS)]
    for t in ths:
        t.start()
    for t in ths:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in ths), "a worker thread did not finish"
    assert not errs, errs
    return res


def test_host_layers_from_many_threads():
    yet, T = _yet()
    specs = [W.random_case(500 + k, 1, 1.0, C, 1 + k % 5, 3000)[2] for k in range(4 * N_THREADS)]
    layouts, precs = ["fused", "compact", "direct", "sparse"], ["fp64", "fp32c"]

    def job(k):
        lay = A.Layer(yet, specs[k], precs[(k // 4) % 2], layouts[k % 4])
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            y = torch.empty(T, dtype=torch.float64, device="cuda")
        A.run_layer(yet, lay, out=y, stream=s)
        pml, tvar = A.pml_tvar(y, RPS, stream=s)
        s.synchronize()
        lay.close()
        return y, pml, tvar

    seq = [job(k) for k in range(len(specs))]
    par = _run_all(job, len(specs))
    for k, (a, b) in enumerate(zip(par, seq)):
        assert torch.equal(a[0], b[0]), k
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]), k
    assert any(bool((b[0] > 0).any()) for b in seq)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_pool_layers_and_batches_from_many_threads(prec):
    yet, T = _yet()
    elts = [W.random_case(700 + j, 1, 1.0, C, 1, 1500 + 250 * j)[2] for j in range(16)]
    P = A.Pool(yet, [e.elt_ids[0] for e in elts], [e.elt_losses[0] for e in elts], prec, max_layers=3 * N_THREADS)
    rng = np.random.default_rng(5)
    queries = []
    for k in range(3 * N_THREADS):
        pick = rng.choice(16, size=int(rng.integers(1, 6)), replace=False).astype(np.int32)
        ret = np.array([elts[p].ret[0] for p in pick])
        lim = np.array([elts[p].lim[0] for p in pick])
        queries.append((pick, ret, lim, 50.0 * k, 1e7, 100.0 * k, 5e7))

    def job(t):
        # three pool layers per thread, run as one batch and one by one
        s = torch.cuda.Stream()
        qs = queries[3 * t:3 * t + 3]
        layers = [P.layer(q[0], q[1], q[2], *q[3:], stream=s) for q in qs]
        with torch.cuda.stream(s):
            ys = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in layers]
            bs = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in layers]
        for lay, y in zip(layers, ys):
            A.run_layer(yet, lay, out=y, stream=s)
        b = A.Batch(yet, layers)
        b.run(bs, stream=s)
        pml, tvar = A.pml_tvar_many(ys, RPS, stream=s)
        s.synchronize()
        b.close()
        for lay in layers:
            lay.close()
        return ys, bs, pml, tvar

    seq = [job(t) for t in range(N_THREADS)]
    assert P.free_slots == 3 * N_THREADS
    par = _run_all(job, N_THREADS)
    assert P.free_slots == 3 * N_THREADS
    for t in range(N_THREADS):
        ys, bs, pml, tvar = par[t]
        for i in range(3):
            assert torch.equal(ys[i], seq[t][0][i]), (t, i)
            assert torch.equal(bs[i], ys[i]), (t, i)
        assert np.array_equal(pml, seq[t][2]) and np.array_equal(tvar, seq[t][3]), t
    P.close()
