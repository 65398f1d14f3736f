"""Batched form at the size the benchmark times: one record pass over
1,000,000 Poisson(1000)-length trials for 64 layers of 1..32 ELTs over a
2,000,000-event catalogue, in the tuned launch shape replayed from its graph.
Every batched YLT is bitwise the single-layer pass of its layer over the
whole YET; the oracle recomputes a sample of trials of every layer,
regenerated on the host from the same seeded blocks; the risk metrics of the
full YLTs agree with the oracle's selection, and their roll-up into programs
and a portfolio is bitwise the oracle's."""
import numpy as np
import pytest
import torch

from gpu_cases import assert_close_to_oracle, oracle_run
from oracle import oracle
from paper_1412_4556_amd import ara as A
from paper_1412_4556_amd import workloads as W

pytestmark = pytest.mark.gpu

N_SAMPLE = 200
RPS = (100.0, 250.0, 1000.0)


@pytest.fixture(scope="module")
def batch_paper():
    wl = W.batch_layers()
    ids, off = W.yet_full(wl.yet)
    t_ids = torch.from_numpy(ids).cuda()
    t_off = torch.from_numpy(off).cuda()
    del ids
    yet = A.Yet(t_ids, t_off, wl.yet.n_trials, wl.yet.catalog_size)
    rng = np.random.default_rng(4556)
    sample = np.unique(np.concatenate([[0, wl.yet.n_trials - 1],
                                       rng.choice(wl.yet.n_trials, N_SAMPLE, replace=False)]))
    sub_ids, sub_off = W.yet_subset(wl.yet, sample, off)
    return wl, yet, sample, sub_ids, sub_off


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_batch_paper_scale(batch_paper, prec):
    wl, yet, sample, sub_ids, sub_off = batch_paper
    T, C = wl.yet.n_trials, wl.yet.catalog_size
    print(f"batch paper scale {prec}: {len(wl.layers)} layers, {T} trials", flush=True)
    layers = [A.Layer(yet, s, prec, "fused") for s in wl.layers]
    outs = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in layers]
    b = A.Batch(yet, layers)
    b.run(outs)  # tunes the launch shape
    for o in outs:
        o.fill_(-1.0)
    b.run(outs)  # replays the captured graph in the tuned shape
    torch.cuda.synchronize()
    threads, per_cu = b.launch_config
    assert threads % 64 == 0 and per_cu >= 1
    rows = torch.from_numpy(sample).cuda()
    y = torch.empty(T, dtype=torch.float64, device="cuda")
    for l, (lay, o) in enumerate(zip(layers, outs)):
        A.run_layer(yet, lay, out=y)
        torch.cuda.synchronize()
        assert torch.equal(o, y), f"layer {l}: batched YLT differs from the single-layer pass"
        ref = oracle_run(sub_ids, sub_off, len(sample), C, 0, wl.layers[l])
        assert_close_to_oracle(o[rows].cpu().numpy(), ref, prec)
    # risk metrics of 16 of the full batched YLTs in one call
    pick = list(range(0, len(outs), 4))
    gp, gt = A.pml_tvar_many([outs[i] for i in pick], RPS)
    for r, i in enumerate(pick):
        yh = outs[i].cpu().numpy()
        op, ot = oracle.pml_tvar(yh, RPS)
        assert np.array_equal(gp[r], op), i
        assert np.allclose(gt[r], ot, rtol=1e-12, atol=0), i
    assert sum(int((o > 0).sum()) for o in outs) > 0
    # roll-up as the benchmark times it: programs of 8 consecutive layers,
    # then the portfolio of the programs, bitwise the oracle's
    groups = [l * 8 // len(outs) for l in range(len(outs))]
    progs = A.rollup(outs, groups, 8)
    pfolio = A.rollup(progs, [0] * 8, 1)
    torch.cuda.synchronize()
    host = [o.cpu().numpy() for o in outs]
    ref_p = oracle.rollup(host, groups, 8)
    ref_f = oracle.rollup(ref_p, [0] * 8, 1)
    for g in range(8):
        assert np.array_equal(progs[g].cpu().numpy(), ref_p[g]), g
    assert np.array_equal(pfolio[0].cpu().numpy(), ref_f[0])
    b.close()
    for lay in layers:
        lay.close()
