"""Roll-up of layer year losses into programs and a portfolio on the GPU
(ara_rollup) against the oracle's roll-up.

The roll-up adds binary64 tables in a fixed order, so on the same inputs it
must match the oracle bitwise; from the layer passes onwards the program
tables are within the sum of the layers' tolerances (tol * G per trial)."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_cases import TOL, gpu_layer_run, oracle_run
from oracle import oracle
from paper_1412_4556_amd import _lib as L
from paper_1412_4556_amd import ara as A
from paper_1412_4556_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _spec(d):
    return W.LayerSpec([np.array(e["ids"], np.int32) for e in d["elts"]],
                       [np.array(e["losses"], np.float64) for e in d["elts"]],
                       np.array([e["ret"] for e in d["elts"]], np.float64),
                       np.array([e["lim"] for e in d["elts"]], np.float64),
                       d["occ_ret"], d["occ_lim"], d["agg_ret"], d["agg_lim"])


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


@pytest.mark.parametrize("prec,layout", [("fp64", "fused"), ("fp32c", "fused"), ("fp64", "compact"),
                                         ("fp32c", "direct")])
def test_rollup_worked_example(prec, layout):
    """Hand-worked program and portfolio (integers: exact in every form)."""
    g = json.load(open(GOLD))
    off = np.zeros(len(g["trials"]) + 1, np.int64)
    np.cumsum([len(t) for t in g["trials"]], out=off[1:])
    ids = np.array([e for t in g["trials"] for e in t], np.int32)
    T, C = len(off) - 1, g["catalog_size"]
    y1 = gpu_layer_run(ids, off, T, C, 0, _spec(g), prec, layout)
    y2 = gpu_layer_run(ids, off, T, C, 0, _spec(g["rollup"]["layer2"]), prec, layout)
    ru = g["rollup"]
    assert y2.tolist() == ru["layer2"]["ylt"]
    d2 = _cuda(y2)
    p1, p2 = A.rollup([_cuda(y1), d2, d2], [0, 0, 1], 2)
    (pf,) = A.rollup([p1, p2], [0, 0], 1)
    torch.cuda.synchronize()
    assert p1.cpu().numpy().tolist() == ru["program_p1_ylt"]
    assert p2.cpu().numpy().tolist() == ru["program_p2_ylt"]
    assert pf.cpu().numpy().tolist() == ru["portfolio_ylt"]
    Ns = sorted(ru["program_p1_pml_tvar"], key=float)
    pml, tvar = A.pml_tvar(p1, [float(N) for N in Ns])
    for i, N in enumerate(Ns):
        assert [pml[i], tvar[i]] == ru["program_p1_pml_tvar"][N]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_rollup_programs_match_oracle(prec):
    """Five ragged layers into four programs (one without layers): bitwise the
    oracle's roll-up of the same tables, and within tolerance of the oracle's
    roll-up of the oracle's layer tables."""
    T, C = 3001, 20000
    groups, n_groups = [0, 1, 0, 3, 1], 4
    gpu, ref, gross = [], [], []
    ids, off, _ = W.random_case(30, T, 150.0, C, 1, 2500)  # the programs' one YET
    for i, seed in enumerate((31, 32, 33, 34, 35)):
        spec = W.random_case(seed, T, 150.0, C, 3 + i, 2500)[2]  # terms sized for such trials
        gpu.append(gpu_layer_run(ids, off, T, C, 0, spec, prec, "fused"))
        r = oracle_run(ids, off, T, C, 0, spec)
        ref.append(r["ylt"])
        gross.append(r["gross"])
    outs = A.rollup([_cuda(y) for y in gpu], groups, n_groups)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    same = oracle.rollup(gpu, groups, n_groups)
    for g in range(n_groups):
        assert np.array_equal(got[g], same[g]), g
    assert not got[2].any()
    want = oracle.rollup(ref, groups, n_groups)
    gsum = oracle.rollup(gross, groups, n_groups)
    for g in range(n_groups):
        assert np.all(np.abs(got[g] - want[g]) <= TOL[prec] * gsum[g] * 1.0001), g


def test_rollup_full_size_bitwise():
    """64 tables of 1,000,003 trials (a ragged tail beyond the grid) into 8
    programs of 8, then a portfolio: bitwise the oracle's roll-up."""
    T = 1_000_003
    gen = torch.Generator(device="cuda").manual_seed(7)
    ylts = [torch.rand(T, dtype=torch.float64, device="cuda", generator=gen) * 1e7 for _ in range(64)]
    for y in ylts[::5]:
        y[y < 5e6] = 0.0
    groups = [l // 8 for l in range(64)]
    progs = A.rollup(ylts, groups, 8)
    (pf,) = A.rollup(progs, [0] * 8, 1)
    torch.cuda.synchronize()
    host = [y.cpu().numpy() for y in ylts]
    want = oracle.rollup(host, groups, 8)
    for g in range(8):
        assert np.array_equal(progs[g].cpu().numpy(), want[g]), g
    (wpf,) = oracle.rollup(want, [0] * 8, 1)
    assert np.array_equal(pf.cpu().numpy(), wpf)


def test_rollup_errors_and_empty():
    y = torch.zeros(100, dtype=torch.float64, device="cuda")
    z = torch.zeros(100, dtype=torch.float64, device="cuda")
    with pytest.raises(L.AraError) as ei:
        A.rollup([y], [1], 1)
    assert ei.value.name == "ARA_ERR_INVALID_ARG"
    with pytest.raises(L.AraError) as ei:
        A.rollup([y], [0], 1, out=[y])
    assert ei.value.name == "ARA_ERR_INVALID_ARG"
    buf = torch.zeros(150, dtype=torch.float64, device="cuda")
    with pytest.raises(L.AraError) as ei:
        A.rollup([buf[:100]], [0], 1, out=[buf[50:]])  # the output overlaps the input's second half
    assert ei.value.name == "ARA_ERR_INVALID_ARG"
    with pytest.raises(L.AraError) as ei:
        A.rollup([y, buf[:100]], [0, 1], 2, out=[z, z])
    assert ei.value.name == "ARA_ERR_INVALID_ARG"
    with pytest.raises(L.AraError) as ei:
        A.rollup([y] * 65, [0] * 65, 1)
    assert ei.value.name == "ARA_ERR_INVALID_ARG"
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    (o,) = A.rollup([e, e], [0, 0], 1)
    torch.cuda.synchronize()
    assert o.numel() == 0
