"""Parity of the HIP trial pass (through the C-ABI) with the CPU oracle.

Tolerances: every trial's |y - y_oracle| <= tol * G, G the trial's gross
looked-up loss, tol = 1e-12 in FP64 and 1e-6 in FP32C; integer-valued cases
must match bitwise.  Layouts must agree with each other bitwise.
"""
import json
import os

import numpy as np
import pytest
import torch

from gpu_cases import TOL, assert_close_to_oracle, assert_risk_close, gpu_layer_run, oracle_run
from oracle import oracle
from paper_1412_4556_amd import _lib as L
from paper_1412_4556_amd import ara as A
from paper_1412_4556_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
PRECS = ["fp64", "fp32c"]
LAYOUTS = ["direct", "sparse", "compact", "fused"]


def _golden():
    g = json.load(open(GOLD))
    spec = W.LayerSpec([np.array(e["ids"], np.int32) for e in g["elts"]],
                       [np.array(e["losses"], np.float64) for e in g["elts"]],
                       np.array([e["ret"] for e in g["elts"]], np.float64),
                       np.array([e["lim"] for e in g["elts"]], np.float64),
                       g["occ_ret"], g["occ_lim"], g["agg_ret"], g["agg_lim"])
    off = np.zeros(len(g["trials"]) + 1, np.int64)
    np.cumsum([len(t) for t in g["trials"]], out=off[1:])
    ids = np.array([e for t in g["trials"] for e in t], np.int32)
    return g, spec, ids, off


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("layout", LAYOUTS)
def test_worked_example(prec, layout):
    g, spec, ids, off = _golden()
    T = len(off) - 1
    y = gpu_layer_run(ids, off, T, g["catalog_size"], 0, spec, prec, layout)
    assert y.tolist() == g["ylt"]
    y2, cum, net = gpu_layer_run(ids, off, T, g["catalog_size"], 0, spec, prec, layout, events=True)
    assert y2.tolist() == g["ylt"]
    assert [cum[off[i]:off[i + 1]].tolist() for i in range(T)] == g["event_cum"]
    assert [net[off[i]:off[i + 1]].tolist() for i in range(T)] == g["event_net"]
    y3, mx = gpu_layer_run(ids, off, T, g["catalog_size"], 0, spec, prec, layout, max_occ=True)
    assert y3.tolist() == g["ylt"]
    assert mx.tolist() == g["occ_max"]


def test_worked_example_occurrence_basis_pml_tvar():
    from fractions import Fraction
    g, *_ = _golden()
    q = g["occ_max_pml_tvar"]
    pml, tvar = A.pml_tvar(torch.tensor(g["occ_max"], dtype=torch.float64, device="cuda"), q["return_periods"])
    assert pml.tolist() == q["pml"]
    assert np.allclose(tvar, [float(Fraction(t)) for t in q["tvar"]], rtol=1e-15, atol=0)


def test_worked_example_pml_tvar():
    g, *_ = _golden()
    y = torch.tensor(g["ylt"], dtype=torch.float64, device="cuda")
    pml, tvar = A.pml_tvar(y, g["pml_tvar"]["return_periods"])
    assert pml.tolist() == g["pml_tvar"]["pml"]
    assert tvar.tolist() == g["pml_tvar"]["tvar"]


# ----------------------------------------------------------------------------- configured workloads
@pytest.fixture(scope="module")
def tiny():
    wl = W.plain_tiny()
    ids, off = W.yet_full(wl.yet)
    spec = wl.layers[0]
    ref = oracle_run(ids, None, wl.yet.n_trials, wl.yet.catalog_size, wl.yet.fixed_len, spec)
    return wl, ids, spec, ref


def test_plain_tiny_all_layouts(tiny):
    wl, ids, spec, ref = tiny
    T, C, K = wl.yet.n_trials, wl.yet.catalog_size, wl.yet.fixed_len
    assert (ref["ylt"] > 0).mean() > 0.1  # the terms leave a non-degenerate YLT
    results = {}
    for prec in PRECS:
        ys = {}
        for layout in LAYOUTS:
            ys[layout] = gpu_layer_run(ids, None, T, C, K, spec, prec, layout)
            results[(prec, layout)] = assert_close_to_oracle(ys[layout], ref, prec)
        for layout in LAYOUTS[1:]:
            assert np.array_equal(ys[layout], ys["direct"]), (prec, layout)
    print(results)
    # risk metrics: on the GPU's own YLT the selection is exact and the mean
    # is within binary64 rounding; against the oracle's YLT they move by at
    # most the largest per-trial error
    y = gpu_layer_run(ids, None, T, C, K, spec, "fp64", "compact")
    gp, gt = A.pml_tvar(torch.from_numpy(y).cuda(), wl.return_periods)
    op, ot = oracle.pml_tvar(y, wl.return_periods)
    assert np.array_equal(gp, op)
    assert np.allclose(gt, ot, rtol=1e-12, atol=0)
    rp, rt = oracle.pml_tvar(ref["ylt"], wl.return_periods)
    assert_risk_close(gp, gt, rp, rt, "fp64", ref)


@pytest.mark.parametrize("layout", ["fused", "compact"])
@pytest.mark.parametrize("prec", PRECS)
def test_precision_workload(prec, layout):
    wl = W.precision_poisson()
    ids, off = W.yet_full(wl.yet)
    T, C = wl.yet.n_trials, wl.yet.catalog_size
    for spec in wl.layers:
        ref = oracle_run(ids, off, T, C, 0, spec)
        y = gpu_layer_run(ids, off, T, C, 0, spec, prec, layout)
        stats = assert_close_to_oracle(y, ref, prec)
        gp, gt = A.pml_tvar(torch.from_numpy(y).cuda(), wl.return_periods)
        rp, rt = oracle.pml_tvar(ref["ylt"], wl.return_periods)
        risk = assert_risk_close(gp, gt, rp, rt, prec, ref)
        print(spec.name, prec, layout, stats, risk)
        if spec.name == "pareto_uncapped_elt":
            assert (ref["ylt"] > 0).mean() > 0.01


# ----------------------------------------------------------------------------- edge cases
EDGE = [
    # id, kwargs of random_case, misalign
    ("empties", dict(seed=31, n_trials=500, mean_len=30.0, catalog=800, n_elts=4, elt_size=200, empty_frac=0.3), False),
    ("short_trials", dict(seed=32, n_trials=700, mean_len=2.0, catalog=300, n_elts=3, elt_size=100), False),
    ("long_trials", dict(seed=33, n_trials=40, mean_len=3000.0, catalog=5000, n_elts=5, elt_size=1500), False),
    ("misaligned_ids", dict(seed=34, n_trials=300, mean_len=57.0, catalog=900, n_elts=3, elt_size=300), True),
    ("one_trial", dict(seed=35, n_trials=1, mean_len=999.0, catalog=600, n_elts=2, elt_size=300), False),
    ("catalog_one", dict(seed=36, n_trials=50, mean_len=10.0, catalog=1, n_elts=2, elt_size=1), False),
    ("max_elts", dict(seed=37, n_trials=200, mean_len=100.0, catalog=3000, n_elts=32, elt_size=300), False),
    ("one_elt", dict(seed=38, n_trials=300, mean_len=100.0, catalog=3000, n_elts=1, elt_size=2000), False),
    ("open_terms", dict(seed=39, n_trials=300, mean_len=100.0, catalog=3000, n_elts=4, elt_size=800, terms="open"), False),
    ("counting", dict(seed=40, n_trials=300, mean_len=100.0, catalog=3000, n_elts=4, elt_size=800, terms="counting",
                      integer_losses=True), False),
    # catalogues above 2^20 events: the fused pass's block filter covers
    # several events per bit and a hashed filter is probed as well
    ("hashed_filter_1.1M", dict(seed=44, n_trials=1500, mean_len=400.0, catalog=1_100_000, n_elts=6, elt_size=40_000),
     False),
    ("hashed_filter_3M_misaligned", dict(seed=45, n_trials=1200, mean_len=350.0, catalog=3_000_000, n_elts=8,
                                         elt_size=60_000), True),
    # trials longer than a 1,024-event group: the YLT pass reads the group,
    # then the rest of the trial one 256-event chunk at a time
    ("wide_groups_hashed", dict(seed=47, n_trials=900, mean_len=1000.0, catalog=2_000_000, n_elts=8,
                                elt_size=30_000), False),
]


@pytest.mark.parametrize("name,kw,misalign", EDGE, ids=[e[0] for e in EDGE])
@pytest.mark.parametrize("prec", PRECS)
def test_edge_cases(name, kw, misalign, prec):
    ids, off, spec = W.random_case(**kw)
    T, C = kw["n_trials"], kw["catalog"]
    ref = oracle_run(ids, off, T, C, 0, spec, want_event_cum=True, want_event_net=True, want_occ_max=True)
    ys = [gpu_layer_run(ids, off, T, C, 0, spec, prec, lay, ids_misalign=misalign) for lay in LAYOUTS]
    assert_close_to_oracle(ys[0], ref, prec)
    for other in ys[1:]:
        assert np.array_equal(ys[0], other)
    # occurrence basis: the largest occurrence loss per trial, every layout;
    # with binary64 layers it is exactly the oracle's (a maximum of bitwise
    # equal occurrence losses)
    for lay in LAYOUTS:
        y, mx = gpu_layer_run(ids, off, T, C, 0, spec, prec, lay, ids_misalign=misalign, max_occ=True)
        assert np.array_equal(y, ys[0])
        if prec == "fp64":
            assert np.array_equal(mx, ref["occ_max"]), lay
        else:
            assert np.all(np.abs(mx - ref["occ_max"]) <= TOL[prec] * ref["gross"]), lay
    y, cum, net = gpu_layer_run(ids, off, T, C, 0, spec, prec, "fused", events=True, ids_misalign=misalign)
    assert_close_to_oracle(y, ref, prec)
    # the fused per-event pass is bitwise the generic one (compact layout)
    y2, cum2, net2 = gpu_layer_run(ids, off, T, C, 0, spec, prec, "compact", events=True, ids_misalign=misalign)
    assert np.array_equal(y, y2) and np.array_equal(cum, cum2) and np.array_equal(net, net2)
    gross_ev = np.repeat(ref["gross"], np.diff(off))
    assert np.all(np.abs(cum - ref["event_cum"]) <= TOL[prec] * gross_ev)
    assert np.all(np.abs(net - ref["event_net"]) <= 2 * TOL[prec] * gross_ev)


@pytest.mark.parametrize("K", [0, 1, 3, 7, 256, 1000, 1001])
@pytest.mark.parametrize("misalign", [False, True])
def test_fixed_length_trials(K, misalign):
    """Trials without an offsets array, of lengths that are and are not
    multiples of 4, with aligned and unaligned IDs, on every layout."""
    T, C = 257, 2000
    rng = np.random.default_rng(K)
    ids = rng.integers(0, C, size=T * K, dtype=np.int32)
    _, _, spec = W.random_case(41, 1, 1.0, C, 4, 600)
    ref = oracle_run(ids, None, T, C, K, spec)
    for prec in PRECS:
        ys = [gpu_layer_run(ids, None, T, C, K, spec, prec, lay, ids_misalign=misalign and K > 0)
              for lay in ("compact", "fused")]
        assert_close_to_oracle(ys[0], ref, prec)
        assert np.array_equal(ys[0], ys[1])


def test_fixed_length_large_catalog():
    """The paper's shape at 3,000 trials: 1,000 events per trial (no offsets
    array), a 2,000,000-event catalogue and 16 ELTs of 20,000 events, so the
    fixed-length fused pass runs with both LDS filters."""
    T, K, C = 3000, 1000, 2_000_000
    rng = np.random.default_rng(46)
    ids = rng.integers(0, C, size=T * K, dtype=np.int32)
    _, _, spec = W.random_case(46, 1, 1.0, C, 16, 20_000)
    ref = oracle_run(ids, None, T, C, K, spec)
    for prec in PRECS:
        ys = [gpu_layer_run(ids, None, T, C, K, spec, prec, lay) for lay in ("compact", "fused")]
        assert_close_to_oracle(ys[0], ref, prec)
        assert np.array_equal(ys[0], ys[1])
        assert (ys[1] > 0).mean() > 0.05


def test_largest_catalog():
    """Event IDs up to 2^31 - 2 (catalogue 2^31 - 1, the largest accepted):
    the fused table has 2^31 entries and each block-filter bit covers 2^11
    events; every layout and precision against the oracle."""
    C = 2**31 - 1
    rng = np.random.default_rng(47)
    elt_ids = [np.unique(rng.integers(0, C, 1200)).astype(np.int32)[:1000] for _ in range(3)]
    elt_ids[0][:2] = [0, C - 1]
    elt_ids[0] = np.unique(elt_ids[0]).astype(np.int32)
    losses = [np.round(rng.lognormal(8, 1.5, len(e)), 2) for e in elt_ids]
    spec = W.LayerSpec(elt_ids, losses, np.full(3, 100.0), np.full(3, 1e6), 50.0, 5e6, 1e3, 1e8)
    T = 300
    lens = rng.poisson(40, T)
    off = np.zeros(T + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    pool = np.concatenate(elt_ids)
    ids = np.where(rng.random(off[-1]) < 0.5, rng.choice(pool, off[-1]), rng.integers(0, C, off[-1])).astype(np.int32)
    ids[off[0]:off[0] + 2] = [C - 1, 0]
    ref = oracle_run(ids, off, T, C, 0, spec)
    assert (ref["ylt"] > 0).mean() > 0.5
    for prec, layout in (("fp64", "fused"), ("fp32c", "fused"), ("fp64", "compact"), ("fp64", "sparse")):
        y = gpu_layer_run(ids, off, T, C, 0, spec, prec, layout)
        assert_close_to_oracle(y, ref, prec)
        torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", PRECS)
def test_integer_cases_are_bitwise(prec):
    for seed in (51, 52, 53):
        ids, off, spec = W.random_case(seed, 400, 300.0, 4000, 4, 1500, integer_losses=True, max_int_loss=60)
        ref = oracle_run(ids, off, 400, 4000, 0, spec, want_event_cum=True, want_event_net=True)
        for layout in LAYOUTS:
            y = gpu_layer_run(ids, off, 400, 4000, 0, spec, prec, layout)
            assert np.array_equal(y, ref["ylt"]), (seed, layout)
        for layout in ("compact", "fused"):
            y, cum, net = gpu_layer_run(ids, off, 400, 4000, 0, spec, prec, layout, events=True)
            assert np.array_equal(y, ref["ylt"]) and np.array_equal(cum, ref["event_cum"])
            assert np.array_equal(net, ref["event_net"])


def test_zero_trials():
    ids = np.zeros(0, np.int32)
    off = np.zeros(1, np.int64)
    _, _, spec = W.random_case(42, 1, 1.0, 100, 2, 50)
    y = gpu_layer_run(ids, off, 0, 100, 0, spec, "fp64", "compact")
    assert y.shape == (0,)


def test_runs_are_deterministic():
    ids, off, spec = W.random_case(43, 2000, 200.0, 20000, 8, 3000)
    a = gpu_layer_run(ids, off, 2000, 20000, 0, spec, "fp32c", "compact")
    b = gpu_layer_run(ids, off, 2000, 20000, 0, spec, "fp32c", "compact")
    assert np.array_equal(a, b)


# ----------------------------------------------------------------------------- risk metrics
@pytest.mark.parametrize("T,N", [(1, 1), (1000, 100), (1000, 250), (997, 10), (100_000, 250), (1_000_000, 100)])
def test_pml_tvar_permutation(T, N):
    y = np.random.default_rng(T).permutation(np.arange(1, T + 1)).astype(np.float64)
    pml, tvar = A.pml_tvar(torch.from_numpy(y).cuda(), [N])
    k = T // N
    assert pml[0] == T - k + 1
    assert tvar[0] == T - (k - 1) / 2


def test_pml_tvar_largest_size():
    """The largest accepted YLT, 2^31 - 1 trials (16 GiB), holding 1..T in
    reverse order: PML_N = T - k + 1 exactly; TVaR_N = T - (k - 1) / 2, exact
    while the tail sum stays below 2^53, else within binary64 summation error."""
    T = 2**31 - 1
    y = torch.arange(T, 0, -1, dtype=torch.float64, device="cuda")
    Ns = [float(T), 1e6, 100.0, 1.0]
    pml, tvar = A.pml_tvar(y, Ns)
    del y
    torch.cuda.empty_cache()
    for i, N in enumerate(Ns):
        k = int(T // N)
        assert pml[i] == T - k + 1, (N, pml[i])
        want = T - (k - 1) / 2
        if k * float(T) < 2.0**53:
            assert tvar[i] == want, (N, tvar[i])
        else:
            assert abs(tvar[i] - want) <= 1e-12 * want, (N, tvar[i], want)


def test_pml_tvar_ties_zeros_negatives():
    rng = np.random.default_rng(7)
    y = np.concatenate([np.zeros(5000), np.full(300, 7.5), rng.lognormal(5, 1, 700), -rng.uniform(0, 5, 100)])
    rng.shuffle(y)
    Ns = [1, 2, 10, 17, 100, 6100]
    gp, gt = A.pml_tvar(torch.from_numpy(y).cuda(), Ns)
    op, ot = oracle.pml_tvar(y, Ns)
    assert np.array_equal(gp, op)
    assert np.allclose(gt, ot, rtol=1e-12, atol=1e-300)


def test_pml_tvar_call_sequence():
    """Calls of different shapes in a row (1, 64 and 5 YLTs; 1 to 16 return
    periods; one call rejected for a NaN in between) each match the oracle:
    nothing of one call's selection state or NaN flag reaches the next."""
    rng = np.random.default_rng(11)
    T = 20_011
    ylts = [np.round(rng.lognormal(12, 1.5, T), 2) for _ in range(64)]
    for y in ylts[::3]:
        y[rng.integers(0, T, 400)] = 0.0
    dev = [torch.from_numpy(y).cuda() for y in ylts]
    shapes = [(1, [250.0]), (64, [1.0, 2.0, 10.0, 100.0, 250.0, 1000.0, 3.0, 7.0, 11.0, 13.0, 17.0, 19.0, 23.0,
                                  29.0, 31.0, 20011.0]),
              (5, [100.0, 250.0]), (1, [2.0, 5.0, 20011.0])]
    for i, (n, Ns) in enumerate(shapes):
        if i == 2:
            bad = dev[0].clone()
            bad[17] = float("nan")
            with pytest.raises(L.AraError) as ei:
                A.pml_tvar(bad, [100.0])
            assert ei.value.name == "ARA_ERR_VALUE"
        if n == 1:
            gp, gt = A.pml_tvar(dev[i], Ns)
            gp, gt = gp[None, :], gt[None, :]
            src = [ylts[i]]
        else:
            gp, gt = A.pml_tvar_many(dev[:n], Ns)
            src = ylts[:n]
        for j, y in enumerate(src):
            op, ot = oracle.pml_tvar(y, Ns)
            assert np.array_equal(gp[j], op), (i, j)
            assert np.allclose(gt[j], ot, rtol=1e-12, atol=0.0), (i, j)


def test_pml_tvar_errors():
    y = torch.ones(10, dtype=torch.float64, device="cuda")
    with pytest.raises(L.AraError) as ei:
        A.pml_tvar(y, [100])
    assert ei.value.name == "ARA_ERR_RP"
    y[3] = float("nan")
    with pytest.raises(L.AraError) as ei:
        A.pml_tvar(y, [2])
    assert ei.value.name == "ARA_ERR_VALUE"


# ----------------------------------------------------------------------------- error paths
@pytest.mark.parametrize("misalign", [0, 1, 2, 3])
def test_yet_validation_reads_every_id(misalign):
    """One out-of-range ID is found wherever it sits: before the first 16-byte
    boundary, in the vector body (in whole 8 KiB chunks and after them) or
    after the last whole granule; large YETs too."""
    for n in (1, 3, 7, 203, 4099, 17_000_017):
        buf = torch.zeros(n + 4, dtype=torch.int32, device="cuda")
        ids = buf[misalign:misalign + n]
        assert ids.data_ptr() % 16 == (buf.data_ptr() + 4 * misalign) % 16
        A.Yet(ids, None, 1, 10, n).close()
        for pos in sorted({0, 1, 2, 3, n // 2, n - 5, n - 4, n - 3, n - 1}):
            if not 0 <= pos < n:
                continue
            ids[pos] = 10
            with pytest.raises(L.AraError) as ei:
                A.Yet(ids, None, 1, 10, n)
            assert ei.value.name == "ARA_ERR_EVENT_RANGE", (n, pos)
            ids[pos] = -1
            with pytest.raises(L.AraError) as ei:
                A.Yet(ids, None, 1, 10, n)
            assert ei.value.name == "ARA_ERR_EVENT_RANGE", (n, pos)
            ids[pos] = 9
            A.Yet(ids, None, 1, 10, n).close()
            ids[pos] = 0


def test_create_errors():
    ids = torch.tensor([0, 1, 2, 5], dtype=torch.int32, device="cuda")
    with pytest.raises(L.AraError) as ei:
        A.Yet(ids, None, 2, 5, 2)
    assert ei.value.name == "ARA_ERR_EVENT_RANGE"
    bad_off = torch.tensor([0, 3, 2, 4], dtype=torch.int64, device="cuda")
    with pytest.raises(L.AraError) as ei:
        A.Yet(ids, bad_off, 3, 10)
    assert ei.value.name == "ARA_ERR_INVALID_ARG"
    yet = A.Yet(ids, None, 2, 10, 2)
    one = lambda ids_, loss: W.LayerSpec([np.array(ids_, np.int32)], [np.array(loss, np.float64)],
                                               np.zeros(1), np.full(1, np.inf), 0.0, np.inf, 0.0, np.inf)
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, one([1, 1], [1.0, 2.0]))
    assert ei.value.name == "ARA_ERR_DUP_EVENT"
    # an event may sit in several ELTs of a layer; a duplicate inside a later
    # ELT is still found (every ID here shares one 64-bit word of the check)
    two = lambda a, b: W.LayerSpec([np.array(a, np.int32), np.array(b, np.int32)],
                                   [np.ones(len(a)), np.ones(len(b))], np.zeros(2), np.full(2, np.inf), 0.0, np.inf,
                                   0.0, np.inf)
    for layout in ("fused", "compact", "direct", "sparse"):
        A.Layer(yet, two([1, 2, 3], [3, 2, 1]), "fp64", layout).close()
        with pytest.raises(L.AraError) as ei:
            A.Layer(yet, two([1, 2], [3, 4, 3]), "fp64", layout)
        assert ei.value.name == "ARA_ERR_DUP_EVENT", layout
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, one([1, 11], [1.0, 2.0]))
    assert ei.value.name == "ARA_ERR_EVENT_RANGE"
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, one([1, 2], [1.0, -2.0]))
    assert ei.value.name == "ARA_ERR_VALUE"
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, one([1, 2], [1.0, float("nan")]))
    assert ei.value.name == "ARA_ERR_VALUE"
    spec = one([1], [1.0]).with_terms(occ_ret=-1.0)
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, spec)
    assert ei.value.name == "ARA_ERR_VALUE"
    big = W.LayerSpec([np.array([i % 10], np.int32) for i in range(33)], [np.ones(1)] * 33, np.zeros(33),
                      np.full(33, np.inf), 0, np.inf, 0, np.inf)
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, big)
    assert ei.value.name == "ARA_ERR_UNSUPPORTED"
    # a valid layer still works after the failures
    lay = A.Layer(yet, one([0, 5], [3.0, 4.0]))
    y = A.run_layer(yet, lay).cpu().numpy()
    assert y.tolist() == [3.0, 4.0]
    # the occurrence-basis entry point needs both output arrays
    import ctypes
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    rc = L.lib().ara_run_layer_max_occurrence(yet.handle, lay.handle, ctypes.c_void_p(out.data_ptr()), None, None)
    assert L.ERRORS.get(rc) == "ARA_ERR_INVALID_ARG"
    rc = L.lib().ara_run_layer_max_occurrence(None, lay.handle, ctypes.c_void_p(out.data_ptr()),
                                              ctypes.c_void_p(out.data_ptr()), None)
    assert L.ERRORS.get(rc) == "ARA_ERR_INVALID_ARG"
    y2, mx = A.run_layer_max_occurrence(yet, lay)
    assert y2.cpu().tolist() == [3.0, 4.0] and mx.cpu().tolist() == [3.0, 4.0]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_fused_build_at_paper_catalogue(prec):
    """The one-launch fused build at the paper's catalogue (2M events, 16 ELTs
    of 20,000): its table gives bitwise the YLT of the compact layout, and it
    finds a duplicate ID, an out-of-range ID and a bad loss anywhere in the
    ELTs (the checks run on the GPU for this layout)."""
    C = 2_000_000
    ids, off, spec = W.random_case(1999, 3000, 400.0, C, 16, 20_000)
    T = len(off) - 1
    yet = A.yet_from_numpy(ids, off, T, C)
    fused = A.Layer(yet, spec, prec, "fused")
    compact = A.Layer(yet, spec, prec, "compact")
    yf = A.run_layer(yet, fused).cpu().numpy()
    yc = A.run_layer(yet, compact).cpu().numpy()
    assert np.array_equal(yf, yc)
    # the same table from a pool of the same ELTs
    P = A.Pool(yet, spec.elt_ids, spec.elt_losses, prec, max_layers=2)
    lp = P.layer(np.arange(16, dtype=np.int32), spec.ret, spec.lim, spec.occ_ret, spec.occ_lim, spec.agg_ret,
                 spec.agg_lim)
    assert np.array_equal(A.run_layer(yet, lp).cpu().numpy(), yf)
    lp.close()
    ref = oracle_run(ids, off, T, C, 0, spec)
    assert_close_to_oracle(yf, ref, prec)

    def broken(j, pos, value=None, loss=None):
        e_ids = [a.copy() for a in spec.elt_ids]
        e_loss = [a.copy() for a in spec.elt_losses]
        if value is not None:
            e_ids[j][pos] = value
        if loss is not None:
            e_loss[j][pos] = loss
        return W.LayerSpec(e_ids, e_loss, spec.ret, spec.lim, spec.occ_ret, spec.occ_lim, spec.agg_ret, spec.agg_lim)

    cases = [(9, 19_990, int(spec.elt_ids[9][5]), None, "ARA_ERR_DUP_EVENT"),
             (0, 0, int(spec.elt_ids[0][19_999]), None, "ARA_ERR_DUP_EVENT"),
             (15, 19_999, C, None, "ARA_ERR_EVENT_RANGE"),
             (3, 7, -5, None, "ARA_ERR_EVENT_RANGE"),
             (0, 11_111, None, float("inf"), "ARA_ERR_VALUE"),
             (12, 3, None, float("nan"), "ARA_ERR_VALUE"),
             (7, 19_000, None, -1e-300, "ARA_ERR_VALUE")]
    for j, pos, value, loss, want in cases:
        with pytest.raises(L.AraError) as ei:
            A.Layer(yet, broken(j, pos, value, loss), prec, "fused")
        assert ei.value.name == want, (j, pos, value, loss)
    # an ID in several ELTs of the layer is allowed
    e_ids = [a.copy() for a in spec.elt_ids]
    in4 = set(spec.elt_ids[4].tolist())
    e_ids[4][0] = next(x for x in spec.elt_ids[3].tolist() if x not in in4)
    ok = W.LayerSpec(e_ids, spec.elt_losses, spec.ret, spec.lim, spec.occ_ret, spec.occ_lim, spec.agg_ret,
                     spec.agg_lim)
    A.Layer(yet, ok, prec, "fused").close()
    # and a valid build still works after the failed ones
    again = A.Layer(yet, spec, prec, "fused")
    assert np.array_equal(A.run_layer(yet, again).cpu().numpy(), yf)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_fused_build_concentrated_elts(prec):
    """ELTs whose events crowd into one 8,192-event range of the catalogue
    (the part one work-group of the one-launch build owns): the table is
    still bitwise the compact layout's, and a duplicate ID or a bad loss
    inside the crowded range is still found."""
    C = 200_000
    rng = np.random.default_rng(2027)
    eids, elos = [], []
    for j in range(8):
        eids.append(rng.choice(8192, size=6000, replace=False).astype(np.int32))  # all in the first range
        elos.append(rng.lognormal(8.0, 2.0, 6000))
    for j in range(2):
        eids.append(rng.choice(C, size=20_000, replace=False).astype(np.int32))
        elos.append(rng.lognormal(8.0, 2.0, 20_000))
    J = len(eids)
    ret = np.array([np.quantile(l, 0.1) for l in elos])
    lim = np.array([np.quantile(l, 0.9) for l in elos])
    spec = W.LayerSpec(eids, elos, ret, lim, 500.0, 1e6, 1e4, 1e8)
    T = 2000
    ids = np.concatenate([rng.integers(0, 8192, size=T * 200 // 2), rng.integers(0, C, size=T * 200 // 2)]).astype(np.int32)
    rng.shuffle(ids)
    yet = A.Yet(torch.from_numpy(ids).cuda(), None, T, C, 200)
    yf = A.run_layer(yet, A.Layer(yet, spec, prec, "fused")).cpu().numpy()
    yc = A.run_layer(yet, A.Layer(yet, spec, prec, "compact")).cpu().numpy()
    assert np.array_equal(yf, yc)
    assert (yf > 0).mean() > 0.05
    # the same table built from a device pool of the ELTs
    P = A.Pool(yet, eids, elos, prec, max_layers=1)
    lp = P.layer(np.arange(J, dtype=np.int32), ret, lim, 500.0, 1e6, 1e4, 1e8)
    assert np.array_equal(A.run_layer(yet, lp).cpu().numpy(), yf)
    lp.close()
    ref = oracle_run(ids, None, T, C, 200, spec)
    assert_close_to_oracle(yf, ref, prec)
    bad_ids = [a.copy() for a in eids]
    bad_ids[3][5999] = bad_ids[3][17]
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, W.LayerSpec(bad_ids, elos, ret, lim, 500.0, 1e6, 1e4, 1e8), prec, "fused")
    assert ei.value.name == "ARA_ERR_DUP_EVENT"
    bad_los = [a.copy() for a in elos]
    bad_los[5][100] = float("nan")
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, W.LayerSpec(eids, bad_los, ret, lim, 500.0, 1e6, 1e4, 1e8), prec, "fused")
    assert ei.value.name == "ARA_ERR_VALUE"


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_fused_build_more_ranges_than_list_counters(prec):
    """A catalogue of 40M events: 4,883 ranges of 8,192 events, more than
    the build's per-work-group range counters, so every entry reserves its
    place in its range's list with an atomic of its own.  The table is
    bitwise the compact layout's (from the host and from a device pool),
    the oracle's within tolerance, and a duplicate ID is still found."""
    C = 40_000_000
    rng = np.random.default_rng(2029)
    eids = [rng.choice(C, size=3000, replace=False).astype(np.int32) for _ in range(4)]
    # 500 events in two ELTs of the layer (ELT 2 keeps 3,000 distinct IDs)
    eids[2] = np.concatenate([eids[1][:500], rng.permutation(np.setdiff1d(eids[2], eids[1][:500]))[:2500]])
    assert all(len(np.unique(e)) == 3000 for e in eids)
    elos = [rng.lognormal(8.0, 2.0, 3000) for _ in range(4)]
    ret = np.array([np.quantile(l, 0.1) for l in elos])
    lim = np.array([np.quantile(l, 0.9) for l in elos])
    spec = W.LayerSpec(eids, elos, ret, lim, 500.0, 1e6, 1e4, 1e8)
    T = 500
    lens = rng.poisson(60, T)
    off = np.zeros(T + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    pool = np.concatenate(eids)
    ids = np.where(rng.random(off[-1]) < 0.6, rng.choice(pool, off[-1]), rng.integers(0, C, off[-1])).astype(np.int32)
    yet = A.yet_from_numpy(ids, off, T, C)
    yf = A.run_layer(yet, A.Layer(yet, spec, prec, "fused")).cpu().numpy()
    yc = A.run_layer(yet, A.Layer(yet, spec, prec, "compact")).cpu().numpy()
    assert np.array_equal(yf, yc)
    assert (yf > 0).mean() > 0.1
    P = A.Pool(yet, eids, elos, prec, max_layers=1)
    lp = P.layer(np.arange(4, dtype=np.int32), ret, lim, 500.0, 1e6, 1e4, 1e8)
    assert np.array_equal(A.run_layer(yet, lp).cpu().numpy(), yf)
    lp.close()
    ref = oracle_run(ids, off, T, C, 0, spec)
    assert_close_to_oracle(yf, ref, prec)
    bad_ids = [a.copy() for a in eids]
    bad_ids[0][2999] = bad_ids[0][0]
    with pytest.raises(L.AraError) as ei:
        A.Layer(yet, W.LayerSpec(bad_ids, elos, ret, lim, 500.0, 1e6, 1e4, 1e8), prec, "fused")
    assert ei.value.name == "ARA_ERR_DUP_EVENT"


@pytest.mark.parametrize("C", [8191, 8192, 8193, 16384, 24577])
def test_fused_build_range_boundaries(C):
    """Catalogues around multiples of the build's 8,192-event ranges (the
    last range holding only the zero slot when the catalogue is a multiple,
    a single event past a multiple): the GPU-built table gives bitwise the
    compact layout's YLT, from host ELTs and from a device pool, in both
    precisions, with events at both ends of every range."""
    rng = np.random.default_rng(C)
    edges = np.array([e for g in range(0, C, 8192) for e in (g, g + 1, g + 8191) if e < C] + [C - 1], np.int64)
    eids = []
    for j in range(3):
        rest = rng.choice(C, size=min(C // 3, 3000), replace=False)
        eids.append(np.unique(np.concatenate([edges, rest])).astype(np.int32))
    elos = [rng.lognormal(8.0, 1.5, len(e)) for e in eids]
    ret = np.array([np.quantile(l, 0.1) for l in elos])
    lim = np.array([np.quantile(l, 0.95) for l in elos])
    spec = W.LayerSpec(eids, elos, ret, lim, 100.0, 1e6, 1e3, 1e8)
    T = 400
    lens = rng.poisson(50, T)
    off = np.zeros(T + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    ids = np.where(rng.random(off[-1]) < 0.3, rng.choice(edges, off[-1]), rng.integers(0, C, off[-1])).astype(np.int32)
    yet = A.yet_from_numpy(ids, off, T, C)
    ref = oracle_run(ids, off, T, C, 0, spec)
    for prec in PRECS:
        yf = A.run_layer(yet, A.Layer(yet, spec, prec, "fused")).cpu().numpy()
        yc = A.run_layer(yet, A.Layer(yet, spec, prec, "compact")).cpu().numpy()
        assert np.array_equal(yf, yc), prec
        P = A.Pool(yet, eids, elos, prec, max_layers=1)
        lp = P.layer(np.arange(3, dtype=np.int32), ret, lim, 100.0, 1e6, 1e3, 1e8)
        assert np.array_equal(A.run_layer(yet, lp).cpu().numpy(), yf), prec
        lp.close()
        assert_close_to_oracle(yf, ref, prec)


def test_layer_from_flat_arrays():
    """The binding's flat-array constructor (the ELTs as ara_create_layer
    takes them) builds the same layer as the per-ELT spec, and rejects terms
    that do not match the ELT count."""
    ids, off, spec = W.random_case(77, 300, 40.0, 5000, 3, 600)
    T = len(off) - 1
    yet = A.yet_from_numpy(ids, off, T, 5000)
    terms = (spec.ret, spec.lim, spec.occ_ret, spec.occ_lim, spec.agg_ret, spec.agg_lim)
    for prec in PRECS:
        a = A.run_layer(yet, A.Layer(yet, spec, prec, "fused")).cpu().numpy()
        b = A.run_layer(yet, A.Layer.from_flat(yet, *spec.concat(), *terms, prec, "fused")).cpu().numpy()
        assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        A.Layer.from_flat(yet, *spec.concat(), spec.ret[:2], spec.lim, *terms[2:])
