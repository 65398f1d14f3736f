"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a hand-worked example, a
closed form that reduces the pass to a library routine, an invariant of the
method (Section III), or exact rational arithmetic on tiny inputs.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from fractions import Fraction

from exact_ref import exact_layer, exact_occ_max
from oracle import oracle
from paper_1412_4556_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
U64 = 2.0 ** -53


def _golden_layer(g):
    return W.LayerSpec([np.array(e["ids"], np.int32) for e in g["elts"]],
                       [np.array(e["losses"], np.float64) for e in g["elts"]],
                       np.array([e["ret"] for e in g["elts"]], np.float64),
                       np.array([e["lim"] for e in g["elts"]], np.float64),
                       g["occ_ret"], g["occ_lim"], g["agg_ret"], g["agg_lim"])


def _flatten(trials):
    off = np.zeros(len(trials) + 1, np.int64)
    np.cumsum([len(t) for t in trials], out=off[1:])
    ids = np.array([e for t in trials for e in t], np.int32)
    return ids, off


def _run(ids, off, C, layer, **kw):
    return oracle.run_layer(ids, off, len(off) - 1, 0, C, layer, **kw)


# ----------------------------------------------------------------------------- hand-worked example
def test_worked_example_exact():
    g = json.load(open(GOLD))
    lay = _golden_layer(g)
    ids, off = _flatten(g["trials"])
    r = _run(ids, off, g["catalog_size"], lay, want_event_net=True, want_event_cum=True)
    assert r["ylt"].tolist() == g["ylt"]
    cum = [r["event_cum"][off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)]
    assert cum == g["event_cum"]
    assert r["occ_sum"].tolist() == g["occ_sum"]
    net = [r["event_net"][off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)]
    assert net == g["event_net"]
    # order dependence of the per-event split, order independence of the total
    pid, poff = _flatten([g["permuted_trial"]["events"]])
    rp = _run(pid, poff, g["catalog_size"], lay, want_event_net=True)
    assert rp["event_net"].tolist() == g["permuted_trial"]["event_net"]
    assert rp["ylt"].tolist() == [g["permuted_trial"]["ylt"]]
    # open terms: plain sums of looked-up losses
    ro = _run(ids, off, g["catalog_size"], lay.open_terms())
    assert ro["ylt"].tolist() == g["open_terms_ylt"]


def test_worked_example_occ_max():
    """Per-trial largest occurrence loss (occurrence basis), by hand."""
    g = json.load(open(GOLD))
    lay = _golden_layer(g)
    ids, off = _flatten(g["trials"])
    r = _run(ids, off, g["catalog_size"], lay, want_occ_max=True)
    assert r["occ_max"].tolist() == g["occ_max"]
    q = g["occ_max_pml_tvar"]
    pml, tvar = oracle.pml_tvar(r["occ_max"], q["return_periods"])
    assert pml.tolist() == q["pml"]
    assert tvar.tolist() == [float(Fraction(t)) for t in q["tvar"]]


def test_worked_example_pml_tvar():
    g = json.load(open(GOLD))
    pml, tvar = oracle.pml_tvar(np.array(g["ylt"], np.float64), g["pml_tvar"]["return_periods"])
    assert pml.tolist() == g["pml_tvar"]["pml"]
    assert tvar.tolist() == g["pml_tvar"]["tvar"]


# ----------------------------------------------------------------------------- exact brute force
CASES = [
    # seed, trials, mean_len, catalog, elts, elt_size, integer, terms, empty_frac
    (1, 40, 12.0, 30, 3, 12, False, "random", 0.1),
    (2, 50, 8.0, 20, 4, 10, False, "random", 0.2),
    (3, 30, 15.0, 25, 1, 20, False, "random", 0.0),
    (4, 40, 10.0, 30, 4, 15, True, "random", 0.1),
    (5, 25, 20.0, 30, 2, 30, False, "open", 0.0),
    (6, 25, 20.0, 30, 3, 9, True, "counting", 0.1),
    (7, 50, 5.0, 12, 4, 12, False, "random", 0.3),
]


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_oracle_matches_exact_rationals(case):
    seed, T, L, C, J, n, integer, terms, empty = case
    ids, off, lay = W.random_case(seed, T, L, C, J, n, integer_losses=integer, terms=terms, empty_frac=empty)
    r = _run(ids, off, C, lay, want_event_net=True)
    ey, eS, eG, enet = exact_layer(ids, off, lay)
    for i in range(T):
        K = int(off[i + 1] - off[i])
        G = float(eG[i])
        bound = (K + J + 3) * U64 * G * 1.01
        assert abs(r["ylt"][i] - float(ey[i])) <= bound, (i, r["ylt"][i], float(ey[i]))
        assert abs(r["occ_sum"][i] - float(eS[i])) <= bound
        assert r["gross"][i] == pytest.approx(G, rel=1e-12, abs=0)
        if integer:
            assert r["ylt"][i] == float(ey[i])
    # largest occurrence loss per trial
    rm = _run(ids, off, C, lay, want_occ_max=True)["occ_max"]
    em = exact_occ_max(ids, off, lay)
    for i in range(T):
        assert abs(rm[i] - float(em[i])) <= (J + 3) * U64 * float(eG[i]) * 1.01
        if integer:
            assert rm[i] == float(em[i])
    # per-event increments: sum of increments = year loss; each within bound
    for k in range(len(ids)):
        assert abs(r["event_net"][k] - float(enet[k])) <= (len(ids) + J + 3) * U64 * max(float(sum(eG)), 1.0)


# ----------------------------------------------------------------------------- closed forms
def _presence_and_totals(lay, C):
    w = np.zeros(C)
    present = np.zeros(C, bool)
    for e, l in zip(lay.elt_ids, lay.elt_losses):
        np.add.at(w, e, l)
        present[e] = True
    return w, present


def _count_matrix(ids, off, C):
    T = len(off) - 1
    rows = np.repeat(np.arange(T), np.diff(off))
    return sp.csr_matrix((np.ones(len(ids)), (rows, ids)), shape=(T, C))


@pytest.mark.parametrize("integer", [True, False])
def test_open_terms_reduce_to_sparse_matvec(integer):
    """Zero retentions and infinite limits: year loss = sum over the trial's
    events of the event's total loss over the ELTs (a count-matrix product)."""
    C = 5000
    ids, off, lay = W.random_case(11, 300, 200.0, C, 5, 800, integer_losses=integer, max_int_loss=1000,
                                  terms="open")
    w, _ = _presence_and_totals(lay, C)
    expect = _count_matrix(ids, off, C) @ w
    r = _run(ids, off, C, lay)
    if integer:
        assert np.array_equal(r["ylt"], expect)
    else:
        K = np.diff(off)
        assert np.all(np.abs(r["ylt"] - expect) <= (K + 8) * U64 * expect * 1.01)
    assert np.array_equal(r["ylt"], r["occ_sum"])


def test_counting_form_counts_present_events():
    """Open per-ELT terms, occurrence limit 1, losses >= 1: each occurrence of
    an event present in at least one ELT contributes exactly 1."""
    C = 3000
    ids, off, lay = W.random_case(12, 400, 150.0, C, 4, 300, integer_losses=True, terms="counting")
    _, present = _presence_and_totals(lay, C)
    counts = np.add.reduceat(present[ids].astype(np.int64), off[:-1]) * (np.diff(off) > 0)
    r = _run(ids, off, C, lay)
    assert np.array_equal(r["ylt"], counts.astype(np.float64))


def test_aggregate_terms_saturate():
    C = 2000
    ids, off, lay = W.random_case(13, 500, 100.0, C, 3, 400)
    base = _run(ids, off, C, lay.with_terms(agg_ret=0.0, agg_lim=np.inf))
    S = base["occ_sum"]
    R3 = float(np.quantile(S, 0.3))
    L3 = float(np.quantile(S, 0.8) - R3)
    r = _run(ids, off, C, lay.with_terms(agg_ret=R3, agg_lim=L3))
    assert np.all(r["ylt"] <= L3)
    assert np.all(r["ylt"][S >= R3 + L3] == L3)
    assert np.all(r["ylt"][S <= R3] == 0.0)
    assert np.all(r["ylt"] >= 0.0)
    mid = (S > R3) & (S < R3 + L3)
    assert mid.any()
    assert np.allclose(r["ylt"][mid], S[mid] - R3, rtol=0, atol=4 * U64 * S.max())


def test_occurrence_limit_bounds():
    C = 2000
    ids, off, lay = W.random_case(14, 300, 100.0, C, 3, 400)
    lay = lay.with_terms(agg_ret=0.0, agg_lim=np.inf)
    r = _run(ids, off, C, lay)
    K = np.diff(off)
    assert np.all(r["occ_sum"] <= K * lay.occ_lim * (1 + 1e-12))
    assert np.all(r["occ_sum"] <= r["gross"] * (1 + 1e-12))


def test_additivity_over_elts():
    """Open terms and integer losses: ELTs A and B together give the sum of the
    year losses of A and B separately, exactly."""
    C = 4000
    ids, off, lay = W.random_case(15, 300, 120.0, C, 6, 700, integer_losses=True, max_int_loss=500, terms="open")
    a = W.LayerSpec(lay.elt_ids[:3], lay.elt_losses[:3], lay.ret[:3], lay.lim[:3], 0.0, np.inf, 0.0, np.inf)
    b = W.LayerSpec(lay.elt_ids[3:], lay.elt_losses[3:], lay.ret[3:], lay.lim[3:], 0.0, np.inf, 0.0, np.inf)
    ya = _run(ids, off, C, a)["ylt"]
    yb = _run(ids, off, C, b)["ylt"]
    yab = _run(ids, off, C, lay)["ylt"]
    assert np.array_equal(yab, ya + yb)


# ----------------------------------------------------------------------------- invariants
def _perturbed(lay, what, rng):
    J = lay.n_elts
    if what == "ret":
        return lay.with_terms(ret=lay.ret * rng.uniform(1.0, 2.0, J)), -1
    if what == "lim":
        return lay.with_terms(lim=lay.lim * rng.uniform(1.0, 2.0, J)), +1
    if what == "occ_ret":
        return lay.with_terms(occ_ret=lay.occ_ret * 1.7 + 1.0), -1
    if what == "occ_lim":
        return lay.with_terms(occ_lim=lay.occ_lim * 1.5), +1
    if what == "agg_ret":
        return lay.with_terms(agg_ret=lay.agg_ret * 1.5 + 1.0), -1
    if what == "agg_lim":
        return lay.with_terms(agg_lim=lay.agg_lim * 1.5), +1
    if what == "loss":
        l2 = W.LayerSpec(lay.elt_ids, [l * rng.uniform(1.0, 1.5, len(l)) for l in lay.elt_losses], lay.ret, lay.lim,
                         lay.occ_ret, lay.occ_lim, lay.agg_ret, lay.agg_lim)
        return l2, +1
    raise ValueError(what)


@pytest.mark.parametrize("what", ["ret", "lim", "occ_ret", "occ_lim", "agg_ret", "agg_lim", "loss"])
def test_monotone_in_terms_and_losses(what):
    C = 3000
    ids, off, lay = W.random_case(16, 400, 120.0, C, 4, 600)
    rng = np.random.default_rng(99)
    base = _run(ids, off, C, lay)["ylt"]
    lay2, sign = _perturbed(lay, what, rng)
    y2 = _run(ids, off, C, lay2)["ylt"]
    tol = 1e-12 * np.maximum(base, y2).max()
    if sign > 0:
        assert np.all(y2 >= base - tol)
    else:
        assert np.all(y2 <= base + tol)
    assert np.any(y2 != base)
    p1, t1 = oracle.pml_tvar(base, [10, 50])
    p2, t2 = oracle.pml_tvar(y2, [10, 50])
    assert np.all(sign * (p2 - p1) >= -tol) and np.all(sign * (t2 - t1) >= -tol)


def test_year_loss_is_order_invariant():
    C = 2000
    ids, off, lay = W.random_case(17, 200, 80.0, C, 3, 300, integer_losses=True)
    rng = np.random.default_rng(5)
    shuffled = ids.copy()
    for i in range(len(off) - 1):
        rng.shuffle(shuffled[off[i]:off[i + 1]])
    r0 = _run(ids, off, C, lay, want_event_net=True)
    r1 = _run(shuffled, off, C, lay, want_event_net=True)
    assert np.array_equal(r0["ylt"], r1["ylt"])
    # increments are non-negative and add up to the year loss
    assert np.all(r0["event_net"] >= 0)
    sums = np.add.reduceat(r0["event_net"], off[:-1]) * (np.diff(off) > 0)
    assert np.array_equal(sums, r0["ylt"])


def test_trials_are_independent():
    C = 2000
    ids, off, lay = W.random_case(18, 300, 60.0, C, 3, 300)
    full = _run(ids, off, C, lay)
    pick = np.array([5, 17, 200, 3, 299, 0])
    sub_ids = np.concatenate([ids[off[t]:off[t + 1]] for t in pick])
    sub_off = np.zeros(len(pick) + 1, np.int64)
    np.cumsum(np.diff(off)[pick], out=sub_off[1:])
    sub = _run(sub_ids, sub_off, C, lay)
    assert np.array_equal(sub["ylt"], full["ylt"][pick])


def test_fixed_length_equals_offsets_form():
    C = 1000
    ids, off, lay = W.random_case(19, 100, 50, C, 3, 200, fixed_len=True)
    a = _run(ids, off, C, lay)["ylt"]
    b = oracle.run_layer(ids, None, 100, 50, C, lay)["ylt"]
    assert np.array_equal(a, b)


def test_threads_do_not_change_results():
    C = 3000
    ids, off, lay = W.random_case(20, 2000, 40.0, C, 4, 500)
    a = _run(ids, off, C, lay, n_threads=1)["ylt"]
    b = _run(ids, off, C, lay, n_threads=4)["ylt"]
    assert np.array_equal(a, b)


# ----------------------------------------------------------------------------- risk metrics
@pytest.mark.parametrize("T,N", [(1000, 100), (1000, 250), (997, 10), (50, 50), (12, 1)])
def test_pml_tvar_on_a_permutation(T, N):
    """YLT a permutation of 1..T: the k-th largest is T-k+1 and the mean of the
    top k is T-(k-1)/2."""
    y = np.random.default_rng(T).permutation(np.arange(1, T + 1)).astype(np.float64)
    pml, tvar = oracle.pml_tvar(y, [N])
    k = T // N
    assert pml[0] == T - k + 1
    assert tvar[0] == T - (k - 1) / 2


def test_pml_tvar_order_relations():
    y = np.random.default_rng(3).lognormal(10, 2, 5000)
    y[y < np.quantile(y, 0.6)] = 0.0
    Ns = [2, 5, 10, 100, 250, 1000, 5000]
    pml, tvar = oracle.pml_tvar(y, Ns)
    assert np.all(tvar >= pml)
    assert np.all(np.diff(pml) >= 0) and np.all(np.diff(tvar) >= 0)
    assert pml[-1] == tvar[-1] == y.max()


def test_pml_tvar_rejects_short_ylt():
    with pytest.raises(oracle.OracleError):
        oracle.pml_tvar(np.ones(10), [100])


# ----------------------------------------------------------------------------- input checks
def test_oracle_rejects_bad_elts():
    ids = np.array([0, 1, 2], np.int32)
    off = np.array([0, 3], np.int64)
    dup = W.LayerSpec([np.array([1, 1], np.int32)], [np.array([1.0, 2.0])], np.zeros(1), np.full(1, np.inf),
                      0, np.inf, 0, np.inf)
    with pytest.raises(oracle.OracleError, match="-3"):
        _run(ids, off, 5, dup)
    rng_bad = W.LayerSpec([np.array([7], np.int32)], [np.array([1.0])], np.zeros(1), np.full(1, np.inf),
                          0, np.inf, 0, np.inf)
    with pytest.raises(oracle.OracleError, match="-2"):
        _run(ids, off, 5, rng_bad)


# ----------------------------------------------------------------------------- occurrence basis
def test_occ_max_closed_forms_and_bounds():
    """Open terms: the largest occurrence loss of a trial is the largest total
    loss (over the ELTs) of its events.  Counting form: 1 if the trial holds an
    event present in some ELT, else 0.  Always 0 <= occ_max <= min(S, FT2 limit)."""
    C = 4000
    ids, off, lay = W.random_case(12, 400, 60.0, C, 4, 700, integer_losses=True, max_int_loss=500, terms="open",
                                  empty_frac=0.05)
    w, present = _presence_and_totals(lay, C)
    r = _run(ids, off, C, lay, want_occ_max=True)
    expect = np.array([w[ids[off[i]:off[i + 1]]].max() if off[i + 1] > off[i] else 0.0 for i in range(len(off) - 1)])
    assert np.array_equal(r["occ_max"], expect)
    ids, off, lay = W.random_case(13, 400, 20.0, C, 3, 300, integer_losses=True, terms="counting", empty_frac=0.1)
    _, present = _presence_and_totals(lay, C)
    r = _run(ids, off, C, lay, want_occ_max=True)
    expect = np.array([float(present[ids[off[i]:off[i + 1]]].any()) for i in range(len(off) - 1)])
    assert np.array_equal(r["occ_max"], expect)
    ids, off, lay = W.random_case(14, 300, 80.0, C, 5, 900)
    r = _run(ids, off, C, lay, want_occ_max=True)
    assert np.all(r["occ_max"] >= 0.0)
    assert np.all(r["occ_max"] <= lay.occ_lim)
    assert np.all(r["occ_max"] <= r["occ_sum"])
    # order of events inside a trial does not matter
    rng = np.random.default_rng(5)
    pid = ids.copy()
    for i in range(len(off) - 1):
        rng.shuffle(pid[off[i]:off[i + 1]])
    assert np.array_equal(_run(pid, off, C, lay, want_occ_max=True)["occ_max"], r["occ_max"])


# ----------------------------------------------------------------------------- roll-up of layers into programs
def _golden_layer2(g):
    l2 = g["rollup"]["layer2"]
    return W.LayerSpec([np.array(e["ids"], np.int32) for e in l2["elts"]],
                       [np.array(e["losses"], np.float64) for e in l2["elts"]],
                       np.array([e["ret"] for e in l2["elts"]], np.float64),
                       np.array([e["lim"] for e in l2["elts"]], np.float64),
                       l2["occ_ret"], l2["occ_lim"], l2["agg_ret"], l2["agg_lim"])


def test_rollup_worked_example():
    """Hand-worked second layer, program and portfolio (integers: exact)."""
    g = json.load(open(GOLD))
    ids, off = _flatten(g["trials"])
    y1 = _run(ids, off, g["catalog_size"], _golden_layer(g))["ylt"]
    r2 = _run(ids, off, g["catalog_size"], _golden_layer2(g))
    ru = g["rollup"]
    assert r2["occ_sum"].tolist() == ru["layer2"]["occ_sum"]
    assert r2["ylt"].tolist() == ru["layer2"]["ylt"]
    p1, p2 = oracle.rollup([y1, r2["ylt"], r2["ylt"]], [0, 0, 1], 2)
    assert p1.tolist() == ru["program_p1_ylt"]
    assert p2.tolist() == ru["program_p2_ylt"]
    (pf,) = oracle.rollup([p1, p2], [0, 0], 1)
    assert pf.tolist() == ru["portfolio_ylt"]
    for N, (pml, tvar) in ru["program_p1_pml_tvar"].items():
        op, ot = oracle.pml_tvar(p1, [float(N)])
        assert (op[0], ot[0]) == (pml, tvar)


def test_rollup_of_open_layers_is_the_union_layer():
    """Open terms and integer losses: the roll-up of layers over ELT sets A and
    B is the year loss of one layer over A and B together, exactly (an
    independent route through the pass itself)."""
    C = 4000
    ids, off, lay = W.random_case(21, 300, 120.0, C, 7, 700, integer_losses=True, max_int_loss=500, terms="open")
    parts = [(0, 2), (2, 3), (3, 7)]
    ylts = []
    for a, b in parts:
        part = W.LayerSpec(lay.elt_ids[a:b], lay.elt_losses[a:b], lay.ret[a:b], lay.lim[a:b], 0.0, np.inf, 0.0, np.inf)
        ylts.append(_run(ids, off, C, part)["ylt"])
    whole = _run(ids, off, C, lay)["ylt"]
    (prog,) = oracle.rollup(ylts, [0, 0, 0], 1)
    assert np.array_equal(prog, whole)


def test_rollup_groups_and_tvar_subadditivity():
    """A group without inputs is zero, a one-input group is its input, and the
    mean of the k largest year losses of a sum is at most the sum of the
    inputs' means (true of any top-k mean)."""
    rng = np.random.default_rng(5)
    T = 4000
    ylts = []
    for i in range(5):
        y = rng.lognormal(11, 1.5, T)
        y[rng.random(T) < 0.5] = 0.0
        ylts.append(y)
    groups = [1, 1, 3, 1, 1]
    out = oracle.rollup(ylts, groups, 4)
    assert not out[0].any() and not out[2].any()
    assert np.array_equal(out[3], ylts[2])
    Ns = [2.0, 10.0, 100.0, 250.0, 1000.0]
    _, tsum = oracle.pml_tvar(out[1], Ns)
    parts = [oracle.pml_tvar(ylts[i], Ns)[1] for i in (0, 1, 3, 4)]
    assert np.all(tsum <= np.sum(parts, axis=0) * (1 + 1e-12))
    with pytest.raises(oracle.OracleError):
        oracle.rollup(ylts, [0, 0, 0, 0, 4], 4)
