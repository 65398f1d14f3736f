"""The oracle pins must catch plausible mistakes.

Each case copies the oracle's C source into a temporary directory, plants one
mistake by text substitution, compiles it, and checks that the hand-worked
example or the exact-rational brute force rejects the mutant.  The committed
oracle is never modified.
"""
import json
import os
import subprocess

import numpy as np
import pytest

from exact_ref import exact_layer
from oracle import oracle
from paper_1412_4556_amd import workloads as W
from test_oracle_pins import GOLD, _flatten, _golden_layer

SRC = os.path.join(os.path.dirname(oracle.__file__), "ara_oracle.c")
U64 = 2.0 ** -53

MUTANTS = {
    "ft1_dropped": [("e += clamp_excess(l, ret[j], lim[j]);", "e += l;")],
    "ft1_swapped": [("e += clamp_excess(l, ret[j], lim[j]);", "e += clamp_excess(l, lim[j], ret[j]);")],
    "ft2_dropped": [("double o = clamp_excess(e, occ_ret, occ_lim);", "double o = e;")],
    "ft3_per_event": [("S += o;", "S += clamp_excess(o, agg_ret, agg_lim);")],
    "event_loss_not_reset": [("double S = 0.0, G = 0.0, A_prev = 0.0, M = 0.0;",
                              "double S = 0.0, G = 0.0, A_prev = 0.0, M = 0.0, ec = 0.0;"),
                             ("double e = 0.0;", "double e = ec;"),
                             ("double o = clamp_excess(e, occ_ret, occ_lim);",
                              "double o = clamp_excess(e, occ_ret, occ_lim); ec = e;")],
    "wrong_lookup_index": [("double l = table[(size_t)j * C + (size_t)E];",
                            "double l = table[(size_t)j * C + (size_t)((E + 1) % (int32_t)C)];")],
    "retention_sign": [("double v = x - retention;", "double v = x + retention;")],
    "missing_max_zero": [("if (v < 0.0) v = 0.0;", "")],
    "missing_limit": [("if (v > limit) v = limit;", "")],
    "last_event_dropped": [("for (int64_t k = begin; k < end; ++k)", "for (int64_t k = begin; k + 1 < end; ++k)")],
    "agg_retention_dropped": [("ylt[i] = clamp_excess(S, agg_ret, agg_lim);", "ylt[i] = clamp_excess(S, 0.0, agg_lim);")],
    "elt_order_offset": [("table[(size_t)j * C + (size_t)e] = elt_losses[pos];",
                          "table[(size_t)j * C + (size_t)e] = elt_losses[pos > 0 ? pos - 1 : pos];")],
    "occ_max_before_ft2": [("if (o > M) M = o;", "if (e > M) M = e;")],
    "occ_max_last_not_largest": [("if (o > M) M = o;", "M = o;")],
}


def _build_mutant(tmp_path, name, subs):
    src = open(SRC).read()
    for a, b in subs:
        assert a in src, (name, a)
        src = src.replace(a, b)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"lib{name}.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-o", str(so), str(c)])
    return oracle.load_library(str(so))


def _pins_hold(lib) -> bool:
    g = json.load(open(GOLD))
    lay = _golden_layer(g)
    ids, off = _flatten(g["trials"])
    try:
        r = oracle.run_layer(ids, off, len(off) - 1, 0, g["catalog_size"], lay, lib=lib, want_event_net=True)
    except oracle.OracleError:
        return False
    if r["ylt"].tolist() != g["ylt"] or r["occ_sum"].tolist() != g["occ_sum"]:
        return False
    rm = oracle.run_layer(ids, off, len(off) - 1, 0, g["catalog_size"], lay, lib=lib, want_occ_max=True)
    if rm["occ_max"].tolist() != g["occ_max"]:
        return False
    ro = oracle.run_layer(ids, off, len(off) - 1, 0, g["catalog_size"], lay.open_terms(), lib=lib)
    if ro["ylt"].tolist() != g["open_terms_ylt"]:
        return False
    for seed in (1, 4, 7):
        ids, off, lay = W.random_case(seed, 30, 10.0, 25, 3, 10, integer_losses=(seed == 4), empty_frac=0.1)
        r = oracle.run_layer(ids, off, len(off) - 1, 0, 25, lay, lib=lib)
        ey, _, eG, _ = exact_layer(ids, off, lay)
        for i in range(len(off) - 1):
            bound = (int(off[i + 1] - off[i]) + 8) * U64 * float(eG[i]) * 1.01
            if abs(r["ylt"][i] - float(ey[i])) > bound:
                return False
    return True


def test_unmutated_copy_passes(tmp_path):
    assert _pins_hold(_build_mutant(tmp_path, "identity", []))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, name):
    assert not _pins_hold(_build_mutant(tmp_path, name, MUTANTS[name]))
