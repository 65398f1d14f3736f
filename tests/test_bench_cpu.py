"""The benchmark's CPU-baseline leg (no GPU needed): the oracle's timing, its
single-thread figure, and the parity report it makes against a given YLT."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
from oracle import oracle  # noqa: E402
from paper_1412_4556_amd import workloads as W  # noqa: E402


def test_cpu_baseline_reports_parity_against_a_given_ylt():
    wl = W.plain_tiny()
    spec = wl.layers[0]
    ids, off = W.yet_subset(wl.yet, np.arange(wl.yet.n_trials))
    ref = oracle.run_layer(ids, off, wl.yet.n_trials, 0, wl.yet.catalog_size, spec, n_threads=4)
    y = ref["ylt"].copy()
    y[7] += 1e-13 * ref["gross"][7]  # within 1e-12 * G
    y[9] += 1e-9 * ref["gross"][9]   # beyond it
    rps = [100.0, 250.0]
    pml, tvar = oracle.pml_tvar(y, rps)
    res = bench.cpu_baseline(wl, spec, 0.2, gpu_ylt=y, gpu_pml_tvar=(pml, tvar), rps=rps)
    assert res["kind"] == "oracle" and res["unit"] == "lookups/s" and res["value"] > 0 and res["cores"] >= 1
    assert res["single_thread"]["cores"] == 1 and res["single_thread"]["value"] > 0
    par = res["parity"]
    assert par["trials_compared"] == wl.yet.n_trials
    assert par["trials_over_1e-12_gross"] == 1
    assert par["bitwise_equal_trials"] == wl.yet.n_trials - 2
    assert 9e-10 < par["max_err_over_gross"] < 1.1e-9
    assert "pml_max_rel_err" in par and "tvar_max_rel_err" in par
