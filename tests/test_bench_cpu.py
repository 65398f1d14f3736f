"""The benchmark's CPU-baseline leg (no GPU needed): the oracle's timing, its
single-thread figure, the host description, and the error reports it makes
against given YLTs (FP64 and FP32C on the timed workload's sample, and the
precision workload in full)."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
from oracle import oracle  # noqa: E402
from paper_1412_4556_amd import workloads as W  # noqa: E402


def test_cpu_baseline_reports_parity_against_given_ylts():
    wl = W.plain_tiny()
    spec = wl.layers[0]
    ids, off = W.yet_subset(wl.yet, np.arange(wl.yet.n_trials))
    ref = oracle.run_layer(ids, off, wl.yet.n_trials, 0, wl.yet.catalog_size, spec, n_threads=4)
    y = ref["ylt"].copy()
    y[7] += 1e-13 * ref["gross"][7]  # within 1e-12 * G
    y[9] += 1e-9 * ref["gross"][9]   # beyond it
    y32 = ref["ylt"] * (1 + 3e-7)    # an FP32C-sized error on every trial
    rps = [100.0, 250.0]
    pml, tvar = oracle.pml_tvar(y, rps)
    pml32, tvar32 = oracle.pml_tvar(y32, rps)
    # the precision workload: the oracle's own tables, one of them perturbed
    w = W.precision_poisson()
    pids, poff = W.yet_subset(w.yet, np.arange(w.yet.n_trials))
    runs = {}
    for lay in w.layers:
        r = oracle.run_layer(pids, poff, w.yet.n_trials, 0, w.yet.catalog_size, lay, n_threads=4)
        runs[(lay.name, "fp64_fused")] = (r["ylt"], oracle.pml_tvar(r["ylt"], list(w.return_periods)))
        yp = r["ylt"] * (1 + 2e-7)
        runs[(lay.name, "fp32c_fused")] = (yp, oracle.pml_tvar(yp, list(w.return_periods)))
    res = bench.cpu_baseline(wl, spec, 0.2, gpu_ylt=y, gpu_pml_tvar=(pml, tvar), rps=rps, gpu_ylt32=y32,
                             gpu_pml_tvar32=(pml32, tvar32), precision=(w, pids, poff, runs))
    assert res["kind"] == "oracle" and res["unit"] == "lookups/s" and res["value"] > 0 and res["cores"] >= 1
    assert res["host"]["threads_used"] == res["cores"] and res["host"]["logical_cpus"] >= 1
    assert res["single_thread"]["cores"] == 1 and res["single_thread"]["value"] > 0
    par = res["parity"]
    assert par["trials_compared"] == wl.yet.n_trials
    f64 = par["fp64"]
    assert f64["trials_over_tol_gross"] == 1
    assert f64["bitwise_equal_trials"] == wl.yet.n_trials - 2
    assert 9e-10 < f64["max_err_over_gross"] < 1.1e-9
    assert len(f64["pml_rel_err"]) == 2 and len(f64["tvar_rel_err"]) == 2
    f32 = par["fp32c"]
    assert abs(f32["max_rel_err"] - 3e-7) < 1e-9 and abs(f32["mean_rel_err"] - 3e-7) < 1e-9
    assert f32["trials_over_tol_gross"] == 0
    assert all(abs(v - 3e-7) < 1e-9 for v in f32["pml_rel_err"])
    pw = res["precision_workload"]["layers"]
    for lay in w.layers:
        assert pw[lay.name]["fp64_fused"]["max_rel_err"] == 0.0
        assert pw[lay.name]["fp64_fused"]["bitwise_equal_trials"] == w.yet.n_trials
        assert abs(pw[lay.name]["fp32c_fused"]["max_rel_err"] - 2e-7) < 1e-9
