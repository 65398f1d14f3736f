#!/usr/bin/env python3
"""Benchmark of the Aggregate Risk Analysis trial pass on one MI355X.

Workload: the paper's experiment shape (Section IV) -- a YET of 1,000,000
trials x 1,000 events over a 2,000,000-event catalogue and one layer of 16
ELTs x 20,000 events (lognormal(10, 2) losses, per-ELT retention/limit at the
10th/90th percentile, occurrence 1e5/1e7, aggregate 1e6/5e7), synthetic and
seeded, resident in HBM before timing starts.

One step = the layer's fused table built on the GPU from its 16 ELTs, which
are resident in HBM (steps 1-3 of the method for every catalogue event: the
per-ELT terms, the sum over the ELTs, the occurrence terms), the trial pass
over every trial (the cumulative sum and the aggregate terms, YLT written to
HBM), and PML/TVaR at 1-in-100 and 1-in-250 returned to the host.  The timed
steps are pipelined: step i + 1 is queued before step i's PML/TVaR is read on
the host (the line also gives the time per step one at a time).  Prints one
JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1412_4556_amd", "csrc", "ara_kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "k_trial_pass_fused_counters_plain_1M_trials_x_1000_events_16_elts.md")


def measured_traffic():
    """HBM bytes per launch of the fused pass from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    import re

    try:
        text = open(COUNTERS).read()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
        if f"kernel_source_sha256_16: {sha}" not in text:
            return None
        return float(re.search(r"traffic_bytes_per_launch: ([0-9.e+]+)", text).group(1))
    except (OSError, AttributeError):
        return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def host_cpus():
    """What the host offers this process: logical CPUs, the CPUs it may run
    on, and the thread count the machine sets for OpenMP (on a host shared
    by several GPUs: the CPU share of one GPU)."""
    try:
        aff = len(os.sched_getaffinity(0))
    except Exception:
        aff = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    return {"logical_cpus": os.cpu_count(), "affinity_cpus": aff, "omp_num_threads": omp,
            "cpu_model": cpu_model()}


def host_threads():
    """Threads of the CPU baseline: every CPU this process may run on, capped
    by OMP_NUM_THREADS when the machine sets it (a GPU's share of the host)."""
    info = host_cpus()
    n = info["affinity_cpus"]
    if info["omp_num_threads"]:
        try:
            n = min(n, int(info["omp_num_threads"]))
        except ValueError:
            pass
    return max(1, n)


def time_layer(A, torch, yet, lay, ylt, steps, warmup, rps, with_pml=True):
    """Wall time per step and mean kernel time (HIP events on the launch stream)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        A.run_layer(yet, lay, out=ylt)
        if with_pml:
            A.pml_tvar(ylt, rps)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    res = None
    for i in range(steps):
        evs[i][0].record(stream)
        A.run_layer(yet, lay, out=ylt)
        evs[i][1].record(stream)
        if with_pml:
            res = A.pml_tvar(ylt, rps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms = [a.elapsed_time(b) for a, b in evs]
    return (t1 - t0) * 1e3 / steps, sum(k_ms) / len(k_ms), min(k_ms), res


def time_step(A, torch, yet, pool, spec, ylt, steps, warmup, rps, pipelined=True):
    """The headline step (fused table from the device-resident ELTs, trial
    pass, PML/TVaR to the host).  Returns the wall time per step, the mean
    build and pass times (HIP events on the launch stream), the fastest pass
    and the last step's PML/TVaR.

    pipelined: step i + 1 is queued before step i's PML/TVaR is read on the
    host (PML/TVaR into device memory with the entry point that allocates
    nothing, an asynchronous copy into pinned host memory and an event per
    step; two table slots of the pool alternate), so the GPU does not wait
    for the host between steps.  Otherwise every step ends with the
    synchronous ara_pml_tvar before the next one is issued."""
    import numpy as np

    stream = torch.cuda.current_stream()
    idx = np.arange(spec.n_elts, dtype=np.int32)
    r = len(rps)
    dev = torch.empty(2 * r, dtype=torch.float64, device="cuda")
    host = [torch.empty(2 * r, dtype=torch.float64, pin_memory=True) for _ in range(2)]
    done = [torch.cuda.Event() for _ in range(2)]

    def launch(i, ev=None):
        if ev:
            ev[0].record(stream)
        lay = pool.layer(idx, spec.ret, spec.lim, spec.occ_ret, spec.occ_lim, spec.agg_ret, spec.agg_lim,
                         stream=stream)
        if ev:
            ev[1].record(stream)
        A.run_layer(yet, lay, out=ylt, stream=stream)
        if ev:
            ev[2].record(stream)
        if not pipelined:
            res = A.pml_tvar(ylt, rps, stream=stream)
            lay.close()  # the slot's next build is queued behind this pass on the same stream
            return res
        A.pml_tvar_many_noalloc([ylt], rps, dev[:r], dev[r:], stream=stream)
        with torch.cuda.stream(stream):
            host[i % 2].copy_(dev, non_blocking=True)
        done[i % 2].record(stream)
        return (i, lay)

    def finish(p):
        i, lay = p
        done[i % 2].synchronize()
        out = host[i % 2].numpy().copy()
        lay.close()
        return out[:r], out[r:]

    def run(n, evs=None):
        res, prev = None, None
        for i in range(n):
            p = launch(i, evs[i] if evs else None)
            if not pipelined:
                res = p
                continue
            if prev is not None:
                res = finish(prev)
            prev = p
        if prev is not None:
            res = finish(prev)
        return res

    run(warmup)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    res = run(steps, evs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b_ms = [e[0].elapsed_time(e[1]) for e in evs]
    p_ms = [e[1].elapsed_time(e[2]) for e in evs]
    return (t1 - t0) * 1e3 / steps, sum(b_ms) / steps, sum(p_ms) / steps, min(p_ms), res


def error_report(y, ref, tol, gpu_pml_tvar=None, rps=()):
    """Error of a GPU year loss table against the oracle's, per trial:
    relative to the oracle's year loss (over trials where it is > 0), to the
    trial's gross looked-up loss G and to its cumulative occurrence loss S;
    and, with the GPU's PML/TVaR, their relative error against the oracle's
    values from its own table."""
    import numpy as np

    from oracle import oracle

    err = np.abs(np.asarray(y) - ref["ylt"])
    pos = ref["ylt"] > 0
    rel = err[pos] / ref["ylt"][pos]
    spos = ref["occ_sum"] > 0
    out = {"trials": int(len(err)),
           "max_rel_err": float(rel.max()) if pos.any() else 0.0,
           "mean_rel_err": float(rel.mean()) if pos.any() else 0.0,
           "max_err_over_gross": float((err / np.maximum(ref["gross"], 1e-300)).max()) if len(err) else 0.0,
           "max_err_over_S": float((err[spos] / ref["occ_sum"][spos]).max()) if spos.any() else 0.0,
           "trials_over_tol_gross": int((err > tol * ref["gross"]).sum()),
           "bitwise_equal_trials": int((np.asarray(y) == ref["ylt"]).sum())}
    if gpu_pml_tvar is not None:
        op, ot = oracle.pml_tvar(ref["ylt"], rps)
        gp, gt = gpu_pml_tvar
        nz = lambda a: np.where(a == 0, 1.0, np.abs(a))
        out["pml_rel_err"] = [float(v) for v in np.abs(np.asarray(gp) - op) / nz(op)]
        out["tvar_rel_err"] = [float(v) for v in np.abs(np.asarray(gt) - ot) / nz(ot)]
    return out


def precision_runs(A, W, torch):
    """The precision workload (10k Poisson(1000) trials, 4 ELTs of Pareto
    losses, two term sets) through the GPU in both precisions: host copies
    of every YLT and its PML/TVaR, for the CPU leg's comparison."""
    import numpy as np

    w = W.precision_poisson()
    ids, off = W.yet_subset(w.yet, np.arange(w.yet.n_trials))
    yet = A.yet_from_numpy(ids, off, w.yet.n_trials, w.yet.catalog_size)
    out = {}
    for lay_spec in w.layers:
        for prec, layout in (("fp64", "fused"), ("fp32c", "fused"), ("fp32c", "compact")):
            lay = A.Layer(yet, lay_spec, prec, layout)
            y = A.run_layer(yet, lay)
            pt = A.pml_tvar(y, list(w.return_periods))
            out[(lay_spec.name, f"{prec}_{layout}")] = (y.cpu().numpy(), pt)
            lay.close()
    yet.close()
    return w, ids, off, out


def cpu_baseline(wl, spec, target_s, gpu_ylt=None, gpu_pml_tvar=None, rps=(), gpu_ylt32=None,
                 gpu_pml_tvar32=None, precision=None, single_full=False):
    """The oracle on a bounded sample of the same workload, on the host cores;
    with the GPU's YLT of the timed pass, also the GPU's error on the sample
    (|y - y_oracle| / G per trial, G the trial's gross looked-up loss) and,
    when the sample is the whole workload, PML/TVaR against the oracle's."""
    import numpy as np

    from oracle import oracle
    from paper_1412_4556_amd import workloads as W

    threads = host_threads()
    cpus = host_cpus()
    J = spec.n_elts

    def run(n, n_threads=threads):
        ids, off = W.yet_subset(wl.yet, np.arange(n))
        t = time.perf_counter()
        r = oracle.run_layer(ids, off, n, 0, wl.yet.catalog_size, spec, n_threads=n_threads)
        return time.perf_counter() - t, int(off[-1]), r

    probe = min(2000 * threads, wl.yet.n_trials)
    dt, ev, _ = run(probe)
    n = int(min(wl.yet.n_trials, max(probe, probe * target_s / max(dt, 1e-3))))
    dt, ev, ref = run(n)
    res = {"value": ev * J / dt, "unit": "lookups/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n} of {wl.yet.n_trials} trials ({ev} trial-events x {J} ELTs), FP64, "
                     f"OpenMP over trials, {dt:.1f} s incl. direct-table build",
           "cpu_model": cpus["cpu_model"], "seconds": dt,
           "host": {**cpus, "threads_used": threads,
                    "threads_rule": "every CPU of the process's affinity, capped by OMP_NUM_THREADS when set "
                                    "(the CPU share of one GPU on a shared host)"}}
    # the same loop on one core (the paper's sequential form), on a smaller sample
    n1 = int(min(wl.yet.n_trials, max(100, n / threads / 4)))
    dt1, ev1, _ = run(n1, 1)
    res["single_thread"] = {"value": ev1 * J / dt1, "unit": "lookups/s", "cores": 1,
                            "sample": f"first {n1} trials ({ev1} trial-events x {J} ELTs), {dt1:.1f} s "
                                      f"incl. direct-table build"}
    if single_full:
        # the whole workload on one core (the paper's sequential form; minutes),
        # in eight consecutive blocks of trials, each reported as it ends
        n_blk = 8
        edges = np.linspace(0, wl.yet.n_trials, n_blk + 1).astype(np.int64)
        dtf, evf = 0.0, 0
        for k in range(n_blk):
            ids, off = W.yet_subset(wl.yet, np.arange(edges[k], edges[k + 1]))
            t = time.perf_counter()
            oracle.run_layer(ids, off, int(edges[k + 1] - edges[k]), 0, wl.yet.catalog_size, spec, n_threads=1)
            dtf += time.perf_counter() - t
            evf += int(off[-1])
            log(f"single-thread oracle over the whole workload: block {k + 1}/{n_blk}, {dtf:.1f} s so far")
        res["single_thread_full"] = {"value": evf * J / dtf, "unit": "lookups/s", "cores": 1, "seconds": dtf,
                                     "sample": f"all {wl.yet.n_trials} trials ({evf} trial-events x {J} ELTs), "
                                               f"in {n_blk} consecutive blocks of trials, each incl. its "
                                               f"direct-table build"}
    # and whole on the two small workloads (parity: 10k x 1000 events, 4 ELTs;
    # precision: 10k Poisson(1000) trials, 4 ELTs of Pareto losses)
    small = {}
    for w in (W.plain_tiny(), W.precision_poisson()):
        ids, off = W.yet_subset(w.yet, np.arange(w.yet.n_trials))
        lay = w.layers[0]
        t = time.perf_counter()
        oracle.run_layer(ids, off, w.yet.n_trials, 0, w.yet.catalog_size, lay, n_threads=1)
        dts = time.perf_counter() - t
        small[w.name] = {"value": int(off[-1]) * lay.n_elts / dts, "unit": "lookups/s", "seconds": dts}
    res["single_thread_small_workloads"] = small
    if gpu_ylt is not None:
        whole = n == wl.yet.n_trials
        par = {"trials_compared": n,
               "fp64": error_report(gpu_ylt[:n], ref, 1e-12, gpu_pml_tvar if whole else None, rps)}
        if gpu_ylt32 is not None:
            par["fp32c"] = error_report(gpu_ylt32[:n], ref, 1e-6, gpu_pml_tvar32 if whole else None, rps)
        res["parity"] = par
    if precision is not None:
        # the precision workload in full: FP64 and FP32C against the oracle
        w, ids, off, runs = precision
        rp = list(w.return_periods)
        rep = {}
        for lay_spec in w.layers:
            ref = oracle.run_layer(ids, off, w.yet.n_trials, 0, w.yet.catalog_size, lay_spec, n_threads=threads)
            rep[lay_spec.name] = {form: error_report(y, ref, 1e-12 if form.startswith("fp64") else 1e-6, pt, rp)
                                  for (name, form), (y, pt) in runs.items() if name == lay_spec.name}
        res["precision_workload"] = {"workload": w.name, "return_periods": rp, "layers": rep}
    return res


def batch_leg(A, W, torch, n_trials, steps, precision="fp64"):
    """64 layers over one YET of Poisson(1000)-length trials: one batched pass
    (records built once, launch shape tuned, graph replayed) against 64
    sequential single-layer passes over the same YET."""
    import numpy as np

    wl = W.batch_layers(n_trials)
    log(f"batch leg: generating YET of {n_trials} Poisson(1000) trials, {len(wl.layers)} layers")
    ids, off = W.yet_full(wl.yet)
    t_ids = torch.from_numpy(ids).cuda()
    t_off = torch.from_numpy(off).cuda()
    n_events = len(ids)
    del ids
    yet = A.Yet(t_ids, t_off, wl.yet.n_trials, wl.yet.catalog_size)
    t0 = time.perf_counter()
    layers = [A.Layer(yet, s, precision, "fused") for s in wl.layers]
    layer_build_s = time.perf_counter() - t0
    T = wl.yet.n_trials
    outs = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in layers]
    seq = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in layers]
    t0 = time.perf_counter()
    batch = A.Batch(yet, layers)
    batch_build_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    batch.run(outs)
    torch.cuda.synchronize()
    first_run_ms = (time.perf_counter() - t0) * 1e3
    stream = torch.cuda.current_stream()

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(n):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    batch_ms = timed(lambda: batch.run(outs), steps)
    seq_ms = timed(lambda: [A.run_layer(yet, l, out=o) for l, o in zip(layers, seq)], max(1, steps // 2))
    same = all(torch.equal(a, b) for a, b in zip(outs, seq))
    # small batches (dense records, one pass per group of 4 layers) of the
    # first n layers against their single-layer passes
    single = [timed(lambda l=l, o=o: A.run_layer(yet, l, out=o), 3) for l, o in zip(layers[:16], seq[:16])]
    small = []
    for n in (2, 4, 8, 16):
        sb = A.Batch(yet, layers[:n])
        so = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in range(n)]
        sb.run(so)
        ms = timed(lambda: sb.run(so), 3)
        small.append({"n_layers": n, "batched_ms": ms, "single_passes_ms": sum(single[:n]),
                      "speedup": sum(single[:n]) / ms, "launch_group_chunks": sb.launch_group,
                      "bitwise_equal_to_single": all(torch.equal(a, b) for a, b in zip(so, seq[:n]))})
        log(f"batch leg: {n} layers batched {ms:.2f} ms vs {sum(single[:n]):.2f} ms as single passes")
        sb.close()
        del so
    J = [s.n_elts for s in wl.layers]
    lt = len(layers) * T
    log(f"batch leg: batched {batch_ms:.2f} ms vs sequential {seq_ms:.2f} ms ({seq_ms / batch_ms:.1f}x), "
        f"bitwise equal {same}")
    res = {"workload": wl.name, "n_layers": len(layers), "n_trials": T, "n_events": n_events,
           "elts_total": int(sum(J)), "precision": precision,
           "batched_ms": batch_ms, "sequential_ms": seq_ms, "speedup": seq_ms / batch_ms,
           "batched_layer_trials_per_s": lt / (batch_ms * 1e-3),
           "sequential_layer_trials_per_s": lt / (seq_ms * 1e-3),
           "batched_lookups_per_s": float(sum(J)) * n_events / (batch_ms * 1e-3),
           "launch_config": list(batch.launch_config), "launch_group_chunks": batch.launch_group,
           "record_bytes": batch.device_bytes,
           "batch_build_ms": batch_build_ms, "first_run_ms_incl_tuning": first_run_ms,
           "layer_build_s_total": layer_build_s, "bitwise_equal_to_sequential": bool(same),
           "small_batches": small}
    # programs of 8 layers each, then the portfolio of the 8 programs, and
    # their PML/TVaR (100 and 250 years)
    progs = [torch.empty(T, dtype=torch.float64, device="cuda") for _ in range(8)]
    pfolio = [torch.empty(T, dtype=torch.float64, device="cuda")]
    groups = [l * 8 // len(layers) for l in range(len(layers))]

    def roll():
        A.rollup(outs, groups, 8, out=progs)
        A.rollup(progs, [0] * 8, 1, out=pfolio)

    roll_ms = timed(roll, 5)
    ppml, ptvar = A.pml_tvar_many(progs + pfolio, [100.0, 250.0])
    roll_bytes = (len(layers) + 8 + 8 + 1) * T * 8
    res["rollup"] = {"programs": 8, "layers_per_program": len(layers) // 8, "ms": round(roll_ms, 4),
                     "gbps": round(roll_bytes / (roll_ms * 1e-3) / 1e9, 1),
                     "program_pml": ppml[:8].tolist(), "program_tvar": ptvar[:8].tolist(),
                     "portfolio_pml": ppml[8].tolist(), "portfolio_tvar": ptvar[8].tolist()}
    log(f"batch leg: roll-up into 8 programs and a portfolio {roll_ms:.3f} ms")
    batch.close()
    for l in layers:
        l.close()
    yet.close()
    del t_ids, t_off, outs, seq, progs, pfolio
    torch.cuda.empty_cache()
    return res


def serving_leg(A, W, torch, n_trials, rates, max_layers=128, n_queries=1000, budget_s=330.0):
    """Poisson-arriving ad hoc layer queries (1..16 ELTs of a 256-ELT pool,
    random occurrence/aggregate terms) against a resident YET of Poisson(1000)
    trials: continuous batching against one query at a time."""
    from paper_1412_4556_amd import serve as S

    y, pool = W.serving_pool(n_trials)
    log(f"serving leg: generating YET of {n_trials} Poisson(1000) trials, pool of {len(pool.ids)} ELTs")
    ids, off = W.yet_full(y)
    t_ids = torch.from_numpy(ids).cuda()
    t_off = torch.from_numpy(off).cuda()
    del ids
    yet = A.Yet(t_ids, t_off, y.n_trials, y.catalog_size)
    P = A.Pool(yet, pool.ids, pool.losses, "fp64", max_layers=max_layers)
    srv = S.BatchingServer(yet, P)
    min_batch = srv.warm_up(W.serving_queries(pool, srv.max_batch, 1e6, stream=999))
    log(f"serving leg: record pass wins from {min_batch} layers per group")
    warm = W.serving_queries(pool, 40, 2000.0, stream=998)
    srv.serve(S.make_queries(warm))
    S.serve_one_at_a_time(yet, P, S.make_queries(warm))
    out = []
    t_start = time.perf_counter()
    # fastest rates first; a rate's two runs take about 2 n / rate seconds,
    # and a run that would not fit the time budget gets fewer queries (said
    # in its record)
    for i, rate in sorted(enumerate(rates), key=lambda x: -x[1]):
        n = n_queries
        left = budget_s - (time.perf_counter() - t_start)
        if 2.0 * n / rate > left:
            n = max(100, int(left * rate / 2.0))
        items = W.serving_queries(pool, n, rate, stream=i)
        b = srv.serve(S.make_queries(items), progress=lambda k: log(f"serving {rate:.0f}/s batched: {k}/{n}"))
        log(f"serving {rate:.0f}/s batched: done")
        o = S.serve_one_at_a_time(yet, P, S.make_queries(items),
                                  progress=lambda k: log(f"serving {rate:.0f}/s one at a time: {k}/{n}"))
        log(f"serving {rate:>6.0f}/s x {n}: batched p50 {b['p50_ms']:.2f} p99 {b['p99_ms']:.2f} ms "
            f"{b['layers_per_s']:.0f} layers/s (mean batch {b['mean_batch']:.1f}); one-at-a-time p50 "
            f"{o['p50_ms']:.2f} p99 {o['p99_ms']:.2f} ms {o['layers_per_s']:.0f} layers/s")
        out.append({"rate_per_s": rate, "n_queries": n, "reduced_for_time": n < n_queries, "batched": b,
                    "one_at_a_time": o})
    res = {"workload": f"serving_{n_trials}_trials_pool_{len(pool.ids)}_elts", "n_trials": y.n_trials,
           "n_events": int(off[-1]), "pool_elts": len(pool.ids), "layer_slots": max_layers,
           "pool_device_bytes": P.device_bytes, "return_periods": [100.0, 250.0],
           "record_pass_from_layers": min_batch, "rates": out}
    srv.close()
    P.close()
    yet.close()
    del t_ids, t_off
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32c"])
    ap.add_argument("--trials", type=int, default=1_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-single-thread-full", action="store_true",
                    help="also time the oracle on one core over the whole workload (minutes)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-trials", type=int, default=1_000_000)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-trials", type=int, default=500_000)
    ap.add_argument("--serving-rates", default="10,30,100,300,1000,3000")
    ap.add_argument("--serving-queries", type=int, default=1000, help="queries per rate (after warm-up)")
    ap.add_argument("--serving-budget-s", type=float, default=330.0,
                    help="wall-clock budget of the serving sweep; slow rates past it run fewer queries")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB 5 times (counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration > 0:
        import torch

        n = int(args.copy_calibration * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n * 4, "launches": 5}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (trials would shard by trial "
              "range across GPUs, with one exchange of the local top-k for PML/TVaR)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1412_4556_amd import ara as A
    from paper_1412_4556_amd import workloads as W

    wl = W.plain_paper(args.trials)
    spec = wl.layers[0]
    T, K, J = wl.yet.n_trials, wl.yet.fixed_len, spec.n_elts
    log(f"generating YET {T} x {K} over {wl.yet.catalog_size} events")
    ids, _ = W.yet_full(wl.yet)
    t_ids = torch.from_numpy(ids).cuda()
    del ids
    yet = A.Yet(t_ids, None, T, wl.yet.catalog_size, K)
    ylt = torch.empty(T, dtype=torch.float64, device="cuda")
    rps = list(wl.return_periods)
    lookups = float(T) * K * J
    # the layer's ELTs, resident in HBM like the YET (a pool of 16 ELTs)
    pool = A.Pool(yet, spec.elt_ids, spec.elt_losses, args.precision, max_layers=2)
    ms_step, b_ms, k_ms, k_min, (pml, tvar) = time_step(A, torch, yet, pool, spec, ylt, args.steps, args.warmup,
                                                        rps)
    # the same steps one at a time (each waits for its PML/TVaR before the
    # next is issued): the latency of one step, with the host's turnaround
    ms_sync, _, _, _, (pml_s, tvar_s) = time_step(A, torch, yet, pool, spec, ylt, args.steps, args.warmup, rps,
                                                  pipelined=False)
    assert np.array_equal(pml_s, pml) and np.array_equal(tvar_s, tvar), "pipelined and synchronous steps differ"
    ylt_host = ylt.cpu().numpy()  # the timed steps' YLT, for the parity check against the oracle
    # the same layer built from host ELTs (upload over PCIe, checks, table),
    # outside the step; the second build is the steady-state cost
    # (from the ELTs as the C ABI takes them, every ELT's entries back to
    # back in host memory; joining the spec's per-ELT arrays is not timed)
    flat = spec.concat()
    terms = (spec.ret, spec.lim, spec.occ_ret, spec.occ_lim, spec.agg_ret, spec.agg_lim)
    A.Layer.from_flat(yet, *flat, *terms, args.precision, "fused").close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lay = A.Layer.from_flat(yet, *flat, *terms, args.precision, "fused", spec=spec)
    torch.cuda.synchronize()
    host_build_ms = (time.perf_counter() - t0) * 1e3
    log(f"layer: {J} ELTs, layout {lay.layout}, precision {lay.precision}, {lay.device_bytes} device bytes")
    algo_bytes = T * K * 4 + T * 8 + lay.device_bytes
    achieved = algo_bytes / (k_ms * 1e-3) / 1e9
    log(f"step {ms_step:.3f} ms pipelined, {ms_sync:.3f} ms one at a time (table build {b_ms:.3f} ms, "
        f"trial pass {k_ms:.3f} ms, min {k_min:.3f}), "
        f"{achieved:.0f} GB/s; layer from host ELTs {host_build_ms:.3f} ms")
    # the step's table is bitwise the one built from the host ELTs
    y2 = A.run_layer(yet, lay)
    assert torch.equal(y2, ylt), "pool-built and host-built layers differ"
    del y2
    # FP32C: the same step, and its YLT for the error report
    other = "fp32c" if args.precision == "fp64" else "fp64"
    pool2 = A.Pool(yet, spec.elt_ids, spec.elt_losses, other, max_layers=2)
    ylt2 = torch.empty(T, dtype=torch.float64, device="cuda")
    ms2, b2, k2, _, pt2 = time_step(A, torch, yet, pool2, spec, ylt2, args.steps, args.warmup, rps)
    ylt2_host = ylt2.cpu().numpy()
    log(f"{other} step {ms2:.3f} ms (table build {b2:.3f} ms, trial pass {k2:.3f} ms)")
    pool2.close()
    del ylt2
    precision = precision_runs(A, W, torch) if not args.no_cpu_baseline else None

    extras = {}
    if not args.no_extras:
        for prec, layout, steps in (("fp32c", "fused", args.steps), ("fp64", "compact", 5), ("fp32c", "compact", 5),
                                    ("fp64", "direct", 3), ("fp32c", "direct", 3), ("fp64", "sparse", 2)):
            if prec == args.precision and layout == "fused":
                continue
            l2 = A.Layer(yet, spec, prec, layout)
            _, kx, _, _ = time_layer(A, torch, yet, l2, ylt, steps, 1, rps, with_pml=False)
            extras[f"{prec}_{l2.layout}"] = {"kernel_ms": round(kx, 4), "lookups_per_s": lookups / (kx * 1e-3),
                                             "table_bytes": l2.device_bytes}
            log(f"extra {prec}/{l2.layout}: kernel {kx:.3f} ms")
            l2.close()
        # per-event outputs (the cumulative-sum scan), FP64
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        A.run_layer_events(yet, lay, want_cum=False, want_net=True)
        torch.cuda.synchronize()
        ev0.record()
        out = A.run_layer_events(yet, lay, want_cum=False, want_net=True)
        ev1.record()
        torch.cuda.synchronize()
        extras["per_event_net_output"] = {"kernel_ms": round(ev0.elapsed_time(ev1), 4)}
        del out
        # occurrence basis: YLT plus the largest occurrence loss per trial
        A.run_layer_max_occurrence(yet, lay)
        torch.cuda.synchronize()
        ms_occ = []
        for _ in range(5):
            ev0.record()
            _, mx = A.run_layer_max_occurrence(yet, lay)
            ev1.record()
            torch.cuda.synchronize()
            ms_occ.append(ev0.elapsed_time(ev1))
        opml, otvar = A.pml_tvar(mx, rps)
        extras["max_occurrence_output"] = {"kernel_ms": round(sorted(ms_occ)[2], 4),
                                           "occurrence_pml": [float(v) for v in opml],
                                           "occurrence_tvar": [float(v) for v in otvar]}
        del mx
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            A.pml_tvar(ylt, rps)
        extras["pml_tvar_ms"] = round((time.perf_counter() - t) * 200, 4)
        # a plain read-only pass over the same 4 GB: the YET validation that
        # ara_create_yet runs (every ID read once with 16-byte loads, a range
        # check), timed on the host around the synchronous create call
        A.Yet(t_ids, None, T, wl.yet.catalog_size, K).close()
        ms_rd = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            A.Yet(t_ids, None, T, wl.yet.catalog_size, K).close()
            ms_rd.append((time.perf_counter() - t0) * 1e3)
        rd_ms = sorted(ms_rd)[2]
        rd_gbps = t_ids.numel() * 4 / (rd_ms * 1e-3) / 1e9
        extras["hbm_read_probe"] = {"what": "YET validation in ara_create_yet: 4.0e9 bytes read once, host clock incl. "
                                            "the call", "ms": round(rd_ms, 4), "gbps": round(rd_gbps, 1),
                                    "trial_pass_frac_of_it": round(achieved / rd_gbps, 3)}
        log(f"read probe: {rd_gbps:.0f} GB/s; the trial pass reaches {achieved / rd_gbps:.2f} of it")

    lay_layout, lay_prec = lay.layout, lay.precision
    del t_ids
    pool.close()
    yet.close()
    lay.close()
    torch.cuda.empty_cache()
    batch = None
    if not args.no_batch:
        batch = batch_leg(A, W, torch, args.batch_trials, max(3, args.steps // 4))

    serving = None
    if not args.no_serving:
        serving = serving_leg(A, W, torch, args.serving_trials,
                              [float(r) for r in args.serving_rates.split(",") if r],
                              n_queries=args.serving_queries, budget_s=args.serving_budget_s)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        y64, y32 = (ylt_host, ylt2_host) if args.precision == "fp64" else (ylt2_host, ylt_host)
        p64, p32 = ((pml, tvar), pt2) if args.precision == "fp64" else (pt2, (pml, tvar))
        cpu = cpu_baseline(wl, spec, args.cpu_seconds, gpu_ylt=y64, gpu_pml_tvar=p64, rps=rps, gpu_ylt32=y32,
                           gpu_pml_tvar32=p32, precision=precision, single_full=args.cpu_single_thread_full)
        log(f"cpu baseline {cpu['value']:.3e} lookups/s on {cpu['cores']} threads")

    rec = {
        "metric": "trial-events x ELT lookups/sec",
        "value": lookups / (ms_step * 1e-3),
        "unit": "lookups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_synchronous": ms_sync,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f32c-scan+f64-aggregate",
        "data": "synthetic (seeded; the paper's YET/ELT shapes, its data are not public)",
        "config": {"workload": wl.name, "n_trials": T, "events_per_trial": K, "catalog": wl.yet.catalog_size,
                   "elts": J, "elt_size": 20_000, "layout": lay_layout, "precision": lay_prec,
                   "return_periods": rps},
        "trial_events_per_s": T * K / (ms_step * 1e-3),
        "lookups_are": ("equivalent: each step builds the layer's fused table from its device-resident ELTs "
                        "(the J ELT losses of every catalogue event through FT1, summed, through FT2) and the "
                        "trial pass reads one entry per trial-event"),
        "step_parts_ms": {"table_build_from_device_elts": b_ms, "trial_pass": k_ms,
                          "pml_tvar_and_host_overheads": ms_step - b_ms - k_ms},
        "layer_build_from_host_elts_ms": host_build_ms,
        "value_with_host_elt_build": lookups / ((ms_step - b_ms + host_build_ms) * 1e-3),
        "other_precision_step": {"precision": other, "ms_per_step": ms2, "value": lookups / (ms2 * 1e-3),
                                 "table_build_ms": b2, "trial_pass_ms": k2},
        "kernel_ms": k_ms,
        "hbm_gbps_algorithmic": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBPS,
                     "traffic": measured_traffic() if (lay_layout == "fused" and lay_prec == "fp64" and T == 1_000_000)
                     else None,
                     "kernel": "k_trial_pass_fused" if lay_layout == "fused" else "k_trial_pass",
                     "algorithmic_bytes": algo_bytes},
        "cpu_baseline": cpu,
        "pml": pml.tolist(),
        "tvar": tvar.tolist(),
        "device": torch.cuda.get_device_name(0),
        "extras": extras,
        "batch": batch,
        "serving": serving,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
