"""Helpers shared by the GPU tests: run a case through the C-ABI and through
the oracle on the same seeded inputs, and compare."""
import numpy as np
import torch

from oracle import oracle
from paper_1412_4556_amd import ara as A

TOL = {"fp64": 1e-12, "fp32c": 1e-6}


def gpu_layer_run(ids, off, T, C, K, spec, prec, layout, events=False, ids_misalign=False, max_occ=False):
    """YLT (and per-event outputs) of the HIP path, copied to the host."""
    if ids_misalign:
        # place the IDs one element into a bigger buffer: not 16-byte aligned
        buf = torch.empty(len(ids) + 1, dtype=torch.int32, device="cuda")
        buf[1:] = torch.from_numpy(np.ascontiguousarray(ids, np.int32)).cuda()
        t_ids = buf[1:]
        assert t_ids.data_ptr() % 16 != 0
    else:
        t_ids = torch.from_numpy(np.ascontiguousarray(ids, np.int32)).cuda()
    t_off = None if off is None else torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda()
    yet = A.Yet(t_ids, t_off, T, C, K)
    lay = A.Layer(yet, spec, prec, layout)
    if events:
        y, cum, net = A.run_layer_events(yet, lay)
        torch.cuda.synchronize()
        out = (y.cpu().numpy(), cum.cpu().numpy(), net.cpu().numpy())
    elif max_occ:
        y, mx = A.run_layer_max_occurrence(yet, lay)
        torch.cuda.synchronize()
        out = (y.cpu().numpy(), mx.cpu().numpy())
    else:
        y = A.run_layer(yet, lay)
        torch.cuda.synchronize()
        out = y.cpu().numpy()
    lay.close()
    yet.close()
    return out


def assert_close_to_oracle(y, ref, prec, what="ylt"):
    """|y - y_ref| <= tol * G_i per trial, G_i the trial's gross looked-up
    loss; in FP64 the year loss also within 1e-12 of the trial's cumulative
    occurrence loss S_i (every occurrence loss is the oracle's to the bit,
    only the order of the per-trial sum differs: (K - 1) u S_i)."""
    tol = TOL[prec]
    G = ref["gross"]
    err = np.abs(y - ref[what])
    bad = err > tol * G
    assert not bad.any(), (f"{what}: {bad.sum()} trials over {tol}*G; worst trial {int(np.argmax(err / np.maximum(G, 1e-300)))}"
                           f" err {err.max():.3e}")
    if prec == "fp64" and what == "ylt":
        S = ref["occ_sum"]
        bad = err > 1e-12 * S
        assert not bad.any(), f"ylt: {bad.sum()} trials over 1e-12*S; worst err {err[bad].max():.3e}"
    pos = ref[what] > 0
    rel = float((err[pos] / ref[what][pos]).max()) if pos.any() else 0.0
    scaled = float((err / np.maximum(G, 1e-300)).max()) if len(G) else 0.0
    return {"max_err_over_gross": scaled, "max_rel_err": rel}


def oracle_run(ids, off, T, C, K, spec, **kw):
    return oracle.run_layer(ids, off, T, K, C, spec, n_threads=8, **kw)


def assert_risk_close(gp, gt, rp, rt, prec, ref):
    """PML/TVaR of the GPU's YLT against the oracle's values from its own YLT:
    in FP64 within 1e-12 of their own size (exactly equal where the oracle's
    value is 0); in FP32C within 1e-6 of the largest gross trial loss (the
    per-trial bound; PML and TVaR move by at most the largest per-trial
    error)."""
    gp, gt, rp, rt = (np.asarray(a, np.float64) for a in (gp, gt, rp, rt))
    if prec == "fp64":
        for g, r in ((gp, rp), (gt, rt)):
            assert np.all(np.abs(g - r) <= 1e-12 * np.abs(r)), (g, r)
    else:
        bound = TOL[prec] * ref["gross"].max()
        assert np.all(np.abs(gp - rp) <= bound) and np.all(np.abs(gt - rt) <= bound)
    nz = lambda a: np.where(a == 0, 1.0, np.abs(a))
    return {"pml_rel_err": (np.abs(gp - rp) / nz(rp)).tolist(), "tvar_rel_err": (np.abs(gt - rt) / nz(rt)).tolist()}
