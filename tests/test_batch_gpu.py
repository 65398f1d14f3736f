"""Batched pass: many layers over one YET in one launch.

Every layer's YLT from the batch must be bitwise the one of its own
single-layer pass, and within tolerance of the oracle."""
import numpy as np
import pytest
import torch

from gpu_cases import TOL, assert_close_to_oracle, oracle_run
from paper_1412_4556_amd import _lib as L
from paper_1412_4556_amd import ara as A
from paper_1412_4556_amd import workloads as W

pytestmark = pytest.mark.gpu


def _layers(seed, n, C, max_j, elt_size):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        J = int(rng.integers(1, max_j + 1))
        _, _, spec = W.random_case(seed * 1000 + i, 1, 1.0, C, J, elt_size)
        out.append(spec)
    return out


def _yet(ids, off, T, C, K=0, misalign=False):
    if misalign:
        buf = torch.empty(len(ids) + 1, dtype=torch.int32, device="cuda")
        buf[1:] = torch.from_numpy(np.ascontiguousarray(ids, np.int32)).cuda()
        t_ids = buf[1:]
    else:
        t_ids = torch.from_numpy(np.ascontiguousarray(ids, np.int32)).cuda()
    t_off = None if off is None else torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda()
    return A.Yet(t_ids, t_off, T, C, K)


CASES = [
    # name, trials, mean_len, catalog, n_layers, max_elts, elt_size, fixed_len, misalign
    # (up to 16 layers: dense records in passes of up to 4 layers; above: sparse records)
    ("poisson_12", 3000, 200.0, 20000, 12, 8, 3000, False, False),
    ("poisson_16", 2000, 250.0, 20000, 16, 6, 2000, False, False),
    ("poisson_17", 2000, 250.0, 20000, 17, 6, 2000, False, False),
    ("poisson_3", 2500, 300.0, 40000, 3, 8, 5000, False, False),
    ("fixed_2", 900, 512, 30000, 2, 5, 5000, True, False),
    ("one_layer", 1500, 100.0, 10000, 1, 4, 2000, False, False),
    ("poisson_64", 2000, 300.0, 50000, 64, 6, 4000, False, False),
    ("fixed_1000", 600, 1000, 30000, 9, 5, 5000, True, False),
    ("fixed_7_misaligned", 700, 7, 3000, 5, 4, 600, True, True),
    ("empties", 1500, 20.0, 5000, 7, 3, 800, False, False),
    # sparse records in every YET form (fixed length, misaligned IDs, empty trials)
    ("fixed_1000_40", 500, 1000, 30000, 40, 5, 3000, True, False),
    ("fixed_7_20", 600, 7, 3000, 20, 4, 600, True, False),
    ("fixed_7_misaligned_20", 700, 7, 3000, 20, 4, 600, True, True),
    ("fixed_12_misaligned_33", 400, 12, 2000, 33, 6, 400, True, True),
    ("empties_24", 1500, 20.0, 5000, 24, 3, 800, False, False),
]


# Pass forms of sparse batches: the tuner's choice, or forced: the grouped
# pass (8 chunks per step) and the pipelined pass (one chunk per step, loads
# staged over three steps).  Batches of up to 16 layers take the dense form
# whatever the force (the dense passes have their own tests below).
FORMS = {"tuned": None, "grouped": "256,1,8", "pipelined": "256,1,1"}


def _force(monkeypatch, form):
    if FORMS[form]:
        monkeypatch.setenv("ARA_BATCH_LAUNCH", FORMS[form])
    else:
        monkeypatch.delenv("ARA_BATCH_LAUNCH", raising=False)


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_batch_equals_single_layer_passes(case, prec, form, monkeypatch):
    name, T, L_, C, n, max_j, esz, fixed, mis = case
    if form != "tuned" and n <= 16:
        pytest.skip("dense form: the forced shape does not apply")
    _force(monkeypatch, form)
    if fixed:
        rng = np.random.default_rng(T)
        K = int(L_)
        ids = rng.integers(0, C, size=T * K, dtype=np.int32)
        off = None
    else:
        K = 0
        ids, off, _ = W.random_case(T, T, L_, C, 1, 1, empty_frac=0.2 if name.startswith("empties") else 0.0)
    specs = _layers(hash(name) % 1000, n, C, max_j, esz)
    yet = _yet(ids, off, T, C, K, mis)
    layers = [A.Layer(yet, s, prec, "fused") for s in specs]
    singles = [A.run_layer(yet, l).cpu().numpy() for l in layers]
    batch = A.Batch(yet, layers)
    outs = batch.run()
    torch.cuda.synchronize()
    threads, per_cu = batch.launch_config
    assert threads % 64 == 0 and per_cu >= 1
    assert batch.launch_group in (1, 2, 4, 8)
    if form != "tuned":
        assert (threads, per_cu, batch.launch_group) == tuple(int(x) for x in FORMS[form].split(","))
    for l in range(n):
        assert np.array_equal(outs[l].cpu().numpy(), singles[l]), (name, l)
    # a second run (graph replay) into new buffers gives the same bits
    outs2 = batch.run()
    torch.cuda.synchronize()
    for l in range(n):
        assert np.array_equal(outs2[l].cpu().numpy(), singles[l])
    # oracle on a few layers
    for l in (0, n // 2, n - 1):
        ref = oracle_run(ids, off, T, C, K, specs[l])
        assert_close_to_oracle(singles[l], ref, prec)


@pytest.mark.parametrize("form", list(FORMS))
def test_batch_overflow_records(form, monkeypatch):
    """Dense ELTs over a small catalogue: most events sit in more layers than a
    record holds inline, so the overflow entries carry most of the losses
    (several blocks of four per event)."""
    _force(monkeypatch, form)
    T, C = 800, 500
    ids, off, _ = W.random_case(77, T, 60.0, C, 1, 1)
    specs = []
    for i in range(64):
        _, _, s = W.random_case(900 + i, 1, 1.0, C, 1, 400, terms="open", integer_losses=True)
        specs.append(s)
    yet = _yet(ids, off, T, C)
    for prec in ("fp64", "fp32c"):
        layers = [A.Layer(yet, s, prec, "fused") for s in specs]
        outs = A.run_layers(yet, layers)
        for l in (0, 13, 63):
            ref = oracle_run(ids, off, T, C, 0, specs[l])
            assert np.array_equal(outs[l].cpu().numpy(), ref["ylt"])  # integer losses: exact
        for l in range(64):
            assert np.array_equal(outs[l].cpu().numpy(), A.run_layer(yet, layers[l]).cpu().numpy())


def test_batch_errors():
    ids, off, spec = W.random_case(5, 100, 10.0, 1000, 2, 200)
    yet = _yet(ids, off, 100, 1000)
    fused = A.Layer(yet, spec, "fp64", "fused")
    compact = A.Layer(yet, spec, "fp64", "compact")
    f32 = A.Layer(yet, spec, "fp32c", "fused")
    with pytest.raises(L.AraError) as ei:
        A.Batch(yet, [fused, compact])
    assert ei.value.name == "ARA_ERR_UNSUPPORTED"
    with pytest.raises(L.AraError) as ei:
        A.Batch(yet, [fused, f32])
    assert ei.value.name == "ARA_ERR_INVALID_ARG"
    with pytest.raises(L.AraError) as ei:
        A.Batch(yet, [fused] * 65)
    assert ei.value.name == "ARA_ERR_UNSUPPORTED"
    b = A.Batch(yet, [fused, fused])  # the same layer twice is allowed
    o = b.run()
    assert np.array_equal(o[0].cpu().numpy(), o[1].cpu().numpy())


def test_batch_over_empty_yet():
    ids = np.zeros(0, np.int32)
    off = np.zeros(11, np.int64)
    _, _, spec = W.random_case(6, 1, 1.0, 100, 2, 50)
    yet = _yet(ids, off, 10, 100)
    lay = A.Layer(yet, spec, "fp64", "fused")
    outs = A.Batch(yet, [lay, lay]).run([torch.full((10,), 7.0, dtype=torch.float64, device="cuda") for _ in range(2)])
    assert all(np.array_equal(o.cpu().numpy(), np.zeros(10)) for o in outs)


def _disjoint_layers(n, C, size, seed):
    """n one-ELT layers over disjoint event ranges: no event is non-zero in
    more than one layer, so the batch needs no overflow entries."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(n):
        ids = np.arange(l * size, (l + 1) * size, dtype=np.int32) % C
        out.append(W.LayerSpec([ids], [rng.uniform(1.0, 100.0, size)], np.zeros(1), np.full(1, np.inf),
                               0.0, np.inf, 0.0, np.inf))
    return out


def _shared_layers(n, C, seed):
    """n layers that all hold one ELT covering the whole catalogue (each with
    its own terms): every event is non-zero in all n layers, so every record
    spills n - 6 (FP64) or n - 5 (FP32C) entries into the overflow area."""
    rng = np.random.default_rng(seed)
    ids = np.arange(C, dtype=np.int32)
    out = []
    for l in range(n):
        loss = rng.uniform(1.0, 1000.0, C)
        out.append(W.LayerSpec([ids], [loss], np.array([float(l)]), np.array([900.0 - l]), float(l), 2000.0,
                               float(10 * l), 1e7))
    return out


@pytest.mark.parametrize("n", [12, 20])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_batch_rebuild_same_size_larger_overflow(prec, n):
    """Regression: a batch that replayed a captured graph and is then rebuilt
    with the same number of layers but more overflow entries (its overflow
    area is reallocated) must not replay the old graph's pointers; a run on a
    second stream right after one on the first, and a rebuild right after a
    run, are ordered after the earlier run by the library."""
    T, C = 2500, 3000
    ids, off, _ = W.random_case(4242, T, 150.0, C, 1, 1)
    yet = _yet(ids, off, T, C)
    few = [A.Layer(yet, s, prec, "fused") for s in _disjoint_layers(n, C, 200, 1)]
    many_specs = _shared_layers(n, C, 2)
    many = [A.Layer(yet, s, prec, "fused") for s in many_specs]
    single_few = [A.run_layer(yet, l).cpu().numpy() for l in few]
    single_many = [A.run_layer(yet, l).cpu().numpy() for l in many]
    b = A.Batch(yet, few)
    small_bytes = b.device_bytes
    outs = b.run()
    outs = b.run(outs)  # the second run replays the captured graph
    torch.cuda.synchronize()
    for l in range(n):
        assert np.array_equal(outs[l].cpu().numpy(), single_few[l]), ("few", l)
    # no synchronisation between the run above and this rebuild
    outs_a = b.run()
    b.rebuild(many)
    if n > 16:
        assert b.device_bytes > small_bytes  # the overflow area was reallocated
    s2 = torch.cuda.Stream()
    outs_b = b.run(stream=s2)
    outs_c = b.run()  # default stream right after a run on s2
    torch.cuda.synchronize()
    for l in range(n):
        assert np.array_equal(outs_a[l].cpu().numpy(), single_few[l]), ("before rebuild", l)
        assert np.array_equal(outs_b[l].cpu().numpy(), single_many[l]), ("after rebuild", l)
        assert np.array_equal(outs_c[l].cpu().numpy(), single_many[l]), ("after rebuild, other stream", l)
    for l in (0, n - 1):
        ref = oracle_run(ids, off, T, C, 0, many_specs[l])
        assert_close_to_oracle(outs_b[l].cpu().numpy(), ref, prec)
    # and back to the layers without overflow (no reallocation this time)
    b.rebuild(few)
    outs_d = b.run()
    torch.cuda.synchronize()
    for l in range(n):
        assert np.array_equal(outs_d[l].cpu().numpy(), single_few[l]), ("rebuilt back", l)
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_batch_rebuild_across_forms(prec):
    """One batch object rebuilt between the dense form (up to 16 layers, in
    passes of up to 4) and the sparse one, and between dense widths, without
    synchronising in between: every run bitwise its layers' own passes."""
    T, C = 1800, 8000
    ids, off, _ = W.random_case(99, T, 120.0, C, 1, 1, empty_frac=0.05)
    yet = _yet(ids, off, T, C)
    specs = _layers(5, 40, C, 6, 1500)
    layers = [A.Layer(yet, sp, prec, "fused") for sp in specs]
    singles = [A.run_layer(yet, l).cpu().numpy() for l in layers]
    b = A.Batch(yet, layers[:2])
    pending = []
    for lo, hi in ((0, 2), (3, 40), (1, 4), (5, 21), (7, 23), (2, 18), (0, 1), (9, 13), (0, 40)):
        if b.n_layers != hi - lo or lo != 0:
            b.rebuild(layers[lo:hi])
        outs = b.run()
        pending.append((lo, hi, outs))
    torch.cuda.synchronize()
    for lo, hi, outs in pending:
        for k, o in enumerate(outs):
            assert np.array_equal(o.cpu().numpy(), singles[lo + k]), (lo, hi, k)
    b.close()


def test_batch_tuned_shape_fits_every_layer_count(monkeypatch):
    """A launch shape tuned for one layer count is reused for the other
    counts of its power-of-two bucket; its work-group is narrowed when the
    per-wave accumulators of a larger count would not fit the LDS (512
    threads fit 33 FP64 layers, not 64)."""
    T, C = 1234, 6000
    ids, off, _ = W.random_case(1234, T, 80.0, C, 1, 1)
    yet = _yet(ids, off, T, C)
    layers = [A.Layer(yet, sp, "fp64", "fused") for sp in _layers(8, 64, C, 3, 800)]
    singles = [A.run_layer(yet, l).cpu().numpy() for l in layers]
    monkeypatch.setenv("ARA_BATCH_LAUNCH", "512,1,8")
    b = A.Batch(yet, layers[:33])
    outs = b.run()
    assert b.launch_config == (512, 1) and b.launch_group == 8
    b.rebuild(layers)  # the forced shape, narrowed for 64 layers
    outs64 = b.run()
    threads, _ = b.launch_config
    assert threads <= 256
    torch.cuda.synchronize()
    for l in range(33):
        assert np.array_equal(outs[l].cpu().numpy(), singles[l])
    for l in range(64):
        assert np.array_equal(outs64[l].cpu().numpy(), singles[l])
    b.close()
    # a tuned shape remembered for 33 layers, reused (narrowed if needed) for 64
    monkeypatch.delenv("ARA_BATCH_LAUNCH")
    b = A.Batch(yet, layers[:33])
    b.run()
    b.rebuild(layers)
    outs64 = b.run()
    threads, per_cu = b.launch_config
    assert (threads // 64) * 64 * 65 * 8 <= 160 * 1024
    torch.cuda.synchronize()
    for l in range(64):
        assert np.array_equal(outs64[l].cpu().numpy(), singles[l])
    b.close()
