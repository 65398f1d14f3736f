"""The seeded generators: deterministic, and any trial subset regenerates
exactly the slice of the full YET (the full-size parity tests rely on it)."""
import numpy as np

from paper_1412_4556_amd import workloads as W


def _small(spec, n):
    return W.YetSpec(spec.workload, n, spec.catalog_size, spec.fixed_len, spec.poisson_mean)


def test_yet_subset_matches_full_fixed_and_poisson():
    for base in (W.plain_paper().yet, W.batch_layers(n_trials=1000, n_layers=1).yet):
        spec = _small(base, 150_000)  # spans several generator blocks
        ids, off = W.yet_full(spec)
        if off is None:
            off = np.arange(spec.n_trials + 1, dtype=np.int64) * spec.fixed_len
        pick = np.array([0, 1, 65_535, 65_536, 65_537, 131_071, 149_999, 7])
        sub_ids, sub_off = W.yet_subset(spec, pick)
        for i, t in enumerate(pick):
            assert np.array_equal(sub_ids[sub_off[i]:sub_off[i + 1]], ids[off[t]:off[t + 1]])
        assert ids.min() >= 0 and ids.max() < spec.catalog_size


def test_generators_are_deterministic():
    a = W.plain_tiny()
    b = W.plain_tiny()
    assert all(np.array_equal(x, y) for x, y in zip(a.layers[0].elt_ids, b.layers[0].elt_ids))
    assert all(np.array_equal(x, y) for x, y in zip(a.layers[0].elt_losses, b.layers[0].elt_losses))
    assert np.array_equal(a.layers[0].ret, b.layers[0].ret)
    ia, _ = W.yet_full(a.yet)
    ib, _ = W.yet_full(b.yet)
    assert np.array_equal(ia, ib)


def test_elts_are_dictionaries_and_terms_in_range():
    wl = W.plain_tiny()
    lay = wl.layers[0]
    for ids, losses, r, u in zip(lay.elt_ids, lay.elt_losses, lay.ret, lay.lim):
        assert len(np.unique(ids)) == len(ids)
        assert np.all(losses > 0) and 0 <= r < u
        assert np.isclose(r, np.percentile(losses, 10)) and np.isclose(u, np.percentile(losses, 90))


def test_serving_queries_pick_pool_members():
    y, pool = W.serving_pool(n_trials=10)
    items = W.serving_queries(pool, 50, 100.0)
    times = [t for t, _, _ in items]
    assert np.all(np.diff(times) > 0)
    for _, spec, pick in items:
        assert 1 <= len(pick) <= 16 and len(np.unique(pick)) == len(pick)
        for j, p in enumerate(pick):
            assert spec.elt_ids[j] is pool.ids[p]
