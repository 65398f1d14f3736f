"""PML/TVaR without allocation (ara_pml_tvar_many_noalloc): the entry point
whose scratch is a static device array of the library, for callers that
cannot allocate.  Its results must be bitwise those of ara_pml_tvar_many on
the same YLTs, call after call, also when a call is smaller than the one
before it (the shared scratch keeps the earlier call's contents)."""
import numpy as np
import pytest
import torch

from oracle import oracle
from paper_1412_4556_amd import _lib as L
from paper_1412_4556_amd import ara as A

pytestmark = pytest.mark.gpu


def _ylts(seed, n, T):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        y = rng.lognormal(12.0, 2.0, T)
        y[rng.uniform(size=T) < 0.3] = 0.0  # many zeros and ties, as after aggregate retentions
        y[: T // 50] = np.round(y[: T // 50], -4)
        out.append(torch.from_numpy(y).cuda())
    return out


def _noalloc(ylts, rps, stream=None):
    n = len(ylts)
    pml = torch.full((n, len(rps)), -1.0, dtype=torch.float64, device="cuda")
    tvar = torch.full((n, len(rps)), -1.0, dtype=torch.float64, device="cuda")
    A.pml_tvar_many_noalloc(ylts, rps, pml, tvar, stream=stream)
    return pml, tvar


def test_noalloc_equals_pml_tvar_many_two_calls():
    big = _ylts(1, 8, 300_000)
    small = _ylts(2, 2, 40_000)
    rp_big = [10.0, 100.0, 250.0, 1000.0, 5000.0]
    rp_small = [100.0, 250.0]
    for ylts, rps in ((big, rp_big), (small, rp_small)):
        pml, tvar = _noalloc(ylts, rps)
        torch.cuda.synchronize()
        want_pml, want_tvar = A.pml_tvar_many(ylts, rps)
        got_pml, got_tvar = pml.cpu().numpy(), tvar.cpu().numpy()
        assert np.array_equal(got_pml, want_pml), (len(ylts), rps)
        assert np.array_equal(got_tvar, want_tvar), (len(ylts), rps)
        # and the oracle's definition (k-th largest, mean of the k largest)
        for i, y in enumerate(ylts):
            rp_, rt_ = oracle.pml_tvar(y.cpu().numpy(), rps)
            assert np.array_equal(got_pml[i], rp_)
            assert np.all(np.abs(got_tvar[i] - rt_) <= 1e-12 * np.abs(rt_))


def test_noalloc_calls_in_a_row_on_one_stream():
    """Calls queued back to back on one stream without waiting: each starts
    from the state it clears, whatever the previous call left."""
    s = torch.cuda.Stream()
    sets = [(_ylts(10 + i, 1 + i % 3, 20_000 + 7_000 * i), [50.0, 200.0][: 1 + i % 2]) for i in range(6)]
    with torch.cuda.stream(s):
        outs = [_noalloc(y, rp, stream=s) for y, rp in sets]
    s.synchronize()
    for (y, rp), (pml, tvar) in zip(sets, outs):
        want_pml, want_tvar = A.pml_tvar_many(y, rp)
        assert np.array_equal(pml.cpu().numpy(), want_pml)
        assert np.array_equal(tvar.cpu().numpy(), want_tvar)


def test_noalloc_nan_and_limits():
    ylts = _ylts(3, 3, 5_000)
    ylts[1][17] = float("nan")
    pml, tvar = _noalloc(ylts, [10.0, 100.0])
    torch.cuda.synchronize()
    p, t = pml.cpu().numpy(), tvar.cpu().numpy()
    assert np.all(np.isnan(p[1])) and np.all(np.isnan(t[1]))
    want_pml, want_tvar = A.pml_tvar_many([ylts[0], ylts[2]], [10.0, 100.0])
    assert np.array_equal(p[[0, 2]], want_pml) and np.array_equal(t[[0, 2]], want_tvar)
    # the next call, without the NaN, is clean again
    ylts[1][17] = 1.0
    pml, tvar = _noalloc(ylts, [10.0, 100.0])
    torch.cuda.synchronize()
    want_pml, want_tvar = A.pml_tvar_many(ylts, [10.0, 100.0])
    assert np.array_equal(pml.cpu().numpy(), want_pml) and np.array_equal(tvar.cpu().numpy(), want_tvar)
    # beyond the static scratch: rejected on the host, nothing launched
    many = _ylts(4, 5, 1_000)
    with pytest.raises(L.AraError) as ei:
        _noalloc(many * 3, [2.0] * 9)  # 135 selections
    assert ei.value.name == "ARA_ERR_UNSUPPORTED"
    with pytest.raises(L.AraError) as ei:
        _noalloc(many[:1], [2000.0])  # k = floor(1000 / 2000) = 0
    assert ei.value.name == "ARA_ERR_RP"
