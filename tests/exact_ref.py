"""Exact-arithmetic brute force of the trial pass, for pinning the oracle on tiny inputs.

Every float input is converted exactly to a ``fractions.Fraction``; the four
steps of Section III (lookup, per-ELT terms and cross-ELT sum, occurrence
terms, cumulative sum and aggregate terms) are then evaluated without any
rounding.  ELT lookups use a plain dict per ELT.  Infinite limits are kept as
``None`` (no cap).
"""
from fractions import Fraction
import math


def _F(x):
    return None if math.isinf(x) else Fraction(x)


def _clamp(x, r, u):
    v = x - r
    if v < 0:
        v = Fraction(0)
    if u is not None and v > u:
        v = u
    return v


def exact_layer(ids, offsets, layer):
    """Return (ylt, occ_sum, gross, event_net) as lists of Fractions."""
    tables = [dict(zip(map(int, e), map(Fraction, l))) for e, l in zip(layer.elt_ids, layer.elt_losses)]
    ret = [Fraction(r) for r in layer.ret]
    lim = [_F(u) for u in layer.lim]
    R2, L2 = Fraction(layer.occ_ret), _F(layer.occ_lim)
    R3, L3 = Fraction(layer.agg_ret), _F(layer.agg_lim)
    ylt, occ, gross, net = [], [], [], []
    for i in range(len(offsets) - 1):
        S = Fraction(0)
        G = Fraction(0)
        A_prev = Fraction(0)
        for k in range(int(offsets[i]), int(offsets[i + 1])):
            E = int(ids[k])
            e = Fraction(0)
            for j, t in enumerate(tables):
                l = t.get(E, Fraction(0))
                G += l
                e += _clamp(l, ret[j], lim[j])
            S += _clamp(e, R2, L2)
            A = _clamp(S, R3, L3)
            net.append(A - A_prev)
            A_prev = A
        ylt.append(_clamp(S, R3, L3))
        occ.append(S)
        gross.append(G)
    return ylt, occ, gross, net


def exact_occ_max(ids, offsets, layer):
    """Largest occurrence loss (after the occurrence terms) of each trial, as
    Fractions; 0 for an empty trial."""
    tables = [dict(zip(map(int, e), map(Fraction, l))) for e, l in zip(layer.elt_ids, layer.elt_losses)]
    ret = [Fraction(r) for r in layer.ret]
    lim = [_F(u) for u in layer.lim]
    R2, L2 = Fraction(layer.occ_ret), _F(layer.occ_lim)
    out = []
    for i in range(len(offsets) - 1):
        M = Fraction(0)
        for k in range(int(offsets[i]), int(offsets[i + 1])):
            E = int(ids[k])
            e = Fraction(0)
            for j, t in enumerate(tables):
                e += _clamp(t.get(E, Fraction(0)), ret[j], lim[j])
            M = max(M, _clamp(e, R2, L2))
        out.append(M)
    return out
