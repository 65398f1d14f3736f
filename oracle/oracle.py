"""CPU oracle for the Aggregate Risk Analysis trial pass -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It wraps the plain sequential float64 C implementation in
``ara_oracle.c`` (Section III of the paper: Algorithm 1 and its four steps) and
adds the risk metrics read from the Year Loss Table.

Roll-up (the paper nests layers in programs and programs in a portfolio,
Section III, without saying how their results combine; the reading used
here): the year loss of a program in a trial is the sum of its layers' year
losses in that trial, added in binary64 in layer order starting from 0; a
portfolio rolls up its programs the same way.

Risk metrics (the paper names PML and TVaR without defining them; the
reading used here): for a return period of N years over T trials, with
k = floor(T / N) >= 1,
  PML_N  = the k-th largest year loss,
  TVaR_N = the mean of the k largest year losses.
The oracle sorts with ``numpy.sort`` and sums the tail with ``math.fsum``
(correctly rounded), then divides by k.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ara_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str):
    """Open an oracle shared library (the default one, or a test's rebuild of it)."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64, i32, d = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.oracle_run_layer.argtypes = [P, P, i64, i64, i32, i32, P, P, P, P, P, d, d, d, d, ctypes.c_int,
                                     P, P, P, P, P, P]
    lib.oracle_run_layer.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def run_layer(ids: np.ndarray, offsets: Optional[np.ndarray], n_trials: int, events_per_trial: int,
              catalog_size: int, layer, n_threads: int = 1, want_event_net: bool = False, lib=None,
              want_event_cum: bool = False, want_occ_max: bool = False):
    """Run one layer over a YET.

    Returns a dict with ``ylt`` (year loss per trial), ``occ_sum`` (the
    cumulative occurrence loss S before the aggregate terms), ``gross`` (sum of
    every looked-up loss before any term, used as the error scale) and, if
    asked, ``event_net`` (per-event increments of the aggregate-net loss) and
    ``event_cum`` (the cumulative occurrence loss S after each event) and
    ``occ_max`` (the largest occurrence loss of each trial, 0 if empty).
    """
    lib = _load() if lib is None else lib
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    off = None if offsets is None else np.ascontiguousarray(offsets, dtype=np.int64)
    eids, elos, sizes = layer.concat()
    eids = np.ascontiguousarray(eids, np.int32)
    elos = np.ascontiguousarray(elos, np.float64)
    sizes = np.ascontiguousarray(sizes, np.int64)
    ret = np.ascontiguousarray(layer.ret, np.float64)
    lim = np.ascontiguousarray(layer.lim, np.float64)
    ylt = np.zeros(n_trials, np.float64)
    occ = np.zeros(n_trials, np.float64)
    gross = np.zeros(n_trials, np.float64)
    ev = np.zeros(len(ids), np.float64) if want_event_net else None
    ec = np.zeros(len(ids), np.float64) if want_event_cum else None
    om = np.zeros(n_trials, np.float64) if want_occ_max else None
    rc = lib.oracle_run_layer(_ptr(ids), _ptr(off), n_trials, events_per_trial, catalog_size, layer.n_elts,
                              _ptr(eids), _ptr(elos), _ptr(sizes), _ptr(ret), _ptr(lim),
                              layer.occ_ret, layer.occ_lim, layer.agg_ret, layer.agg_lim, int(n_threads),
                              _ptr(ylt), _ptr(occ), _ptr(gross), _ptr(ec), _ptr(ev), _ptr(om))
    if rc != 0:
        raise OracleError(f"oracle_run_layer failed with status {rc}")
    out = {"ylt": ylt, "occ_sum": occ, "gross": gross}
    if want_event_net:
        out["event_net"] = ev
    if want_event_cum:
        out["event_cum"] = ec
    if want_occ_max:
        out["occ_max"] = om
    return out


def tail_k(n_trials: int, return_period: float) -> int:
    """Number of tail trials for a return period: k = floor(T / N)."""
    return int(math.floor(n_trials / return_period))


def pml_tvar(ylt: np.ndarray, return_periods: Sequence[float]):
    """PML and TVaR for each return period, as (pml array, tvar array)."""
    y = np.sort(np.asarray(ylt, dtype=np.float64))[::-1]
    T = len(y)
    pml, tvar = [], []
    for N in return_periods:
        k = tail_k(T, N)
        if k < 1:
            raise OracleError(f"return period {N} exceeds the number of trials {T}")
        pml.append(float(y[k - 1]))
        tvar.append(math.fsum(y[:k].tolist()) / k)
    return np.array(pml), np.array(tvar)


def rollup(ylts: Sequence[np.ndarray], groups: Sequence[int], n_groups: int):
    """Year loss tables of n_groups groups (programs, or a portfolio): group g
    is the trial-by-trial sum of the input tables l with groups[l] == g, added
    in increasing l from 0.0 (a group without inputs is all zero)."""
    if len(ylts) != len(groups):
        raise OracleError("one group index per input table")
    T = len(ylts[0]) if len(ylts) else 0
    out = [np.zeros(T, np.float64) for _ in range(n_groups)]
    for l, g in enumerate(groups):
        if not 0 <= g < n_groups:
            raise OracleError(f"group index {g} outside 0 .. {n_groups - 1}")
        y = np.asarray(ylts[l], dtype=np.float64)
        if len(y) != T:
            raise OracleError("input tables differ in length")
        out[g] = out[g] + y  # one binary64 addition per trial
    return out

