"""Python interface of libara: the same operations as the C ABI, on torch
tensors that live in HIP device memory.

torch only supplies device memory and the current stream; every step of the
trial pass runs in the HIP kernels of libara.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

PRECISIONS = {"fp64": L.ARA_FP64, "fp32c": L.ARA_FP32C}
LAYOUTS = {"auto": L.ARA_LAYOUT_AUTO, "direct": L.ARA_LAYOUT_DIRECT, "sparse": L.ARA_LAYOUT_SPARSE,
           "compact": L.ARA_LAYOUT_COMPACT, "fused": L.ARA_LAYOUT_FUSED}
LAYOUT_NAMES = {v: k for k, v in LAYOUTS.items()}


def _stream(stream: Optional[torch.cuda.Stream] = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _vp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Yet:
    """A device-resident Year Event Table (borrows the given tensors)."""

    def __init__(self, event_ids: torch.Tensor, offsets: Optional[torch.Tensor], n_trials: int,
                 catalog_size: int, events_per_trial: int = 0, stream=None):
        if event_ids.dtype != torch.int32 or not event_ids.is_cuda or not event_ids.is_contiguous():
            raise ValueError("event_ids must be a contiguous int32 device tensor")
        if offsets is not None and (offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous()):
            raise ValueError("offsets must be a contiguous int64 device tensor")
        self.event_ids = event_ids
        self.offsets = offsets
        self.n_trials = int(n_trials)
        self.catalog_size = int(catalog_size)
        self.events_per_trial = int(events_per_trial)
        self.n_events = int(event_ids.numel())
        h = ctypes.c_void_p()
        L.check(L.lib().ara_create_yet(ctypes.c_void_p(event_ids.data_ptr()),
                                       ctypes.c_void_p(offsets.data_ptr()) if offsets is not None else None,
                                       self.n_trials, self.events_per_trial, self.catalog_size,
                                       ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            L.lib().ara_destroy_yet(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Layer:
    """A layer's ELTs and terms, copied into library-owned device memory."""

    def __init__(self, yet: Yet, spec, precision: str = "fp64", layout: str = "auto"):
        ids, losses, sizes = spec.concat()
        self._create(yet, ids, losses, sizes, spec.ret, spec.lim, spec.occ_ret, spec.occ_lim, spec.agg_ret,
                     spec.agg_lim, precision, layout)
        self.spec = spec

    @classmethod
    def from_flat(cls, yet: Yet, ids, losses, sizes, ret, lim, occ_ret, occ_lim, agg_ret, agg_lim,
                  precision: str = "fp64", layout: str = "auto", spec=None) -> "Layer":
        """The layer from its ELTs as ara_create_layer takes them: every ELT's
        IDs and losses back to back (ELT j: sizes[j] entries, in layer order)."""
        obj = cls.__new__(cls)
        obj._create(yet, ids, losses, sizes, ret, lim, occ_ret, occ_lim, agg_ret, agg_lim, precision, layout)
        obj.spec = spec
        return obj

    def _create(self, yet, ids, losses, sizes, ret, lim, occ_ret, occ_lim, agg_ret, agg_lim, precision, layout):
        ids, losses, sizes = _np(ids, np.int32), _np(losses, np.float64), _np(sizes, np.int64)
        ret, lim = _np(ret, np.float64), _np(lim, np.float64)
        if len(ret) != len(sizes) or len(lim) != len(sizes):
            raise ValueError("one retention and one limit per ELT")
        h = ctypes.c_void_p()
        L.check(L.lib().ara_create_layer(yet.handle, int(len(sizes)), _vp(ids), _vp(losses), _vp(sizes), _vp(ret),
                                         _vp(lim), float(occ_ret), float(occ_lim), float(agg_ret), float(agg_lim),
                                         PRECISIONS[precision], LAYOUTS[layout], ctypes.byref(h)))
        self._h = h
        self.yet = yet

    @classmethod
    def _wrap(cls, handle, yet, spec):
        obj = cls.__new__(cls)
        obj._h = handle
        obj.yet = yet
        obj.spec = spec
        return obj

    @property
    def handle(self):
        return self._h

    @property
    def device_bytes(self) -> int:
        return int(L.lib().ara_layer_device_bytes(self._h))

    @property
    def layout(self) -> str:
        return LAYOUT_NAMES[int(L.lib().ara_layer_layout(self._h))]

    @property
    def precision(self) -> str:
        return {0: "fp64", 1: "fp32c"}[int(L.lib().ara_layer_precision(self._h))]

    def close(self):
        if getattr(self, "_h", None):
            L.lib().ara_destroy_layer(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """ELTs resident on the device; layers are built from them on the GPU."""

    def __init__(self, yet: Yet, elt_ids, elt_losses, precision: str = "fp64", max_layers: int = 64):
        sizes = _np([len(a) for a in elt_ids], np.int64)
        ids = _np(np.concatenate(elt_ids), np.int32)
        losses = _np(np.concatenate(elt_losses), np.float64)
        h = ctypes.c_void_p()
        L.check(L.lib().ara_create_pool(yet.handle, len(elt_ids), _vp(ids), _vp(losses), _vp(sizes),
                                        PRECISIONS[precision], int(max_layers), ctypes.byref(h)))
        self._h = h
        self.yet = yet
        self.n_elts = len(elt_ids)
        self.max_layers = int(max_layers)

    @property
    def free_slots(self) -> int:
        return int(L.lib().ara_pool_free_slots(self._h))

    @property
    def device_bytes(self) -> int:
        return int(L.lib().ara_pool_device_bytes(self._h))

    def layer(self, elt_index, ret, lim, occ_ret, occ_lim, agg_ret, agg_lim, stream=None, spec=None) -> Layer:
        """Build a fused layer on the GPU (asynchronous on the stream); raises
        AraError(ARA_ERR_OOM) when every slot is taken."""
        idx = _np(elt_index, np.int32)
        r, u = _np(ret, np.float64), _np(lim, np.float64)
        h = ctypes.c_void_p()
        L.check(L.lib().ara_create_layer_from_pool(self._h, len(idx), _vp(idx), _vp(r), _vp(u), float(occ_ret),
                                                   float(occ_lim), float(agg_ret), float(agg_lim),
                                                   ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
        return Layer._wrap(h, self.yet, spec)

    def close(self):
        if getattr(self, "_h", None):
            L.lib().ara_destroy_pool(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_out(t: torch.Tensor, n: int, name: str):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{name} must be a contiguous float64 device tensor of >= {n} elements")


def run_layer(yet: Yet, layer: Layer, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """YLT of one layer (float64 [n_trials]); asynchronous on the stream."""
    if out is None:
        out = torch.empty(yet.n_trials, dtype=torch.float64, device=yet.event_ids.device)
    _check_out(out, yet.n_trials, "out")
    L.check(L.lib().ara_run_layer(yet.handle, layer.handle, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(_stream(stream))))
    return out


def run_layer_events(yet: Yet, layer: Layer, want_cum: bool = True, want_net: bool = True, stream=None):
    """(ylt, event_cum or None, event_net or None)."""
    dev = yet.event_ids.device
    ylt = torch.empty(yet.n_trials, dtype=torch.float64, device=dev)
    cum = torch.empty(yet.n_events, dtype=torch.float64, device=dev) if want_cum else None
    net = torch.empty(yet.n_events, dtype=torch.float64, device=dev) if want_net else None
    L.check(L.lib().ara_run_layer_events(yet.handle, layer.handle, ctypes.c_void_p(ylt.data_ptr()),
                                         ctypes.c_void_p(cum.data_ptr()) if cum is not None else None,
                                         ctypes.c_void_p(net.data_ptr()) if net is not None else None,
                                         ctypes.c_void_p(_stream(stream))))
    return ylt, cum, net


def run_layer_max_occurrence(yet: Yet, layer: Layer, stream=None):
    """(ylt, max_occ): the YLT and, per trial, the largest occurrence loss
    (float64 [n_trials] each); asynchronous on the stream."""
    dev = yet.event_ids.device
    ylt = torch.empty(yet.n_trials, dtype=torch.float64, device=dev)
    mx = torch.empty(yet.n_trials, dtype=torch.float64, device=dev)
    L.check(L.lib().ara_run_layer_max_occurrence(yet.handle, layer.handle, ctypes.c_void_p(ylt.data_ptr()),
                                                 ctypes.c_void_p(mx.data_ptr()), ctypes.c_void_p(_stream(stream))))
    return ylt, mx


class Batch:
    """Several fused layers prepared for one pass over the YET."""

    def __init__(self, yet: Yet, layers: Sequence[Layer]):
        n = len(layers)
        hs = (ctypes.c_void_p * n)(*[l.handle.value for l in layers])
        h = ctypes.c_void_p()
        L.check(L.lib().ara_create_batch(yet.handle, hs, n, ctypes.byref(h)))
        self._h = h
        self.yet = yet
        self.n_layers = n

    @property
    def handle(self):
        return self._h

    @property
    def device_bytes(self) -> int:
        return int(L.lib().ara_batch_device_bytes(self._h))

    @property
    def launch_config(self):
        t, w = ctypes.c_int32(), ctypes.c_int32()
        L.check(L.lib().ara_batch_launch_config(self._h, ctypes.byref(t), ctypes.byref(w)))
        return int(t.value), int(w.value)

    @property
    def launch_group(self) -> int:
        """256-event chunks per load step chosen for the pass (0 before the first run)."""
        g = ctypes.c_int32()
        L.check(L.lib().ara_batch_launch_group(self._h, ctypes.byref(g)))
        return int(g.value)

    def rebuild(self, layers: Sequence[Layer]):
        n = len(layers)
        hs = (ctypes.c_void_p * n)(*[l.handle.value for l in layers])
        L.check(L.lib().ara_batch_rebuild(self._h, hs, n))
        self.n_layers = n

    def run(self, outs: Optional[Sequence[torch.Tensor]] = None, stream=None):
        if outs is None:
            outs = [torch.empty(self.yet.n_trials, dtype=torch.float64, device=self.yet.event_ids.device)
                    for _ in range(self.n_layers)]
        if len(outs) != self.n_layers:
            raise ValueError("one output tensor per layer")
        for o in outs:
            _check_out(o, self.yet.n_trials, "outs[i]")
        ps = (ctypes.c_void_p * self.n_layers)(*[o.data_ptr() for o in outs])
        L.check(L.lib().ara_run_batch(self._h, ps, ctypes.c_void_p(_stream(stream))))
        return list(outs)

    def close(self):
        if getattr(self, "_h", None):
            L.lib().ara_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_layers(yet: Yet, layers: Sequence[Layer], outs: Optional[Sequence[torch.Tensor]] = None, stream=None):
    """YLTs of several layers in one pass (one-shot batch; synchronous)."""
    n = len(layers)
    if outs is None:
        outs = [torch.empty(yet.n_trials, dtype=torch.float64, device=yet.event_ids.device) for _ in range(n)]
    for o in outs:
        _check_out(o, yet.n_trials, "outs[i]")
    hs = (ctypes.c_void_p * n)(*[l.handle.value for l in layers])
    ps = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    L.check(L.lib().ara_run_layers(yet.handle, hs, ps, n, ctypes.c_void_p(_stream(stream))))
    return list(outs)


def pml_tvar(ylt: torch.Tensor, return_periods: Sequence[float], stream=None):
    """(pml, tvar) numpy arrays for the return periods; synchronous."""
    _check_out(ylt, ylt.numel(), "ylt")
    rp = _np(list(return_periods), np.float64)
    pml = np.zeros(len(rp))
    tvar = np.zeros(len(rp))
    L.check(L.lib().ara_pml_tvar(ctypes.c_void_p(ylt.data_ptr()), int(ylt.numel()), _vp(rp), len(rp), _vp(pml),
                                 _vp(tvar), ctypes.c_void_p(_stream(stream))))
    return pml, tvar


def pml_tvar_many(ylts: Sequence[torch.Tensor], return_periods: Sequence[float], stream=None):
    """(pml, tvar) numpy arrays [n_ylts][n_rp] for YLTs of equal length; synchronous."""
    n = len(ylts)
    T = ylts[0].numel()
    for y in ylts:
        _check_out(y, T, "ylt")
    ps = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ylts])
    rp = _np(list(return_periods), np.float64)
    pml = np.zeros((n, len(rp)))
    tvar = np.zeros((n, len(rp)))
    L.check(L.lib().ara_pml_tvar_many(ps, n, int(T), _vp(rp), len(rp), _vp(pml), _vp(tvar),
                                      ctypes.c_void_p(_stream(stream))))
    return pml, tvar


def pml_tvar_many_noalloc(ylts: Sequence[torch.Tensor], return_periods: Sequence[float], pml: torch.Tensor,
                          tvar: torch.Tensor, stream=None):
    """PML/TVaR into the device tensors pml, tvar (float64 [n_ylts, n_rp],
    caller-allocated) with the library's static scratch: asynchronous, the
    library allocates nothing."""
    n = len(ylts)
    T = ylts[0].numel()
    for y in ylts:
        _check_out(y, T, "ylt")
    rp = _np(list(return_periods), np.float64)
    _check_out(pml, n * len(rp), "pml")
    _check_out(tvar, n * len(rp), "tvar")
    ps = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ylts])
    L.check(L.lib().ara_pml_tvar_many_noalloc(ps, n, int(T), _vp(rp), len(rp), ctypes.c_void_p(pml.data_ptr()),
                                              ctypes.c_void_p(tvar.data_ptr()), ctypes.c_void_p(_stream(stream))))
    return pml, tvar


def rollup(ylts: Sequence[torch.Tensor], groups: Sequence[int], n_groups: int, out=None, stream=None):
    """Year loss tables of n_groups groups: group g is the trial-by-trial sum of
    ylts[l] for groups[l] == g, in increasing l (ara_rollup); asynchronous."""
    n = len(ylts)
    T = ylts[0].numel() if n else 0
    for y in ylts:
        _check_out(y, T, "ylt")
    if out is None:
        dev = ylts[0].device if n else "cuda"
        out = [torch.empty(T, dtype=torch.float64, device=dev) for _ in range(max(n_groups, 0))]
    if len(out) != max(n_groups, 0):
        raise ValueError("one output table per group")
    for o in out:
        _check_out(o, T, "out")
    ps = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ylts])
    gs = _np(list(groups), np.int32)
    if len(gs) != n:
        raise ValueError("one group index per input table")
    os_ = (ctypes.c_void_p * max(n_groups, 1))(*[o.data_ptr() for o in out])
    L.check(L.lib().ara_rollup(ps, n, _vp(gs), int(n_groups), int(T), os_, ctypes.c_void_p(_stream(stream))))
    return list(out)


def yet_from_numpy(ids: np.ndarray, offsets: Optional[np.ndarray], n_trials: int, catalog_size: int,
                   events_per_trial: int = 0, device: str = "cuda") -> Yet:
    """Copy a host YET to the device and register it."""
    t_ids = torch.from_numpy(np.ascontiguousarray(ids, np.int32)).to(device)
    t_off = None if offsets is None else torch.from_numpy(np.ascontiguousarray(offsets, np.int64)).to(device)
    return Yet(t_ids, t_off, n_trials, catalog_size, events_per_trial)
