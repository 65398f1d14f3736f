"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1412_4556_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ara.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ara_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["ara_create_yet", "ara_create_layer", "ara_run_layer", "ara_pml_tvar", "ara_run_layers",
              "ara_run_layer_events", "ara_destroy_yet", "ara_destroy_layer", "ara_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), "binding signatures and header disagree"


def test_abi_version_and_error_string():
    lib = L.lib()
    assert lib.ara_abi_version() == 1
    assert isinstance(lib.ara_last_error(), bytes)


def test_argument_checks_without_device_work():
    lib = L.lib()
    h = ctypes.c_void_p()
    # NULL out pointer / NULL yet / bad sizes are rejected before any HIP call
    assert lib.ara_create_yet(None, None, 10, 10, 100, None, None) == -1
    assert lib.ara_create_yet(None, None, -1, 10, 100, None, ctypes.byref(h)) == -1
    assert lib.ara_create_yet(None, None, 10, 10, 0, None, ctypes.byref(h)) == -1
    assert b"catalog" in lib.ara_last_error()
    sizes = np.array([1], np.int64)
    r = np.zeros(1)
    u = np.full(1, np.inf)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.ara_create_layer(None, 1, None, None, vp(sizes), vp(r), vp(u), 0, np.inf, 0, np.inf, 0, 0,
                                ctypes.byref(h)) == -1
    assert lib.ara_run_layer(None, None, None, None) == -1
    assert lib.ara_run_layer_events(None, None, None, None, None, None) == -1
    assert lib.ara_pml_tvar(None, 10, None, 1, None, None, None) == -1
    rp = np.array([100.0])
    pml = np.zeros(1)
    tv = np.zeros(1)
    fake = ctypes.c_void_p(16)  # never dereferenced: the size check fails first
    assert lib.ara_pml_tvar(fake, 0, vp(rp), 1, vp(pml), vp(tv), None) == -1
    assert lib.ara_pml_tvar(fake, 10, vp(rp), 0, vp(pml), vp(tv), None) == -1
    assert lib.ara_pml_tvar(fake, 10, vp(rp), 1, vp(pml), vp(tv), None) == -7  # floor(10/100) = 0
    assert lib.ara_layer_device_bytes(None) == 0
    assert lib.ara_layer_layout(None) == -1
    lib.ara_destroy_layer(None)
    lib.ara_destroy_yet(None)


def test_binding_raises_named_errors():
    with pytest.raises(L.AraError) as ei:
        L.check(-3)
    assert ei.value.name == "ARA_ERR_DUP_EVENT"
