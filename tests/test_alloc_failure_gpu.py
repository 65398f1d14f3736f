"""An injected device-allocation failure is reported as ARA_ERR_OOM and
leaves the library usable (run in a child process: the injection is read
from the environment once)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
from paper_1412_4556_amd import ara as A, _lib as L, workloads as W
ids, off, spec = W.random_case(3, 200, 50.0, 5000, 3, 800)
yet = A.yet_from_numpy(ids, off, 200, 5000)          # allocation 1: validation flags
try:
    A.Layer(yet, spec, "fp64", "compact")             # allocations 2..: the second one fails
    print("NO-ERROR")
except L.AraError as e:
    print("ERR", e.name)
y = torch.arange(1, 101, dtype=torch.float64, device="cuda")
p, t = A.pml_tvar(y, [10])                            # still works (its scratch is not injected)
print("PML", p[0], t[0])
"""


def test_injected_allocation_failure():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, ARA_FAULT_ALLOC_AFTER="2")
    r = subprocess.run([sys.executable, "-c", CHILD, root], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "ERR ARA_ERR_OOM" in r.stdout
    assert "PML 91.0 95.5" in r.stdout
