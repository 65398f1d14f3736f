"""Injected failures, each run in a child process (an injection is read
from the environment once): a device-allocation failure is reported as
ARA_ERR_OOM and leaves the library usable; batch graph captures that fail
leave the batched pass running by direct launches, bitwise as before."""
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


CAPTURE_CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
from paper_1412_4556_amd import ara as A, workloads as W
ids, off, _ = W.random_case(4, 3000, 120.0, 20000, 1, 1)
T = len(off) - 1
yet = A.yet_from_numpy(ids, off, T, 20000)
for n in (3, 20):  # dense records, then sparse records
    specs = [W.random_case(40 + k, 1, 1.0, 20000, 1 + k % 3, 2500)[2] for k in range(n)]
    layers = [A.Layer(yet, sp, "fp64", "fused") for sp in specs]
    singles = [A.run_layer(yet, l) for l in layers]
    b = A.Batch(yet, layers)
    for rep in range(5):  # three failed captures, then direct launches
        outs = b.run()
        torch.cuda.synchronize()
        assert all(torch.equal(o, s) for o, s in zip(outs, singles)), (n, rep)
    b.close()
    for l in layers:
        l.close()
print("BATCHES-OK")
"""


def test_failed_graph_captures_fall_back_to_direct_launches():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, ARA_FAULT_CAPTURE="1")
    r = subprocess.run([sys.executable, "-c", CAPTURE_CHILD, root], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "BATCHES-OK" in r.stdout, r.stdout[-2000:]
