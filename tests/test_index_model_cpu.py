"""The kernels' index arithmetic, checked on the CPU: tests/index_model.cpp
runs the index functions the kernels call
(paper_1412_4556_amd/csrc/ara_index.h).  YET loads of the fused and batched
passes, over trials of every length 0..1001 at every start modulo 4 and
fixed-length YETs: every 16-byte load stays within the YET's last granule,
the clamp never moves a load holding trial elements, and each event is taken
exactly once.  The fused table build, over catalogue sizes from 1 to
2^31 - 1: every event's range and offset give back the event, each range's
count sits in its own block-filter word inside the filter, and each range's
entry list stays inside the range's part of the table."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_load_indexing_model(tmp_path):
    exe = tmp_path / "index_model"
    src = os.path.join(HERE, "index_model.cpp")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", src, "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok"), out.stdout
