"""The YET load indexing of the fused and batched passes, checked on the CPU:
tests/index_model.cpp runs the index functions the kernels call
(paper_1412_4556_amd/csrc/ara_index.h) over trials of every length 0..1001 at
every start modulo 4, and fixed-length YETs, and checks that every 16-byte
load stays within the YET's last granule, that the clamp never moves a load
holding trial elements, and that each event is taken exactly once."""
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
