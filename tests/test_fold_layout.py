"""The folded kx = 0 column of the spectral sweep (no GPU): the device-side
maps between workspace slots and half-spectrum bins, compiled for the host
from the library's own header and checked for consistency and completeness
(tests/fold_layout_check.cpp)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1001_1588_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_fold_layout_maps(tmp_path):
    exe = str(tmp_path / "fold_layout_check")
    subprocess.run(["hipcc", "-std=c++17", "-O1", "--offload-arch=gfx950", "-I", CSRC,
                    os.path.join(HERE, "fold_layout_check.cpp"), "-o", exe], check=True, capture_output=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout
