"""Tile order of the GEMM kernels checked on the host: the windowed XCD
placement is a bijection for every grid size, and the tile map covers a
ragged multi-problem table exactly once.  The index functions are compiled
for the host with hipcc; no device code runs."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_tile_order(tmp_path):
    exe = str(tmp_path / "tile_order_check")
    src = os.path.join(HERE, "host", "tile_order_check.hip")
    flags = ["-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops"]
    subprocess.run([HIPCC] + flags + [src, "-o", exe], check=True, timeout=600, capture_output=True)
    out = subprocess.run([exe], check=True, timeout=300, capture_output=True, text=True).stdout
    assert out.strip().endswith("bad=0"), out
