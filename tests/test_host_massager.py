"""Host algebra of the Smith massager path (massager_host.hpp): the modular
Smith form with transforms over Z/sZ (Section 2.2, Phase 2, item 2) checked
against determinantal divisors of tiny integer matrices, E P R = diag(d),
-U P R = [D 0] and U M = -I modulo the orders, word and big-integer rings
agreeing, and the p-adic top-digit conversion; compiled with g++ and the
address/undefined-behaviour sanitizers (host code only)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_massager_host_algebra(tmp_path):
    exe = str(tmp_path / "massager_check")
    src = os.path.join(HERE, "host", "massager_check.cpp")
    flags = ["-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(["g++"] + flags + [src, "-o", exe], check=True, timeout=300)
    out = subprocess.run([exe], check=True, timeout=300, capture_output=True, text=True).stdout
    assert out.strip().endswith("bad=0"), out
