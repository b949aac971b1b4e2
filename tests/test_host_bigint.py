"""Host code of the Smith-form driver: the big-integer routines (Lehmer gcd,
extended gcd, rational reconstruction) checked against plain Euclid and
round trips, compiled with g++ and the address/undefined-behaviour
sanitizers (host code only)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_bigint_lehmer(tmp_path):
    exe = str(tmp_path / "bigint_check")
    src = os.path.join(HERE, "host", "bigint_check.cpp")
    flags = ["-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(["g++"] + flags + [src, "-o", exe], check=True, timeout=300)
    out = subprocess.run([exe], check=True, timeout=300, capture_output=True, text=True).stdout
    assert out.strip().endswith("bad=0"), out
