"""The C-ABI library loads and exports every entry point include/rns.h
declares; host-only routines behave as documented.  No GPU needed."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rns.h")
LIB = os.path.join(ROOT, "paper_2605_19254_amd", "librns.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)
    skip = {"sizeof", "defined"}
    return sorted(set(n for n in names if n not in skip and not n.startswith("RNS")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2605_19254_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "modmatmul_batched" in names and "crt_reconstruct" in names and "rns_reduce" in names
    assert "smith_form" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_every_export():
    import paper_2605_19254_amd.binding as b
    assert sorted(b.EXPORTS) == _declared()


def test_host_routines():
    import paper_2605_19254_amd as rg
    from oracle import primes as op
    assert rg.rns_primes_below(1 << 26, 30) == op.largest_primes_below(1 << 26, 30)
    assert rg.rns_primes_below(20, 4) == [19, 17, 13, 11]
    with pytest.raises(rg.RnsError):
        rg.rns_primes_below(8, 5)
    assert rg.rns_strerror(0) == "ok"
    assert "bound" in rg.rns_strerror(4)


def test_ctx_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2605_19254_amd as rg
    with pytest.raises(rg.RnsError) as e:
        rg.Context(device=0, L=4)
    assert e.value.status == 3
