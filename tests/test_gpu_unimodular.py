"""GPU unimodularity certificate (rns_unimodular_certify, Section 2.2, Phase 3)
against the oracle (oracle/unimodular.py):

* the residue Z_e after k double-plus-one steps equals the oracle's, entry
  for entry, for the same X (the primes the call reports), at sizes that span
  several product tiles and a ragged tail, entries up to 2^20;
* the verdict equals the definition |det D| = 1: unimodular L U products up to
  n = 3000 (the full-size cases are checked by the verdict, which a wrong
  residue at any step would break: a non-unimodular twin with det 2 must come
  out False after exactly the needed steps), det = +-2, 3 and a large prime,
  D singular modulo a prime of X, a zero column, n = 0 and 1;
* the bound error (n max|D| >= 2^61).

Inputs: seeded numpy generators; unimodular matrices are L U with L, U unit
triangular with entries in {-1, 0, 1}, rows and columns permuted.
"""
import math
import sys

import numpy as np
import pytest

from oracle import unimodular as ou
from oracle import smith as osm

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_19254_amd as rg
    return rg


@pytest.fixture(scope="module")
def ctx(rg):
    c = rg.Context(device=0, L=24)
    yield c
    c.close()


def _lu(n, seed, det=1):
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-1, 2, size=(n, n)), -1) + np.eye(n, dtype=np.int64)
    U = np.triu(rng.integers(-1, 2, size=(n, n)), 1) + np.eye(n, dtype=np.int64)
    L[n - 1, :] *= det
    # |entries| <= 2 n < 2^53: the double product is exact (and fast)
    D = np.rint(L.astype(np.float64) @ U.astype(np.float64)).astype(np.int64)
    pr, pc = rng.permutation(n), rng.permutation(n)
    return np.ascontiguousarray(D[pr][:, pc]).astype(np.int64)


@pytest.mark.parametrize("n,seed,amp,steps", [
    (1, 1, 50, 2), (5, 2, 50, 3), (37, 3, 50, 3), (70, 4, 1 << 20, 2), (130, 5, 50, 2), (131, 6, 7, 1),
])
def test_residues_match_oracle(ctx, rg, n, seed, amp, steps):
    _say("unimodular residues", n, seed, amp, steps)
    rng = np.random.default_rng(seed)
    while True:
        d = rng.integers(-amp, amp + 1, size=(n, n), dtype=np.int64)
        if n > 40 or abs(osm.bareiss_det(d.tolist())) > 1:
            break
    first = rg.unimodular_certify(ctx, d, max_steps=0)
    primes = first.info["x_prime"]
    X = math.prod(primes)
    assert X >= 4 * n * n * int(np.abs(d).max())
    for k in range(steps + 1):
        res = rg.unimodular_certify(ctx, d, max_steps=k, want_z=True)
        assert res.info["x_prime"] == primes
        want = ou.high_order_residue(d.tolist(), primes, k)
        assert want is not None
        got = res.Z.tolist()
        assert got == want, (n, k)
        if k and any(any(r) for r in want):
            assert res.verdict is None or res.verdict is False


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (16, 2), (64, 3), (200, 4), (701, 5)])
def test_unimodular_verdicts(ctx, rg, n, seed):
    _say("unimodular verdict", n)
    d = _lu(n, seed)
    res = rg.unimodular_certify(ctx, d)
    assert res.verdict is True and res.info["reason"] == 0
    assert res.info["steps"] <= res.info["steps_needed"]
    if n <= 64:
        assert ou.is_unimodular(d.tolist())


@pytest.mark.parametrize("det", [2, -2, 3, 1000003])
def test_not_unimodular(ctx, rg, det):
    for n in (1, 9, 150):
        _say("not unimodular", n, det)
        d = _lu(n, 100 + n, det=det)
        if n <= 9:
            assert abs(osm.bareiss_det(d.tolist())) == abs(det)
        res = rg.unimodular_certify(ctx, d)
        assert res.verdict is False and res.info["reason"] == 1
        assert res.info["steps"] == res.info["steps_needed"]


def test_full_size_pair(ctx, rg):
    n = 3000
    _say("unimodular full size", n)
    d = _lu(n, 7)
    res = rg.unimodular_certify(ctx, d)
    assert res.verdict is True
    _say("  steps", res.info["steps"], "of", res.info["steps_needed"], "seconds", res.info["seconds"])
    d2 = _lu(n, 7, det=2)
    res2 = rg.unimodular_certify(ctx, d2)
    assert res2.verdict is False and res2.info["steps"] == res2.info["steps_needed"]


def test_degenerate_cases(ctx, rg):
    _say("unimodular degenerate cases")
    assert rg.unimodular_certify(ctx, np.zeros((0, 0), dtype=np.int64)).verdict is True
    assert rg.unimodular_certify(ctx, np.array([[-1]], dtype=np.int64)).verdict is True
    assert rg.unimodular_certify(ctx, np.array([[0]], dtype=np.int64)).info["reason"] == 3
    p0 = rg.unimodular_certify(ctx, _lu(4, 1)).info["x_prime"][0]
    d = _lu(12, 9, det=p0)                              # p0 | det D
    res = rg.unimodular_certify(ctx, d)
    assert res.verdict is False and res.info["reason"] == 2
    z = _lu(10, 3)
    z[:, 4] = 0
    res = rg.unimodular_certify(ctx, z)
    assert res.verdict is False and res.info["reason"] == 3
    big = _lu(8, 2)
    big[0, 0] = 1 << 59
    with pytest.raises(rg.RnsError) as e:
        rg.unimodular_certify(ctx, big)
    assert e.value.status == 4                         # RNS_EBOUND
