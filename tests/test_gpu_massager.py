"""GPU Smith massager (rns_smith_massager): S against the oracle's Smith form
and (U, M, T, S) through Section 4.2's checks (oracle/massager.py):
divisibility, A M S^-1 and (T + U M) S^-1 integral, T unit upper triangular,
|det A| = prod s_i, and Definition 1 with W = -T^-1 U.  The massager comes
back reduced (row i of U modulo s_i) and certified by Phase 3 (B unimodular
by high-order residues); the forced failure drops the last batch, so the
certificate itself must reject the non-maximal massager and restart.

Inputs: the Section 4.1 family A_ij = i^j mod n (synth.vandermonde_mod) for
the primes 17..53 (oracle computed here) and n = 101, 199 (stored oracle
values, tests/golden/smith_vandermonde.json); several batches are forced by
a first batch of one invariant (RNS_MASSAGER_R0=1); random matrices (one
nontrivial invariant); a unimodular matrix; the edge cases n = 0, n < 16,
singular input; a forced certificate failure (restart).
"""
import json
import os
import random
import sys

import numpy as np
import pytest

import synth
from oracle import massager as om, smith as osm

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "smith_vandermonde.json")


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


@pytest.fixture(scope="module")
def ctx_small_batches(rg):
    os.environ["RNS_MASSAGER_R0"] = "1"
    try:
        c = rg.Context(device=0, L=24)
    finally:
        del os.environ["RNS_MASSAGER_R0"]
    yield c
    c.close()


def _check_massager(a, res, det_abs=None):
    S = res.s
    c = om.checks(a, res.U, res.M, res.T, S, det_abs=det_abs)
    assert all(c.values()), c
    W = om.definition1_W(res.U, res.T)
    assert om.definition1(a, res.M, W, S)
    # reduced entries: M and T columns mod s_j, U rows mod s_i
    n = len(S)
    assert res.stats["cert_kind"] == 1 and res.stats["uc_dim"] >= n
    for j in range(n):
        for i in range(n):
            assert 0 <= res.U[j, i] < S[j] or (S[j] == 1 and res.U[j, i] == 0)
            assert 0 <= res.M[i, j] < max(S[j], 1) or (S[j] == 1 and res.M[i, j] == 0)
            if i != j:
                assert 0 <= res.T[i, j] < max(S[j], 1) or (S[j] == 1 and res.T[i, j] == 0)


@pytest.mark.parametrize("n", [17, 19, 23, 29, 31, 37, 41, 43, 47, 53])
def test_vandermonde_family_matches_oracle(ctx, rg, n):
    _say("massager vandermonde", n)
    a = synth.vandermonde_mod(n)
    res = rg.smith_massager(ctx, a, seed=n)
    assert res.s == osm.smith_form(a)
    assert res.stats["path"] == 2 and res.stats["cert_exact"] == 1
    _check_massager(a, res)


@pytest.mark.parametrize("n", [37, 43, 53, 61])
def test_several_batches(ctx_small_batches, rg, n):
    """A first batch of one invariant: the projection then runs through one
    or more earlier batches (the B update of Definition 2)."""
    _say("massager several batches", n)
    a = synth.vandermonde_mod(n)
    res = rg.smith_massager(ctx_small_batches, a, seed=3)
    assert res.s == osm.smith_form(a)
    assert res.stats["batches"] >= 3
    _check_massager(a, res)


def test_vandermonde_golden(ctx, rg):
    """The Section 4.1 family at n = 101, 199, 211, 307 and 503: S equals the
    oracle's (stored by tests/golden/make_smith_golden.py --vandermonde);
    up to n = 199 also the massager's checks in exact integers, with
    |det A| from the oracle (above that the Python-integer products take
    minutes; Phase 3's certificate still covers them)."""
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        n = case["n"]
        _say("massager vandermonde golden", n)
        a = synth.vandermonde_mod(n)
        res = rg.smith_massager(ctx, a, seed=1, fetch=("U", "M", "T") if n <= 199 else ())
        want = [1] * case["ones"] + [int(v) for v in case["tail"]]
        assert res.s == want
        assert res.s[-1].bit_length() == int(case["tail"][-1]).bit_length()
        assert res.stats["cert_kind"] == 1 and res.stats["cert_exact"] == 1
        if n <= 199:
            _check_massager(a, res, det_abs=int(case["det_abs"]))


@pytest.mark.parametrize("n,seed", [(20, 1), (64, 2), (100, 3)])
def test_random_matrices(ctx, rg, n, seed):
    _say("massager random", n, seed)
    rng = np.random.default_rng(seed)
    while True:
        a = rng.integers(-99, 100, size=(n, n), dtype=np.int64)
        if osm.bareiss_det(a.tolist()) != 0:
            break
    res = rg.smith_massager(ctx, a, seed=seed)
    assert res.s == osm.smith_form(a.tolist())
    _check_massager(a, res)


@pytest.mark.parametrize("name,factors", [
    ("a 20-bit prime plane", (2, 3, 2, 5, 1048573, 2, 7)),
    ("powers of two only", (2, 2, 2, 4, 2, 8, 2, 2)),
    ("15-bit and 10-bit prime planes", (32749, 1009, 2, 3)),
])
def test_word_moduli_planted(ctx, rg, name, factors):
    """Planted chains whose s_n fits a word: every batch runs the local Smith
    forms on the GPU, with an odd prime plane of Montgomery products, a pure
    power of two, and several prime powers combined by the CRT."""
    _say("massager planted word moduli:", name)
    pl = synth.planted_small(28, seed=3, factors=factors, cap=(1 << 31) - 1)
    res = rg.smith_massager(ctx, pl.a, seed=2)
    assert res.s == pl.s
    _check_massager(pl.a, res)


def test_unimodular_matrix(ctx, rg):
    _say("massager unimodular")
    n = 24
    rng = random.Random(5)
    P = [[int(i == j) for j in range(n)] for i in range(n)]
    for _ in range(2 * n):
        i, j = rng.sample(range(n), 2)
        f = rng.choice([-1, 1])
        P[i] = [x + f * y for x, y in zip(P[i], P[j])]
    a = np.array(P, dtype=np.int64)
    assert abs(osm.bareiss_det(P)) == 1
    res = rg.smith_massager(ctx, a, seed=0)
    assert res.s == [1] * n
    _check_massager(a, res)
    assert all(res.U[i, j] == 0 and res.M[i, j] == 0 for i in range(n) for j in range(n))


def test_seeds_agree_and_restart(ctx, rg):
    _say("massager seeds and forced restart")
    a = synth.vandermonde_mod(41)
    want = osm.smith_form(a)
    for seed in (1, 2, 3):
        assert rg.smith_massager(ctx, a, seed=seed).s == want
    ctx.force_cert_failures(1)
    res = rg.smith_massager(ctx, a, seed=9)
    assert res.stats["restarts"] >= 1
    assert res.stats["uc_rejects"] >= 1 and res.stats["cert_kind"] == 1
    assert res.s == want
    _check_massager(a, res)


def test_edge_cases(ctx, rg):
    _say("massager edge cases")
    empty = rg.smith_massager(ctx, np.zeros((0, 0), dtype=np.int64))
    assert empty.s == []
    with pytest.raises(rg.RnsError) as e:
        rg.smith_massager(ctx, synth.vandermonde_mod(13))
    assert e.value.status == 8                       # RNS_ENOTSUP below n = 16
    sing = synth.vandermonde_mod(29)
    sing[5] = sing[3]
    with pytest.raises(rg.RnsError) as e:
        rg.smith_massager(ctx, sing)
    assert e.value.status == 6                       # RNS_ESINGULAR


def test_determinant_certificate_form(ctx, rg):
    """The determinant certificate (|det A| = prod s_i from det A mod primes),
    which Phase 3 takes where the linearized B is beyond the residue
    certificate's limits, selected here with RNS_MASSAGER_CERT=det."""
    _say("massager determinant certificate form")
    a = synth.vandermonde_mod(43)
    os.environ["RNS_MASSAGER_CERT"] = "det"
    try:
        res = rg.smith_massager(ctx, a, seed=4)
        ctx.force_cert_failures(1)
        res2 = rg.smith_massager(ctx, a, seed=5)
    finally:
        del os.environ["RNS_MASSAGER_CERT"]
    want = osm.smith_form(a)
    assert res.s == want and res.stats["cert_kind"] == 0 and res.stats["cert_exact"] == 1
    assert res2.s == want and res2.stats["restarts"] >= 1 and res2.stats["cert_kind"] == 0
    S = res.s
    c = om.checks(a, res.U, res.M, res.T, S)
    assert all(c.values()), c


@pytest.mark.parametrize("n", [120, 400])
def test_planted_many_invariants(ctx, rg, n):
    """Planted invariants (A = U diag(s) V from factors among the primes below
    100) with n random row and column operations, so that n max|A| stays
    below the massager's 2^36 (the planted workload's 4n operations give
    entries of 2^42 at n = 2000, beyond it): nearly every s_i nontrivial (111
    of 120, 370 of 400), S equal to the planted invariants, certified by B's
    unimodularity; at n = 120 (U, M, T) also pass Section 4.2's checks.
    The massager refuses the 4n-operation matrix with RNS_ENOTSUP."""
    _say("massager planted", n)
    pl = synth.planted_smith(n, seed=0, ops_per_dim=1)
    assert int(np.abs(pl.a).max()) * n < (1 << 36)
    res = rg.smith_massager(ctx, pl.a, seed=0, fetch=("U", "M", "T") if n <= 120 else ())
    assert res.s == pl.s
    assert res.stats["cert_kind"] == 1 and res.stats["uc_rejects"] == 0
    if n <= 120:
        _check_massager(pl.a, res)
    else:
        big = synth.planted_smith(n, seed=0)
        with pytest.raises(rg.RnsError) as e:
            rg.smith_massager(ctx, big.a)
        assert e.value.status == 8                   # RNS_ENOTSUP
