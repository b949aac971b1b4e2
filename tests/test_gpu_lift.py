"""GPU p-adic lifting step (rns_lift_step: the Smith-form driver's step
kernels) against the oracle's Dixon step (oracle/lift.py), bit-exact.

Small cases cover every kernel form (vector units; matrix cores with int16
and int32 A; packed and unpacked right-hand sides) with ragged n.  Two cases
at n = 43690, the largest n the matrix-core step accepts, put every int32
digit sum at its bound: balanced digits of -8421504 are (-128, -128, -128, 0),
so with C and Rm made of it the shift-group-2 sum of C Rm reaches
3 * 2^14 * 43690 = 2^31 - 32768; and A X with A = 32639 (signed digits 127,
127) and X = 50331647 (digits 255, 255, 255, 2) takes every pair sum to
127 * 255 * 43690.
"""
import sys

import numpy as np
import pytest

from oracle import lift as olift, primes as op

pytestmark = pytest.mark.gpu

P = op.largest_primes_below(1 << 26, 3)


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_19254_amd as rg
    return torch, torch.device("cuda:0"), rg


def _run(env, C, A, Rt, p, form):
    """Runs the GPU step; Rt is [t][n] (the entry's layout)."""
    torch, dev, rg = env
    X, Rn, Rnm, bad, used = rg.lift_step(torch.from_numpy(C.astype(np.int32)).to(dev),
                                         torch.from_numpy(A).to(dev), torch.from_numpy(Rt).to(dev), p, form=form)
    torch.cuda.synchronize()
    return X.cpu().numpy().astype(np.uint32), Rn.cpu().numpy(), Rnm.cpu().numpy().astype(np.uint32), bad, used


def _check(env, C, A, Rt, p, form):
    X, Rn, Rnm, bad, used = _run(env, C, A, Rt, p, form)
    wX, wRn, wRnm, exact = olift.step(C, A, Rt.T, p)
    assert np.array_equal(X, wX.T)
    assert np.array_equal(Rn, np.asarray(wRn, dtype=np.int64).T)
    assert np.array_equal(Rnm, wRnm.T)
    assert bad == (not exact)
    return used


@pytest.mark.parametrize("n", [17, 100, 333, 1029])
@pytest.mark.parametrize("t", [1, 3, 4, 5, 8, 16])
@pytest.mark.parametrize("form", ["vector", "mfma"])
@pytest.mark.parametrize("abound", [1 << 10, 1 << 20])
def test_step_random_matches_oracle(env, n, t, form, abound):
    _say("lift step random", n, t, form, abound)
    rng = np.random.default_rng(n * 31 + t)
    p = P[t % 3]
    C = rng.integers(0, p, size=(n, n)).astype(np.uint32)
    A = rng.integers(-abound, abound + 1, size=(n, n), dtype=np.int64)
    Rt = rng.integers(-(1 << 40), 1 << 40, size=(t, n), dtype=np.int64)
    used = _check(env, C, A, Rt, p, form)
    rg = env[2]
    if form == "vector":
        assert used & (rg.binding.LIFT_C_MFMA | rg.binding.LIFT_AX_MFMA) == 0
    else:
        assert used & rg.binding.LIFT_C_MFMA
        int16 = abound < 32640
        assert bool(used & rg.binding.LIFT_A_INT16) == int16
        assert bool(used & rg.binding.LIFT_AX_MFMA) == int16
        assert bool(used & rg.binding.LIFT_PACKED) == (int16 and t <= 4)


@pytest.mark.parametrize("edge,int16", [(32639, True), (32640, False)])
def test_step_int16_edge(env, edge, int16):
    """A stored as int16 exactly while every |a| < 32640 (two signed byte
    digits), as int32 from 32640 on; both give the oracle's step."""
    _say("lift step int16 edge", edge)
    rng = np.random.default_rng(edge)
    n, t, p = 200, 4, P[0]
    C = rng.integers(0, p, size=(n, n)).astype(np.uint32)
    A = rng.choice(np.array([edge, -edge, 0, 1, -1, 255, -256], dtype=np.int64), size=(n, n))
    Rt = rng.integers(-(1 << 30), 1 << 30, size=(t, n), dtype=np.int64)
    used = _check(env, C, A, Rt, p, "mfma")
    rg = env[2]
    assert bool(used & rg.binding.LIFT_A_INT16) == int16
    assert bool(used & rg.binding.LIFT_AX_MFMA) == int16


@pytest.mark.parametrize("t", [4, 9])
def test_step_with_true_inverse_is_exact(env, t):
    """C = A^-1 mod p (the driver's case): every division is exact and the
    flag stays clear; two steps chained through R'."""
    _say("lift step true inverse", t)
    rng = np.random.default_rng(11)
    n, p = 70, P[1]
    while True:
        A = rng.integers(-1000, 1001, size=(n, n), dtype=np.int64)
        try:
            C = olift.inverse_mod_p(A, p)
            break
        except ValueError:
            continue
    Rt = rng.integers(-128, 129, size=(t, n), dtype=np.int64)
    for _ in range(2):
        X, Rn, Rnm, bad, _used = _run(env, C, A, Rt, p, "mfma")
        wX, wRn, wRnm, exact = olift.step(C, A, Rt.T, p)
        assert exact and not bad
        assert np.array_equal(X, wX.T) and np.array_equal(Rn, np.asarray(wRn, np.int64).T)
        Rt = np.ascontiguousarray(Rn)


NMAX = 43690


def _large_case(env, C, A, Rt_full, p, ts, forms):
    torch, dev, rg = env
    tC = torch.from_numpy(C.view(np.int32)).to(dev)
    tA = torch.from_numpy(A).to(dev)
    _say("  uploaded")
    for t in ts:
        Rt = np.ascontiguousarray(Rt_full[:t])
        wX, wRn, wRnm, exact = olift.step(C, A, Rt.T, p)
        _say("  oracle done t =", t)
        for form in forms:
            X, Rn, Rnm, bad, used = rg.lift_step(tC, tA, torch.from_numpy(Rt).to(dev), p, form=form)
            torch.cuda.synchronize()
            _say("  gpu done", t, form, "kernels", used)
            assert np.array_equal(X.cpu().numpy().astype(np.uint32), wX.T)
            assert np.array_equal(Rn.cpu().numpy(), np.asarray(wRn, np.int64).T)
            assert np.array_equal(Rnm.cpu().numpy().astype(np.uint32), wRnm.T)
            assert bad == (not exact)
            if form == "mfma":
                assert used & rg.binding.LIFT_C_MFMA and used & rg.binding.LIFT_AX_MFMA
                assert bool(used & rg.binding.LIFT_PACKED) == (t <= 4)
    del tC, tA
    torch.cuda.empty_cache()


def test_step_crm_sums_at_bound_n43690(env):
    """C Rm with every shift-group-2 int32 sum at 3 * 2^14 * 43690."""
    _say("lift step n=43690, C Rm digit sums at their bound")
    n, p = NMAX, P[0]
    v = -8421504                                   # balanced digits (-128, -128, -128, 0)
    C = np.full((n, n), p + v, dtype=np.uint32)
    rng = np.random.default_rng(1)
    C[1:5] = rng.integers(0, p, size=(4, n)).astype(np.uint32)     # a few ordinary rows
    A = np.empty((n, n), dtype=np.int64)
    A[:] = rng.integers(-32639, 32640, size=(1, n))
    Rt = np.full((9, n), v, dtype=np.int64)
    _large_case(env, C, A, Rt, p, ts=(4, 9), forms=("mfma", "vector"))


def test_step_ax_sums_at_bound_n43690(env):
    """A X with A = 32639 and X = 50331647 (C = I, so X = Rm): every digit-pair
    sum at 127 * 255 * 43690."""
    _say("lift step n=43690, A X digit sums at their bound")
    n, p = NMAX, P[2]
    C = np.zeros((n, n), dtype=np.uint32)
    C[np.arange(n), np.arange(n)] = 1
    A = np.full((n, n), 32639, dtype=np.int64)
    A[7] = -32639
    Rt = np.full((9, n), 50331647, dtype=np.int64)
    _large_case(env, C, A, Rt, p, ts=(4, 9), forms=("mfma",))
