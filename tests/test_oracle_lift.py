"""Pins for the oracle's Dixon lifting step (oracle/lift.py).

The step is checked against what the lifting must satisfy, not against a
retyping of its formula: the p-adic identity A (sum_i X_i p^i) = R_0 - p^K R_K
over K steps, the rational solution A^-1 b (SymPy) agreeing with the lifted
digits modulo p^K, brute force on tiny inputs, and the inverse mod p against
SymPy's.
"""
import numpy as np
import pytest
import sympy

from oracle import lift, primes as op

P = op.largest_primes_below(1 << 26, 1)[0]


def _rand_nonsingular(n, bound, seed):
    rng = np.random.default_rng(seed)
    while True:
        a = rng.integers(-bound, bound + 1, size=(n, n), dtype=np.int64)
        if sympy.Matrix(a.tolist()).det() % P != 0:
            return a


def test_inverse_mod_p_against_sympy():
    a = _rand_nonsingular(9, 50, 1)
    want = np.array(sympy.Matrix(a.tolist()).inv_mod(P).tolist(), dtype=np.int64)
    assert np.array_equal(lift.inverse_mod_p(a, P).astype(np.int64), want)
    with pytest.raises(ValueError):
        lift.inverse_mod_p(np.zeros((3, 3), np.int64), P)


def test_step_brute_force_tiny():
    rng = np.random.default_rng(2)
    for trial in range(20):
        n, t = int(rng.integers(1, 6)), int(rng.integers(1, 4))
        p = [97, 101, P][trial % 3]
        C = rng.integers(0, p, size=(n, n)).astype(np.uint32)
        A = rng.integers(-300, 301, size=(n, n), dtype=np.int64)
        R = rng.integers(-10**6, 10**6, size=(n, t), dtype=np.int64)
        X, Rn, Rnm, exact = lift.step(C, A, R, p)
        ok = True
        for i in range(n):
            for c in range(t):
                x = sum(int(C[i, k]) * (int(R[k, c]) % p) for k in range(n)) % p
                assert int(X[i, c]) == x
        for i in range(n):
            for c in range(t):
                num = int(R[i, c]) - sum(int(A[i, k]) * int(X[k, c]) for k in range(n))
                ok &= num % p == 0
                q = abs(num) // p * (1 if num >= 0 else -1)
                assert int(Rn[i, c]) == q and int(Rnm[i, c]) == q % p
        assert exact == ok


@pytest.mark.parametrize("n,t,bound", [(12, 3, 99), (30, 5, 1 << 10)])
def test_lifting_identity_and_rational_solution(n, t, bound):
    a = _rand_nonsingular(n, bound, n)
    C = lift.inverse_mod_p(a, P)
    rng = np.random.default_rng(7)
    b = rng.integers(-128, 129, size=(n, t), dtype=np.int64)
    R = b.copy()
    K = 6
    acc = np.zeros((n, t), dtype=object)
    pk = 1
    for _ in range(K):
        X, R, _, exact = lift.step(C, a, R, P)
        assert exact                           # C = A^-1 mod p: every division is exact
        acc = acc + X.astype(object) * pk
        pk *= P
    # A (sum X_i p^i) = b - p^K R_K over the integers
    lhs = a.astype(object).dot(acc)
    assert np.array_equal(lhs, b.astype(object) - pk * R.astype(object))
    # the lifted digits are A^-1 b mod p^K (SymPy's rational solution)
    sol = sympy.Matrix(a.tolist()).LUsolve(sympy.Matrix(b.tolist()))
    for i in range(n):
        for c in range(t):
            q = sympy.Rational(sol[i, c])
            want = int(q.p) * pow(int(q.q), -1, pk) % pk
            assert int(acc[i, c]) % pk == want


def test_inexact_division_is_flagged():
    n = 6
    a = _rand_nonsingular(n, 20, 3)
    C = lift.inverse_mod_p(a, P).astype(np.int64)
    C[0, 0] = (C[0, 0] + 1) % P                # no longer the inverse mod p
    R = np.ones((n, 2), dtype=np.int64)
    _, _, _, exact = lift.step(C.astype(np.uint32), a, R, P)
    assert not exact
