"""Pins of the massager oracle (oracle/massager.py): Eq. (1) multiplied out
factor by factor against its block form, massagers known in closed form
(A = diag(s); A = P diag(s) Q with unimodular P, Q, where M = Q^-1, U = -Q,
and the same with any unit upper triangular T), and planted mistakes that
each check must catch."""
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import massager as om, smith as osm


def _unimodular(n, rng, ops=None):
    """A product of elementary operations with multipliers in [-2, 2]."""
    P = [[int(i == j) for j in range(n)] for i in range(n)]
    for _ in range(ops or 3 * n):
        i, j = rng.sample(range(n), 2)
        f = rng.randint(-2, 2)
        P[i] = [a + f * b for a, b in zip(P[i], P[j])]
    return P


def _inverse(P):
    """Exact inverse (Fractions, Gauss-Jordan); integral for unimodular P."""
    n = len(P)
    M = [[Fraction(v) for v in P[i]] + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for c in range(n):
        r = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[r] = M[r], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    out = [[M[i][n + j] for j in range(n)] for i in range(n)]
    assert all(v.denominator == 1 for row in out for v in row)
    return [[int(v) for v in row] for row in out]


def _mul(X, Y):
    return [[sum(a * b for a, b in zip(r, c)) for c in zip(*Y)] for r in X]


def _planted(n, s, seed):
    rng = random.Random(seed)
    P, Q = _unimodular(n, rng), _unimodular(n, rng)
    D = [[s[i] if i == j else 0 for j in range(n)] for i in range(n)]
    A = _mul(_mul(P, D), Q)
    M = _inverse(Q)
    U = [[-v for v in row] for row in Q]
    T = [[int(i == j) for j in range(n)] for i in range(n)]
    return A, U, M, T


def test_eq1_product_equals_block_form():
    rng = random.Random(3)
    for n in (1, 2, 4):
        S = [1] * n
        for i in range(n):
            S[i] = S[i - 1] * rng.randint(1, 4) if i else rng.randint(1, 3)
        A = [[rng.randint(-5, 5) for _ in range(n)] for _ in range(n)]
        U = [[rng.randint(-5, 5) for _ in range(n)] for _ in range(n)]
        M = [[rng.randint(-5, 5) for _ in range(n)] for _ in range(n)]
        T = [[(1 if i == j else (rng.randint(-3, 3) if j > i else 0)) for j in range(n)] for i in range(n)]
        B = om.massaged_matrix(A, U, M, T, S)
        AM, UM = _mul(A, M), _mul(U, M)
        for i in range(n):
            for j in range(n):
                assert B[i][j] == A[i][j]
                assert B[i][n + j] == Fraction(AM[i][j], S[j])
                assert B[n + i][j] == U[i][j]
                assert B[n + i][n + j] == Fraction(T[i][j] + UM[i][j], S[j])


def test_diagonal_matrix_trivial_massager():
    s = [1, 2, 6, 12, 60]
    n = len(s)
    A = [[s[i] if i == j else 0 for j in range(n)] for i in range(n)]
    I = [[int(i == j) for j in range(n)] for i in range(n)]
    U = [[-v for v in row] for row in I]
    c = om.checks(A, U, I, I, s)
    assert all(c.values()), c
    B = om.massaged_matrix(A, U, I, I, s)
    assert om.is_integral(B)
    assert abs(osm.bareiss_det([[int(v) for v in row] for row in B])) == 1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_planted_massager_and_definition1(seed):
    s = [1, 1, 2, 2, 6, 30, 30 * 7]
    A, U, M, T = _planted(len(s), s, seed)
    c = om.checks(A, U, M, T, s)
    assert all(c.values()), c
    B = om.massaged_matrix(A, U, M, T, s)
    assert om.is_integral(B)
    assert abs(osm.bareiss_det([[int(v) for v in row] for row in B])) == 1
    assert om.definition1(A, M, om.definition1_W(U, T), s)
    assert osm.smith_form(A) == s
    # Any unit upper triangular T with U' = T U gives another massager.
    rng = random.Random(seed + 10)
    n = len(s)
    T2 = [[(1 if i == j else (rng.randint(-4, 4) if j > i else 0)) for j in range(n)] for i in range(n)]
    U2 = _mul(T2, U)
    c2 = om.checks(A, U2, M, T2, s)
    assert all(c2.values()), c2
    assert om.is_integral(om.massaged_matrix(A, U2, M, T2, s))
    assert om.definition1(A, M, om.definition1_W(U2, T2), s)


def test_planted_mistakes_are_caught():
    s = [1, 2, 6, 6, 60]
    n = len(s)
    A, U, M, T = _planted(n, s, 7)
    assert all(om.checks(A, U, M, T, s).values())
    M2 = [row[:] for row in M]
    M2[0][4] += 1                                   # s_5 = 60 > 1
    c = om.checks(A, U, M2, T, s)
    assert not c["AMS_integral"]
    assert not om.is_integral(om.massaged_matrix(A, U, M2, T, s))
    U2 = [row[:] for row in U]
    U2[3] = [-v for v in U2[3]]                     # a sign flipped
    assert not om.checks(A, U2, M, T, s)["TUMS_integral"]
    assert not om.checks(A, U, M, T, [1, 2, 6, 6, 30])["unimodular"]
    T2 = [row[:] for row in T]
    T2[4][1] = 5
    assert not om.checks(A, U, M, T2, s)["T_unit_upper"]
    assert not om.checks(A, U, M, T, [1, 6, 2, 6, 60])["divisibility"]
    assert not om.definition1(A, M, [[-v for v in row] for row in om.definition1_W(U, T)], s)


def test_checks_match_integrality_of_eq1():
    """AMS and TUMS both hold exactly when B of Eq. (1) is integral."""
    rng = random.Random(11)
    s = [1, 2, 2, 12]
    A, U, M, T = _planted(len(s), s, 5)
    for _ in range(30):
        M2 = [row[:] for row in M]
        U2 = [row[:] for row in U]
        i, j = rng.randrange(4), rng.randrange(4)
        if rng.random() < 0.5:
            M2[i][j] += rng.choice([-2, -1, 1, 2, 12, 24])
        else:
            U2[i][j] += rng.choice([-1, 1, 2, 12])
        c = om.checks(A, U2, M2, T, s)
        assert om.is_integral(om.massaged_matrix(A, U2, M2, T, s)) == (c["AMS_integral"] and c["TUMS_integral"])
