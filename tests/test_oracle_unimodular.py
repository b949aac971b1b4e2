"""Pins of oracle/unimodular.py (Section 2.2, Phase 3) against what the
mathematics fixes, computed by other means:

* the definition: the certificate's verdict equals |det D| = 1 (fraction-free
  determinant) on random unimodular and non-unimodular matrices, including
  det = +-2, +-3, a multiple of a prime of X, and singular ones;
* the residue identity: for every precision e = 2^k - 1 reached, the
  approximant implied by the residue, D^-1 (I - X^e Z_e), is an integer
  matrix (D^-1 from SymPy's exact rational inverse), and |Z_e| <= N max|D|;
* for a unimodular D, Z_e = 0 as soon as X^e > 4 max|D^-1| (the true entries,
  from SymPy), and the approximant then equals D^-1;
* C = D^-1 mod X against SymPy's inverse_mod; Hadamard's bound against the
  true adjugate;
* partial linearization: |det| of the linearized matrix equals |det B|
  (SymPy), its entries stay below 2^lam, its size is as stated.

A dropped term, a wrong sign or a transposed product in the step breaks the
integrality of D^-1 (I - X^e Z_e), which is checked at every step.
"""
import math
import random

import numpy as np
import pytest
import sympy

from oracle import unimodular as ou
from oracle import smith as osm

PRIMES2 = [67108859, 67108837]          # X for the pins: two primes below 2^26
PRIMES1 = [1000003]


def _rand_unimodular(n, rng, ops=None, mult=3):
    a = [[int(i == j) for j in range(n)] for i in range(n)]
    for _ in range(ops if ops is not None else 3 * n) if n >= 2 else ():
        i, j = rng.sample(range(n), 2)
        f = rng.randint(-mult, mult)
        if rng.random() < 0.5:
            a[i] = [x + f * y for x, y in zip(a[i], a[j])]
        else:
            for r in range(n):
                a[r][i] += f * a[r][j]
    if rng.random() < 0.5:
        a[0] = [-v for v in a[0]]
    return a


def _with_det(n, det, rng):
    u = _rand_unimodular(n, rng)
    d = [[int(i == j) for j in range(n)] for i in range(n)]
    d[n - 1][n - 1] = det
    # U diag(1, .., det) V
    v = _rand_unimodular(n, rng)
    return (np.array(u, dtype=object).dot(np.array(d, dtype=object)).dot(np.array(v, dtype=object))).tolist()


def _sympy_inv(d):
    return sympy.Matrix(d).inv()


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (5, 2), (12, 3), (24, 4)])
def test_unimodular_matrices_certify(n, seed):
    rng = random.Random(seed)
    d = _rand_unimodular(n, rng)
    assert abs(osm.bareiss_det(d)) == 1
    ok, steps = ou.certify(d, PRIMES2)
    assert ok and ou.is_unimodular(d)
    assert steps <= ou.steps_needed(d, math.prod(PRIMES2))


@pytest.mark.parametrize("det", [2, -2, 3, -3, 6, 101, -(2**31 - 1)])
def test_non_unimodular_rejected(det):
    rng = random.Random(abs(det))
    for n in (1, 3, 9):
        d = _with_det(n, det, rng)
        assert osm.bareiss_det(d) in (det, -det)
        ok, steps = ou.certify(d, PRIMES2)
        assert not ok and not ou.is_unimodular(d)
        assert steps == ou.steps_needed(d, math.prod(PRIMES2))


def test_singular_modulo_x_and_singular():
    rng = random.Random(7)
    p = PRIMES2[1]
    d = _with_det(6, p, rng)                      # p | det D: no inverse mod X
    assert ou.inverse_mod(d, PRIMES2) is None
    assert ou.certify(d, PRIMES2) == (False, 0)
    z = [[0] * 4 for _ in range(4)]
    z[0][0] = z[1][1] = z[2][2] = 1                # zero column
    assert ou.certify(z, PRIMES2) == (False, 0)
    assert ou.certify([], PRIMES2) == (True, 0)


def test_agrees_with_definition_on_random_small_matrices():
    rng = random.Random(11)
    seen = {True: 0, False: 0}
    for trial in range(120):
        n = rng.randint(1, 5)
        if trial % 3 == 0:
            d = _rand_unimodular(n, rng, mult=2)
        else:
            d = [[rng.randint(-2, 2) for _ in range(n)] for _ in range(n)]
        det = osm.bareiss_det(d)
        if det == 0:
            continue
        ok, _ = ou.certify(d, PRIMES2)
        assert ok == (abs(det) == 1), (d, det)
        seen[ok] += 1
    assert seen[True] >= 20 and seen[False] >= 20


@pytest.mark.parametrize("n,seed", [(3, 1), (8, 2), (16, 3)])
def test_residue_identity_and_bound(n, seed):
    """D^-1 (I - X^e Z_e) integral and |Z_e| <= N max|D| at every step, for a
    D that is not unimodular (so the residues stay nonzero)."""
    rng = random.Random(seed)
    while True:
        d = [[rng.randint(-50, 50) for _ in range(n)] for _ in range(n)]
        det = osm.bareiss_det(d)
        if det != 0 and math.gcd(det, math.prod(PRIMES2)) == 1 and abs(det) > 1:
            break
    X = math.prod(PRIMES2)
    assert X >= 4 * n * n * ou.max_abs(d)
    dinv = _sympy_inv(d)
    beta = n * ou.max_abs(d)
    for steps in range(0, 5):
        z = ou.high_order_residue(d, PRIMES2, steps)
        e = (1 << steps) - 1
        assert ou.max_abs(z) <= beta
        implied = dinv * (sympy.eye(n) - X ** e * sympy.Matrix(z))
        assert all(v.is_integer for v in implied), steps
        # the implied approximant stays below X^e in absolute value
        if e > 0:
            assert max(abs(int(v)) for v in implied) < X ** e


@pytest.mark.parametrize("n,seed", [(4, 5), (10, 6), (20, 7)])
def test_unimodular_residue_vanishes_at_true_precision(n, seed):
    rng = random.Random(seed)
    d = _rand_unimodular(n, rng, mult=4)
    dinv = _sympy_inv(d)
    hmax = max(abs(int(v)) for v in dinv)
    X = math.prod(PRIMES1)
    for steps in range(0, 12):
        e = (1 << steps) - 1
        z = ou.high_order_residue(d, PRIMES1, steps)
        if X ** e > 4 * hmax:
            assert ou.max_abs(z) == 0, steps
            break
    else:
        pytest.fail("precision never reached")


def test_inverse_mod_and_adjugate_bound_against_sympy():
    rng = random.Random(9)
    X = math.prod(PRIMES2)
    for n in (1, 2, 6, 11):
        while True:
            d = [[rng.randint(-30, 30) for _ in range(n)] for _ in range(n)]
            if math.gcd(osm.bareiss_det(d), X) == 1:
                break
        c = ou.inverse_mod(d, PRIMES2)
        ref = sympy.Matrix(d).inv_mod(X)
        assert all((int(c[i][j]) - int(ref[i, j])) % X == 0 for i in range(n) for j in range(n))
        assert all(abs(v) <= (X - 1) // 2 for row in c for v in row)
        if n > 1:
            adj = sympy.Matrix(d).adjugate()
            h = max(abs(int(v)) for v in adj)
            assert math.log2(max(h, 1)) <= ou.log2_adjugate_bound(d) + 1e-9


@pytest.mark.parametrize("lam,seed", [(4, 1), (8, 2), (16, 3)])
def test_linearization_keeps_det(lam, seed):
    rng = random.Random(seed)
    n = 6
    b = [[rng.randint(-9, 9) for _ in range(n)] for _ in range(n)]
    big = [1, 4]
    for r in big:
        b[r] = [rng.randint(-(1 << 60), 1 << 60) for _ in range(n)]
    b[4][2] = 0
    lin = ou.linearize_rows(b, big, lam)
    det_b = sympy.Matrix(b).det()
    det_l = sympy.Matrix(lin).det()
    assert abs(det_l) == abs(det_b) and det_b != 0
    assert ou.max_abs(lin) <= (1 << lam)
    widths = [max(abs(v).bit_length() for v in b[r]) for r in big]
    assert len(lin) == n + sum(max(1, -(-w // lam)) - 1 for w in widths)
    # a unimodular B stays unimodular
    rng2 = random.Random(seed + 100)
    u = _rand_unimodular(5, rng2, mult=1 << 20)
    lu = ou.linearize_rows(u, range(5), lam)
    assert ou.max_abs(lu) <= (1 << lam)
    assert ou.is_unimodular(u) and ou.is_unimodular(lu) and ou.certify(lu, PRIMES2)[0]
    u[2] = [2 * v for v in u[2]]
    lu = ou.linearize_rows(u, range(5), lam)
    assert not ou.is_unimodular(lu) and not ou.certify(lu, PRIMES2)[0]
