"""Pins for the oracle's determinant and Smith form.

Independent checks: Leibniz determinants and determinantal divisors by brute
force (tiny n), SymPy (the paper's own cross-check, Section 4.2), the largest
invariant factor as the common denominator of A^{-1}, planted invariants, the
divisibility chain and |det A| = prod s_i (Section 4.2, checks 1 and 4).
"""
import itertools
import json
import os
from math import gcd

import numpy as np
import pytest
import sympy
from sympy import QQ, ZZ, Matrix, ilcm
from sympy.matrices.normalforms import invariant_factors
from sympy.polys.matrices import DomainMatrix

from oracle import smith
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def _leibniz(a):
    n = len(a)
    total = 0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        term = -1 if inv % 2 else 1
        for i in range(n):
            term *= int(a[i][perm[i]])
        total += term
    return total


def _determinantal_divisor_smith(a):
    """s_k = D_k / D_{k-1}, D_k = gcd of all k x k minors (brute force)."""
    n = len(a)
    D = [1]
    for k in range(1, n + 1):
        g = 0
        for rows in itertools.combinations(range(n), k):
            for cols in itertools.combinations(range(n), k):
                g = gcd(g, _leibniz([[a[i][j] for j in cols] for i in rows]))
        D.append(g)
    return [D[k] // D[k - 1] for k in range(1, n + 1)]


def test_bareiss_against_leibniz():
    rng = np.random.default_rng(20)
    for n in range(1, 6):
        for _ in range(30):
            a = rng.integers(-9, 10, size=(n, n))
            assert smith.bareiss_det(a) == _leibniz(a.tolist())
    # a zero leading pivot forces a row exchange
    a = [[0, 2, 1], [3, 1, 4], [5, 9, 2]]
    assert smith.bareiss_det(a) == _leibniz(a)


def test_bareiss_against_sympy():
    rng = np.random.default_rng(21)
    for n in (7, 12, 20):
        a = rng.integers(-99, 100, size=(n, n))
        assert smith.bareiss_det(a) == int(Matrix(a.tolist()).det(method="berkowitz"))


def test_smith_brute_force_tiny():
    rng = np.random.default_rng(22)
    count = 0
    while count < 120:
        n = int(rng.integers(1, 5))
        a = rng.integers(-9, 10, size=(n, n))
        if _leibniz(a.tolist()) == 0:
            continue
        assert smith.smith_form(a) == _determinantal_divisor_smith(a.tolist()), a
        count += 1
    # structured cases: diagonal (needs the gcd/lcm reordering), scalar multiples
    for diag in ([6, 4], [12, 18, 8], [2, 3, 5, 7], [9, 3, 27, 1]):
        a = np.diag(diag)
        assert smith.smith_form(a) == _determinantal_divisor_smith(a.tolist())
    a = 6 * np.eye(3, dtype=np.int64)
    assert smith.smith_form(a) == [6, 6, 6]
    assert smith.smith_form(np.array([[-5]])) == [5]


@pytest.mark.parametrize("n", [3, 5, 7, 11, 13, 17, 19, 23, 29])
def test_smith_vandermonde_mod_vs_sympy(n):
    # Section 4.2: the paper compares against SymPy for prime n <= 53.
    # SymPy 1.14's invariant_factors stalls above n = 29 on this family; the
    # larger n are pinned in the next test.
    a = synth.vandermonde_mod(n)
    s = smith.smith_form(a)
    f = [abs(int(v)) for v in invariant_factors(Matrix(a.tolist()), domain=ZZ)]
    assert s == f


def _largest_factor_from_inverse(a):
    n = a.shape[0]
    inv = DomainMatrix.from_list_sympy(n, n, a.tolist()).convert_to(QQ).inv()
    den = 1
    for row in inv.to_list():
        for v in row:
            den = ilcm(den, QQ.to_sympy(v).q)
    return int(den)


@pytest.mark.parametrize("n", [31, 37, 41, 43, 47, 53])
def test_smith_vandermonde_mod_large(n):
    # s_n is the least d with d A^{-1} integral; s_1 is the gcd of all entries;
    # prod s_i = |det A| with det from SymPy's domain elimination.
    a = synth.vandermonde_mod(n)
    s = smith.smith_form(a)
    assert smith.is_divisor_chain(s)
    assert s[-1] == _largest_factor_from_inverse(a)
    g = 0
    for v in a.flatten().tolist():
        g = gcd(g, int(v))
    assert s[0] == g
    det = int(DomainMatrix.from_list_sympy(n, n, a.tolist()).convert_to(ZZ).det())
    prod = 1
    for v in s:
        prod *= v
    assert prod == abs(det)


def test_paper_facts_fixture_is_consistent():
    facts = json.load(open(GOLDEN))
    assert facts["vandermonde_mod_sn_bits"]["bits"] == 4083
    for n in facts["vandermonde_mod_checked_primes"]["primes"]:
        assert sympy.isprime(n)


@pytest.mark.parametrize("n,seed", [(8, 0), (24, 1), (40, 2), (64, 3)])
def test_smith_planted(n, seed):
    pl = synth.planted_smith(n, seed=seed)
    assert smith.smith_form(pl.a) == pl.s


def test_planted_generator_is_unimodular_transform():
    # det U = det V = 1, so |det A| = prod s (sympy determinant)
    pl = synth.planted_smith(12, seed=4)
    prod = 1
    for v in pl.s:
        prod *= v
    assert abs(int(Matrix(pl.a.tolist()).det(method="berkowitz"))) == prod
    assert smith.is_divisor_chain(pl.s)


def test_smith_random_invariants():
    rng = np.random.default_rng(23)
    for n in (10, 25):
        a = rng.integers(-99, 100, size=(n, n))
        s = smith.smith_form(a)
        assert smith.is_divisor_chain(s)
        assert s[-1] == _largest_factor_from_inverse(a)
        prod = 1
        for v in s:
            prod *= v
        assert prod == abs(smith.bareiss_det(a))


def test_singular_raises():
    a = np.array([[1, 2], [2, 4]])
    with pytest.raises(smith.Singular):
        smith.smith_form(a)
    assert smith.bareiss_det(np.zeros((3, 3), dtype=np.int64)) == 0


def test_small_smith_workload_is_nonsingular():
    a = synth.small_smith(seed=0)
    assert a.shape == (64, 64) and a.min() >= -99 and a.max() <= 99
    s = smith.smith_form(a)
    assert smith.is_divisor_chain(s)
    assert s[-1] == _largest_factor_from_inverse(a)
