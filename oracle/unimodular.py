"""Oracle: unimodularity certification by high-order X-adic residues
(Section 2.2, Phase 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Phase 3 decides whether the final massaged matrix B of Eq. (1) is unimodular;
the paper names the deterministic certification of Pauderis and Storjohann,
built on double-plus-one X-adic lifting, without describing it.  This module
writes out the reading used here, for an integer N x N matrix D:

* X is a product of primes with D invertible modulo X (otherwise p | det D
  for some prime p of X and D is not unimodular) and X >= 4 N^2 max|D|.
  C = D^-1 mod X.
* High-order residues.  Start from Z_0 = I (the approximant 0 of D^-1 at
  precision X^0: I - D 0 = X^0 Z_0).  One double-plus-one step maps a residue
  Z at precision e, I - D P = X^e Z for some integer P = D^-1 mod X^e, to one
  at precision 2e + 1:

      Y = Z Z,   K = cmod(C Y, X),   Z' = (Y - D K) / X        (exact)

  because D^-1 = P + X^e D^-1 Z gives D^-1 = P (I + X^e Z) + X^2e D^-1 Y and
  D^-1 Y = K + X D^-1 Z' (K = D^-1 Y mod X).  With |Z| <= N max|D| and
  X >= 4 N^2 max|D| the new residue stays within that bound, and the implied
  approximant P stays below X^e in absolute value (its fresh digit is
  symmetric and its carries are a quarter of the previous bound).
* Certificate.  Z_e = 0 means D P = I: D^-1 = P is integral and D is
  unimodular.  Conversely, if D is unimodular then D^-1 is integral with
  entries at most the Hadamard bound H of the (N-1)-minors; once
  X^e >= 4 H, D^-1 - P is a multiple of X^e smaller than X^e in absolute
  value, hence 0, and Z_e = X^-e D (D^-1 - P) = 0.  So D is unimodular
  exactly when Z_e = 0 after k steps with 2^k - 1 >= log_X(4 H).

Every matrix here is a list of lists of Python ints; products use numpy's
object-dtype dot (exact).  `is_unimodular` is the definition (|det D| = 1 by
fraction-free elimination); the other functions follow the steps above.
`linearize_rows` is the partial linearization that brings the massaged matrix
to small entries with the same |det|.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import smith as osmith


def _obj(x) -> np.ndarray:
    a = np.empty((len(x), len(x[0]) if len(x) else 0), dtype=object)
    for i, row in enumerate(x):
        for j, v in enumerate(row):
            a[i, j] = int(v)
    return a


def _mm(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    if a.shape[0] == 0:
        return a.copy()
    return np.dot(a, b)


def cmod(x: int, X: int) -> int:
    """Symmetric residue of x modulo an odd X: the r = x mod X with |r| <= (X-1)/2."""
    r = x % X
    return r - X if r > (X - 1) // 2 else r


def is_unimodular(d) -> bool:
    """The definition: |det D| = 1 (Bareiss elimination, exact)."""
    return abs(osmith.bareiss_det(_rows(d))) == 1


def _rows(d) -> List[List[int]]:
    return [[int(v) for v in row] for row in d]


def inverse_mod_prime(d, p: int) -> Optional[List[List[int]]]:
    """D^-1 mod p by Gauss-Jordan elimination over Z/p; None if D is singular mod p."""
    n = len(d)
    m = [[int(v) % p for v in row] + [int(i == j) for j in range(n)] for i, row in enumerate(d)]
    for c in range(n):
        piv = next((r for r in range(c, n) if m[r][c] % p), None)
        if piv is None:
            return None
        m[c], m[piv] = m[piv], m[c]
        inv = pow(m[c][c], -1, p)
        m[c] = [(v * inv) % p for v in m[c]]
        for r in range(n):
            if r != c and m[r][c]:
                f = m[r][c]
                m[r] = [(a - f * b) % p for a, b in zip(m[r], m[c])]
    return [row[n:] for row in m]


def inverse_mod(d, primes: Sequence[int]) -> Optional[List[List[int]]]:
    """D^-1 mod X, X = prod(primes) (distinct primes), symmetric entries, by the
    CRT of the inverses modulo each prime; None if D is singular mod one of them."""
    n = len(d)
    X = math.prod(primes)
    inv = [inverse_mod_prime(d, p) for p in primes]
    if any(v is None for v in inv):
        return None
    out = [[0] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            x = 0
            for p, ip in zip(primes, inv):
                mp = X // p
                x += ip[i][j] * mp * pow(mp, -1, p)
            out[i][j] = cmod(x, X)
    return out


def max_abs(d) -> int:
    return max((abs(int(v)) for row in d for v in row), default=0)


def log2_adjugate_bound(d) -> float:
    """log2 of H = prod_c ||col_c||_2 / min_c ||col_c||_2, Hadamard's bound on
    every (N-1)-minor of D (deleting a row only shortens the columns)."""
    n = len(d)
    if n <= 1:
        return 0.0
    logs = []
    for c in range(n):
        s = sum(int(d[r][c]) ** 2 for r in range(n))
        if s == 0:
            return math.inf
        logs.append(0.5 * math.log2(s))
    return sum(logs) - min(logs)


def steps_needed(d, X: int) -> int:
    """Smallest k with (2^k - 1) log2 X >= log2(4 H)."""
    need = (log2_adjugate_bound(d) + 2.0) / math.log2(X)
    k = 0
    while (1 << k) - 1 < need:
        k += 1
    return k


def residue_step(d: np.ndarray, c: np.ndarray, X: int, z: np.ndarray) -> np.ndarray:
    """One double-plus-one step: Z' = (Z Z - D cmod(C Z Z, X)) / X, exact."""
    y = _mm(z, z)
    k = _mm(c, y)
    k = np.vectorize(lambda v: cmod(int(v), X), otypes=[object])(k) if k.size else k
    r = y - _mm(d, k)
    for v in r.flat:
        assert int(v) % X == 0, "inexact division by X"
    return r // X if r.size else r


def high_order_residue(d, primes: Sequence[int], steps: int) -> Optional[List[List[int]]]:
    """Z_e after `steps` double-plus-one steps from Z_0 = I (e = 2^steps - 1);
    None if D is singular modulo a prime of X."""
    n = len(d)
    X = math.prod(primes)
    c = inverse_mod(d, primes)
    if c is None:
        return None
    D, C = _obj(d), _obj(c) if n else np.empty((0, 0), dtype=object)
    z = _obj([[int(i == j) for j in range(n)] for i in range(n)]) if n else np.empty((0, 0), dtype=object)
    for _ in range(steps):
        z = residue_step(D, C, X, z)
    return [[int(v) for v in row] for row in z]


def certify(d, primes: Sequence[int]) -> Tuple[bool, int]:
    """The certificate: (unimodular?, steps run).  Singular modulo X or a zero
    column: not unimodular, 0 steps.  Otherwise steps until Z = 0 (unimodular)
    or until the precision reaches 4 H (not unimodular)."""
    n = len(d)
    if n == 0:
        return True, 0
    X = math.prod(primes)
    if X < 4 * n * n * max_abs(d):
        raise ValueError("X below 4 N^2 max|D|")
    if math.isinf(log2_adjugate_bound(d)):
        return False, 0
    c = inverse_mod(d, primes)
    if c is None:
        return False, 0
    D, C = _obj(d), _obj(c)
    z = _obj([[int(i == j) for j in range(n)] for i in range(n)])
    k_max = steps_needed(d, X)
    for k in range(1, k_max + 1):
        z = residue_step(D, C, X, z)
        if all(int(v) == 0 for v in z.flat):
            return True, k
    return False, k_max


def linearize_rows(b, rows: Sequence[int], lam: int) -> List[List[int]]:
    """Partial linearization of the listed rows of a square integer matrix B:
    row r = sum_l 2^(lam l) r_l (digits r_l of the absolute values, carrying
    each entry's sign, |r_l| < 2^lam) becomes the rows r_0 .. r_{k-1} plus
    k - 1 new columns holding 2^lam on the superdiagonal and -1 on the
    diagonal of the digit rows.  Adding 2^lam times digit row l+1 to digit
    row l from the last upwards turns the first digit row back into r and
    leaves a single -1 in each new column, so |det| is unchanged and the
    result is unimodular exactly when B is.  Rows not listed stay as they are
    (with zeros in the new columns)."""
    n = len(b)
    base = 1 << lam
    digits = {}
    for r in rows:
        row = [int(v) for v in b[r]]
        width = max((abs(v).bit_length() for v in row), default=0)
        k = max(1, -(-width // lam))
        dr = []
        for l in range(k):
            dr.append([(1 if v >= 0 else -1) * ((abs(v) >> (lam * l)) & (base - 1)) for v in row])
        digits[r] = dr
    extra = sum(len(v) - 1 for v in digits.values())
    N = n + extra
    out = []
    col = n
    for r in range(n):
        if r not in digits:
            out.append([int(v) for v in b[r]] + [0] * extra)
            continue
        dr = digits[r]
        k = len(dr)
        for l in range(k):
            row = dr[l] + [0] * extra
            if l > 0:
                row[col + l - 1] = -1
            if l < k - 1:
                row[col + l] = base
            out.append(row)
        col += k - 1
    assert len(out) == N and all(len(r) == N for r in out)
    return out
