"""Oracle: the Smith normal form of a nonsingular integer matrix (Section 1).

For nonsingular A in Z^{n x n} the Smith form is the unique
S = diag(s_1, ..., s_n), s_i > 0, s_1 | s_2 | ... | s_n, with U A V = S for
unimodular U, V.  The oracle computes it as follows.

1. d = |det A| by fraction-free (Bareiss) elimination, exact over Z.
   d = 0 means A is singular, which the method does not cover.
2. Because d * A^{-1} is integral, d Z^n lies inside the column lattice of A,
   so Z^n / A Z^n = (Z/dZ)^n / (image of A mod d).  The matrix is therefore
   reduced mod d and diagonalised by unimodular row and column operations built
   from extended gcds, reducing every entry mod d after each operation (adding a
   multiple of d to one entry subtracts a vector of d Z^n from a column, which
   leaves the quotient unchanged).
3. A diagonal entry e turns into the cyclic factor Z / gcd(e, d) (gcd(0, d) = d).
4. The diagonal is brought into divisibility order with the identity
   diag(a, b) ~ diag(gcd(a, b), lcm(a, b)).

This is the textbook "Smith form modulo a multiple of the determinant".  It
shares nothing with the massager method of Section 2; it is only the definition
of S made computable.
"""
from __future__ import annotations

from math import gcd
from typing import List, Sequence

import numpy as np


class Singular(ValueError):
    pass


def bareiss_det(a) -> int:
    """Exact determinant by Bareiss fraction-free elimination (row pivoting)."""
    m = [[int(v) for v in row] for row in np.asarray(a).tolist()]
    n = len(m)
    if n == 0:
        return 1
    sign = 1
    prev = 1
    for k in range(n - 1):
        if m[k][k] == 0:
            piv = next((i for i in range(k + 1, n) if m[i][k] != 0), None)
            if piv is None:
                return 0
            m[k], m[piv] = m[piv], m[k]
            sign = -sign
        akk = m[k][k]
        for i in range(k + 1, n):
            aik = m[i][k]
            row_i = m[i]
            row_k = m[k]
            for j in range(k + 1, n):
                # Sylvester's identity: the division is exact.
                row_i[j] = (row_i[j] * akk - aik * row_k[j]) // prev
            row_i[k] = 0
        prev = akk
    return sign * m[n - 1][n - 1]


def xgcd(a: int, b: int):
    """(g, x, y) with x*a + y*b = g = gcd(a, b) >= 0."""
    x0, y0, x1, y1 = 1, 0, 0, 1
    while b:
        q, r = divmod(a, b)
        a, b = b, r
        x0, x1 = x1, x0 - q * x1
        y0, y1 = y1, y0 - q * y1
    if a < 0:
        a, x0, y0 = -a, -x0, -y0
    return a, x0, y0


def _pivot_op(a: int, b: int):
    """(g, x, y) for the 2x2 unimodular operation [[x, y], [-b/g, a/g]] that maps
    (a, b) to (g, 0).  When a divides b the operation is the plain elimination
    x = 1, y = 0, which leaves the pivot row (column) untouched."""
    if a != 0 and b % a == 0:
        return a, 1, 0
    return xgcd(a, b)


def _diagonalise_mod(m: List[List[int]], d: int) -> List[int]:
    """Diagonalise the square matrix m over Z/dZ by unimodular integer row and
    column operations; returns the diagonal (entries in [0, d))."""
    n = len(m)
    for k in range(n):
        while True:
            # Clear column k below the pivot with 2x2 unimodular row operations.
            for i in range(k + 1, n):
                b = m[i][k]
                if b == 0:
                    continue
                a = m[k][k]
                g, x, y = _pivot_op(a, b)
                ag, bg = a // g, b // g
                rk, ri = m[k], m[i]
                for j in range(k, n):
                    u, v = rk[j], ri[j]
                    rk[j] = (x * u + y * v) % d
                    ri[j] = (-bg * u + ag * v) % d
            # Clear row k right of the pivot with 2x2 unimodular column operations.
            dirty = False
            for j in range(k + 1, n):
                b = m[k][j]
                if b == 0:
                    continue
                a = m[k][k]
                g, x, y = _pivot_op(a, b)
                ag, bg = a // g, b // g
                for i in range(k, n):
                    u, v = m[i][k], m[i][j]
                    m[i][k] = (x * u + y * v) % d
                    m[i][j] = (-bg * u + ag * v) % d
                    if i > k and m[i][k] != 0:
                        dirty = True
            if not dirty:
                break
    return [m[i][i] for i in range(n)]


def _divisibility_order(g: List[int]) -> List[int]:
    """diag(g) -> Smith form, by diag(a, b) ~ diag(gcd, lcm) on every pair."""
    g = list(g)
    n = len(g)
    for i in range(n):
        for j in range(i + 1, n):
            a, b = g[i], g[j]
            h = gcd(a, b)
            g[i], g[j] = h, (a // h) * b if h else 0
    return g


def smith_form(a) -> List[int]:
    """Invariant factors s_1 | ... | s_n of a nonsingular integer matrix.
    Raises Singular when det A = 0."""
    a = np.asarray(a)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("square matrix expected")
    if n == 0:
        return []
    d = abs(bareiss_det(a))
    if d == 0:
        raise Singular("matrix is singular")
    if d == 1:
        return [1] * n
    m = [[int(v) % d for v in row] for row in a.tolist()]
    diag = _diagonalise_mod(m, d)
    g = [gcd(e, d) for e in diag]            # gcd(0, d) = d
    s = _divisibility_order(g)
    prod = 1
    for v in s:
        prod *= v
    assert prod == d, "invariant factors must multiply to |det A|"
    return s


def is_divisor_chain(s: Sequence[int]) -> bool:
    return all(int(s[i + 1]) % int(s[i]) == 0 for i in range(len(s) - 1)) and all(int(v) > 0 for v in s)


def det_mod(a, p: int) -> int:
    """det A mod p in [0, p) (from the exact determinant)."""
    return bareiss_det(a) % int(p)
