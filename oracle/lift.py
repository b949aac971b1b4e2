"""Oracle: one step of Dixon's p-adic lifting.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3 names Dixon's p-adic lifting as the solver behind the method's
linear systems (rational solving, and the integrality certification of the
Phase 2 projections in Section 2.2).  Given C = A^-1 mod p and a residual R
(initially the right-hand sides), one step computes

    X  = C (R mod p) mod p          (the next p-adic digit of A^-1 R)
    R' = (R - A X) / p              (exact: A X = R mod p when C = A^-1 mod p)

so that after K steps A (X_0 + p X_1 + ... + p^(K-1) X_(K-1)) = R_0 - p^K R_K.
The functions below are that definition written out.  For a C that is not
the inverse of A mod p the division is inexact; the step then reports it and
takes the quotient rounded toward zero (the convention of the HIP step
kernels' error path, fixed here so that such inputs can still be compared
entry by entry).

Matrices are in the mathematical layout: A, C are n x n, R and X are n x t
(one column per right-hand side).
"""
from __future__ import annotations

import numpy as np

from . import native, rns


def digit(C: np.ndarray, R: np.ndarray, p: int) -> np.ndarray:
    """X = C (R mod p) mod p, uint32 n x t.  C holds residues in [0, p)."""
    p = int(p)
    Rm = np.mod(np.asarray(R, dtype=np.int64), np.int64(p)).astype(np.uint32)
    C = np.asarray(C, dtype=np.uint32)
    if native.available():
        return native.modmatmul(C, Rm, p)
    return rns.modmatmul(C, Rm, p)


def _trunc_div(num: np.ndarray, p: int) -> np.ndarray:
    """num / p rounded toward zero, elementwise (int64 or object)."""
    q = abs(num) // p
    return np.where(num < 0, -q, q)


def residual(A: np.ndarray, X: np.ndarray, R: np.ndarray, p: int, rows=None):
    """R' = (R - A X) / p for the given rows (all when None), with the flag
    "p divides every R - A X".  Exact integers: int64 when every partial sum
    provably fits (n max|A| max|X| + max|R| < 2^63), Python integers otherwise.
    Returns (R' int64 or object, R' mod p uint32, exact)."""
    p = int(p)
    A = np.asarray(A, dtype=np.int64)
    X = np.asarray(X).astype(np.int64)
    R = np.asarray(R, dtype=np.int64)
    if rows is not None:
        rows = np.asarray(rows)
        A = A[rows]
        R = R[rows]
    n = A.shape[1]
    amax = max(abs(int(A.max())), abs(int(A.min()))) if A.size else 0
    xmax = int(X.max()) if X.size else 0
    rmax = max(abs(int(R.max())), abs(int(R.min()))) if R.size else 0
    if n * amax * xmax + rmax < (1 << 63):
        AX = native.exact_matmul(A, X) if native.available() else A @ X
        num = R - AX
    else:
        num = R.astype(object) - A.astype(object).dot(X.astype(object))
    exact = bool(np.all(num % p == 0))
    Rn = _trunc_div(num, p)
    Rnm = np.mod(Rn, p).astype(np.uint32)
    return Rn, Rnm, exact


def step(C: np.ndarray, A: np.ndarray, R: np.ndarray, p: int):
    """One lifting step: (X, R', R' mod p, exact)."""
    X = digit(C, R, p)
    Rn, Rnm, exact = residual(A, X, R, p)
    return X, Rn, Rnm, exact


def inverse_mod_p(A: np.ndarray, p: int) -> np.ndarray:
    """A^-1 mod p by Gauss-Jordan elimination over Z/pZ in Python integers
    (small n only).  Raises ValueError when p divides det A."""
    p = int(p)
    n = A.shape[0]
    M = [[int(v) % p for v in A[i]] + [1 if j == i else 0 for j in range(n)] for i in range(n)]
    for c in range(n):
        piv = next((r for r in range(c, n) if M[r][c]), None)
        if piv is None:
            raise ValueError("singular mod p")
        M[c], M[piv] = M[piv], M[c]
        inv = pow(M[c][c], -1, p)
        M[c] = [v * inv % p for v in M[c]]
        for r in range(n):
            if r != c and M[r][c]:
                f = M[r][c]
                M[r] = [(v - f * w) % p for v, w in zip(M[r], M[c])]
    return np.array([row[n:] for row in M], dtype=np.uint32)
