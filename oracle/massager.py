"""Oracle: what a Smith massager must satisfy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.1 defines a Smith massager of a nonsingular integer A with Smith
form S in two equivalent ways:

* Definition 1: a pair (S, F) with A F = 0 modulo S (column j of A F divisible
  by s_j) and an integer W with W F = I modulo S (column-wise again).
* Eq. (1): a tuple (U, M, T, S) of n x n integer matrices, T unit upper
  triangular and S in Smith form, such that the 2n x 2n matrix

      B = diag(A, I) [I 0; U I] [I M; 0 T] diag(I, S^-1)

  is integral; the massager is maximal exactly when B is unimodular, i.e.
  when det S = |det A| (the product gives det B det S = det A).

Section 4.2 checks a returned massager by divisibility of the s_i, by
integrality of A M S^-1 and (T + U M) S^-1 (the two non-trivial blocks of B),
and by |det A| / prod s_i = 1.  The functions below write these out with
exact integers (Python ints); `massaged_matrix` multiplies out Eq. (1) with
exact fractions, factor by factor, as the definition states it.

Reading of the sign in Definition 1's remark that W = T^-1 U: with Eq. (1)
as printed, (T + U M) S^-1 integral gives T^-1 U M = -I modulo S, so the W of
Definition 1 is -T^-1 U here (`definition1_W`).
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import smith as osmith


def _mat(x) -> List[List[int]]:
    return [[int(v) for v in row] for row in x]


def _mul(X, Y) -> List[List]:
    """Exact product of integer (or Fraction) matrices (numpy object dot)."""
    return np.array(X, dtype=object).dot(np.array(Y, dtype=object)).tolist()


def massaged_matrix(A, U, M, T, S: Sequence[int]) -> List[List[Fraction]]:
    """B of Eq. (1) as exact fractions: the four factors multiplied in order."""
    A, U, M, T = _mat(A), _mat(U), _mat(M), _mat(T)
    n = len(A)
    N = 2 * n

    def block(tl, tr, bl, br):
        out = [[Fraction(0)] * N for _ in range(N)]
        for i in range(n):
            for j in range(n):
                out[i][j] = Fraction(tl[i][j])
                out[i][n + j] = Fraction(tr[i][j])
                out[n + i][j] = Fraction(bl[i][j])
                out[n + i][n + j] = Fraction(br[i][j])
        return out

    I = [[int(i == j) for j in range(n)] for i in range(n)]
    Z = [[0] * n for _ in range(n)]
    Sinv = [[Fraction(1, int(S[i])) if i == j else Fraction(0) for j in range(n)] for i in range(n)]
    F1 = block(A, Z, Z, I)
    F2 = block(I, Z, U, I)
    F3 = block(I, M, Z, T)
    F4 = block(I, Z, Z, Sinv)
    return _mul(_mul(_mul(F1, F2), F3), F4)


def is_integral(B) -> bool:
    return all(Fraction(v).denominator == 1 for row in B for v in row)


def checks(A, U, M, T, S: Sequence[int], det_abs: Optional[int] = None) -> Dict[str, bool]:
    """Section 4.2's checks of a massager (U, M, T, S) of A, plus the shape
    conditions of Eq. (1) (T unit upper triangular, S positive).  |det A| is
    the Bareiss determinant unless given (det_abs, e.g. a stored oracle value)."""
    A, U, M, T = _mat(A), _mat(U), _mat(M), _mat(T)
    S = [int(v) for v in S]
    n = len(A)
    AM = _mul(A, M)
    UM = _mul(U, M)
    out = {
        "positive": all(v > 0 for v in S),
        "divisibility": all(S[i + 1] % S[i] == 0 for i in range(n - 1)),
        "AMS_integral": all(AM[i][j] % S[j] == 0 for i in range(n) for j in range(n)),
        "TUMS_integral": all((T[i][j] + UM[i][j]) % S[j] == 0 for i in range(n) for j in range(n)),
        "T_unit_upper": all(T[i][i] == 1 for i in range(n)) and all(T[i][j] == 0 for i in range(n) for j in range(i)),
    }
    prod = 1
    for v in S:
        prod *= v
    out["unimodular"] = (abs(osmith.bareiss_det(A)) if det_abs is None else int(det_abs)) == prod
    return out


def definition1_W(U, T) -> List[List[int]]:
    """W = -T^-1 U (T unit upper triangular: back substitution over Z)."""
    U, T = _mat(U), _mat(T)
    n = len(T)
    W = [[0] * len(U[0]) for _ in range(n)]
    for i in range(n - 1, -1, -1):
        for c in range(len(U[0])):
            v = U[i][c] - sum(T[i][k] * W[k][c] for k in range(i + 1, n))
            W[i][c] = v
    return [[-v for v in row] for row in W]


def definition1(A, F, W, S: Sequence[int]) -> bool:
    """A F = 0 and W F = I, both column-wise modulo S (Definition 1)."""
    A, F, W = _mat(A), _mat(F), _mat(W)
    S = [int(v) for v in S]
    n = len(A)
    AF = _mul(A, F)
    WF = _mul(W, F)
    return all(AF[i][j] % S[j] == 0 for i in range(n) for j in range(n)) and all(
        (WF[i][j] - (1 if i == j else 0)) % S[j] == 0 for i in range(n) for j in range(n))
