"""Oracle: the Residue Number System product of Section 3.1.

An integer matrix is reduced modulo each of L primes, the L residue matrices
are multiplied independently modulo their prime, and the integer result is
rebuilt by the Chinese Remainder Theorem.  Each function below is the plain
definition of one of those steps.
"""
from __future__ import annotations

from math import gcd, isqrt
from typing import Iterable, Sequence

import numpy as np

from . import native


# --------------------------------------------------------------------------
# Reduction (Section 3.1: each entry is reduced modulo each prime).
# --------------------------------------------------------------------------

def reduce(x: np.ndarray, primes: Sequence[int]) -> np.ndarray:
    """r_j = x mod p_j in [0, p_j) (floor semantics for negative x).

    x: int64 array of any shape.  Returns uint32 [L, *x.shape].
    numpy's ``mod`` with a positive divisor is the floor-mod, the same
    convention as Python's ``%``.
    """
    x = np.asarray(x, dtype=np.int64)
    out = np.empty((len(primes),) + x.shape, dtype=np.uint32)
    for j, p in enumerate(primes):
        out[j] = np.mod(x, np.int64(p))
    return out


def reduce_int(x: int, primes: Sequence[int]) -> list[int]:
    """The same for one Python integer of any size."""
    return [x % int(p) for p in primes]


# --------------------------------------------------------------------------
# Modular product (Section 3.1: one independent product per prime).
# --------------------------------------------------------------------------

# With residues below 2^26 each product is below 2^52, so 2048 of them sum
# below 2^63: the int64 partial sums over K-chunks of this length are exact.
_K_CHUNK = 2048


def modmatmul(a: np.ndarray, b: np.ndarray, p: int) -> np.ndarray:
    """C = (A @ B) mod p for residue matrices A (m x k), B (k x n) in [0, p).

    p < 2^26.  The sum over k is split into chunks of 2048 terms, each summed
    exactly in int64 and reduced mod p; the reduced chunk sums are added.
    Returns uint32 (m x n) in [0, p).
    """
    p = int(p)
    assert p < (1 << 26)
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    m, k = a.shape
    k2, n = b.shape
    assert k == k2
    acc = np.zeros((m, n), dtype=np.int64)
    for k0 in range(0, k, _K_CHUNK):
        part = a[:, k0:k0 + _K_CHUNK] @ b[k0:k0 + _K_CHUNK, :]
        acc = np.mod(acc + np.mod(part, p), p)
    return acc.astype(np.uint32)


def modmatmul_planes(a_res: np.ndarray, b_res: np.ndarray,
                     primes: Sequence[int], use_native: bool = True) -> np.ndarray:
    """Plane-by-plane product: C[j] = A[j] @ B[j] mod p_j, uint32 [L, m, n]."""
    out = []
    for j, p in enumerate(primes):
        if use_native and native.available():
            out.append(native.modmatmul(a_res[j], b_res[j], int(p)))
        else:
            out.append(modmatmul(a_res[j], b_res[j], int(p)))
    return np.stack(out) if out else np.zeros((0,) + (a_res.shape[1], b_res.shape[2]), np.uint32)


def modmatmul_entry(a_row: np.ndarray, b_col: np.ndarray, p: int) -> int:
    """One entry, sum_k a_row[k] * b_col[k] mod p, in Python integers."""
    return sum(int(x) * int(y) for x, y in zip(a_row, b_col)) % int(p)


# --------------------------------------------------------------------------
# Exact integer product (the quantity the RNS product represents).
# --------------------------------------------------------------------------

def exact_matmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """C = A @ B over the integers.  int64 when every |C_ij| provably fits
    (max|A| * max|B| * k < 2^63), otherwise a Python-int object array."""
    a = np.asarray(a)
    b = np.asarray(b)
    k = a.shape[1]
    ma = int(np.abs(a.astype(object)).max()) if a.size else 0
    mb = int(np.abs(b.astype(object)).max()) if b.size else 0
    if ma * mb * k < (1 << 63) and a.dtype == np.int64 and b.dtype == np.int64:
        if native.available():
            return native.exact_matmul(a, b)
        return a @ b
    ao = a.astype(object)
    bo = b.astype(object)
    return ao.dot(bo)


def exact_entry(a_row, b_col) -> int:
    return sum(int(x) * int(y) for x, y in zip(a_row, b_col))


# --------------------------------------------------------------------------
# Chinese remaindering (Section 3.1: the integer result is reconstructed
# from the L residues).
# --------------------------------------------------------------------------

class CRTBasis:
    """Lagrange form of the CRT: x = sum_j r_j * (M/p_j) * ((M/p_j)^-1 mod p_j)
    mod M, with M = prod p_j.  The result is then moved to the symmetric range
    [-(M-1)/2, (M-1)/2] (M is odd, so there is no tie)."""

    def __init__(self, primes: Sequence[int]):
        self.primes = [int(p) for p in primes]
        m = 1
        for p in self.primes:
            m *= p
        self.M = m
        self.weights = []
        for p in self.primes:
            mj = m // p
            self.weights.append(mj * pow(mj % p, -1, p))

    def reconstruct(self, residues: Iterable[int]) -> int:
        x = sum(int(r) * w for r, w in zip(residues, self.weights)) % self.M
        if x > (self.M - 1) // 2:
            x -= self.M
        return x


def crt(residues: Sequence[int], primes: Sequence[int]) -> int:
    return CRTBasis(primes).reconstruct(residues)


def crt_planes(res: np.ndarray, primes: Sequence[int]) -> np.ndarray:
    """Entry-wise CRT of uint32 planes [L, ...] -> object array of Python ints."""
    basis = CRTBasis(primes)
    L = res.shape[0]
    flat = res.reshape(L, -1)
    out = np.empty(flat.shape[1], dtype=object)
    for e in range(flat.shape[1]):
        out[e] = basis.reconstruct(flat[:, e])
    return out.reshape(res.shape[1:])


# --------------------------------------------------------------------------
# Output encoding: W little-endian 64-bit words, two's complement.
# --------------------------------------------------------------------------

class Overflow(ValueError):
    pass


def to_words(x: int, W: int) -> list[int]:
    """Two's-complement encoding of x in W 64-bit words, least significant
    first.  Raises Overflow when x is outside [-2^(64W-1), 2^(64W-1))."""
    lim = 1 << (64 * W - 1)
    if not (-lim <= x < lim):
        raise Overflow(x)
    u = x % (1 << (64 * W))
    return [(u >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(W)]


def from_words(words: Sequence[int]) -> int:
    u = 0
    for i, w in enumerate(words):
        u |= int(w) << (64 * i)
    W = len(words)
    if u >> (64 * W - 1):
        u -= 1 << (64 * W)
    return u


# --------------------------------------------------------------------------
# How many primes a result needs.
# --------------------------------------------------------------------------

def primes_needed(bound: int, primes: Sequence[int]) -> int:
    """Smallest L with prod_{j<L} p_j >= 2*bound + 1, so that every integer of
    absolute value at most ``bound`` is recovered from its residues."""
    m = 1
    for L, p in enumerate(primes, start=1):
        m *= int(p)
        if m >= 2 * bound + 1:
            return L
    raise ValueError("basis too short for bound")


def hadamard_bound(a: np.ndarray) -> int:
    """Hadamard's bound on |det A|: the smaller of the products of the row and
    the column Euclidean norms, as ceil(sqrt(prod of squared norms))."""
    ao = np.asarray(a).astype(object)
    rows = 1
    for i in range(ao.shape[0]):
        rows *= sum(int(v) * int(v) for v in ao[i, :])
    cols = 1
    for j in range(ao.shape[1]):
        cols *= sum(int(v) * int(v) for v in ao[:, j])
    sq = min(rows, cols)
    r = isqrt(sq)
    if r * r < sq:
        r += 1
    return r


def product_entry_bound(a: np.ndarray, b: np.ndarray) -> int:
    """A bound on max |(A B)_ij|: max row norm of A times max column norm of B
    (Cauchy-Schwarz), rounded up."""
    ao = np.asarray(a).astype(object)
    bo = np.asarray(b).astype(object)
    ra = max((sum(int(v) * int(v) for v in ao[i, :]) for i in range(ao.shape[0])), default=0)
    cb = max((sum(int(v) * int(v) for v in bo[:, j]) for j in range(bo.shape[1])), default=0)
    sq = ra * cb
    r = isqrt(sq)
    if r * r < sq:
        r += 1
    return r


def coprime(primes: Sequence[int]) -> bool:
    ps = [int(p) for p in primes]
    return all(gcd(ps[i], ps[j]) == 1 for i in range(len(ps)) for j in range(i + 1, len(ps)))
