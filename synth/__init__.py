"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lays them out; it holds none of the
arithmetic of the method (no reduction, no products, no reconstruction, no
Smith form).  Both the CPU oracle and the GPU path receive the arrays built
here, so no random-number parity between the two sides is ever needed.

Every generator uses numpy's ``default_rng`` (PCG64) with an explicit seed.

Workloads (sizes and value ranges follow the paper's setting of an exact
multi-modular product over word-size primes, Section 3.1, and its test family
of Section 4.1):

* ``square_pair``      -- two n x n int64 matrices, entries uniform in [-b, b]
                          (the n = 4096, b = 2^20 product is the headline one).
* ``small_smith``      -- one 64 x 64 matrix, entries uniform in [-99, 99].
* ``planted_smith``    -- A = U diag(s) V with U, V products of random
                          elementary operations and a planted divisor chain s.
* ``uneven_batch``     -- many independent products of log-uniform size.
* ``serving_stream``   -- Poisson arrivals of Smith-form requests.
* ``vandermonde_mod``  -- the family A_ij = i^j mod n of Section 4.1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

# The 25 primes below 100; used only as a pool to draw planted factors from.
PRIMES_BELOW_100 = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47,
                    53, 59, 61, 67, 71, 73, 79, 83, 89, 97)


def uniform_matrix(rows: int, cols: int, bound: int, seed: int) -> np.ndarray:
    """Entries i.i.d. uniform in [-bound, bound], int64, C-contiguous."""
    rng = np.random.default_rng(seed)
    return rng.integers(-bound, bound + 1, size=(rows, cols), dtype=np.int64)


def square_pair(n: int = 4096, bound: int = 1 << 20, seed_a: int = 0,
                seed_b: int = 1):
    """The single large product: A from seed_a, B from seed_b."""
    return (uniform_matrix(n, n, bound, seed_a),
            uniform_matrix(n, n, bound, seed_b))


def uniform_residues(primes, rows: int, cols: int, seed: int) -> np.ndarray:
    """Stress input: plane j uniform in [0, primes[j]), uint32 [L, rows, cols]."""
    rng = np.random.default_rng(seed)
    out = np.empty((len(primes), rows, cols), dtype=np.uint32)
    for j, p in enumerate(primes):
        out[j] = rng.integers(0, int(p), size=(rows, cols), dtype=np.int64)
    return out


def small_smith(seed: int = 0, attempt: int = 0, n: int = 64,
                bound: int = 99) -> np.ndarray:
    """The small Smith-form input.  ``attempt`` k returns the (k+1)-th draw of
    the same generator, so a caller that finds a draw singular asks for the
    next one."""
    rng = np.random.default_rng(seed)
    a = None
    for _ in range(attempt + 1):
        a = rng.integers(-bound, bound + 1, size=(n, n), dtype=np.int64)
    return a


@dataclass
class Planted:
    a: np.ndarray          # int64 n x n
    s: List[int]           # planted invariant factors, ascending, s_i | s_{i+1}
    attempts: int = 1


def planted_chain(n: int, rng: np.random.Generator, events: int = 5) -> List[int]:
    """Divisor chain: ``events`` times, pick a position q uniform in [1, n] and a
    prime from the pool, and multiply s_q, ..., s_n by it."""
    s = [1] * n
    for _ in range(events):
        q = int(rng.integers(1, n + 1))
        f = PRIMES_BELOW_100[int(rng.integers(0, len(PRIMES_BELOW_100)))]
        for i in range(q - 1, n):
            s[i] *= f
    return s


def _random_ops(n: int, count: int, rng: np.random.Generator):
    i = rng.integers(0, n, size=count)
    j = rng.integers(0, n - 1, size=count)
    j = j + (j >= i)                      # uniform over j != i
    c = rng.choice(np.array([-3, -2, -1, 1, 2, 3], dtype=np.int64), size=count)
    return i, j, c


def planted_smith(n: int, seed: int = 0, ops_per_dim: int = 4,
                  limit_bits: int = 62, max_attempts: int = 8) -> Planted:
    """A = U diag(s) V, U (V) the product of ops_per_dim*n random row (column)
    operations x_i += c x_j, i != j, c in {+-1, +-2, +-3}; det U = det V = 1.
    The operations are applied to diag(s) directly (columns first, then rows),
    which builds U (diag(s) V) without forming U or V.  A draw whose entries
    reach 2^limit_bits at any point is redrawn from the same generator."""
    rng = np.random.default_rng(seed)
    lim = 1 << limit_bits
    for attempt in range(1, max_attempts + 1):
        s = planted_chain(n, rng)
        a = np.zeros((n, n), dtype=np.int64)
        a[np.arange(n), np.arange(n)] = np.array(s, dtype=np.int64)
        ok = True
        ci, cj, cc = _random_ops(n, ops_per_dim * n, rng)
        for i, j, c in zip(ci, cj, cc):            # column ops: col_i += c col_j
            col = a[:, i] + c * a[:, j]
            if np.abs(col).max() >= lim // 4:
                ok = False
                break
            a[:, i] = col
        if ok:
            ri, rj, rc = _random_ops(n, ops_per_dim * n, rng)
            for i, j, c in zip(ri, rj, rc):        # row ops: row_i += c row_j
                row = a[i, :] + c * a[j, :]
                if np.abs(row).max() >= lim // 4:
                    ok = False
                    break
                a[i, :] = row
        if ok:
            return Planted(a=a, s=s, attempts=attempt)
    raise RuntimeError("planted_smith: entries kept exceeding the int64 limit")


def planted_small(n: int, seed: int = 0, factors=(2, 3, 2, 5, 2, 7, 3, 2), ops_per_dim: int = 2,
                  cap: int = 1 << 20) -> Planted:
    """A = U diag(s) V with small entries and several invariants above 1: the
    k-th factor multiplies s_{n-k}, ..., s_n (k = 1, 2, ...), so the last
    len(factors) invariants are nontrivial and form a divisor chain.  U and V
    are products of ops_per_dim*n random operations x_i += c x_j, c = +-1 (on
    columns, then rows of diag(s)); an operation that would make an entry
    reach ``cap`` is skipped, so |a_ij| < cap."""
    rng = np.random.default_rng(seed)
    s = [1] * n
    for k, f in enumerate(factors, start=1):
        for i in range(n - k, n):
            s[i] *= f
    a = np.zeros((n, n), dtype=np.int64)
    a[np.arange(n), np.arange(n)] = np.array(s, dtype=np.int64)
    for axis in (1, 0):
        i = rng.integers(0, n, size=ops_per_dim * n)
        j = rng.integers(0, n - 1, size=ops_per_dim * n)
        j = j + (j >= i)
        c = rng.choice(np.array([-1, 1], dtype=np.int64), size=ops_per_dim * n)
        for ii, jj, cc in zip(i, j, c):
            if axis == 1:
                new = a[:, ii] + cc * a[:, jj]
                if np.abs(new).max() < cap:
                    a[:, ii] = new
            else:
                new = a[ii, :] + cc * a[jj, :]
                if np.abs(new).max() < cap:
                    a[ii, :] = new
    return Planted(a=a, s=s)


@dataclass
class Problem:
    m: int
    n: int
    k: int
    a: np.ndarray
    b: np.ndarray


def uneven_sizes(count: int = 512, lo: int = 32, hi: int = 1024,
                 seed: int = 0) -> List[int]:
    """n_i = round(exp(U(ln lo, ln hi)))."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return [int(round(math.exp(x))) for x in u]


def uneven_batch(count: int = 512, lo: int = 32, hi: int = 1024,
                 bound: int = 1 << 16, seed: int = 0) -> List[Problem]:
    """Independent square products of log-uniform size, entries in [-bound, bound]."""
    sizes = uneven_sizes(count, lo, hi, seed)
    rng = np.random.default_rng(seed + 1)
    out = []
    for n in sizes:
        a = rng.integers(-bound, bound + 1, size=(n, n), dtype=np.int64)
        b = rng.integers(-bound, bound + 1, size=(n, n), dtype=np.int64)
        out.append(Problem(n, n, n, a, b))
    return out


@dataclass
class Request:
    rid: int
    arrival: float      # seconds from stream start
    n: int
    seed: int


@dataclass
class ServingStream:
    rate: float
    requests: List[Request] = field(default_factory=list)


def serving_stream(count: int, rate: float, lo: int = 100, hi: int = 4000,
                   tail_n: int = 10007, tail_at: int = 50,
                   seed: int = 0) -> ServingStream:
    """Poisson arrivals (exponential gaps of mean 1/rate); sizes log-uniform in
    [lo, hi]; one request of size tail_n at position tail_at (0 disables)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    reqs = []
    for r in range(count):
        n = int(round(math.exp(u[r])))
        if tail_n and r == tail_at:
            n = tail_n
        reqs.append(Request(r, float(t[r]), n, seed * 1000003 + r))
    return ServingStream(rate, reqs)


def request_matrix(req: Request, bound: int = 1 << 10, attempt: int = 0) -> np.ndarray:
    """The matrix of one serving request (redraw with attempt+1 if singular)."""
    return small_smith(seed=req.seed, attempt=attempt, n=req.n, bound=bound)


def vandermonde_mod(n: int) -> np.ndarray:
    """A_ij = i^j mod n for 0 <= i, j < n, with 0^0 = 1 (Section 4.1)."""
    a = np.empty((n, n), dtype=np.int64)
    for i in range(n):
        v = 1 % n
        for j in range(n):
            a[i, j] = v
            v = (v * i) % n
    return a
