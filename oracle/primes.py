"""Oracle: the RNS basis (Section 3.1, the bullet on exact double-precision
accumulation, which takes primes consecutively below a bound).

Reading: the basis is the L largest primes strictly below the bound, in
descending order; the bound is 2^26 for every workload here (the paper derives
its bound from a full-length dot product; the GPU paths block the dot product
instead, so the bound is fixed).
"""
from __future__ import annotations

from math import isqrt


def is_prime(x: int) -> bool:
    """Trial division by every odd number up to sqrt(x)."""
    if x < 2:
        return False
    if x % 2 == 0:
        return x == 2
    for d in range(3, isqrt(x) + 1, 2):
        if x % d == 0:
            return False
    return True


def largest_primes_below(bound: int, count: int) -> list[int]:
    """The ``count`` largest primes p < bound, descending."""
    out = []
    x = bound - 1
    while len(out) < count:
        if x < 2:
            raise ValueError("not enough primes below bound")
        if is_prime(x):
            out.append(x)
        x -= 1
    return out


def product(primes) -> int:
    m = 1
    for p in primes:
        m *= int(p)
    return m
