"""Pins for the oracle's basis, reduction, modular product, CRT and encoding.

Each check compares the oracle with something other than itself: a library
routine (sympy), brute force on tiny inputs, a closed form, or an invariant.
"""
import random

import numpy as np
import pytest
import sympy
from sympy.ntheory.modular import crt as sympy_crt

from oracle import native, primes as op, rns
import synth

P26 = 1 << 26


# ---------------------------------------------------------------- primes --

def test_is_prime_matches_sympy():
    for x in range(0, 5000):
        assert op.is_prime(x) == sympy.isprime(x), x
    rng = random.Random(1)
    for _ in range(300):
        x = rng.randrange(P26 - 100000, P26)
        assert op.is_prime(x) == sympy.isprime(x), x


def test_basis_is_the_largest_primes_below_2_26():
    got = op.largest_primes_below(P26, 26)
    want = []
    x = P26
    for _ in range(26):
        x = sympy.prevprime(x)
        want.append(x)
    assert got == want
    # consecutive: no prime is skipped between the 26th and 2^26
    assert len(list(sympy.primerange(got[-1], P26))) == 26
    assert got[0] == 67108859 and got[23] == 67108493
    assert op.product(got[:24]).bit_length() == 624
    assert rns.coprime(got)


# ---------------------------------------------------------------- reduce --

def test_reduce_invariants_and_extremes():
    ps = op.largest_primes_below(P26, 5) + [3, 7]
    rng = np.random.default_rng(3)
    x = rng.integers(-(1 << 63), (1 << 63) - 1, size=500, dtype=np.int64)
    x = np.concatenate([x, np.array([0, 1, -1, -(1 << 63), (1 << 63) - 1,
                                     ps[0], -ps[0], ps[0] - 1, -(ps[0] - 1)],
                                    dtype=np.int64)])
    r = rns.reduce(x, ps)
    for j, p in enumerate(ps):
        for e, xv in enumerate(x.tolist()):
            rv = int(r[j, e])
            assert 0 <= rv < p
            assert (xv - rv) % p == 0
    assert int(rns.reduce(np.array([-1]), [ps[0]])[0, 0]) == ps[0] - 1
    assert int(rns.reduce(np.array([ps[0]]), [ps[0]])[0, 0]) == 0


# ------------------------------------------------------------- modmatmul --

def _brute(a, b, p):
    m, k = a.shape
    n = b.shape[1]
    c = np.zeros((m, n), dtype=np.uint32)
    for i in range(m):
        for j in range(n):
            s = 0
            for t in range(k):
                s += int(a[i, t]) * int(b[t, j])
            c[i, j] = s % p
    return c


@pytest.mark.parametrize("use_native", [False, True])
def test_modmatmul_brute_force_tiny(use_native):
    ps = op.largest_primes_below(P26, 3) + [2, 3, 97]
    rng = np.random.default_rng(5)
    for trial in range(40):
        m, k, n = (int(v) for v in rng.integers(1, 8, size=3))
        p = ps[trial % len(ps)]
        a = rng.integers(0, p, size=(m, k)).astype(np.uint32)
        b = rng.integers(0, p, size=(k, n)).astype(np.uint32)
        got = native.modmatmul(a, b, p) if use_native else rns.modmatmul(a, b, p)
        assert np.array_equal(got, _brute(a, b, p))


@pytest.mark.parametrize("use_native", [False, True])
def test_modmatmul_closed_forms(use_native):
    p = 67108859
    f = native.modmatmul if use_native else rns.modmatmul
    rng = np.random.default_rng(6)
    b = rng.integers(0, p, size=(37, 29)).astype(np.uint32)
    # identity: I B = B
    assert np.array_equal(f(np.eye(37, dtype=np.uint32), b, p), b)
    # all entries p-1: (p-1)^2 = 1 mod p, so every entry is k mod p; k crosses
    # the 2048-term chunk boundary twice.
    for k in (1, 2047, 2048, 2049, 5000):
        a = np.full((3, k), p - 1, dtype=np.uint32)
        bb = np.full((k, 2), p - 1, dtype=np.uint32)
        assert np.all(f(a, bb, p) == k % p)
    # k = 1: outer product
    u = rng.integers(0, p, size=(6, 1)).astype(np.uint32)
    v = rng.integers(0, p, size=(1, 5)).astype(np.uint32)
    want = np.array([[int(x) * int(y) % p for y in v[0]] for x in u[:, 0]], dtype=np.uint32)
    assert np.array_equal(f(u, v, p), want)


def test_modmatmul_native_equals_numpy_and_exact_product():
    p = 67108837
    rng = np.random.default_rng(7)
    a = rng.integers(0, p, size=(33, 4500)).astype(np.uint32)
    b = rng.integers(0, p, size=(4500, 21)).astype(np.uint32)
    c1 = rns.modmatmul(a, b, p)
    c2 = native.modmatmul(a, b, p)
    assert np.array_equal(c1, c2)
    # exact product in Python integers, reduced at the end
    exact = a.astype(object).dot(b.astype(object))
    assert np.array_equal(np.vectorize(lambda v: v % p)(exact).astype(np.uint32), c1)


def test_exact_matmul_against_python_ints():
    rng = np.random.default_rng(8)
    a = rng.integers(-(1 << 20), (1 << 20) + 1, size=(17, 300), dtype=np.int64)
    b = rng.integers(-(1 << 20), (1 << 20) + 1, size=(300, 13), dtype=np.int64)
    want = a.astype(object).dot(b.astype(object))
    assert np.array_equal(rns.exact_matmul(a, b).astype(object), want)
    # entries too large for int64 go through Python integers
    big = np.full((2, 3), (1 << 40), dtype=np.int64)
    bigb = np.full((3, 2), (1 << 40), dtype=np.int64)
    out = rns.exact_matmul(big, bigb)
    assert out[0, 0] == 3 * (1 << 80)


# ------------------------------------------------------------------- CRT --

def test_crt_round_trip_including_endpoints():
    ps = op.largest_primes_below(P26, 24)
    basis = rns.CRTBasis(ps)
    M = basis.M
    h = (M - 1) // 2
    rng = random.Random(9)
    xs = [0, 1, -1, h, -h, h - 1, -h + 1] + [rng.randrange(-h, h + 1) for _ in range(200)]
    for x in xs:
        assert basis.reconstruct(rns.reduce_int(x, ps)) == x


def test_crt_brute_force_small_primes():
    ps = [3, 5, 7, 11]
    M = 3 * 5 * 7 * 11
    for x in range(-(M - 1) // 2, (M - 1) // 2 + 1):
        r = [x % p for p in ps]
        # brute force: the unique value in the symmetric range with these residues
        cand = [y for y in range(-(M - 1) // 2, (M - 1) // 2 + 1)
                if all(y % p == rv for p, rv in zip(ps, r))]
        assert cand == [x]
        assert rns.crt(r, ps) == x


def test_crt_agrees_with_sympy():
    ps = op.largest_primes_below(P26, 10)
    rng = random.Random(10)
    for _ in range(100):
        r = [rng.randrange(p) for p in ps]
        x = rns.crt(r, ps)
        y, M = sympy_crt(ps, r)
        y = int(y)
        if y > (int(M) - 1) // 2:
            y -= int(M)
        assert x == y


def test_crt_redundant_primes_small_values():
    # |x| < 2^52 is fixed by three primes; the other 21 residues must agree.
    ps = op.largest_primes_below(P26, 24)
    rng = random.Random(11)
    for _ in range(50):
        x = rng.randrange(-(1 << 52), 1 << 52)
        r = rns.reduce_int(x, ps)
        assert rns.crt(r[:3], ps[:3]) == x
        assert rns.crt(r, ps) == x


def test_crt_planes_matches_scalar():
    ps = op.largest_primes_below(P26, 4)
    res = synth.uniform_residues(ps, 3, 5, seed=12)
    out = rns.crt_planes(res, ps)
    for i in range(3):
        for j in range(5):
            assert out[i, j] == rns.crt([int(res[l, i, j]) for l in range(4)], ps)


# -------------------------------------------------------------- encoding --

def test_words_encoding():
    assert rns.to_words(0, 1) == [0]
    assert rns.to_words(-1, 1) == [0xFFFFFFFFFFFFFFFF]
    assert rns.to_words(-1, 3) == [0xFFFFFFFFFFFFFFFF] * 3
    assert rns.to_words(1 << 64, 2) == [0, 1]
    assert rns.to_words(-(1 << 64), 2) == [0, 0xFFFFFFFFFFFFFFFF]
    assert rns.to_words((1 << 63) - 1, 1) == [0x7FFFFFFFFFFFFFFF]
    assert rns.to_words(-(1 << 63), 1) == [0x8000000000000000]
    with pytest.raises(rns.Overflow):
        rns.to_words(1 << 63, 1)
    with pytest.raises(rns.Overflow):
        rns.to_words(-(1 << 63) - 1, 1)
    rng = random.Random(13)
    for _ in range(100):
        W = rng.randrange(1, 6)
        x = rng.randrange(-(1 << (64 * W - 1)), 1 << (64 * W - 1))
        assert rns.from_words(rns.to_words(x, W)) == x


# ---------------------------------------------------------------- bounds --

def test_primes_needed_and_hadamard():
    ps = op.largest_primes_below(P26, 30)
    assert rns.primes_needed(1, ps) == 1
    assert rns.primes_needed((ps[0] - 1) // 2, ps) == 1
    assert rns.primes_needed((ps[0] + 1) // 2, ps) == 2
    # diagonal matrix: Hadamard's bound is |det| exactly
    d = np.diag(np.array([3, -5, 7, 2], dtype=np.int64))
    assert rns.hadamard_bound(d) == 210
    # Sylvester-Hadamard matrix of order 4: |det| = 4^(4/2) = 16, bound is tight
    h2 = np.array([[1, 1], [1, -1]], dtype=np.int64)
    h4 = np.kron(h2, h2)
    assert rns.hadamard_bound(h4) == 16
    assert abs(int(sympy.Matrix(h4.tolist()).det())) == 16
    # the bound holds on random matrices
    rng = np.random.default_rng(14)
    for _ in range(10):
        a = rng.integers(-9, 10, size=(6, 6))
        assert abs(int(sympy.Matrix(a.tolist()).det())) <= rns.hadamard_bound(a)


# ------------------------------------------- single entries and plane stacks --
# modmatmul_entry and exact_entry are the expected values of sampled checks at
# sizes where whole products are too slow; modmatmul_planes is the per-prime
# loop of the CPU baseline.  Each is pinned here against brute force, closed
# forms and the whole-matrix routines above.

def test_modmatmul_entry_brute_force_and_closed_forms():
    rng = np.random.default_rng(21)
    ps = op.largest_primes_below(P26, 2) + [5, 97]
    for trial in range(30):
        p = ps[trial % len(ps)]
        m, k, n = (int(v) for v in rng.integers(1, 7, size=3))
        a = rng.integers(0, p, size=(m, k)).astype(np.uint32)
        b = rng.integers(0, p, size=(k, n)).astype(np.uint32)
        want = _brute(a, b, p)
        for i in range(m):
            for j in range(n):
                assert rns.modmatmul_entry(a[i], b[:, j], p) == int(want[i, j])
    p = 67108859
    # (p-1)^2 = 1 mod p: a k-term row of p-1 against a column of p-1 gives k
    for k in (1, 2048, 4099):
        row = np.full(k, p - 1, dtype=np.uint32)
        assert rns.modmatmul_entry(row, row, p) == k % p
    # 2^25 * 2^25 = 2^50: the value mod p depends on p, so a swapped prime shows
    assert rns.modmatmul_entry(np.array([1 << 25]), np.array([1 << 25]), p) == (1 << 50) % p
    # an empty sum is 0
    assert rns.modmatmul_entry(np.zeros(0, np.uint32), np.zeros(0, np.uint32), p) == 0


def test_modmatmul_entry_matches_whole_products():
    p = 67108837
    rng = np.random.default_rng(22)
    a = rng.integers(0, p, size=(5, 3000)).astype(np.uint32)
    b = rng.integers(0, p, size=(3000, 4)).astype(np.uint32)
    c = native.modmatmul(a, b, p)
    for i in range(5):
        for j in range(4):
            assert rns.modmatmul_entry(a[i], b[:, j], p) == int(c[i, j])
    # row and column roles: entry (i, j) uses row i of A and column j of B
    a2 = np.arange(6, dtype=np.uint32).reshape(2, 3)
    b2 = np.array([[1, 0], [0, 0], [0, 10]], dtype=np.uint32)
    assert rns.modmatmul_entry(a2[1], b2[:, 1], 97) == (5 * 10) % 97
    assert rns.modmatmul_entry(a2[0], b2[:, 0], 97) == 0


def test_exact_entry_pins():
    rng = np.random.default_rng(23)
    a = rng.integers(-(1 << 20), (1 << 20) + 1, size=(4, 777), dtype=np.int64)
    b = rng.integers(-(1 << 20), (1 << 20) + 1, size=(777, 3), dtype=np.int64)
    c = native.exact_matmul(a, b)
    for i in range(4):
        for j in range(3):
            want = 0
            for t in range(777):
                want += int(a[i, t]) * int(b[t, j])
            assert rns.exact_entry(a[i], b[:, j]) == want == int(c[i, j])
    # closed forms: a row of ones sums the column; values beyond int64 stay exact
    col = np.array([3, -7, 11, 2**40], dtype=np.int64)
    assert rns.exact_entry(np.ones(4, np.int64), col) == 3 - 7 + 11 + 2**40
    big = np.full(8, (1 << 62), dtype=np.int64)
    assert rns.exact_entry(big, big) == 8 * (1 << 124)
    assert rns.exact_entry(np.array([-(1 << 63)], np.int64), np.array([-1], np.int64)) == 1 << 63


@pytest.mark.parametrize("use_native", [False, True])
def test_modmatmul_planes_prime_per_plane(use_native):
    ps = op.largest_primes_below(P26, 5)
    rng = np.random.default_rng(24)
    L, m, k, n = 5, 3, 4, 2
    a = np.stack([rng.integers(0, p, size=(m, k)) for p in ps]).astype(np.uint32)
    b = np.stack([rng.integers(0, p, size=(k, n)) for p in ps]).astype(np.uint32)
    got = rns.modmatmul_planes(a, b, ps, use_native=use_native)
    assert got.shape == (L, m, n) and got.dtype == np.uint32
    for j, p in enumerate(ps):
        assert np.array_equal(got[j], _brute(a[j], b[j], p)), j
    # plane j must be reduced by prime j: 2^25 * 2^25 = 2^50 differs per prime
    one = np.full((L, 1, 1), 1 << 25, dtype=np.uint32)
    got = rns.modmatmul_planes(one, one, ps, use_native=use_native)
    assert [int(v) for v in got[:, 0, 0]] == [(1 << 50) % p for p in ps]
    assert len(set(int(v) for v in got[:, 0, 0])) == L
    # no primes: an empty stack of the right shape
    assert rns.modmatmul_planes(a[:0], b[:0], [], use_native=use_native).shape == (0, m, n)
