"""The stored Smith forms (tests/golden/smith_lifting.json and
smith_vandermonde.json, written by the oracle's Smith form) checked by facts
that do not go through that code: the invariants form a divisor chain whose
first member is the gcd of A's entries, and their product is |det A|
(Definition 1's S has the same determinant as A up to sign), tested modulo
three primes near 2^31 with det A mod p from Gaussian elimination over GF(p)
on A rebuilt from its seeded generator.  A dropped, doubled or altered
invariant changes the product modulo all three primes (short of a multiple
of their product)."""
import json
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
PRIMES = (2147483647, 2147483629, 2147483587)          # the three largest below 2^31


def det_mod(a: np.ndarray, p: int) -> int:
    """det a mod p by elimination over GF(p); every product stays below 2^62."""
    m = np.mod(np.asarray(a, dtype=np.int64), p)
    n = m.shape[0]
    det = 1
    for k in range(n):
        nz = np.nonzero(m[k:, k])[0]
        if nz.size == 0:
            return 0
        r = k + int(nz[0])
        if r != k:
            m[[k, r]] = m[[r, k]]
            det = -det
        d = int(m[k, k])
        det = det * d % p
        f = m[k + 1:, k] * pow(d, p - 2, p) % p
        m[k + 1:, k:] = (m[k + 1:, k:] - np.outer(f, m[k, k:]) % p) % p
    return det % p


def _cases():
    out = []
    with open(os.path.join(HERE, "golden", "smith_lifting.json")) as f:
        for c in json.load(f)["cases"]:
            out.append(pytest.param("lifting", c, id="%s-%d" % (c["gen"], c["n"])))
    with open(os.path.join(HERE, "golden", "smith_vandermonde.json")) as f:
        for c in json.load(f)["cases"]:
            out.append(pytest.param("vandermonde", c, id="vandermonde-%d" % c["n"]))
    return out


def _matrix(kind, c):
    if kind == "vandermonde":
        return synth.vandermonde_mod(c["n"])
    if c["gen"] == "small_smith":
        return synth.small_smith(seed=c["seed"], attempt=c["attempt"], n=c["n"], bound=c["bound"])
    return synth.planted_small(c["n"], seed=c["seed"]).a


def test_det_mod_pins():
    """det_mod itself: the identity, a swap, a singular matrix and a 3 x 3
    determinant by hand."""
    p = PRIMES[0]
    assert det_mod(np.eye(5, dtype=np.int64), p) == 1
    assert det_mod(np.array([[0, 1], [1, 0]]), p) == p - 1
    assert det_mod(np.array([[1, 2], [2, 4]]), p) == 0
    assert det_mod(np.array([[2, -3, 1], [2, 0, -1], [1, 4, 5]]), p) == 49


@pytest.mark.parametrize("kind,c", _cases())
def test_stored_smith_form(kind, c):
    a = _matrix(kind, c)
    n = c["n"]
    tail = [int(v) for v in c["tail"]]
    assert a.shape == (n, n) and c["ones"] + len(tail) == n
    assert all(v > 1 for v in tail)
    assert all(tail[i + 1] % tail[i] == 0 for i in range(len(tail) - 1))
    s1 = 1 if c["ones"] else tail[0]
    assert math.gcd(*(int(v) for v in np.unique(np.abs(a)))) == s1
    prod = math.prod(tail)
    if "det_abs" in c:
        assert int(c["det_abs"]) == prod
    for p in PRIMES:
        d = det_mod(a, p)
        assert prod % p in (d, (p - d) % p), (kind, n, p)
