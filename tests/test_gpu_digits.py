"""The matrix-core conversions (digits_gemm.hip) against the oracle, bit-exact:
the exact CRT (crt_reconstruct without a bound), the multiword reduction
(rns_reduce_mw) and the RNS base conversion (rns_base_convert), over prime
counts that select every kernel shape (1 to 64 source primes), ragged
shapes, and the values where the floating-point correction is ambiguous
(|x| next to (M-1)/2, where the sum of y_j / p_j is next to a half-integer).

Expected values: oracle.rns (Lagrange CRT over Python integers, floor-mod
reduction)."""
import sys

import numpy as np
import pytest

from oracle import primes as op, rns as orns

pytestmark = pytest.mark.gpu

NP = 140
PRIMES = op.largest_primes_below(1 << 26, NP)


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_19254_amd as rg
    ctx = rg.Context(device=0, L=NP)
    yield torch, torch.device("cuda:0"), rg, ctx
    ctx.close()


def _residues_of(vals, ps, rows, cols):
    """int32 planes [L, rows, cols] of the Python integers vals (row-major)."""
    out = np.empty((len(ps), rows * cols), dtype=np.int64)
    for e, v in enumerate(vals):
        out[:, e] = orns.reduce_int(v, ps)
    return out.reshape(len(ps), rows, cols).astype(np.int32)


def _values(rng, M, n, with_edges=True):
    """n symmetric-range integers: uniform over the whole range, plus the
    edges: 0, +-1, +-(M-1)/2 and its neighbours, +-M/2 (1 - 2^-45) (a sum of
    y_j / p_j within 2^-40 of a half-integer)."""
    h = (M - 1) // 2
    vals = [int.from_bytes(rng.bytes((M.bit_length() + 7) // 8 + 1), "little") % M - h for _ in range(n)]
    if with_edges:
        edges = [0, 1, -1, h, -h, h - 1, -h + 1, h - 12345, -h + 777, M // 2 - (M >> 45), -(M // 2) + (M >> 45),
                 M // 2 - (M >> 41), (1 << 63) - 1, -(1 << 63)]
        for i, v in enumerate(edges):
            if abs(v) <= h:
                vals[(7 * i) % n] = v
    return vals


@pytest.mark.parametrize("L", [1, 2, 7, 16, 17, 20, 24, 32, 33, 40, 48, 49, 64])
def test_crt_exact_matrix_cores(env, L):
    torch, dev, rg, ctx = env
    rng = np.random.default_rng(L)
    begin = (3 * L) % (NP - L)
    ps = PRIMES[begin:begin + L]
    M = orns.CRTBasis(ps).M
    rows, cols = 5, 131
    vals = _values(rng, M, rows * cols)
    res = torch.from_numpy(_residues_of(vals, ps, rows, cols)).to(dev)
    for W in (1, 2, (M.bit_length() + 64) // 64, 32):
        _say("crt matrix cores", L, W)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
        out = rg.crt_reconstruct(ctx, res, prime_begin=begin, L=L, W=W, status=status)
        got = out.cpu().numpy().reshape(rows * cols, W)
        over = False
        for e, v in enumerate(vals):
            try:
                want = orns.to_words(v, W)
            except orns.Overflow:
                over = True
                want = [(v % (1 << (64 * W))) >> (64 * w) & 0xFFFFFFFFFFFFFFFF for w in range(W)]
            assert [int(x) & 0xFFFFFFFFFFFFFFFF for x in got[e]] == want, (L, W, e, v)
        assert bool(status.item()) == over, (L, W)


@pytest.mark.parametrize("W", [1, 2, 3, 7, 8, 9, 10, 20, 31, 32])
def test_reduce_multiword_matrix_cores(env, W):
    """Every prime count up to 140 in groups of 32 (the launch's grid.y)."""
    torch, dev, rg, ctx = env
    _say("reduce multiword matrix cores", W)
    rng = np.random.default_rng(200 + W)
    rows, cols = 7, 67
    lim = 1 << (64 * W - 1)
    vals = [int.from_bytes(rng.bytes(8 * W), "little") - lim for _ in range(rows * cols)]
    for i, v in enumerate([-lim, lim - 1, 0, -1, 1, lim // 3, -(lim // 5), (1 << 64) - 1, -(1 << 64)]):
        if -lim <= v < lim:
            vals[5 * i] = v
    words = np.array([orns.to_words(v, W) for v in vals], dtype=np.uint64).reshape(rows, cols, W)
    x = torch.from_numpy(words.view(np.int64)).to(dev)
    for begin, L in ((0, NP), (11, 33), (100, 1)):
        res = rg.rns_reduce_mw(ctx, x, prime_begin=begin, L=L)
        torch.cuda.synchronize()
        got = res.cpu().numpy().astype(np.int64).reshape(L, -1)
        for j, p in enumerate(PRIMES[begin:begin + L]):
            assert np.array_equal(got[j], np.array([v % p for v in vals], dtype=np.int64)), (W, begin, j)


@pytest.mark.parametrize("L1,b1,L2,b2", [(24, 0, 24, 24), (8, 5, 40, 60), (64, 40, 3, 1), (33, 100, 17, 7),
                                         (16, 30, 20, 20), (1, 2, 5, 9)])
def test_base_convert(env, L1, b1, L2, b2):
    """Residues in one primes range -> residues of the same symmetric integer
    in another (overlapping ranges included): with a bound (the one-pass
    Lagrange form with the floating-point correction) and without (exact CRT,
    then the multiword reduction)."""
    torch, dev, rg, ctx = env
    rng = np.random.default_rng(L1 * 1000 + L2)
    ps, qs = PRIMES[b1:b1 + L1], PRIMES[b2:b2 + L2]
    M = orns.CRTBasis(ps).M
    rows, cols = 3, 129
    # with a bound: |x| <= B, B = M/2 (1 - 2^-38)
    B = (M // 2) - (M >> 38)
    vals = [int(v) for v in rng.integers(-(1 << 62), 1 << 62, size=rows * cols)]
    vals = [v * (B >> 62) // 1 if B >> 62 else v % (B + 1) * (1 if v >= 0 else -1) for v in vals]
    vals[:4] = [0, -1, B, -B]
    res = torch.from_numpy(_residues_of(vals, ps, rows, cols)).to(dev)
    _say("base convert with bound", L1, L2)
    out = rg.base_convert(ctx, res, b1, b2, L2, L=L1, bound=B)
    got = out.cpu().numpy().astype(np.int64).reshape(L2, -1)
    for i, q in enumerate(qs):
        assert np.array_equal(got[i], np.array([v % q for v in vals], dtype=np.int64)), (i, q)
    # without: the whole symmetric range, its edges included
    vals = _values(rng, M, rows * cols)
    res = torch.from_numpy(_residues_of(vals, ps, rows, cols)).to(dev)
    _say("base convert exact", L1, L2)
    out = rg.base_convert(ctx, res, b1, b2, L2, L=L1)
    got = out.cpu().numpy().astype(np.int64).reshape(L2, -1)
    for i, q in enumerate(qs):
        assert np.array_equal(got[i], np.array([v % q for v in vals], dtype=np.int64)), (i, q)
    assert ctx.status() == 0


def test_crt_mixed_radix_form_still_exact(rg=None):
    """The mixed-radix (Garner) kernel, selected with RNS_CRT_GARNER=1 when a
    context is created, gives the same words as the matrix-core form."""
    import os
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_19254_amd as rg
    _say("crt garner vs matrix cores")
    dev = torch.device("cuda:0")
    ps = PRIMES[:24]
    M = orns.CRTBasis(ps).M
    rng = np.random.default_rng(5)
    vals = _values(rng, M, 4 * 200)
    res = torch.from_numpy(_residues_of(vals, ps, 4, 200)).to(dev)
    os.environ["RNS_CRT_GARNER"] = "1"
    try:
        cg = rg.Context(device=0, L=24)
    finally:
        del os.environ["RNS_CRT_GARNER"]
    cm = rg.Context(device=0, L=24)
    try:
        a = rg.crt_reconstruct(cg, res, L=24, W=10)
        b = rg.crt_reconstruct(cm, res, L=24, W=10)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert cg.status() == 0 and cm.status() == 0
    finally:
        cg.close()
        cm.close()


@pytest.mark.parametrize("L,W", [(2, 1), (24, 10), (24, 4), (40, 17), (64, 28)])
def test_crt_limb_form_matches_oracle(L, W):
    """The exact Lagrange form on 32-bit limbs (k_crt_exact, selected with
    RNS_CRT_FORM=limbs when a context is created) against the oracle's CRT:
    full-range values (both signs, the endpoints +-(M-1)/2, values beyond W
    words that must raise the status word) with ragged row lengths."""
    import os
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_19254_amd as rg
    _say("crt limb form", L, W)
    dev = torch.device("cuda:0")
    ps = PRIMES[:L]
    M = orns.CRTBasis(ps).M
    rng = np.random.default_rng(L * 100 + W)
    rows, cols = 3, 201
    vals = _values(rng, M, rows * cols)
    vals[0], vals[1], vals[2] = (M - 1) // 2, -((M - 1) // 2), 0
    res = torch.from_numpy(_residues_of(vals, ps, rows, cols)).to(dev)
    os.environ["RNS_CRT_FORM"] = "limbs"
    try:
        cl = rg.Context(device=0, L=L)
    finally:
        del os.environ["RNS_CRT_FORM"]
    try:
        got = rg.crt_reconstruct(cl, res, L=L, W=W)
        torch.cuda.synchronize()
        words = got.cpu().numpy().reshape(rows * cols, W)
        lim = 1 << (64 * W - 1)
        overflow = False
        for e, v in enumerate(vals):
            if -lim <= v < lim:
                want = [(v >> (64 * k)) & ((1 << 64) - 1) for k in range(W)]
                assert [int(x) for x in words[e].astype(np.uint64)] == want, e
            else:
                overflow = True
        assert (cl.status() != 0) == overflow
    finally:
        cl.close()
