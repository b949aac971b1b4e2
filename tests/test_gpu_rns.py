"""GPU parity of the RNS primitives against the CPU oracle (bit-exact).

Every case prints its name before touching the GPU.  Inputs come from synth
(seeded), expected values from oracle/ only.
"""
import sys

import numpy as np
import pytest

from oracle import native, primes as op, rns as orns
import synth

pytestmark = pytest.mark.gpu

P26 = 1 << 26


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def rg():
    import paper_2605_19254_amd as rg
    return rg


@pytest.fixture(scope="module")
def ctx(rg, torch_dev):
    c = rg.Context(device=0, L=26)
    yield c
    c.close()


PRIMES = op.largest_primes_below(P26, 26)


def _res(rng, ps, rows, cols, edge=False):
    out = np.empty((len(ps), rows, cols), dtype=np.int64)
    for j, p in enumerate(ps):
        out[j] = rng.integers(0, p, size=(rows, cols))
        if edge:
            special = np.array([0, 1, p - 1, (p - 1) // 2, (p + 1) // 2, 2, p - 2], dtype=np.int64)
            mask = rng.random((rows, cols)) < 0.3
            out[j][mask] = rng.choice(special, size=int(mask.sum()))
    return out.astype(np.int32)


def _modmatmul(ctx, rg, probs, path):
    """modmatmul_batched on a path, or a plan with a forced INT8 kernel
    variant for paths named int8-v<variant>."""
    if path.startswith("int8-v"):
        plan = rg.GemmPlan(ctx, probs, path="int8")
        plan.set_variant(int(path[len("int8-v"):]))
        plan.execute()
        plan.close()
    else:
        rg.modmatmul_batched(ctx, probs, path=path)


# ------------------------------------------------------------------ reduce --

@pytest.mark.parametrize("rows,cols,begin,L", [(1, 1, 0, 1), (3, 300, 0, 24), (257, 129, 2, 24),
                                               (64, 64, 0, 26)])
def test_reduce_matches_oracle(ctx, rg, torch_dev, rows, cols, begin, L):
    torch, dev = torch_dev
    _say("reduce", rows, cols, begin, L)
    rng = np.random.default_rng(rows * 1000 + cols)
    x = rng.integers(-(1 << 63), (1 << 63) - 1, size=(rows, cols), dtype=np.int64)
    flat = x.reshape(-1)
    ext = [0, 1, -1, -(1 << 63), (1 << 63) - 1, PRIMES[0], -PRIMES[0], 1 << 42, -(1 << 42), (1 << 21) - 1]
    flat[:min(len(ext), flat.size)] = ext[:flat.size]
    got = rg.rns_reduce(ctx, torch.from_numpy(x).to(dev), prime_begin=begin, L=L).cpu().numpy()
    want = orns.reduce(x, PRIMES[begin:begin + L]).astype(np.int32)
    assert np.array_equal(got, want)


def test_reduce_strided_and_empty(ctx, rg, torch_dev):
    torch, dev = torch_dev
    _say("reduce strided")
    rng = np.random.default_rng(7)
    big = rng.integers(-(1 << 40), 1 << 40, size=(50, 80), dtype=np.int64)
    xt = torch.from_numpy(big).to(dev)[5:45, 10:70]     # row stride 80
    out = torch.full((4, 40, 64), -1, dtype=torch.int32, device=dev)[:, :, :60]
    rg.rns_reduce(ctx, xt, prime_begin=0, L=4, out=out)
    want = orns.reduce(big[5:45, 10:70], PRIMES[:4]).astype(np.int32)
    assert np.array_equal(out.cpu().numpy(), want)
    e = torch.empty((0, 5), dtype=torch.int64, device=dev)
    assert rg.rns_reduce(ctx, e, L=3).shape == (3, 0, 5)


@pytest.mark.parametrize("W", [1, 2, 5, 10, 32])
def test_reduce_multiword(ctx, rg, torch_dev, W):
    """rns_reduce_mw against the oracle's residues of the Python integers
    (random words plus the extremes of the W-word range), a strided view,
    and the round trip through crt_reconstruct where the 26 primes cover the
    W-word range (W <= 10); W = 1 agrees with rns_reduce."""
    torch, dev = torch_dev
    _say("reduce multiword", W)
    rng = np.random.default_rng(100 + W)
    rows, cols, extra = 19, 70, 3
    words = rng.integers(0, 1 << 64, size=(rows, cols + extra, W), dtype=np.uint64)
    lim = 1 << (64 * W - 1)
    special = [v for v in (-lim, lim - 1, 0, -1, 1, -(lim // 2), (1 << 64) - 1, -(1 << 64)) if -lim <= v < lim]
    for idx, v in enumerate(special):
        words[idx % rows, idx, :] = np.array(orns.to_words(v, W), dtype=np.uint64)
    words[rows - 1, cols - 1, :] = np.array(orns.to_words(-lim, W), dtype=np.uint64)   # last entry of the view
    x = torch.from_numpy(words.view(np.int64)).to(dev)[:, :cols, :]
    res = rg.rns_reduce_mw(ctx, x, L=26)
    torch.cuda.synchronize()
    got = res.cpu().numpy()
    ints = [[orns.from_words([int(w) for w in words[i, c]]) for c in range(cols)] for i in range(rows)]
    for j, p in enumerate(PRIMES):
        want = np.array([[v % p for v in row] for row in ints], dtype=np.int64)
        assert np.array_equal(got[j].astype(np.int64), want), j
    if W <= 10:
        back = rg.crt_reconstruct(ctx, res, L=26, W=W)
        assert np.array_equal(back.cpu().numpy().reshape(rows, cols, W).view(np.uint64), words[:, :cols, :])
    if W == 1:
        x1 = x[:, :, 0]
        assert torch.equal(rg.rns_reduce(ctx, x1, L=26), res)
    assert ctx.status() == 0


def test_reduce_multiword_errors(ctx, rg, torch_dev):
    import ctypes
    from paper_2605_19254_amd import binding
    torch, dev = torch_dev
    _say("reduce multiword errors")
    x = torch.zeros((2, 3, 33), dtype=torch.int64, device=dev)
    out = torch.empty((1, 2, 3), dtype=torch.int32, device=dev)
    for W in (0, 33):
        assert binding._lib_reduce_mw(ctx.handle, x.data_ptr(), W, 2, 3, 3, 0, 1, out.data_ptr(), 3, 6,
                                      None) == binding.EINVAL
    assert binding._lib_reduce_mw(ctx.handle, x.data_ptr(), 2, 2, 3, 3, 25, 2, out.data_ptr(), 3, 6,
                                  None) == binding.EINVAL          # primes past the basis
    assert binding._lib_reduce_mw(ctx.handle, x.data_ptr(), 2, 0, 3, 3, 0, 1, out.data_ptr(), 3, 6,
                                  None) == binding.OK              # empty is a no-op


# --------------------------------------------------------------- modmatmul --

SHAPES = [(1, 1, 1), (1, 5, 1), (16, 16, 64), (17, 33, 70), (64, 128, 64), (65, 129, 65),
          (100, 200, 300), (130, 257, 129), (7, 300, 1000), (300, 7, 2100)]


@pytest.mark.parametrize("path", ["int8", "fp64"])
@pytest.mark.parametrize("m,n,k", SHAPES)
def test_modmatmul_matches_oracle(ctx, rg, torch_dev, path, m, n, k):
    torch, dev = torch_dev
    _say("modmatmul", path, m, n, k)
    rng = np.random.default_rng(m * 7 + n * 13 + k)
    begin, L = (0, 3) if m * n * k > 1e6 else (20, 6)
    ps = PRIMES[begin:begin + L]
    a = _res(rng, ps, m, k, edge=True)
    b = _res(rng, ps, k, n, edge=True)
    c = torch.full((L, m, n), -1, dtype=torch.int32, device=dev)
    _modmatmul(ctx, rg, [rg.GemmProblem(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), c, begin)], path)
    got = c.cpu().numpy()
    for j, p in enumerate(ps):
        want = native.modmatmul(a[j].astype(np.uint32), b[j].astype(np.uint32), p).astype(np.int32)
        assert np.array_equal(got[j], want), (path, j)


@pytest.mark.parametrize("path", ["int8", "fp64"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (65, 129, 130), (130, 300, 128), (40, 70, 0)])
def test_modmatmul_subtract(ctx, rg, torch_dev, path, m, n, k):
    """C := C - A B mod p (RNS_GEMM_SUBTRACT) against the oracle's product."""
    torch, dev = torch_dev
    _say("modmatmul subtract", path, m, n, k)
    rng = np.random.default_rng(m + 3 * n + 5 * k)
    begin, L = 4, 5
    ps = PRIMES[begin:begin + L]
    a = _res(rng, ps, m, k, edge=True)
    b = _res(rng, ps, k, n, edge=True)
    c0 = _res(rng, ps, m, n, edge=True)
    c = torch.from_numpy(c0.copy()).to(dev)
    ta = torch.from_numpy(a).to(dev) if k else torch.empty((L, m, 0), dtype=torch.int32, device=dev)
    tb = torch.from_numpy(b).to(dev) if k else torch.empty((L, 0, n), dtype=torch.int32, device=dev)
    _modmatmul(ctx, rg, [rg.GemmProblem(ta, tb, c, begin, subtract=True)], path)
    got = c.cpu().numpy()
    for j, p in enumerate(ps):
        prod = native.modmatmul(a[j].astype(np.uint32), b[j].astype(np.uint32), p).astype(np.int64) if k else 0
        want = ((c0[j].astype(np.int64) - prod) % p).astype(np.int32)
        assert np.array_equal(got[j], want), (path, j)


@pytest.mark.parametrize("path", ["int8", "fp64"])
def test_modmatmul_worst_case_values(ctx, rg, torch_dev, path):
    """All residues at the balanced extremes: every digit product and every
    8-term block sits at its bound."""
    torch, dev = torch_dev
    _say("modmatmul worst", path)
    ps = PRIMES[:2] + PRIMES[23:24]
    L, m, n, k = 3, 64, 128, 4096 + 64
    a = np.empty((L, m, k), dtype=np.int32)
    b = np.empty((L, k, n), dtype=np.int32)
    rng = np.random.default_rng(3)
    for j, p in enumerate(ps):
        h = (p - 1) // 2
        a[j] = rng.choice(np.array([h, h + 1, p - 1, 1], dtype=np.int64), size=(m, k))
        b[j] = rng.choice(np.array([h, h + 1], dtype=np.int64), size=(k, n))
    c = torch.empty((L, m, n), dtype=torch.int32, device=dev)
    pb = [0, 1, 23]
    for j in range(L):
        _modmatmul(ctx, rg, [rg.GemmProblem(torch.from_numpy(a[j:j + 1]).to(dev),
                                            torch.from_numpy(b[j:j + 1]).to(dev),
                                            c[j:j + 1], pb[j])], path)
    got = c.cpu().numpy()
    for j, p in enumerate(ps):
        want = native.modmatmul(a[j].astype(np.uint32), b[j].astype(np.uint32), p).astype(np.int32)
        assert np.array_equal(got[j], want)


def _digit_extremes(p):
    """Residues mod p whose balanced base-256 digits sit at their bounds, and
    the residue whose three low digits are all -128 (top digit as large as the
    balanced range allows)."""
    vals = []
    for d in (-128, 127):
        v = d * (1 + 256 + 256 * 256)
        top = ((p - 1) // 2 - abs(v)) // 256 ** 3
        w = v + top * 256 ** 3 if v > 0 else v - top * 256 ** 3
        vals += [v, w]
    low = (-128 * (1 + 256 + 256 * 256)) % p
    return np.array(sorted({v % p for v in vals}), dtype=np.int64), low


@pytest.mark.parametrize("variant", [None, 0, 3])
def test_modmatmul_digit_extremes_at_max_k(ctx, rg, torch_dev, variant):
    """k at the INT8 path's exactness bound, 90% of the entries the residue
    whose low digits are all -128 (every product term of shift group 2 then
    has the same sign): that group's int32 sum reaches 43690 * 3 * 2^14,
    within 2^15 of 2^31; the other entries are drawn from the other extremal
    residues."""
    torch, dev = torch_dev
    path = "int8" if variant is None else "int8-v%d" % variant
    _say("modmatmul digit extremes, k = max", path)
    k = 43690
    m, n = 40, 70
    begin = 9
    p = PRIMES[begin]
    ext, low = _digit_extremes(p)
    rng = np.random.default_rng(17)
    a = np.where(rng.random((1, m, k)) < 0.9, low, rng.choice(ext, size=(1, m, k))).astype(np.int32)
    b = np.where(rng.random((1, k, n)) < 0.9, low, rng.choice(ext, size=(1, k, n))).astype(np.int32)
    c = torch.empty((1, m, n), dtype=torch.int32, device=dev)
    _modmatmul(ctx, rg, [rg.GemmProblem(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), c, begin)], path)
    want = native.modmatmul(a[0].astype(np.uint32), b[0].astype(np.uint32), p).astype(np.int32)
    assert np.array_equal(c.cpu().numpy()[0], want)


def test_context_path_flag(rg, torch_dev):
    """rns_ctx_create flags: RNS_CTX_PATH_FP64 / _INT8 fix what the auto path
    resolves to (also with RNS_CTX_SEPARATE_CRT beside them); both path bits
    together and other flag bits are rejected."""
    import ctypes
    from paper_2605_19254_amd import binding
    torch, dev = torch_dev
    _say("context path flag")
    rng = np.random.default_rng(77)
    ps = PRIMES[:3]
    a = _res(rng, ps, 70, 90, edge=True)
    b = _res(rng, ps, 90, 50, edge=True)
    for path in ("fp64", "int8"):
        with rg.Context(device=0, L=3, path=path) as c:
            out = torch.empty((3, 70, 50), dtype=torch.int32, device=dev)
            prob = rg.GemmProblem(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), out)
            plan = rg.GemmPlan(c, [prob], path="auto")
            assert plan.info()["path"] == path
            plan.execute()
            plan.close()
            got = out.cpu().numpy()
            for j, p in enumerate(ps):
                want = native.modmatmul(a[j].astype(np.uint32), b[j].astype(np.uint32), p).astype(np.int32)
                assert np.array_equal(got[j], want)
    h = ctypes.c_void_p()
    for flags in (3, 7, 8, 1 << 40):
        assert binding._lib_ctx_create(ctypes.byref(h), 0, None, 3, flags) == binding.EINVAL
    for flags in (4, 5, 6):
        assert binding._lib_ctx_create(ctypes.byref(h), 0, None, 3, flags) == binding.OK
        binding._lib_ctx_destroy(h)


def test_modmatmul_batch_equals_single_and_paths_agree(ctx, rg, torch_dev):
    torch, dev = torch_dev
    _say("modmatmul batch")
    rng = np.random.default_rng(11)
    probs, cs_batch = [], []
    specs = [(33, 17, 65, 0, 2), (128, 64, 64, 3, 1), (1, 200, 7, 5, 3), (90, 90, 90, 24, 2)]
    tensors = []
    for (m, n, k, begin, L) in specs:
        ps = PRIMES[begin:begin + L]
        a = torch.from_numpy(_res(rng, ps, m, k)).to(dev)
        b = torch.from_numpy(_res(rng, ps, k, n)).to(dev)
        tensors.append((a, b, begin, L, m, n))
    for path in ("int8", "fp64"):
        batch = [torch.empty((L, m, n), dtype=torch.int32, device=dev) for (_, _, _, L, m, n) in tensors]
        rg.modmatmul_batched(ctx, [rg.GemmProblem(a, b, c, bg) for (a, b, bg, _, _, _), c in zip(tensors, batch)],
                             path=path)
        for (a, b, bg, L, m, n), cb in zip(tensors, batch):
            single = torch.empty((L, m, n), dtype=torch.int32, device=dev)
            rg.modmatmul_batched(ctx, [rg.GemmProblem(a, b, single, bg)], path=path)
            assert torch.equal(single, cb)
        cs_batch.append([c.cpu() for c in batch])
    for x, y in zip(cs_batch[0], cs_batch[1]):
        assert torch.equal(x, y)
    rg.modmatmul_batched(ctx, [], path="int8")   # count 0 is a no-op


def test_modmatmul_k_zero_and_bound(ctx, rg, torch_dev):
    torch, dev = torch_dev
    _say("modmatmul k=0 / bound")
    a = torch.empty((2, 5, 0), dtype=torch.int32, device=dev)
    b = torch.empty((2, 0, 7), dtype=torch.int32, device=dev)
    c = torch.full((2, 5, 7), 9, dtype=torch.int32, device=dev)
    rg.modmatmul_batched(ctx, [rg.GemmProblem(a, b, c)], path="int8")
    assert int(c.abs().sum()) == 0
    big_a = torch.zeros((1, 1, 43691), dtype=torch.int32, device=dev)
    big_b = torch.zeros((1, 43691, 1), dtype=torch.int32, device=dev)
    c1 = torch.empty((1, 1, 1), dtype=torch.int32, device=dev)
    with pytest.raises(rg.RnsError) as e:
        rg.modmatmul_batched(ctx, [rg.GemmProblem(big_a, big_b, c1)], path="int8")
    assert e.value.status == 4
    rg.modmatmul_batched(ctx, [rg.GemmProblem(big_a, big_b, c1)], path="fp64")
    assert int(c1.item()) == 0


# --------------------------------------------------------------------- CRT --

@pytest.mark.parametrize("L,W", [(1, 1), (2, 1), (3, 2), (24, 10), (24, 3), (26, 11), (5, 32)])
def test_crt_garner_matches_oracle(ctx, rg, torch_dev, L, W):
    torch, dev = torch_dev
    _say("crt garner", L, W)
    ps = PRIMES[:L]
    rng = np.random.default_rng(L * 100 + W)
    rows, cols = 9, 150
    res = _res(rng, ps, rows, cols, edge=True)
    basis = orns.CRTBasis(ps)
    h = (basis.M - 1) // 2
    # plant the extremes and values near the sign boundary
    special = [0, 1, -1, h, -h, h - 1, -h + 1, (1 << 63) - 1, -(1 << 63), 1 << 63, -(1 << 63) - 1]
    for e, x in enumerate(special):
        if abs(x) <= h:
            res[:, 0, e] = np.array(orns.reduce_int(x, ps), dtype=np.int64).astype(np.int32)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    out = rg.crt_reconstruct(ctx, torch.from_numpy(res).to(dev), L=L, W=W, status=status)
    got = out.cpu().numpy()
    got = got.reshape(rows, cols, W)
    want_overflow = False
    for i in range(rows):
        for c in range(cols):
            x = basis.reconstruct(res[:, i, c].astype(np.int64))
            try:
                words = orns.to_words(x, W)
            except orns.Overflow:
                want_overflow = True
                words = [(x % (1 << (64 * W))) >> (64 * w) & 0xFFFFFFFFFFFFFFFF for w in range(W)]
            assert [int(v) & 0xFFFFFFFFFFFFFFFF for v in got[i, c]] == words, (i, c, x)
    assert bool(status.item()) == want_overflow


def test_crt_lagrange_with_bound(ctx, rg, torch_dev):
    torch, dev = torch_dev
    _say("crt lagrange")
    rng = np.random.default_rng(21)
    for L, W, bits in [(24, 1, 52), (3, 1, 62), (24, 2, 100), (10, 4, 200)]:
        ps = PRIMES[:L]
        vals = [int(v) for v in rng.integers(-(1 << 62), 1 << 62, size=200)]
        vals = [(v << (bits - 62)) if bits > 62 else (v >> (62 - bits)) for v in vals]
        vals[:4] = [0, -1, (1 << bits) - 1, -((1 << bits) - 1)]
        res = np.ascontiguousarray(np.array([orns.reduce_int(v, ps) for v in vals], dtype=np.int64).T.reshape(L, 1, -1))
        out = rg.crt_reconstruct(ctx, torch.from_numpy(res.astype(np.int32)).to(dev), L=L, W=W,
                                 bound=(1 << bits) - 1)
        got = out.cpu().numpy().reshape(1, -1, W)
        for e, v in enumerate(vals):
            assert [int(x) & 0xFFFFFFFFFFFFFFFF for x in got[0, e]] == orns.to_words(v, W), (L, W, e)


def test_crt_overflow_reported_via_context(ctx, rg, torch_dev):
    torch, dev = torch_dev
    _say("crt overflow ctx")
    ps = PRIMES[:4]
    x = 1 << 70
    res = np.array(orns.reduce_int(x, ps), dtype=np.int64).reshape(4, 1, 1).astype(np.int32)
    assert ctx.status() == 0
    rg.crt_reconstruct(ctx, torch.from_numpy(res).to(dev), L=4, W=1)
    assert ctx.status() == 5
    assert ctx.status() == 0


# --------------------------------------------------------- whole products --

@pytest.mark.parametrize("path", ["int8", "fp64"])
def test_exact_product_small(ctx, rg, torch_dev, path):
    torch, dev = torch_dev
    _say("exact product small", path)
    a, b = synth.square_pair(n=300, bound=1 << 20, seed_a=0, seed_b=1)
    a, b = a[:211, :300].copy(), b[:300, :173].copy()
    ra = rg.rns_reduce(ctx, torch.from_numpy(a).to(dev), L=24)
    rb = rg.rns_reduce(ctx, torch.from_numpy(b).to(dev), L=24)
    rc = torch.empty((24, 211, 173), dtype=torch.int32, device=dev)
    rg.modmatmul_batched(ctx, [rg.GemmProblem(ra, rb, rc)], path=path)
    got = rg.crt_reconstruct(ctx, rc, L=24, W=1, bound=300 << 40).cpu().numpy()
    assert np.array_equal(got, orns.exact_matmul(a, b))
    got2 = rg.crt_reconstruct(ctx, rc, L=24, W=1).cpu().numpy()     # exact form, no bound
    assert np.array_equal(got2, got)
    assert ctx.status() == 0


@pytest.fixture(scope="module")
def n4096_product():
    """The n = 4096 operands of the single-product workload and their exact
    product C = A B from the oracle's plain C loop (every entry)."""
    a, b = synth.square_pair(n=4096, bound=1 << 20, seed_a=0, seed_b=1)
    return a, b, native.exact_matmul(a, b)


@pytest.mark.parametrize("path", ["int8", "fp64", "int8-v0", "int8-v2", "int8-v3"])
def test_exact_product_n4096_full(ctx, rg, torch_dev, n4096_product, path):
    """The full n = 4096, 24-prime product in the benchmark's configuration
    through the boundary calls: every entry of C and every residue of every
    prime plane against the oracle."""
    torch, dev = torch_dev
    _say("exact product n=4096 (all entries)", path)
    n, L = 4096, 24
    a, b, want = n4096_product
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    ra = rg.rns_reduce(ctx, ta, L=L)
    rb = rg.rns_reduce(ctx, tb, L=L)
    rc = torch.empty((L, n, n), dtype=torch.int32, device=dev)
    _modmatmul(ctx, rg, [rg.GemmProblem(ra, rb, rc)], path)
    out = rg.crt_reconstruct(ctx, rc, L=L, W=1, bound=n << 40)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    for j, p in enumerate(PRIMES[:L]):
        assert np.array_equal(rc[j].cpu().numpy(), np.mod(want, p).astype(np.int32)), j
    assert ctx.status() == 0


@pytest.mark.parametrize("path", ["int8", "fp64"])
def test_matmul_plan_n4096_full(ctx, rg, torch_dev, n4096_product, path):
    """The benchmark's step: one whole-product plan over the n = 4096, 24-prime
    product (int64 A and B straight into the tiled operands, GEMM, Lagrange
    CRT), executed twice; every entry against the oracle both times."""
    torch, dev = torch_dev
    _say("whole-product plan n=4096 (all entries)", path)
    n, L = 4096, 24
    a, b, want = n4096_product
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    out = torch.empty((n, n), dtype=torch.int64, device=dev)
    plan = rg.MatmulPlan(ctx, [rg.MatmulProblem(ta, tb, out, prime_begin=0, L=L, bound=n << 40)], path=path)
    plan.execute()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    out.fill_(0)
    plan.execute()                      # a second execution on the resident workspace
    torch.cuda.synchronize()
    assert ctx.status() == 0
    assert np.array_equal(out.cpu().numpy(), want)
    plan.close()


def test_full_range_residues_n4096_stripe(ctx, rg, torch_dev):
    """The stress form of the n = 4096 product: every residue plane uniform in
    [0, p_j) (seeded on the device as in the benchmark), INT8 products of all
    24 primes and the exact mixed-radix CRT into 10 words.  Every residue and
    every CRT output of a 256-row stripe against the oracle (schoolbook
    modmatmul per prime, Lagrange CRT in Python integers)."""
    torch, dev = torch_dev
    _say("full-range residues n=4096 W=10, 256-row stripe")
    n, L, W, rows = 4096, 24, 10, 256
    ps = PRIMES[:L]
    g = torch.Generator(device=dev)
    ra = torch.empty((L, n, n), dtype=torch.int32, device=dev)
    rb = torch.empty_like(ra)
    for j, p in enumerate(ps):
        g.manual_seed(1000 + j)
        ra[j].random_(0, p, generator=g)
        g.manual_seed(2000 + j)
        rb[j].random_(0, p, generator=g)
    rc = torch.empty_like(ra)
    out = torch.empty((n, n, W), dtype=torch.int64, device=dev)
    rg.modmatmul_batched(ctx, [rg.GemmProblem(ra, rb, rc)], path="int8")
    rg.crt_reconstruct(ctx, rc, L=L, W=W, out=out)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    r0 = n // 2 - rows // 2                              # a stripe in the middle of C
    a_s = ra[:, r0:r0 + rows, :].cpu().numpy().astype(np.uint32)
    b_all = rb.cpu().numpy().astype(np.uint32)
    want_res = np.stack([native.modmatmul(a_s[j], b_all[j], p) for j, p in enumerate(ps)])
    got_res = rc[:, r0:r0 + rows, :].cpu().numpy().astype(np.uint32)
    assert np.array_equal(got_res, want_res)
    _say("  residues of the stripe agree; CRT of", rows * n, "entries")
    want = orns.crt_planes(want_res, ps)
    got = rg.words_to_ints(out[r0:r0 + rows].cpu().numpy())
    assert np.array_equal(got, want)
