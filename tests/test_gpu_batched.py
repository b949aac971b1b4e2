"""GPU parity of the batched forms: plans over many uneven products, every
INT8 GEMM variant, whole-product plans with resident residue planes, HIP
graph capture and replay, and the autotuner's cache.

Expected values come from oracle/ only; inputs from synth."""
import os
import sys
import tempfile

import numpy as np
import pytest

from oracle import native, primes as op, rns as orns
import synth

pytestmark = pytest.mark.gpu

PRIMES = op.largest_primes_below(1 << 26, 26)


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


def _uneven_residue_batch(torch, dev, count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    sizes = synth.uneven_sizes(count, lo, hi, seed)
    probs, host = [], []
    for i, n in enumerate(sizes):
        m, k = max(1, n - 3 * (i % 3)), n + (i % 5)
        L = 1 + (i % 3)
        begin = (5 * i) % (26 - L)
        ps = PRIMES[begin:begin + L]
        a = np.stack([rng.integers(0, p, size=(m, k)) for p in ps]).astype(np.int32)
        b = np.stack([rng.integers(0, p, size=(k, n)) for p in ps]).astype(np.int32)
        c = torch.full((L, m, n), -1, dtype=torch.int32, device=dev)
        host.append((a, b, ps))
        probs.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), c, begin))
    return probs, host


def _check_residues(got, a, b, ps):
    for j, p in enumerate(ps):
        want = native.modmatmul(a[j].astype(np.uint32), b[j].astype(np.uint32), p).astype(np.int32)
        assert np.array_equal(got[j], want)


def test_gemm_plan_all_variants_uneven(ctx, rg, torch_dev):
    torch, dev = torch_dev
    _say("gemm plan variants")
    probs, host = _uneven_residue_batch(torch, dev, 24, 5, 300, seed=31)
    gps = [rg.GemmProblem(a, b, c, bg) for a, b, c, bg in probs]
    plan = rg.GemmPlan(ctx, gps, path="int8")
    outs = []
    for v in (0, 1, 2, 3, 4):
        for _, _, c, _ in probs:
            c.fill_(-1)
        plan.set_variant(v)
        plan.execute()
        plan.execute()          # a second run reuses the work counter
        torch.cuda.synchronize()
        outs.append([c.cpu().numpy() for _, _, c, _ in probs])
    for (a, b, ps), got in zip(host, outs[0]):
        _check_residues(got, a, b, ps)
    for v in (1, 2, 3, 4):
        for x, y in zip(outs[0], outs[v]):
            assert np.array_equal(x, y)
    info = plan.info()
    assert info["path"] == "int8" and info["tiles"] > 0
    plan.close()
    fplan = rg.GemmPlan(ctx, gps, path="fp64")
    for _, _, c, _ in probs:
        c.fill_(-1)
    fplan.execute()
    torch.cuda.synchronize()
    for (_, _, c, _), ref in zip(probs, outs[0]):
        assert np.array_equal(c.cpu().numpy(), ref)
    fplan.close()


def test_gemm_plan_empty_and_zero_sized(ctx, rg, torch_dev):
    torch, dev = torch_dev
    _say("gemm plan empty")
    plan = rg.GemmPlan(ctx, [], path="int8")
    plan.execute()
    a = torch.empty((1, 0, 4), dtype=torch.int32, device=dev)
    b = torch.empty((1, 4, 3), dtype=torch.int32, device=dev)
    c = torch.empty((1, 0, 3), dtype=torch.int32, device=dev)
    plan2 = rg.GemmPlan(ctx, [rg.GemmProblem(a, b, c)], path="int8")
    plan2.execute()
    torch.cuda.synchronize()


@pytest.mark.parametrize("with_bound", [True, False])
def test_matmul_plan_uneven_batch(ctx, rg, torch_dev, with_bound):
    torch, dev = torch_dev
    _say("matmul plan", with_bound)
    batch = synth.uneven_batch(count=20, lo=8, hi=200, bound=1 << 16, seed=41)
    probs = []
    for i, pr in enumerate(batch):
        A = torch.from_numpy(pr.a).to(dev)
        B = torch.from_numpy(pr.b).to(dev)
        C = torch.empty((pr.m, pr.n), dtype=torch.int64, device=dev)
        bound = pr.k << 32 if with_bound else 0
        probs.append(rg.MatmulProblem(A, B, C, prime_begin=i % 3, L=2, bound=bound))
    plan = rg.MatmulPlan(ctx, probs, path="int8", W=1)
    plan.execute()
    torch.cuda.synchronize()
    assert ctx.status() == 0
    for pr, p in zip(batch, probs):
        assert np.array_equal(p.C.cpu().numpy(), native.exact_matmul(pr.a, pr.b))
    # alone equals in the batch
    single = rg.MatmulProblem(probs[3].A, probs[3].B, torch.empty_like(probs[3].C), prime_begin=0, L=2,
                              bound=probs[3].bound)
    p1 = rg.MatmulPlan(ctx, [single], path="int8")
    p1.execute()
    torch.cuda.synchronize()
    assert torch.equal(single.C, probs[3].C)
    plan.close()
    p1.close()


def _symmetric_mod(x, M):
    """x mod M in the symmetric range [-(M-1)/2, (M-1)/2] (M odd), elementwise
    over an object array of Python ints."""
    h = (M - 1) // 2
    return np.vectorize(lambda v: (v + h) % M - h, otypes=[object])(x)


@pytest.mark.parametrize("seed", [0, 1])
def test_matmul_plan_fused_crt(ctx, rg, torch_dev, seed):
    """Whole-product plans with one or two primes per problem and one output
    word fuse the CRT into the GEMM launch (both primes of a tile in one
    work-group).  Entries across the whole int64 range, so that products
    exceed p0 p1 and the result is the symmetric residue mod p0 p1; ragged
    shapes over several tiles, k up to 700, prime pairs across the basis (and
    in reversed order of size), L = 1 beside L = 2: every entry against the
    exact product reduced in Python integers, and against the same plan with
    the CRT as its own launch."""
    torch, dev = torch_dev
    _say("fused CRT plan", seed)
    rng = np.random.default_rng(300 + seed)
    lim = np.iinfo(np.int64)
    shapes = [(1, 1, 1), (70, 130, 90), (129, 700, 65), (64, 64, 64), (200, 33, 250), (5, 300, 131)]
    problems, hosts = [], []
    for i, (m, k, n) in enumerate(shapes):
        L = 1 if i % 3 == 2 else 2
        begin = (7 * i + seed) % (26 - L)
        a = rng.integers(lim.min, lim.max, size=(m, k), dtype=np.int64, endpoint=True)
        b = rng.integers(lim.min, lim.max, size=(k, n), dtype=np.int64, endpoint=True)
        if i == 4:   # small entries: products inside the symmetric range
            a = rng.integers(-(1 << 16), 1 << 16, size=(m, k), dtype=np.int64, endpoint=True)
            b = rng.integers(-(1 << 16), 1 << 16, size=(k, n), dtype=np.int64, endpoint=True)
        M = 1
        for p in PRIMES[begin:begin + L]:
            M *= p
        hosts.append((a, b, M))
        problems.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), begin, L))
    exact = [a.astype(object).dot(b.astype(object)) for a, b, _ in hosts]
    # one basis with the primes in increasing order too, so that p0 < p1
    rev = rg.Context(device=0, primes=PRIMES[::-1][:4])
    sep = rg.Context(device=0, L=26, separate_crt=True)
    try:
        for c, reversed_basis in ((ctx, False), (rev, True), (sep, False)):
            probs = []
            for (A, B, begin, L) in problems:
                if reversed_basis:
                    begin = begin % (4 - L + 1)
                probs.append(rg.MatmulProblem(A, B, torch.full((A.shape[0], B.shape[1]), 77, dtype=torch.int64,
                                                               device=dev), prime_begin=begin, L=L))
            plan = rg.MatmulPlan(c, probs, path="int8")
            assert (plan.info()["variant"] == rg.binding.I8_HALF_CRT) == (c is not sep)
            plan.execute()
            torch.cuda.synchronize()
            assert c.status() == 0
            for j, ((a, b, M), p) in enumerate(zip(hosts, probs)):
                if reversed_basis:
                    M = 1
                    for q in c.primes[p.prime_begin:p.prime_begin + p.L]:
                        M *= q
                want = _symmetric_mod(exact[j], M)
                got = p.C.cpu().numpy().astype(object)
                assert np.array_equal(got, want), (j, shapes[j], reversed_basis)
            plan.close()
    finally:
        rev.close()
        sep.close()


def test_matmul_plan_two_primes_beyond_int8_bound(ctx, rg, torch_dev):
    """k = 43691 is beyond the INT8 path's exactness bound: a two-prime plan
    on the auto path takes the FP64 path with a CRT launch of its own (no
    fusion) and is still exact; on the INT8 path it is refused."""
    torch, dev = torch_dev
    _say("two-prime plan, k = 43691")
    rng = np.random.default_rng(17)
    m, k, n = 3, 43691, 5
    a = rng.integers(-(1 << 12), 1 << 12, size=(m, k), dtype=np.int64)
    b = rng.integers(-(1 << 12), 1 << 12, size=(k, n), dtype=np.int64)
    A, B = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    C = torch.zeros((m, n), dtype=torch.int64, device=dev)
    prob = rg.MatmulProblem(A, B, C, prime_begin=3, L=2)
    plan = rg.MatmulPlan(ctx, [prob], path="auto")
    info = plan.info()
    assert info["path"] == "fp64" and info["variant"] != rg.binding.I8_HALF_CRT
    plan.execute()
    torch.cuda.synchronize()
    assert ctx.status() == 0
    assert np.array_equal(C.cpu().numpy(), native.exact_matmul(a, b))
    plan.close()
    with pytest.raises(rg.binding.RnsError) as e:
        rg.MatmulPlan(ctx, [prob], path="int8")
    assert e.value.status == rg.binding.EBOUND


@pytest.mark.parametrize("path", ["int8", "fp64"])
def test_matmul_plan_full_range_int64(ctx, rg, torch_dev, path):
    """Whole-product plans convert int64 operands straight into the tiled
    layouts: entries across the whole int64 range (the extremes included),
    strided A and B, tiles cut by the matrix edges, exact CRT into 3 words;
    every entry against the oracle's Python-integer product."""
    torch, dev = torch_dev
    _say("matmul plan full-range int64", path)
    rng = np.random.default_rng(97)
    lim = np.iinfo(np.int64)
    special = np.array([lim.min, lim.max, 0, -1, 1, lim.min + 1, lim.max - 1, 1 << 42, -(1 << 42),
                        (1 << 21) - 1, -(1 << 21)], dtype=np.int64)
    probs, hosts = [], []
    for i, (m, k, n) in enumerate([(40, 70, 30), (17, 130, 65), (64, 64, 128), (1, 3, 1)]):
        a = rng.integers(lim.min, lim.max, size=(m, k), dtype=np.int64, endpoint=True)
        b = rng.integers(lim.min, lim.max, size=(k, n), dtype=np.int64, endpoint=True)
        ma = rng.random((m, k)) < 0.2
        a[ma] = rng.choice(special, size=int(ma.sum()))
        mb = rng.random((k, n)) < 0.2
        b[mb] = rng.choice(special, size=int(mb.sum()))
        Abig = torch.zeros((m, k + 3), dtype=torch.int64, device=dev)
        Bbig = torch.zeros((k, n + 5), dtype=torch.int64, device=dev)
        Abig[:, :k] = torch.from_numpy(a).to(dev)
        Bbig[:, :n] = torch.from_numpy(b).to(dev)
        C = torch.empty((m, n, 3), dtype=torch.int64, device=dev)
        # |C| <= k 2^126 < 2^134: 6 primes below 2^26 give 155 bits
        probs.append(rg.MatmulProblem(Abig[:, :k], Bbig[:, :n], C, prime_begin=2 * i, L=6))
        hosts.append((a, b))
    plan = rg.MatmulPlan(ctx, probs, path=path, W=3)
    plan.execute()
    torch.cuda.synchronize()
    assert ctx.status() == 0
    for (a, b), p in zip(hosts, probs):
        got = rg.words_to_ints(p.C.cpu().numpy())
        want = a.astype(object).dot(b.astype(object))
        assert np.array_equal(got, want)
    plan.close()


@pytest.mark.parametrize("path", ["int8", "fp64"])
@pytest.mark.parametrize("L", [4, 2])
def test_matmul_plan_degenerate_shapes(ctx, rg, torch_dev, path, L):
    """Whole-product plans with k = 0 (C = 0), empty problems (m = 0 or n = 0)
    and 1 x 1 products in one batch, beside an ordinary product; with two
    primes (the INT8 plan then fuses the CRT into the GEMM) the results are
    the symmetric residues mod p0 p1."""
    torch, dev = torch_dev
    _say("matmul plan degenerate shapes", path, L)
    rng = np.random.default_rng(7)
    shapes = [(5, 0, 7), (0, 4, 3), (6, 4, 0), (1, 1, 1), (33, 65, 17)]
    probs, hosts = [], []
    for m, k, n in shapes:
        a = rng.integers(-(1 << 25), 1 << 25, size=(m, k), dtype=np.int64)
        b = rng.integers(-(1 << 25), 1 << 25, size=(k, n), dtype=np.int64)
        A = torch.from_numpy(a).to(dev) if a.size else torch.zeros((m, k), dtype=torch.int64, device=dev)
        B = torch.from_numpy(b).to(dev) if b.size else torch.zeros((k, n), dtype=torch.int64, device=dev)
        C = torch.full((m, n), 123, dtype=torch.int64, device=dev)
        probs.append(rg.MatmulProblem(A, B, C, prime_begin=0, L=L, bound=max(k, 1) << 50 if L == 4 else 0))
        hosts.append((a, b))
    plan = rg.MatmulPlan(ctx, probs, path=path)
    assert (plan.info()["variant"] == rg.binding.I8_HALF_CRT) == (L == 2 and path == "int8")
    plan.execute()
    torch.cuda.synchronize()
    assert ctx.status() == 0
    M = PRIMES[0] * PRIMES[1]
    for (a, b), p in zip(hosts, probs):
        want = a.astype(object).dot(b.astype(object)) if a.shape[1] else np.zeros((a.shape[0], b.shape[1]), dtype=object)
        if L == 2 and want.size:
            want = _symmetric_mod(want, M)
        assert np.array_equal(p.C.cpu().numpy().astype(object), want)
    plan.close()


def test_matmul_plan_graph_replay(ctx, rg, torch_dev):
    """Capture the whole product (reduce, prep, GEMM, CRT) into a HIP graph and
    replay it several times with eager work in between; every replay must equal
    the eager result for the current inputs.  The plan that fuses the CRT into
    the GEMM, and the plan with a CRT launch of its own in three GEMM
    variants."""
    torch, dev = torch_dev
    _say("graph replay")
    batch = synth.uneven_batch(count=12, lo=16, hi=160, bound=1 << 16, seed=51)
    probs = []
    for pr in batch:
        probs.append(rg.MatmulProblem(torch.from_numpy(pr.a).to(dev), torch.from_numpy(pr.b).to(dev),
                                      torch.empty((pr.m, pr.n), dtype=torch.int64, device=dev),
                                      prime_begin=0, L=2, bound=pr.k << 32))
    want = [native.exact_matmul(pr.a, pr.b) for pr in batch]
    sep = rg.Context(device=0, L=4, separate_crt=True)
    for c, variant in ((ctx, None), (sep, 0), (sep, 2), (sep, 4)):
        plan = rg.MatmulPlan(c, probs, path="int8")
        if variant is None:
            assert plan.info()["variant"] == rg.binding.I8_HALF_CRT
        else:
            plan.set_variant(variant)
        plan.execute()                       # warm-up outside the capture
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.execute()
        torch.cuda.synchronize()
        sign = 1
        for rep in range(4):                 # 4 flips: inputs end as they began
            for p in probs:                  # eager work between replays
                p.A.mul_(-1)
                p.C.fill_(7)
            sign = -sign
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for w, p in zip(want, probs):
                assert np.array_equal(p.C.cpu().numpy(), sign * w), (variant, rep)
        del g
        plan.close()
    assert ctx.status() == 0 and sep.status() == 0
    sep.close()


def test_autotune_and_cache(ctx, rg, torch_dev):
    torch, dev = torch_dev
    _say("autotune")
    probs, host = _uneven_residue_batch(torch, dev, 6, 64, 400, seed=61)
    gps = [rg.GemmProblem(a, b, c, bg) for a, b, c, bg in probs]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        ctx.set_tune_cache(path)
        v = rg.autotune(ctx, gps, path="int8")
        assert v in (0, 1, 2, 3, 4)
        torch.cuda.synchronize()
        for (a, b, ps), (_, _, c, _) in zip(host, probs):
            _check_residues(c.cpu().numpy(), a, b, ps)
        text = open(path).read().split()
        assert text[-1] == str(v) and text[-2].startswith("gfx950/int8/")
        c2 = rg.Context(device=0, L=26)
        c2.set_tune_cache(path)
        plan = rg.GemmPlan(c2, gps, path="int8")
        assert plan.info()["variant"] == v
        plan.close()
        c2.close()
        ctx.set_tune_cache("")


@pytest.fixture(scope="module")
def batch512():
    batch = synth.uneven_batch(count=512, lo=32, hi=1024, bound=1 << 16, seed=0)
    return batch, [native.exact_matmul(pr.a, pr.b) for pr in batch]


@pytest.mark.parametrize("path", ["int8", "fp64"])
def test_matmul_plan_512_uneven_full(ctx, rg, torch_dev, batch512, path):
    """The 512-product workload exactly as the benchmark runs it (n_i
    log-uniform in [32, 1024], seed 0, entries in [-2^16, 2^16], 2 primes
    each, one whole-product plan, autotuned on the INT8 path, replayed from a
    HIP graph): every entry of every product against the oracle's exact
    product."""
    torch, dev = torch_dev
    _say("512 uneven products, all entries", path)
    batch, wants = batch512
    probs = [rg.MatmulProblem(torch.from_numpy(pr.a).to(dev), torch.from_numpy(pr.b).to(dev),
                              torch.empty((pr.m, pr.n), dtype=torch.int64, device=dev),
                              prime_begin=0, L=2, bound=pr.k << 32) for pr in batch]
    plan = rg.MatmulPlan(ctx, probs, path=path)
    if path == "int8":
        plan.autotune()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.execute()
    torch.cuda.synchronize()
    for rep in range(2):
        for p in probs:
            p.C.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert ctx.status() == 0
        for i, (pr, p) in enumerate(zip(batch, probs)):
            assert np.array_equal(p.C.cpu().numpy(), wants[i]), (rep, i, pr.n)
        _say("  replay", rep, "agrees")
    del g
    plan.close()


SMALL_PRIMES = op.largest_primes_below(1 << 15, 8)


@pytest.mark.parametrize("variant", [0, 2, 3, 4])
def test_small_prime_residue_products(rg, torch_dev, variant):
    """A basis of primes below 2^15 (digits 2 and 3 of every balanced residue
    are zero) mixed with two 26-bit primes: every residue of every product
    against the oracle, with residues at 0, 1, p-1 and (p +- 1)/2, ragged
    shapes past the tile edges, k up to 2100, in four GEMM variants."""
    torch, dev = torch_dev
    _say("small primes variant", variant)
    primes = SMALL_PRIMES + PRIMES[:2]
    c = rg.Context(device=0, primes=primes)
    try:
        rng = np.random.default_rng(100 + variant)
        shapes = [(1, 1, 1), (65, 129, 130), (130, 300, 2100), (200, 33, 64), (7, 1000, 257)]
        probs, host = [], []
        for i, (m, n, k) in enumerate(shapes):
            begin, L = (i % 3, 6) if i != 4 else (6, 4)  # the last mixes two small and two big primes
            ps = primes[begin:begin + L]
            a = np.stack([rng.integers(0, p, size=(m, k)) for p in ps])
            b = np.stack([rng.integers(0, p, size=(k, n)) for p in ps])
            for j, p in enumerate(ps):
                mask = rng.random((m, k)) < 0.3
                a[j][mask] = rng.choice(np.array([0, 1, p - 1, (p - 1) // 2, (p + 1) // 2]), size=int(mask.sum()))
            a, b = a.astype(np.int32), b.astype(np.int32)
            C = torch.full((L, m, n), -1, dtype=torch.int32, device=dev)
            probs.append(rg.GemmProblem(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), C, begin))
            host.append((a, b, ps, C))
        plan = rg.GemmPlan(c, probs, path="int8")
        plan.set_variant(variant)
        plan.execute()
        torch.cuda.synchronize()
        for a, b, ps, C in host:
            _check_residues(C.cpu().numpy(), a, b, ps)
        plan.close()
    finally:
        c.close()


def test_small_prime_whole_products(rg, torch_dev):
    """The 512-product batch's shape with three primes below 2^15 per product
    (|C| <= k 2^32 < M / 2 = 2^44.9 / 2): every entry of every product against
    the exact integer product."""
    torch, dev = torch_dev
    _say("small primes whole products")
    c = rg.Context(device=0, primes=SMALL_PRIMES[:3])
    try:
        batch = synth.uneven_batch(count=40, lo=8, hi=300, bound=1 << 16, seed=43)
        probs = []
        for pr in batch:
            probs.append(rg.MatmulProblem(torch.from_numpy(pr.a).to(dev), torch.from_numpy(pr.b).to(dev),
                                          torch.empty((pr.m, pr.n), dtype=torch.int64, device=dev),
                                          prime_begin=0, L=3, bound=pr.k << 32))
        plan = rg.MatmulPlan(c, probs, path="int8")
        plan.autotune()
        plan.execute()
        torch.cuda.synchronize()
        assert c.status() == 0
        for pr, p in zip(batch, probs):
            assert np.array_equal(p.C.cpu().numpy(), native.exact_matmul(pr.a, pr.b))
        plan.close()
    finally:
        c.close()
