"""The allocation-free entry point (modmatmul_batched_noalloc) against
modmatmul_batched on the same inputs, bit-exact, through the C ABI: two calls
in a row, the second smaller (the shared scratch keeps the first call's
contents), both product paths, and the size limit."""
import sys

import numpy as np
import pytest

from oracle import primes as op

pytestmark = pytest.mark.gpu

PRIMES = op.largest_primes_below(1 << 26, 8)


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_19254_amd as rg
    ctx = rg.Context(device=0, L=8)
    yield torch, torch.device("cuda:0"), rg, ctx
    ctx.close()


def _problems(torch, dev, rg, shapes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for (m, k, n, begin, L) in shapes:
        ps = PRIMES[begin:begin + L]
        a = np.stack([rng.integers(0, p, size=(m, k)) for p in ps]).astype(np.int32)
        b = np.stack([rng.integers(0, p, size=(k, n)) for p in ps]).astype(np.int32)
        out.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), begin))
    return out


def _run(torch, rg, ctx, probs, path, noalloc):
    cs = [torch.full((a.shape[0], a.shape[1], b.shape[2]), -1, dtype=torch.int32, device=a.device)
          for a, b, _ in probs]
    gp = [rg.GemmProblem(a, b, c, prime_begin=begin) for (a, b, begin), c in zip(probs, cs)]
    if noalloc:
        rg.modmatmul_batched_noalloc(ctx, gp, path=path)
    else:
        rg.modmatmul_batched(ctx, gp, path=path)
    torch.cuda.synchronize()
    return [c.cpu().numpy() for c in cs]


@pytest.mark.parametrize("path", ["int8", "fp64"])
def test_noalloc_matches_modmatmul_batched(env, path):
    torch, dev, rg, ctx = env
    big = [(300, 517, 250, 0, 3), (64, 1000, 129, 2, 4), (7, 5, 3, 6, 2)]
    small = [(33, 70, 17, 1, 2)]
    for label, shapes, seed in (("first", big, 1), ("second, smaller", small, 2)):
        _say("noalloc", path, label)
        probs = _problems(torch, dev, rg, shapes, seed)
        want = _run(torch, rg, ctx, probs, path, noalloc=False)
        got = _run(torch, rg, ctx, probs, path, noalloc=True)
        for g, w in zip(got, want):
            assert np.array_equal(g, w)


def test_noalloc_rejects_what_does_not_fit(env):
    torch, dev, rg, ctx = env
    _say("noalloc size limit")
    cap = rg.noalloc_scratch_bytes()
    assert cap == 64 << 20
    # 4 planes of a 2048 x 2048 operand as INT8 digit tiles alone need 64 MiB
    n, L = 2048, 4
    a = torch.zeros((L, n, n), dtype=torch.int32, device=dev)
    c = torch.full((L, n, 8), -1, dtype=torch.int32, device=dev)
    b = torch.zeros((L, n, 8), dtype=torch.int32, device=dev)
    with pytest.raises(rg.RnsError) as e:
        rg.modmatmul_batched_noalloc(ctx, [rg.GemmProblem(a, b, c)], path="int8")
    assert e.value.status == rg.binding.ESCRATCH
    torch.cuda.synchronize()
    assert bool((c == -1).all())                          # nothing was written
    # an empty batch is a no-op
    rg.modmatmul_batched_noalloc(ctx, [], path="int8")
