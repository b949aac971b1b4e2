"""GPU Smith-form driver against the oracle (bit-exact invariant factors).

Expected values: oracle.smith (Bareiss determinant + gcd elimination modulo
the determinant) or, for planted inputs, the invariants planted by the
generator."""
import sys

import numpy as np
import pytest

from oracle import smith as osmith
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_19254_amd as rg
    return rg


@pytest.fixture(scope="module")
def ctx(rg):
    c = rg.Context(device=0, L=24)
    yield c
    c.close()


def test_small_smith_workload(ctx, rg):
    _say("smith 64x64 [-99,99] seed 0")
    a = synth.small_smith(seed=0)
    res = rg.smith_form(ctx, a, seed=1)
    assert res.s == osmith.smith_form(a)
    assert res.stats["restarts"] == 0
    assert res.stats["products"] >= 2


@pytest.mark.parametrize("gen,n", [("small", 64), ("planted", 200), ("random", 300)])
def test_smith_on_fp64_product_path(rg, gen, n):
    """A context created with RNS_CTX_PATH_FP64 runs every product of the
    driver (elimination updates, certificates) on the FP64 path; the Smith
    form is the same."""
    _say("smith on the fp64 product path", gen, n)
    if gen == "small":
        a = synth.small_smith(seed=0)
        want = osmith.smith_form(a)
    elif gen == "planted":
        pl = synth.planted_smith(n, seed=3)
        a, want = pl.a, pl.s
    else:
        a = synth.small_smith(seed=5, n=n, bound=1 << 10)
        want = None
    with rg.Context(device=0, L=24, path="fp64") as c64, rg.Context(device=0, L=24, path="int8") as c8:
        r64 = rg.smith_form(c64, a, seed=1)
        r8 = rg.smith_form(c8, a, seed=1)
    assert r64.s == r8.s
    assert osmith.is_divisor_chain(r64.s)
    if want is not None:
        assert r64.s == want


@pytest.mark.parametrize("n", [3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53])
def test_vandermonde_mod_family(ctx, rg, n):
    # Section 4.1 family; Section 4.2 checks primes 3..53.
    _say("smith vandermonde", n)
    a = synth.vandermonde_mod(n)
    res = rg.smith_form(ctx, a, seed=n)
    s = osmith.smith_form(a)
    assert res.s == s
    assert osmith.is_divisor_chain(res.s)


@pytest.mark.parametrize("n,seed", [(2, 0), (5, 1), (10, 2), (20, 3), (33, 4), (48, 5)])
def test_random_small(ctx, rg, n, seed):
    _say("smith random", n, seed)
    rng = np.random.default_rng(100 + seed)
    while True:
        a = rng.integers(-99, 100, size=(n, n), dtype=np.int64)
        if osmith.bareiss_det(a) != 0:
            break
    assert rg.smith_form(ctx, a, seed=seed).s == osmith.smith_form(a)


@pytest.mark.parametrize("n,seed", [(24, 0), (64, 1), (200, 2)])
def test_planted_small(ctx, rg, n, seed):
    _say("smith planted", n, seed)
    pl = synth.planted_smith(n, seed=seed)
    res = rg.smith_form(ctx, pl.a, seed=seed)
    assert res.s == pl.s


def test_planted_n2000(ctx, rg):
    """The planted workload at full size: A = U diag(s) V, n = 2000."""
    _say("smith planted n=2000")
    pl = synth.planted_smith(2000, seed=0)
    res = rg.smith_form(ctx, pl.a, seed=0)
    assert res.s == pl.s
    print("stats", res.stats, flush=True)


def test_structured_and_singular(ctx, rg):
    _say("smith structured")
    for diag in ([6, 4, 9], [12, 18, 8, 1], [2, 3, 5, 7, 11]):
        a = np.diag(np.array(diag, dtype=np.int64))
        assert rg.smith_form(ctx, a).s == osmith.smith_form(a)
    assert rg.smith_form(ctx, np.array([[-7]], dtype=np.int64)).s == [7]
    assert rg.smith_form(ctx, np.zeros((0, 0), dtype=np.int64)).s == []
    sing = np.array([[1, 2, 3], [2, 4, 6], [1, 0, 1]], dtype=np.int64)
    with pytest.raises(rg.RnsError) as e:
        rg.smith_form(ctx, sing)
    assert e.value.status == 6
    with pytest.raises(rg.RnsError) as e:
        rg.smith_form(ctx, np.zeros((4, 4), dtype=np.int64))
    assert e.value.status == 6


def test_las_vegas_restart_forced(ctx, rg):
    """A failed certification (forced from the host) restarts the method and
    still returns the right S (Section 2.2, Phase 3)."""
    _say("smith forced restart")
    a = synth.small_smith(seed=3, n=24)
    want = osmith.smith_form(a)
    ctx.force_cert_failures(2)
    res = rg.smith_form(ctx, a, seed=5)
    assert res.s == want
    assert res.stats["restarts"] >= 2
    ctx.force_cert_failures(0)


def test_result_independent_of_seed(ctx, rg):
    _say("smith seeds")
    a = synth.planted_smith(40, seed=7).a
    r = [rg.smith_form(ctx, a, seed=sd).s for sd in (0, 1, 12345)]
    assert r[0] == r[1] == r[2]


# ------------------------------------------------------- p-adic lifting path --
import json
import os

_GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "smith_lifting.json")))


def _golden_matrix(case):
    if case["gen"] == "small_smith":
        return synth.small_smith(seed=case["seed"], attempt=case["attempt"], n=case["n"], bound=case["bound"])
    return synth.planted_small(case["n"], seed=case["seed"]).a


def _golden_s(case):
    return [1] * case["ones"] + [int(v) for v in case["tail"]]


@pytest.fixture
def lifting_ctx(ctx):
    yield ctx
    ctx.set_smith_path("auto")


@pytest.mark.parametrize("case", _GOLDEN["cases"], ids=lambda c: "%s-n%d" % (c["gen"], c["n"]))
def test_lifting_golden(lifting_ctx, rg, case):
    """Inputs whose invariants are too large for the residue path: the auto
    choice takes p-adic lifting (planted inputs are forced onto it to make the
    projection grow); S equals the oracle's."""
    ctx = lifting_ctx
    _say("smith lifting", case)
    a = _golden_matrix(case)
    if case["gen"] == "planted_small":
        ctx.set_smith_path("lifting")
    res = rg.smith_form(ctx, a, seed=case["seed"])
    assert res.s == _golden_s(case)
    assert res.stats["path"] == 1
    assert res.stats["lift_steps"] > 0
    if case["gen"] == "planted_small":
        assert res.stats["columns"] == 16          # 8 invariants > 1: t grew 4 -> 8 -> 16
    print("stats", res.stats, flush=True)


@pytest.mark.parametrize("n,seed,bound", [(16, 0, 100), (24, 1, 100), (40, 2, 100), (64, 3, 100),
                                          (17, 4, 1 << 15), (33, 5, 1 << 20)])
def test_lifting_forced_matches_oracle(lifting_ctx, rg, n, seed, bound):
    """Forced p-adic lifting against the oracle; entries below 2^15 in
    magnitude take the int16 form of A in the lifting kernels, the larger ones
    (|a| up to 2^15 and 2^20) the int32 form."""
    ctx = lifting_ctx
    _say("smith lifting forced", n, seed, bound)
    rng = np.random.default_rng(500 + seed)
    while True:
        a = rng.integers(-bound + 1, bound, size=(n, n), dtype=np.int64)
        if bound > 100:
            a[0, 0] = bound if seed % 2 == 0 else -bound        # one entry just outside int16
        if osmith.bareiss_det(a) != 0:
            break
    ctx.set_smith_path("lifting")
    res = rg.smith_form(ctx, a, seed=seed)
    assert res.s == osmith.smith_form(a)
    assert res.stats["path"] == 1 and res.stats["cert_exact"] == 1


@pytest.mark.parametrize("edge", [32639, 32700])
def test_lifting_int16_edge_matches_oracle(lifting_ctx, rg, edge):
    """Entries at the edge of the int16 form of A: every |a| <= 32639 splits
    into two signed bytes (here 127 and -127 at the extremes) and takes the
    matrix-core residual update; an entry of 32700, whose high byte would be
    128 in that split, must send A to the int32 form instead."""
    ctx = lifting_ctx
    n = 40
    _say("smith lifting int16 edge", n, edge)
    rng = np.random.default_rng(900 + edge)
    while True:
        a = rng.integers(-32639, 32640, size=(n, n), dtype=np.int64)
        for i in range(6):
            a[i, i] = edge if i % 2 == 0 else -32639
            a[i, n - 1 - i] = 32639
        if osmith.bareiss_det(a) != 0:
            break
    ctx.set_smith_path("lifting")
    res = rg.smith_form(ctx, a, seed=edge)
    assert res.s == osmith.smith_form(a)
    assert res.stats["path"] == 1
    # which form of A and which lifting kernels ran (bit 1: A X on the matrix
    # cores, bit 3: A stored as int16)
    int16 = edge < 32640
    assert res.stats["lift_a_bytes"] == (2 if int16 else 4)
    assert bool(res.stats["lift_kernels"] & rg.binding.LIFT_A_INT16) == int16
    assert bool(res.stats["lift_kernels"] & rg.binding.LIFT_AX_MFMA) == int16
    assert res.stats["lift_kernels"] & rg.binding.LIFT_C_MFMA


def test_lifting_vector_kernels_match(rg, monkeypatch):
    """The lifting products on the vector units (RNS_LIFT_VECTOR=1, read when
    a context is created) give the same invariants as the default matrix-core
    products; both are checked against the stored golden values."""
    case = _GOLDEN["cases"][0]
    _say("smith lifting, vector kernels", case)
    a = _golden_matrix(case)
    monkeypatch.setenv("RNS_LIFT_VECTOR", "1")
    vctx = rg.Context(device=0, L=24)
    monkeypatch.delenv("RNS_LIFT_VECTOR")
    try:
        res = rg.smith_form(vctx, a, seed=case["seed"])
    finally:
        vctx.close()
    assert res.s == _golden_s(case) and res.stats["path"] == 1 and res.stats["lift_steps"] > 0


def test_lifting_restart_seed_and_errors(lifting_ctx, rg):
    ctx = lifting_ctx
    _say("smith lifting restart / seed / singular / not applicable")
    case = _GOLDEN["cases"][0]
    a = _golden_matrix(case)
    want = _golden_s(case)
    ctx.force_cert_failures(2)
    res = rg.smith_form(ctx, a, seed=9)
    ctx.force_cert_failures(0)
    assert res.s == want and res.stats["restarts"] >= 2
    assert rg.smith_form(ctx, a, seed=12345).s == want
    # singular with small entries: every lifting prime divides det A = 0
    sing = synth.small_smith(seed=4, n=32, bound=99).copy()
    sing[5] = sing[7] * 2
    ctx.set_smith_path("lifting")
    with pytest.raises(rg.RnsError) as e:
        rg.smith_form(ctx, sing)
    assert e.value.status == 6
    # entries too large for the lifting path
    big = synth.planted_smith(24, seed=0).a
    with pytest.raises(rg.RnsError) as e:
        rg.smith_form(ctx, big)
    assert e.value.status == 8


def test_largest_invariant_paper_fact(ctx, rg):
    """Section 4.1 prints the size of s_n for A_ij = i^j mod n at n = 1009:
    4083 bits.  Phase 1 on the GPU (p-adic lifting, reconstruction of the
    common denominator) must reproduce it."""
    facts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
    fact = facts["vandermonde_mod_sn_bits"]
    _say("largest invariant, vandermonde n =", fact["n"])
    res = rg.largest_invariant(ctx, synth.vandermonde_mod(fact["n"]), seed=1)
    assert len(res.s) == 1
    assert res.s[0].bit_length() == fact["bits"]


@pytest.mark.parametrize("n", [17, 29, 41, 53])
def test_largest_invariant_matches_oracle(ctx, rg, n):
    _say("largest invariant vs oracle, vandermonde", n)
    a = synth.vandermonde_mod(n)
    assert rg.largest_invariant(ctx, a, seed=n).s == [osmith.smith_form(a)[-1]]


@pytest.mark.parametrize("n", [700, 1100])
def test_lifting_certificate_over_several_panels(lifting_ctx, rg, n):
    """The lifting path at sizes where the determinant elimination of the
    certificate spans two and three 512-column panels (so the in-panel steps,
    the panel rows beyond the panel and the deep Schur-complement update all
    run), with a zero in the (0, 0) position so that the first pivot block
    needs row exchanges.  The planted invariants are the expected values (a
    row permutation does not change S), and the certificate must be exact."""
    ctx = lifting_ctx
    _say("smith lifting, certificate over panels", n)
    pl = synth.planted_small(n, seed=n)
    a = pl.a.copy()
    rows0 = np.nonzero(a[:, 0] == 0)[0]
    assert rows0.size > 0
    a[[0, rows0[0]]] = a[[rows0[0], 0]]
    assert a[0, 0] == 0
    ctx.set_smith_path("lifting")
    res = rg.smith_form(ctx, a, seed=3)
    assert res.s == pl.s
    assert res.stats["path"] == 1 and res.stats["cert_exact"] == 1 and res.stats["cert_primes"] >= 1
