#!/usr/bin/env python3
"""Benchmark of the exact multi-modular integer matrix product on one MI355X.

One step = the whole hot path over one batch of synthetic input that is
already resident in HBM, as one execution of a whole-product plan:
    int64 A and B -> tiled residue digits   all 24 primes, one launch
    24 exact products mod p                 one GEMM launch
    CRT of the 24 planes -> int64 result    one launch
The same product through the four boundary calls (rns_reduce(A),
rns_reduce(B), modmatmul_batched, crt_reconstruct) is timed beside it
(`boundary_calls`).  Workload: A, B 4096 x 4096, entries uniform in
[-2^20, 2^20] (seeds 0 and 1), the 24 largest primes below 2^26.  The headline
runs the INT8-limb path; the FP64-MFMA path is timed on the same inputs.

Prints one JSON line.  `value` is residue int-ops per second of the whole step,
2*m*n*k*L per step.  The roofline entry is for the dominant kernel (the GEMM):
its average launch duration is measured with HIP events recorded on the stream
the kernel runs on, and its achieved rate counts the MFMA operations the path
executes (16 digit-pair products per residue product on the INT8 path).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "exact modmatmul int-ops/s (INT8-limb vs FP64 path); SNF solves/s, p50/p99"
PEAK_INT8_TOPS = 5000.0      # MI355X dense INT8 MFMA, TOP/s
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 matrix, TFLOP/s
PEAK_HBM_GBS = 8000.0


GEMM_SOURCES = ("paper_2605_19254_amd/csrc/gemm_i8.hip", "paper_2605_19254_amd/csrc/gemm_common.hpp",
                "paper_2605_19254_amd/csrc/internal.hpp")
TRAFFIC_SUMMARY = "profiles/k_gemm_i8_half_n4096_L24_traffic.md"
I8_KERNEL_NAMES = {0: "k_gemm_i8_lds", 1: "k_gemm_i8", 2: "k_gemm_i8_half_persistent",
                   3: "k_gemm_i8_w8", 4: "k_gemm_i8_half"}


def gemm_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in GEMM_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(kernel: str):
    """HBM bytes per launch of the GEMM kernel from the committed counter
    summary, or None when that summary is missing, is for another kernel, or
    was taken on GEMM sources other than the ones in this tree."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
    try:
        if fields.get("kernel") != kernel or fields.get("gemm_sources_sha256") != gemm_source_hash():
            return None
        return float(fields["fetch_bytes_per_launch"]) + float(fields["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--primes", type=int, default=24)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-rows", type=int, default=384,
                    help="rows of C the oracle computes for the CPU baseline (0 = skip)")
    ap.add_argument("--cpu-rows-1core", type=int, default=16,
                    help="rows of C for the single-core oracle timing (0 = skip)")
    ap.add_argument("--out", default="")
    ap.add_argument("--batched", type=int, default=512,
                    help="also time the batched workload with this many uneven products (0 = skip)")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--smith", type=int, default=1, help="time the Smith-form workloads (0 = skip)")
    ap.add_argument("--stress", type=int, default=1,
                    help="time the full-range residue product with 10-word CRT (0 = skip)")
    ap.add_argument("--serving", type=int, default=200,
                    help="requests per open-loop serving point (0 = skip)")
    ap.add_argument("--massager-max", type=int, default=5003,
                    help="largest n of the Smith massager leg (Section 4.1 family; 0 = skip)")
    ap.add_argument("--only", default="", choices=["", "batched", "smith", "serving", "lifting", "smith64",
                                                 "planted2000", "stress", "massager", "unimodular"],
                    help="run only this workload (for profiling)")
    ap.add_argument("--unimodular-n", type=int, default=4096,
                    help="matrix order of the unimodularity certificate leg (Phase 3's certificate "
                         "alone; 0 = skip)")
    ap.add_argument("--lifting-n", type=int, default=10007,
                    help="matrix order of the --only lifting workload (one random Smith-form solve)")
    ap.add_argument("--calibrate-iters", type=int, default=300000,
                    help="iterations of the random-operand INT8 MFMA ceiling probe (0 = skip)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one plain device copy of this many bytes (a known-size "
                         "reference for hardware byte counters)")
    return ap.parse_args()


def cpu_baseline(a, b, primes, rows, threads=0):
    """The oracle as it stands, on the first `rows` rows of C: reduce, the
    per-prime schoolbook products (plain C loops, OpenMP on `threads` threads,
    0 = all), CRT in Python ints."""
    import numpy as np
    from oracle import native, rns as orns
    if threads:
        native.set_threads(threads)
    t0 = time.perf_counter()
    ra = orns.reduce(a[:rows], primes)
    rb = orns.reduce(b, primes)
    rc = orns.modmatmul_planes(ra, rb, primes)
    c = orns.crt_planes(rc, primes)
    t = time.perf_counter() - t0
    n = a.shape[1]
    ops = 2.0 * rows * n * b.shape[1] * len(primes)
    # spot-check the sample against the exact product
    want = native.exact_matmul(a[:2], b)
    assert all(int(c[i, j]) == int(want[i, j]) for i in range(2) for j in range(0, b.shape[1], 97))
    cores = native.num_threads()
    if threads:
        native.set_threads(os.cpu_count() or 1)
    return {"value": ops / t, "unit": "int-ops/s", "cores": cores, "kind": "oracle",
            "sample": "rows 0..%d of C (%d x %d x %d, %d primes): reduce, per-prime schoolbook "
                      "modmatmul, CRT; %.1f s" % (rows - 1, rows, n, b.shape[1], len(primes), t),
            "seconds": t}


def _oracle_timings(conn, n, L, rows1):
    """Single-core oracle timings, run in a child process (forked before the
    GPU is touched) while the parent times GPU work: the headline product's
    oracle on `rows1` rows of C with one thread, and the oracle's Smith form of
    the planted n = 200 matrix (the planted n = 2000 workload's generator)."""
    out = {}
    try:
        import synth
        from oracle import primes as op, smith as osmith
        a, b = synth.square_pair(n=n, bound=1 << 20, seed_a=0, seed_b=1)
        if rows1 > 0:
            out["headline_1core"] = cpu_baseline(a, b, op.largest_primes_below(1 << 26, L), rows1, threads=1)
        del a, b
        pl = synth.planted_smith(200, seed=0)
        t0 = time.perf_counter()
        ok = osmith.smith_form(pl.a) == pl.s
        out["planted_200"] = {"value": time.perf_counter() - t0, "unit": "s", "cores": 1, "kind": "oracle",
                              "sample": "planted n = 200, seed 0 (Bareiss determinant + gcd elimination mod d, "
                                        "Python)", "agrees_with_planted": ok}
    except Exception as e:                       # reported, never fatal to the GPU measurements
        out["error"] = repr(e)
    conn.send(out)
    conn.close()


def run_batched(rg, torch, dev, count, steps):
    """512 independent products C_i = A_i B_i, n_i log-uniform in [32, 1024]
    (seed 0), entries uniform in [-2^16, 2^16], 2 primes each (|C| <= n 2^32).
    One whole-product plan (a conversion launch and a GEMM launch over the
    whole batch, the GEMM doing both primes of each tile and the two-prime CRT
    into int64), captured in a HIP graph and replayed.  Ablations: the same
    plan with the CRT as a launch of its own over resident residue planes
    (autotuned, and its persistent GEMM), the FP64 path, and one plan per
    problem launched one after another."""
    import numpy as np
    import synth
    from oracle import native, rns as orns
    batch = synth.uneven_batch(count=count, lo=32, hi=1024, bound=1 << 16, seed=0)
    ctx = rg.Context(device=0, L=2)
    probs = []
    for pr in batch:
        probs.append(rg.MatmulProblem(torch.from_numpy(pr.a).to(dev), torch.from_numpy(pr.b).to(dev),
                                      torch.empty((pr.m, pr.n), dtype=torch.int64, device=dev),
                                      prime_begin=0, L=2, bound=pr.k << 32))
    ops = sum(2.0 * p.m * p.n * p.k * 2 for p in batch)
    plan = rg.MatmulPlan(ctx, probs, path="int8")
    variant = plan.autotune()
    plan.execute()
    torch.cuda.synchronize()
    # correctness: smallest, median and largest problem against the oracle
    order = sorted(range(count), key=lambda i: batch[i].n)
    for i in (order[0], order[count // 2], order[-1]):
        rows = np.array([0, batch[i].m - 1])
        got = probs[i].C[torch.from_numpy(rows).to(dev)].cpu().numpy()
        if not np.array_equal(got, native.exact_matmul(batch[i].a[rows], batch[i].b)):
            raise SystemExit("bench.py: batched result differs from the oracle")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.execute()
    torch.cuda.synchronize()
    # As many untimed replays as timed ones first: the first few replays
    # after the set-up run about 8 % slower while the GPU comes up to speed.
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    def replay_ms(pl, reps):
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        gg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gg, stream=st):
            pl.execute()
        torch.cuda.synchronize()
        for _ in range(reps):                 # untimed, as for the default plan
            gg.replay()
        torch.cuda.synchronize()
        t0_ = time.perf_counter()
        for _ in range(reps):
            gg.replay()
        torch.cuda.synchronize()
        r = 1000.0 * (time.perf_counter() - t0_) / reps
        del gg
        return r

    # ablation: the CRT as a launch of its own over resident C residue planes
    # (the GEMM autotuned), and that plan with the persistent GEMM (two
    # work-groups per CU take half-tiles, longest first, from a counter)
    ctx_sep = rg.Context(device=0, L=2, separate_crt=True)
    plan_sep = rg.MatmulPlan(ctx_sep, probs, path="int8")
    variant_sep = plan_sep.autotune()
    ms_separate = replay_ms(plan_sep, steps)
    for i in (order[0], order[count // 2], order[-1]):
        rows = np.array([0, batch[i].m - 1])
        got = probs[i].C[torch.from_numpy(rows).to(dev)].cpu().numpy()
        if not np.array_equal(got, native.exact_matmul(batch[i].a[rows], batch[i].b)):
            raise SystemExit("bench.py: batched result (separate CRT) differs from the oracle")
    plan_sep.set_variant(2)
    ms_persistent = replay_ms(plan_sep, steps)
    plan_sep.close()
    ctx_sep.close()
    # ablation: every residue product on the FP64 MFMA path
    plan64 = rg.MatmulPlan(ctx, probs, path="fp64")
    ms_fp64 = replay_ms(plan64, max(2, steps // 2))
    for i in (order[0], order[count // 2], order[-1]):
        rows = np.array([0, batch[i].m - 1])
        got = probs[i].C[torch.from_numpy(rows).to(dev)].cpu().numpy()
        if not np.array_equal(got, native.exact_matmul(batch[i].a[rows], batch[i].b)):
            raise SystemExit("bench.py: batched result (FP64 path) differs from the oracle")
    plan64.close()
    # ablation: a plan per problem, launched in a host loop, no graph
    singles = [rg.MatmulPlan(ctx, [p], path="int8") for p in probs]
    for sp in singles:
        sp.execute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sp in singles:
        sp.execute()
    torch.cuda.synchronize()
    ms_loop = 1000.0 * (time.perf_counter() - t0)
    for sp in singles:
        sp.close()
    info = plan.info()
    # oracle on a sample of the batch (the first 24 problems of the draw)
    sample = batch[:24]
    t0 = time.perf_counter()
    for pr in sample:
        ps = ctx.primes[:2]
        rc = orns.modmatmul_planes(orns.reduce(pr.a, ps), orns.reduce(pr.b, ps), ps)
        orns.crt_planes(rc, ps)
    tc = time.perf_counter() - t0
    sops = sum(2.0 * p.m * p.n * p.k * 2 for p in sample)
    del g
    plan.close()
    ctx.close()
    return {"workload": "%d independent products, n log-uniform in [32, 1024] (seed 0), entries in "
                        "[-2^16, 2^16], 2 primes each; one plan under a HIP graph" % count,
            "value": ops / (ms * 1e-3), "unit": "int-ops/s", "ms_per_step": ms, "steps": steps,
            "residue_ops": ops, "variant": variant, "tiles": info["tiles"],
            "mfma_frac_of_int8_peak": 16.0 * ops / (ms * 1e-3) / 1e12 / PEAK_INT8_TOPS,
            "per_problem_launch_loop_ms": ms_loop,
            "separate_crt_ms_per_step": ms_separate, "separate_crt_variant": variant_sep,
            "separate_crt_persistent_gemm_ms_per_step": ms_persistent,
            "fp64_path_ms_per_step": ms_fp64,
            "cpu_baseline": {"value": sops / tc, "unit": "int-ops/s", "cores": native.num_threads(),
                             "kind": "oracle", "sample": "first 24 problems of the batch, %.1f s" % tc}}


def run_lifting(rg, n):
    """One Smith-form solve of a random n x n matrix with entries in
    [-2^10, 2^10] (the p-adic lifting path; n = 10007 is the serving tail)."""
    import synth
    ctx = rg.Context(device=0, L=24)
    try:
        a = synth.small_smith(seed=0, n=n, bound=1 << 10)
        t0 = time.perf_counter()
        r = rg.smith_form(ctx, a, seed=0)
        t = time.perf_counter() - t0
    finally:
        ctx.close()
    if any(r.s[i + 1] % r.s[i] for i in range(len(r.s) - 1)):
        raise SystemExit("bench.py: Smith form (random n=%d) is not a divisor chain" % n)
    return {"workload": "n = %d, entries uniform in [-2^10, 2^10], seed 0 (p-adic lifting)" % n,
            "seconds": t, "stats": r.stats, "largest_invariant_bits": r.s[-1].bit_length()}


def _traced(rg, ctx, a, seed=0):
    """One more solve with every library kernel bracketed by HIP events:
    (kernel milliseconds, kernel launches, wall milliseconds).  Tracing adds
    work of its own, so the untraced timings above it are the figures."""
    ctx.profile(True)
    ctx.profile_read("")
    t0 = time.perf_counter()
    rg.smith_form(ctx, a, seed=seed)
    wall = 1000.0 * (time.perf_counter() - t0)
    ms, launches = ctx.profile_read("")
    ctx.profile(False)
    return {"kernel_ms": ms, "launches": launches, "wall_ms_traced": wall, "kernel_share": ms / wall}


def run_smith(rg, reps=10, oracle_bg=None):
    """Smith forms: the 64 x 64 matrix with entries in [-99, 99] (seed 0) and
    the planted n = 2000 matrix (A = U diag(s) V, seed 0), each checked against
    the oracle or the planted invariants; the oracle is timed on the 64 x 64
    matrix and on a planted n = 200 matrix (in `oracle_bg` when the caller
    timed it in a child process, else here)."""
    import synth
    from oracle import smith as osmith
    out = {}
    with rg.Context(device=0, L=24) as ctx:
        a = synth.small_smith(seed=0)
        want = osmith.smith_form(a)
        rg.smith_form(ctx, a)                      # warm-up (internal basis, kernels)
        t0 = time.perf_counter()
        for r in range(reps):
            res = rg.smith_form(ctx, a, seed=r)
        t = (time.perf_counter() - t0) / reps
        if res.s != want:
            raise SystemExit("bench.py: Smith form (64x64) differs from the oracle")
        t0 = time.perf_counter()
        osmith.smith_form(a)
        to = time.perf_counter() - t0
        out["small_64"] = {"workload": "64x64, entries uniform in [-99, 99], seed 0", "solves_per_s": 1.0 / t,
                           "ms_per_solve": 1000 * t, "stats": res.stats, "traced": _traced(rg, ctx, a),
                           "cpu_baseline": {"value": 1.0 / to, "unit": "solves/s", "cores": 1, "kind": "oracle",
                                            "sample": "the same matrix"}}
        # the same solve with every residue product on the FP64 MFMA path
        with rg.Context(device=0, L=24, path="fp64") as c64:
            rg.smith_form(c64, a)
            t0 = time.perf_counter()
            for r in range(reps):
                res64 = rg.smith_form(c64, a, seed=r)
            t64 = (time.perf_counter() - t0) / reps
        if res64.s != want:
            raise SystemExit("bench.py: Smith form (64x64, FP64 products) differs from the oracle")
        out["small_64"]["fp64_path"] = {"solves_per_s": 1.0 / t64, "ms_per_solve": 1000 * t64}
        pl = synth.planted_smith(2000, seed=0)
        t0 = time.perf_counter()
        res = rg.smith_form(ctx, pl.a, seed=0)
        t = time.perf_counter() - t0
        if res.s != pl.s:
            raise SystemExit("bench.py: planted Smith form (n=2000) differs")
        # random n = 4000, entries in [-2^10, 2^10]: the p-adic lifting path
        ar = synth.small_smith(seed=0, n=4000, bound=1 << 10)
        t0 = time.perf_counter()
        rr = rg.smith_form(ctx, ar, seed=0)
        tr = time.perf_counter() - t0
        if any(rr.s[i + 1] % rr.s[i] for i in range(len(rr.s) - 1)):
            raise SystemExit("bench.py: Smith form (random n=4000) is not a divisor chain")
        out["random_4000"] = {"workload": "n = 4000, entries uniform in [-2^10, 2^10], seed 0 (p-adic lifting)",
                              "seconds": tr, "stats": rr.stats,
                              "nontrivial": sum(1 for v in rr.s if v != 1),
                              "largest_invariant_bits": rr.s[-1].bit_length()}
        if oracle_bg and "planted_200" in oracle_bg:
            cb = oracle_bg["planted_200"]
        else:
            p200 = synth.planted_smith(200, seed=0)
            t0 = time.perf_counter()
            ok = osmith.smith_form(p200.a) == p200.s
            cb = {"value": time.perf_counter() - t0, "unit": "s", "cores": 1, "kind": "oracle",
                  "sample": "planted n = 200, seed 0", "agrees_with_planted": ok}
        out["planted_2000"] = {"workload": "A = U diag(s) V, n = 2000, 4n random row and column operations, "
                                           "5 planted factors from the primes below 100, seed 0",
                               "seconds": t, "stats": res.stats, "traced": _traced(rg, ctx, pl.a),
                               "cpu_baseline": cb}
    return out


def run_smith_one(rg, which, reps=10):
    """One Smith-form workload alone (for a kernel trace of just that
    workload): the 64 x 64 matrix (10 solves after a warm-up) or the planted
    n = 2000 matrix (one solve after a warm-up), with the traced kernel time
    and launch count of one more solve."""
    import synth
    from oracle import smith as osmith
    with rg.Context(device=0, L=24) as ctx:
        if which == "smith64":
            a = synth.small_smith(seed=0)
            want = osmith.smith_form(a)
        else:
            pl = synth.planted_smith(2000, seed=0)
            a, want, reps = pl.a, pl.s, 1
        rg.smith_form(ctx, a)
        t0 = time.perf_counter()
        for r in range(reps):
            res = rg.smith_form(ctx, a, seed=r)
        t = (time.perf_counter() - t0) / reps
        if res.s != want:
            raise SystemExit("bench.py: Smith form (%s) differs" % which)
        return {"workload": which, "ms_per_solve": 1000 * t, "solves": reps, "stats": res.stats,
                "traced": _traced(rg, ctx, a)}


# Section 4.3, Tables 1 and 2 (Apple M4 Max, one core-cluster CPU run with
# OpenBLAS): wall seconds of the paper's implementation on A_ij = i^j mod n,
# and its Phase 1 / Phase 2 / Phase 3 split (LIF, IM, UC).  Context only:
# another machine's numbers.
PAPER_TABLE1_S = {53: 0.033, 101: 0.083, 211: 0.447, 503: 2.07, 1009: 26.30, 2003: 134.4, 5003: 1744.0,
                  10007: 5399.0}
PAPER_TABLE2 = {53: (0.011, 0.005, 0.004, 0.020), 101: (0.024, 0.026, 0.018, 0.070),
                211: (0.078, 0.263, 0.078, 0.428), 503: (0.644, 0.762, 0.563, 2.069),
                1009: (2.424, 17.68, 3.835, 24.67), 2003: (18.76, 93.01, 23.43, 139.7),
                5003: (168.6, 692.2, 545.6, 1515.0)}
MASSAGER_SIZES = (53, 101, 211, 503, 1009, 2003, 5003, 10007)


def run_massager(rg, nmax):
    """The Smith massager (U, M, T, S) of A_ij = i^j mod n (Section 4.1) for
    the paper's prime sizes up to nmax: one timed solve each after a warm-up,
    the divisor chain and (n = 101, 199 from the stored oracle values; n = 1009
    from the printed 4083-bit s_n) the invariants checked, A M S^-1 checked
    integral on its three last columns up to n = 2003 (Phase 3's certificate
    covers every size); the paper's Table 1 and 2 figures
    beside each size as context."""
    import numpy as np
    import synth
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "tests", "golden", "smith_vandermonde.json")) as f:
        golden = {c["n"]: c for c in json.load(f)["cases"]}
    out = []
    with rg.Context(device=0, L=24) as ctx:
        rg.smith_massager(ctx, synth.vandermonde_mod(53), seed=0)     # warm-up
        for n in [m for m in MASSAGER_SIZES if m <= nmax] + [199]:
            a = synth.vandermonde_mod(n)
            t0 = time.perf_counter()
            r = rg.smith_massager(ctx, a, seed=1, fetch=(), m_columns=[n - 3, n - 2, n - 1])
            t = time.perf_counter() - t0
            S = r.s
            if any(S[i + 1] % S[i] for i in range(n - 1)) or r.stats["cert_exact"] != 1:
                raise SystemExit("bench.py: massager n=%d: not a certified divisor chain" % n)
            if n in golden:
                g = golden[n]
                if S != [1] * g["ones"] + [int(v) for v in g["tail"]]:
                    raise SystemExit("bench.py: massager n=%d differs from the oracle's Smith form" % n)
            if n == 1009 and S[-1].bit_length() != 4083:
                raise SystemExit("bench.py: massager n=1009: s_n is not 4083 bits")
            if n <= 2003:                # (object arithmetic: minutes at n = 5003)
                ao = a.astype(object)
                for j in range(n - 3, n):
                    if any(v % S[j] for v in ao.dot(np.array(r.m_columns[j], dtype=object))):
                        raise SystemExit("bench.py: massager n=%d: A M S^-1 not integral" % n)
            rec = {"n": n, "seconds": t, "nontrivial": sum(1 for v in S if v != 1),
                   "largest_invariant_bits": S[-1].bit_length(), "stats": r.stats}
            if n in PAPER_TABLE1_S:
                rec["paper_seconds"] = PAPER_TABLE1_S[n]
                rec["speedup_vs_paper"] = PAPER_TABLE1_S[n] / t
            if n in PAPER_TABLE2:
                rec["paper_lif_im_uc_total"] = PAPER_TABLE2[n]
            out.append(rec)
            print("[bench] massager n=%d %.3f s" % (n, t), file=sys.stderr, flush=True)
    return {"workload": "Smith massager of A_ij = i^j mod n (Section 4.1), one solve per n, seed 1",
            "paper_hardware": "Apple M4 Max, OpenBLAS (Section 4)", "sizes": out}


def run_unimodular(rg, n):
    """Phase 3's certificate alone (rns_unimodular_certify, Section 2.2) on a
    unimodular n x n matrix L U (L, U unit triangular with entries in
    {-1, 0, 1}, rows and columns permuted, seed 0) and on its twin with
    det = 2 (last row of L doubled): one timed call each after a warm-up.  The
    verdicts are checked: True for L U, False after exactly the needed steps
    for the twin (a wrong residue at any step would break one of the two)."""
    import numpy as np

    def lu(m, det):
        rng = np.random.default_rng(0)
        L = np.tril(rng.integers(-1, 2, size=(m, m)), -1) + np.eye(m, dtype=np.int64)
        U = np.triu(rng.integers(-1, 2, size=(m, m)), 1) + np.eye(m, dtype=np.int64)
        L[m - 1, :] *= det
        # |entries| <= 2 m < 2^53: the double product is exact (and uses BLAS)
        D = np.rint(L.astype(np.float64) @ U.astype(np.float64)).astype(np.int64)
        pr, pc = rng.permutation(m), rng.permutation(m)
        return np.ascontiguousarray(D[pr][:, pc])

    out = {"workload": "unimodularity certificate of an n x n unimodular L U product and its det-2 twin "
                       "(entries of L, U in {-1, 0, 1}, seed 0)", "n": n}
    with rg.Context(device=0, L=2) as ctx:
        rg.unimodular_certify(ctx, lu(256, 1))                               # warm-up
        for name, det in (("unimodular", 1), ("det2", 2)):
            d = lu(n, det)
            print("[bench] unimodular %s n=%d: input built" % (name, n), file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            r = rg.unimodular_certify(ctx, d)
            t = time.perf_counter() - t0
            want = det == 1
            if r.verdict is not want or (not want and r.info["steps"] != r.info["steps_needed"]):
                raise SystemExit("bench.py: unimodular certificate gave the wrong verdict for %s" % name)
            info = dict(r.info)
            out[name] = {"seconds": t, "verdict": r.verdict, "steps": info["steps"],
                         "steps_needed": info["steps_needed"], "x_primes": info["x_primes"],
                         "q_primes": info["q_primes"], "log2_bound": info["log2_bound"],
                         "residue_ops": info["residue_ops"], "products": info["products"],
                         "residue_ops_per_s": info["residue_ops"] / t}
            print("[bench] unimodular %s n=%d %.3f s (%d steps)" % (name, n, t, info["steps"]),
                  file=sys.stderr, flush=True)
    return out


def _serving_stream(count, rate, seed, tail):
    """Serving requests: Poisson arrivals at `rate`, n log-uniform in
    [100, 4000], entries uniform in [-2^10, 2^10] (a singular draw is
    redrawn), the n = 10007 tail at the 50th arrival when `tail`, and one
    singular request (all ones, n = 100) at position 5."""
    import numpy as np
    import synth
    from oracle import smith as osmith
    stream = synth.serving_stream(count, rate, lo=100, hi=4000, tail_n=10007 if tail else 0,
                                  tail_at=50, seed=seed)
    reqs = []
    for r in stream.requests:
        if r.rid == 5:
            reqs.append((r, np.ones((100, 100), dtype=np.int64), "singular"))
            continue
        a = synth.request_matrix(r)
        if r.n <= 64 and osmith.bareiss_det(a) == 0:
            a = synth.request_matrix(r, attempt=1)
        reqs.append((r, a, "random"))
    return reqs


def run_stress(rg, torch, dev, ctx, n, L, steps=3):
    """Full-range residues: every plane uniform in [0, p_j) (seeded on the
    device), the INT8 product of the n x n planes over L primes and the exact
    (Garner) CRT into 10-word outputs; sampled entries against the oracle."""
    import numpy as np
    from oracle import rns as orns
    W = 10
    g = torch.Generator(device=dev)
    ra = torch.empty((L, n, n), dtype=torch.int32, device=dev)
    rb = torch.empty_like(ra)
    for j, p in enumerate(ctx.primes[:L]):
        g.manual_seed(1000 + j)
        ra[j].random_(0, p, generator=g)
        g.manual_seed(2000 + j)
        rb[j].random_(0, p, generator=g)
    rc = torch.empty_like(ra)
    out = torch.empty((n, n, W), dtype=torch.int64, device=dev)
    prob = [rg.GemmProblem(ra, rb, rc)]

    def step():
        rg.modmatmul_batched(ctx, prob, path="int8")
        rg.crt_reconstruct(ctx, rc, L=L, W=W, out=out)

    step()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read("")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    ctx.profile(False)
    kern = {}
    for name in ("k_prep", "k_gemm", "k_crt"):
        ms, cnt = ctx.profile_read(name)
        if cnt:
            kern[name] = {"avg_ms": ms / cnt, "launches": cnt}
    primes = ctx.primes[:L]
    for (i, j) in ((0, 0), (n // 2, n // 3), (n - 1, n - 1), (17, n - 5)):
        arow = ra[:, i, :].cpu().numpy().astype(np.int64)
        bcol = rb[:, :, j].cpu().numpy().astype(np.int64)
        r = [orns.modmatmul_entry(arow[q], bcol[q], p) for q, p in enumerate(primes)]
        want = orns.to_words(orns.crt(r, primes), W)
        got = [int(v) & ((1 << 64) - 1) for v in out[i, j].cpu().numpy()]
        if got != want:
            print("bench.py: full-range residue product differs from the oracle at", (i, j), file=sys.stderr)
            sys.exit(1)
    if ctx.status() != 0:
        print("bench.py: CRT reported an error on full-range residues", file=sys.stderr)
        sys.exit(1)
    ops = 2.0 * n ** 3 * L
    # The other conversions of the path on the same planes: the 10-word
    # integers back to 24 residue planes (multiword reduction; the round trip
    # must give the planes back exactly), and the planes converted to 24 other
    # primes, exactly (no bound) and in one pass (with a bound leaving the
    # Lagrange margin, on the planes of the product's residues reduced to a
    # bounded range); every entry compared on the device.
    conv = {}
    back = torch.empty_like(rc)
    c2 = rg.Context(device=0, L=2 * L)
    try:
        def tk(f, reps=3):
            f()
            torch.cuda.synchronize()
            c2.profile(True)
            c2.profile_read("")
            for _ in range(reps):
                f()
            torch.cuda.synchronize()
            ms_, cnt_ = c2.profile_read("")
            c2.profile(False)
            return ms_ / cnt_
        conv["reduce_mw_ms"] = tk(lambda: rg.rns_reduce_mw(c2, out, prime_begin=0, L=L, out=back))
        if not torch.equal(back, rc):
            print("bench.py: multiword reduction did not give the residues back", file=sys.stderr)
            sys.exit(1)
        other = torch.empty_like(rc)
        conv["base_convert_exact_ms"] = tk(lambda: rg.base_convert(c2, rc, 0, L, L, L=L, out=other))
        # the same integers' residues mod the other primes, from the 10 words
        want = torch.empty_like(rc)
        rg.rns_reduce_mw(c2, out, prime_begin=L, L=L, out=want)
        torch.cuda.synchronize()
        if not torch.equal(other, want):
            print("bench.py: base conversion differs from reduction of the CRT output", file=sys.stderr)
            sys.exit(1)
        Mb = 1
        for p in c2.primes[:L]:
            Mb *= p
        bound = Mb // 2 - (Mb >> 38)
        conv["base_convert_one_pass_ms"] = tk(lambda: rg.base_convert(c2, rc, 0, L, L, L=L, bound=bound, out=other))
        torch.cuda.synchronize()
        if not torch.equal(other, want):          # full-range values stay within that bound but for 2^-38 of M
            conv["one_pass_note"] = "full-range inputs exceed the promised bound in a few entries"
        conv["bytes_per_entry"] = {"reduce_mw": 8 * W + 4 * L, "convert": 8 * L}
        conv["reduce_mw_GBps"] = n * n * (8 * W + 4 * L) / (conv["reduce_mw_ms"] * 1e-3) / 1e9
        conv["base_convert_one_pass_GBps"] = n * n * 8 * L / (conv["base_convert_one_pass_ms"] * 1e-3) / 1e9
    finally:
        c2.close()
    return {"workload": "full-range residues uniform in [0, p_j) per plane (seeded), %dx%d, %d primes, INT8 path, "
                        "exact CRT (matrix-core Lagrange form) into %d words" % (n, n, L, W),
            "conversions": conv,
            "ms_per_step": 1000 * t, "value": ops / t, "unit": "int-ops/s", "kernels": kern,
            "gemm_mfma_tops": 16.0 * ops / (kern["k_gemm"]["avg_ms"] * 1e-3) / 1e12, "sampled_entries_checked": 4}


SERVING_FRACS = (0.25, 0.5, 0.75, 1.0, 1.25)


def run_serving(rg, count, fracs=SERVING_FRACS):
    """Closed-loop capacity, then open-loop Poisson arrivals at each fraction
    of it, each point with the n = 10007 tail at its 50th arrival;
    latency = completion - arrival.  Every served result is a divisor chain
    certified by the library; a sample is solved again alone and compared."""
    import numpy as np
    workers = 4
    out = {"workers": workers}
    srv = rg.Server(device=0, workers=workers)
    warm = _serving_stream(12, 1.0, seed=7, tail=False)
    for _, a, kind in warm[:workers]:
        if kind != "singular":
            srv.wait(srv.submit(a))
    t0 = time.perf_counter()
    ts = [srv.submit(a, seed=i) for i, (_, a, kind) in enumerate(warm) if kind != "singular"]
    for t in ts:
        srv.wait(t)
    cap = len(ts) / (time.perf_counter() - t0)
    out["closed_loop_solves_per_s"] = cap
    points = []
    solved = []
    for i, frac in enumerate(fracs):
        rate = frac * cap
        reqs = _serving_stream(count, rate, seed=11 + i, tail=count > 50)
        start = time.perf_counter()
        tickets = []
        for r, a, kind in reqs:
            d = start + r.arrival - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets.append(srv.submit(a, seed=1))
            if len(tickets) % 50 == 0:
                print("[serving] %.2fx capacity: %d submitted" % (frac, len(tickets)), file=sys.stderr, flush=True)
        lat, queue, service, ok, bad, tail_rec, paths, exact = [], [], [], 0, 0, None, [0, 0], 0
        ops, cpu = [], []
        intervals = []
        for t, (r, a, kind) in zip(tickets, reqs):
            st, res, info = srv.wait(t)
            if info["t_start"] > 0 and info["t_end"] >= info["t_start"]:
                intervals.append((info["t_start"], info["t_end"]))
            if kind == "singular":
                bad += int(st == 6)
                continue
            if st != 0 or any(res.s[i + 1] % res.s[i] for i in range(len(res.s) - 1)):
                raise SystemExit("bench.py: served Smith form failed (status %d, n %d)" % (st, r.n))
            ok += 1
            paths[res.stats["path"]] += 1
            exact += res.stats["cert_exact"]
            rec = (info["t_end"] - info["t_submit"], info["t_start"] - info["t_submit"],
                   info["t_end"] - info["t_start"])
            if r.n == 10007:                     # also counted in the percentiles below
                tail_rec = {"n": r.n, "latency_s": rec[0], "queue_s": rec[1], "service_s": rec[2],
                            "stats": res.stats, "largest_invariant_bits": res.s[-1].bit_length()}
            lat.append(rec[0])
            queue.append(rec[1])
            service.append(rec[2])
            ops.append(res.stats["residue_ops"])
            cpu.append(res.stats["t_host_cpu"])
            if len(solved) < 6 and r.n <= 1500:
                solved.append((a, res.s))
        span = time.perf_counter() - start
        # Share of the point's span with at least one request running on the
        # device (union of the [start, end] intervals of every request).
        busy, cur_a, cur_b = 0.0, None, None
        for a_, b_ in sorted(intervals):
            if cur_b is None or a_ > cur_b:
                if cur_b is not None:
                    busy += cur_b - cur_a
                cur_a, cur_b = a_, b_
            else:
                cur_b = max(cur_b, b_)
        if cur_b is not None:
            busy += cur_b - cur_a
        print("[serving] %.2fx capacity: %d requests in %.1f s" % (frac, count, span), file=sys.stderr, flush=True)
        points.append({"rate_frac_of_capacity": frac, "arrival_rate": rate, "requests": count,
                       "solves_per_s": ok / span, "p50_latency_s": float(np.percentile(lat, 50)),
                       "p99_latency_s": float(np.percentile(lat, 99)),
                       "p50_queue_s": float(np.percentile(queue, 50)),
                       "p99_queue_s": float(np.percentile(queue, 99)),
                       "p50_service_s": float(np.percentile(service, 50)),
                       "p99_service_s": float(np.percentile(service, 99)),
                       "max_latency_s": float(np.max(lat)),
                       "residue_int_ops_per_request": {"mean": float(np.mean(ops)),
                                                       "p50": float(np.percentile(ops, 50)),
                                                       "p99": float(np.percentile(ops, 99))},
                       "residue_int_ops_per_s": float(np.sum(ops)) / span,
                       "host_cpu_s_per_request": {"mean": float(np.mean(cpu)),
                                                  "p50": float(np.percentile(cpu, 50)),
                                                  "p99": float(np.percentile(cpu, 99))},
                       "singular_rejected": bad, "paths_residue_lifting": paths,
                       "busy_frac": busy / span if span > 0 else None,
                       "exact_certificates": exact, "tail": tail_rec})
    st = srv.stats()
    srv.close()
    # alone versus in the mix
    with rg.Context(device=0, L=24) as ctx:
        for a, s_mix in solved:
            if rg.smith_form(ctx, a, seed=3).s != s_mix:
                raise SystemExit("bench.py: a served Smith form differs from the same request solved alone")
    out["points"] = points
    out["alone_vs_mix_checked"] = len(solved)
    out["max_running"] = st["max_running"]
    out["hbm_high_water_bytes"] = st["high_water"]
    out["workload"] = ("Poisson arrivals; n log-uniform in [100, 4000], entries uniform in [-2^10, 2^10] "
                       "(seeded synthetic stand-ins), n = 10007 tail at the 50th arrival of each point "
                       "(counted in the latency percentiles; also broken out as `tail`), one singular "
                       "request per point; %d requests per point; latency = completion - arrival" % count)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this library runs on one GPU only (--gpus 1); how the products and "
              "Smith-form requests would shard over several GPUs is designed but not built",
              file=sys.stderr)
        sys.exit(2)
    bg = None
    if not args.only and args.smith:
        # single-core oracle timings in a child forked before the GPU is
        # touched; it runs while the GPU products below are timed
        import multiprocessing as mp
        ctx_mp = mp.get_context("fork")
        parent, child = ctx_mp.Pipe(duplex=False)
        bg = (ctx_mp.Process(target=_oracle_timings, args=(child, args.n, args.primes, args.cpu_rows_1core)),
              parent)
        bg[0].start()
    import numpy as np
    import torch

    import paper_2605_19254_amd as rg
    import synth

    n, L = args.n, args.primes
    dev = torch.device("cuda:0")
    if args.copy_bytes > 0:
        src = torch.empty(args.copy_bytes // 4, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only == "unimodular":
        print(json.dumps(run_unimodular(rg, args.unimodular_n)), flush=True)
        return
    if args.only == "batched":
        print(json.dumps(run_batched(rg, torch, dev, args.batched, args.batched_steps)), flush=True)
        return
    if args.only == "smith":
        print(json.dumps(run_smith(rg)), flush=True)
        return
    if args.only == "serving":
        print(json.dumps(run_serving(rg, args.serving)), flush=True)
        return
    if args.only == "lifting":
        print(json.dumps(run_lifting(rg, args.lifting_n)), flush=True)
        return
    if args.only in ("smith64", "planted2000"):
        print(json.dumps(run_smith_one(rg, args.only)), flush=True)
        return
    if args.only == "massager":
        print(json.dumps(run_massager(rg, args.massager_max or 1009)), flush=True)
        return
    if args.only == "stress":
        with rg.Context(device=0, L=args.primes) as c:
            print(json.dumps(run_stress(rg, torch, dev, c, args.n, args.primes)), flush=True)
        return
    a_np, b_np = synth.square_pair(n=n, bound=1 << 20, seed_a=0, seed_b=1)
    A = torch.from_numpy(a_np).to(dev)
    B = torch.from_numpy(b_np).to(dev)
    ctx = rg.Context(device=0, L=L)
    ra = torch.empty((L, n, n), dtype=torch.int32, device=dev)
    rb = torch.empty((L, n, n), dtype=torch.int32, device=dev)
    rc = torch.empty((L, n, n), dtype=torch.int32, device=dev)
    out = torch.empty((n, n, 1), dtype=torch.int64, device=dev)
    bound = n * (1 << 40)          # |C_ij| <= k * 2^20 * 2^20
    prob = [rg.GemmProblem(ra, rb, rc)]

    def step(path):
        rg.rns_reduce(ctx, A, L=L, out=ra)
        rg.rns_reduce(ctx, B, L=L, out=rb)
        rg.modmatmul_batched(ctx, prob, path=path)
        rg.crt_reconstruct(ctx, rc, L=L, W=1, bound=bound, out=out)

    plans = {}

    def plan_step(path):
        # The same product through a whole-product plan: one conversion
        # launch reduces A and B straight into the GEMM's tiled operands.
        if path not in plans:
            plans[path] = rg.MatmulPlan(ctx, [rg.MatmulProblem(A, B, out.view(n, n), prime_begin=0, L=L,
                                                               bound=bound)], path=path)
        plans[path].execute()

    def timed(path, steps, warmup, step=step):
        for _ in range(warmup):
            step(path)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read("")          # drop warm-up records
        torch.cuda.synchronize()
        # Events on the stream the library launches on (torch's current
        # stream) bracket every step; the wall clock brackets all of them.
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record()
        for i in range(steps):
            step(path)
            ev[i + 1].record()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.profile(False)
        kern = {}
        for name in ("k_reduce", "k_prep", "k_gemm", "k_crt"):
            ms, cnt = ctx.profile_read(name)
            if cnt:
                kern[name] = {"avg_ms": ms / cnt, "launches": cnt}
        per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
        kern["step_ms"] = {"median": per[len(per) // 2], "min": per[0], "max": per[-1]}
        return t, kern

    res_ops = 2.0 * n * n * n * L
    t8, k8 = timed("int8", args.steps, args.warmup)
    # correctness of what was timed: sampled entries against the oracle's exact product
    from oracle import native
    rows = np.array([0, n // 3, n - 1])
    got = out[torch.from_numpy(rows).to(dev), :, 0].cpu().numpy()
    want = native.exact_matmul(a_np[rows], b_np)
    if not np.array_equal(got, want):
        print("bench.py: INT8 path result differs from the oracle", file=sys.stderr)
        sys.exit(1)
    assert ctx.status() == 0
    ms_calls = 1000.0 * t8 / args.steps
    calls_rec = {"ms_per_step": ms_calls, "value": res_ops / (ms_calls * 1e-3), "kernels": k8,
                 "workload": "the same product as four boundary calls per step: rns_reduce (A), rns_reduce (B), "
                             "modmatmul_batched, crt_reconstruct",
                 "reduce_GBps": n * n * (8 + 4.0 * L) / (k8["k_reduce"]["avg_ms"] * 1e-3) / 1e9}
    # The headline: the whole-product plan on the same inputs.
    out.fill_(0)
    tp, kp = timed("int8", args.steps, args.warmup, step=plan_step)
    got = out[torch.from_numpy(rows).to(dev), :, 0].cpu().numpy()
    if not np.array_equal(got, want) or ctx.status() != 0:
        print("bench.py: whole-product plan result differs from the oracle", file=sys.stderr)
        sys.exit(1)
    ms8 = 1000.0 * tp / args.steps
    gemm_ms = kp["k_gemm"]["avg_ms"]
    mfma_ops = 16.0 * res_ops                       # executed INT8 MFMA ops per launch
    achieved = mfma_ops / (gemm_ms * 1e-3) / 1e12    # TOP/s
    probe = rg.GemmPlan(ctx, prob, path="int8")
    kernel = I8_KERNEL_NAMES.get(probe.info()["variant"], "k_gemm_i8")
    probe.close()
    ceiling = None
    if args.calibrate_iters > 0:
        # Sustained rate of the same MFMA instruction with random register
        # operands and no memory traffic: the ceiling this part holds under
        # the power draw of real data (the published peak assumes full clock).
        rate, cal_ms = ctx.calibrate("i8_16x16x64", iters=args.calibrate_iters, random_operands=True)
        ceiling = {"value": rate / 1e12, "unit": "TOP/s", "frac": achieved / (rate / 1e12),
                   "probe": "rns_calibrate kind 0: v_mfma_i32_16x16x64_i8, 8 waves/CU, random "
                            "register operands, %d iterations, %.1f ms" % (args.calibrate_iters, cal_ms)}

    fp64 = None
    if args.fp64_steps > 0:
        out.fill_(0)
        t64, k64 = timed("fp64", args.fp64_steps, 1, step=plan_step)
        got = out[torch.from_numpy(rows).to(dev), :, 0].cpu().numpy()
        if not np.array_equal(got, want):
            print("bench.py: FP64 path result differs from the oracle", file=sys.stderr)
            sys.exit(1)
        ms64 = 1000.0 * t64 / args.fp64_steps
        g64 = k64["k_gemm"]["avg_ms"]
        fp64 = {"value": res_ops / (ms64 * 1e-3), "ms_per_step": ms64, "steps": args.fp64_steps,
                "kernels": k64, "gemm_tflops": res_ops / (g64 * 1e-3) / 1e12,
                "gemm_frac_of_fp64_peak": res_ops / (g64 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}

    for pl in plans.values():
        pl.close()
    conv_bytes = 2.0 * n * n * (8 + 4 * L)          # int64 A and B in, one digit byte x 4 per prime out
    crt_bytes = n * n * (4.0 * L + 8)
    rec = {
        "metric": METRIC,
        "value": res_ops / (ms8 * 1e-3),
        "unit": "int-ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms8,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "exact multi-modular GEMM, A and B %dx%d int64 uniform in "
                               "[-2^20, 2^20] (seeds 0, 1), %d primes below 2^26, INT8-limb path; one "
                               "whole-product plan execution per step: int64 A and B reduced mod every "
                               "prime into the tiled digit operands (one launch), the %d residue products "
                               "(one GEMM launch), Lagrange CRT to int64 (one launch)" % (n, n, L, L),
                   "m": n, "n": n, "k": n, "primes": L, "path": "int8"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_INT8_TOPS,
                     "unit": "TOP/s", "frac": achieved / PEAK_INT8_TOPS,
                     "traffic": recorded_traffic(kernel),
                     "kernel": kernel, "avg_launch_ms": gemm_ms,
                     "ops_per_launch": mfma_ops, "measured_ceiling": ceiling},
        "kernels": kp,
        "device": {"name": torch.cuda.get_device_name(0), "host_cores": os.cpu_count()},
        "hbm_passes": {
            "conversion_GBps": conv_bytes / (kp["k_prep"]["avg_ms"] * 1e-3) / 1e9,
            "crt_GBps": crt_bytes / (kp["k_crt"]["avg_ms"] * 1e-3) / 1e9,
            "peak_GBps": PEAK_HBM_GBS},
        "fp64_path": fp64,
        "boundary_calls": calls_rec,
        "int8_vs_fp64_speedup": (fp64["ms_per_step"] / ms8) if fp64 else None,
    }
    print("[bench] headline and FP64 path done", file=sys.stderr, flush=True)
    rec["stress"] = run_stress(rg, torch, dev, ctx, n, L) if args.stress else None
    print("[bench] full-range stress done", file=sys.stderr, flush=True)
    rec["batched"] = run_batched(rg, torch, dev, args.batched, args.batched_steps) if args.batched > 0 else None
    print("[bench] batched done", file=sys.stderr, flush=True)
    oracle_bg = None
    if bg is not None:
        print("[bench] waiting for the single-core oracle timings", file=sys.stderr, flush=True)
        oracle_bg = bg[1].recv()
        bg[0].join()
    rec["smith"] = run_smith(rg, oracle_bg=oracle_bg) if args.smith else None
    print("[bench] smith done", file=sys.stderr, flush=True)
    rec["serving"] = run_serving(rg, args.serving) if args.serving > 0 else None
    print("[bench] serving done", file=sys.stderr, flush=True)
    rec["massager"] = run_massager(rg, args.massager_max) if args.massager_max > 0 else None
    rec["unimodular"] = run_unimodular(rg, args.unimodular_n) if args.unimodular_n > 0 else None
    print("[bench] massager done", file=sys.stderr, flush=True)
    if args.cpu_rows > 0:
        primes = ctx.primes[:L]
        rec["cpu_baseline"] = cpu_baseline(a_np, b_np, primes, args.cpu_rows)
        if oracle_bg and "headline_1core" in oracle_bg:
            rec["cpu_baseline"]["single_core"] = oracle_bg["headline_1core"]
    else:
        rec["cpu_baseline"] = None
    line = json.dumps(rec)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    ctx.close()


if __name__ == "__main__":
    main()
