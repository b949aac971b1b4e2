"""Writes tests/golden/smith_lifting.json: Smith forms of seeded inputs that
take the p-adic lifting path, computed by the oracle only (Bareiss
determinant and gcd elimination modulo it).  Each case names its generator
in synth/ and its parameters; a planted case is also checked against the
invariants it was built with.  With --vandermonde it writes
tests/golden/smith_vandermonde.json instead: the Smith forms (and |det A|)
of the Section 4.1 family A_ij = i^j mod n for n = 101, 199, 211, 307 and 503,
by the same oracle (or for the sizes given after the flag, replacing those
cases and keeping the others).  Run from the repository root:
    python tests/golden/make_smith_golden.py [--vandermonde [n ...]]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import smith as osmith  # noqa: E402
import synth  # noqa: E402

CASES = [
    {"gen": "small_smith", "n": 80, "seed": 11, "bound": 1024},
    {"gen": "small_smith", "n": 120, "seed": 12, "bound": 1024},
    {"gen": "small_smith", "n": 160, "seed": 13, "bound": 1024},
    {"gen": "small_smith", "n": 240, "seed": 14, "bound": 1024},
    {"gen": "small_smith", "n": 320, "seed": 15, "bound": 1024},
    {"gen": "planted_small", "n": 48, "seed": 3},
    {"gen": "planted_small", "n": 96, "seed": 4},
]


def build(case):
    if case["gen"] == "small_smith":
        attempt = 0
        while True:
            a = synth.small_smith(seed=case["seed"], attempt=attempt, n=case["n"], bound=case["bound"])
            if osmith.bareiss_det(a) != 0:
                return a, attempt
            attempt += 1
    pl = synth.planted_small(case["n"], seed=case["seed"])
    return pl.a, 0


def main():
    out = []
    for case in CASES:
        t = time.time()
        a, attempt = build(case)
        s = osmith.smith_form(a)
        if case["gen"] == "planted_small":
            assert s == synth.planted_small(case["n"], seed=case["seed"]).s, case
        ones = sum(1 for v in s if v == 1)
        rec = dict(case, attempt=attempt, ones=ones, tail=[str(v) for v in s[ones:]],
                   max_abs=int(abs(a).max()))
        out.append(rec)
        print(case, "ones", ones, "nontrivial", len(s) - ones, "bits", s[-1].bit_length(),
              "%.1fs" % (time.time() - t), flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "smith_lifting.json"), "w") as f:
        json.dump({"source": "oracle.smith.smith_form on synth inputs (tests/golden/make_smith_golden.py)",
                   "cases": out}, f, indent=1)


def main_vandermonde(sizes):
    path = os.path.join(ROOT, "tests", "golden", "smith_vandermonde.json")
    kept = []
    if os.path.exists(path):       # cases of other sizes stay as stored
        with open(path) as f:
            kept = [c for c in json.load(f)["cases"] if c["n"] not in sizes]
    out = []
    for n in sizes:
        t = time.time()
        a = synth.vandermonde_mod(n)
        s = osmith.smith_form(a)
        det = abs(osmith.bareiss_det(a))
        prod = 1
        for v in s:
            prod *= v
        assert prod == det and osmith.is_divisor_chain(s), n
        ones = sum(1 for v in s if v == 1)
        out.append({"n": n, "ones": ones, "tail": [str(v) for v in s[ones:]], "det_abs": str(det)})
        print("vandermonde", n, "ones", ones, "bits", s[-1].bit_length(), "%.1fs" % (time.time() - t), flush=True)
    out = sorted(kept + out, key=lambda c: c["n"])
    with open(path, "w") as f:
        json.dump({"source": "oracle.smith.smith_form on synth.vandermonde_mod (tests/golden/make_smith_golden.py "
                             "--vandermonde)", "cases": out}, f, indent=1)


if __name__ == "__main__":
    if "--vandermonde" in sys.argv:
        # sizes after the flag, else the stored set (n = 503 takes the oracle
        # over an hour)
        sizes = [int(a) for a in sys.argv[sys.argv.index("--vandermonde") + 1:]] or [101, 199, 211, 307, 503]
        main_vandermonde(sizes)
    else:
        main()
