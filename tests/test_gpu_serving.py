"""Serving engine: concurrent Smith-form requests on one GPU.  Every result
served in the mix equals the result of the same request alone, and equals the
oracle or the planted invariants; a singular request fails alone; admission
respects the device-memory budget."""
import json
import os
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


def _mix():
    reqs = []
    for n, sd in [(40, 1), (150, 2), (300, 3), (90, 4)]:
        pl = synth.planted_smith(n, seed=sd)
        reqs.append((pl.a, pl.s))
    for n, sd in [(12, 5), (24, 6), (31, 7)]:
        a = synth.small_smith(seed=sd, n=n, bound=1 << 10)
        reqs.append((a, osmith.smith_form(a)))
    # requests whose invariants are too large for the residue path: the p-adic
    # lifting path (its lifting graphs are captured while other requests run);
    # expected values are the oracle's, stored by tests/golden/make_smith_golden.py
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "smith_lifting.json")))
    for case in gold["cases"]:
        if case["gen"] == "small_smith" and case["n"] in (80, 120):
            a = synth.small_smith(seed=case["seed"], attempt=case["attempt"], n=case["n"], bound=case["bound"])
            reqs.append((a, [1] * case["ones"] + [int(v) for v in case["tail"]]))
    sing = np.array([[1, 2, 3, 4, 5]] * 5, dtype=np.int64) + np.arange(5)[:, None]
    sing[4] = sing[0] + sing[1] - sing[2]     # dependent row
    reqs.insert(3, (sing, None))
    return reqs


def test_mix_equals_alone(rg):
    _say("serving mix")
    reqs = _mix()
    srv = rg.Server(device=0, workers=4)
    tickets = [srv.submit(a, seed=i) for i, (a, _) in enumerate(reqs)]
    results = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    with rg.Context(device=0, L=24) as ctx:
        for (a, want), (st, res, info) in zip(reqs, results):
            if want is None:
                assert st == 6 and res is None
                continue
            assert st == 0, info
            assert res.s == want
            assert res.stats["cert_exact"] == 1
            alone = rg.smith_form(ctx, a, seed=99)
            assert alone.s == res.s
            assert info["t_end"] >= info["t_start"] >= info["t_submit"] - 1e-6
    assert stats["max_running"] >= 2
    assert stats["high_water"] <= stats["budget"]
    assert sum(1 for (_, w), (st, r, _) in zip(reqs, results) if r is not None and r.stats["path"] == 1) >= 2


def test_admission_by_footprint(rg):
    _say("serving admission")
    n = 200
    fp = rg.server_footprint(n)
    srv = rg.Server(device=0, workers=4, hbm_budget=int(1.5 * fp))
    pls = [synth.planted_smith(n, seed=s) for s in range(4)]
    tickets = [srv.submit(p.a, seed=i) for i, p in enumerate(pls)]
    out = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    assert stats["max_running"] == 1          # only one request fits the budget
    for p, (st, res, info) in zip(pls, out):
        assert st == 0 and res.s == p.s
    starts = sorted(info["t_start"] for _, _, info in out)
    ends = sorted(info["t_end"] for _, _, info in out)
    assert all(starts[i + 1] >= ends[i] - 1e-6 for i in range(3))   # no overlap


def test_wait_timeout_and_bad_ticket(rg):
    _say("serving wait")
    srv = rg.Server(device=0, workers=1)
    pl = synth.planted_smith(400, seed=9)
    t = srv.submit(pl.a)
    st, res, _ = srv.wait(t, timeout=0.0)
    assert st in (0, 9)                        # done or still running
    if st == 9:
        st, res, _ = srv.wait(t)
    assert st == 0 and res.s == pl.s
    st, res, _ = srv.wait(t)                   # waited once already
    assert st == 1
    srv.close()
