"""GPU parity of shot-list runs: the overflow re-run (shots a capped run
flagged OVERFLOW, sampled again without the cap) and lists in any order over
a mixture's ranges."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from paper_2512_23037_amd import soft
from tests.gpu_helpers import coeff_error, make_ctx, torch

pytestmark = pytest.mark.gpu


def _run_list(ctx, shots):
    t = torch()
    idx = t.from_numpy(np.asarray(shots, dtype=np.int64)).cuda()
    n = len(shots)
    nw = ctx.info()["record_words"]
    outs = [t.zeros((nw, n), dtype=t.int32, device="cuda")] + [t.zeros(n, dtype=t.int32, device="cuda") for _ in range(3)]
    ctx.run_list(idx, *outs)
    t.cuda.synchronize()
    return {k: x.cpu().numpy().view(np.uint32) for k, x in zip(("outcomes", "status", "abort_op", "obs"), outs)}


def _run_range(ctx, shot0, n):
    t = torch()
    nw = ctx.info()["record_words"]
    outs = [t.zeros((nw, n), dtype=t.int32, device="cuda")] + [t.zeros(n, dtype=t.int32, device="cuda") for _ in range(3)]
    ctx.run(shot0, n, *outs)
    t.cuda.synchronize()
    return {k: x.cpu().numpy().view(np.uint32) for k, x in zip(("outcomes", "status", "abort_op", "obs"), outs)}


def test_overflow_rerun_without_the_cap():
    w = workloads.config("cultivation_15q", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 50_000
    ctx = make_ctx(w.text, w.noise, seed=41, cap=8)
    capped = _run_range(ctx, 0, N)
    over = np.nonzero(capped["status"] == soft.OVERFLOW)[0]
    assert len(over) > 100
    ref_capped = circ.batch(41, 0, N, cap=8)
    assert (capped["status"] == ref_capped["status"]).all()
    # the re-run: same shot indices, no cap, kept states for a few of them
    ctx.set_caps(0)
    lo = int(over[0])
    ctx.set_keep(lo, 4096)
    again = _run_list(ctx, over)
    assert (again["status"] != soft.OVERFLOW).all()
    full = circ.batch(41, 0, N)
    for key in ("status", "abort_op", "obs"):
        assert (again[key] == full[key][over]).all(), key
    assert (again["outcomes"] == full["outcomes"][:, over]).all()
    kept = [int(x) for x in over if x < lo + 4096][:20]
    assert len(kept) >= 5
    for shot in kept:
        r = circ.shot(41, int(shot))
        x, z, rr = ctx.read_tableau(int(shot))
        assert (x == r.tab_x).all() and (z == r.tab_z).all() and (rr == r.tab_r).all()
        assert coeff_error(ctx.read_coeffs(int(shot)), r.coeffs) < 1e-10


def test_shot_list_any_order_over_a_mixture():
    m = workloads.mixture(seed=1, total_shots=27 * 2000)
    ctx = soft.Context(0)
    ctx.load_mixture([w.text for w in m["workloads"]], m["models"], m["shot_ends"])
    ctx.set_rng(99)
    rng = np.random.default_rng(4)
    shots = rng.choice(27 * 2000, size=3000, replace=False)       # unsorted, across all ranges
    got = _run_list(ctx, shots)
    circs = {}
    for i, shot in enumerate(shots):
        v = ctx.variant_of(int(shot))
        if v not in circs:
            circs[v] = oracle.Circuit(m["workloads"][v].text, m["models"][v])
        r = circs[v].shot(99, int(shot))
        assert got["status"][i] == r.status and got["abort_op"][i] == r.abort_op, (shot, v)
        rec = [int((got["outcomes"][k >> 5, i] >> (k & 31)) & 1) for k in range(circs[v].n_records)]
        assert rec == r.record, (shot, v)
    c = ctx.counters()
    assert c["shots"] == len(shots)
    per = [ctx.counters(v)["shots"] for v in range(27)]
    ends = [0] + m["shot_ends"]
    want = [int(((shots >= ends[v]) & (shots < ends[v + 1])).sum()) for v in range(27)]
    assert per == want


def test_shot_list_equals_range_run():
    w = workloads.config("cultivation_42q", seed=1)
    ctx = make_ctx(w.text, w.noise, seed=3, bits=32)
    a = _run_range(ctx, 1000, 20000)
    b = _run_list(ctx, np.arange(1000, 21000))
    for key in a:
        assert (a[key] == b[key]).all(), key
