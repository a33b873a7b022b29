"""Deferred T runs (soft_set_deferred_t): a run of T gates with no noise
between them, followed by events that read only the tableau signs, is
skipped; a shot whose check fails before any event reads the coefficients
never needs it; a shot that does need it applies the run late, at the event
that needs it, with the tableau signs the run saw, and a shot whose final
state is kept and still has a run skipped runs again with every run
applied.  Records, statuses, abort ops,
observables, kept final states and pass / discard / logical counts are
identical with deferral on and off, with and without checkpoints, in both
precisions and noise draws; the oracle agrees with it on."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from paper_2512_23037_amd import soft
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import compare_batch, compare_kept, make_ctx, run_gpu

pytestmark = pytest.mark.gpu

SAME = ("shots", "passed", "discarded", "overflow", "numeric", "logical_errors")


def _on_off(build, N, kept=64):
    res = []
    for on in (True, False):
        ctx = build()
        ctx.set_deferred_t(on)
        ctx.set_keep(0, kept)
        out = run_gpu(ctx, 0, N)
        res.append((out, ctx.counters(), [ctx.read_coeffs(s) for s in range(kept)],
                    [ctx.read_tableau(s) for s in range(kept)]))
        ctx.close()
    (a, ca, ka, ta), (b, cb, kb, tb) = res
    for k in ("status", "abort_op", "obs", "outcomes"):
        assert (a[k] == b[k]).all(), k
    for f in SAME:
        assert ca[f] == cb[f], f
    assert ka == kb
    for x, y in zip(ta, tb):
        assert all((u == w).all() for u, w in zip(x, y))
    assert cb["redo_shots"] == 0
    return ca, cb


@pytest.mark.parametrize("bits,mode,prefix", [(32, 1, True), (64, 1, True), (32, 0, False), (64, 0, True),
                                               (32, 1, False)])
def test_defer_on_off_42q(bits, mode, prefix):
    w = workloads.config("cultivation_42q", seed=1)

    def build():
        ctx = make_ctx(w.text, w.noise, seed=20251223, bits=bits)
        ctx.set_noise_mode(mode)
        ctx.set_shared_prefix(prefix)
        return ctx

    on, off = _on_off(build, 400_000, kept=128)
    # shots with a fault before the first T layer skip it and most end at the
    # first check round; the others apply it late
    assert on["redo_shots"] > 0
    assert on["entries_t"] < off["entries_t"]


def test_defer_on_off_15q_both_lists_and_oracle():
    w = workloads.config("cultivation_15q", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 300_000
    for spec in (True, False):
        def build():
            ctx = make_ctx(w.text, w.noise, seed=7)
            ctx.set_speculation(spec)
            return ctx
        _on_off(build, N)
    ctx = make_ctx(w.text, w.noise, seed=7, keep=(0, 256))
    gpu = run_gpu(ctx, 0, N)
    compare_batch(gpu, circ.batch(7, 0, N))
    compare_kept(ctx, circ, 7, range(256))


@pytest.mark.parametrize("seed", range(6))
def test_defer_random_circuits_explicit_words(seed):
    # T gates followed by outcome-fixed measurements and checks, under dense
    # noise: deferred runs, runs applied late, redone kept attempts and kept
    # states against the oracle
    n = 4 + seed % 3
    text, _ = random_circuit(91000 + seed, n, 120, p_t=0.2, p_meas=0.15)
    lines = text.strip().split("\n")
    out = [lines[0]]
    for i, line in enumerate(lines[1:]):
        out.append(line)
        if line.startswith("M ") and i % 3 == 0:
            out.append("DETECTOR 0 %d" % (sum(1 for x in out if x.startswith(("M ", "MPP", "MX", "MR "))) - 1))
    text = "\n".join(out) + "\n"
    noise = {"p1": 0.01, "p2": 0.01, "p_meas": 0.01}
    circ = oracle.Circuit(text, noise)
    N = 2048
    words = random_words(seed, N * circ.words_per_shot).reshape(N, circ.words_per_shot)
    res = []
    for on in (True, False):
        ctx = make_ctx(text, noise, keep=(0, 128))
        ctx.set_deferred_t(on)
        gpu = run_gpu(ctx, 0, N, words)
        compare_batch(gpu, circ.batch(0, 0, N, words=words))
        compare_kept(ctx, circ, 0, range(128), words=words)
        res.append(gpu)
    for k in ("status", "abort_op", "obs", "outcomes"):
        assert (res[0][k] == res[1][k]).all()


def test_defer_mixture_noalloc_and_split():
    import torch
    m = workloads.mixture(seed=1, total_shots=270_000)

    def build_mix():
        ctx = soft.Context(0)
        ctx.load_mixture([w.text for w in m["workloads"]], m["models"], m["shot_ends"])
        ctx.set_rng(3)
        ctx.set_precision(64)
        return ctx

    _on_off(build_mix, 270_000)
    w = workloads.config("cultivation_42q_k12", seed=1)

    def build_split():
        ctx = make_ctx(w.text, w.noise, seed=11, bits=32)
        ctx.set_noise_mode(1)
        ctx.set_tile_memory(3)
        return ctx

    on, _ = _on_off(build_split, 300_000)
    assert on["redo_shots"] > 0
    ctx = build_split()
    ref = run_gpu(ctx, 0, 300_000)
    st = torch.zeros(300_000, dtype=torch.int32, device="cuda")
    ctx.run_noalloc(0, 300_000, None, st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy().view(np.uint32) == ref["status"]).all()


def test_defer_off_with_cap():
    # a support cap is checked on every T: no run is deferred
    w = workloads.config("cultivation_15q", seed=1)
    ctx = make_ctx(w.text, w.noise, seed=5, cap=8)
    run_gpu(ctx, 0, 100_000)
    assert ctx.counters()["redo_shots"] == 0
