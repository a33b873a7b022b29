"""Checkpoints of the noiseless trajectory (soft_set_shared_prefix): up to
the first random measurement every event is deterministic in a shot that no
noise has hit, so such a shot is in the same state as every other at each
checkpoint; the run builds those states once and a shot starts at the last
checkpoint before its first hit, loading the tile only if an event reads it.
With it on and off every output is identical bit for bit -- records,
statuses, abort ops, observables, kept final states, pass / discard /
logical counts, support histograms and the norm check -- in both precisions,
both noise draws, explicit words, mixtures, caps and split tiles; and the
oracle agrees with it on (the other parity tests run with it on, the
default)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from paper_2512_23037_amd import soft
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import compare_batch, compare_kept, make_ctx, run_gpu

pytestmark = pytest.mark.gpu

SAME = ("passed", "discarded", "overflow", "numeric", "logical_errors", "restarts", "noise_slots")


def _on_off(build, N, kept=64, shot0=0):
    res = []
    for on in (True, False):
        ctx = build()
        ctx.set_shared_prefix(on)
        ctx.set_deferred_t(False)  # (deferred T runs change the support histogram: tested apart)
        ctx.set_keep(shot0, kept)
        out = run_gpu(ctx, shot0, N)
        res.append((out, ctx.counters(), [ctx.read_coeffs(s) for s in range(shot0, shot0 + kept)]))
        ctx.close()
    (a, ca, ka), (b, cb, kb) = res
    for k in ("status", "abort_op", "obs", "outcomes"):
        assert (a[k] == b[k]).all(), k
    for f in SAME:
        assert ca[f] == cb[f], f
    assert ca["support_hist"] == cb["support_hist"]
    assert ca["max_norm_dev"] == cb["max_norm_dev"]
    assert ka == kb
    assert cb["prefix_shots"] == 0
    return ca, cb


@pytest.mark.parametrize("bits,mode", [(32, 1), (64, 1), (32, 0), (64, 0)])
def test_prefix_on_off_42q(bits, mode):
    w = workloads.config("cultivation_42q", seed=1)

    def build():
        ctx = make_ctx(w.text, w.noise, seed=20251223, bits=bits)
        ctx.set_noise_mode(mode)
        return ctx

    N = 400_000
    on, off = _on_off(build, N)
    # p = 1e-3 and 499 noise slots before the first T layer: about e^-0.5 of
    # the shots start from a checkpoint, and the kernel runs less T work
    frac = on["prefix_shots"] / N
    assert 0.5 < frac < 0.7, frac
    assert on["entries_t"] < off["entries_t"] and on["events"] < off["events"]


def test_prefix_on_off_15q_full_list_and_oracle():
    # speculation off: the prefix of the circuit-order list, and the oracle's
    # support histogram and counts with it on
    w = workloads.config("cultivation_15q", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 200_000

    def build():
        ctx = make_ctx(w.text, w.noise, seed=7)
        ctx.set_speculation(False)
        return ctx

    on, _ = _on_off(build, N)
    assert on["prefix_shots"] > 0
    ref = circ.batch(7, 0, N)
    ctx = build()
    ctx.set_deferred_t(False)
    ctx.set_keep(0, 128)
    compare_batch(run_gpu(ctx, 0, N), ref)
    compare_kept(ctx, circ, 7, range(128))
    hist = np.bincount(np.floor(np.log2(ref["max_support"])).astype(int), minlength=16)
    assert list(hist[:16]) == ctx.counters()["support_hist"]


def test_prefix_explicit_words_and_caps():
    text = ("QUBITS 6\n" + "".join("H %d\n" % q for q in range(6)) + "T 0\nT 1\nT 2\nTDG 3\nT 4\n"
            "CX 0 1\nT 1\nM 5\nMPP X0*X1\nT 2\nM 3\nTDG 1\nMPP Y2*Z4\n")
    noise = {"p1": 0.02, "p2": 0.02, "p_meas": 0.02, "p_mpp": 0.02}
    circ = oracle.Circuit(text, noise)
    N = 4000
    words = random_words(5, N * circ.words_per_shot).reshape(N, circ.words_per_shot)
    for cap in (0, 8, 16):
        res = []
        for on in (True, False):
            ctx = make_ctx(text, noise, cap=cap, keep=(0, 64))
            ctx.set_shared_prefix(on)
            res.append((run_gpu(ctx, 0, N, words), ctx.counters()))
            compare_batch(res[-1][0], circ.batch(0, 0, N, words=words, cap=cap if cap else 0xFFFFFFFF))
            compare_kept(ctx, circ, 0, range(64), words=words, cap=cap if cap else 0xFFFFFFFF)
        # a cap below the support 2^5 the T layer reaches makes the build
        # overflow before its checkpoint: no shot starts there, and every shot
        # overflows where the oracle's does
        assert (res[0][1]["prefix_shots"] > 0) == (cap == 0)
        for k in ("status", "abort_op", "outcomes"):
            assert (res[0][0][k] == res[1][0][k]).all()


@pytest.mark.parametrize("bits", [32, 64])
def test_checkpoints_long_shots_42q(bits):
    # p = 1e-4: most shots pass every check, so they start at deep
    # checkpoints (the last one is the list's end), some from the end
    # itself; kept states of such shots load the checkpoint's tile
    w = workloads.config("cultivation_42q", seed=1, p=1e-4)

    def build():
        ctx = make_ctx(w.text, w.noise, seed=99, bits=bits)
        ctx.set_noise_mode(1)
        return ctx

    N = 300_000
    on, off = _on_off(build, N, kept=256)
    assert on["prefix_shots"] > 0.8 * N
    assert on["entries_t"] < 0.5 * off["entries_t"]
    circ = oracle.Circuit(w.text, w.noise, noise_mode=1)
    ctx = build()
    ctx.set_keep(0, 128)
    gpu = run_gpu(ctx, 0, 4000)
    ref = circ.batch(99, 0, 4000, tau=1e-12 if bits == 64 else 1e-6)
    diff = (gpu["status"] != ref["status"]) | (gpu["outcomes"] != ref["outcomes"]).any(axis=0)
    assert diff.sum() <= (0 if bits == 64 else 3)
    compare_batch(gpu, ref, skip=diff)
    compare_kept(ctx, circ, 99, [s for s in range(128) if not diff[s]], tol=1e-10 if bits == 64 else 1e-5,
                 tau=1e-12 if bits == 64 else 1e-6)


def test_prefix_mixture_and_split_tiles():
    m = workloads.mixture(seed=1, total_shots=270_000)

    def build_mix():
        ctx = soft.Context(0)
        ctx.load_mixture([w.text for w in m["workloads"]], m["models"], m["shot_ends"])
        ctx.set_rng(3)
        ctx.set_precision(64)
        return ctx

    on, _ = _on_off(build_mix, 270_000)
    assert on["prefix_shots"] > 0
    w = workloads.config("cultivation_42q_k12", seed=1)

    def build_split():
        ctx = make_ctx(w.text, w.noise, seed=11, bits=32)
        ctx.set_noise_mode(1)
        ctx.set_tile_memory(3)
        return ctx

    on, _ = _on_off(build_split, 300_000)
    assert on["prefix_shots"] > 0


def test_prefix_noalloc_and_graph_replays():
    import torch
    w = workloads.config("cultivation_42q", seed=1)
    ctx = make_ctx(w.text, w.noise, seed=5, bits=32)
    ctx.set_noise_mode(1)
    ref = run_gpu(ctx, 0, 200_000)
    c_ref = ctx.counters()
    st = torch.zeros(200_000, dtype=torch.int32, device="cuda")
    ctx.run_noalloc(0, 200_000, None, st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy().view(np.uint32) == ref["status"]).all()
    assert ctx.counters()["prefix_shots"] == c_ref["prefix_shots"] > 0
    # replays of the captured graph (reset, prefix build, sampler) with eager
    # work between them give the same results every time
    for _ in range(3):
        again = run_gpu(ctx, 0, 200_000)
        torch.ones(1 << 20, device="cuda").sum().item()
        assert (again["status"] == ref["status"]).all()
    assert ctx.graph_info()["instantiations"] <= 2
