"""GPU parity with the coefficient tiles in device memory (HBM) instead of
LDS, and on the span-12 member of the 42-qubit family (support up to 2^12)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import compare_batch, compare_kept, make_ctx, run_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", range(6))
def test_memory_tiles_random_circuits(seed):
    n = 2 + seed
    text, _ = random_circuit(52000 + seed, n, 90)
    circ = oracle.Circuit(text)
    N = 256
    words = random_words(seed, N * circ.words_per_shot).reshape(N, circ.words_per_shot)
    ctx = make_ctx(text, keep=(0, N))
    ctx.set_tile_memory(2)
    assert ctx.launch_shape()["tiles_in_memory"] == 1
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


def test_memory_tiles_cultivation_15q():
    w = workloads.config("cultivation_15q", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 200_000
    ctx = make_ctx(w.text, w.noise, seed=21, keep=(0, 128))
    ctx.set_tile_memory(2)
    gpu = run_gpu(ctx, 0, N)
    compare_batch(gpu, circ.batch(21, 0, N))
    compare_kept(ctx, circ, 21, range(128))


@pytest.mark.parametrize("bits,tol", [(64, 1e-10), (32, 1e-5)])
def test_span12_both_tile_placements(bits, tol):
    w = workloads.config("cultivation_42q_k12", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 2000
    outs = {}
    for mode in (1, 2):
        ctx = make_ctx(w.text, w.noise, seed=13, bits=bits, keep=(0, 64))
        ctx.set_tile_memory(mode)
        assert ctx.info()["k_max"] == 12
        outs[mode] = run_gpu(ctx, 0, N)
        tau = 1e-12 if bits == 64 else 1e-6
        ref = circ.batch(13, 0, N, tau=tau)
        diff = (outs[mode]["status"] != ref["status"]) | (outs[mode]["outcomes"] != ref["outcomes"]).any(axis=0)
        # FP64 bit-exact; FP32 may flip an outcome whose draw is within 1e-5
        # of its probability (the guard band of the 42-qubit subset test)
        assert diff.sum() <= (0 if bits == 64 else 3)
        compare_batch(outs[mode], ref, skip=diff)
        worst = compare_kept(ctx, circ, 13, [s for s in range(64) if not diff[s]], tol=tol, tau=tau)
        print("bits %d mode %d worst %.3g" % (bits, mode, worst))
        ctx.close()
    # the two placements run the same arithmetic: identical results
    for k in ("status", "abort_op", "obs", "outcomes"):
        assert (outs[1][k] == outs[2][k]).all(), k


def _wide_circuit(seed, n=10, length=160):
    """A random circuit whose span reaches at least 2^8 (a split tile needs
    k_max >= 8): T on fresh |+> qubits first, then random ops."""
    text, _ = random_circuit(seed, n, length, p_t=0.18, p_diag=0.04, p_if=0.04, p_meas=0.05)
    lines = text.strip().split("\n")
    head = ["H %d\nT %d" % (q, q) for q in range(n)]
    return "\n".join([lines[0]] + head + lines[1:]) + "\n"


@pytest.mark.parametrize("seed,lds_log2", [(0, 7), (1, 8), (2, 0), (3, 7)])
def test_split_tiles_random_circuits(seed, lds_log2):
    # the low 2^L entries in LDS, the others in a device-memory slab
    text = _wide_circuit(53000 + seed)
    circ = oracle.Circuit(text)
    N = 192
    words = random_words(seed, N * circ.words_per_shot).reshape(N, circ.words_per_shot)
    ctx = make_ctx(text, keep=(0, N))
    assert ctx.info()["k_max"] >= 8
    ctx.set_tile_memory(3, lds_log2)
    sh = ctx.launch_shape()
    assert sh["tiles_in_memory"] == 2
    if lds_log2:
        assert sh["lds_bytes_per_wave"] >= 16 << lds_log2
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


@pytest.mark.parametrize("bits", [64, 32])
def test_split_tiles_trace_step_by_step(bits):
    text = _wide_circuit(54000, n=9, length=70)
    lines = text.strip().split("\n")
    circ = oracle.Circuit(text)
    words = random_words(3, circ.words_per_shot)
    ctx = make_ctx(text, bits=bits)
    ctx.set_tile_memory(3, 7)
    ctx.set_trace(0, ctx.info()["events"])
    run_gpu(ctx, 0, 1, words.reshape(1, -1))
    steps = 0
    tol = 1e-10 if bits == 64 else 1e-5
    for step in range(ctx.info()["events"]):
        t = ctx.read_trace(step)
        if t is None:
            break
        prefix = "\n".join(lines[: t["op"] + 2]) + "\n"
        pc = oracle.Circuit(prefix)
        r = pc.shot(0, 0, words=words[: pc.words_per_shot], tau=1e-12 if bits == 64 else 1e-6)
        assert (t["r"] == r.tab_r).all(), step
        keys = set(t["coeffs"]) | set(r.coeffs)
        err = max([abs(t["coeffs"].get(a, 0) - r.coeffs.get(a, 0)) for a in keys] + [0.0])
        assert err < tol, (step, err)
        steps += 1
    assert steps >= 10


@pytest.mark.parametrize("bits", [64, 32])
def test_split_equals_lds_on_42q(bits):
    # the 42-qubit workload (span 10) in device memory and with splits at
    # L = 7, 8, 9: the same arithmetic in the same order, so results equal
    # the LDS run bit for bit (FP32 runs its butterfly pairs at spans 8-10 as
    # one pass there, the LDS run as two)
    w = workloads.config("cultivation_42q", seed=1)
    N = 300_000
    outs = {}
    for mode, L in ((1, 0), (2, 0), (3, 7), (3, 8), (3, 9)):
        ctx = make_ctx(w.text, w.noise, seed=17, bits=bits, keep=(0, 32))
        ctx.set_noise_mode(1)
        ctx.set_tile_memory(mode, L)
        outs[(mode, L)] = (run_gpu(ctx, 0, N), [ctx.read_coeffs(s) for s in range(32)], ctx.counters())
        ctx.close()
    base, base_c, base_n = outs[(1, 0)]
    for key, (o, cf, cn) in outs.items():
        for k in ("status", "abort_op", "obs", "outcomes"):
            assert (o[k] == base[k]).all(), (key, k)
        assert cf == base_c, key
        for f in ("passed", "discarded", "logical_errors", "restarts", "entries_t"):
            assert cn[f] == base_n[f], (key, f)


@pytest.mark.parametrize("bits,tol", [(64, 1e-10), (32, 1e-5)])
def test_span12_split_tiles(bits, tol):
    # the scale run's circuit (support cap 2^12) with the low 2^10 / 2^11
    # entries in LDS and the rest spilled to device memory: against the
    # oracle, and equal to the all-LDS placement bit for bit
    w = workloads.config("cultivation_42q_k12", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 2000
    tau = 1e-12 if bits == 64 else 1e-6
    ref = circ.batch(13, 0, N, tau=tau)
    outs = {}
    for L in (0, 10, 11):
        ctx = make_ctx(w.text, w.noise, seed=13, bits=bits, keep=(0, 64))
        ctx.set_tile_memory(1 if L == 0 else 3, L)
        outs[L] = run_gpu(ctx, 0, N)
        diff = (outs[L]["status"] != ref["status"]) | (outs[L]["outcomes"] != ref["outcomes"]).any(axis=0)
        assert diff.sum() <= (0 if bits == 64 else 3)
        compare_batch(outs[L], ref, skip=diff)
        compare_kept(ctx, circ, 13, [s for s in range(64) if not diff[s]], tol=tol, tau=tau)
        ctx.close()
    for L in (10, 11):
        for k in ("status", "abort_op", "obs", "outcomes"):
            assert (outs[L][k] == outs[0][k]).all(), (L, k)


def test_split_tiles_autotune_and_gaps_at_scale():
    # autotune over LDS, device-memory and split placements on the span-12
    # circuit; whatever it picks, 10^6 gap-sampled FP32 shots equal the LDS run
    w = workloads.config("cultivation_42q_k12", seed=1)
    N = 1_000_000
    res = []
    for tune in (False, True):
        ctx = make_ctx(w.text, w.noise, seed=99, bits=32)
        ctx.set_noise_mode(1)
        if tune:
            ctx.autotune(1 << 20)
            print("autotuned shape", ctx.launch_shape())
        else:
            ctx.set_tile_memory(1)
        res.append((run_gpu(ctx, 0, N), ctx.counters()))
        ctx.close()
    for k in ("status", "abort_op", "obs", "outcomes"):
        assert (res[0][0][k] == res[1][0][k]).all(), k
    for f in ("passed", "discarded", "logical_errors"):
        assert res[0][1][f] == res[1][1][f], f
