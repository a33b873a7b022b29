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
