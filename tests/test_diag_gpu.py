"""GPU parity of the one-pass diagonal gates (CS, CSDG, CPHASE, RZ, CCZ, CCX
and DIAG on 1-3 qubits): the kernel runs each gate's Z-string expansion
U = sum_g c_g Z^g in one pass over the tile (one coset of the terms' shifts
per group of lanes).  Tableaux, records, statuses, abort ops and observables
bit-exact against the oracle; coefficients within 1e-10 (FP64) / 1e-5 (FP32)
relative to the oracle's 2-norm."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import compare_batch, compare_kept, make_ctx, run_gpu

pytestmark = pytest.mark.gpu


def _words(circ, n, seed):
    return random_words(seed, n * circ.words_per_shot).reshape(n, circ.words_per_shot)


@pytest.mark.parametrize("seed", range(20))
def test_diagonal_gates_explicit_words(seed):
    n = 1 + seed % 8
    text, _ = random_circuit(66000 + seed, n, 90, p_diag=0.15, p_t=0.08)
    circ = oracle.Circuit(text)
    N = 256
    words = _words(circ, N, seed)
    ctx = make_ctx(text, keep=(0, N))
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


@pytest.mark.parametrize("seed,bits", [(0, 64), (1, 64), (2, 32), (3, 32)])
def test_diagonal_gates_model_noise_philox(seed, bits):
    text, _ = random_circuit(67000 + seed, 6, 200, p_diag=0.1, p_msc=0.1)
    noise = {"p1": 3e-3, "p2": 3e-3, "p_idle": 1e-3, "p_meas": 3e-3, "p_reset": 3e-3, "p_mpp": 3e-3}
    circ = oracle.Circuit(text, noise)
    N = 20000
    ctx = make_ctx(text, noise, seed=8 + seed, bits=bits, keep=(0, 256))
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(8 + seed, 0, N)
    if bits == 64:
        compare_batch(gpu, ref)
        compare_kept(ctx, circ, 8 + seed, range(256))
    else:
        diff = (gpu["status"] != ref["status"]) | (gpu["outcomes"] != ref["outcomes"]).any(axis=0)
        assert diff.sum() <= 3
        compare_batch(gpu, ref, skip=diff)
        compare_kept(ctx, circ, 8 + seed, [s for s in range(256) if not diff[s]], tol=1e-5, tau=1e-6)


@pytest.mark.parametrize("seed", range(4))
def test_diagonal_gates_with_caps(seed):
    # a support cap below what a CCZ or CS layer reaches: OVERFLOW at the
    # same op as the oracle (one-pass gates count only their final support)
    lines = ["QUBITS 6"] + ["H %d" % q for q in range(6)] + ["CCZ 0 1 2", "CS 3 4", "T 5", "CCZ 3 4 5",
                                                             "RZ 0.3 0", "M 0", "DIAG 2 1 5 0 0.4 0.9 -1.2"]
    text = "\n".join(lines) + "\n"
    noise = {"p1": 0.02, "p2": 0.02}
    circ = oracle.Circuit(text, noise)
    cap = [4, 8, 32, 64][seed]
    ref = circ.batch(3, 0, 4000, cap=cap)
    assert (ref["status"] == oracle.OVERFLOW).any() or cap == 64
    ctx = make_ctx(text, noise, seed=3, cap=cap, keep=(0, 64))
    compare_batch(run_gpu(ctx, 0, 4000), ref)
    compare_kept(ctx, circ, 3, range(64), cap=cap)


@pytest.mark.parametrize("seed", range(4))
def test_diagonal_gates_trace_step_by_step(seed):
    # the step-by-step check (Sec. V-B) across diagonal gates: after every
    # event the GPU state equals the oracle's state for the same prefix
    n = 3 + seed % 3
    text, _ = random_circuit(68000 + seed, n, 60, p_diag=0.2)
    lines = text.strip().split("\n")
    circ = oracle.Circuit(text)
    words = random_words(seed, circ.words_per_shot)
    ctx = make_ctx(text)
    ctx.set_trace(0, ctx.info()["events"])
    run_gpu(ctx, 0, 1, words.reshape(1, -1))
    steps = 0
    for step in range(ctx.info()["events"]):
        t = ctx.read_trace(step)
        if t is None:
            break
        prefix = "\n".join(lines[: t["op"] + 2]) + "\n"
        pc = oracle.Circuit(prefix)
        r = pc.shot(0, 0, words=words[: pc.words_per_shot])
        assert (t["x"] == r.tab_x).all() and (t["z"] == r.tab_z).all() and (t["r"] == r.tab_r).all(), step
        keys = set(t["coeffs"]) | set(r.coeffs)
        err = max([abs(t["coeffs"].get(a, 0) - r.coeffs.get(a, 0)) for a in keys] + [0.0])
        assert err < 1e-10, (step, lines[t["op"] + 1], err)
        steps += 1
    assert steps >= 5


def test_diagonal_gates_in_device_memory_tiles():
    text, _ = random_circuit(69000, 7, 120, p_diag=0.15, p_t=0.1)
    circ = oracle.Circuit(text)
    N = 128
    words = _words(circ, N, 5)
    ctx = make_ctx(text, keep=(0, N))
    ctx.set_tile_memory(2)
    assert ctx.launch_shape()["tiles_in_memory"] == 1
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


def test_ccz_one_pass_equals_seven_t_form_on_gpu():
    # the one-pass CCZ and its seven-T phase polynomial written out give the
    # same records and final states on the GPU (and both equal the oracle)
    seven = ("T 0\nT 1\nT 2\nCX 0 1\nTDG 1\nCX 0 1\nCX 0 2\nTDG 2\nCX 0 2\nCX 1 2\nTDG 2\nCX 1 2\n"
             "CX 0 2\nCX 1 2\nT 2\nCX 1 2\nCX 0 2\n")
    prep = "QUBITS 4\nH 0\nH 1\nH 2\nT 1\nCX 2 3\nH 3\n"
    tail = "MPP X0*X1\nM 2\nMPP Y1*Z3\n"
    a_txt, b_txt = prep + "CCZ 0 1 2\n" + tail, prep + seven + tail
    N = 4096
    res = []
    for t in (a_txt, b_txt):
        ctx = make_ctx(t, seed=12, keep=(0, 64))
        res.append((ctx, run_gpu(ctx, 0, N)))
    for key in ("status", "outcomes"):
        assert (res[0][1][key] == res[1][1][key]).all()
    for s in range(64):
        ca, cb = res[0][0].read_coeffs(s), res[1][0].read_coeffs(s)
        keys = set(ca) | set(cb)
        assert max(abs(ca.get(k, 0) - cb.get(k, 0)) for k in keys) < 1e-10
