"""GPU parity of classically controlled gates (IF) and gate teleportation.

`IF r0,r1,.. GATE` applies GATE when the XOR of the record bits is 1,
`IF r0&r1&.. GATE` when all of them are 1.  A conditional Pauli flips tableau
signs; a conditional diagonal gate (S, SDG, T, TDG, CZ, CS, CCZ, CPHASE, RZ,
DIAG) acts on the coefficients by its Z-string expansion, so the x/z frame is
the same in every shot and the span grows in every shot (zeros where the gate
did not fire).  Tableaux, records, statuses, abort ops and observables must be
bit-exact against the oracle; coefficients within 1e-10 (FP64) / 1e-5 (FP32)
relative to the oracle's 2-norm.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import compare_batch, compare_kept, make_ctx, run_gpu

pytestmark = pytest.mark.gpu


def _words(circ, n, seed):
    return random_words(seed, n * circ.words_per_shot).reshape(n, circ.words_per_shot)


@pytest.mark.parametrize("seed", range(24))
def test_conditional_gates_explicit_words(seed):
    n = 2 + seed % 7
    text, _ = random_circuit(71000 + seed, n, 90, p_if=0.2, p_diag=0.06, p_t=0.1, p_meas=0.12)
    assert "IF " in text
    circ = oracle.Circuit(text)
    N = 256
    words = _words(circ, N, seed)
    ctx = make_ctx(text, keep=(0, N))
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


@pytest.mark.parametrize("seed,bits", [(0, 64), (1, 64), (2, 32), (3, 32)])
def test_conditional_gates_model_noise_philox(seed, bits):
    text, _ = random_circuit(72000 + seed, 6, 200, p_if=0.12, p_diag=0.05, p_msc=0.05)
    noise = {"p1": 3e-3, "p2": 3e-3, "p_idle": 1e-3, "p_meas": 3e-3, "p_reset": 3e-3, "p_mpp": 3e-3}
    circ = oracle.Circuit(text, noise)
    N = 20000
    ctx = make_ctx(text, noise, seed=21 + seed, bits=bits, keep=(0, 256))
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(21 + seed, 0, N)
    if bits == 64:
        compare_batch(gpu, ref)
        compare_kept(ctx, circ, 21 + seed, range(256))
    else:
        # FP32: an outcome may differ only near a tie (u within 1e-5 of p0)
        diff = (gpu["status"] != ref["status"]) | (gpu["outcomes"] != ref["outcomes"]).any(axis=0)
        assert diff.sum() <= 3
        compare_batch(gpu, ref, skip=diff)
        compare_kept(ctx, circ, 21 + seed, [s for s in range(256) if not diff[s]], tol=1e-5, tau=1e-6)


@pytest.mark.parametrize("seed", range(4))
def test_conditional_gates_trace_step_by_step(seed):
    # after every event the GPU state equals the oracle's state for the same
    # prefix (the step-by-step check of the paper's validation)
    n = 3 + seed % 3
    text, _ = random_circuit(73000 + seed, n, 60, p_if=0.25, p_meas=0.15, p_diag=0.05)
    # a CCX line is H, CCZ, H: written out, every traced event ends a line,
    # so the state after it is the state of a circuit prefix
    lines = []
    for line in text.strip().split("\n"):
        tok = line.split()
        if "CCX" in tok:
            t = tok[-1]
            lines += ["H %s" % t, line.replace("CCX", "CCZ"), "H %s" % t]
        else:
            lines.append(line)
    text = "\n".join(lines) + "\n"
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


@pytest.mark.parametrize("cap", [2, 4, 8])
def test_conditional_gates_with_caps(cap):
    # a conditional CCZ that fires can pass the cap; one that does not fire
    # never does (the oracle skips it, and the kernel only zero-fills)
    text = ("QUBITS 6\nH 0\nH 1\nH 2\nH 3\nM 3\nH 4\nM 4\nIF 0 CCZ 0 1 2\nIF 0&1 CS 1 5\nH 5\n"
            "IF 1 T 5\nIF 0,1 T 0\nMPP X0*X1\nM 2\n")
    noise = {"p1": 0.05, "p2": 0.05}
    circ = oracle.Circuit(text, noise)
    ref = circ.batch(4, 0, 4000, cap=cap)
    assert (ref["status"] == oracle.OVERFLOW).any() and (ref["status"] != oracle.OVERFLOW).any()
    ctx = make_ctx(text, noise, seed=4, cap=cap, keep=(0, 64))
    compare_batch(run_gpu(ctx, 0, 4000), ref)
    compare_kept(ctx, circ, 4, range(64), cap=cap)


def test_conditional_gates_in_device_memory_tiles():
    text, _ = random_circuit(74000, 7, 120, p_if=0.2, p_diag=0.08, p_t=0.1, p_meas=0.12)
    circ = oracle.Circuit(text)
    N = 128
    words = _words(circ, N, 6)
    ctx = make_ctx(text, keep=(0, N))
    ctx.set_tile_memory(2)
    assert ctx.launch_shape()["tiles_in_memory"] == 1
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


CCZ_TELEPORT = (
    # |CCZ> = CCZ|+++> on ancillas 3, 4, 5; CX data i -> ancilla i; M
    # ancillas; corrections CZ for each single outcome bit, Z for each pair
    "H 3\nH 4\nH 5\nCCZ 3 4 5\nCX 0 3\nCX 1 4\nCX 2 5\nM 3\nM 4\nM 5\n"
    "IF 0 CZ 1 2\nIF 1 CZ 0 2\nIF 2 CZ 0 1\nIF 0&1 Z 2\nIF 0&2 Z 1\nIF 1&2 Z 0\n")


@pytest.mark.parametrize("seed", range(3))
def test_ccz_teleportation_every_branch_on_gpu(seed):
    # every outcome branch of CCZ teleportation: the GPU state equals the
    # oracle's, and (noise off) equals the direct CCZ up to a global phase on
    # the data, which the oracle pins already check against the statevector
    prep, _ = random_circuit(9400 + seed, 3, 30, p_meas=0, p_mpp=0, p_reset=0)
    body = prep.split("\n", 1)[1]
    text = "QUBITS 6\n" + body + CCZ_TELEPORT + "MPP X0*Y1\nM 2\n"
    circ = oracle.Circuit(text)
    rows = []
    for branch in itertools.product((0, 1), repeat=3):
        rows.append([0 if b == 0 else 2 ** 32 - 1 for b in branch] + [0x1234567, 0x89ABCDEF])
    words = np.array(rows, dtype=np.uint32)
    ctx = make_ctx(text, keep=(0, 8))
    gpu = run_gpu(ctx, 0, 8, words)
    ref = circ.batch(0, 0, 8, words=words)
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 0, range(8), words=words)
    assert sorted({tuple((gpu["outcomes"][0, s] >> np.arange(3)) & 1) for s in range(8)}) == \
        sorted(itertools.product((0, 1), repeat=3))


def test_teleported_t_layer_with_noise_fp32_and_fp64():
    # a teleported T / T-dagger layer on three data qubits under circuit-level
    # noise: GPU against oracle in both precisions
    tele = ("QUBITS 6\nH 0\nH 1\nH 2\nCX 0 1\nH 3\nT 3\nH 4\nT 4\nH 5\nTDG 5\n"
            "CX 0 3\nCX 1 4\nCX 2 5\nM 3\nM 4\nM 5\nIF 0 S 0\nIF 1 S 1\nIF 2 SDG 2\n"
            "MPP X0*X1*X2\nDETECTOR 0 3\nM 0\nM 1\nOBSERVABLE 0 4 5\n")
    noise = {"p1": 2e-3, "p2": 2e-3, "p_meas": 2e-3, "p_mpp": 2e-3}
    circ = oracle.Circuit(tele, noise)
    N = 50000
    ref = circ.batch(31, 0, N)
    for bits in (64, 32):
        ctx = make_ctx(tele, noise, seed=31, bits=bits, keep=(0, 128))
        gpu = run_gpu(ctx, 0, N)
        if bits == 64:
            compare_batch(gpu, ref)
            compare_kept(ctx, circ, 31, range(128))
        else:
            diff = (gpu["status"] != ref["status"]) | (gpu["outcomes"] != ref["outcomes"]).any(axis=0)
            assert diff.sum() <= 3
            compare_batch(gpu, ref, skip=diff)
            compare_kept(ctx, circ, 31, [s for s in range(128) if not diff[s]], tol=1e-5, tau=1e-6)


def test_conditional_gates_with_gap_sampling():
    text, _ = random_circuit(75000, 6, 160, p_if=0.15, p_diag=0.05)
    noise = {"p1": 4e-3, "p2": 4e-3, "p_meas": 4e-3, "p_mpp": 4e-3}
    circ = oracle.Circuit(text, noise, noise_mode=1)
    N = 20000
    ctx = make_ctx(text, noise, seed=41, keep=(0, 64))
    ctx.set_noise_mode(1)
    compare_batch(run_gpu(ctx, 0, N), circ.batch(41, 0, N))
    compare_kept(ctx, circ, 41, range(64))


def test_if_parse_errors_on_gpu_compiler():
    from paper_2512_23037_amd import soft
    for bad, frag in (("QUBITS 2\nIF 0 S 1\n", "not yet measured"), ("QUBITS 2\nM 0\nIF 0,0&0 S 1\n", "not both"),
                      ("QUBITS 2\nM 0\nIF 0 H 1\n", "neither"), ("QUBITS 2\nM 0\nIF 0\n", "record bits and a gate"),
                      ("QUBITS 2\nM 0\nIF 0 CZ 1 1\n", "repeated"), ("QUBITS 2\nM 0\nIF 0 S 1 0\n", "arguments")):
        ctx = soft.Context(0)
        with pytest.raises(soft.SoftError, match=frag):
            ctx.load_circuit(bad)
            ctx.info()
