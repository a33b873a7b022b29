"""GPU parity on the widest registers and spans the library accepts: 64 qubits
(every bit of the sign words, qubit 63 included) and coefficient spans of 14
to 19 dimensions held in device-memory tiles.  Tableaux, records, statuses,
abort ops and observables bit-exact against the oracle; coefficients within
1e-10 (FP64) / 1e-5 (FP32) of the oracle's, relative to its 2-norm."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import compare_batch, compare_kept, make_ctx, run_gpu

pytestmark = pytest.mark.gpu


def wide_circuit(seed, p_t=0.02, length=900):
    text, _ = random_circuit(65000 + seed, 64, length, p_t=p_t, p_meas=0.05, p_mpp=0.04, p_reset=0.03)
    lines = text.strip().split("\n")
    # make sure qubit 63 is measured, reset and entangled with qubit 0
    lines += ["H 63", "CX 63 0", "T 63", "MPP X63*Z0", "M 63", "R 63", "DETECTOR 0 %d" % 0,
              "OBSERVABLE 0 1 2"]
    return "\n".join(lines) + "\n"


def _words(circ, n, seed):
    return np.stack([random_words(seed * 1000 + i, circ.words_per_shot) for i in range(n)])


@pytest.mark.parametrize("seed", range(8))
def test_64_qubits_explicit_words(seed):
    text = wide_circuit(seed)
    circ = oracle.Circuit(text)
    assert circ.n_qubits == 64
    N = 256
    words = _words(circ, N, seed)
    ctx = make_ctx(text, keep=(0, N))
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


@pytest.mark.parametrize("seed,bits", [(0, 64), (2, 64), (5, 32), (6, 64)])
def test_64_qubits_model_noise_philox(seed, bits):
    text = wide_circuit(seed)
    noise = {"p1": 0.004, "p2": 0.004, "p_idle": 0.0, "p_meas": 0.004, "p_reset": 0.004, "p_mpp": 0.004}
    circ = oracle.Circuit(text, noise)
    N = 8192
    ctx = make_ctx(text, noise, seed=77 + seed, bits=bits, keep=(0, 256))
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(77 + seed, 0, N)
    if bits == 64:
        compare_batch(gpu, ref)
        compare_kept(ctx, circ, 77 + seed, range(256))
    else:
        diff = (gpu["status"] != ref["status"]) | (gpu["outcomes"] != ref["outcomes"]).any(axis=0)
        assert diff.sum() <= 2
        compare_batch(gpu, ref, skip=diff)
        compare_kept(ctx, circ, 77 + seed, [s for s in range(256) if not diff[s]], tol=1e-5, tau=1e-6)
    # the sign words reach bit 63: some shot ends with a flipped sign there
    signs = set()
    for s in range(64):
        _, _, r = ctx.read_tableau(s)
        signs.add((int(r[63]), int(r[127])))
    assert len(signs) > 1


@pytest.mark.parametrize("seed,p_t,bits", [(3, 0.02, 64), (3, 0.02, 32), (1, 0.03, 64), (3, 0.03, 32)])
def test_wide_spans_in_device_memory(seed, p_t, bits):
    # spans of 14 (LDS cannot hold the FP64 tile) and 18-19 dimensions: the
    # tiles live in device memory, one slab per wave
    text = wide_circuit(seed, p_t=p_t)
    circ = oracle.Circuit(text)
    N = 12
    words = _words(circ, N, seed + 50)
    ctx = make_ctx(text, bits=bits, keep=(0, N), tau=1e-12 if bits == 64 else 1e-6)
    info = ctx.info()
    assert info["k_max"] >= 14
    ctx.set_tile_memory(0)
    assert ctx.launch_shape()["tiles_in_memory"] == 1
    gpu = run_gpu(ctx, 0, N, words)
    ref = circ.batch(0, 0, N, words=words, tau=1e-12 if bits == 64 else 1e-6)
    assert ref["max_support"].max() >= 1 << 13
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 0, range(N), words=words, tol=1e-10 if bits == 64 else 1e-5,
                 tau=1e-12 if bits == 64 else 1e-6)
