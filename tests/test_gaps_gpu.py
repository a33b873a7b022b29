"""GPU parity of gap sampling (noise mode 1): the kernel's candidate walk over
the gap table and its thinning must give the oracle's mode-1 shots bit for bit
(records, statuses, abort ops, observables, tableaux; coefficients to 1e-10 in
FP64).  The circuits cover thinned and unthinned slots, many candidates per
shot (stream-2 words past one 256-word block), gaps past 64 and past 4096
table entries, mixtures with a table per variant, speculation restarts and
the lane-parallel measurement runs."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from paper_2512_23037_amd import soft
from tests.gen_small import random_circuit
from tests.gpu_helpers import compare_batch, compare_kept, make_ctx, run_gpu

pytestmark = pytest.mark.gpu


def _gap_ctx(text, noise=None, **kw):
    ctx = make_ctx(text, noise, **kw)
    ctx.set_noise_mode(1)
    return ctx


@pytest.mark.parametrize("seed", range(12))
def test_random_noisy_circuits_gaps(seed):
    n = 2 + seed % 6
    text, _ = random_circuit(41000 + seed, n, 120, p_msc=0.1 if seed % 3 == 0 else 0.0)
    rng = np.random.default_rng(seed)
    lines = text.strip().split("\n")
    out = [lines[0]]
    for line in lines[1:]:
        out.append(line)
        if rng.random() < 0.2:
            out.append("TICK")
    text = "\n".join(out) + "\n"
    # distinct rates per kind: most candidates are thinned
    noise = {"p1": 0.02, "p2": 0.05, "p_idle": 0.01, "p_meas": 0.03, "p_reset": 0.015, "p_mpp": 0.04}
    circ = oracle.Circuit(text, noise, noise_mode=1)
    N = 2048
    ctx = _gap_ctx(text, noise, seed=7 + seed, keep=(500, 64))
    gpu = run_gpu(ctx, 500, N)
    compare_batch(gpu, circ.batch(7 + seed, 500, N))
    compare_kept(ctx, circ, 7 + seed, range(500, 564))


@pytest.mark.parametrize("p", [0.2, 2e-4])
def test_long_single_qubit_chain(p):
    # 6000 noise slots of one rate on one qubit, read out after each: with
    # p = 0.2 a shot has ~1200 candidates (stream-2 words far past the first
    # 256), with p = 2e-4 most gaps run past 4096 table entries.
    n = 6000
    text = "QUBITS 1\n" + "XERR %r 0\nM 0\nR 0\n" % p * n
    circ = oracle.Circuit(text, noise_mode=1)
    N = 4096
    ctx = _gap_ctx(text, None, seed=3)
    gpu = run_gpu(ctx, 0, N)
    compare_batch(gpu, circ.batch(3, 0, N))
    hits = int(np.unpackbits(gpu["outcomes"].view(np.uint8)).sum())
    assert abs(hits / N - n * p) < 6 * np.sqrt(n * p / N)


def test_heavy_thinning_chain():
    # One slot at 0.3 sets p_max; 3000 slots at 1e-3 accept one candidate in 300.
    text = "QUBITS 2\nXERR 0.3 1\n" + "XERR 0.001 0\nM 0\nR 0\n" * 3000 + "M 1\n"
    circ = oracle.Circuit(text, noise_mode=1)
    N = 4096
    ctx = _gap_ctx(text, None, seed=9)
    gpu = run_gpu(ctx, 0, N)
    compare_batch(gpu, circ.batch(9, 0, N))


def test_cultivation_15q_gaps():
    w = workloads.config("cultivation_15q", seed=1)
    circ = oracle.Circuit(w.text, w.noise, noise_mode=1)
    N = 200_000
    ctx = _gap_ctx(w.text, w.noise, seed=17, keep=(0, 128))
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(17, 0, N)
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 17, range(128))
    c = ctx.counters()
    assert c["passed"] == int((ref["status"] == 0).sum())
    assert c["logical_errors"] == int(((ref["status"] == 0) & (ref["obs"] != 0)).sum())


def test_cultivation_42q_gaps_with_restarts():
    # Dense model noise breaks T / T-dagger cancellations: restarted shots
    # redraw the same candidates.
    w = workloads.config("cultivation_42q", seed=1)
    noise = {k: (v * 8 if v else v) for k, v in w.noise.items()}
    circ = oracle.Circuit(w.text, noise, noise_mode=1)
    N = 3000
    ctx = _gap_ctx(w.text, noise, seed=23, keep=(0, 64))
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(23, 0, N)
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 23, range(64))
    assert ctx.counters()["restarts"] > 0
    assert len(np.unique(ref["abort_op"])) > 5


def test_full_size_sampled_shots_gaps():
    # The benchmark's workload at full size in FP32 with gap sampling.
    w = workloads.config("cultivation_42q", seed=1)
    circ = oracle.Circuit(w.text, w.noise, noise_mode=1)
    N = 2_000_000
    ctx = _gap_ctx(w.text, w.noise, seed=5, bits=32)
    gpu = run_gpu(ctx, 0, N)
    c = ctx.counters()
    assert c["shots"] == N and c["passed"] == int((gpu["status"] == 0).sum())
    rng = np.random.default_rng(1)
    for shot in rng.choice(N, size=150, replace=False):
        r = circ.shot(5, int(shot))
        assert gpu["status"][shot] == r.status and gpu["abort_op"][shot] == r.abort_op
        rec = [int((gpu["outcomes"][k >> 5, shot] >> (k & 31)) & 1) for k in range(circ.n_records)]
        assert rec == r.record


def test_mixture_gaps_per_variant_tables():
    total = 27 * 800
    m = workloads.mixture(seed=1, total_shots=total)
    ctx = soft.Context(0)
    ctx.load_mixture([w.text for w in m["workloads"]], m["models"], m["shot_ends"])
    ctx.set_rng(41)
    ctx.set_noise_mode(1)
    gpu = run_gpu(ctx, 0, total)
    lo = 0
    cache = {}
    for v, (w, mod, hi) in enumerate(zip(m["workloads"], m["models"], m["shot_ends"])):
        key = (w.name, mod["p1"])
        if key not in cache:
            cache[key] = oracle.Circuit(w.text, mod, noise_mode=1)
        c = cache[key]
        ref = c.batch(41, lo, hi - lo)
        nw = (c.n_records + 31) // 32
        sub = {k: (x[:nw, lo:hi] if x.ndim == 2 else x[lo:hi]) for k, x in gpu.items()}
        compare_batch(sub, ref)
        lo = hi


def test_mode_switch_and_explicit_words():
    w = workloads.config("cultivation_15q", seed=1)
    ctx = make_ctx(w.text, w.noise, seed=4)
    a0 = run_gpu(ctx, 0, 20000)
    ctx.set_noise_mode(1)
    a1 = run_gpu(ctx, 0, 20000)
    ref1 = oracle.Circuit(w.text, w.noise, noise_mode=1).batch(4, 0, 20000)
    compare_batch(a1, ref1)
    ctx.set_noise_mode(0)
    compare_batch(run_gpu(ctx, 0, 20000), a0)
    # explicit words take the per-slot form in either mode
    circ = oracle.Circuit(w.text, w.noise)
    rng = np.random.default_rng(2)
    words = rng.integers(0, 2**32, size=(512, circ.words_per_shot), dtype=np.uint64).astype(np.uint32)
    ctx.set_noise_mode(1)
    compare_batch(run_gpu(ctx, 0, 512, words), circ.batch(0, 0, 512, words=words))
    with pytest.raises(soft.SoftError):
        ctx.set_noise_mode(2)
