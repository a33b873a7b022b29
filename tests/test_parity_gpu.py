"""GPU parity: the HIP sampler (through the C ABI) against the CPU oracle on
the same seeded inputs.  Tableaux, outcomes, statuses, abort ops and
observables bit-exact; coefficients within 1e-10 (FP64) / 1e-5 (FP32) of the
oracle's, relative to its 2-norm."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from paper_2512_23037_amd import soft
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import (compare_batch, compare_kept, compare_kept_many, guard_band_flips, make_ctx,
                               oracle_shots, run_gpu, torch)

pytestmark = pytest.mark.gpu


def _words(circ, n, seed):
    return random_words(seed, n * circ.words_per_shot).reshape(n, circ.words_per_shot)


@pytest.mark.parametrize("seed", range(24))
def test_random_circuits_explicit_words(seed):
    n = 1 + seed % 8
    text, _ = random_circuit(31000 + seed, n, 90)
    circ = oracle.Circuit(text)
    N = 128
    words = _words(circ, N, seed)
    ctx = make_ctx(text, keep=(0, N))
    gpu = run_gpu(ctx, 0, N, words)
    ref = circ.batch(0, 0, N, words=words)
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 0, range(N), words=words)


@pytest.mark.parametrize("seed", range(16))
def test_msc_ops_explicit_words(seed):
    # X-basis readouts and resets, measure-and-reset, H_XY / H_NXY and
    # record-controlled Paulis, with explicit noise ops and words
    n = 1 + seed % 6
    text, _ = random_circuit(61000 + seed, n, 90, p_msc=0.25)
    if seed % 2:
        lines = text.strip().split("\n")
        noisy = [lines[0]]
        for ln in lines[1:]:
            noisy.append(ln)
            q = ln.split()[-1]
            if q.isdigit():
                noisy.append("ZERR 0.05 %s" % q if seed % 4 == 1 else "DEP1 0.05 %s" % q)
        text = "\n".join(noisy) + "\n"
    circ = oracle.Circuit(text)
    N = 256
    words = _words(circ, N, seed)
    ctx = make_ctx(text, keep=(0, N))
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


@pytest.mark.parametrize("seed", range(10))
def test_ccz_ccx_explicit_words(seed):
    # CCZ / Toffoli lowered to their phase polynomial of seven T/T-dagger
    n = 3 + seed % 5
    text, _ = random_circuit(63000 + seed, n, 70, p_ccz=0.12)
    circ = oracle.Circuit(text)
    N = 256
    words = _words(circ, N, seed)
    ctx = make_ctx(text, keep=(0, N))
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(N), words=words)


@pytest.mark.parametrize("seed", range(3))
def test_long_records_in_lds(seed):
    # More than 128 record bits: words beyond the four scalar-register words
    # live in LDS, and beyond eight words the outputs go out directly;
    # detectors and feedback read bits across all of them.
    rng = np.random.default_rng(seed)
    text, _ = random_circuit(64000 + seed, 4, 700, p_meas=0.5, p_t=0.05, p_mpp=0.02, p_reset=0.0)
    lines = text.strip().split("\n")
    out, n_rec = [lines[0]], 0
    for ln in lines[1:]:
        out.append(ln)
        if ln.startswith(("M ", "MPP ")):
            n_rec += 1
            if n_rec > 10 and rng.random() < 0.04:
                r = sorted(rng.choice(n_rec, size=3, replace=False))
                out.append("DETECTOR %d %s" % (int(rng.integers(2)), " ".join(str(x) for x in r)))
            if n_rec > 5 and rng.random() < 0.05:
                out.append("XIF %d %d" % (int(rng.integers(n_rec)), int(rng.integers(4))))
    out.append("OBSERVABLE 0 %s" % " ".join(str(x) for x in range(0, n_rec, 7)))
    text = "\n".join(out) + "\n"
    circ = oracle.Circuit(text)
    assert circ.n_records > 300
    N = 512
    words = _words(circ, N, seed)
    ctx = make_ctx(text, keep=(0, 64))
    assert ctx.info()["record_words"] > 8
    gpu = run_gpu(ctx, 0, N, words)
    compare_batch(gpu, circ.batch(0, 0, N, words=words))
    compare_kept(ctx, circ, 0, range(64), words=words)


def test_msc_ops_model_noise_philox():
    text, _ = random_circuit(62000, 5, 200, p_msc=0.2, p_ccz=0.03)
    assert "CC" in text
    noise = {"p1": 2e-3, "p2": 4e-3, "p_idle": 1e-3, "p_meas": 5e-3, "p_reset": 5e-3, "p_mpp": 5e-3}
    circ = oracle.Circuit(text, noise)
    N = 20000
    ctx = make_ctx(text, noise, seed=8, keep=(0, 128))
    gpu = run_gpu(ctx, 0, N)
    compare_batch(gpu, circ.batch(8, 0, N))
    compare_kept(ctx, circ, 8, range(128))


@pytest.mark.parametrize("seed", range(16))
def test_random_noisy_circuits_philox(seed):
    n = 2 + seed % 6
    text, _ = random_circuit(32000 + seed, n, 80)
    rng = np.random.default_rng(seed)
    lines = text.strip().split("\n")
    out = [lines[0]]
    for line in lines[1:]:
        out.append(line)
        if rng.random() < 0.2:
            out.append("TICK")
    text = "\n".join(out) + "\n"
    noise = {k: 0.03 for k in ("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp")}
    cap = [0, 1, 2, 4][seed % 4]
    circ = oracle.Circuit(text, noise)
    N = 512
    ctx = make_ctx(text, noise, seed=99 + seed, cap=cap, keep=(1000, 64))
    gpu = run_gpu(ctx, 1000, N)
    ref = circ.batch(99 + seed, 1000, N, cap=cap if cap else 0xFFFFFFFF)
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 99 + seed, range(1000, 1064), cap=cap if cap else 0xFFFFFFFF)


def test_clifford_t_8q_full():
    w = workloads.config("clifford_t_8q", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 10000
    ctx = make_ctx(w.text, w.noise, seed=2024, keep=(0, 512))
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(2024, 0, N)
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 2024, range(512))
    c = ctx.counters()
    assert c["shots"] == N
    assert c["passed"] == int((ref["status"] == 0).sum())
    assert c["discarded"] == int((ref["status"] == 1).sum())


def test_cultivation_15q_full():
    w = workloads.config("cultivation_15q", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 1_000_000
    ctx = make_ctx(w.text, w.noise, seed=7, keep=(0, 256))
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(7, 0, N)
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 7, range(256))
    c = ctx.counters()
    assert c["passed"] == int((ref["status"] == 0).sum())
    assert c["logical_errors"] == int(((ref["status"] == 0) & (ref["obs"] != 0)).sum())
    hist = np.bincount(np.floor(np.log2(ref["max_support"])).astype(int), minlength=16)
    # The speculative list runs the commuting T gates of a layer in another
    # order and may hold smaller supports than the circuit's order; the full
    # list's supports are the oracle's.
    spec_hist = c["support_hist"]
    assert sum(spec_hist) == N and max(np.nonzero(spec_hist)[0]) <= max(np.nonzero(hist)[0])
    # (with deferred T runs off: a shot that a check ends with a T run skipped
    # reports the supports it computed)
    ctx.set_speculation(False)
    ctx.set_deferred_t(False)
    run_gpu(ctx, 0, N)
    assert list(hist[:16]) == ctx.counters()["support_hist"]


@pytest.mark.parametrize("workload,rate", [("cultivation_15q", 0.03), ("cultivation_15q", 0.004),
                                           ("cultivation_42q", 0.002)])
def test_measurement_runs_with_dense_noise(workload, rate):
    # Runs of outcome-fixed measurements (checks and resets) are evaluated one
    # member per lane; noise hits between members must reach exactly the
    # members after them, and a failing check inside a run must end the shot
    # there.  Explicit words put a hit on each noise slot with probability
    # `rate`, far above the model's p, so most runs see hits inside them.
    w = workloads.config(workload, seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 4096
    rng = np.random.default_rng([len(workload), int(rate * 1e4)])
    thr = int(w.noise["p1"] * 2**32)  # every slot of these circuits has p = p1
    hit = rng.random((N, circ.n_noise_slots)) < rate
    nw = np.where(hit, rng.integers(0, thr, size=hit.shape), rng.integers(thr, 2**32, size=hit.shape))
    mw = rng.integers(0, 2**32, size=(N, circ.n_meas_slots))
    words = np.concatenate([nw, mw], axis=1).astype(np.uint32)
    ctx = make_ctx(w.text, w.noise, keep=(0, 256))
    gpu = run_gpu(ctx, 0, N, words)
    ref = circ.batch(0, 0, N, words=words)
    compare_batch(gpu, ref)
    compare_kept(ctx, circ, 0, range(256), words=words[:256])
    # shots end at many different checks, not only the first
    assert len(np.unique(ref["abort_op"])) > 5
    # the dense noise breaks T / T-dagger cancellations: restarted shots
    assert ctx.counters()["restarts"] > 0


@pytest.mark.parametrize("workload,bits", [("cultivation_15q", 64), ("cultivation_42q", 64), ("cultivation_42q", 32)])
def test_speculative_lists_equal_full_lists(workload, bits):
    # The span-truncating event list (with restarts where noise broke a
    # cancellation) gives the full list's results: records, statuses, abort
    # ops and observables bit for bit, kept coefficients to rounding.
    w = workloads.config(workload, seed=1)
    N = 200_000
    outs, kept = {}, {}
    for spec in (True, False):
        ctx = make_ctx(w.text, w.noise, seed=31, bits=bits, keep=(0, 128))
        ctx.set_speculation(spec)
        outs[spec] = run_gpu(ctx, 0, N)
        kept[spec] = [ctx.read_coeffs(s_) for s_ in range(128)]
        c = ctx.counters()
        if spec:
            assert 0 < c["restarts"] < N // 10
        else:
            assert c["restarts"] == 0
        ctx.close()
    diff = (outs[True]["status"] != outs[False]["status"]) | (outs[True]["outcomes"] != outs[False]["outcomes"]).any(axis=0)
    # FP32: an outcome may flip only at a near-tie of the two summation orders
    assert diff.sum() == 0 if bits == 64 else diff.sum() <= 2
    keep = ~diff
    for key in ("abort_op", "obs"):
        assert (outs[True][key][keep] == outs[False][key][keep]).all()
    tol = 1e-10 if bits == 64 else 1e-5
    for s_ in range(128):
        if keep[s_]:
            from tests.gpu_helpers import coeff_error
            assert coeff_error(kept[True][s_], kept[False][s_]) < tol


def test_speculation_noiseless_never_restarts():
    w = workloads.config("cultivation_42q", seed=1)
    ctx = make_ctx(w.text, None, seed=2)
    gpu = run_gpu(ctx, 0, 100_000)
    assert (gpu["status"] == 0).all() and (gpu["obs"] == 0).all()
    assert ctx.counters()["restarts"] == 0


@pytest.mark.parametrize("noise_mode", [0, 1])
@pytest.mark.parametrize("bits,tol", [(64, 1e-10), (32, 1e-5)])
def test_cultivation_42q_oracle_subset(bits, tol, noise_mode):
    # The precision configuration's oracle subset: shots 0..9999 of the
    # 42-qubit workload, FP64 and FP32, per-slot draws and gap sampling.
    # Records, statuses, abort ops and observables of every shot bit-exact
    # (FP32: a shot may differ only where a draw lies within 1e-5 of the
    # oracle's probability); kept tableaux and coefficients of every passed
    # shot and of every fifth other shot.
    w = workloads.config("cultivation_42q", seed=1)
    circ = oracle.Circuit(w.text, w.noise, noise_mode=noise_mode)
    N = 10000
    seed = 11 + noise_mode
    ctx = make_ctx(w.text, w.noise, seed=seed, bits=bits, keep=(0, N))
    ctx.set_noise_mode(noise_mode)
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(seed, 0, N)
    diff = (gpu["status"] != ref["status"]) | (gpu["outcomes"] != ref["outcomes"]).any(axis=0)
    if bits == 64:
        assert not diff.any()
    else:
        flips = np.nonzero(diff)[0]
        assert len(flips) <= 5
        res = oracle_shots(circ, seed, flips)
        assert all(guard_band_flips(circ, seed, list(zip(flips, res)))), \
            "FP32 outcome flip outside the guard band"
    compare_batch(gpu, ref, skip=diff)
    passed = np.nonzero((ref["status"] == oracle.PASSED) & ~diff)[0]
    assert len(passed) > 50
    others = [s for s in range(0, N, 5) if not diff[s] and ref["status"][s] != oracle.PASSED]
    shots = sorted(set(passed.tolist()) | set(others))
    assert len(shots) >= 1000
    worst = compare_kept_many(ctx, circ, seed, shots, tol=tol, tau=1e-12 if bits == 64 else 1e-6)
    print("bits=%d mode=%d: %d kept shots (%d passed), worst coefficient error %.3g, %d guard-band flips"
          % (bits, noise_mode, len(shots), len(passed), worst, int(diff.sum())))


def test_full_size_sampled_shots():
    # The benchmark's workload and launch shape at full size; sampled shots
    # are checked one by one against the oracle, the rest by invariants.
    w = workloads.config("cultivation_42q", seed=1)
    circ = oracle.Circuit(w.text, w.noise)
    N = 2_000_000
    ctx = make_ctx(w.text, w.noise, seed=5, bits=32)
    gpu = run_gpu(ctx, 0, N)
    c = ctx.counters()
    assert c["shots"] == N
    assert c["passed"] + c["discarded"] + c["overflow"] + c["numeric"] == N
    assert c["passed"] == int((gpu["status"] == 0).sum())
    assert ((gpu["status"] == 0) == (gpu["abort_op"] == soft.NO_ABORT)).all()
    assert c["max_norm_dev"] < 1e-4
    rng = np.random.default_rng(0)
    for shot in rng.choice(N, size=150, replace=False):
        r = circ.shot(5, int(shot))
        assert gpu["status"][shot] == r.status and gpu["abort_op"][shot] == r.abort_op
        rec = [int((gpu["outcomes"][k >> 5, shot] >> (k & 31)) & 1) for k in range(circ.n_records)]
        assert rec == r.record


def test_shard_determinism_and_graph_replay():
    w = workloads.config("cultivation_15q", seed=3)
    ctx = make_ctx(w.text, w.noise, seed=21)
    a = run_gpu(ctx, 0, 40000)
    b1 = run_gpu(ctx, 0, 20000)
    b2 = run_gpu(ctx, 20000, 20000)
    for key in ("status", "abort_op", "obs"):
        assert (a[key] == np.concatenate([b1[key], b2[key]])).all()
    assert (a["outcomes"] == np.concatenate([b1["outcomes"], b2["outcomes"]], axis=1)).all()
    t = torch()
    # the same graph replayed, with the program's own eager work in between
    outs = soft.sample(ctx, 0, 40000)
    for rep in range(4):
        _ = (t.randn(4096, device="cuda") * 2.0).sum().item()
        for o in outs:
            o.zero_()
        ctx.run(0, 40000, *outs)
        t.cuda.synchronize()
        assert (outs[1].cpu().numpy().view(np.uint32) == a["status"]).all()
        got = outs[0].cpu().numpy().view(np.uint32)[: a["outcomes"].shape[0]]
        assert (got == a["outcomes"]).all()


def test_parse_errors_and_degenerate_inputs():
    ctx = soft.Context(0)
    for bad in ("H 0\n", "QUBITS 2\nH 2\n", "QUBITS 2\nCX 1 1\n", "QUBITS 2\nFOO 1\n", "QUBITS 2\nDETECTOR 0 0\n",
                "QUBITS 2\nDEP1 1.5 0\n", "QUBITS 2\nMPP X0*X0\n", "QUBITS 65\n"):
        with pytest.raises(soft.SoftError) as ei:
            ctx.load_circuit(bad)
        assert ei.value.code == soft.SOFT_EPARSE
        with pytest.raises(ValueError):
            oracle.Circuit(bad)
    # empty circuit, zero shots, Clifford-only, p = 1 and p below 2^-32
    for text, noise in (("QUBITS 1\n", {}), ("QUBITS 3\nH 0\nCX 0 1\nM 1\nM 0\n", {}),
                        ("QUBITS 2\nH 0\nT 0\nCX 0 1\nM 0\nM 1\n", {"p1": 1.0, "p2": 1.0}),
                        ("QUBITS 2\nH 0\nT 0\nM 0\n", {"p1": 1e-10})):
        circ = oracle.Circuit(text, noise)
        ctx = make_ctx(text, noise, seed=3, keep=(0, 16))
        ctx.run(0, 0, None, None)
        gpu = run_gpu(ctx, 0, 300)
        compare_batch(gpu, circ.batch(3, 0, 300))
        compare_kept(ctx, circ, 3, range(16))


def test_autotune_keeps_results():
    w = workloads.config("cultivation_15q", seed=1)
    ctx = make_ctx(w.text, w.noise, seed=4)
    base = run_gpu(ctx, 0, 20000)
    ctx.autotune(20000)
    shape = ctx.launch_shape()
    assert 1 <= shape["waves_per_block"] <= 4
    tuned = run_gpu(ctx, 0, 20000)
    for key in ("status", "abort_op", "obs", "outcomes"):
        assert (base[key] == tuned[key]).all()


@pytest.mark.parametrize("seed", range(8))
def test_trace_matches_oracle_step_by_step(seed):
    # The paper's step-by-step cross-check (Sec. V-B): after every event the
    # GPU tableau and coefficient vector equal the oracle's for the same prefix.
    n = 2 + seed % 5
    text, _ = random_circuit(41000 + seed, n, 70, p_msc=0.15 if seed >= 4 else 0.0)
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
        if t["final"] and r.status != oracle.PASSED:
            assert t["status"] == r.status
        assert (t["x"] == r.tab_x).all() and (t["z"] == r.tab_z).all() and (t["r"] == r.tab_r).all(), step
        keys = set(t["coeffs"]) | set(r.coeffs)
        err = max([abs(t["coeffs"].get(a, 0) - r.coeffs.get(a, 0)) for a in keys] + [0.0])
        assert err < 1e-10, (step, lines[t["op"] + 1], err)
        steps += 1
    assert steps >= 5


@pytest.mark.parametrize("mode", [0, 1])
def test_work_counters_closed_forms(mode):
    # T on a fresh |+> qubit adds a span coordinate: the k-th such T writes
    # 2^(k+1) tile entries; a second T on the same qubit is a butterfly over
    # the 2^k entries.  No measurement, no noise: every shot runs every event.
    # The whole list is a shared T prefix: with it on (the default) every
    # shot starts at its end and runs no T work; off, every shot runs it.
    N = 5000
    text = "QUBITS 5\n" + "".join("H %d\n" % q for q in range(5)) + "".join("T %d\n" % q for q in range(5)) + "T 0\n"
    ctx = make_ctx(text, None, seed=3)
    ctx.set_noise_mode(mode)
    run_gpu(ctx, 0, N)
    c = ctx.counters()
    assert c["entries_t"] == 0 and c["events"] == 0 and c["prefix_shots"] == N
    ctx.set_shared_prefix(False)
    run_gpu(ctx, 0, N)
    c = ctx.counters()
    assert c["entries_t"] == N * ((2 + 4 + 8 + 16 + 32) + 32)
    assert c["entries_m"] == 0 and c["events"] == N * 6 and c["noise_slots"] == 0 and c["prefix_shots"] == 0
    # one measurement pass over the 2^5 entries per shot, and a noise table of
    # 3 slots drawn once per shot (per slot: the 3 words; gap sampling: one
    # 256-word block of stream 2)
    text2 = text + "DEP1 0.1 1\nDEP1 0.2 2\nDEP1 0.3 3\nMPP X0\n"
    ctx2 = make_ctx(text2, None, seed=3)
    ctx2.set_noise_mode(mode)
    ctx2.set_shared_prefix(False)
    run_gpu(ctx2, 0, N)
    c2 = ctx2.counters()
    assert c2["entries_t"] == c["entries_t"] and c2["events"] == N * 7
    assert c2["entries_m"] == N * 32
    assert c2["noise_slots"] == N * (3 if mode == 0 else 256)


def test_graph_reused_across_batches():
    # A scan of equal batches launched back to back without synchronizing:
    # one instantiated graph per slot serves every batch (only the sampler
    # node's arguments change), and the batches equal one large run.
    w = workloads.config("cultivation_15q", seed=3)
    t = torch()
    big = make_ctx(w.text, w.noise, seed=29)
    ref = run_gpu(big, 0, 160000)
    ctx = make_ctx(w.text, w.noise, seed=29)
    nb, B = 16, 10000
    outs = [soft.sample(ctx, b * B, B) for b in range(nb)]
    t.cuda.synchronize()
    gi = ctx.graph_info()
    assert gi["launches"] == nb and gi["instantiations"] <= 2
    nw = ref["outcomes"].shape[0]
    for b, (oc, st, ab, ob) in enumerate(outs):
        sl = slice(b * B, (b + 1) * B)
        assert (st.cpu().numpy().view(np.uint32) == ref["status"][sl]).all(), b
        assert (ab.cpu().numpy().view(np.uint32) == ref["abort_op"][sl]).all(), b
        assert (ob.cpu().numpy().view(np.uint32) == ref["obs"][sl]).all(), b
        assert (oc.cpu().numpy().view(np.uint32)[:nw] == ref["outcomes"][:, sl]).all(), b
    # the last batch's counters are its own
    c = ctx.counters()
    assert c["shots"] == B
    assert c["passed"] == int((ref["status"][(nb - 1) * B:] == 0).sum())
    # a different precision instantiates again; going back reuses a slot
    ctx.set_precision(32)
    run_gpu(ctx, 0, B)
    ctx.set_precision(64)
    again = run_gpu(ctx, 0, B)
    assert (again["status"] == ref["status"][:B]).all()
    assert ctx.graph_info()["instantiations"] <= 4


@pytest.mark.parametrize("bits,mode", [(32, 1), (64, 1), (32, 0), (64, 0)])
def test_lean_kernel_equals_full_kernel(bits, mode):
    # A launch with no kept states and no trace runs the lean kernel (those
    # paths compiled out); keeping a few states switches to the full one.
    # Records, statuses, abort ops, observables and the pass / discard /
    # logical counts are the same either way.
    w = workloads.config("cultivation_42q", seed=1)
    res = []
    for keep in (None, (7, 16)):
        ctx = make_ctx(w.text, w.noise, seed=20251223, bits=bits, keep=keep)
        ctx.set_noise_mode(mode)
        res.append((run_gpu(ctx, 0, 400_000), ctx.counters()))
        ctx.close()
    (a, ca), (b, cb) = res
    for k in ("status", "abort_op", "obs", "outcomes"):
        assert (a[k] == b[k]).all(), k
    for f in ("shots", "passed", "discarded", "overflow", "numeric", "logical_errors", "restarts"):
        assert ca[f] == cb[f], f
