"""GPU parity on random feature-rich circuits under random library options.

Each seed draws a circuit (Cliffords, T/T-dagger, Z and Pauli-product
measurements, resets, the extended measurement-and-reset set, record-controlled
Paulis, CCZ/CCX, diagonal gates, classically controlled gates, detectors and
an observable), a uniform noise rate, and one setting of every option that
must not change results: per-slot or gap-sampled noise, FP64 or FP32
coefficients, speculative lists, checkpoints of the noiseless trajectory,
deferred T runs, and the tile placement (automatic, LDS, device memory,
split).  Records, statuses, abort ops and observables are compared with the
oracle on 1500 shots (FP64 bit-exact; FP32 may differ only where a
measurement's uniform lies within 1e-5 of the oracle's probability), and the
final tableau and coefficients of shots 0..63 (1e-10 FP64, 1e-5 FP32).
A second group runs the same circuits in FP64 through the other ways in:
shot offsets up to 2^40, support caps (overflow statuses, counters and the
tableau at the abort), shot lists in any order, explicit per-shot words, and
the no-alloc entry point against the regular one.  A third group puts 2-6 of
these circuits and noise models in one mixed launch, and a fourth checks the
state after every event of one shot against the oracle on the prefix."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2512_23037_amd import soft
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import (coeff_error, compare_batch, compare_kept, compare_kept_many, guard_band_flips, make_ctx,
                               run_gpu, torch)

pytestmark = pytest.mark.gpu

N = 1500
KEPT = 64
REC_OPS = ("M ", "MPP", "MX ", "MR ", "MRX")


def draw_case(seed):
    """The circuit text, noise model and options of one seed."""
    rng = np.random.default_rng(seed)
    big = seed % 3 == 0
    n = int(rng.integers(2, 15 if big else 11))
    length = int(rng.integers(60, 500 if big else 240))
    text, _ = random_circuit(880000 + seed, n, length, p_t=float(rng.uniform(0.05, 0.3)),
                             p_meas=float(rng.uniform(0.03, 0.12)), p_msc=0.05, p_ccz=0.02 if n >= 3 else 0.0,
                             p_diag=0.03, p_if=0.03)
    lines = text.strip().split("\n")
    head = []
    if n <= 10 and rng.random() < 0.5:  # grow the span early
        head = ["H %d\nT %d" % (q, q) for q in range(n)]
    out = [lines[0]] + head
    nrec = 0
    pdet = float(rng.choice([0.0, 0.03, 0.1]))
    for line in lines[1:]:
        out.append(line)
        if line.startswith(REC_OPS):
            nrec += 1
            if rng.random() < pdet:
                k = int(rng.integers(1, min(3, nrec) + 1))
                recs = rng.choice(nrec, size=k, replace=False)
                out.append("DETECTOR %d %s" % (int(rng.integers(2)), " ".join(str(int(r)) for r in recs)))
    if nrec:
        out.append("OBSERVABLE 0 %d" % int(rng.integers(nrec)))
    text = "\n".join(out) + "\n"
    p = float(rng.choice([0.0, 0.002, 0.01, 0.03]))
    noise = {"p1": p, "p2": p, "p_meas": p, "p_reset": p, "p_mpp": p}
    opts = {"mode": int(rng.integers(2)), "bits": 64 if rng.random() < 0.7 else 32}
    opts["spec"], opts["prefix"], opts["defer"] = (bool(rng.integers(2)) for _ in range(3))
    opts["tile"] = int(rng.integers(4))
    opts["lds_log2"] = 7 if rng.random() < 0.5 else 0
    return text, noise, opts


def run_case(seed):
    text, noise, o = draw_case(seed)
    circ = oracle.Circuit(text, noise, noise_mode=o["mode"])
    ctx = make_ctx(text, noise, seed=seed, bits=o["bits"], keep=(0, KEPT))
    ctx.set_noise_mode(o["mode"])
    ctx.set_speculation(o["spec"])
    ctx.set_shared_prefix(o["prefix"])
    ctx.set_deferred_t(o["defer"])
    kmax = ctx.info()["k_max"]
    tile = 2 if (o["tile"] == 3 and kmax < 8) else o["tile"]  # a split tile needs a span of 2^8
    ctx.set_tile_memory(tile, o["lds_log2"] if tile == 3 else 0)
    print("seed %d n=%d k_max=%d %s noise %g tile %d" % (seed, circ.n_qubits, kmax, o, noise["p1"], tile), flush=True)
    gpu = run_gpu(ctx, 0, N)
    ref = circ.batch(seed, 0, N)
    if o["bits"] == 64:
        compare_batch(gpu, ref)
        compare_kept_many(ctx, circ, seed, list(range(KEPT)))
    else:
        diff = (gpu["status"] != ref["status"]) | (gpu["abort_op"] != ref["abort_op"]) | (gpu["obs"] != ref["obs"])
        if ref["outcomes"].size:
            diff |= (gpu["outcomes"] != ref["outcomes"]).any(axis=0)
        bad = np.nonzero(diff)[0]
        assert len(bad) <= 10
        res = [circ.shot(seed, int(s)) for s in bad]
        assert all(guard_band_flips(circ, seed, list(zip(bad, res)))), "FP32 difference outside the guard band"
        compare_batch(gpu, ref, skip=diff)
        compare_kept_many(ctx, circ, seed, [s for s in range(KEPT) if not diff[s]], tol=1e-5, tau=1e-6)
    ctx.close()


@pytest.mark.parametrize("chunk", range(12))
def test_random_circuits_random_options(chunk):
    for seed in range(150 + 16 * chunk, 150 + 16 * (chunk + 1)):
        run_case(seed)


def _outs(ctx, n):
    t = torch()
    nw = ctx.info()["record_words"]
    return [t.zeros((max(nw, 1), n), dtype=t.int32, device="cuda")] + \
        [t.zeros(n, dtype=t.int32, device="cuda") for _ in range(3)]


def _host(outs, nw):
    d = {k: x.cpu().numpy().view(np.uint32) for k, x in zip(("outcomes", "status", "abort_op", "obs"), outs)}
    d["outcomes"] = d["outcomes"][:nw]
    return d


def run_entry_case(seed):
    text, noise, o = draw_case(seed)
    rng = np.random.default_rng(10 ** 6 + seed)
    kind = int(rng.integers(4))  # offset, cap, list, explicit words + no-alloc
    circ = oracle.Circuit(text, noise, noise_mode=o["mode"])
    n = 1000
    print("seed %d kind %d n=%d %s" % (seed, kind, circ.n_qubits, o), flush=True)
    if kind == 0:
        shot0 = int(rng.integers(1, 1 << 40))
        ctx = make_ctx(text, noise, seed=seed, keep=(shot0 + 7, 32))
        ctx.set_noise_mode(o["mode"])
        ctx.set_deferred_t(o["defer"])
        compare_batch(run_gpu(ctx, shot0, n), circ.batch(seed, shot0, n))
        compare_kept_many(ctx, circ, seed, list(range(shot0 + 7, shot0 + 39)))
    elif kind == 1:
        cap = int(2 ** rng.integers(0, 7))
        ctx = make_ctx(text, noise, seed=seed, cap=cap, keep=(0, 32))
        ctx.set_noise_mode(o["mode"])
        gpu = run_gpu(ctx, 0, n)
        ref = circ.batch(seed, 0, n, cap=cap)
        compare_batch(gpu, ref)
        assert ctx.counters()["overflow"] == int((ref["status"] == oracle.OVERFLOW).sum())
        for s in range(32):
            r = circ.shot(seed, s, cap=cap)
            x, z, rr = ctx.read_tableau(s)
            assert (x == r.tab_x).all() and (z == r.tab_z).all() and (rr == r.tab_r).all(), "tableau of shot %d" % s
    elif kind == 2:
        shots = rng.choice(1 << 36, size=n, replace=False).astype(np.int64)
        ctx = make_ctx(text, noise, seed=seed)
        ctx.set_noise_mode(o["mode"])
        ctx.set_deferred_t(o["defer"])
        ctx.set_shared_prefix(o["prefix"])
        nw = ctx.info()["record_words"]
        outs = _outs(ctx, n)
        ctx.run_list(torch().from_numpy(shots).cuda(), *outs)
        torch().cuda.synchronize()
        gpu = _host(outs, nw)
        for i in rng.choice(n, size=100, replace=False):
            r = circ.batch(seed, int(shots[i]), 1)
            for k in ("status", "abort_op", "obs"):
                assert gpu[k][i] == r[k][0], (k, int(shots[i]))
            if nw:
                assert (gpu["outcomes"][:, i] == r["outcomes"][:, 0]).all(), ("outcomes", int(shots[i]))
    else:
        circ0 = oracle.Circuit(text, noise)
        words = random_words(seed, n * circ0.words_per_shot).reshape(n, circ0.words_per_shot)
        ctx = make_ctx(text, noise, seed=seed, keep=(0, 64))
        ctx.set_deferred_t(o["defer"])
        compare_batch(run_gpu(ctx, 0, n, words), circ0.batch(0, 0, n, words=words))
        compare_kept(ctx, circ0, 0, range(64), words=words)
        ctx.close()
        ctx = make_ctx(text, noise, seed=seed)
        ctx.set_noise_mode(o["mode"])
        ref = run_gpu(ctx, 0, n)
        nw = ctx.info()["record_words"]
        outs = _outs(ctx, n)
        ctx.run_noalloc(0, n, *outs)
        torch().cuda.synchronize()
        got = _host(outs, nw)
        for k in ("status", "abort_op", "obs", "outcomes"):
            assert (got[k] == ref[k]).all(), ("no-alloc", k)
    ctx.close()


@pytest.mark.parametrize("chunk", range(4))
def test_random_circuits_every_entry(chunk):
    for seed in range(600 + 16 * chunk, 600 + 16 * (chunk + 1)):
        run_entry_case(seed)


def run_mixture_case(seed):
    """2-6 of the random circuits and noise models in one launch (random range
    sizes, the first variant's options): each range against its own variant's
    oracle, per-variant counters, and the states around the first boundary."""
    rng = np.random.default_rng(2 * 10 ** 6 + seed)
    nv = int(rng.integers(2, 7))
    cases = [draw_case(5000 + seed * 8 + j) for j in range(nv)]
    ends = [int(x) for x in np.cumsum(rng.integers(50, 500, size=nv))]
    o = cases[0][2]
    keys = ("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp")
    models = [{k: c[1].get(k, 0.0) for k in keys} for c in cases]
    print("seed %d: %d variants, %d shots, %s" % (seed, nv, ends[-1], o), flush=True)
    ctx = soft.Context(0)
    ctx.load_mixture([c[0] for c in cases], models, ends)
    ctx.set_rng(seed)
    ctx.set_precision(64)
    ctx.set_noise_mode(o["mode"])
    ctx.set_speculation(o["spec"])
    ctx.set_shared_prefix(o["prefix"])
    ctx.set_deferred_t(o["defer"])
    tile = 2 if (o["tile"] == 3 and ctx.info()["k_max"] < 8) else o["tile"]
    ctx.set_tile_memory(tile, o["lds_log2"] if tile == 3 else 0)
    b = ends[0]
    ctx.set_keep(b - 16, 32)
    gpu = run_gpu(ctx, 0, ends[-1])
    lo, circs = 0, []
    for v, ((text, _, _), hi) in enumerate(zip(cases, ends)):
        circ = oracle.Circuit(text, models[v], noise_mode=o["mode"])
        circs.append(circ)
        ref = circ.batch(seed, lo, hi - lo)
        sub = {k: (x[:, lo:hi] if x.ndim == 2 else x[lo:hi]) for k, x in gpu.items()}
        nw = (circ.n_records + 31) // 32
        assert not sub["outcomes"][nw:].any(), "record words past the variant's records must stay 0"
        sub["outcomes"] = sub["outcomes"][:nw]
        compare_batch(sub, ref)
        cv = ctx.counters(v)
        assert cv["shots"] == hi - lo and cv["passed"] == int((ref["status"] == 0).sum()), v
        lo = hi
    for shot in range(b - 16, b + 16):
        r = circs[ctx.variant_of(shot)].shot(seed, shot)
        x, z, rr = ctx.read_tableau(shot)
        assert (x == r.tab_x).all() and (z == r.tab_z).all() and (rr == r.tab_r).all(), shot
        assert coeff_error(ctx.read_coeffs(shot), r.coeffs) < 1e-10, shot
    ctx.close()


@pytest.mark.parametrize("chunk", range(2))
def test_random_mixtures(chunk):
    for seed in range(16 * chunk, 16 * (chunk + 1)):
        run_mixture_case(seed)


def run_trace_case(seed):
    """The state after every event of one shot (Sec. V-B's step-by-step
    check) against the oracle run on the circuit's prefix.  Even seeds drop
    the detectors so that the shot runs every event."""
    text, _, o = draw_case(seed)
    if seed % 2 == 0:
        text = "\n".join(x for x in text.strip().split("\n") if not x.startswith("DETECTOR")) + "\n"
    lines = text.strip().split("\n")
    circ = oracle.Circuit(text)
    words = random_words(seed, circ.words_per_shot)
    bits = o["bits"]
    tau = 1e-12 if bits == 64 else 1e-6
    ctx = make_ctx(text, bits=bits, tau=tau)
    kmax = ctx.info()["k_max"]
    tile = 2 if (o["tile"] == 3 and kmax < 8) else o["tile"]
    if tile == 1 and kmax > 12:
        tile = 0
    ctx.set_tile_memory(tile, o["lds_log2"] if tile == 3 else 0)
    events = ctx.info()["events"]
    ctx.set_trace(0, events)
    run_gpu(ctx, 0, 1, words.reshape(1, -1))
    steps = 0
    for step in range(events):
        t = ctx.read_trace(step)
        if t is None:
            break
        upto = lines[: t["op"] + 2]
        tok = upto[-1].split() if t["op"] + 1 < len(lines) else []
        if "CCX" in tok:  # the event is the CCZ of H_t CCZ H_t
            i = tok.index("CCX")
            upto[-1] = "H %s\n%s" % (tok[i + 3], " ".join(tok[:i] + ["CCZ"] + tok[i + 1:]))
        pc = oracle.Circuit("\n".join(upto) + "\n")
        r = pc.shot(0, 0, words=words[: pc.words_per_shot], tau=tau)
        if t["final"] and r.status != oracle.PASSED:
            assert t["status"] == r.status, step
        assert (t["x"] == r.tab_x).all() and (t["z"] == r.tab_z).all() and (t["r"] == r.tab_r).all(), step
        assert coeff_error(t["coeffs"], r.coeffs) < (1e-10 if bits == 64 else 1e-5), (step, upto[-1])
        steps += 1
    ctx.close()
    return steps


@pytest.mark.parametrize("chunk", range(2))
def test_random_traces_step_by_step(chunk):
    steps = sum(run_trace_case(seed) for seed in range(16 * chunk, 16 * (chunk + 1)))
    assert steps > 500
