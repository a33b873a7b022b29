"""GPU parity of the speculative event lists on bracket circuits: a T/T-dagger
layer, a commuting check round, and the inverse layer in another order (held
back and emitted latest-opened first, with the span dropped step by step),
optionally with idle noise inside the inverse layer.  Results with speculation
must equal the oracle's and the full list's bit for bit (FP64), caps that
force OVERFLOW included."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import coeff_error, compare_batch, compare_kept, make_ctx, run_gpu

pytestmark = pytest.mark.gpu


SHAPES = [(7, 8, 3, [7, 4], 4), (9, 6, 3, [9, 5], 6), (8, 6, 2, [8], 6), (10, 6, 3, [10, 6, 3], 6)]


def bracket_circuit(seed: int):
    """A small cultivation-shaped circuit whose inverse layers run in another
    order than their layers (and, for every third seed, with a TICK inside)."""
    nd, na, rz, br, w = SHAPES[seed % len(SHAPES)]
    order = "shuffled_tick" if seed % 3 == 0 else "shuffled"
    return workloads.cultivation_shaped(100 + seed, nd, na, rz, br, check_weight=w, inverse_order=order)


@pytest.mark.parametrize("seed", range(12))
def test_bracket_circuits_match_oracle_and_full_list(seed):
    text = bracket_circuit(seed).text
    p = [0.0, 0.002, 0.02][seed % 3]
    noise = {"p1": p, "p2": p, "p_idle": p, "p_meas": p, "p_reset": p, "p_mpp": p}
    circ = oracle.Circuit(text, noise)
    N = 20000
    ref = circ.batch(40 + seed, 0, N)
    outs = {}
    for spec in (True, False):
        ctx = make_ctx(text, noise, seed=40 + seed, keep=(0, 64))
        ctx.set_speculation(spec)
        outs[spec] = run_gpu(ctx, 0, N)
        compare_batch(outs[spec], ref)
        compare_kept(ctx, circ, 40 + seed, range(64))
        c = ctx.counters()
        if not spec or p == 0.0:
            assert c["restarts"] == 0
        if spec and p == 0.02:
            assert c["restarts"] > 0
        ctx.close()
    for key in ("status", "abort_op", "obs", "outcomes"):
        assert (outs[True][key] == outs[False][key]).all()


@pytest.mark.parametrize("seed", [1, 4, 7])
def test_bracket_circuits_capped(seed):
    # Caps below the layer's peak support: shots overflow in the T layer, and
    # the speculative list (which visits other supports in the inverse layer)
    # must report the full list's statuses and abort ops.
    text = bracket_circuit(seed).text
    noise = {"p1": 0.01, "p2": 0.01, "p_idle": 0.0, "p_meas": 0.01, "p_reset": 0.01, "p_mpp": 0.0}
    circ = oracle.Circuit(text, noise)
    N = 8000
    for cap in (4, 16):
        ref = circ.batch(9, 0, N, cap=cap)
        ctx = make_ctx(text, noise, seed=9, cap=cap)
        compare_batch(run_gpu(ctx, 0, N), ref)
        ctx.close()


@pytest.mark.parametrize("noise_mode,bits", [(0, 64), (1, 64), (1, 32)])
def test_42q_speculative_list_equals_full_list(noise_mode, bits):
    # The benchmark workload at scale: the speculative list (reordered layers,
    # folded drops, fused runs of doublings and of dropping butterflies) must
    # give the full list's records, statuses, abort ops and observables for
    # every shot (FP64; FP32 may differ only at near-ties of the two summation
    # orders), with restarts where noise broke a cancellation, and the same
    # final coefficients for the 512 kept shots (restarted ones among them):
    # within 1e-10 in FP64, 1e-5 in FP32.
    w = workloads.config("cultivation_42q", seed=1)
    N = 2_000_000
    K = 512
    outs, restarts, kept = {}, {}, {}
    for spec in (True, False):
        ctx = make_ctx(w.text, w.noise, seed=20251223, bits=bits, keep=(0, K))
        ctx.set_noise_mode(noise_mode)
        ctx.set_speculation(spec)
        outs[spec] = run_gpu(ctx, 0, N)
        restarts[spec] = ctx.counters()["restarts"]
        kept[spec] = [ctx.read_coeffs(s_) for s_ in range(K)]
        if spec:
            # the kept range itself holds restarted shots
            run_gpu(ctx, 0, K)
            assert ctx.counters()["restarts"] > 0
        ctx.close()
    assert restarts[False] == 0 and restarts[True] > 0
    diff = (outs[True]["status"] != outs[False]["status"]) | (outs[True]["outcomes"] != outs[False]["outcomes"]).any(axis=0)
    assert diff.sum() == 0 if bits == 64 else diff.sum() <= 4
    for key in ("status", "abort_op", "obs"):
        assert (outs[True][key][~diff] == outs[False][key][~diff]).all(), key
    tol = 1e-10 if bits == 64 else 1e-5
    worst = 0.0
    for s_ in range(K):
        if not diff[s_]:
            err = coeff_error(kept[True][s_], kept[False][s_])
            assert err < tol, (s_, err)
            worst = max(worst, err)
    print("bits=%d mode=%d worst speculative-vs-full coefficient difference %.3g" % (bits, noise_mode, worst))
