"""soft_run_noalloc (the entry point for callers that cannot allocate device
memory) against soft_run, through the C ABI: two calls in a row, the second
with fewer shots, must give soft_run's records, statuses, abort ops,
observables and counters bit for bit -- with LDS tiles and with
device-memory tiles or the device-memory parts of split tiles in the static
scratch -- and the call must build no
graph.  Also its error paths: no circuit, kept states on, slabs of one
block larger than the scratch."""
from __future__ import annotations

import numpy as np
import pytest

import workloads
from paper_2512_23037_amd import soft
from tests.gen_small import random_circuit, random_words
from tests.gpu_helpers import make_ctx

pytestmark = pytest.mark.gpu

FIELDS = ("shots", "passed", "discarded", "overflow", "numeric", "logical_errors", "restarts", "prefix_shots")
# work run, and the supports and norms of what was computed: the same when
# both calls start the same shots from checkpoints (the no-alloc call keeps
# checkpoint slots only while they fit its scratch; a shot started elsewhere
# may skip a different set of deferred T runs)
WORK = ("entries_t", "entries_m", "noise_slots", "events", "redo_shots")


def _outputs(ctx, n):
    import torch
    nw = max(ctx.info()["record_words"], 1)
    return [torch.full((nw, n), -7, dtype=torch.int32, device="cuda")] + \
        [torch.full((n,), -7, dtype=torch.int32, device="cuda") for _ in range(3)]


def _run(ctx, shot0, n, noalloc):
    import torch
    outs = _outputs(ctx, n)
    (ctx.run_noalloc if noalloc else ctx.run)(shot0, n, *outs)
    torch.cuda.synchronize()
    c = ctx.counters()
    return [o.cpu().numpy().view(np.uint32) for o in outs], c


def _same(a, b):
    (oa, ca), (ob, cb) = a, b
    for x, y in zip(oa, ob):
        assert (x == y).all()
    same_start = ca["prefix_shots"] == cb["prefix_shots"]
    for f in FIELDS + (WORK if same_start else ()):
        if f == "prefix_shots" and not same_start:
            continue
        assert ca[f] == cb[f], f
    if same_start:
        assert list(ca["support_hist"]) == list(cb["support_hist"])
        assert ca["max_norm_dev"] == cb["max_norm_dev"]
    return same_start


@pytest.mark.parametrize("tiles", [1, 2, 3])
@pytest.mark.parametrize("bits", [32, 64])
def test_noalloc_equals_soft_run_two_calls(tiles, bits):
    w = workloads.config("cultivation_42q", seed=1)
    ctx = soft.Context(0)
    ctx.load_noise(**w.noise)
    ctx.load_circuit(w.text)
    ctx.set_rng(20251223)
    ctx.set_precision(bits)
    ctx.set_noise_mode(1)
    ctx.set_tile_memory(tiles)
    for shot0, n in ((1000, 300000), (5, 40000)):  # the second call is smaller
        ref = _run(ctx, shot0, n, noalloc=False)
        g0 = ctx.graph_info()
        got = _run(ctx, shot0, n, noalloc=True)
        assert ctx.graph_info() == g0  # no graph built or launched
        assert _same(got, ref)  # one circuit: its checkpoint slots fit the scratch
        assert ref[1]["shots"] == n and ref[1]["discarded"] > 0


def test_noalloc_explicit_words_and_mixture():
    text, _ = random_circuit(81000, 6, 150, p_diag=0.05, p_if=0.05)
    ctx = make_ctx(text)
    info = ctx.info()
    stride = info["noise_slots"] + info["meas_slots"]
    import torch
    for n in (3000, 700):
        words = torch.from_numpy(random_words(n, n * stride).view(np.int32)).cuda()
        ctx.set_uniforms(words, n, info["noise_slots"], info["meas_slots"])
        _same(_run(ctx, 0, n, True), _run(ctx, 0, n, False))
        del words
    ctx.set_uniforms(None)
    mix = workloads.mixture(seed=1, total_shots=200000)
    m = soft.Context(0)
    m.load_mixture([w.text for w in mix["workloads"]], mix["models"], mix["shot_ends"])
    m.set_rng(3)
    m.set_precision(64)
    for shot0, n in ((0, 200000), (50000, 60000)):
        _same(_run(m, shot0, n, True), _run(m, shot0, n, False))


def test_noalloc_error_paths():
    import torch
    w = workloads.config("cultivation_15q", seed=1)
    ctx = soft.Context(0)
    status = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(soft.SoftError, match="no circuit"):
        ctx.run_noalloc(0, 16, None, status)
    ctx.load_noise(**w.noise)
    ctx.load_circuit(w.text)  # uploads the tables
    outs = _outputs(ctx, 16)
    ctx.set_keep(0, 4)
    with pytest.raises(soft.SoftError, match="kept states"):
        ctx.run_noalloc(0, 16, *outs)
    ctx.set_keep(0, 0)
    ctx.run_noalloc(0, 16, *outs)
    ctx.run_noalloc(0, 0)  # nothing to do
    # span 20 in FP64 with device-memory tiles: one wave's slab is 16 MiB,
    # four waves per block need more than the scratch's 32 MiB
    big = "QUBITS 20\n" + "".join("H %d\nT %d\n" % (q, q) for q in range(20)) + "M 0\n"
    b = soft.Context(0)
    b.load_circuit(big)
    b.set_precision(64)
    b.set_tile_memory(2)
    b.set_caps(0, 4, 1, 1)
    outs = _outputs(b, 4)
    with pytest.raises(soft.SoftError, match="scratch holds"):
        b.run_noalloc(0, 4, *outs)
