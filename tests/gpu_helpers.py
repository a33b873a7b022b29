"""Shared helpers of the GPU parity tests: run the HIP sampler through the
C ABI and the oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2512_23037_amd import soft

KEYS = ("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp")


def torch():
    import torch as _t
    return _t


def make_ctx(text, noise=None, seed=0, bits=64, cap=0, keep=None, tau=-1.0, shape=(0, 0, 0)):
    ctx = soft.Context(0)
    ctx.load_noise(**{k: (noise or {}).get(k, 0.0) for k in KEYS})
    ctx.load_circuit(text)
    ctx.set_rng(seed)
    ctx.set_precision(bits)
    ctx.set_prune(tau)
    ctx.set_caps(cap, *shape)
    if keep is not None:
        ctx.set_keep(*keep)
    return ctx


def run_gpu(ctx, shot0, n, words=None):
    t = torch()
    info = ctx.info()
    wt = None
    if words is not None:
        wt = t.from_numpy(np.ascontiguousarray(words, dtype=np.uint32).view(np.int32)).cuda()
        ctx.set_uniforms(wt, n, info["noise_slots"], info["meas_slots"])
    else:
        ctx.set_uniforms(None)
    outs = soft.sample(ctx, shot0, n)
    t.cuda.synchronize()
    res = {name: x.cpu().numpy().view(np.uint32) for name, x in zip(("outcomes", "status", "abort_op", "obs"), outs)}
    res["outcomes"] = res["outcomes"][: info["record_words"]]
    del wt
    return res


def compare_batch(gpu, ref, skip=None):
    """Bit-exact comparison of outcomes, status, abort op and observables.
    `skip`: boolean mask of shots to leave out."""
    keep = np.ones(len(ref["status"]), dtype=bool) if skip is None else ~skip
    assert (gpu["status"][keep] == ref["status"][keep]).all(), _first_diff(gpu["status"], ref["status"], keep)
    assert (gpu["abort_op"][keep] == ref["abort_op"][keep]).all(), _first_diff(gpu["abort_op"], ref["abort_op"], keep)
    assert (gpu["obs"][keep] == ref["obs"][keep]).all()
    if ref["outcomes"].size:
        assert (gpu["outcomes"][:, keep] == ref["outcomes"][:, keep]).all(), "outcome records differ"


def _first_diff(a, b, keep):
    idx = np.nonzero((a != b) & keep)[0]
    return "first differing shot %s: gpu %s vs oracle %s" % (idx[:5], a[idx[:5]], b[idx[:5]])


def coeff_error(got: dict, ref: dict) -> float:
    """max_alpha |v_gpu - v_ref| / ||v_ref||_2 over the union of supports."""
    keys = set(got) | set(ref)
    norm = np.sqrt(sum(abs(v) ** 2 for v in ref.values())) or 1.0
    return max([abs(got.get(k, 0) - ref.get(k, 0)) for k in keys] + [0.0]) / norm


def compare_kept(ctx, circ, seed, shots, words=None, tol=1e-10, cap=0xFFFFFFFF, tau=1e-12):
    worst = 0.0
    stride = circ.words_per_shot
    for i, shot in enumerate(shots):
        w = None if words is None else words[i * stride:(i + 1) * stride] if words.ndim == 1 else words[i]
        r = circ.shot(seed, shot, words=w, tau=tau, cap=cap)
        x, z, rr = ctx.read_tableau(shot)
        assert (x == r.tab_x).all() and (z == r.tab_z).all(), "tableau x/z differ at shot %d" % shot
        assert (rr == r.tab_r).all(), "tableau signs differ at shot %d" % shot
        err = coeff_error(ctx.read_coeffs(shot), r.coeffs)
        assert err <= tol, "shot %d coefficient error %g" % (shot, err)
        worst = max(worst, err)
    return worst


def oracle_shots(circ, seed, shots, tau=1e-12, cap=0xFFFFFFFF, threads=16):
    """Oracle results of single shots, computed on a pool of host threads (the
    oracle's C calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as pool:
        return list(pool.map(lambda s: circ.shot(seed, int(s), tau=tau, cap=cap), shots))


def compare_kept_many(ctx, circ, seed, shots, tol=1e-10, tau=1e-12):
    """compare_kept for Philox-drawn shots, with the oracle on host threads.
    Returns the largest coefficient error."""
    worst = 0.0
    for shot, r in zip(shots, oracle_shots(circ, seed, shots, tau=tau)):
        x, z, rr = ctx.read_tableau(int(shot))
        assert (x == r.tab_x).all() and (z == r.tab_z).all(), "tableau x/z differ at shot %d" % shot
        assert (rr == r.tab_r).all(), "tableau signs differ at shot %d" % shot
        err = coeff_error(ctx.read_coeffs(int(shot)), r.coeffs)
        assert err <= tol, "shot %d coefficient error %g" % (shot, err)
        worst = max(worst, err)
    return worst


def guard_band_flips(circ, seed, ref_p0_shots, band=1e-5):
    """For each listed oracle result (shot, ShotResult): True when some
    measurement's uniform lies within `band` of the oracle's P(+1), i.e. an
    FP32 run may take the other branch there (the near-tie rule)."""
    out = []
    for shot, r in ref_p0_shots:
        near = False
        for slot in range(circ.n_meas_slots):
            p = r.p0[slot]
            if np.isnan(p):
                continue
            blk = oracle.philox([slot >> 2, int(shot) & 0xFFFFFFFF, int(shot) >> 32, 1],
                                [seed & 0xFFFFFFFF, seed >> 32])
            u = (float(blk[slot & 3]) + 0.5) / 2 ** 32
            near |= abs(u - p) < band
        out.append(near)
    return out
