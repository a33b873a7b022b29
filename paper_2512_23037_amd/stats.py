"""Statistics layer over the sampler: long runs in batches, logical error
rates with intervals, discard rates, and throughput sweeps.

* ``wilson``: the Wilson score interval of a binomial proportion.
* ``bayes_factor_interval``: the LER hypotheses whose binomial likelihood is
  within a given factor (1000 in the paper's Sec. IV figures) of the
  maximum-likelihood hypothesis.
* ``run_batches``: run shots [shot0, shot0 + total) of a loaded context in
  launches of ``batch`` shots (each launch is the library's captured graph),
  summing the device counters of every variant.
* ``noise_scan``: one circuit at several noise rates, as the variants of one
  mixture, so every batch is a single persistent launch; reports per rate the
  LER with both intervals, the discard rate and the throughput.

Everything here is host-side bookkeeping: the shots themselves run in the
HIP kernels behind the C ABI.
"""
from __future__ import annotations

import math
import time

Z95 = 1.959963984540054  # two-sided 95% normal quantile


def wilson(k: int, n: int, z: float = Z95) -> tuple[float, float]:
    """Wilson score interval for k successes in n trials."""
    if n <= 0:
        return (0.0, 1.0)
    ph = k / n
    den = 1.0 + z * z / n
    mid = (ph + z * z / (2 * n)) / den
    half = z * math.sqrt(ph * (1.0 - ph) / n + z * z / (4.0 * n * n)) / den
    return (max(0.0, mid - half), min(1.0, mid + half))


def _loglik(k: int, n: int, p: float) -> float:
    out = 0.0
    if k:
        out += k * math.log(p) if p > 0.0 else -math.inf
    if n - k:
        out += (n - k) * math.log1p(-p) if p < 1.0 else -math.inf
    return out


def bayes_factor_interval(k: int, n: int, factor: float = 1000.0) -> tuple[float, float]:
    """[lo, hi] = {p : L(p_hat) / L(p) <= factor} for the binomial likelihood
    L(p) = p^k (1-p)^(n-k), found by bisection on each side of p_hat = k/n."""
    if n <= 0:
        return (0.0, 1.0)
    ph = k / n
    target = _loglik(k, n, ph) - math.log(factor)

    def root(a: float, b: float) -> float:
        # log L(a) >= target > log L(b) (or the reverse); 200 halvings reach double precision
        fa = _loglik(k, n, a) >= target
        for _ in range(200):
            m = 0.5 * (a + b)
            if (_loglik(k, n, m) >= target) == fa:
                a = m
            else:
                b = m
        return 0.5 * (a + b)

    lo = 0.0 if k == 0 or _loglik(k, n, 0.0) >= target else root(ph, 0.0)
    hi = 1.0 if k == n or _loglik(k, n, 1.0) >= target else root(ph, 1.0)
    return (lo, hi)


def run_batches(ctx, shot0: int, total: int, batch: int, stream=None, progress=None) -> dict:
    """Run `total` shots in launches of at most `batch` shots with status-only
    outputs; return the summed counters per variant and the elapsed time."""
    import torch

    nv = 1 if ctx._ends is None else len(ctx._ends)
    status = torch.empty(min(batch, total), dtype=torch.int32, device="cuda")
    sums = [None] * nv
    stream = stream or torch.cuda.current_stream()
    torch.cuda.synchronize()
    g0 = ctx.graph_info()
    t0 = time.perf_counter()
    done = 0
    while done < total:
        n = min(batch, total - done)
        ctx.run(shot0 + done, n, status=status, stream=stream)
        for v in range(nv):  # reading the counters synchronizes the stream
            c = ctx.counters(v)
            if sums[v] is None:
                sums[v] = dict(c)
            else:
                for key, val in c.items():
                    if key == "support_hist":
                        sums[v][key] = [a + b for a, b in zip(sums[v][key], val)]
                    elif key == "max_norm_dev":
                        sums[v][key] = max(sums[v][key], val)
                    else:
                        sums[v][key] += val
        done += n
        if progress:
            progress(done, total, time.perf_counter() - t0)
    g1 = ctx.graph_info()
    return {"variants": sums, "seconds": time.perf_counter() - t0,
            "graph_instantiations": g1["instantiations"] - g0["instantiations"],
            "launches": g1["launches"] - g0["launches"]}


def rates(c: dict) -> dict:
    """LER (logical errors among passed shots) with its intervals, and the
    discard rate, from one counter dict."""
    k, n = int(c["logical_errors"]), int(c["passed"])
    return {"shots": int(c["shots"]), "passed": n, "logical_errors": k,
            "discard_rate": c["discarded"] / max(1, c["shots"]),
            "ler": k / n if n else float("nan"),
            "ler_wilson95": wilson(k, n), "ler_bayes1000": bayes_factor_interval(k, n),
            "overflow": int(c["overflow"]), "numeric": int(c["numeric"])}


def noise_scan(text: str, ps, shots_per_p: int, batch: int, bits: int = 32, seed: int = 0,
               noise_keys=("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp"), progress=None,
               autotune: int = 0, noise_mode: int = 0) -> list[dict]:
    """One circuit at each rate of `ps` (uniform circuit-level noise), run as
    the variants of one mixture over consecutive global shot ranges.  With
    autotune > 0 the launch shape and tile placement are tuned on that many
    shots first (outside the timed scan)."""
    from . import soft

    ctx = soft.Context(0)
    ends = [shots_per_p * (i + 1) for i in range(len(ps))]
    ctx.load_mixture([text] * len(ps), [{k: p for k in noise_keys} for p in ps], ends)
    ctx.set_rng(seed)
    ctx.set_precision(bits)
    ctx.set_noise_mode(noise_mode)
    if autotune:
        ctx.autotune(autotune)
    shape = ctx.launch_shape()
    res = run_batches(ctx, 0, shots_per_p * len(ps), batch, progress=progress)
    rows = []
    for p, c in zip(ps, res["variants"]):
        r = rates(c)
        r["p"] = p
        rows.append(r)
    total = shots_per_p * len(ps)
    for r in rows:
        r["scan_shots_per_s"] = total / res["seconds"]
        r["launch"] = shape
    ctx.close()
    return rows


def batch_sweep(ctx, sizes, reps: int = 3) -> list[dict]:
    """Throughput against the number of shots per launch (the saturation
    curve): for each size, the best of `reps` timed launches."""
    import torch

    out = []
    status = torch.empty(max(sizes), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    for n in sizes:
        ctx.run(0, n, status=status, stream=stream)  # warm-up and graph capture
        best = math.inf
        for r in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.run(0, n, status=status, stream=stream)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
        out.append({"shots": n, "seconds": best, "shots_per_s": n / best})
    return out


def p_sweep(text: str, ps, shots: int, bits: int = 32, seed: int = 0, noise_mode: int = 0, reps: int = 3,
            noise_keys=("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp")) -> list[dict]:
    """Throughput against the noise rate (uniform circuit-level noise at each
    p of `ps`): one context per rate, `shots` per launch, the best of `reps`
    timed launches after a warm-up, with the discard rate and the work per
    shot from the device counters of the last launch.  Noise changes where
    shots stop, so it changes the work per shot."""
    import torch

    from . import soft

    out = []
    stream = torch.cuda.current_stream()
    status = torch.empty(shots, dtype=torch.int32, device="cuda")
    for p in ps:
        ctx = soft.Context(0)
        ctx.load_noise(**{k: p for k in noise_keys})
        ctx.load_circuit(text)
        ctx.set_rng(seed)
        ctx.set_precision(bits)
        ctx.set_noise_mode(noise_mode)
        ctx.run(0, shots, status=status, stream=stream)  # warm-up and graph capture
        best = math.inf
        for r in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.run((r + 1) * shots, shots, status=status, stream=stream)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
        c = ctx.counters()
        n = max(1, int(c["shots"]))
        out.append({"p": p, "shots": shots, "seconds": best, "shots_per_s": shots / best,
                    "discard_rate": c["discarded"] / n, "ler": c["logical_errors"] / max(1, c["passed"]),
                    "t_entries_per_shot": c["entries_t"] / n, "events_per_shot": c["events"] / n,
                    "noise_words_per_shot": c["noise_slots"] / n, "restarts": int(c["restarts"])})
        ctx.close()
    return out
