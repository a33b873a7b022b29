"""Command line for long runs: a noise scan with logical error rates and
intervals, a throughput-against-batch-size sweep, or a throughput-against-
noise-rate sweep.

  python -m paper_2512_23037_amd.scan --circuit FILE --p 2.5e-4,5e-4,1e-3 \\
         --shots-per-p 1000000000 --batch 10000000 --bits 32
  python -m paper_2512_23037_amd.scan --workload cultivation_42q --p 1e-3 --sweep 4096,65536,1048576
  python -m paper_2512_23037_amd.scan --workload cultivation_42q --p 1e-4,1e-3,1e-2 --p-sweep --shots-per-p 1e7

(--workload names a generator of the repository's `workloads` module.)

One JSON line per noise rate (or per batch size) on stdout, progress on
stderr.
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2512_23037_amd.scan")
    src = ap.add_mutually_exclusive_group(required=True)
    src.add_argument("--circuit", help="circuit text file")
    src.add_argument("--workload", help="name of a seeded generator in the workloads module (seed 1)")
    ap.add_argument("--p", default="1e-3", help="comma-separated circuit-level noise rates")
    ap.add_argument("--shots-per-p", type=float, default=1e7)
    ap.add_argument("--batch", type=float, default=1e7)
    ap.add_argument("--bits", type=int, default=32)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--sweep", default="", help="comma-separated shots per launch: throughput sweep instead of a scan")
    ap.add_argument("--autotune", type=float, default=0, help="tune the launch shape on this many shots first")
    ap.add_argument("--p-sweep", action="store_true",
                    help="throughput at each noise rate, --shots-per-p shots per launch (instead of a scan)")
    ap.add_argument("--noise-mode", type=int, default=0, choices=(0, 1),
                    help="0: a noise word per location, 1: gap sampling")
    args = ap.parse_args(argv)
    if args.circuit:
        text = open(args.circuit).read()
    else:
        import workloads
        text = workloads.config(args.workload, seed=1).text
    ps = [float(x) for x in args.p.split(",") if x]

    import torch  # noqa: F401  (loads the HIP runtime before the library)

    from . import soft, stats

    if args.p_sweep:
        for row in stats.p_sweep(text, ps, int(args.shots_per_p), bits=args.bits, seed=args.seed,
                                 noise_mode=args.noise_mode):
            row.update({"bits": args.bits, "noise_mode": args.noise_mode})
            print(json.dumps(row), flush=True)
        return 0

    if args.sweep:
        sizes = [int(float(x)) for x in args.sweep.split(",") if x]
        ctx = soft.Context(0)
        ctx.load_noise(**{k: ps[0] for k in ("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp")})
        ctx.load_circuit(text)
        ctx.set_rng(args.seed)
        ctx.set_precision(args.bits)
        ctx.set_noise_mode(args.noise_mode)
        for row in stats.batch_sweep(ctx, sizes):
            row.update({"p": ps[0], "bits": args.bits})
            print(json.dumps(row), flush=True)
        return 0

    def progress(done, total, secs):
        print("scan: %d / %d shots, %.1f s" % (done, total, secs), file=sys.stderr, flush=True)

    rows = stats.noise_scan(text, ps, int(args.shots_per_p), int(args.batch), bits=args.bits, seed=args.seed,
                            progress=progress, autotune=int(args.autotune), noise_mode=args.noise_mode)
    for r in rows:
        r["bits"] = args.bits
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
