"""Benchmark of the SVT linearized fit on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one svt_fit_events request over the scaled-up plain-fit workload
(3000 events x 64 roads, 1-4 hits per layer, 72 sectors, lattice constants,
planted tracks; 192,000 roads, ~7.5 M combinations) with inputs and results
resident in HBM.  Inputs rotate over distinct copies so that the timed
passes read HBM rather than the 256 MB last-level cache.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(batch) -> int:
    """Bytes the method must move once: every input word read once, every
    result word written once (constants: 12 KB, once per launch)."""
    nr, ne, nh = batch.n_roads, batch.n_events, batch.n_hits
    inputs = 4 * (ne + 1) + nr * (1 + 4 + 4 + 4) + 4 + 2 * nh
    outputs = nr * (4 + 4 + 4 + 8 + 12 + 4) + 4 * ne
    consts = 72 * 42 * 4
    return inputs + outputs + consts


def cpu_baseline(batch, consts, min_seconds=10.0, max_reps=50):
    import oracle
    oracle.build(force=False)
    threads = max(1, min(16, os.cpu_count() or 1))
    total = 0
    reps = 0
    t0 = time.perf_counter()
    while reps < max_reps:
        rc, out, summ = oracle.fit_batch(batch, consts, n_threads=threads, comb_offsets=False)
        assert rc == 0
        total += summ["total_comb"]
        reps += 1
        if time.perf_counter() - t0 >= min_seconds and reps >= 3:
            break
    dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "combinations/s", "cores": threads, "kind": "oracle",
            "sample": f"full 3000-event batch x {reps} passes ({dt:.1f} s), OpenMP over events"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--copies", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the fit path has no cross-GPU step)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_0380_amd import svt, synth

    batch, consts = synth.cfg2()
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    info = ctx.device_info()
    copies = [svt.to_device(batch) for _ in range(args.copies)]
    results = [svt.DeviceResults(batch.n_events, batch.n_roads) for _ in range(args.copies)]
    bstructs = [c.struct() for c in copies]
    rstructs = [r.struct() for r in results]
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()

    def run(n, collect):
        tickets = []
        dev_ns = []
        total = 0
        for i in range(n):
            k = i % args.copies
            tickets.append(ctx.submit(bstructs[k], rstructs[k], stream))
            if len(tickets) > 32:
                st, s = ctx.result(tickets.pop(0), -1)
                svt.check(st, "fit")
                total += s.total_comb
                dev_ns.append(s.device_ns)
        for t in tickets:
            st, s = ctx.result(t, -1)
            svt.check(st, "fit")
            total += s.total_comb
            dev_ns.append(s.device_ns)
        return total, dev_ns

    run(args.warmup, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total, dev_ns = run(args.steps, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ms_per_step = elapsed * 1e3 / args.steps
    fits_per_s = total / elapsed
    kernel_s = float(np.mean(dev_ns)) * 1e-9
    alg = algorithmic_bytes(batch)
    achieved = alg / kernel_s / 1e9
    line = {
        "metric": "fitted combinations/s (+ p50/p99 per-burst latency, batched vs plain)",
        "value": fits_per_s,
        "unit": "combinations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/fp64-exact",
        "data": "synthetic (seeded generator; paper's CDF data not available)",
        "config": {"workload": "scaled-up plain fit: 3000 events x 64 roads, 1-4 hits/layer, "
                               "72 sectors, lattice constants, half the roads with a planted track",
                   "n_roads": batch.n_roads, "n_hits": batch.n_hits,
                   "combinations": int(total // args.steps), "chi2_cut": consts.chi2_cut,
                   "device": info["arch"], "compute_units": info["compute_units"],
                   "tuning": ctx.tuning(), "input_copies": args.copies},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel_us": kernel_s * 1e6, "algorithmic_bytes": alg},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(batch, consts, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
