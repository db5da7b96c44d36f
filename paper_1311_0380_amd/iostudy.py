"""I/O study on one GPU: host <-> device transfer latency for pageable,
pinned and mapped buffers, and the round trip (copy in + fit + copy out) of
trigger-sized bursts with the share of it spent moving data -- the one-GPU
analog of the paper's transfer measurements (Sec. 4.2: total latency versus
packet size, and the fraction spent in data transfer).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import svt

KIND_NAMES = {svt.SVT_MEM_PAGEABLE: "pageable", svt.SVT_MEM_PINNED: "pinned",
              svt.SVT_MEM_MAPPED: "mapped", svt.SVT_MEM_DEVICE: "device"}
DEFAULT_SIZES = tuple(4096 << (2 * i) for i in range(8))     # 4 KB .. 64 MB


def transfer_sweep(ctx: svt.Context, sizes=DEFAULT_SIZES, reps=15):
    rows = []
    for kind in (svt.SVT_MEM_PAGEABLE, svt.SVT_MEM_PINNED, svt.SVT_MEM_MAPPED):
        for direction in (0, 1):
            for n in sizes:
                us = svt.svt_io_probe(ctx.handle, kind, direction, n, reps)
                rows.append(dict(kind=KIND_NAMES[kind], dir="h2d" if direction == 0 else "d2h",
                                 bytes=int(n), us=us, gbs=n / us / 1e3))
    return rows


def _host_copy(batch, kind):
    """The batch's arrays in host memory of the given kind (mapped = pinned
    memory that the kernel reads in place)."""
    out = {}
    for f in svt.BATCH_FIELDS:
        t = torch.from_numpy(np.ascontiguousarray(getattr(batch, f)))
        out[f] = t.pin_memory() if kind in (svt.SVT_MEM_PINNED, svt.SVT_MEM_MAPPED) else t.clone()
    return out


def _results(ne, nr, kind):
    if kind == svt.SVT_MEM_DEVICE:
        return svt.DeviceResults(ne, nr)
    if kind == svt.SVT_MEM_PAGEABLE:
        r = svt.DeviceResults(ne, nr, device="cpu")
    else:
        r = svt.DeviceResults(ne, nr, pin=True)
    r.mem_kind = kind
    return r


def round_trip(ctx: svt.Context, batch, event_counts=(1, 10, 100, 300, 1000, 3000), reps=7,
               kinds=(svt.SVT_MEM_PAGEABLE, svt.SVT_MEM_PINNED, svt.SVT_MEM_MAPPED)):
    """For bursts of the first n events: device time of the whole request
    (copies included) per memory kind, the device-resident fit time, and the
    share of the round trip spent on data movement."""
    rows = []
    stream = torch.cuda.current_stream().cuda_stream
    for n in event_counts:
        sub = batch.select_events(0, min(n, batch.n_events))
        nbytes = sub.nbytes()
        db = svt.to_device(sub)
        dr = _results(sub.n_events, sub.n_roads, svt.SVT_MEM_DEVICE)
        fit_ns = []
        for _ in range(reps + 1):
            t = ctx.submit(db.struct(), dr.struct(), stream)
            st, s = ctx.result(t, -1)
            svt.check(st)
            fit_ns.append(s.device_ns)
        fit_us = float(np.median(fit_ns[1:])) / 1e3
        for kind in kinds:
            host = _host_copy(sub, kind)
            b = svt.svt_event_batch(sub.n_events, sub.n_roads, sub.n_hits, kind,
                                    *[host[f].data_ptr() for f in svt.BATCH_FIELDS])
            res = _results(sub.n_events, sub.n_roads, kind)
            dev_ns, wall = [], []
            for _ in range(reps + 1):
                t0 = time.perf_counter()
                t = ctx.submit(b, res.struct(), stream)
                st, s = ctx.result(t, -1)
                wall.append(time.perf_counter() - t0)
                svt.check(st)
                dev_ns.append(s.device_ns)
            rt_us = float(np.median(dev_ns[1:])) / 1e3
            rows.append(dict(events=sub.n_events, input_bytes=int(nbytes), kind=KIND_NAMES[kind],
                             round_trip_us=rt_us, wall_us=float(np.median(wall[1:])) * 1e6,
                             fit_us=fit_us,
                             transfer_share=max(0.0, 1.0 - fit_us / rt_us) if rt_us > 0 else None))
    return rows


def main():
    """python -m paper_1311_0380_amd.iostudy [--kind pageable|pinned|mapped|all]
    Transfer latencies (median of --reps, timed by events on the context's
    stream) as one JSON line, for profiling the transfers on their own."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--kind", default="all", choices=["pageable", "pinned", "mapped", "all"])
    ap.add_argument("--reps", type=int, default=9)
    args = ap.parse_args()
    kinds = [k for k, name in KIND_NAMES.items() if args.kind in (name, "all") and
             k != svt.SVT_MEM_DEVICE]
    ctx = svt.Context(0)
    try:
        rows = []
        for kind in kinds:
            for direction in (0, 1):
                for n in DEFAULT_SIZES:
                    us = svt.svt_io_probe(ctx.handle, kind, direction, n, args.reps)
                    rows.append(dict(kind=KIND_NAMES[kind], dir="h2d" if direction == 0 else "d2h",
                                     bytes=int(n), us=us, gbs=n / us / 1e3))
        print(json.dumps({"reps": args.reps, "transfers": rows}))
    finally:
        ctx.close()


if __name__ == "__main__":
    main()
