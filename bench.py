"""Benchmark of the SVT linearized fit on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]
                [--sections fit,list,unpack,uneven,serve,io,shadow]

Headline step = one svt_fit_events request over the scaled-up plain-fit
workload (3000 events x 64 roads, 1-4 hits per layer, 72 sectors, lattice
constants, half the roads with a planted track: 192,000 roads, ~7.5 M
combinations), inputs and results resident in HBM.  Inputs rotate over
distinct copies so timed passes read HBM rather than the 256 MB last-level
cache.  Further sections measure the list of every passing combination,
the unpack of a packed word stream, the uneven-batch plan against per-event launches, the serving loop (p50/p99
per burst, batched against plain), the transfer study and the float shadow.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import collections
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n_events, n_roads, n_hits, n_sectors=72):
    """Bytes the method must move once: every input word read once, every
    result word written once, the constants once."""
    inputs = 4 * (n_events + 1) + n_roads * (1 + 4 + 4 + 4) + 4 + 2 * n_hits
    outputs = n_roads * (4 + 4 + 4 + 8 + 12 + 4) + 4 * n_events
    return inputs + outputs + n_sectors * 42 * 4


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("svt_fit.hip", "svt_rows.h", "svt_internal.h"):
        with open(os.path.join(ROOT, "paper_1311_0380_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the kernel source that is built now; else None."""
    path = os.path.join(ROOT, "profiles", "fit_kernel_3000ev_hbm_counters.md")
    try:
        kv = {}
        for line in open(path):
            if "=" in line and not line.startswith(("|", "`", "cd ")):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_sha256_prefix") != kernel_source_hash():
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q))


def cpu_baseline(batch, consts, min_seconds=10.0, max_reps=5000):
    import oracle
    oracle.build(force=False)
    threads = max(1, min(16, os.cpu_count() or 1))
    total = reps = 0
    t0 = time.perf_counter()
    while reps < max_reps:
        rc, _, summ = oracle.fit_batch(batch, consts, n_threads=threads, comb_offsets=False)
        assert rc == 0
        total += summ["total_comb"]
        reps += 1
        if time.perf_counter() - t0 >= min_seconds and reps >= 3:
            break
    dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "combinations/s", "cores": threads, "kind": "oracle",
            "sample": f"the full 3000-event batch, {reps} passes in {dt:.1f} s "
                      f"(OpenMP over events, {threads} threads)"}


def section_fit(args, svt, synth, torch):
    batch, consts = synth.cfg2()
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    info = ctx.device_info()
    copies = [svt.to_device(batch) for _ in range(args.copies)]
    results = [svt.DeviceResults(batch.n_events, batch.n_roads) for _ in range(args.copies)]
    bs = [c.struct() for c in copies]
    rs = [r.struct() for r in results]
    stream = torch.cuda.current_stream().cuda_stream
    if args.time_every < 1 or args.steps < args.time_every:
        raise SystemExit("--time-every must be at least 1 and at most --steps "
                         "(the roofline needs timed launches)")
    if args.fit_streams < 1 or args.copies % args.fit_streams:
        # request i reuses the buffers of request i - copies: same stream, so in order
        raise SystemExit("--fit-streams must be at least 1 and divide --copies")
    # requests alternate over independent streams (default priority), so that
    # one launch's tail and set-up overlap the next one's row loops
    streams = [torch.cuda.Stream() for _ in range(args.fit_streams)]
    handles = [s.cuda_stream for s in streams]
    # dispatch events on one request in time_every: a start timestamp costs
    # the host about 11 us per launch, the completion alone about 3 us
    ctx.set_timing(args.time_every)
    h, sub, fin = ctx.handle, svt.lib.svt_fit_events, svt.lib.svt_result
    b_refs = [ctypes.byref(b) for b in bs]
    r_refs = [ctypes.byref(r) for r in rs]
    s_ptrs = [ctypes.c_void_p(x) for x in handles]
    tk, summ = ctypes.c_int64(0), svt.svt_summary()
    tk_ref, summ_ref = ctypes.byref(tk), ctypes.byref(summ)
    torch.cuda.synchronize()

    def run(n):
        # the C calls with their argument objects built once: the loop's own
        # host cost stays well below a request's device time
        pend, dev_ns, total = collections.deque(), [], 0

        def collect(t):
            st = fin(h, t, -1, summ_ref)
            svt.check(st, "fit")
            dev_ns.append(summ.device_ns)
            return summ.total_comb

        for i in range(n):
            st = sub(h, b_refs[i % args.copies], r_refs[i % args.copies], s_ptrs[i % len(s_ptrs)], tk_ref)
            svt.check(st, "svt_fit_events")
            pend.append(tk.value)
            if len(pend) > 32:
                total += collect(pend.popleft())
        while pend:
            total += collect(pend.popleft())
        return total, dev_ns

    run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total, dev_ns = run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(1)
    # one request at a time: the request's own device time without queueing
    iso = []
    for i in range(20):
        t = ctx.submit(bs[i % args.copies], rs[i % args.copies], stream)
        st, s = ctx.result(t, -1)
        iso.append(s.device_ns)
    timed = [d for d in dev_ns if d > 0]
    kernel_s = float(np.mean(timed)) * 1e-9
    alg = algorithmic_bytes(batch.n_events, batch.n_roads, batch.n_hits)
    achieved = alg / kernel_s / 1e9
    effective = alg * args.steps / elapsed / 1e9   # launches overlap: bytes per wall second
    out = dict(
        value=total / elapsed, ms_per_step=elapsed * 1e3 / args.steps,
        combinations=int(total // args.steps),
        config={"workload": "scaled-up plain fit: 3000 events x 64 roads, 1-4 hits per layer, "
                            "72 sectors, lattice constants, half the roads with a planted track",
                "n_events": batch.n_events, "n_roads": batch.n_roads, "n_hits": batch.n_hits,
                "combinations": int(total // args.steps), "chi2_cut": consts.chi2_cut,
                "device": info["arch"], "compute_units": info["compute_units"],
                "tuning": ctx.tuning(), "input_copies": args.copies, "streams": args.fit_streams},
        roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                  "kernel_us": kernel_s * 1e6, "algorithmic_bytes": alg,
                  "timed_launches": len(timed),
                  "effective_gbs": effective, "effective_frac": effective / HBM_PEAK_GBS,
                  "isolated_request_us_p50": pct(iso, 50) / 1e3},
        batch=batch, consts=consts)
    ctx.close()
    return out


def list_algorithmic_bytes(n_roads, n_hits, entries):
    """Bytes a passing-combination list must move: the pass counts in (4 B per
    road), the road offsets out (8 B), the roads in (13 B: sector, hit counts,
    hit offset, XFT words) and their hits (2 B each), and 24 B per entry
    (index, chi2, three fit rows)."""
    return n_roads * (4 + 8 + 13) + 2 * n_hits + 24 * entries


def section_list(args, svt, synth, torch):
    """Every passing combination of the 3000-event batch: one svt_list_passing
    request after a fit, inputs and list in HBM."""
    batch, consts = synth.cfg2()
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    db = svt.to_device(batch)
    res = svt.DeviceResults(batch.n_events, batch.n_roads)
    st, _, _ = ctx.fit(db, res)
    svt.check(st, "fit")
    cap = int(res.npass.sum().item())
    lst = svt.DevicePassList(batch.n_roads, cap)
    b, l = db.struct(), lst.struct()
    stream = torch.cuda.current_stream().cuda_stream

    def once():
        st, t = svt.svt_list_passing(ctx.handle, b, res.npass.data_ptr(), l, stream)
        svt.check(st, "svt_list_passing")
        st, s = ctx.result(t, -1)
        svt.check(st, "list")
        return s

    for _ in range(5):
        once()
    dev, wall = [], []
    for _ in range(args.list_reps):
        t0 = time.perf_counter()
        s = once()
        wall.append(time.perf_counter() - t0)
        dev.append(s.device_ns)
    ctx.close()
    entries = int(s.total_pass)
    alg = list_algorithmic_bytes(batch.n_roads, batch.n_hits, entries)
    req_s = pct(dev, 50) * 1e-9
    return {"workload": "every passing combination of the 3000-event x 64-road batch "
                        "(road offsets from the fit's pass counts, then the list)",
            "entries": entries, "combinations_evaluated": int(s.total_comb),
            "request_device_us_p50": req_s * 1e6, "request_wall_us_p50": pct(wall, 50) * 1e6,
            "entries_per_s": entries / req_s, "algorithmic_bytes": alg,
            "achieved_gbs": alg / req_s / 1e9, "hbm_frac": alg / req_s / 1e9 / HBM_PEAK_GBS,
            "timed": "events around the request: the offsets scan (two small kernels) "
                     "and the list kernel"}


def section_unpack(args, svt, synth, torch):
    """Unpack of the 3000-event batch's packed word stream into the CSR
    batch: from device memory, from host-mapped memory read in place (zero
    copy) and from pageable memory (DMA copy first); then unpack + fit from
    host-mapped memory."""
    batch, consts = synth.cfg2()
    words = synth.pack_stream(batch)
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    caps = (batch.n_events, batch.n_roads, batch.n_hits)
    w32 = torch.from_numpy(words.view(np.int32))
    srcs = {"device": (w32.cuda(), svt.SVT_MEM_DEVICE), "mapped": (w32.pin_memory(), svt.SVT_MEM_MAPPED),
            "pageable": (words, svt.SVT_MEM_PAGEABLE)}
    out_bytes = 4 * (batch.n_events + 1) + 13 * batch.n_roads + 4 + 2 * batch.n_hits
    in_bytes = 4 * len(words)
    res = {"workload": "the 3000-event x 64-road batch as a packed word stream "
                       f"({len(words)} words, {in_bytes} B) unpacked into the CSR batch ({out_bytes} B)",
           "words": len(words), "stream_bytes": in_bytes, "batch_bytes": out_bytes}
    for name, (src, kind) in srcs.items():
        for _ in range(3):
            st, s, _ = ctx.unpack_stream(src, mem_kind=kind, caps=caps)
            svt.check(st, "unpack")
        dev, wall = [], []
        for _ in range(args.unpack_reps):
            t0 = time.perf_counter()
            st, s, _ = ctx.unpack_stream(src, mem_kind=kind, caps=caps)
            wall.append(time.perf_counter() - t0)
            dev.append(s.device_ns)
        d = pct(dev, 50) * 1e-9
        res[name] = {"request_device_us_p50": d * 1e6, "request_wall_us_p50": pct(wall, 50) * 1e6,
                     "gbs": (in_bytes + out_bytes) / d / 1e9}
    # ingest: unpack from host-mapped words, then fit the unpacked batch
    src, kind = srcs["mapped"]
    dres = svt.DeviceResults(batch.n_events, batch.n_roads)
    wall = []
    for i in range(args.unpack_reps + 3):
        t0 = time.perf_counter()
        st, s, db = ctx.unpack_stream(src, mem_kind=kind, caps=caps)
        svt.check(st, "unpack")
        st, fs, _ = ctx.fit(db, dres)
        svt.check(st, "fit")
        if i >= 3:
            wall.append(time.perf_counter() - t0)
    res["mapped_unpack_then_fit_wall_us_p50"] = pct(wall, 50) * 1e6
    ctx.close()
    res["timed"] = ("device time: events around the request (three passes over the words, plus the "
                    "DMA copy for pageable words)")
    return res


def section_uneven(args, svt, synth, torch, uneven):
    batch, consts = synth.cfg3()
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    db = svt.to_device(batch)
    dr = svt.DeviceResults(batch.n_events, batch.n_roads)
    best, table = uneven.autotune(ctx, db, dr, reps=5)
    plan = uneven.Plan(ctx, batch.n_events, batch.n_roads, batch.n_hits, best)
    b, r = db.struct(), dr.struct()
    inb, outb = plan.inb, plan.outb
    plan.fit(b, r)                       # inputs now in the plan's buffers
    inb.n_events, inb.n_roads, inb.n_hits = batch.n_events, batch.n_roads, batch.n_hits
    # wall times with no request timed (neither form needs device times
    # there); device times in runs of their own
    ctx.set_timing(0)
    lat = []
    for _ in range(args.uneven_reps):
        t0 = time.perf_counter()
        st, s = plan.fit(inb, outb)
        lat.append(time.perf_counter() - t0)
        svt.check(st)
    per = uneven.PerEventBatches(batch)
    per.run(ctx)                         # warm
    plain_wall = []
    for _ in range(3):
        w, _, _ = per.run(ctx)
        plain_wall.append(w)
    ctx.set_timing(1)
    dev = []
    for _ in range(args.uneven_reps):
        st, s = plan.fit(inb, outb)
        dev.append(s.device_ns)
    _, plain_dev, _ = per.run(ctx)
    plan.close()
    ctx.close()
    total = int(np.prod(batch.nhits.astype(np.int64), axis=1).sum())
    return {"workload": "uneven batching: 10000 events, roads/event geometric (mean 16, max 256), "
                        "hits/layer Poisson(1.5) clipped to [1, 8]",
            "combinations": total, "tuning": best, "tuning_candidates": len(table),
            "batched_graph_us_p50": pct(lat, 50) * 1e6, "batched_graph_us_p99": pct(lat, 99) * 1e6,
            "batched_graph_device_us_p50": pct(dev, 50) / 1e3,
            "plain_per_event_batch_us_p50": pct(plain_wall, 50) * 1e6,
            "plain_per_event_device_us_p50": pct(plain_dev, 50) / 1e3,
            "plain_per_event_device_us_p99": pct(plain_dev, 99) / 1e3,
            "batched_fits_per_s": total / pct(lat, 50),
            "plain_fits_per_s": total / pct(plain_wall, 50)}


def section_serve(args, svt, synth, torch, serve):
    batch, consts = synth.cfg2(seed=5)
    out = {"workload": "trigger serving: Poisson bursts of 1-3000 events (log-uniform), "
                       "events shaped as the 3000-event plain fit, pinned host pool",
           "loads": []}
    import gc
    pool = serve.HostPool(batch)
    comb_road = np.prod(batch.nhits.astype(np.int64), axis=1)
    comb_cum = np.concatenate([[0], np.cumsum(comb_road)])[batch.road_offsets.astype(np.int64)]
    for load, nb_batched, nb_plain in ((1e4, args.serve_bursts[0], args.serve_bursts[0]),
                                       (1e5, args.serve_bursts[1], args.serve_bursts[1]),
                                       (1e6, args.serve_bursts[2], args.serve_bursts[2] // 2)):
        rng = np.random.default_rng(int(load) % 1000 + 5)
        arr = serve.make_arrivals(rng, nb_batched, load, pool.batch.n_events)
        ctx = svt.Context(0, 4 << 30)
        ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
        ctx.set_timing(0)                  # latencies come from the host clock
        srv = serve.Server(serve.LibraryDevice(ctx, 4), pool, n_slots=4, max_events=6000)
        srv.warm()                         # staging buffers for the largest launches
        srv.run(arr[:8])
        srv.launch_sizes.clear()
        gc.collect()
        gc.disable()                       # no collector pauses inside the serving loop
        try:
            t0 = time.perf_counter()
            recs = srv.run(arr)
            wall = time.perf_counter() - t0
        finally:
            gc.enable()
        ev = sum(r.e1 - r.e0 for r in recs)
        comb = sum(int(comb_cum[r.e1] - comb_cum[r.e0]) for r in recs)
        st_b = serve.latency_stats(recs)
        plain = serve.PlainServer(ctx, pool, window=32)
        gc.collect()
        gc.disable()
        try:
            precs = plain.run(arr[:nb_plain], time_limit=60.0)
        finally:
            gc.enable()
        st_p = serve.latency_stats(precs)
        ctx.close()
        out["loads"].append({"events_per_s": load, "bursts": len(recs),
                             "batched": dict(st_b, launches=len(srv.launch_sizes),
                                             mean_events_per_launch=float(np.mean(srv.launch_sizes)),
                                             events_per_s_served=ev / wall,
                                             fits_per_s=comb / wall),
                             "plain": dict(st_p, bursts=len(precs))})
        log(f"serve load {load:g}: batched p50 {st_b.get('p50_us', 0):.0f} us p99 "
            f"{st_b.get('p99_us', 0):.0f} us | plain p50 {st_p.get('p50_us', 0):.0f} us "
            f"p99 {st_p.get('p99_us', 0):.0f} us")
    return out


def section_io(args, svt, synth, torch, iostudy):
    batch, consts = synth.cfg2(seed=5)
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    sweep = iostudy.transfer_sweep(ctx, reps=9)
    rt = iostudy.round_trip(ctx, batch, reps=5)
    ctx.close()
    return {"transfers": sweep, "round_trip": rt}


def section_shadow(args, svt, synth, torch, shadow):
    h = synth.helix_tracks(args.shadow_tracks, seed=4)
    coef, off = synth.pilot_constants(h)
    # start away from the optimum, as before a calibration
    rng = np.random.default_rng(5)
    coef = (coef * (1 + rng.normal(0, 0.02, coef.shape))).astype(np.float32)
    off = (off + rng.normal(0, 5.0, off.shape)).astype(np.float32)
    ctx = svt.Context(0)
    tr = shadow.ShadowTracks.from_helix(h, (1 / 400.0, 1 / 1e4, 1.0))
    A = torch.tensor(coef, device="cuda")
    b = torch.tensor(off, device="cuda")
    for _ in range(3):
        shadow.forward(ctx.handle, tr, A, b)
        shadow.backward(ctx.handle, tr, A, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        shadow.forward(ctx.handle, tr, A, b)
    e1.record()
    torch.cuda.synchronize()
    fwd_us = e0.elapsed_time(e1) * 1e3 / reps
    e0.record()
    for _ in range(reps):
        shadow.backward(ctx.handle, tr, A, b)
    e1.record()
    torch.cuda.synchronize()
    bwd_us = e0.elapsed_time(e1) * 1e3 / reps
    t0 = time.perf_counter()
    res = shadow.calibrate(ctx.handle, tr, A, b, steps=args.shadow_steps, lr=args.shadow_lr, lam=10.0,
                           record_every=max(1, args.shadow_steps // 5))
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / args.shadow_steps
    ci, oi, sh, status = shadow.requantize(ctx.handle, res.coef, res.offset)
    torch.cuda.synchronize()
    ctx.close()
    nbytes = h.x.shape[0] * (6 + 3) * 4
    return {"workload": f"float-shadow calibration: {h.x.shape[0]} helix tracks, 72 sectors",
            "forward_us": fwd_us, "backward_us": bwd_us,
            "backward_gbs": nbytes / (bwd_us * 1e-6) / 1e9,
            "calibration_step_ms": step_ms, "loss_history": res.history,
            "requantize_status": int(status.item()),
            "shifts": [int(v) for v in sh.cpu().numpy()[:8]]}


def section_copy(args, torch):
    """A plain device-to-device copy of known size: the yardstick that turns
    the HBM counters of a profile into bytes."""
    n = 512 << 20
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    return {"bytes_read": n, "bytes_written": n, "us": us, "gbs": 2 * n / us / 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--copies", type=int, default=32)
    ap.add_argument("--fit-streams", type=int, default=2,
                    help="streams the fit requests of the timed region alternate over")
    ap.add_argument("--time-every", type=int, default=8,
                    help="fit requests of the timed region that carry dispatch events: one in N")
    ap.add_argument("--sections", default="fit,list,unpack,uneven,serve,io,shadow")
    ap.add_argument("--list-reps", type=int, default=50)
    ap.add_argument("--unpack-reps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--uneven-reps", type=int, default=50)
    ap.add_argument("--serve-bursts", type=lambda s: [int(v) for v in s.split(",")],
                    default=[40, 150, 400])
    ap.add_argument("--shadow-tracks", type=int, default=1000000)
    ap.add_argument("--shadow-steps", type=int, default=50)
    ap.add_argument("--shadow-lr", type=float, default=1e-4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the fit path has no cross-GPU step)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_0380_amd import iostudy, serve, shadow, svt, synth, uneven

    sections = set(args.sections.split(","))
    log("section fit")
    fit = section_fit(args, svt, synth, torch)
    line = {
        "metric": "fitted combinations/s (+ p50/p99 per-burst latency, batched vs plain)",
        "value": fit["value"], "unit": "combinations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": fit["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32 fit rows, fp64 exact chi2",
        "data": "synthetic (seeded generators; the paper's CDF data is not available)",
        "config": fit["config"], "roofline": fit["roofline"],
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(fit["batch"], fit["consts"], args.cpu_seconds)
    if "list" in sections:
        log("section list")
        line["list"] = section_list(args, svt, synth, torch)
    if "unpack" in sections:
        log("section unpack")
        line["unpack"] = section_unpack(args, svt, synth, torch)
    if "uneven" in sections:
        log("section uneven")
        line["uneven"] = section_uneven(args, svt, synth, torch, uneven)
    if "serve" in sections:
        log("section serve")
        line["serve"] = section_serve(args, svt, synth, torch, serve)
        p = {f"{int(l['events_per_s'])}": {"batched_p50_us": l["batched"].get("p50_us"),
                                            "batched_p99_us": l["batched"].get("p99_us"),
                                            "plain_p50_us": l["plain"].get("p50_us"),
                                            "plain_p99_us": l["plain"].get("p99_us")}
             for l in line["serve"]["loads"]}
        line["per_burst_latency_us"] = p
    if "io" in sections:
        log("section io")
        line["io"] = section_io(args, svt, synth, torch, iostudy)
    if "shadow" in sections:
        log("section shadow")
        line["shadow"] = section_shadow(args, svt, synth, torch, shadow)
    if "copy" in sections:
        log("section copy")
        line["copy"] = section_copy(args, torch)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
