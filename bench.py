"""Benchmark of the SVT linearized fit on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]
                [--sections fit,sweep,list,unpack,uneven,serve,io,shadow]

Headline step = one pass of the fit over the scaled-up plain-fit workload
(3000 events x 64 roads, 1-4 hits per layer, 72 sectors, lattice constants,
half the roads with a planted track: 192,000 roads, ~7.5 M combinations),
inputs and results resident in HBM.  The K timed passes run back to back as
ring runs of up to 100 passes (one multi-pass fit launch and one reduction
kernel each, enqueued on the stream), and rotate over 32
input copies so that they read HBM rather than the 256 MB last-level cache;
at least 2000 untimed passes of the same rings come first, whatever --warmup
asks for, so that the clocks have settled.
The per-request form (one svt_fit_events call per pass) is reported beside
it.  Further sections: the paper's sweep (1-3000 events x 2048 combinations,
with the oracle on one and on all host threads), the list of every passing
combination, the unpack of a packed word stream, the uneven-batch plan
against per-event launches, the serving loop (p50/p99 per burst, batched
against plain), the transfer study and the float shadow.  Prints one JSON
line.
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


# untimed passes before the timed region, whatever --warmup asks for (about
# 17 ms of fit work: the chip's clocks settle within some 20 ms of it)
WARM_PASSES = 2000
# untimed regions shaped as the timed one, run just before it
PRE_REGIONS = 3


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("svt_fit.hip", "svt_rows.h", "svt_internal.h"):
        with open(os.path.join(ROOT, "paper_1311_0380_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per pass over the 3000-event batch from the committed counter
    summary, if it was taken on the kernel source that is built now; else
    None."""
    path = os.path.join(ROOT, "profiles", "fit_kernel_3000ev_hbm_counters.md")
    try:
        kv = {}
        for line in open(path):
            if "=" in line and not line.startswith(("|", "`", "cd ")):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_sha256_prefix") != kernel_source_hash():
            return None
        return int(kv["traffic_bytes_per_pass"])
    except (OSError, KeyError, ValueError):
        return None


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q))


def host_cpu():
    """The host's CPU as the oracle sees it: model name, logical CPUs, the
    CPUs this process may run on, and the threads an OpenMP run uses (the
    affinity set, capped by OMP_NUM_THREADS when that is set: a GPU job's
    share of a shared host)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    threads = affinity
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        threads = min(threads, int(omp))
    return {"model": model, "nproc": os.cpu_count() or 1, "affinity": affinity,
            "threads": max(1, threads)}


def oracle_rate(batch, consts, threads, min_seconds, min_reps=3, max_reps=100):
    """Oracle passes over one batch until min_seconds have passed (at least
    min_reps, at most max_reps); returns (combinations/s, median seconds per
    pass, passes)."""
    import oracle
    times, total = [], 0
    t_all = time.perf_counter()
    while len(times) < max_reps:
        t0 = time.perf_counter()
        rc, _, summ = oracle.fit_batch(batch, consts, n_threads=threads, comb_offsets=False)
        times.append(time.perf_counter() - t0)
        assert rc == 0
        total += summ["total_comb"]
        if time.perf_counter() - t_all >= min_seconds and len(times) >= min_reps:
            break
    return total / sum(times), float(np.median(times)), len(times)


def cpu_baseline(batch, consts, min_seconds=10.0):
    """The oracle on the host: all the threads this process may use over the
    full 3000-event batch, and one thread over its first 300 events."""
    import oracle
    oracle.build(force=False)
    cpu = host_cpu()
    rate, med, reps = oracle_rate(batch, consts, cpu["threads"], min_seconds)
    sub = batch.select_events(0, 300)
    rate1, med1, reps1 = oracle_rate(sub, consts, 1, min_seconds / 2)
    return {"value": rate, "unit": "combinations/s", "cores": cpu["threads"], "kind": "oracle",
            "sample": f"the full 3000-event batch, {reps} passes, median {med * 1e3:.0f} ms per pass "
                      f"(OpenMP over events, {cpu['threads']} threads)",
            "single_thread": {"value": rate1, "unit": "combinations/s", "cores": 1,
                              "sample": f"the batch's first 300 events, {reps1} passes, median "
                                        f"{med1 * 1e3:.1f} ms per pass"},
            "cpu_model": cpu["model"], "nproc": cpu["nproc"], "affinity": cpu["affinity"]}


def make_rings(svt, ctx, bs, rs, steps, per_ring, per_launch=0):
    """Rings covering `steps` passes: full rings of per_ring passes (each
    starting at a different copy) and one ring for the remainder; per_launch
    passes per kernel launch (0: the library's choice)."""
    sizes = [per_ring] * (steps // per_ring) + ([steps % per_ring] if steps % per_ring else [])
    rings = []
    for i, n in enumerate(sizes):
        rot = (i * per_ring) % len(bs)
        order = list(range(rot, len(bs))) + list(range(rot))
        nb = min(n, len(bs))
        st, ring = svt.svt_ring_create(ctx, [bs[j] for j in order[:nb]], [rs[j] for j in order[:nb]],
                                       n, per_launch)
        svt.check(st, "svt_ring_create")
        rings.append((ring, n))
    return rings


def run_rings(svt, ctx, rings, stream, repeat=1):
    """Replay the rings in order, at most three runs in flight (a ring runs
    once at a time); returns (combinations, device ns per run)."""
    pend, total, dev = collections.deque(), 0, []
    for _ in range(repeat):
        for ring, n in rings:
            st, t = svt.svt_ring_run(ring, stream)
            while st == svt.SVT_E_AGAIN and pend:   # this ring's previous run is in flight
                st2, s = svt.svt_result(ctx, pend.popleft(), -1)
                svt.check(st2, "ring")
                total += s.total_comb
                dev.append(s.device_ns)
                st, t = svt.svt_ring_run(ring, stream)
            svt.check(st, "svt_ring_run")
            pend.append(t)
            while len(pend) > 2:
                st2, s = svt.svt_result(ctx, pend.popleft(), -1)
                svt.check(st2, "ring")
                total += s.total_comb
                dev.append(s.device_ns)
    while pend:
        st2, s = svt.svt_result(ctx, pend.popleft(), -1)
        svt.check(st2, "ring")
        total += s.total_comb
        dev.append(s.device_ns)
    return total, dev


def section_fit(args, svt, synth, torch):
    """Headline: passes of the fit over the 3000-event batch, back to back.
    The timed region runs exactly --steps passes as ring runs of at most
    --ring-passes passes each over --copies rotating input copies (the
    paper's repeated passes over one sample, Sec. 4.1, in steady state).
    The per-request form (one svt_fit_events per pass, over two streams)
    is measured beside it."""
    batch, consts = synth.cfg2()
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    info = ctx.device_info()
    copies = [svt.to_device(batch) for _ in range(args.copies)]
    results = [svt.DeviceResults(batch.n_events, batch.n_roads) for _ in range(args.copies)]
    bs = [c.struct() for c in copies]
    rs = [r.struct() for r in results]
    stream = torch.cuda.current_stream().cuda_stream
    per_ring = max(1, min(args.ring_passes, args.steps))
    timed = make_rings(svt, ctx.handle, bs, rs, args.steps, per_ring, args.passes_per_launch)
    shapes = [svt.svt_ring_info(r) for r, _ in timed]
    per_launch = shapes[0][1]
    launches = sum(x[2] for x in shapes)
    # warm-up: the timed rings themselves, at least --warmup passes and never
    # fewer than WARM_PASSES (the chip takes some 20 ms of this work to reach
    # its steady clocks; a short --warmup would otherwise time the ramp)
    warm = max(args.warmup, WARM_PASSES)
    warm_repeat = max(1, -(-warm // args.steps))
    run_rings(svt, ctx.handle, timed, stream, repeat=warm_repeat)
    torch.cuda.synchronize()
    # and three untimed regions shaped as the timed one (each from a
    # synchronized start): the first two such regions after the long warm-up
    # ran slower on the host side (20-pass regions, wall time per pass:
    # 12.7, 11.6, then 9.7-9.8 us, at the same device time)
    for _ in range(PRE_REGIONS):
        run_rings(svt, ctx.handle, timed, stream)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    total, dev = run_rings(svt, ctx.handle, timed, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for ring, _ in timed:
        svt.svt_ring_destroy(ring)
    passes = args.steps
    kernel_s = sum(dev) * 1e-9 / passes          # per pass
    launch_s = sum(dev) * 1e-9 / launches        # per kernel launch
    # a longer run of the same rings' shape for the steady-state check
    requests = section_fit_requests(args, svt, ctx, bs, rs, torch)
    alg = algorithmic_bytes(batch.n_events, batch.n_roads, batch.n_hits)
    traffic = measured_traffic()
    # one launch covers passes / launches passes of alg bytes each
    achieved = alg * passes / launches / launch_s / 1e9
    out = dict(
        value=total / elapsed, ms_per_step=elapsed * 1e3 / passes,
        combinations=int(total // passes),
        config={"workload": "scaled-up plain fit: 3000 events x 64 roads, 1-4 hits per layer, "
                            "72 sectors, lattice constants, half the roads with a planted track",
                "step": "one pass of the fit over the batch; the timed passes run back to back "
                        f"as ring runs of up to {per_ring} passes over {args.copies} "
                        f"rotating input copies, {per_launch} passes per kernel launch",
                "chunks": "12 events per chunk (three 256-road sub-chunks per block) in a "
                          "launch's passes, 4 in its last passes (enough to fill the grid once, "
                          "at most a quarter of them)",
                "n_events": batch.n_events, "n_roads": batch.n_roads, "n_hits": batch.n_hits,
                "combinations": int(total // passes), "chi2_cut": consts.chi2_cut,
                "device": info["arch"], "compute_units": info["compute_units"],
                "tuning": ctx.tuning(), "input_copies": args.copies, "ring_passes": per_ring,
                "passes_per_launch": per_launch,
                "warmup_passes_run": (warm_repeat + PRE_REGIONS) * args.steps},
        roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": achieved / HBM_PEAK_GBS,
                  "traffic": None if traffic is None else traffic * passes // launches,
                  "kernel_us": launch_s * 1e6, "kernel_us_per_pass": kernel_s * 1e6,
                  "algorithmic_bytes": alg * passes // launches, "algorithmic_bytes_per_pass": alg,
                  "passes_per_launch": per_launch, "timed_launches": launches,
                  "kernel_us_basis": "device time of the timed ring runs (events around each "
                                     "run on its stream) / kernel launches: back-to-back "
                                     "fit kernels on one stream, the gaps between them and the "
                                     "small kernel that reduces each run's block partials "
                                     "included"},
        requests=requests, batch=batch, consts=consts)
    ctx.close()
    return out


def section_fit_requests(args, svt, ctx, bs, rs, torch):
    """One svt_fit_events request per pass, alternating over two streams
    (launches overlap), one request in --time-every timed by its own
    dispatch; then 20 isolated requests."""
    streams = [torch.cuda.Stream() for _ in range(args.fit_streams)]
    handles = [s.cuda_stream for s in streams]
    ctx.set_timing(args.time_every)
    h, sub, fin = ctx.handle, svt.lib.svt_fit_events, svt.lib.svt_result
    b_refs = [ctypes.byref(b) for b in bs]
    r_refs = [ctypes.byref(r) for r in rs]
    s_ptrs = [ctypes.c_void_p(x) for x in handles]
    tk, summ = ctypes.c_int64(0), svt.svt_summary()
    tk_ref, summ_ref = ctypes.byref(tk), ctypes.byref(summ)
    n_req = max(args.steps, 200)

    def run(n):
        pend, dev_ns, total = collections.deque(), [], 0

        def collect(t):
            st = fin(h, t, -1, summ_ref)
            svt.check(st, "fit")
            dev_ns.append(summ.device_ns)
            return summ.total_comb

        for i in range(n):
            st = sub(h, b_refs[i % len(bs)], r_refs[i % len(bs)], s_ptrs[i % len(s_ptrs)], tk_ref)
            svt.check(st, "svt_fit_events")
            pend.append(tk.value)
            if len(pend) > 32:
                total += collect(pend.popleft())
        while pend:
            total += collect(pend.popleft())
        return total, dev_ns

    run(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total, dev_ns = run(n_req)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(1)
    stream = torch.cuda.current_stream().cuda_stream
    iso = []
    for i in range(20):
        t = ctx.submit(bs[i % len(bs)], rs[i % len(bs)], stream)
        st, s = ctx.result(t, -1)
        iso.append(s.device_ns)
    timed = [d for d in dev_ns if d > 0]
    return {"requests": n_req, "streams": args.fit_streams, "us_per_request": elapsed * 1e6 / n_req,
            "combinations_per_s": total / elapsed,
            "dispatch_timed_us_mean": float(np.mean(timed)) / 1e3, "dispatch_timed": len(timed),
            "isolated_request_us_p50": pct(iso, 50) / 1e3,
            "note": "a dispatch timed by its own events measures at least 3.9 us (an empty "
                    "kernel measures the same)"}


def section_sweep(args, svt, synth, torch, iostudy):
    """The paper's benchmark shape (Sec. 4.1): 2048 combinations per event,
    1 to 3000 events.  Per size: device time of a pass (rings of 100 passes),
    end-to-end time of a request with pinned host inputs and results, the
    stages (DMA in, unpack of the packed words, fit, DMA out) and the oracle
    on one thread and on all threads, with the speed-ups."""
    import oracle
    oracle.build(force=False)
    cpu = host_cpu()
    ctx = svt.Context(0)
    stream = torch.cuda.current_stream().cuda_stream
    rows = []
    for ne in args.sweep_events:
        batch, consts = synth.paper_sweep(ne)
        ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
        comb = int(np.prod(batch.nhits.astype(np.int64), axis=1).sum())
        n_copy = 8
        dbs = [svt.to_device(batch) for _ in range(n_copy)]
        drs = [svt.DeviceResults(batch.n_events, batch.n_roads) for _ in range(n_copy)]
        rings = make_rings(svt, ctx.handle, [d.struct() for d in dbs], [r.struct() for r in drs],
                           100, 100)
        run_rings(svt, ctx.handle, rings, stream)
        _, dev = run_rings(svt, ctx.handle, rings, stream, repeat=3)
        for ring, _ in rings:
            svt.svt_ring_destroy(ring)
        fit_us = float(np.median(dev)) / 1e3 / 100
        # end to end: pinned host inputs and results, one request at a time
        pin_b = {f: torch.from_numpy(np.ascontiguousarray(getattr(batch, f))).pin_memory()
                 for f in svt.BATCH_FIELDS}
        hb = svt.svt_event_batch(batch.n_events, batch.n_roads, batch.n_hits, svt.SVT_MEM_PINNED,
                                 *[pin_b[f].data_ptr() for f in svt.BATCH_FIELDS])
        pres = svt.DeviceResults(batch.n_events, batch.n_roads, pin=True)
        hr = pres.struct()
        e2e, wall = [], []
        for i in range(args.sweep_reps + 5):
            t0 = time.perf_counter()
            t = ctx.submit(hb, hr, stream)
            st, s = ctx.result(t, -1)
            svt.check(st, "sweep request")
            if i >= 5:
                wall.append(time.perf_counter() - t0)
                e2e.append(s.device_ns / 1e3)
        # stages: DMA of the CSR batch in, unpack of the packed words (device),
        # the fit, DMA of the results out
        in_bytes = batch.nbytes()
        out_bytes = batch.n_roads * 36 + 4 * batch.n_events
        h2d = svt.svt_io_probe(ctx.handle, svt.SVT_MEM_PINNED, 0, in_bytes, 21)
        d2h = svt.svt_io_probe(ctx.handle, svt.SVT_MEM_PINNED, 1, out_bytes, 21)
        words = torch.from_numpy(synth.pack_stream(batch).view(np.int32)).cuda()
        caps = (batch.n_events, batch.n_roads, batch.n_hits)
        unp = []
        for i in range(23):
            st, s, _ = ctx.unpack_stream(words, mem_kind=svt.SVT_MEM_DEVICE, caps=caps)
            svt.check(st, "unpack")
            if i >= 3:
                unp.append(s.device_ns / 1e3)
        # the oracle: one thread, and every thread this process may use
        budget = args.sweep_cpu_seconds
        r1, m1, n1 = oracle_rate(batch, consts, 1, budget, min_reps=3)
        ra, ma, na = oracle_rate(batch, consts, cpu["threads"], budget, min_reps=3)
        e2e_us = float(np.median(e2e))
        row = {"events": ne, "combinations": comb, "gpu_fit_us": fit_us,
               "gpu_fits_per_s": comb / (fit_us * 1e-6),
               "gpu_end_to_end_us": e2e_us, "gpu_end_to_end_wall_us": float(np.median(wall)) * 1e6,
               "end_to_end_fits_per_s": comb / (e2e_us * 1e-6),
               "stages_us": {"h2d": h2d, "unpack": float(np.median(unp)), "fit": fit_us,
                             "d2h": d2h},
               "cpu_1thread_us": m1 * 1e6, "cpu_1thread_reps": n1,
               "cpu_all_us": ma * 1e6, "cpu_all_reps": na, "cpu_threads": cpu["threads"],
               "speedup_fit_vs_1thread": m1 * 1e6 / fit_us,
               "speedup_end_to_end_vs_1thread": m1 * 1e6 / e2e_us,
               "speedup_fit_vs_all_threads": ma * 1e6 / fit_us}
        rows.append(row)
        log(f"sweep {ne:5d} events: fit {fit_us:7.2f} us, end to end {e2e_us:8.1f} us, "
            f"cpu 1 thread {m1 * 1e6:10.0f} us, all {ma * 1e6:9.0f} us")
    ctx.close()
    return {"workload": "paper shape: events x 8 roads x 4 hits per layer (2048 combinations "
                        "per event), lattice constants, half the roads with a planted track",
            "cpu_model": cpu["model"], "rows": rows,
            "timed": "fit: device time of rings of 100 passes over 8 copies / 100; end to end: "
                     "device time of one request with pinned host inputs and results (copies "
                     "included), median of --sweep-reps; stages from separate DMA probes and "
                     "unpack requests; oracle: median pass"}


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
            "timed": "events around the request: the tile sums of npass (one small kernel) "
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
                                       (1e6, args.serve_bursts[2], args.serve_bursts[2])):
        rng = np.random.default_rng(int(load) % 1000 + 5)
        arr = serve.make_arrivals(rng, nb_batched, load, pool.batch.n_events)
        ctx = svt.Context(0, 4 << 30)
        ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
        ctx.set_timing(0)                  # latencies come from the host clock
        srv = serve.Server(serve.LibraryDevice(ctx, 4), pool, n_slots=4, max_events=6000)
        srv.warm()                         # staging buffers for the largest launches
        srv.run(arr[:8])
        srv.launch_sizes.clear()
        srv.fill_seconds = 0.0
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
            precs = plain.run(arr[:nb_plain], time_limit=args.serve_plain_seconds)
        finally:
            gc.enable()
        st_p = serve.latency_stats(precs)
        ctx.close()
        out["loads"].append({"events_per_s": load, "bursts": len(recs),
                             "batched": dict(st_b, launches=len(srv.launch_sizes),
                                             mean_events_per_launch=float(np.mean(srv.launch_sizes)),
                                             events_per_s_served=ev / wall,
                                             fits_per_s=comb / wall,
                                             host_fill_share=srv.fill_seconds / wall,
                                             wall_s=wall),
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
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--copies", type=int, default=32)
    ap.add_argument("--passes-per-launch", type=int, default=0,
                    help="fit passes per kernel launch in the rings (0: the library's choice)")
    ap.add_argument("--ring-passes", type=int, default=100,
                    help="passes per ring run in the timed region")
    ap.add_argument("--fit-streams", type=int, default=2,
                    help="streams the fit requests of the timed region alternate over")
    ap.add_argument("--time-every", type=int, default=8,
                    help="fit requests of the timed region that carry dispatch events: one in N")
    ap.add_argument("--sections", default="fit,sweep,list,unpack,uneven,serve,io,shadow")
    ap.add_argument("--sweep-events", type=lambda s: [int(v) for v in s.split(",")],
                    default=[1, 10, 100, 500, 1000, 2000, 3000])
    ap.add_argument("--sweep-reps", type=int, default=100)
    ap.add_argument("--sweep-cpu-seconds", type=float, default=1.5)
    ap.add_argument("--list-reps", type=int, default=50)
    ap.add_argument("--unpack-reps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--uneven-reps", type=int, default=50)
    ap.add_argument("--serve-bursts", type=lambda s: [int(v) for v in s.split(",")],
                    default=[2000, 2000, 2000],
                    help="bursts per offered load (10k, 100k, 1M events/s), batched form")
    ap.add_argument("--serve-plain-seconds", type=float, default=15.0,
                    help="time cap of the plain per-event form per load (its burst count is reported)")
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
        "config": fit["config"], "roofline": fit["roofline"], "requests": fit["requests"],
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(fit["batch"], fit["consts"], args.cpu_seconds)
    if "sweep" in sections:
        log("section sweep")
        line["sweep"] = section_sweep(args, svt, synth, torch, iostudy)
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
