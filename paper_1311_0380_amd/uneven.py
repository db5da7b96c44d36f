"""Uneven batches: one persistent graph-captured launch (a plan) with a launch
shape chosen by a grid search, against a per-event launch baseline.

Marshalling and timing only; every fit runs in the library's kernels.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from . import svt

CACHE_PATH = os.environ.get(
    "SVT_TUNE_CACHE",
    os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "build",
                 "svt_tune.json"))


CACHE_VERSION = "shapes7"     # bump when the candidate set or the kernels change


def workload_signature(n_events, n_roads, n_hits, ncomb_total=None):
    rpe = n_roads / max(1, n_events)
    hpr = n_hits / max(1, n_roads)
    key = f"ev{int(np.log2(max(1, n_events)))}_rpe{rpe:.0f}_hpr{hpr:.1f}"
    if ncomb_total is not None:
        key += f"_cpr{ncomb_total / max(1, n_roads):.0f}"
    return key


def candidates(n_events, n_roads):
    """Launch shapes to try: chunks of about 128..512 roads, cyclic or
    blocked, or each block's events found by road count (schedule 3), each
    with a few occupancies."""
    rpe = max(1.0, n_roads / max(1, n_events))
    out = []
    for e in (1, 2, 4, 8, 16, 32, 64, 128, 256):
        if 128 <= e * rpe <= 512 or (e == 1 and rpe > 512):
            for bpc in (3, 4, 5):
                for sch in (1, 2):
                    out.append(dict(events_per_chunk=e, blocks_per_cu=bpc, schedule=sch, kernel=1))
    for bpc in (3, 4, 5):
        out.append(dict(events_per_chunk=256, blocks_per_cu=bpc, schedule=3, kernel=1))
    return out


def _time_fit(ctx: svt.Context, bstruct, rstruct, reps, stream):
    ts = []
    for _ in range(reps):
        t = ctx.submit(bstruct, rstruct, stream)
        st, s = ctx.result(t, -1)
        svt.check(st, "fit")
        ts.append(s.device_ns)
    return float(np.median(ts))


def autotune(ctx: svt.Context, dbatch: svt.DeviceBatch, dres: svt.DeviceResults, reps=7,
             signature=None, use_cache=True, arch_key=None):
    """Grid search over (events per chunk, blocks per CU, schedule); returns
    (best tuning dict, table of (tuning, median device ns)).  Cached by
    (device arch, compute units, workload signature)."""
    info = ctx.device_info()
    arch_key = arch_key or f"{info['arch']}_{info['compute_units']}cu"
    signature = signature or workload_signature(dbatch.n_events, dbatch.n_roads, dbatch.n_hits)
    key = f"{arch_key}/{signature}/{CACHE_VERSION}"
    cache = {}
    if use_cache and os.path.exists(CACHE_PATH):
        try:
            with open(CACHE_PATH) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]["best"], cache[key]["table"]
    saved = ctx.tuning()
    stream = torch.cuda.current_stream().cuda_stream
    b, r = dbatch.struct(), dres.struct()
    table = []
    try:
        for cand in candidates(dbatch.n_events, dbatch.n_roads):
            ctx.set_tuning(**cand)
            _time_fit(ctx, b, r, 2, stream)
            table.append((cand, _time_fit(ctx, b, r, reps, stream)))
    finally:
        ctx.set_tuning(**saved)
    best = min(table, key=lambda t: t[1])[0]
    if use_cache:
        cache[key] = {"best": best, "table": table}
        os.makedirs(os.path.dirname(CACHE_PATH), exist_ok=True)
        tmp = CACHE_PATH + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, CACHE_PATH)
    return best, table


class Plan:
    """A graph-captured persistent fit with capacity for a batch shape."""

    def __init__(self, ctx: svt.Context, max_events, max_roads, max_hits, tuning=None):
        t = tuning or {}
        self.ctx = ctx
        self.handle = svt.svt_plan_create(ctx.handle, max_events, max_roads, max_hits,
                                          t.get("events_per_chunk", 0), t.get("blocks_per_cu", 0),
                                          t.get("schedule", 0), t.get("kernel", 0))
        self.inb, self.outb = svt.svt_plan_buffers(self.handle)

    def close(self):
        if self.handle:
            svt.svt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, bstruct, rstruct, stream=None):
        st, t = svt.svt_plan_fit(self.handle, bstruct, rstruct, stream)
        svt.check(st, "svt_plan_fit")
        return t

    def fit(self, bstruct, rstruct, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        t = self.submit(bstruct, rstruct, stream)
        return self.ctx.result(t, -1)


class PerEventBatches:
    """Every event of a batch as its own self-contained device batch (its own
    CSR offsets), sharing one upload; results land in full-size buffers."""

    def __init__(self, batch, device="cuda"):
        ne = batch.n_events
        ro = batch.road_offsets.astype(np.int64)
        ho = batch.hit_offsets.astype(np.int64)
        self.ne = ne
        self.r0 = ro[:-1].copy()
        self.nr = np.diff(ro)
        self.h0 = ho[ro[:-1]]
        self.nh = ho[ro[1:]] - self.h0
        # per-event road offsets [0, nr] and rebased hit offsets
        self.ro_ev = np.stack([np.zeros(ne, np.int64), self.nr], axis=1).astype(np.int32)
        self.ho_start = (ro[:-1] + np.arange(ne)).astype(np.int64)   # position in ho_ev
        ho_ev = np.empty(batch.n_roads + ne, np.int64)
        for e in range(ne):
            a, b = int(ro[e]), int(ro[e + 1])
            ho_ev[self.ho_start[e]:self.ho_start[e] + (b - a) + 1] = ho[a:b + 1] - ho[a]
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.d_ro = t(self.ro_ev)
        self.d_ho = t(ho_ev.astype(np.int32))
        self.d_sector = t(batch.sector)
        self.d_nhits = t(batch.nhits)
        self.d_hits = t(batch.hits)
        self.d_xft = t(batch.xft)
        self.res = svt.DeviceResults(ne, batch.n_roads, device=device)
        self._structs = None

    def structs(self):
        if self._structs is None:
            out = []
            rs = self.res
            for e in range(self.ne):
                r0, nr, h0, nh = int(self.r0[e]), int(self.nr[e]), int(self.h0[e]), int(self.nh[e])
                b = svt.svt_event_batch(
                    1, nr, nh, svt.SVT_MEM_DEVICE,
                    self.d_ro.data_ptr() + 8 * e,
                    self.d_sector.data_ptr() + r0,
                    self.d_nhits.data_ptr() + 4 * r0,
                    self.d_ho.data_ptr() + 4 * int(self.ho_start[e]),
                    self.d_hits.data_ptr() + 2 * h0,
                    self.d_xft.data_ptr() + 4 * r0)
                r = svt.svt_results(rs.ncomb.data_ptr() + 4 * r0, rs.npass.data_ptr() + 4 * r0,
                                    rs.best.data_ptr() + 4 * r0, rs.chi2.data_ptr() + 8 * r0,
                                    rs.params.data_ptr() + 12 * r0,
                                    rs.hit_index.data_ptr() + 4 * r0,
                                    rs.ntracks.data_ptr() + 4 * e, None, svt.SVT_MEM_DEVICE, 0)
                out.append((b, r))
            self._structs = out
        return self._structs

    def run(self, ctx: svt.Context, stream=None, window=48):
        """Launch every event separately (in order, up to `window` in flight);
        returns (wall seconds, per-event device ns, per-event completion
        seconds after the start)."""
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        structs = self.structs()
        dev_ns = np.zeros(self.ne)
        done_t = np.zeros(self.ne)
        pending = []
        t0 = time.perf_counter()
        for e, (b, r) in enumerate(structs):
            pending.append((e, ctx.submit(b, r, stream)))
            while len(pending) >= window:
                e0, tk = pending.pop(0)
                st, s = ctx.result(tk, -1)
                svt.check(st, "per-event fit")
                dev_ns[e0] = s.device_ns
                done_t[e0] = time.perf_counter() - t0
        for e0, tk in pending:
            st, s = ctx.result(tk, -1)
            svt.check(st, "per-event fit")
            dev_ns[e0] = s.device_ns
            done_t[e0] = time.perf_counter() - t0
        return time.perf_counter() - t0, dev_ns, done_t
