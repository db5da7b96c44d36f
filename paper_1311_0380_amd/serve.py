"""Trigger-style serving loop: bursts of events arrive open-loop (Poisson) and
are fitted with continuous batching.

A burst is a contiguous range of events of a host event pool (the detector
read-out buffer).  Bursts that are waiting when a launch slot frees up are
merged into one batch (offsets rebased) and submitted; several launches are in
flight at once on separate streams, so their work overlaps on the device.
Admission is by device memory: the library returns SVT_E_NOMEM when the
staging of a launch does not fit the context's budget next to the launches
in flight, and the bursts then wait for a completion.  Per-burst latency is
completion (results on the host) minus arrival.

The plain baseline launches every event of every burst separately.

Marshalling, scheduling and timing only: every fit runs in the library.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import synth


@dataclasses.dataclass
class BurstRecord:
    idx: int
    arrival: float
    e0: int
    e1: int
    submit: float = -1.0
    done: float = -1.0
    launch: int = -1

    @property
    def latency(self):
        return self.done - self.arrival


def make_arrivals(rng, n_bursts, events_per_s, pool_events, max_events=3000):
    """Open-loop Poisson arrivals of bursts with log-uniform sizes; each burst
    is a random contiguous range of the event pool."""
    sizes = np.minimum(synth.burst_sizes(rng, n_bursts, max_events), pool_events)
    t = synth.poisson_arrivals(rng, n_bursts, events_per_s, synth.log_uniform_mean(max_events))
    starts = (rng.random(n_bursts) * (pool_events - sizes + 1)).astype(np.int64)
    return [(float(t[i]), int(starts[i]), int(starts[i] + sizes[i])) for i in range(n_bursts)]


class HostPool:
    """Events in page-locked host memory, with the prefix sums that locate a
    contiguous event range."""

    def __init__(self, batch, pin=True):
        import torch
        self.batch = batch
        self.ro = batch.road_offsets.astype(np.int64)
        self.ho = batch.hit_offsets.astype(np.int64)

        def pinned(a):
            t = torch.from_numpy(np.ascontiguousarray(a))
            return t.pin_memory() if pin else t

        self.t = {f: pinned(getattr(batch, f)) for f in
                  ("road_offsets", "sector", "nhits", "hit_offsets", "hits", "xft")}
        self.a = {f: v.numpy() for f, v in self.t.items()}

    def counts(self, e0, e1):
        r0, r1 = int(self.ro[e0]), int(self.ro[e1])
        return e1 - e0, r1 - r0, int(self.ho[r1] - self.ho[r0])


class LaunchBuffers:
    """Pinned input and result buffers of one launch slot."""

    def __init__(self, max_events, max_roads, max_hits, pin_memory=True):
        import torch

        def pin(shape, dt):
            t = torch.empty(shape, dtype=dt)
            return t.pin_memory() if pin_memory else t

        self.max = (max_events, max_roads, max_hits)
        self.ro = pin(max_events + 1, torch.int32)
        self.sector = pin(max(1, max_roads), torch.uint8)
        self.nhits = pin((max(1, max_roads), 4), torch.uint8)
        self.ho = pin(max_roads + 1, torch.int32)
        self.hits = pin(max(1, max_hits), torch.int16)
        self.xft = pin((max(1, max_roads), 2), torch.int16)
        self.ncomb = pin(max(1, max_roads), torch.int32)
        self.npass = pin(max(1, max_roads), torch.int32)
        self.best = pin(max(1, max_roads), torch.int32)
        self.chi2 = pin(max(1, max_roads), torch.int64)
        self.params = pin((max(1, max_roads), 3), torch.int32)
        self.hit_index = pin((max(1, max_roads), 4), torch.uint8)
        self.ntracks = pin(max_events, torch.int32)
        self.n = (0, 0, 0)

    def fill(self, pool: HostPool, ranges):
        """Merge event ranges of the pool into this slot (offsets rebased)."""
        ne = nr = nh = 0
        ro, ho = self.ro.numpy(), self.ho.numpy()
        ro[0] = 0
        ho[0] = 0
        for e0, e1 in ranges:
            r0, r1 = int(pool.ro[e0]), int(pool.ro[e1])
            h0, h1 = int(pool.ho[r0]), int(pool.ho[r1])
            k_e, k_r, k_h = e1 - e0, r1 - r0, h1 - h0
            ro[ne + 1:ne + k_e + 1] = pool.ro[e0 + 1:e1 + 1] - r0 + nr
            ho[nr + 1:nr + k_r + 1] = pool.ho[r0 + 1:r1 + 1] - h0 + nh
            self.sector.numpy()[nr:nr + k_r] = pool.a["sector"][r0:r1]
            self.nhits.numpy()[nr:nr + k_r] = pool.a["nhits"][r0:r1]
            self.xft.numpy()[nr:nr + k_r] = pool.a["xft"][r0:r1]
            self.hits.numpy()[nh:nh + k_h] = pool.a["hits"][h0:h1]
            ne, nr, nh = ne + k_e, nr + k_r, nh + k_h
        self.n = (ne, nr, nh)

    def structs(self):
        from . import svt
        ne, nr, nh = self.n
        b = svt.svt_event_batch(ne, nr, nh, svt.SVT_MEM_PINNED, self.ro.data_ptr(),
                                self.sector.data_ptr(), self.nhits.data_ptr(), self.ho.data_ptr(),
                                self.hits.data_ptr(), self.xft.data_ptr())
        r = svt.svt_results(self.ncomb.data_ptr(), self.npass.data_ptr(), self.best.data_ptr(),
                            self.chi2.data_ptr(), self.params.data_ptr(),
                            self.hit_index.data_ptr(), self.ntracks.data_ptr(), None,
                            svt.SVT_MEM_PINNED, 0)
        return b, r

    def results(self, road_lo=0, road_hi=None, ev_lo=0, ev_hi=None):
        ne, nr, _ = self.n
        road_hi = nr if road_hi is None else road_hi
        ev_hi = ne if ev_hi is None else ev_hi
        sl = slice(road_lo, road_hi)
        out = dict(ncomb=self.ncomb.numpy()[sl].copy(), npass=self.npass.numpy()[sl].copy(),
                   best=self.best.numpy()[sl].copy(),
                   chi2=self.chi2.numpy()[sl].view(np.uint64).copy(),
                   params=self.params.numpy()[sl].copy(),
                   hit_index=self.hit_index.numpy()[sl].copy(),
                   ntracks=self.ntracks.numpy()[ev_lo:ev_hi].copy())
        return out


class LibraryDevice:
    """The fit library through its pinned-memory path; one stream per slot."""

    NOMEM = -3

    def __init__(self, ctx, n_slots):
        import torch
        self.ctx = ctx
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]

    def submit(self, slot, bufs: LaunchBuffers):
        from . import svt
        b, r = bufs.structs()
        st, t = svt.svt_fit_events(self.ctx.handle, b, r, self.streams[slot].cuda_stream)
        return st, t

    def poll(self, ticket):
        from . import svt
        st, s = svt.svt_result(self.ctx.handle, ticket, 0)
        if st == svt.SVT_E_AGAIN:
            return False, 0
        return True, st


class Server:
    """Continuous batching over n_slots launch slots."""

    def __init__(self, device, pool: HostPool, n_slots=4, max_events=6000, max_roads=None,
                 max_hits=None, clock=time.perf_counter, keep_results=False, spin=0.0,
                 pin_memory=True):
        rpe = max(1, pool.batch.n_roads // max(1, pool.batch.n_events))
        hpr = max(1, pool.batch.n_hits // max(1, pool.batch.n_roads))
        self.max_events = max_events
        self.max_roads = max_roads or max_events * rpe * 2
        self.max_hits = max_hits or self.max_roads * hpr * 2
        self.device = device
        self.pool = pool
        self.bufs = [LaunchBuffers(max_events, self.max_roads, self.max_hits, pin_memory)
                     for _ in range(n_slots)]
        self.clock = clock
        self.keep_results = keep_results
        self.spin = spin
        self.results = {}
        self.launch_sizes = []
        self.fill_seconds = 0.0   # host time spent merging bursts into launch buffers

    def warm(self):
        """One full-size launch per slot, all in flight together, so that the
        device's staging pool holds buffers for the largest launches before
        the first burst arrives."""
        ranges, ne, nr, nh = [], 0, 0, 0
        while True:
            ce, cr, ch = self.pool.counts(0, self.pool.batch.n_events)
            room = (self.max_events - ne, self.max_roads - nr, self.max_hits - nh)
            if ce <= room[0] and cr <= room[1] and ch <= room[2]:
                ranges.append((0, self.pool.batch.n_events))
                ne, nr, nh = ne + ce, nr + cr, nh + ch
                continue
            # the largest prefix of the pool that still fits
            lo, hi = 0, self.pool.batch.n_events
            while lo < hi:
                mid = (lo + hi + 1) // 2
                ce, cr, ch = self.pool.counts(0, mid)
                if ce <= room[0] and cr <= room[1] and ch <= room[2]:
                    lo = mid
                else:
                    hi = mid - 1
            if lo:
                ranges.append((0, lo))
            break
        tickets = []
        for slot in range(len(self.bufs)):
            self.bufs[slot].fill(self.pool, ranges)
            st, t = self.device.submit(slot, self.bufs[slot])
            if st != 0:
                raise RuntimeError(f"warm-up submit failed with status {st}")
            tickets.append(t)
        for t in tickets:
            while True:
                self.clock()
                fin, st = self.device.poll(t)
                if fin:
                    if st != 0:
                        raise RuntimeError(f"warm-up launch failed with status {st}")
                    break

    def run(self, arrivals):
        """Serve the bursts; returns their records (latencies in seconds)."""
        recs = [BurstRecord(i, a, e0, e1) for i, (a, e0, e1) in enumerate(arrivals)]
        order = sorted(range(len(recs)), key=lambda i: recs[i].arrival)
        nxt = 0
        queue = collections.deque()
        busy = {}            # slot -> (ticket, [record indices])
        free = list(range(len(self.bufs)))
        done = 0
        n_launch = 0
        t0 = self.clock()
        while done < len(recs):
            now = self.clock() - t0
            while nxt < len(order) and recs[order[nxt]].arrival <= now:
                queue.append(order[nxt])
                nxt += 1
            # admit: every free slot takes the waiting bursts that fit in it
            while free and queue:
                slot = free[-1]
                take, ne, nr, nh = [], 0, 0, 0
                while queue:
                    r = recs[queue[0]]
                    ce, cr, ch = self.pool.counts(r.e0, r.e1)
                    if take and (ne + ce > self.max_events or nr + cr > self.max_roads or
                                 nh + ch > self.max_hits):
                        break
                    take.append(queue.popleft())
                    ne, nr, nh = ne + ce, nr + cr, nh + ch
                t_fill = self.clock()
                self.bufs[slot].fill(self.pool, [(recs[i].e0, recs[i].e1) for i in take])
                self.fill_seconds += self.clock() - t_fill
                st, ticket = self.device.submit(slot, self.bufs[slot])
                if st != 0:
                    for i in reversed(take):
                        queue.appendleft(i)
                    if (st == self.device.NOMEM or st == -5) and busy:
                        break          # wait for a completion to free memory / a ticket
                    raise RuntimeError(f"submit failed with status {st} with nothing in flight")
                free.pop()
                t_sub = self.clock() - t0
                for i in take:
                    recs[i].submit = t_sub
                    recs[i].launch = n_launch
                self.launch_sizes.append(ne)
                busy[slot] = (ticket, take)
                n_launch += 1
            # complete
            progressed = False
            for slot in list(busy):
                ticket, take = busy[slot]
                fin, st = self.device.poll(ticket)
                if not fin:
                    continue
                if st != 0:
                    raise RuntimeError(f"launch failed with status {st}")
                t_done = self.clock() - t0
                if self.keep_results:
                    self._demux(slot, take, recs)
                for i in take:
                    recs[i].done = t_done
                done += len(take)
                del busy[slot]
                free.append(slot)
                progressed = True
            if not progressed and self.spin:
                time.sleep(self.spin)
        return recs

    def _demux(self, slot, take, recs):
        bufs = self.bufs[slot]
        ev = rd = 0
        for i in take:
            r = recs[i]
            ce, cr, _ = self.pool.counts(r.e0, r.e1)
            self.results[i] = bufs.results(rd, rd + cr, ev, ev + ce)
            ev += ce
            rd += cr


class PlainServer:
    """Baseline: every event of every burst is its own launch (FIFO, one
    stream, up to `window` launches in flight)."""

    def __init__(self, ctx, pool: HostPool, window=32, clock=time.perf_counter):
        import torch
        from . import svt
        self.ctx = ctx
        self.pool = pool
        self.window = window
        self.clock = clock
        b = pool.batch
        ne = b.n_events
        ro, ho = pool.ro, pool.ho
        # per-event CSR offsets in pinned memory: [0, n_roads_e] and rebased hit offsets
        self.ro_ev = torch.from_numpy(np.stack([np.zeros(ne, np.int64), np.diff(ro)], 1)
                                      .astype(np.int32)).pin_memory()
        ho_ev = np.empty(b.n_roads + ne, np.int32)
        self.ho_start = (ro[:-1] + np.arange(ne)).astype(np.int64)
        for e in range(ne):
            a, c = int(ro[e]), int(ro[e + 1])
            ho_ev[self.ho_start[e]:self.ho_start[e] + (c - a) + 1] = ho[a:c + 1] - ho[a]
        self.ho_ev = torch.from_numpy(ho_ev).pin_memory()
        pin = lambda shape, dt: torch.zeros(shape, dtype=dt).pin_memory()
        nr = b.n_roads
        self.res = dict(ncomb=pin(nr, torch.int32), npass=pin(nr, torch.int32),
                        best=pin(nr, torch.int32), chi2=pin(nr, torch.int64),
                        params=pin((nr, 3), torch.int32), hit_index=pin((nr, 4), torch.uint8),
                        ntracks=pin(ne, torch.int32))
        self.stream = torch.cuda.Stream()
        self.svt = svt

    def _structs(self, e):
        svt, p = self.svt, self.pool
        r0, r1 = int(p.ro[e]), int(p.ro[e + 1])
        h0, h1 = int(p.ho[r0]), int(p.ho[r1])
        b = svt.svt_event_batch(1, r1 - r0, h1 - h0, svt.SVT_MEM_PINNED,
                                self.ro_ev.data_ptr() + 8 * e,
                                p.t["sector"].data_ptr() + r0, p.t["nhits"].data_ptr() + 4 * r0,
                                self.ho_ev.data_ptr() + 4 * int(self.ho_start[e]),
                                p.t["hits"].data_ptr() + 2 * h0, p.t["xft"].data_ptr() + 4 * r0)
        R = self.res
        r = svt.svt_results(R["ncomb"].data_ptr() + 4 * r0, R["npass"].data_ptr() + 4 * r0,
                            R["best"].data_ptr() + 4 * r0, R["chi2"].data_ptr() + 8 * r0,
                            R["params"].data_ptr() + 12 * r0, R["hit_index"].data_ptr() + 4 * r0,
                            R["ntracks"].data_ptr() + 4 * e, None, svt.SVT_MEM_PINNED, 0)
        return b, r

    def run(self, arrivals, time_limit=None):
        svt = self.svt
        recs = [BurstRecord(i, a, e0, e1) for i, (a, e0, e1) in enumerate(arrivals)]
        order = sorted(range(len(recs)), key=lambda i: recs[i].arrival)
        inflight = collections.deque()     # (ticket, record index, last event of the burst?)
        t0 = self.clock()
        st_handle = self.stream.cuda_stream

        def drain(keep):
            while len(inflight) > keep:
                tk, i, last = inflight.popleft()
                st, _ = svt.svt_result(self.ctx.handle, tk, -1)
                svt.check(st, "plain fit")
                if last:
                    recs[i].done = self.clock() - t0

        for i in order:
            r = recs[i]
            while self.clock() - t0 < r.arrival:
                drain(0) if inflight else None
            r.submit = self.clock() - t0
            for e in range(r.e0, r.e1):
                b, rr = self._structs(e)
                while True:
                    st, tk = svt.svt_fit_events(self.ctx.handle, b, rr, st_handle)
                    if st != svt.SVT_E_AGAIN:
                        break
                    drain(len(inflight) - 1)
                svt.check(st, "plain submit")
                inflight.append((tk, i, e == r.e1 - 1))
                drain(self.window)
            if time_limit is not None and self.clock() - t0 > time_limit:
                break
        drain(0)
        return [r for r in recs if r.done >= 0]


def latency_stats(recs):
    lat = np.array([r.latency for r in recs if r.done >= 0]) * 1e6
    if lat.size == 0:
        return dict(n=0)
    return dict(n=int(lat.size), p50_us=float(np.percentile(lat, 50)),
                p99_us=float(np.percentile(lat, 99)), max_us=float(lat.max()),
                mean_us=float(lat.mean()))
