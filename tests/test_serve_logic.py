"""Serving loop logic on the CPU with a simulated device: open-loop arrivals,
FIFO admission, continuous batching while launches are in flight, admission
by a device-memory budget, and per-burst demultiplexing."""
import numpy as np

from paper_1311_0380_amd import serve, synth


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-6          # every look at the clock advances it by 1 us
        return self.t


class SimDevice:
    """Completes a launch `cost(roads)` seconds after its submission; refuses
    launches whose bytes would exceed the budget next to those in flight."""

    NOMEM = -3

    def __init__(self, clock, budget_bytes, per_road_s=2e-8, fixed_s=20e-6):
        self.clock, self.budget = clock, budget_bytes
        self.per_road, self.fixed = per_road_s, fixed_s
        self.inflight = {}
        self.next = 1
        self.submitted = []

    def submit(self, slot, bufs):
        ne, nr, nh = bufs.n
        need = 70 * nr + 2 * nh + 8 * ne
        if sum(b for _, b in self.inflight.values()) + need > self.budget:
            return self.NOMEM, 0
        t = self.next
        self.next += 1
        self.inflight[t] = (self.clock.t + self.fixed + self.per_road * nr, need)
        self.submitted.append((slot, bufs.n))
        return 0, t

    def poll(self, ticket):
        end, _ = self.inflight[ticket]
        if self.clock.t < end:
            return False, 0
        del self.inflight[ticket]
        return True, 0


def pool_batch():
    b, _ = synth.cfg2(seed=9, n_events=400)
    return b


def test_every_burst_completes_once_in_fifo_order():
    clock = FakeClock()
    pool = serve.HostPool(pool_batch(), pin=False)
    dev = SimDevice(clock, budget_bytes=1 << 30)
    srv = serve.Server(dev, pool, n_slots=3, max_events=500, clock=clock, pin_memory=False)
    rng = np.random.default_rng(1)
    arr = serve.make_arrivals(rng, 200, 2e5, pool.batch.n_events, max_events=300)
    recs = srv.run(arr)
    assert all(r.done > r.arrival and r.submit >= r.arrival for r in recs)
    # FIFO: submission order follows arrival order
    subs = sorted(recs, key=lambda r: r.arrival)
    assert all(a.submit <= b.submit for a, b in zip(subs, subs[1:]))
    assert sum(srv.launch_sizes) == sum(r.e1 - r.e0 for r in recs)


def test_bursts_merge_while_device_is_busy():
    clock = FakeClock()
    pool = serve.HostPool(pool_batch(), pin=False)
    dev = SimDevice(clock, budget_bytes=1 << 30, per_road_s=2e-7)
    srv = serve.Server(dev, pool, n_slots=1, max_events=2000, clock=clock, pin_memory=False)
    arr = [(i * 1e-6, i, i + 3) for i in range(50)]      # much faster than one launch
    recs = srv.run(arr)
    launches = {r.launch for r in recs}
    assert len(launches) < len(recs)                    # continuous batching merged bursts
    assert max(srv.launch_sizes) > 3


def test_budget_limits_bytes_in_flight():
    clock = FakeClock()
    pool = serve.HostPool(pool_batch(), pin=False)
    budget = 70 * 64 * 60 + 2 * 64 * 60 * 16 + 8 * 60
    dev = SimDevice(clock, budget_bytes=budget, per_road_s=1e-7)
    srv = serve.Server(dev, pool, n_slots=4, max_events=50, clock=clock, pin_memory=False)
    arr = [(0.0, 10 * i, 10 * i + 10) for i in range(30)]
    peak = []
    orig = dev.submit

    def watch(slot, bufs):
        st, t = orig(slot, bufs)
        peak.append(sum(b for _, b in dev.inflight.values()))
        return st, t
    dev.submit = watch
    recs = srv.run(arr)
    assert len(recs) == 30 and max(peak) <= budget


def test_demux_slices_match_merged_layout():
    clock = FakeClock()
    b = pool_batch()
    pool = serve.HostPool(b, pin=False)
    bufs = serve.LaunchBuffers(100, 10000, 200000, pin_memory=False)
    ranges = [(5, 9), (100, 101), (30, 42)]
    bufs.fill(pool, ranges)
    merged = synth.concat([b.select_events(e0, e1) for e0, e1 in ranges])
    ne, nr, nh = bufs.n
    assert (ne, nr, nh) == (merged.n_events, merged.n_roads, merged.n_hits)
    assert np.array_equal(bufs.ro.numpy()[:ne + 1], merged.road_offsets)
    assert np.array_equal(bufs.ho.numpy()[:nr + 1], merged.hit_offsets)
    assert np.array_equal(bufs.hits.numpy()[:nh], merged.hits)
    assert np.array_equal(bufs.sector.numpy()[:nr], merged.sector)
    assert np.array_equal(bufs.nhits.numpy()[:nr], merged.nhits)
    assert np.array_equal(bufs.xft.numpy()[:nr], merged.xft)


def test_arrivals_shape():
    rng = np.random.default_rng(3)
    arr = serve.make_arrivals(rng, 5000, 1e5, 3000)
    t = np.array([a for a, _, _ in arr])
    sizes = np.array([e1 - e0 for _, e0, e1 in arr])
    assert np.all(np.diff(t) > 0) and sizes.min() >= 1 and sizes.max() <= 3000
    rate = sizes.sum() / t[-1]
    assert 0.8e5 < rate < 1.25e5


def test_warm_fills_every_slot_to_the_launch_limits():
    clock = FakeClock()
    pool = serve.HostPool(pool_batch(), pin=False)
    dev = SimDevice(clock, budget_bytes=1 << 30)
    srv = serve.Server(dev, pool, n_slots=3, max_events=900, clock=clock, pin_memory=False)
    srv.warm()
    assert sorted(s for s, _ in dev.submitted) == [0, 1, 2]
    for _, (ne, nr, nh) in dev.submitted:
        assert ne <= srv.max_events and nr <= srv.max_roads and nh <= srv.max_hits
        # two whole pools (800 events) plus the largest prefix that still fits
        assert ne == 900 or nr > srv.max_roads - 70 or nh > srv.max_hits - 70 * 16
    assert not dev.inflight
