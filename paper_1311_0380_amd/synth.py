"""Seeded synthetic inputs for the SVT linearized track fit.

This module only *produces inputs*: events made of roads, roads made of hits,
per-sector constant sets and the chi2 cut.  It holds none of the fit's
arithmetic (no fit rows, no chi2, no combination enumeration); both the CPU
oracle and the HIP library consume what it returns.

Shapes follow the paper's problem statement (Sec. 2: roads found per event,
one hit per layer per combination, per-sector constants f_i, q_i) and the
Sec. 4 workload, in which every event has the same road and combination
counts and batches run from 1 to 3000 events.  The paper's own data (CDF SVT events and
constant files) is not available; these generators stand in for it.

Conventions used throughout:
  * a road has 4 combinatorial silicon layers plus 2 XFT words; the fit input of
    a combination is x = (h0, h1, h2, h3, xft0, xft1), each in [0, 4096);
  * constants per sector s: coef[s] is 6x6 (rows 0..2 parameter words d0, phi,
    curvature; rows 3..5 chi2 constraint components), offset[s] has 6 entries;
  * hits of a road are stored layer-major: the n0 layer-0 hits, then n1
    layer-1 hits, and so on.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

HIT_RANGE = 4096          # hit and XFT words are 12-bit: [0, 4096)
N_LAYERS = 4              # combinatorial silicon layers per road
N_INPUTS = 6              # 4 silicon hits + 2 XFT words
N_SECTORS = 72
MAX_HITS_PER_LAYER = 16

# Track model used to build exact-recovery constants.  Rows are the six fit
# inputs (4 silicon layers at relative radii 1, 2, 3, 6, then the XFT
# curvature word and the XFT phi word); columns are the track parameters
# theta = (d, phi, c).  Integer entries so that hits on a track are integers.
TRACK_H = np.array([[6, 1, 1],
                    [3, 1, 2],
                    [2, 1, 3],
                    [1, 1, 6],
                    [0, 0, 1],
                    [0, 1, 12]], dtype=np.int64)

# Integer left-null basis of TRACK_H (NULL_N @ TRACK_H == 0).
NULL_N = np.array([[0, -1, 2, -1, 2, 0],
                   [-1, 3, -1, -1, 4, 0],
                   [-1, 3, 1, -5, -2, 2]], dtype=np.int64)

# Integer left inverse of TRACK_H scaled by 5 (LEFT_INV5 @ TRACK_H == 5 I),
# built from input rows 0, 3 and 4.
LEFT_INV5 = np.zeros((3, 6), dtype=np.int64)
LEFT_INV5[:, [0, 3, 4]] = np.array([[1, -1, 5],
                                    [-1, 6, -35],
                                    [0, 0, 5]], dtype=np.int64)
RECOVERY_SCALE = 5

CUT_CFG1 = 1 << 42
CUT_LATTICE = 1 << 32


@dataclasses.dataclass
class Batch:
    """One batch of events in CSR/SoA layout (host numpy arrays)."""
    road_offsets: np.ndarray   # int32 [n_events + 1]
    sector: np.ndarray         # uint8 [n_roads]
    nhits: np.ndarray          # uint8 [n_roads, 4]
    hit_offsets: np.ndarray    # int32 [n_roads + 1]
    hits: np.ndarray           # int16 [n_hits]
    xft: np.ndarray            # int16 [n_roads, 2]
    # generator bookkeeping (not fit inputs): which roads carry a planted track,
    # the planted track's hit position per layer (-1 for random roads), theta.
    track_road: np.ndarray = None
    track_pos: np.ndarray = None
    track_theta: np.ndarray = None

    @property
    def n_events(self) -> int:
        return int(self.road_offsets.shape[0] - 1)

    @property
    def n_roads(self) -> int:
        return int(self.sector.shape[0])

    @property
    def n_hits(self) -> int:
        return int(self.hits.shape[0])

    def nbytes(self) -> int:
        return sum(int(a.nbytes) for a in (self.road_offsets, self.sector, self.nhits,
                                            self.hit_offsets, self.hits, self.xft))

    def select_events(self, e0: int, e1: int) -> "Batch":
        """Events [e0, e1) as a self-contained batch (offsets rebased)."""
        r0, r1 = int(self.road_offsets[e0]), int(self.road_offsets[e1])
        h0, h1 = int(self.hit_offsets[r0]), int(self.hit_offsets[r1])
        sub = Batch(
            road_offsets=(self.road_offsets[e0:e1 + 1] - r0).astype(np.int32),
            sector=self.sector[r0:r1].copy(),
            nhits=self.nhits[r0:r1].copy(),
            hit_offsets=(self.hit_offsets[r0:r1 + 1] - h0).astype(np.int32),
            hits=self.hits[h0:h1].copy(),
            xft=self.xft[r0:r1].copy())
        if self.track_road is not None:
            sub.track_road = self.track_road[r0:r1].copy()
            sub.track_pos = self.track_pos[r0:r1].copy()
            sub.track_theta = self.track_theta[r0:r1].copy()
        return sub


@dataclasses.dataclass
class Constants:
    coef: np.ndarray     # int32 [n_sectors, 6, 6]
    offset: np.ndarray   # int32 [n_sectors, 6]
    chi2_cut: int
    x0: np.ndarray = None  # int64 [n_sectors, 6] lattice origin (lattice constants only)

    @property
    def n_sectors(self) -> int:
        return int(self.coef.shape[0])


def concat(batches) -> Batch:
    """Concatenate batches event-wise (offsets rebased)."""
    batches = list(batches)
    ro, ho = [np.zeros(1, np.int64)], [np.zeros(1, np.int64)]
    rbase = hbase = 0
    for b in batches:
        ro.append(b.road_offsets[1:].astype(np.int64) + rbase)
        ho.append(b.hit_offsets[1:].astype(np.int64) + hbase)
        rbase += b.n_roads
        hbase += b.n_hits
    return Batch(road_offsets=np.concatenate(ro).astype(np.int32),
                 sector=np.concatenate([b.sector for b in batches]),
                 nhits=np.concatenate([b.nhits for b in batches]).reshape(-1, 4),
                 hit_offsets=np.concatenate(ho).astype(np.int32),
                 hits=np.concatenate([b.hits for b in batches]),
                 xft=np.concatenate([b.xft for b in batches]).reshape(-1, 2))


# --------------------------------------------------------------------------
# constants
# --------------------------------------------------------------------------
# ---- packed word stream ------------------------------------------------------
# A self-defined stand-in for the raw input the paper's unpack step reads
# (the SVT word format itself is not available).  32-bit words, the top two
# bits a tag:
#   3 event header : bits 29..0 zero; the roads up to the next event header
#                    belong to this event
#   2 road header  : bits 29..22 sector, bits 19..0 the hit counts of layers
#                    0..3 (5 bits each, layer 0 lowest), bits 21..20 zero
#   1 XFT word     : bits 11..0 first XFT word, bits 23..12 second, 29..24 zero
#   0 hit word     : two hits of the road (layer-major order), bits 11..0 the
#                    first, bits 23..12 the second (zero in a road's last word
#                    when its hit count is odd), bits 29..24 zero
# A road is its header, its XFT word and ceil(hits / 2) hit words.
STREAM_HIT, STREAM_XFT, STREAM_ROAD, STREAM_EVENT = 0, 1, 2, 3


def pack_stream(batch: "Batch") -> np.ndarray:
    """The batch as a packed word stream (uint32)."""
    ne, nr = batch.n_events, batch.n_roads
    nh = batch.nhits.astype(np.int64).reshape(nr, 4)
    tot = nh.sum(axis=1)
    length = 2 + (tot + 1) // 2                        # words per road
    ro = batch.road_offsets.astype(np.int64)
    cl = np.concatenate([[0], np.cumsum(length)])
    ev_words = 1 + cl[ro[1:]] - cl[ro[:-1]]
    ev_start = np.concatenate([[0], np.cumsum(ev_words)])
    words = np.zeros(int(ev_start[-1]), np.uint32)
    words[ev_start[:-1]] = np.uint32(STREAM_EVENT << 30)
    ev_of_road = np.repeat(np.arange(ne), np.diff(ro))
    road_start = ev_start[ev_of_road] + 1 + cl[:-1] - cl[ro[ev_of_road]]
    counts = nh[:, 0] | (nh[:, 1] << 5) | (nh[:, 2] << 10) | (nh[:, 3] << 15)
    words[road_start] = ((STREAM_ROAD << 30) | (batch.sector.astype(np.int64) << 22) |
                         counts).astype(np.uint32)
    xf = batch.xft.astype(np.int64).reshape(nr, 2)
    words[road_start + 1] = ((STREAM_XFT << 30) | (xf[:, 1] << 12) | xf[:, 0]).astype(np.uint32)
    ho = batch.hit_offsets.astype(np.int64)
    road_of_hit = np.repeat(np.arange(nr), np.diff(ho))
    j = np.arange(batch.n_hits) - ho[road_of_hit]
    widx = road_start[road_of_hit] + 2 + j // 2
    val = (batch.hits.astype(np.int64) << (12 * (j % 2))).astype(np.uint32)
    np.bitwise_or.at(words, widx, val)
    return words


def uniform_constants(rng: np.random.Generator, n_sectors=N_SECTORS, lo=-1024, hi=1024,
                      chi2_cut=CUT_CFG1) -> Constants:
    """Constants drawn uniformly from [lo, hi) (the small plain-fit workload)."""
    coef = rng.integers(lo, hi, size=(n_sectors, 6, 6), dtype=np.int64).astype(np.int32)
    offset = rng.integers(lo, hi, size=(n_sectors, 6), dtype=np.int64).astype(np.int32)
    return Constants(coef=coef, offset=offset, chi2_cut=int(chi2_cut))


def lattice_constants(rng: np.random.Generator, n_sectors=N_SECTORS, m_range=40, k_range=20,
                      x0_range=8, chi2_cut=CUT_LATTICE) -> Constants:
    """Constants under which hits on a linear track have exactly zero chi2.

    Per sector: constraint rows C = M N (so C H = 0) and parameter rows
    F = LEFT_INV5 + K N (so F H = 5 I), with random integer mixing matrices
    M, K; offsets place the track manifold at an integer origin x0:
    b = -(A x0).  For x = x0 + H theta this gives parameter words 5 theta and
    constraint components 0.
    """
    m = rng.integers(-m_range, m_range + 1, size=(n_sectors, 3, 3), dtype=np.int64)
    k = rng.integers(-k_range, k_range + 1, size=(n_sectors, 3, 3), dtype=np.int64)
    x0 = rng.integers(-x0_range, x0_range + 1, size=(n_sectors, 6), dtype=np.int64)
    c_rows = m @ NULL_N                       # [S,3,6]
    f_rows = LEFT_INV5[None] + k @ NULL_N     # [S,3,6]
    coef = np.concatenate([f_rows, c_rows], axis=1)   # [S,6,6]
    assert np.abs(coef).max() < 1024
    offset = -np.einsum("skj,sj->sk", coef, x0)
    return Constants(coef=coef.astype(np.int32), offset=offset.astype(np.int32),
                     chi2_cut=int(chi2_cut), x0=x0)


# --------------------------------------------------------------------------
# events
# --------------------------------------------------------------------------
def _draw_theta(rng, x0_rows: np.ndarray) -> np.ndarray:
    """Integer track parameters with every input word inside [0, 4096)."""
    n = x0_rows.shape[0]
    theta = np.zeros((n, 3), np.int64)
    todo = np.arange(n)
    while todo.size:
        t = np.stack([rng.integers(0, 341, todo.size),
                      rng.integers(0, 1001, todo.size),
                      rng.integers(0, 251, todo.size)], axis=1)
        x = x0_rows[todo] + t @ TRACK_H.T
        ok = np.all((x >= 0) & (x < HIT_RANGE), axis=1)
        theta[todo[ok]] = t[ok]
        todo = todo[~ok]
    return theta


def make_events(rng: np.random.Generator, roads_per_event: np.ndarray, nhits: np.ndarray,
                n_sectors: int, track_mask: np.ndarray = None,
                consts: Constants = None) -> Batch:
    """Build a batch from per-event road counts and per-road hit counts.

    roads_per_event: int [n_events]; nhits: int [n_roads, 4];
    track_mask: bool [n_roads] roads that carry one planted track (requires
    lattice constants, whose x0 places the track manifold).
    """
    roads_per_event = np.asarray(roads_per_event, np.int64)
    n_roads = int(roads_per_event.sum())
    nhits = np.asarray(nhits, np.int64).reshape(n_roads, 4)
    road_offsets = np.zeros(roads_per_event.size + 1, np.int64)
    np.cumsum(roads_per_event, out=road_offsets[1:])
    per_road = nhits.sum(axis=1)
    hit_offsets = np.zeros(n_roads + 1, np.int64)
    np.cumsum(per_road, out=hit_offsets[1:])
    n_hits = int(hit_offsets[-1])
    sector = rng.integers(0, n_sectors, n_roads)
    hits = rng.integers(0, HIT_RANGE, n_hits)
    xft = rng.integers(0, HIT_RANGE, (n_roads, 2))
    track_pos = np.full((n_roads, 4), -1, np.int64)
    theta = np.zeros((n_roads, 3), np.int64)
    if track_mask is None:
        track_mask = np.zeros(n_roads, bool)
    track_mask = np.asarray(track_mask, bool) & np.all(nhits > 0, axis=1)
    tr = np.nonzero(track_mask)[0]
    if tr.size:
        assert consts is not None and consts.x0 is not None
        th = _draw_theta(rng, consts.x0[sector[tr]])
        theta[tr] = th
        xtrue = consts.x0[sector[tr]] + th @ TRACK_H.T       # [T,6]
        # layer start offsets inside each road (layer-major)
        lstart = hit_offsets[tr][:, None] + np.concatenate(
            [np.zeros((tr.size, 1), np.int64), np.cumsum(nhits[tr], axis=1)[:, :3]], axis=1)
        pos = (rng.random((tr.size, 4)) * nhits[tr]).astype(np.int64)
        track_pos[tr] = pos
        # noise hits in a track road's layer differ from the true word
        for layer in range(4):
            seg_lo = lstart[:, layer]
            seg_n = nhits[tr, layer]
            idx = np.repeat(seg_lo, seg_n) + _ragged_arange(seg_n)
            want = np.repeat(xtrue[:, layer], seg_n)
            clash = hits[idx] == want
            while clash.any():
                hits[idx[clash]] = rng.integers(0, HIT_RANGE, int(clash.sum()))
                clash = hits[idx] == want
            hits[seg_lo + pos[:, layer]] = xtrue[:, layer]
        xft[tr] = xtrue[:, 4:6]
    return Batch(road_offsets=road_offsets.astype(np.int32),
                 sector=sector.astype(np.uint8),
                 nhits=nhits.astype(np.uint8),
                 hit_offsets=hit_offsets.astype(np.int32),
                 hits=hits.astype(np.int16),
                 xft=xft.astype(np.int16),
                 track_road=track_mask, track_pos=track_pos, track_theta=theta)


def _ragged_arange(counts: np.ndarray) -> np.ndarray:
    counts = np.asarray(counts, np.int64)
    if counts.size == 0:
        return np.zeros(0, np.int64)
    ends = np.cumsum(counts)
    starts = np.repeat(ends - counts, counts)
    return np.arange(int(ends[-1]), dtype=np.int64) - starts


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def cfg1(seed: int = 1, n_events: int = 100):
    """Small plain fit: 100 events x 8 roads, 1-2 hits per layer, uniform
    constants in [-2^10, 2^10), cut 2^42."""
    rng = np.random.default_rng(seed)
    consts = uniform_constants(rng)
    rpe = np.full(n_events, 8)
    nh = rng.integers(1, 3, (int(rpe.sum()), 4))
    return make_events(rng, rpe, nh, consts.n_sectors), consts


def cfg2(seed: int = 2, n_events: int = 3000, roads_per_event: int = 64,
         tracks_per_event: int = 32):
    """Scaled-up plain fit: 3000 events x 64 roads, 1-4 hits per layer,
    lattice constants, half of each event's roads carry a planted track."""
    rng = np.random.default_rng(seed)
    consts = lattice_constants(rng)
    rpe = np.full(n_events, roads_per_event)
    n_roads = int(rpe.sum())
    nh = rng.integers(1, 5, (n_roads, 4))
    mask = np.zeros((n_events, roads_per_event), bool)
    order = rng.random((n_events, roads_per_event)).argsort(axis=1)
    np.put_along_axis(mask, order[:, :tracks_per_event], True, axis=1)
    return make_events(rng, rpe, nh, consts.n_sectors, mask.ravel(), consts), consts


def cfg3(seed: int = 3, n_events: int = 10000):
    """Uneven batching: roads/event Geometric(1/16) on {1,..} clipped to 256,
    hits/layer Poisson(1.5) clipped to [1, 8], lattice constants, each road
    carries a planted track with probability 1/2."""
    rng = np.random.default_rng(seed)
    consts = lattice_constants(rng)
    rpe = np.minimum(rng.geometric(1.0 / 16.0, n_events), 256)
    n_roads = int(rpe.sum())
    nh = np.clip(rng.poisson(1.5, (n_roads, 4)), 1, 8)
    mask = rng.random(n_roads) < 0.5
    return make_events(rng, rpe, nh, consts.n_sectors, mask, consts), consts


def paper_sweep(n_events: int, seed: int = 6):
    """The paper's benchmark shape (Sec. 4): every event has 2048
    combinations (8 roads x 4 hits in each of 4 layers), lattice constants,
    half the roads with a planted track."""
    rng = np.random.default_rng(seed)
    consts = lattice_constants(rng)
    rpe = np.full(n_events, 8)
    nh = np.full((n_events * 8, 4), 4)
    mask = np.zeros((n_events, 8), bool)
    mask[:, :4] = True
    return make_events(rng, rpe, nh, consts.n_sectors, mask.ravel(), consts), consts


PAPER_SWEEP_EVENTS = (1, 10, 100, 500, 1000, 2000, 3000)


def random_small(rng: np.random.Generator, n_events: int, max_roads: int, max_hits: int,
                 n_sectors: int, allow_empty: bool = True, consts: Constants = None,
                 track_frac: float = 0.0) -> Batch:
    """Tiny irregular batches for exhaustive checks (empty events and empty
    layers allowed)."""
    lo_r = 0 if allow_empty else 1
    rpe = rng.integers(lo_r, max_roads + 1, n_events)
    n_roads = int(rpe.sum())
    lo_h = 0 if allow_empty else 1
    nh = rng.integers(lo_h, max_hits + 1, (n_roads, 4))
    mask = rng.random(n_roads) < track_frac if track_frac > 0 else None
    return make_events(rng, rpe, nh, n_sectors, mask, consts)


# --------------------------------------------------------------------------
# trigger-style bursts (serving workload)
# --------------------------------------------------------------------------
def burst_sizes(rng: np.random.Generator, n: int, max_events: int = 3000) -> np.ndarray:
    """Burst sizes log-uniform on [1, max_events]: floor(exp(U[0, ln(max+1))))."""
    s = np.floor(np.exp(rng.uniform(0.0, math.log(max_events + 1), n))).astype(np.int64)
    return np.clip(s, 1, max_events)


def poisson_arrivals(rng: np.random.Generator, n: int, events_per_s: float,
                     mean_events_per_burst: float) -> np.ndarray:
    """Open-loop arrival times (seconds) of n bursts at the offered event rate."""
    rate = events_per_s / mean_events_per_burst
    return np.cumsum(rng.exponential(1.0 / rate, n))


def log_uniform_mean(max_events: int = 3000) -> float:
    """Expected burst size of burst_sizes() (exact sum over the integer support)."""
    L = math.log(max_events + 1)
    k = np.arange(1, max_events + 1, dtype=np.float64)
    p = (np.log(np.minimum(k + 1, max_events + 1)) - np.log(k)) / L
    return float((k * p).sum())


# --------------------------------------------------------------------------
# helix tracks for the float-shadow calibration workload
# --------------------------------------------------------------------------
@dataclasses.dataclass
class HelixGeometry:
    radii_cm: tuple = (3.0, 5.0, 7.0, 10.0)   # silicon layers
    xft_radius_cm: float = 100.0              # XFT reference radius; Rmax = this radius
    n_sectors: int = 72                       # phi sectors of 5 degrees (sector set at layer 2)
    pitch_um: float = 4.0                     # silicon word unit (local arc length)
    word_center: float = 2048.0
    sigma_um: float = 10.0                    # silicon hit smearing
    d0_sigma_um: float = 50.0
    xft_phi_unit_urad: float = 300.0          # XFT phi word unit (local angle at Rmax)
    xft_curv_words: float = 2000.0            # words per unit of curvature * Rmax
    xft_sigma_words: float = 1.0              # XFT word smearing
    # parameter-word units of the truth (d0 [um], local phi0 [urad], curvature * Rmax * 1e3)
    truth_scale: tuple = (1.0, 1.0, 1000.0)


@dataclasses.dataclass
class HelixTracks:
    x: np.ndarray              # float64 [N, 6] unquantized input words
    xq: np.ndarray             # int16 [N, 6] words rounded to integers (clipped to [0, 4095])
    truth: np.ndarray          # float64 [N, 3] parameter words (d0 um, phi0 urad, 1e3 c Rmax)
    sector: np.ndarray         # int32 [N] ascending (tracks grouped by sector)
    sector_offsets: np.ndarray # int32 [n_sectors + 1] tracks of sector s: [off[s], off[s+1])
    kept: np.ndarray           # bool [N] all six rounded words inside [0, 4096)
    dropped: int               # generated tracks removed because a word left [0, 4096)


def helix_tracks(n: int, seed: int = 4, geom: HelixGeometry = None) -> HelixTracks:
    """Charged tracks in the transverse plane for the calibration workload.

    d0 ~ N(0, 50 um), phi0 ~ U[0, 2 pi), curvature ~ U[-1, 1] / Rmax with Rmax
    the XFT radius; silicon hits smeared with N(0, 10 um).  Each input word
    is a local coordinate inside the track's 5 degree phi sector (the sector
    is the one the track crosses at layer 2): silicon words are the arc
    position / pitch + 2048 at each layer radius; the XFT words are the
    curvature and the local phi at the XFT radius.  The circle / cylinder
    intersection is exact.  Tracks with a word outside [0, 4096) after
    rounding are dropped (and counted); the rest are returned grouped by
    sector.
    """
    g = geom or HelixGeometry()
    rng = np.random.default_rng(seed)
    want = n
    xs, ts, ss = [], [], []
    dropped = 0
    width = 2.0 * np.pi / g.n_sectors
    rmax = g.xft_radius_cm
    while want > 0:
        m = int(want * 1.05) + 16
        d0 = rng.normal(0.0, g.d0_sigma_um, m) * 1e-4                 # cm
        phi0 = rng.uniform(0.0, 2.0 * np.pi, m)
        curv = rng.uniform(-1.0, 1.0, m) / rmax                         # signed 1/R in 1/cm

        def phi_at(r):
            # azimuth where a circle of curvature curv, impact parameter d0 and
            # direction phi0 at closest approach crosses radius r
            arg = (curv * r) / 2.0 + (d0 / r) * (1.0 + curv * d0 / 2.0) / (1.0 + curv * d0)
            return phi0 + np.arcsin(np.clip(arg, -1.0, 1.0))

        sector = np.floor(np.mod(phi_at(g.radii_cm[2]), 2.0 * np.pi) / width).astype(np.int64)
        sector = np.minimum(sector, g.n_sectors - 1)
        center = (sector + 0.5) * width
        x = np.zeros((m, 6))
        for layer, r in enumerate(g.radii_cm):
            dphi = np.angle(np.exp(1j * (phi_at(r) - center)))
            arc_um = dphi * r * 1e4 + rng.normal(0.0, g.sigma_um, m)
            x[:, layer] = arc_um / g.pitch_um + g.word_center
        x[:, 4] = curv * rmax * g.xft_curv_words + g.word_center \
            + rng.normal(0.0, g.xft_sigma_words, m)
        dphi_x = np.angle(np.exp(1j * (phi_at(rmax) - center)))
        x[:, 5] = dphi_x * 1e6 / g.xft_phi_unit_urad + g.word_center \
            + rng.normal(0.0, g.xft_sigma_words, m)
        truth = np.stack([d0 * 1e4 * g.truth_scale[0],
                          np.angle(np.exp(1j * (phi0 - center))) * 1e6 * g.truth_scale[1],
                          curv * rmax * g.truth_scale[2]], axis=1)
        ok = np.all((np.rint(x) >= 0) & (np.rint(x) < HIT_RANGE), axis=1)
        dropped += int((~ok).sum())
        take = np.nonzero(ok)[0][:want]
        xs.append(x[take]); ts.append(truth[take]); ss.append(sector[take])
        want -= take.size
    x = np.concatenate(xs); truth = np.concatenate(ts); sector = np.concatenate(ss)
    order = np.argsort(sector, kind="stable")
    x, truth, sector = x[order], truth[order], sector[order]
    off = np.zeros(g.n_sectors + 1, np.int64)
    np.add.at(off, sector + 1, 1)
    off = np.cumsum(off)
    xq = np.rint(x)
    return HelixTracks(x=x, xq=np.clip(xq, 0, HIT_RANGE - 1).astype(np.int16), truth=truth,
                       sector=sector.astype(np.int32), sector_offsets=off.astype(np.int32),
                       kept=np.ones(x.shape[0], bool), dropped=dropped)


def pilot_constants(h: HelixTracks, frac: float = 0.02, seed: int = 7):
    """Starting constants for calibration from a small pilot sample (the role
    nominal geometry constants play before a calibration): per sector, least
    squares of the truth on the words for rows 0..2, and the three
    smallest-variance directions of the words (unit rows, centred) for rows
    3..5.  float32 [S,6,6], [S,6]."""
    rng = np.random.default_rng(seed)
    n_s = h.sector_offsets.shape[0] - 1
    coef = np.zeros((n_s, 6, 6))
    off = np.zeros((n_s, 6))
    for s in range(n_s):
        a, e = int(h.sector_offsets[s]), int(h.sector_offsets[s + 1])
        take = rng.choice(np.arange(a, e), size=max(32, int((e - a) * frac)), replace=False)
        X = h.x[take]
        Xa = np.hstack([X, np.ones((X.shape[0], 1))])
        sol, *_ = np.linalg.lstsq(Xa, h.truth[take], rcond=None)
        coef[s, :3] = sol[:6].T
        off[s, :3] = sol[6]
        mu = X.mean(axis=0)
        _, vec = np.linalg.eigh(np.cov((X - mu).T))
        coef[s, 3:] = vec[:, :3].T
        off[s, 3:] = -coef[s, 3:] @ mu
    return coef.astype(np.float32), off.astype(np.float32)
