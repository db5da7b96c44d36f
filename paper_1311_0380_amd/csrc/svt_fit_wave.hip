// Wave-autonomous SVT fit kernel for gfx950 (arXiv:1311.0380, Sec. 2 and
// Sec. 2.1).
//
// Every wavefront is an independent worker: it takes a chunk of consecutive
// events (so each event, and its track count, belongs to one wavefront) and
// fits its roads in sub-chunks of at most 64 roads, one road per lane, with
// no block-wide barrier after the constants are staged.  Waves of a CU are
// therefore free to be in different phases: one loads while another fits.
//
//   A  lane = road: load and validate the road; one wave scan places its hits
//      and its (i0, i1) rows in the wave's LDS; a radix sort of the roads by
//      (n3, n2) orders the row list so that 64 consecutive rows share their
//      inner trip counts; the constant part of the constraint rows
//      b + A[:,4] x4 + A[:,5] x5 is formed from the sector's constants.
//   B  lane = row (i0, i1): every (i2, i3) combination in the row loops of
//      svt_rows.h; the row's best goes to its road with one LDS 64-bit
//      atomicMin on chi2 << 16 | i0 << 12 | i1 << 8 | i2 << 4 | i3, whose
//      order is the order of (chi2, combination index) since every n_l <= 16.
//   C  lane = road: decode the winner, recompute its parameter rows 0..2 in
//      int32, write the road's results, count tracks per event.
#include <hip/hip_ext.h>

#include "svt_internal.h"
#include "svt_rows.h"

namespace svt {
namespace {

constexpr int kWRoads = 64;       // roads per wave sub-chunk (one per lane)
constexpr int kWHitCap = 768;     // staged hit words per wave sub-chunk (>= 64)
constexpr int kWRowCap = 512;     // (i0, i1) rows per wave sub-chunk (>= 256)
constexpr int kWStage = kWHitCap / 64;
constexpr int kWaves = kBlock / 64;

struct WaveLds {
    double road[kWRoads][6];            // base of rows 3..5, packed road info, 2 pad
                                        // (48-byte stride: no LDS bank-group clash)
    unsigned long long key[kWRoads];    // best key of each road
    uint32_t np[kWRoads];               // passing combinations of each road
    uint32_t evcnt[kWRoads];            // tracks of each event of the chunk
    uint16_t row[kWRowCap];             // road | i0 << 6 | i1 << 10
    int16_t hit[kWHitCap + 16];         // staged hit words (+ pad read by row loops)
};

struct Acc {
    uint64_t comb = 0, pass = 0;
    uint32_t tracks = 0;
    uint32_t err_road = 0xFFFFFFFFu, err_event = 0xFFFFFFFFu;
};

// Fit roads [s, re) of the wave's chunk from road s on; returns how many
// roads were fitted (at least one).  ro_e holds road_offsets[eb + lane] for
// lanes 0..ne (the chunk's event boundaries).
template <bool F>
__device__ int wave_sub(const FitArgs &a, WaveLds &W, const double *s_pb, int32_t s, int32_t re,
                        int32_t n_roads, int32_t n_hits, int32_t n_sectors, double cut,
                        int32_t ne, int32_t ro_e, Acc &acc)
{
    const int lane = threadIdx.x & 63;
    const int32_t r = s + lane;
    const bool inr = r < re;

    uint32_t sec = 0, nh4 = 0, x2 = 0;
    int32_t h0 = 0, h1 = 0;
    if (inr) {
        sec = a.sector[r];
        nh4 = a.nhits4[r];
        h0 = a.hit_offsets[r];
        h1 = a.hit_offsets[r + 1];
        x2 = a.xft2[r];
    }
    const uint32_t n0 = nh4 & 255u, n1 = (nh4 >> 8) & 255u, n2 = (nh4 >> 16) & 255u,
                   n3 = nh4 >> 24;
    const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
    const uint32_t sum = n0 + n1 + n2 + n3;
    bool ok = inr && sec < (uint32_t)n_sectors && n0 <= 16 && n1 <= 16 && n2 <= 16 && n3 <= 16;
    ok = ok && h0 >= 0 && h1 <= n_hits && (int64_t)h1 - (int64_t)h0 == (int64_t)sum;
    ok = ok && (r != 0 || h0 == 0) && (r != n_roads - 1 || h1 == n_hits);
    ok = ok && xa >= 0 && xa < 4096 && xb >= 0 && xb < 4096;
    if (inr && !ok) acc.err_road = min(acc.err_road, (uint32_t)r);
    // the sector's constants for the base of rows 3..5, in flight with the
    // hit words below
    double cb[9];
    {
        const double *src = a.cst_base + (size_t)(ok ? sec : 0u) * kCstBaseStride;
#pragma unroll
        for (int q = 0; q < 9; ++q) cb[q] = src[q];
    }

    // hits (<= 64 per road) and rows (<= 256 per road) of the roads before
    // this one, packed in one 32-bit scan (totals stay below 2^16)
    const uint32_t nh = ok ? sum : 0u;
    const uint32_t rows = (ok && n2 * n3 > 0) ? n0 * n1 : 0u;
    const uint32_t pk = nh | (rows << 16);
    const uint32_t incl = wave_incl_scan(pk);
    const uint32_t hb = (incl - pk) & 0xFFFFu, rend = incl >> 16;
    const bool fits = inr && hb + nh <= (uint32_t)kWHitCap && rend <= (uint32_t)kWRowCap;
    const int L = __popcll(__ballot(fits));          // fits is a prefix of the lanes
    const bool active = lane < L;
    const uint32_t T = __builtin_amdgcn_readlane(incl & 0xFFFFu, L - 1);
    const uint32_t R = __builtin_amdgcn_readlane(rend, L - 1);
    const int32_t hs = clampi(__builtin_amdgcn_readfirstlane(h0), 0, n_hits);

    // stage the hit words (coalesced), checking each word's range
    int16_t v[kWStage];
#pragma unroll
    for (int q = 0; q < kWStage; ++q) {
        const int32_t t = lane + q * 64, g = hs + t;
        v[q] = (t < (int32_t)T && g < n_hits) ? a.hits[g] : (int16_t)0;
    }
    bool bad_hit = false;
#pragma unroll
    for (int q = 0; q < kWStage; ++q) {
        const int32_t t = lane + q * 64;
        if (t < (int32_t)T) {
            W.hit[t] = v[q];
            bad_hit |= v[q] < 0 || v[q] >= 4096;
        }
    }

    // the road's record: base of rows 3..5 (exact in int32, held as fp64)
    // and its packed counts, hit base and sector
    if (active) {
        const double b3 = fma(cb[3], (double)xb, fma(cb[0], (double)xa, cb[6]));
        const double b4 = fma(cb[4], (double)xb, fma(cb[1], (double)xa, cb[7]));
        const double b5 = fma(cb[5], (double)xb, fma(cb[2], (double)xa, cb[8]));
        const unsigned long long info = (unsigned long long)(ok ? nh4 : 0u) |
                                        ((unsigned long long)hb << 32) |
                                        ((unsigned long long)(ok ? sec : 0u) << 48);
        W.road[lane][0] = b3;
        W.road[lane][1] = b4;
        W.road[lane][2] = b5;
        W.road[lane][3] = __longlong_as_double((long long)info);
        W.key[lane] = ~0ull;
        W.np[lane] = 0u;
    }

    // order the roads by (n3, n2) with a stable radix sort across the lanes,
    // over the key bits that occur (roads without rows hold no rows, so
    // where they land does not matter)
    const uint32_t rows_a = active ? rows : 0u;
    const uint32_t k2 = rows_a ? n2 - 1u : 0u, k3 = rows_a ? n3 - 1u : 0u;
    const uint32_t m2 = wave_max(k2), m3 = wave_max(k3);
    const uint32_t b2 = m2 ? 32u - (uint32_t)__builtin_clz(m2) : 0u;
    const uint32_t b3 = m3 ? 32u - (uint32_t)__builtin_clz(m3) : 0u;
    uint32_t pv = (((k3 << 4) | k2) << 8) | (uint32_t)lane;
    for (uint32_t t = 0; t < b2 + b3; ++t) {
        const uint32_t bit = t < b2 ? t : 4u + (t - b2);
        const bool one = (pv >> (8 + bit)) & 1u;
        const uint64_t m1 = __ballot(one);
        const uint32_t n_zero = 64u - (uint32_t)__popcll(m1);
        const uint32_t dst = one ? n_zero + lanes_below(m1) : lanes_below(~m1);
        pv = (uint32_t)__builtin_amdgcn_ds_permute((int)(dst << 2), (int)pv);
    }
    const int src = (int)(pv & 63u);
    const uint32_t rows_s = (uint32_t)__shfl((int)rows_a, src, 64);
    const uint32_t ex_s = wave_incl_scan(rows_s) - rows_s;
    const uint32_t rbase = (uint32_t)__builtin_amdgcn_ds_permute(src << 2, (int)ex_s);
    if (rows_a) {
        uint32_t w = rbase;
        for (uint32_t i0 = 0; i0 < n0; ++i0)
            for (uint32_t i1 = 0; i1 < n1; ++i1, ++w)
                W.row[w] = (uint16_t)((uint32_t)lane | (i0 << 6) | (i1 << 10));
    }
    wave_sync();

    if (__ballot(bad_hit)) {
        // a hit word out of range: each road checks its own staged words
        if (active && ok) {
            for (uint32_t t = 0; t < nh; ++t) {
                const int16_t h = W.hit[hb + t];
                if (h < 0 || h >= 4096) {
                    acc.err_road = min(acc.err_road, (uint32_t)r);
                    break;
                }
            }
        }
    }

    // B: every combination of every row
    const double lim = F ? cut + 0.5 : cut;
    for (uint32_t w0 = 0; w0 < R; w0 += 64) {
        const uint32_t idx = w0 + (uint32_t)lane;
        const bool act = idx < R;
        const uint32_t d = W.row[act ? idx : R - 1];
        const uint32_t j = d & 63u, i0 = (d >> 6) & 15u, i1 = (d >> 10) & 15u;
        const double b3 = W.road[j][0], b4 = W.road[j][1], b5 = W.road[j][2];
        const unsigned long long info = (unsigned long long)__double_as_longlong(W.road[j][3]);
        const uint32_t rn = (uint32_t)info, hbj = (uint32_t)(info >> 32) & 0xFFFFu,
                       sj = (uint32_t)(info >> 48);
        const uint32_t rn0 = rn & 255u, rn1 = (rn >> 8) & 255u, rn2 = (rn >> 16) & 255u,
                       rn3 = rn >> 24;
        const double *cs = s_pb + sj * kCstPbStride;   // [col][row], columns 0..3 of rows 3..5
        const double h0v = (double)W.hit[hbj + i0], h1v = (double)W.hit[hbj + rn0 + i1];
        Row st;
        st.z3 = fma(cs[3], h1v, fma(cs[0], h0v, b3));
        st.z4 = fma(cs[4], h1v, fma(cs[1], h0v, b4));
        st.z5 = fma(cs[5], h1v, fma(cs[2], h0v, b5));
        st.a3 = cs[6];
        st.a4 = cs[7];
        st.a5 = cs[8];
        st.c3 = cs[9];
        st.c4 = cs[10];
        st.c5 = cs[11];
        st.best = F ? __builtin_inf() : cut + 1.0;
        st.bidx = 0xFFFFFFFFu;
        st.np = 0;
        run_row<F>(st, W.hit, hbj + rn0 + rn1, hbj + rn0 + rn1 + rn2, rn2, rn3, lim);
        if (act) {
            unsigned long long key;
            if (row_key<F>(st, cut, (i0 << 12) | (i1 << 8), 4u, 0u, key)) atomicMin(&W.key[j], key);
            if (st.np) atomicAdd(&W.np[j], st.np);
        }
    }
    wave_sync();

    // the road's event: largest e < ne with road_offsets[eb + e] <= r (every
    // lane takes part: a lane reads other lanes' boundaries)
    int ev = 0;
#pragma unroll
    for (int b = 32; b > 0; b >>= 1) {
        const int cand = ev + b;
        const int32_t v = __shfl(ro_e, cand < ne ? cand : ne, 64);
        ev = (cand < ne && v <= r) ? cand : ev;
    }

    // C: results of each road.  Its counts, hit base and sector come back
    // from LDS (zero counts for a malformed road give the same outputs as
    // the road's error path), which keeps phase A's values out of phase B.
    if (active) {
        const unsigned long long info =
            (unsigned long long)__double_as_longlong(W.road[lane][3]);
        const uint32_t c4 = (uint32_t)info, hb = (uint32_t)(info >> 32) & 0xFFFFu,
                       sec = (uint32_t)(info >> 48);
        const uint32_t n0 = c4 & 255u, n1 = (c4 >> 8) & 255u, n2 = (c4 >> 16) & 255u,
                       n3 = c4 >> 24;
        const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
        const unsigned long long key = W.key[lane];
        const uint32_t np = W.np[lane];
        const bool found = key != ~0ull;
        int32_t bk = -1;
        uint64_t c2 = ~0ull;
        int32_t p[3] = {0, 0, 0};
        uint32_t hi4 = 0xFFFFFFFFu;
        if (found) {
            const uint32_t i0 = (uint32_t)(key >> 12) & 15u, i1 = (uint32_t)(key >> 8) & 15u,
                           i2 = (uint32_t)(key >> 4) & 15u, i3 = (uint32_t)key & 15u;
            c2 = key >> 16;
            bk = (int32_t)(((i0 * n1 + i1) * n2 + i2) * n3 + i3);
            hi4 = i0 | (i1 << 8) | (i2 << 16) | (i3 << 24);
            const uint32_t x[6] = {(uint32_t)(int32_t)W.hit[hb + i0],
                                   (uint32_t)(int32_t)W.hit[hb + n0 + i1],
                                   (uint32_t)(int32_t)W.hit[hb + n0 + n1 + i2],
                                   (uint32_t)(int32_t)W.hit[hb + n0 + n1 + n2 + i3],
                                   (uint32_t)xa, (uint32_t)xb};
            // parameter rows 0..2, exact in int32 by the load-time bound
            const int32_t *ci = a.cst_par + (size_t)sec * kCstParStride;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                uint32_t acc32 = (uint32_t)ci[k * 8 + 6];
#pragma unroll
                for (int col = 0; col < 6; ++col)
                    acc32 += (uint32_t)__mul24(ci[k * 8 + col], (int32_t)x[col]);
                p[k] = (int32_t)acc32;
            }
            atomicAdd(&W.evcnt[ev], 1u);
        }
        // written once, never read back here: streaming stores
        __builtin_nontemporal_store((int32_t)(n0 * n1 * n2 * n3), &a.ncomb[r]);
        __builtin_nontemporal_store((int32_t)np, &a.npass[r]);
        __builtin_nontemporal_store(bk, &a.best[r]);
        __builtin_nontemporal_store(c2, &a.chi2[r]);
        __builtin_nontemporal_store(p[0], &a.params[3 * (int64_t)r + 0]);
        __builtin_nontemporal_store(p[1], &a.params[3 * (int64_t)r + 1]);
        __builtin_nontemporal_store(p[2], &a.params[3 * (int64_t)r + 2]);
        __builtin_nontemporal_store(hi4, &a.hit_index4[r]);
        acc.comb += n0 * n1 * n2 * n3;
        acc.pass += np;
        acc.tracks += found ? 1u : 0u;
    }
    wave_sync();
    return L;
}

// The chunks of this wavefront: 1 = cyclic (chunk c -> wave c mod waves),
// 2 = blocked (each wave a contiguous range).
struct ChunkRange {
    int32_t c0, step, c1;
};

__device__ __forceinline__ ChunkRange chunk_range(const FitArgs &a, int32_t n_chunks)
{
    const int32_t gw = (int32_t)blockIdx.x * kWaves + (int32_t)(threadIdx.x >> 6);
    const int32_t nw = (int32_t)gridDim.x * kWaves;
    if (a.schedule == 2)
        return ChunkRange{(int32_t)((int64_t)n_chunks * gw / nw), 1,
                          (int32_t)((int64_t)n_chunks * (gw + 1) / nw)};
    return ChunkRange{gw, nw, n_chunks};
}

// Event boundaries of chunk c: lane e holds road_offsets[c * E + e] for
// e <= ne, a large value above.
__device__ __forceinline__ int32_t chunk_bounds(const FitArgs &a, int32_t c, int32_t n_events)
{
    const int lane = threadIdx.x & 63;
    const int32_t eb = c * a.events_per_chunk;
    const int32_t ne = min(a.events_per_chunk, n_events - eb);
    return lane <= ne ? a.road_offsets[eb + lane] : 0x7FFFFFFF;
}

template <bool F>
__device__ __forceinline__ void run_chunks(const FitArgs &a, WaveLds &W, const double *s_pb,
                                           int32_t n_events, int32_t n_roads, int32_t n_hits,
                                           const ChunkRange cr, int32_t ro_first, Acc &acc)
{
    const int lane = threadIdx.x & 63;
    const int32_t E = a.events_per_chunk;
    const int32_t c0 = cr.c0, step = cr.step, c1 = cr.c1;
    for (int32_t c = c0; c < c1; c += step) {
        const int32_t eb = c * E;
        const int32_t ne = min(E, n_events - eb);
        // event boundaries: lane e holds road_offsets[eb + e] for e <= ne
        const int32_t ro_e = c == c0 ? ro_first : chunk_bounds(a, c, n_events);
        const int32_t ro_n = __shfl_down(ro_e, 1, 64);
        if (lane < ne) {
            const int32_t e = eb + lane;
            const bool bad = ro_e < 0 || ro_n < ro_e || ro_n > n_roads || (e == 0 && ro_e != 0) ||
                             (e == n_events - 1 && ro_n != n_roads);
            if (bad) acc.err_event = min(acc.err_event, (uint32_t)e);
        }
        const int32_t ra = clampi(__builtin_amdgcn_readfirstlane(ro_e), 0, n_roads);
        const int32_t rb = clampi(__builtin_amdgcn_readlane(ro_e, ne), ra, n_roads);
        W.evcnt[lane] = 0u;
        wave_sync();
        for (int32_t s = ra; s < rb;)
            s += wave_sub<F>(a, W, s_pb, s, rb, n_roads, n_hits, a.n_sectors, a.cut_d, ne, ro_e,
                             acc);
        if (lane < ne) a.ntracks[eb + lane] = (int32_t)W.evcnt[lane];
        wave_sync();
    }
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
fit_wave_kernel(FitArgs a)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    __shared__ WaveLds s_w[kWaves];
    const int tid = threadIdx.x;

    int32_t n_events = a.n_events, n_roads = a.n_roads, n_hits = a.n_hits;
    if (a.sizes != nullptr) {
        n_events = a.sizes->n_events;
        n_roads = a.sizes->n_roads;
        n_hits = a.sizes->n_hits;
    }
    // the first chunk's event boundaries are in flight while the columns 0..3
    // of every sector's constraint rows are staged in LDS
    const int32_t n_chunks =
        n_events > 0 ? (n_events + a.events_per_chunk - 1) / a.events_per_chunk : 0;
    const ChunkRange cr = chunk_range(a, n_chunks);
    const int32_t ro_first = cr.c0 < cr.c1 ? chunk_bounds(a, cr.c0, n_events) : 0;
    double *s_pb = reinterpret_cast<double *>(s_dyn);
    for (int i = tid; i < a.n_sectors * kCstPbStride; i += kBlock) s_pb[i] = a.cst_pb[i];
    __syncthreads();

    Acc acc;
    WaveLds &W = s_w[tid >> 6];
    if (a.frac_key)
        run_chunks<true>(a, W, s_pb, n_events, n_roads, n_hits, cr, ro_first, acc);
    else
        run_chunks<false>(a, W, s_pb, n_events, n_roads, n_hits, cr, ro_first, acc);

    // block sums -> host-mapped partials (the host reduces them)
    const int lane = tid & 63, wid = tid >> 6;
    uint64_t comb = acc.comb, pass = acc.pass;
    uint32_t trk = acc.tracks, er = acc.err_road, ee = acc.err_event;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        comb += __shfl_xor(comb, off, 64);
        pass += __shfl_xor(pass, off, 64);
        trk += __shfl_xor(trk, off, 64);
        er = min(er, (uint32_t)__shfl_xor(er, off, 64));
        ee = min(ee, (uint32_t)__shfl_xor(ee, off, 64));
    }
    __shared__ BlockPartial s_part[kWaves];
    if (lane == 0) s_part[wid] = BlockPartial{comb, pass, trk, er, ee, 0};
    __syncthreads();
    if (tid == 0) {
        BlockPartial p = s_part[0];
        for (int w = 1; w < kWaves; ++w) {
            p.comb += s_part[w].comb;
            p.pass += s_part[w].pass;
            p.tracks += s_part[w].tracks;
            p.err_road = min(p.err_road, s_part[w].err_road);
            p.err_event = min(p.err_event, s_part[w].err_event);
        }
        p.seq = request_seq(a);
        a.partials[blockIdx.x] = p;
    }
}

}  // namespace

hipError_t prepare_fit_wave()
{
    const int max_dyn = 256 * kCstPbStride * (int)sizeof(double);
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fit_wave_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn);
}

hipError_t launch_fit_wave(const FitArgs &a, int grid, hipStream_t stream, hipEvent_t start,
                           hipEvent_t stop)
{
    const size_t dyn = (size_t)a.n_sectors * kCstPbStride * sizeof(double);
    if (start != nullptr || stop != nullptr)
        hipExtLaunchKernelGGL(fit_wave_kernel, dim3(grid), dim3(kBlock), (uint32_t)dyn, stream,
                              start, stop, 0u, a);
    else
        hipLaunchKernelGGL(fit_wave_kernel, dim3(grid), dim3(kBlock), dyn, stream, a);
    return hipGetLastError();
}

}  // namespace svt
