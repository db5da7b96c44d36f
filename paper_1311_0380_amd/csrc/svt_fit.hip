// Fused SVT fit kernel for gfx950 (arXiv:1311.0380, Sec. 2 / Sec. 2.1).
//
// One persistent grid.  Work item = a chunk of `events_per_chunk` consecutive
// events, so every event (and its track count) belongs to exactly one block.
// A chunk's roads are processed in sub-chunks of at most kSubRoads roads whose
// hits (kHitCap) and (i0, i1) rows (kRowCap) fit in LDS:
//
//   A  one thread per road: load + validate the road, prefix sums give each
//      road its slot in the LDS hit table and row list.  The road's two
//      layers with the fewest hits index its rows (c, d) and the other two
//      (a, b) are looped over inside each row, which gives the fewest and
//      longest rows.  Rows are binned by (n_a, n_b) so that a wavefront's
//      rows share their inner trip counts; the hits are staged in LDS
//      (coalesced, flattened); the constraint rows' constant part
//      b + A[:,4] x4 + A[:,5] x5 is formed.
//   B  one thread per row (i_c, i_d): z = base + A[:,c] h_c + A[:,d] h_d,
//      then every (i_a, i_b) combination in the row loops of svt_rows.h.
//      The row's best is merged into the road with one LDS atomicMin on the
//      key chi2 << 16 | i0 << 12 | i1 << 8 | i2 << 4 | i3, whose order is
//      the order of (chi2, combination index k) because each i_l < n_l <= 16.
//   C  one thread per road: decode the winner, recompute its parameter rows
//      0..2 exactly in int32, write the road's results, count tracks per event.
//
// Each block writes its partial sums to host-mapped memory; the host reduces
// them when the request completes.
#include <hip/hip_ext.h>

#include "svt_internal.h"
#include "svt_rows.h"

namespace svt {
namespace {

constexpr int kBins = 17 * 17;   // (n2, n3) in 0..16 x 0..16
constexpr int kWaves = kBlock / 64;
static_assert(kMaxEventsPerChunk <= kBlock, "one thread per event of a chunk");

// Inclusive scans across the wavefront: of two packed 32-bit counters
// (neither half may overflow), and of one 64-bit value.
__device__ __forceinline__ uint64_t wave_incl_scan_pair(uint64_t x)
{
    const uint32_t lo = wave_incl_scan((uint32_t)x), hi = wave_incl_scan((uint32_t)(x >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t t = __shfl_up(x, off, 64);
        if (lane >= off) x += t;
    }
    return x;
}

// Block-wide exclusive scan: of packed 32-bit pairs (PAIR) or of 64-bit values.
template <bool PAIR>
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t *s_warp, uint64_t &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t incl = PAIR ? wave_incl_scan_pair(v) : wave_incl_scan64(v);
    if (lane == 63) s_warp[wid] = incl;
    __syncthreads();
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        uint64_t s = s_warp[w];
        before += (w < wid) ? s : 0;
        tot += s;
    }
    total = tot;
    __syncthreads();
    return before + incl - v;
}

// Sums of a wavefront, kept as uniform values (wave reductions at the end of
// every sub-chunk keep them out of the per-lane registers).
struct Acc {
    uint64_t comb = 0, pass = 0;
    uint32_t tracks = 0;
    uint32_t err_road = 0xFFFFFFFFu, err_event = 0xFFFFFFFFu;
};

struct Shared {
    double base[3][kSubRoads];              // b + A[:,4] x4 + A[:,5] x5, rows 3..5
    // per road: staged hit index of the first hit of layers a, b (x) and
    // c, d (y); n_a | n_b << 8 | (a | b << 2 | c << 4 | d << 6) << 16 (z);
    // sector (w)
    uint4 rec[kSubRoads];
    unsigned long long key[kSubRoads];      // best key of each road
    uint32_t n4[kSubRoads];                 // packed hit counts of each road
    uint32_t np[kSubRoads];                 // passing combinations of each road
    uint16_t hb[kSubRoads];                 // first staged hit of each road
    uint16_t row[kRowCap];                  // road | i0 << 8 | i1 << 12, binned by (n2, n3)
    int16_t hit[kHitCap + 16];              // staged hit words (+ pad read by row loops)
    uint32_t bin[kBins];
    uint32_t bstart[kBins];
    int32_t evro[kMaxEventsPerChunk + 1];
    uint32_t evcnt[kMaxEventsPerChunk];
    uint64_t warp[kWaves];
    uint32_t fitc[kWaves];
    int32_t misc[4];
};

constexpr int kStage = kHitCap / kBlock;    // staged hits per thread

// Process the roads [s, rb) of the current chunk starting at road s; returns
// how many roads were fitted (at least one when s < rb).
template <bool F>
__device__ int process_sub(const FitArgs &a, Shared &S, const double *s_cd, int32_t s, int32_t rb,
                           int32_t n_roads, int32_t n_hits, int32_t n_sectors, int32_t ne,
                           double cut, Acc &acc)
{
    const int tid = threadIdx.x;
    const int32_t r = s + tid;
    const bool inr = r < rb;

    // one round of loads: the sub-chunk's hit range (uniform), each thread's
    // road, and a speculative copy of the hits the next kSubRoads roads hold
    const int32_t s_end = min(rb, s + kSubRoads);
    const int32_t hs = clampi(a.hit_offsets[s], 0, n_hits);
    const int32_t he = clampi(a.hit_offsets[s_end], hs, n_hits);
    const int32_t t_pre = min(he - hs, kHitCap);
    uint32_t sec = 0, nh4 = 0, x2 = 0;
    int32_t h0 = 0, h1 = 0;
    if (inr) {
        sec = a.sector[r];
        nh4 = a.nhits4[r];
        h0 = a.hit_offsets[r];
        h1 = a.hit_offsets[r + 1];
        x2 = a.xft2[r];
    }
    int16_t v[kStage];
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
        const int t = tid + q * kBlock;
        v[q] = t < t_pre ? a.hits[hs + t] : (int16_t)0;
    }

    const uint32_t n0 = nh4 & 255u, n1 = (nh4 >> 8) & 255u, n2 = (nh4 >> 16) & 255u,
                   n3 = nh4 >> 24;
    const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
    const uint32_t sum = n0 + n1 + n2 + n3;
    bool ok = inr && sec < (uint32_t)n_sectors && n0 <= 16 && n1 <= 16 && n2 <= 16 && n3 <= 16;
    ok = ok && h0 >= 0 && h1 <= n_hits && (int64_t)h1 - (int64_t)h0 == (int64_t)sum;
    ok = ok && (r != 0 || h0 == 0) && (r != n_roads - 1 || h1 == n_hits);
    ok = ok && xa >= 0 && xa < 4096 && xb >= 0 && xb < 4096;
    acc.err_road = min(acc.err_road, wave_min(inr && !ok ? (uint32_t)r : 0xFFFFFFFFu));

    const uint32_t nh = ok ? sum : 0u;
    // row layers c < d: the two with the fewest hits (ties to the lower
    // layer); inner layers a < b: the other two
    uint32_t rowmask = 0;
    {
        const uint32_t nl[4] = {n0, n1, n2, n3};
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            uint32_t rk = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (m != l) rk += (nl[m] < nl[l] || (nl[m] == nl[l] && m < l)) ? 1u : 0u;
            rowmask |= (rk < 2 ? 1u : 0u) << l;
        }
    }
    // the layers and their counts are derived again where they are used,
    // which keeps only the mask live across the scan's barriers
    auto lay = [](uint32_t m, int q) {   // q = 0..3: c, d, a, b
        return q == 0 ? (uint32_t)__builtin_ctz(m)
             : q == 1 ? 31u - (uint32_t)__builtin_clz(m)
             : q == 2 ? (uint32_t)__builtin_ctz(m ^ 15u) : 31u - (uint32_t)__builtin_clz(m ^ 15u);
    };
    auto cnt = [](uint32_t c4, uint32_t l) { return (c4 >> (8 * l)) & 255u; };
    auto off = [](uint32_t c4, uint32_t l) {   // hits of the layers before l
        return ((c4 & ((1u << (8 * l)) - 1u)) * 0x01010101u) >> 24;
    };
    const uint32_t rows =
        (ok && n0 * n1 * n2 * n3 > 0) ? cnt(nh4, lay(rowmask, 0)) * cnt(nh4, lay(rowmask, 1)) : 0u;
    // block scan of (hits, rows); the roads that fit are a prefix of the
    // block, counted per wave and summed across the scan's second barrier
    const uint64_t pk = (uint64_t)nh | ((uint64_t)rows << 32);
    const uint64_t incl = wave_incl_scan_pair(pk);
    const int lane = tid & 63, wid = tid >> 6;
    if (lane == 63) S.warp[wid] = incl;
    __syncthreads();
    uint64_t before = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) before += (w < wid) ? S.warp[w] : 0ull;
    const uint64_t ex = before + incl - pk;
    const uint32_t hb = (uint32_t)ex, rbase = (uint32_t)(ex >> 32);
    const bool fits = inr && hb + nh <= (uint32_t)kHitCap && rbase + rows <= (uint32_t)kRowCap;
    const uint32_t wfit = (uint32_t)__popcll(__ballot(fits));
    if (lane == 0) S.fitc[wid] = wfit;
    __syncthreads();
    int L = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) L += (int)S.fitc[w];
    const bool active = tid < L;   // fits is a prefix of the block

    if (tid == L - 1) {
        S.misc[1] = (int32_t)(hb + nh);           // hits of the sub-chunk
        S.misc[3] = (int32_t)(rbase + rows);      // rows of the sub-chunk
    }
    const uint32_t bkey = cnt(nh4, lay(rowmask, 3)) * 17u + cnt(nh4, lay(rowmask, 2));   // n_b major
    uint32_t boff = 0;
    if (active) {
        S.hb[tid] = (uint16_t)hb;
        {
            const uint32_t lc = lay(rowmask, 0), ld = lay(rowmask, 1), la = lay(rowmask, 2),
                           lb = lay(rowmask, 3);
            S.rec[tid] = make_uint4((hb + off(nh4, la)) | ((hb + off(nh4, lb)) << 16),
                                    (hb + off(nh4, lc)) | ((hb + off(nh4, ld)) << 16),
                                    cnt(nh4, la) | (cnt(nh4, lb) << 8) |
                                        ((la | (lb << 2) | (lc << 4) | (ld << 6)) << 16),
                                    ok ? sec : 0u);
        }
        S.n4[tid] = ok ? nh4 : 0u;
        S.key[tid] = ~0ull;
        S.np[tid] = 0;
        if (rows) boff = atomicAdd(&S.bin[bkey], rows);
        if (ok) {
            // constant part of the constraint rows, exact in int32
            const double *cs = s_cd + sec * kCstStride;
            const int32_t *cb = reinterpret_cast<const int32_t *>(cs) + kCstIntB;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                S.base[k][tid] = fma(cs[15 + k], (double)xb, fma(cs[12 + k], (double)xa, (double)cb[k]));
        }
    }
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
        const int t = tid + q * kBlock;
        if (t < t_pre) S.hit[t] = v[q];
    }
    __syncthreads();
    const int32_t T = S.misc[1], total_rows = S.misc[3];
    // range of the hit words: the speculative copy, then hits it did not
    // cover (only possible with inconsistent offsets), each checked by the
    // thread that holds it
    int32_t bad_t = INT32_MAX;
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
        const int t = tid + q * kBlock;
        if (t < T && t < t_pre && (v[q] < 0 || v[q] >= 4096)) bad_t = min(bad_t, t);
    }
    for (int t = t_pre + tid; t < T; t += kBlock) {
        const int32_t g = hs + t;
        const int16_t h = g < n_hits ? a.hits[g] : (int16_t)0;
        S.hit[t] = h;
        if (h < 0 || h >= 4096) bad_t = min(bad_t, t);
    }
    uint32_t bad_hit_road = 0xFFFFFFFFu;
    if (bad_t != INT32_MAX) {
        int lo = 0, hi = L;     // last road with hb <= bad_t
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if ((int32_t)S.hb[mid] <= bad_t) lo = mid; else hi = mid;
        }
        bad_hit_road = (uint32_t)(s + lo);
    }
    acc.err_road = min(acc.err_road, wave_min(bad_hit_road));
    // bin starts: every wavefront scans the 289 bins itself (lane l holds
    // bins 5l .. 5l+4) and fetches its roads' starts across lanes, so no
    // barrier separates the scan from the row lists
    uint32_t bstart;
    {
        uint32_t vb[5], loc = 0;
        const int lb = (tid & 63) * 5;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            vb[q] = lb + q < kBins ? S.bin[lb + q] : 0u;
            loc += vb[q];
        }
        uint32_t run = wave_incl_scan(loc) - loc;
        // every wavefront writes the same starts, so a wavefront reading
        // after its own writes sees the right value whoever wrote last
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            if (lb + q < kBins) S.bstart[lb + q] = run;
            run += vb[q];
        }
        wave_sync();
        bstart = S.bstart[bkey];
    }

    // rows of the road, in (i_c, i_d) order, at its place in the binned list
    if (active && rows) {
        // the road's rows at [w, w + rows): an odd first slot alone, then
        // two rows per 32-bit store
        uint32_t w = bstart + boff, ic = 0, id = 0, k = 0;
        const uint32_t base = (uint32_t)tid, nd = cnt(nh4, lay(rowmask, 1));
        if (w & 1u) {
            S.row[w++] = (uint16_t)base;
            k = 1;
            id = 1 == nd ? 0u : 1u;
            ic = 1 == nd ? 1u : 0u;
        }
        for (; k + 1 < rows; k += 2, w += 2) {
            const uint32_t ra = base | (ic << 8) | (id << 12);
            if (++id == nd) { id = 0; ++ic; }
            const uint32_t rb2 = base | (ic << 8) | (id << 12);
            if (++id == nd) { id = 0; ++ic; }
            *reinterpret_cast<uint32_t *>(&S.row[w]) = ra | (rb2 << 16);
        }
        if (k < rows) S.row[w] = (uint16_t)(base | (ic << 8) | (id << 12));
    }
    __syncthreads();
    for (int i = tid; i < kBins; i += kBlock) S.bin[i] = 0;   // ready for the next sub-chunk

    // B: every combination of every row
    for (int idx0 = 0; idx0 < total_rows; idx0 += kBlock) {
        if (idx0 + (tid & ~63) >= total_rows) continue;   // whole wavefront idle
        const int idx = idx0 + tid;
        const bool act = idx < total_rows;
        const uint32_t d = S.row[act ? idx : total_rows - 1];
        const uint32_t j = d & 255u, ic = (d >> 8) & 15u, id = (d >> 12) & 15u;
        const uint4 rc = S.rec[j];
        const uint32_t rn2 = rc.z & 255u, rn3 = (rc.z >> 8) & 255u;
        const uint32_t la = (rc.z >> 16) & 3u, lb = (rc.z >> 18) & 3u, lc = (rc.z >> 20) & 3u,
                       ld = (rc.z >> 22) & 3u;
        // sector constants: column l of rows 3..5 at cs[3 l .. 3 l + 2]
        const double *cs = s_cd + rc.w * kCstStride;
        const double *ka = cs + 3 * la, *kb = cs + 3 * lb, *kc = cs + 3 * lc, *kd = cs + 3 * ld;
        const double hc = (double)S.hit[(rc.y & 0xFFFFu) + ic], hd = (double)S.hit[(rc.y >> 16) + id];
        Row st;
        st.z3 = fma(kd[0], hd, fma(kc[0], hc, S.base[0][j]));
        st.z4 = fma(kd[1], hd, fma(kc[1], hc, S.base[1][j]));
        st.z5 = fma(kd[2], hd, fma(kc[2], hc, S.base[2][j]));
        st.a3 = ka[0];
        st.a4 = ka[1];
        st.a5 = ka[2];
        st.c3 = kb[0];
        st.c4 = kb[1];
        st.c5 = kb[2];
        st.best = F ? __builtin_inf() : cut + 1.0;
        st.bidx = 0xFFFFFFFFu;
        st.np = 0;
        run_row<F>(st, S.hit, rc.x & 0xFFFFu, rc.x >> 16, rn2, rn3, F ? cut + 0.5 : cut);
        if (act) {
            // the row's indices and layers come back from LDS rather than
            // staying live across the row loops
            const uint32_t d2 = S.row[idx];
            const uint32_t j2 = d2 & 255u, lay = S.rec[j2].z >> 16;
            const uint32_t rowbits = (((d2 >> 8) & 15u) << (12u - 4u * ((lay >> 4) & 3u))) |
                                     (((d2 >> 12) & 15u) << (12u - 4u * ((lay >> 6) & 3u)));
            unsigned long long key;
            if (row_key<F>(st, cut, rowbits, 12u - 4u * (lay & 3u), 12u - 4u * ((lay >> 2) & 3u), key))
                atomicMin(&S.key[j2], key);
            if (st.np) atomicAdd(&S.np[j2], st.np);
        }
    }
    __syncthreads();

    // C: results of each road.  Its counts, hit base and sector come back
    // from LDS (zero counts for a malformed road give the same outputs as
    // the road's error path), which keeps phase A's values out of phase B.
    uint32_t my_comb = 0, my_pass = 0, my_track = 0;
    if (active) {
        const uint32_t c4 = S.n4[tid], hb = S.hb[tid], sec = S.rec[tid].w;
        const uint32_t n0 = c4 & 255u, n1 = (c4 >> 8) & 255u, n2 = (c4 >> 16) & 255u,
                       n3 = c4 >> 24;
        const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
        const unsigned long long key = S.key[tid];
        const uint32_t np = S.np[tid];
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
            const uint32_t x[6] = {(uint32_t)(int32_t)S.hit[hb + i0],
                                   (uint32_t)(int32_t)S.hit[hb + n0 + i1],
                                   (uint32_t)(int32_t)S.hit[hb + n0 + n1 + i2],
                                   (uint32_t)(int32_t)S.hit[hb + n0 + n1 + n2 + i3],
                                   (uint32_t)xa, (uint32_t)xb};
            // parameter rows 0..2, exact in int32 by the load-time bound
            const int32_t *ci = reinterpret_cast<const int32_t *>(s_cd + sec * kCstStride);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                uint32_t acc32 = (uint32_t)ci[kCstIntPB + k];
#pragma unroll
                for (int col = 0; col < 6; ++col)
                    acc32 += (uint32_t)__mul24(ci[kCstIntP + col * 3 + k], (int32_t)x[col]);
                p[k] = (int32_t)acc32;
            }
        }
        // results are written once and not read again by this kernel:
        // streaming stores keep them from filling (and later flushing) L2
        __builtin_nontemporal_store((int32_t)(n0 * n1 * n2 * n3), &a.ncomb[r]);
        __builtin_nontemporal_store((int32_t)np, &a.npass[r]);
        __builtin_nontemporal_store(bk, &a.best[r]);
        __builtin_nontemporal_store(c2, &a.chi2[r]);
        __builtin_nontemporal_store(p[0], &a.params[3 * (int64_t)r + 0]);
        __builtin_nontemporal_store(p[1], &a.params[3 * (int64_t)r + 1]);
        __builtin_nontemporal_store(p[2], &a.params[3 * (int64_t)r + 2]);
        __builtin_nontemporal_store(hi4, &a.hit_index4[r]);
        if (found) {
            int lo = 0, hi = ne;   // events [lo, hi): largest e with evro[e] <= r
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (S.evro[mid] <= r) lo = mid; else hi = mid;
            }
            atomicAdd(&S.evcnt[lo], 1u);
        }
        my_comb = n0 * n1 * n2 * n3;
        my_pass = np;
        my_track = found ? 1u : 0u;
    }
    acc.comb += wave_sum(my_comb);      // each at most 64 * 2^16
    acc.pass += wave_sum(my_pass);
    acc.tracks += wave_sum(my_track);
    __syncthreads();
    return L;
}

// The first event e in [0, n_events] with road_offsets[e] >= t, found by one
// wavefront: each round probes 64 evenly spaced events of the interval left
// and keeps the gap where the comparison turns (three rounds for 10^4
// events).  Every lane returns the same value.  For offsets that are not
// nondecreasing the result is still some event in [0, n_events].
__device__ __forceinline__ int32_t first_event_at(const int32_t *road_offsets, int32_t n_events, int64_t t)
{
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    int32_t lo = -1, hi = n_events;   // the answer lies in (lo, hi]
    while (hi - lo > 1) {
        const int32_t step = (hi - lo - 1 + 63) / 64;
        const int32_t p = lo + (lane + 1) * step;
        const bool ge = p >= hi || (int64_t)road_offsets[p] >= t;
        const uint64_t m = __ballot(ge);
        if (m == 0) {
            lo = __builtin_amdgcn_readlane(p, 63);
        } else {
            const int j = __ffsll((unsigned long long)m) - 1;
            const int32_t pj = __builtin_amdgcn_readlane(p, j);
            lo = j > 0 ? __builtin_amdgcn_readlane(p, j - 1) : lo;
            hi = pj < hi ? pj : hi;
        }
    }
    return hi;
}

// Static schedules (no shared counter): 1 = cyclic (chunk c -> block c mod
// grid), 2 = blocked (block b owns a contiguous range of chunks); schedule 3
// (balanced by roads) is set up in the kernel.
__device__ __forceinline__ void chunk_range(int32_t n_chunks, int32_t schedule, int32_t &first,
                                            int32_t &step, int32_t &last)
{
    if (schedule == 2) {
        const int64_t g = gridDim.x, b = blockIdx.x;
        first = (int32_t)((int64_t)n_chunks * b / g);
        last = (int32_t)((int64_t)n_chunks * (b + 1) / g);
        step = 1;
    } else {
        first = blockIdx.x;
        last = n_chunks;
        step = gridDim.x;
    }
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
fit_kernel(FitArgs a)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    __shared__ Shared S;
    const int tid = threadIdx.x;

    int32_t n_events = a.n_events, n_roads = a.n_roads, n_hits = a.n_hits;
    uint32_t seq = a.seq;
    if (a.sizes != nullptr) {
        n_events = a.sizes->n_events;
        n_roads = a.sizes->n_roads;
        n_hits = a.sizes->n_hits;
        seq = a.sizes->seq;
    }
    if (a.seq_dev != nullptr) seq = *a.seq_dev;
    const int32_t n_sectors = a.n_sectors;
    double *s_cd = reinterpret_cast<double *>(s_dyn);

    Acc acc;
    const double cut = a.cut_d;
    const int32_t E = a.events_per_chunk;
    // sector constants -> LDS: a copy of the image built at load time
    const uint4 *csrc = reinterpret_cast<const uint4 *>(a.cst_block);
    uint4 *cdst = reinterpret_cast<uint4 *>(s_cd);
    const int n16 = n_sectors * kCstBytesPerSector / 16;

    int32_t c_first, c_step, c_last;
    // chunk c covers events [e_base + c E, min(e_base + (c + 1) E, e_end))
    int32_t e_base = 0, e_end = n_events;
    if (a.schedule == 3) {
        // balanced by roads: block b takes the events whose first road lies
        // in [b R / G, (b + 1) R / G) (R roads, G blocks), found by wavefronts
        // 0 and 1; chunks of at most E events then split that range
        // meanwhile wavefronts 2 and 3 stage the sector constants and check
        // a share of the event offsets: every event's offsets are checked by
        // some block whatever the partition, so that malformed offsets cannot
        // escape the check
        const int wid = (int)(__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6);
        const int64_t G = gridDim.x, b = blockIdx.x;
        uint32_t bad_event = 0xFFFFFFFFu;
        if (wid < 2) {
            const int64_t bb = b + wid;
            const int32_t e = bb >= G ? n_events
                                      : first_event_at(a.road_offsets, n_events, (int64_t)n_roads * bb / G);
            if (tid == wid * 64) S.misc[wid] = e;
        } else {
            const int t2 = tid - 128;
            const int32_t per = (int32_t)((n_events + G - 1) / G);
            for (int32_t e = (int32_t)(b * per) + t2; e < min((int64_t)n_events, (b + 1) * per); e += 128) {
                const int32_t lo = a.road_offsets[e], hi = a.road_offsets[e + 1];
                const bool bad = lo < 0 || hi < lo || hi > n_roads || (e == 0 && lo != 0) ||
                                 (e == n_events - 1 && hi != n_roads);
                if (bad) bad_event = min(bad_event, (uint32_t)e);
            }
            for (int i = t2; i < n16; i += 128) cdst[i] = csrc[i];
        }
        acc.err_event = min(acc.err_event, wave_min(bad_event));
        __syncthreads();
        e_base = clampi(S.misc[0], 0, n_events);
        e_end = clampi(S.misc[1], e_base, n_events);
        c_first = 0;
        c_step = 1;
        c_last = (e_end - e_base + E - 1) / E;
        __syncthreads();   // S.misc is reused by the sub-chunks
    } else {
        const int32_t n_chunks = n_events > 0 ? (n_events + E - 1) / E : 0;
        chunk_range(n_chunks, a.schedule, c_first, c_step, c_last);
    }

    // the first chunk's event boundaries are in flight while the sector
    // constants are staged
    int32_t ev0 = 0, ev1 = 0;
    if (c_first < c_last) {
        const int32_t e0 = e_base + c_first * E, ne = min(E, e_end - e0);
        if (tid <= ne) ev0 = a.road_offsets[e0 + tid];
        if (tid + kBlock <= ne) ev1 = a.road_offsets[e0 + tid + kBlock];
    }

    if (a.schedule != 3)
        for (int i = tid; i < n16; i += kBlock) cdst[i] = csrc[i];
    for (int i = tid; i < kBins; i += kBlock) S.bin[i] = 0;

    if (c_first < c_last) {
        const int32_t ne = min(E, e_end - (e_base + c_first * E));
        if (tid <= ne) S.evro[tid] = ev0;
        if (tid + kBlock <= ne) S.evro[tid + kBlock] = ev1;
    }
    for (int32_t c = c_first; c < c_last; c += c_step) {
        const int32_t e0 = e_base + c * E;
        const int32_t ne = min(E, e_end - e0);
        if (c != c_first)
            for (int i = tid; i <= ne; i += kBlock) S.evro[i] = a.road_offsets[e0 + i];
        if (tid < ne) S.evcnt[tid] = 0;   // ne <= kMaxEventsPerChunk = kBlock
        __syncthreads();
        const int32_t ra = clampi(S.evro[0], 0, n_roads);
        const int32_t rb = clampi(S.evro[ne], ra, n_roads);
        for (int32_t s = ra; s < rb;)
            s += a.frac_key ? process_sub<true>(a, S, s_cd, s, rb, n_roads, n_hits, n_sectors, ne, cut, acc)
                            : process_sub<false>(a, S, s_cd, s, rb, n_roads, n_hits, n_sectors, ne, cut, acc);
        uint32_t bad_event = 0xFFFFFFFFu;
        for (int i = tid; i < ne; i += kBlock) {
            const int32_t e = e0 + i, lo = S.evro[i], hi = S.evro[i + 1];
            const bool bad = lo < 0 || hi < lo || hi > n_roads || (e == 0 && lo != 0) ||
                             (e == n_events - 1 && hi != n_roads);
            if (bad) bad_event = min(bad_event, (uint32_t)e);
            a.ntracks[e] = (int32_t)S.evcnt[i];
        }
        acc.err_event = min(acc.err_event, wave_min(bad_event));
        __syncthreads();
    }

    // block sums -> host-mapped partials (the host reduces them); the
    // wavefront sums are uniform already.  Lane and wave ids are recomputed
    // here rather than kept live across the whole kernel.
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int wid = (int)(__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6);
    __shared__ BlockPartial s_part[kWaves];
    if (lane == 0)
        s_part[wid] = BlockPartial{acc.comb, acc.pass, acc.tracks, acc.err_road, acc.err_event, 0};
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
        p.seq = seq;
        a.partials[blockIdx.x] = p;
    }
}

// ---------------------------------------------------------------------------
// comb_offsets: exclusive prefix sum of ncomb (int64), three small passes
// ---------------------------------------------------------------------------
constexpr int kScanTile = kBlock * 8;

__global__ void __launch_bounds__(kBlock) scan_tiles(const int32_t *ncomb, int32_t n, int64_t *tile_sum)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        const int64_t g = base + i;
        if (g < n) s += ncomb[g];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ int64_t w[kWaves];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < kWaves; ++q) t += w[q];
        tile_sum[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kBlock) scan_tile_sums(int64_t *tile_sum, int32_t n_tiles)
{
    __shared__ uint64_t warp[kWaves];
    int64_t carry = 0;
    for (int32_t b0 = 0; b0 < n_tiles; b0 += kBlock) {
        const int32_t b = b0 + threadIdx.x;
        const int64_t v = b < n_tiles ? tile_sum[b] : 0;
        uint64_t tot;
        const int64_t ex = (int64_t)block_excl_scan<false>((uint64_t)v, warp, tot);
        if (b < n_tiles) tile_sum[b] = carry + ex;
        carry += (int64_t)tot;
    }
    if (threadIdx.x == 0) tile_sum[n_tiles] = carry;
}

__global__ void __launch_bounds__(kBlock) scan_apply(const int32_t *ncomb, int32_t n,
                                                     const int64_t *tile_sum, int64_t *out)
{
    __shared__ uint64_t warp[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t carry = tile_sum[blockIdx.x];
    for (int i0 = 0; i0 < kScanTile; i0 += kBlock) {
        const int64_t g = base + i0 + threadIdx.x;
        const int64_t v = g < n ? ncomb[g] : 0;
        uint64_t tot;
        const int64_t ex = (int64_t)block_excl_scan<false>((uint64_t)v, warp, tot);
        if (g < n) out[g] = carry + ex;
        carry += (int64_t)tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_sum[gridDim.x];
}

__global__ void zero_i64(int64_t *p)
{
    if (threadIdx.x == 0) p[0] = 0;
}

__global__ void copy_seq(const uint32_t *src, uint32_t *dst)
{
    if (threadIdx.x == 0) *dst = *src;
}

}  // namespace

hipError_t prepare_fit()
{
    const int max_dyn = 256 * kCstBytesPerSector;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fit_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn);
}

hipError_t launch_fit(const FitArgs &a, int grid, size_t dyn_lds, hipStream_t stream,
                      hipEvent_t start, hipEvent_t stop)
{
    if (start != nullptr || stop != nullptr)
        hipExtLaunchKernelGGL(fit_kernel, dim3(grid), dim3(kBlock), (uint32_t)dyn_lds, stream, start,
                              stop, 0u, a);
    else
        hipLaunchKernelGGL(fit_kernel, dim3(grid), dim3(kBlock), dyn_lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_copy_seq(const uint32_t *src, uint32_t *dst, hipStream_t stream)
{
    hipLaunchKernelGGL(copy_seq, dim3(1), dim3(64), 0, stream, src, dst);
    return hipGetLastError();
}

size_t comb_offsets_scratch_bytes(int32_t n_roads)
{
    const int64_t tiles = ((int64_t)n_roads + kScanTile - 1) / kScanTile;
    return (size_t)(tiles + 1) * sizeof(int64_t);
}

hipError_t launch_comb_offsets(const int32_t *ncomb, int64_t *comb_offsets, int32_t n_roads,
                               int64_t *scratch, hipStream_t stream)
{
    const int32_t tiles = (int32_t)(((int64_t)n_roads + kScanTile - 1) / kScanTile);
    if (tiles == 0) {
        hipLaunchKernelGGL(zero_i64, dim3(1), dim3(64), 0, stream, comb_offsets);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(scan_tiles, dim3(tiles), dim3(kBlock), 0, stream, ncomb, n_roads, scratch);
    hipLaunchKernelGGL(scan_tile_sums, dim3(1), dim3(kBlock), 0, stream, scratch, tiles);
    hipLaunchKernelGGL(scan_apply, dim3(tiles), dim3(kBlock), 0, stream, ncomb, n_roads, scratch,
                       comb_offsets);
    return hipGetLastError();
}

}  // namespace svt
