// Fused SVT fit kernel for gfx950 (arXiv:1311.0380, Sec. 2 / Sec. 2.1).
//
// Five 256-thread blocks per CU (96 VGPRs and no spills, 31 KB of LDS each;
// the sector constants are read from device memory through the caches).
// Values the compiler would hoist out of the chunk loop and hold (and spill
// at 96 VGPRs) are made where they are used: the thread's index through
// fresh_tid, the cut's limits, the chunk's event indices.  Work item = a
// chunk of `events_per_chunk` consecutive events, so every event (and its
// track count) belongs to exactly one block.  A chunk's roads are processed in
// sub-chunks of at most kSubRoads roads whose hits (kHitCap) and rows
// (kRowCap) fit in LDS:
//
//   A  one thread per road: load + validate the road, prefix sums give each
//      road its slot in the LDS hit table and row list.  The road's two
//      layers with the fewest hits index its rows (c, d) and the other two
//      (a, b) are looped over inside each row, which gives the fewest and
//      longest rows.  Rows are binned by (n_b, n_a), largest first, so that
//      a wavefront's rows share their inner trip counts; the hits are staged
//      in LDS (coalesced, flattened); the constraint rows' constant part
//      b + A[:,4] x4 + A[:,5] x5 is formed.
//   B  one thread per row (i_c, i_d): z = base + A[:,c] h_c + A[:,d] h_d,
//      then every (i_a, i_b) combination in the row loops of svt_rows.h.
//      The row's best is merged into the road with one LDS atomicMin on the
//      key chi2 << 16 | i0 << 12 | i1 << 8 | i2 << 4 | i3, whose order is
//      the order of (chi2, combination index k) because each i_l < n_l <= 16.
//   C  one thread per road: decode the winner, recompute its parameter rows
//      0..2 exactly in int32, write the road's results, count tracks per event.
//
// Each block writes its partial sums to the request's partials (host-mapped
// for a request, device memory reduced on the device for a ring); the host
// reads them when the request completes.
#include <hip/hip_ext.h>

#include "svt_internal.h"
#include "svt_rows.h"

namespace svt {
namespace {
// The thread's index through a value the compiler cannot see through, so
// that values derived from it are made where used, not hoisted and held.
__device__ __forceinline__ int fresh_tid()
{
    // the wavefront's index is uniform (a scalar register); the lane's
    // index is made anew, so no vector register holds the thread's index
    const int wid = (int)(__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6);
    int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    asm volatile("" : "+v"(lane));
    return wid * 64 + lane;
}

constexpr int kBins = 16 * 16;   // inner trip counts (n_a, n_b), each 1..16
constexpr int kWaves = kBlock / 64;
constexpr int kHitVecs = kHitCap / 8;            // 16-byte groups of the staged hit window
constexpr int kVecsPerThread = kHitVecs / kBlock;
static_assert(kMaxEventsPerChunk <= kBlock, "one thread per event of a chunk");
static_assert(kHitVecs % kBlock == 0, "the hit window is a whole number of 16-byte groups per thread");

// Inclusive scan across the wavefront of one 64-bit value.
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

// Block-wide exclusive scan of 64-bit values (the comb_offsets kernels).
__device__ uint64_t block_excl_scan64(uint64_t v, uint64_t *s_warp, uint64_t &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t incl = wave_incl_scan64(v);
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
    int32_t base[3][kSubRoads];             // b + A[:,4] x4 + A[:,5] x5, rows 3..5 (exact in int32)
    // per road, what its rows need (indices into the hit window and into
    // the constants image, in doubles):
    //   x  first hit of row layer c | of d << 16
    //   y  first hit of inner layer a | of b << 16
    //   z  column c of rows 3..5 | column d << 16
    //   w  column a | column b << 16
    uint4 ra[kSubRoads];
    uint32_t shape[kSubRoads];              // n_a | n_b << 5 | key place of a << 10 | of b << 14
    unsigned long long key[kSubRoads];      // best key of each road
    uint32_t np[kSubRoads];                 // passing combinations of each road
    uint32_t n4[kSubRoads];                 // hit counts of each road (0 if malformed)
    uint32_t info[kSubRoads];               // window position of its first hit | sector << 16
    uint32_t x2[kSubRoads];                 // the road's XFT words
    // rows, binned by (n_b, n_a): road | i_c << 8 | i_d << 12 | the row's key bits << 16
    uint32_t row[kRowCap];
    __align__(16) int16_t hit[kHitCap + 16];   // staged hit window (+ pad read by row loops)
    __align__(16) uint32_t bin[kBins];
    int32_t evro[kMaxEventsPerChunk + 1];   // event road offsets of the chunk
    uint32_t evcnt[kMaxEventsPerChunk];
    uint32_t wrows[kWaves];                 // rows of each wavefront's roads
    uint32_t wout[kWaves];                  // first lane of each wavefront outside the window
    uint32_t wfit[kWaves];                  // first lane of each wavefront that does not fit
    int32_t misc[4];                        // [2]: a staged word is out of range; [3]: rows
    uint32_t seq;                           // the request's sequence number
};

// LDS per block (Shared and write_partial's per-wavefront partials): five
// blocks (twenty wavefronts, the VGPR limit at 96) share a CU's 160 KB; LDS
// is allocated in 512-byte granules.
static_assert(((sizeof(Shared) + sizeof(BlockPartial) * kWaves + 511) / 512) * 512 * 5 <= 160 * 1024,
              "five blocks per CU");

// OR across the wavefront (all lanes active), as a uniform value.
__device__ __forceinline__ uint32_t wave_or(uint32_t x)
{
    x |= dpp<kRowShr + 1, 0xF, true>(x);
    x |= dpp<kRowShr + 2, 0xF, true>(x);
    x |= dpp<kRowShr + 4, 0xF, true>(x);
    x |= dpp<kRowShr + 8, 0xF, true>(x);
    x |= dpp<kRowBcast15, 0xA, false>(x);
    x |= dpp<kRowBcast31, 0xC, false>(x);
    return __builtin_amdgcn_readlane(x, 63);
}

// Small rows of different trip counts in one wavefront (N2 and N3 at least
// every lane's n2 and n3).  Indices past a lane's lists read the words that
// follow them (the window carries a pad); those combinations get an
// infinite index fraction, so they neither pass nor win, and the count
// needs no mask.  The minimum keeps i3 / 256 per combination and adds
// i2 / 16 once per i2.
template <int N2, int N3>
__device__ __forceinline__ void frac_small_masked(Row &st, const int16_t *hit, uint32_t p2, uint32_t p3,
                                                  uint32_t n2, uint32_t n3, double lim)
{
    double h2[N2], h3[N3], f3[N3];
#pragma unroll
    for (int i = 0; i < N2; ++i) h2[i] = (double)hit[p2 + i];
#pragma unroll
    for (int i = 0; i < N3; ++i) {
        h3[i] = (double)hit[p3 + i];
        f3[i] = (uint32_t)i < n3 ? i * (1.0 / 256) : __builtin_inf();
    }
#pragma unroll
    for (int i2 = 0; i2 < N2; ++i2) {
        if (i2 == 0 || (uint32_t)i2 < n2) {
            const double q3 = fma(st.a3, h2[i2], st.z3);
            const double q4 = fma(st.a4, h2[i2], st.z4);
            const double q5 = fma(st.a5, h2[i2], st.z5);
            double bi = __builtin_inf();
#pragma unroll
            for (int i3 = 0; i3 < N3; ++i3) {
                const double y3 = fma(st.c3, h3[i3], q3);
                const double y4 = fma(st.c4, h3[i3], q4);
                const double y5 = fma(st.c5, h3[i3], q5);
                const double v = fma(y5, y5, fma(y4, y4, fma(y3, y3, f3[i3])));
                count_le(st.np, v, lim);
                bi = dmin(bi, v);
            }
            st.best = dmin(st.best, i2 == 0 ? bi : bi + i2 * (1.0 / 16));
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The row loops of one wavefront: its rows are sorted by (n3, n2), largest
// first, so when every lane has the same n3 the first lane holds the largest
// n2; otherwise the largest of each comes from one OR of one-hot bits.
template <bool F>
__device__ __forceinline__ void run_rows(Row &st, const int16_t *hit, uint32_t p2, uint32_t p3,
                                         uint32_t rn2, uint32_t rn3, double lim)
{
    const uint32_t n3f = __builtin_amdgcn_readfirstlane(rn3);
    const uint32_t n3l = __builtin_amdgcn_readlane(rn3, 63);
    const bool uni = n3f == n3l;
    uint32_t n2m = __builtin_amdgcn_readfirstlane(rn2), n3m = n3f;
    if (!uni) {
        const uint32_t m = wave_or((1u << (rn2 - 1u)) | (1u << (rn3 + 15u)));
        n2m = 32u - (uint32_t)__builtin_clz((m & 0xFFFFu) | 1u);
        n3m = 32u - (uint32_t)__builtin_clz((m >> 16) | 1u);
    }
    if constexpr (F) {
        if (n2m <= 4 && n3m <= 4) {
            const uint32_t sel = ((n2m - 1) << 2) | (n3m - 1);
#define SVT_SMALL(N2, N3)                                                         \
    case ((N2 - 1) << 2) | (N3 - 1):                                              \
        if (uni) frac_small<N2, N3>(st, hit, p2, p3, rn2, lim);                   \
        else frac_small_masked<N2, N3>(st, hit, p2, p3, rn2, rn3, lim);           \
        return;
            switch (sel) {
                SVT_SMALL(1, 1) SVT_SMALL(1, 2) SVT_SMALL(1, 3) SVT_SMALL(1, 4)
                SVT_SMALL(2, 1) SVT_SMALL(2, 2) SVT_SMALL(2, 3) SVT_SMALL(2, 4)
                SVT_SMALL(3, 1) SVT_SMALL(3, 2) SVT_SMALL(3, 3) SVT_SMALL(3, 4)
                SVT_SMALL(4, 1) SVT_SMALL(4, 2) SVT_SMALL(4, 3) SVT_SMALL(4, 4)
            default: break;
            }
#undef SVT_SMALL
        }
    }
    if (uni) {
#define SVT_CASE(N)                                                          \
    case N:                                                                  \
        if constexpr (F) frac_uniform<N>(st, hit, p2, p3, rn2, n2m, lim);    \
        else gen_uniform<N>(st, hit, p2, p3, rn2, n2m, lim);                 \
        break;
        switch (n3f) {
            SVT_CASE(1) SVT_CASE(2) SVT_CASE(3) SVT_CASE(4) SVT_CASE(5) SVT_CASE(6)
            SVT_CASE(7) SVT_CASE(8) SVT_CASE(9) SVT_CASE(10) SVT_CASE(11) SVT_CASE(12)
            SVT_CASE(13) SVT_CASE(14) SVT_CASE(15) SVT_CASE(16)
        default: break;
        }
#undef SVT_CASE
    } else {
        if constexpr (F) frac_mixed(st, hit, p2, p3, rn2, rn3, n2m, n3m, lim);
        else gen_mixed(st, hit, p2, p3, rn2, rn3, n2m, n3m, lim);
    }
}

// The launch arguments through a pointer the compiler cannot see through, so
// that their loads are repeated where the fields are used rather than hoisted
// to the kernel's start and held (or spilled) in scalar registers throughout.
typedef const __attribute__((address_space(4))) FitArgs ConstArgs;
__device__ __forceinline__ const FitArgs &fresh_args(const FitArgs &a)
{
    // (the address is uniform; readfirstlane keeps it in scalar registers
    // wherever the compiler cannot tell)
    const uint64_t v = reinterpret_cast<uint64_t>((ConstArgs *)&a);
    uint64_t u = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v) |
                 ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32);
    asm volatile("" : "+s"(u));
    return *(const FitArgs *)reinterpret_cast<ConstArgs *>(u);
}

// Hit words a in [0, 4096): no bit of 15..12 set in either half of a word pair.
__device__ __forceinline__ bool words_ok(uint32_t pair) { return (pair & 0xF000F000u) == 0u; }

// One sub-chunk's inputs, loaded ahead of their use: the words of the road
// of each thread and the thread's share of the hit window.
struct SubIn {
    uint32_t sec, nh4, x2;
    int32_t h0, h1;
    uint4 hv[kVecsPerThread];
};

// The hit window of the sub-chunk that starts at road s of a chunk ending at
// road rb: from the first road's first hit, rounded down to a 16-byte
// boundary, to the end of the last road the sub-chunk can hold (at least the
// first road's end), at most kHitCap words.  A road inside the window finds
// its hits at their offset from the window's start.  window_loads issues the
// three offsets it needs, one per lane (lanes 0, 1 and 2 of the result), so
// that nothing waits for them before window_of reads them.
__device__ __forceinline__ int32_t window_loads(const FitArgs &a, int32_t s, int32_t rb)
{
    const int lane = fresh_tid() & 63;
    const int32_t s_end = min(rb, s + kSubRoads);
    return a.hit_offsets[lane == 1 ? s_end : (lane == 2 ? s + 1 : s)];
}

__device__ __forceinline__ void window_of(int32_t raw, int32_t n_hits, int32_t &hw, int32_t &W)
{
    const int32_t hs = clampi(__builtin_amdgcn_readlane(raw, 0), 0, n_hits);
    const int32_t he = max(__builtin_amdgcn_readlane(raw, 1), __builtin_amdgcn_readlane(raw, 2));
    hw = hs & ~7;
    W = min(clampi(he, hs, n_hits) - hw, kHitCap);
}

// The words of road s + tid (zeros past rb).
__device__ __forceinline__ void road_loads(const FitArgs &a, int32_t s, int32_t rb, SubIn &in)
{
    const int32_t r = s + (int32_t)fresh_tid();
    in.sec = 0;
    in.nh4 = 0;
    in.x2 = 0;
    in.h0 = 0;
    in.h1 = 0;
    if (r < rb) {
        in.sec = a.sector[r];
        in.nh4 = a.nhits4[r];
        in.h0 = a.hit_offsets[r];
        in.h1 = a.hit_offsets[r + 1];
        in.x2 = a.xft2[r];
    }
}

// The thread's 16-byte groups of the window [hw, hw + W) (zeros past it).
__device__ __forceinline__ void window_loads_hits(const FitArgs &a, int32_t hw, int32_t W, int32_t n_hits,
                                                  bool vec, SubIn &in)
{
    const int tid = fresh_tid();
#pragma unroll
    for (int q = 0; q < kVecsPerThread; ++q) {
        int32_t t = 8 * (tid + q * kBlock);
        // recomputed per sub-chunk: a per-lane address hoisted out of the
        // chunk loop would stay live across the row loops
        asm volatile("" : "+v"(t));
        in.hv[q] = make_uint4(0u, 0u, 0u, 0u);
        if (vec && t < W && hw + t + 8 <= n_hits) {
            // a whole 16-byte group of the array; in the window's last group
            // the words past the window are zeroed
            uint4 v = *reinterpret_cast<const uint4 *>(a.hits + hw + t);
            if (t + 8 > W) {
                const int32_t nv = W - t;
                auto keep = [nv](int d) {
                    return nv >= 2 * d + 2 ? 0xFFFFFFFFu : (nv == 2 * d + 1 ? 0xFFFFu : 0u);
                };
                v.x &= keep(0);
                v.y &= keep(1);
                v.z &= keep(2);
                v.w &= keep(3);
            }
            in.hv[q] = v;
        } else if (t < W) {
            // the array's last, partial group (or a hits array that is not
            // 16-byte aligned): word by word, all eight loads in flight at
            // once (indices clamped into the array, which holds at least the
            // window), zeros past the window
            uint32_t w[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) w[i] = (uint16_t)a.hits[min(hw + t + i, n_hits - 1)];
#pragma unroll
            for (int i = 0; i < 8; ++i) w[i] = t + i < W ? w[i] : 0u;
            in.hv[q] = make_uint4(w[0] | (w[1] << 16), w[2] | (w[3] << 16), w[4] | (w[5] << 16),
                                  w[6] | (w[7] << 16));
        }
    }
}

// Phase A of the sub-chunk of roads [s, rb) (one thread per road): validate
// the roads, order their layers, place their rows in the binned row list,
// stage the window and the per-road records in LDS.  Returns L, the roads
// that fit (a prefix of the sub-chunk, at least one when s < rb), and the
// sub-chunk's rows.
template <bool F>
__device__ __forceinline__ int sub_a(Shared &S, const double *cst, int32_t s, int32_t rb,
                                     int32_t n_roads, int32_t n_hits, int32_t n_sectors,
                                     const SubIn &in, int32_t hw, int32_t W, Acc &acc,
                                     int32_t &total_rows_out)
{
    const int tid = fresh_tid();
    const int lane = tid & 63, wid = tid >> 6;
    const int32_t r = s + tid;
    const bool inr = r < rb;
    const uint32_t sec = in.sec, nh4 = in.nh4, x2 = in.x2;
    const int32_t h0 = in.h0, h1 = in.h1;
    const uint32_t n0 = nh4 & 255u, n1 = (nh4 >> 8) & 255u, n2 = (nh4 >> 16) & 255u,
                   n3 = nh4 >> 24;
    const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
    const uint32_t sum = n0 + n1 + n2 + n3;
    bool ok = inr && sec < (uint32_t)n_sectors && n0 <= 16 && n1 <= 16 && n2 <= 16 && n3 <= 16;
    ok = ok && h0 >= 0 && h1 <= n_hits && (int64_t)h1 - (int64_t)h0 == (int64_t)sum;
    ok = ok && (r != 0 || h0 == 0) && (r != n_roads - 1 || h1 == n_hits);
    ok = ok && xa >= 0 && xa < 4096 && xb >= 0 && xb < 4096;
    acc.err_road = min(acc.err_road, wave_min(inr && !ok ? (uint32_t)r : 0xFFFFFFFFu));

    // row layers c < d: the two with the fewest hits (ties to the lower
    // layer); inner layers a < b: the other two.  Keys n << 2 | layer are
    // distinct, so a min / max network orders them.
    const uint32_t k0 = n0 << 2, k1 = (n1 << 2) | 1u, k2 = (n2 << 2) | 2u, k3 = (n3 << 2) | 3u;
    const uint32_t lo01 = min(k0, k1), hi01 = max(k0, k1), lo23 = min(k2, k3), hi23 = max(k2, k3);
    const uint32_t q1 = min(lo01, lo23), q4 = max(hi01, hi23);
    const uint32_t m1 = max(lo01, lo23), m2 = min(hi01, hi23);
    const uint32_t q2 = min(m1, m2), q3 = max(m1, m2);
    const bool rsw = (q1 & 3u) > (q2 & 3u), isw = (q3 & 3u) > (q4 & 3u);
    const uint32_t kc = rsw ? q2 : q1, kd = rsw ? q1 : q2, ka = isw ? q4 : q3, kb = isw ? q3 : q4;
    const uint32_t nh = ok ? sum : 0u;
    const uint32_t rows = (ok && (q1 >> 2) != 0u) ? (kc >> 2) * (kd >> 2) : 0u;
    const int32_t pos = h0 - hw;
    const bool in_window = nh == 0u || (pos >= 0 && pos + (int32_t)nh <= W);

    // rows before each road (the row list's capacity) and the first road
    // outside the window, per wavefront
    const uint32_t incl = wave_incl_scan(rows);
    const uint64_t out = __ballot(inr && !in_window);
    if (lane == 63) S.wrows[wid] = incl;
    if (lane == 0) S.wout[wid] = out ? (uint32_t)__ffsll((unsigned long long)out) - 1u : 64u;
    // stage the window (checking each word's range on the way)
    bool bad_word = false;
#pragma unroll
    for (int q = 0; q < kVecsPerThread; ++q) {
        const int32_t t = 8 * (tid + q * kBlock);
        if (t < W) {
            *reinterpret_cast<uint4 *>(&S.hit[t]) = in.hv[q];
            bad_word |= !words_ok(in.hv[q].x | in.hv[q].y | in.hv[q].z | in.hv[q].w);
        }
    }
    if (bad_word) S.misc[2] = 1;
    __syncthreads();
    uint32_t before = 0, total = 0, first_out = kBlock;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t t = S.wrows[w], o = S.wout[w];
        before += w < wid ? t : 0u;
        total += t;
        first_out = (first_out == (uint32_t)kBlock && o < 64u) ? (uint32_t)(w * 64) + o : first_out;
    }
    const uint32_t rbase = before + incl - rows;
    // the roads that fit (their hits inside the window, their rows inside
    // the row list) are a prefix [0, L) of the sub-chunk
    int L = min(kBlock, rb - s);
    if (total > (uint32_t)kRowCap || first_out < (uint32_t)kBlock) {
        const bool fit = inr && in_window && rbase + rows <= (uint32_t)kRowCap;
        const uint64_t m = __ballot(!fit);
        if (lane == 0) S.wfit[wid] = m ? (uint32_t)__ffsll((unsigned long long)m) - 1u : 64u;
        __syncthreads();
        L = kBlock;
#pragma unroll
        for (int w = kWaves - 1; w >= 0; --w) {
            const uint32_t f = S.wfit[w];
            L = f < 64u ? w * 64 + (int)f : L;
        }
    }
    const bool active = tid < L;
    if (tid == L - 1) S.misc[3] = (int32_t)(rbase + rows);    // rows of the sub-chunk

    const uint32_t lc = kc & 3u, ld = kd & 3u, la = ka & 3u, lb = kb & 3u;
    // bins in descending (n_b, n_a): the largest rows come first, and the
    // last, partial pass over the row list (which one wavefront runs while
    // the others wait at the barrier) takes the smallest
    const uint32_t bkey = 255u - (((kb >> 2) - 1u) * 16u + ((ka >> 2) - 1u));
    uint32_t boff = 0;
    if (active) {
        // window positions of each layer's first hit (layer-major lists)
        auto lpos = [&](uint32_t l) {
            return (uint32_t)pos + (((nh4 & ((1u << (8u * l)) - 1u)) * 0x01010101u) >> 24);
        };
        const uint32_t cb = (ok ? sec : 0u) * (uint32_t)kCstStride;
        S.ra[tid] = make_uint4(lpos(lc) | (lpos(ld) << 16), lpos(la) | (lpos(lb) << 16),
                               (cb + 3u * lc) | ((cb + 3u * ld) << 16),
                               (cb + 3u * la) | ((cb + 3u * lb) << 16));
        S.shape[tid] = (ka >> 2) | ((kb >> 2) << 5) | ((12u - 4u * la) << 10) | ((12u - 4u * lb) << 14);
        // (made here: a constant hoisted out of the chunk loop is spilled)
        uint32_t none = 0xFFFFFFFFu;
        asm volatile("" : "+v"(none));
        S.key[tid] = ((unsigned long long)none << 32) | none;
        S.np[tid] = 0;
        S.n4[tid] = ok ? nh4 : 0u;
        S.info[tid] = (uint32_t)pos | (sec << 16);
        S.x2[tid] = x2;
        if (rows) boff = atomicAdd(&S.bin[bkey], rows);
        if (ok) {
            // constant part of the constraint rows, exact in int32
            const double *cs = cst + sec * kCstStride;
            const int32_t *cbi = reinterpret_cast<const int32_t *>(cs) + kCstIntB;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                S.base[k][tid] =
                    (int32_t)fma(cs[15 + k], (double)xb, fma(cs[12 + k], (double)xa, (double)cbi[k]));
        }
    }
    __syncthreads();
    const int32_t total_rows = S.misc[3];
    if (S.misc[2]) {
        // a word out of range in the window: each road checks its own words
        bool bad = false;
        if (active && nh)
            for (uint32_t i = 0; i < nh; ++i) {
                const int16_t w = S.hit[pos + (int32_t)i];
                bad |= w < 0 || w >= 4096;
            }
        acc.err_road = min(acc.err_road, wave_min(bad ? (uint32_t)r : 0xFFFFFFFFu));
    }
    // bin starts: every wavefront scans the 256 bins itself (lane l holds
    // bins 4l .. 4l+3); all write the same starts, so a wavefront reading
    // after its own writes sees the right value whoever wrote last
    uint32_t bstart;
    {
        const uint4 vb = *reinterpret_cast<const uint4 *>(&S.bin[4 * lane]);
        const uint32_t loc = vb.x + vb.y + vb.z + vb.w;
        const uint32_t run = wave_incl_scan(loc) - loc;
        // the start of bin 4 l + i is lane l's run plus its first i counts
        const int o = (int)(bkey >> 2);
        const uint32_t i = bkey & 3u;
        const uint32_t r0 = (uint32_t)__shfl((int)run, o, 64), b0 = (uint32_t)__shfl((int)vb.x, o, 64),
                       b1 = (uint32_t)__shfl((int)vb.y, o, 64), b2 = (uint32_t)__shfl((int)vb.z, o, 64);
        bstart = r0 + (i > 0 ? b0 : 0u) + (i > 1 ? b1 : 0u) + (i > 2 ? b2 : 0u);
    }
    // the road's rows, in (i_c, i_d) order, at its place in the binned list;
    // each carries its key bits (i_c and i_d at their layers' places)
    // (the entry is tid + i_c A + i_d B with A, B the place values of i_c
    // and i_d; after each i_d it steps by B, and after the last i_d of an
    // i_c by A - (n_d - 1) B)
    if (active && rows) {
        const uint32_t nd = kd >> 2;
        const uint32_t B = (1u << 12) | (1u << (28u - 4u * ld));
        const uint32_t wrap = ((1u << 8) | (1u << (28u - 4u * lc))) - nd * B;
        uint32_t *dst = &S.row[bstart + boff];
        uint32_t e = (uint32_t)tid, left = nd;
        for (uint32_t k = 0; k < rows; ++k) {
            dst[k] = e;
            --left;
            e += left ? B : wrap + B;
            left = left ? left : nd;
        }
    }
    __syncthreads();
    S.bin[tid] = 0;   // ready for the next sub-chunk (kBins == kBlock)
    if (tid == 0) S.misc[2] = 0;
    total_rows_out = total_rows;
    return __builtin_amdgcn_readfirstlane(L);
}

// Phase B: every combination of every row (one thread per row).
template <bool F>
__device__ __forceinline__ void sub_b(Shared &S, const double *cst, int32_t total_rows, double cut)
{
    const int tid = fresh_tid();
    // (the cut through an opaque copy: limits made here, not held from the
    // kernel's start)
    asm volatile("" : "+v"(cut));
    const double lim = F ? cut + 0.5 : cut;
    for (int idx0 = 0; idx0 < total_rows; idx0 += kBlock) {
        if (idx0 + (tid & ~63) >= total_rows) continue;   // whole wavefront idle
        const int idx = idx0 + tid;
        const bool act = idx < total_rows;
        const uint32_t d = S.row[act ? idx : total_rows - 1];
        const uint32_t j = d & 255u, ic = (d >> 8) & 15u, id = (d >> 12) & 15u;
        const uint4 ra = S.ra[j];
        const uint32_t shp = S.shape[j];
        const double *cc = cst + (ra.z & 0xFFFFu), *cd = cst + (ra.z >> 16);
        const double *ca = cst + (ra.w & 0xFFFFu), *cb = cst + (ra.w >> 16);
        const double hc = (double)S.hit[(ra.x & 0xFFFFu) + ic], hd = (double)S.hit[(ra.x >> 16) + id];
        Row st;
        st.z3 = fma(cd[0], hd, fma(cc[0], hc, (double)S.base[0][j]));
        st.z4 = fma(cd[1], hd, fma(cc[1], hc, (double)S.base[1][j]));
        st.z5 = fma(cd[2], hd, fma(cc[2], hc, (double)S.base[2][j]));
        st.a3 = ca[0];
        st.a4 = ca[1];
        st.a5 = ca[2];
        st.c3 = cb[0];
        st.c4 = cb[1];
        st.c5 = cb[2];
        st.best = F ? __builtin_inf() : cut + 1.0;
        st.bidx = 0xFFFFFFFFu;
        st.np = 0;
        run_rows<F>(st, S.hit, ra.y & 0xFFFFu, ra.y >> 16, shp & 31u, (shp >> 5) & 31u, lim);
        if (act) {
            // the key places come back from LDS rather than staying live
            // across the row loops
            const uint32_t shp2 = S.shape[j];
            unsigned long long key;
            if (row_key<F>(st, cut, d >> 16, (shp2 >> 10) & 15u, (shp2 >> 14) & 15u, key))
                atomicMin(&S.key[j], key);
            if (st.np) atomicAdd(&S.np[j], st.np);
        }
    }
    __syncthreads();
}

// Phase C: the results of the sub-chunk's fitted roads [s, s + L) (one
// thread per road) and their tracks counted per event of the chunk (event
// road offsets evro, ne events).
__device__ __forceinline__ void sub_c(const FitArgs &a, Shared &S, const double *cst, int32_t s,
                                      int32_t L, int32_t ne, const int32_t *evro, Acc &acc)
{
    const int tid = fresh_tid();
    const int32_t r = s + tid;
    const bool active = tid < L;
    const uint32_t x2 = active ? S.x2[tid] : 0u;
    const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
    // Each road's counts, first hit and sector come back from LDS (zero
    // counts for a malformed road give the same outputs as the road's error
    // path), which keeps phase A's values out of phase B.
    uint32_t my_comb = 0, my_pass = 0, my_track = 0;
    if (active) {
        const uint32_t c4 = S.n4[tid];
        const uint32_t c0 = c4 & 255u, c1 = (c4 >> 8) & 255u, c2n = (c4 >> 16) & 255u,
                       c3 = c4 >> 24;
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
            bk = (int32_t)(((i0 * c1 + i1) * c2n + i2) * c3 + i3);
            hi4 = i0 | (i1 << 8) | (i2 << 16) | (i3 << 24);
            const uint32_t inf = S.info[tid];
            const int32_t hp = (int32_t)(inf & 0xFFFFu);
            const uint32_t x[6] = {(uint32_t)(int32_t)S.hit[hp + i0],
                                   (uint32_t)(int32_t)S.hit[hp + c0 + i1],
                                   (uint32_t)(int32_t)S.hit[hp + c0 + c1 + i2],
                                   (uint32_t)(int32_t)S.hit[hp + c0 + c1 + c2n + i3],
                                   (uint32_t)xa, (uint32_t)xb};
            // parameter rows 0..2, exact in int32 by the load-time bound
            const int32_t *ci = reinterpret_cast<const int32_t *>(cst + (inf >> 16) * kCstStride);
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
        __builtin_nontemporal_store((int32_t)(c0 * c1 * c2n * c3), &a.ncomb[r]);
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
                if (evro[mid] <= r) lo = mid; else hi = mid;
            }
            atomicAdd(&S.evcnt[lo], 1u);
        }
        my_comb = c0 * c1 * c2n * c3;
        my_pass = np;
        my_track = found ? 1u : 0u;
    }
    acc.comb += wave_sum(my_comb);      // each at most 64 * 2^16
    acc.pass += wave_sum(my_pass);
    acc.tracks += wave_sum(my_track);
    __syncthreads();
}

// Process the roads [s, rb) of the current chunk starting at road s; returns
// how many roads were fitted (at least one when s < rb).
template <bool F>
__device__ int process_sub(const FitArgs &a_in, Shared &S, const double *cst, int32_t s, int32_t rb,
                           int32_t n_roads, int32_t n_hits, int32_t n_sectors, int32_t ne,
                           double cut, bool vec, Acc &acc)
{
    const FitArgs &a = fresh_args(a_in);
    const int tid = fresh_tid();
    int32_t hw, W;
    const int32_t wraw = window_loads(a, s, rb);
    SubIn in;
    road_loads(a, s, rb, in);
    window_of(wraw, n_hits, hw, W);
    window_loads_hits(a, hw, W, n_hits, vec, in);
    int32_t total_rows;
    const int L = sub_a<F>(S, cst, s, rb, n_roads, n_hits, n_sectors, in, hw, W, acc, total_rows);
    sub_b<F>(S, cst, total_rows, cut);
    sub_c(a, S, cst, s, L, ne, S.evro, acc);
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
__device__ __forceinline__ void chunk_range(int32_t n_chunks, int32_t schedule, int32_t blk,
                                            int32_t nblk, int32_t &first, int32_t &step,
                                            int32_t &last)
{
    if (schedule == 2) {
        const int64_t g = nblk, b = blk;
        first = (int32_t)((int64_t)n_chunks * b / g);
        last = (int32_t)((int64_t)n_chunks * (b + 1) / g);
        step = 1;
    } else {
        first = blk;
        last = n_chunks;
        step = nblk;
    }
}

// The block's sums of one batch -> its partials[blk] in host-mapped memory
// (the host reduces them); the wavefront sums are uniform already.  Lane and
// wave ids are recomputed here rather than kept live across the whole kernel.
// Every thread calls it (one barrier).
__device__ __forceinline__ void write_partial(const FitArgs &a, int32_t blk, const Acc &acc,
                                              const uint32_t &seq)
{
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int wid = (int)(__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6);
    __shared__ BlockPartial s_part[kWaves];
    if (lane == 0)
        s_part[wid] = BlockPartial{acc.comb, acc.pass, acc.tracks, acc.err_road, acc.err_event, 0};
    __syncthreads();
    if (threadIdx.x == 0) {
        BlockPartial p = s_part[0];
        for (int w = 1; w < kWaves; ++w) {
            p.comb += s_part[w].comb;
            p.pass += s_part[w].pass;
            p.tracks += s_part[w].tracks;
            p.err_road = min(p.err_road, s_part[w].err_road);
            p.err_event = min(p.err_event, s_part[w].err_event);
        }
        p.seq = seq;
        a.partials[blk] = p;
    }
}

// One block's share of one batch: block blk of the nblk blocks the batch is
// spread over.
__device__ __forceinline__ void fit_block(const FitArgs &a_in, const int32_t blk, const int32_t nblk)
{
    const FitArgs &a = fresh_args(a_in);
    __shared__ __align__(16) Shared S;

    // sizes and sequence number: from the launch arguments, or read once per
    // block from the plan's host-mapped descriptor (all four words in one
    // load: reads of one host word by every block queue behind each other)
    // or the ring's device word
    int32_t n_events = a.n_events, n_roads = a.n_roads, n_hits = a.n_hits;
    uint32_t seq = a.seq;
    if (a.sizes != nullptr) {
        const uint4 sz = *reinterpret_cast<const uint4 *>(a.sizes);
        n_events = (int32_t)sz.x;
        n_roads = (int32_t)sz.y;
        n_hits = (int32_t)sz.z;
        seq = sz.w;
    } else if (a.seq_dev != nullptr) {
        seq = *a.seq_dev;
    }
    // kept in LDS until the block's sums are written (not in a register
    // across the whole kernel)
    if (fresh_tid() == 0) S.seq = seq;
    const int32_t n_sectors = a.n_sectors;
    // the sector constants, read through the caches (device memory)
    typedef const __attribute__((address_space(1))) double GlobalDouble;
    const double *cst = (const double *)(GlobalDouble *)a.cst_block;

    Acc acc;
    const double cut = a.cut_d;
    const int32_t E = a.events_per_chunk;

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
        const int64_t G = nblk, b = blk;
        uint32_t bad_event = 0xFFFFFFFFu;
        if (wid < 2) {
            const int64_t bb = b + wid;
            const int32_t e = bb >= G ? n_events
                                      : first_event_at(a.road_offsets, n_events, (int64_t)n_roads * bb / G);
            if (fresh_tid() == wid * 64) S.misc[wid] = e;
        } else {
            const int t2 = fresh_tid() - 128;
            const int32_t per = (int32_t)((n_events + G - 1) / G);
            for (int32_t e = (int32_t)(b * per) + t2; e < min((int64_t)n_events, (b + 1) * per); e += 128) {
                const int32_t lo = a.road_offsets[e], hi = a.road_offsets[e + 1];
                const bool bad = lo < 0 || hi < lo || hi > n_roads || (e == 0 && lo != 0) ||
                                 (e == n_events - 1 && hi != n_roads);
                if (bad) bad_event = min(bad_event, (uint32_t)e);
            }
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
        chunk_range(n_chunks, a.schedule, blk, nblk, c_first, c_step, c_last);
    }

    // the first chunk's event boundaries
    int32_t ev0 = 0, ev1 = 0;
    if (c_first < c_last) {
        const int32_t e0 = e_base + c_first * E, ne = min(E, e_end - e0);
        const int tid = fresh_tid();
        if (tid <= ne) ev0 = a.road_offsets[e0 + tid];
        if (tid + kBlock <= ne) ev1 = a.road_offsets[e0 + tid + kBlock];
    }

    static_assert(kBins == kBlock, "one bin per thread");
    S.bin[fresh_tid()] = 0;
    if (fresh_tid() == 0) S.misc[2] = 0;
    // 16-byte hit loads need a 16-byte aligned hits array
    const bool vec = (reinterpret_cast<uintptr_t>(a.hits) & 15u) == 0u;

    if (c_first < c_last) {
        const int32_t ne = min(E, e_end - (e_base + c_first * E));
        const int tid = fresh_tid();
        if (tid <= ne) S.evro[tid] = ev0;
        if (tid + kBlock <= ne) S.evro[tid + kBlock] = ev1;
    }
    for (int32_t c = c_first; c < c_last; c += c_step) {
        const int32_t e0 = e_base + c * E;
        const int32_t ne = min(E, e_end - e0);
        if (c != c_first) {
            // (an index made here: one carried from chunk to chunk is spilled)
            const int it = fresh_tid();
            for (int i = it; i <= ne; i += kBlock) S.evro[i] = a.road_offsets[e0 + i];
        }
        if (fresh_tid() < ne) S.evcnt[fresh_tid()] = 0;   // ne <= kMaxEventsPerChunk = kBlock
        __syncthreads();
        const int32_t ra = clampi(S.evro[0], 0, n_roads);
        const int32_t rb = clampi(S.evro[ne], ra, n_roads);
        for (int32_t s = ra; s < rb;)
            s += a.frac_key ? process_sub<true>(a, S, cst, s, rb, n_roads, n_hits, n_sectors, ne, cut, vec, acc)
                            : process_sub<false>(a, S, cst, s, rb, n_roads, n_hits, n_sectors, ne, cut, vec, acc);
        uint32_t bad_event = 0xFFFFFFFFu;
        // (the thread's first event made here, not held across the sub-chunks)
        const int i0 = fresh_tid();
        for (int i = i0; i < ne; i += kBlock) {
            const int32_t e = e0 + i, lo = S.evro[i], hi = S.evro[i + 1];
            const bool bad = lo < 0 || hi < lo || hi > n_roads || (e == 0 && lo != 0) ||
                             (e == n_events - 1 && hi != n_roads);
            if (bad) bad_event = min(bad_event, (uint32_t)e);
            a.ntracks[e] = (int32_t)S.evcnt[i];
        }
        acc.err_event = min(acc.err_event, wave_min(bad_event));
        __syncthreads();
    }

    write_partial(a, blk, acc, S.seq);
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5)))
fit_kernel(FitArgs a)
{
    // the argument is read in place, in the kernel argument segment (where
    // it is the first argument): its address must not escape, or it would be
    // copied to private memory
    (void)a;
    ConstArgs *pa = (ConstArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    fit_block(*(const FitArgs *)pa, (int32_t)blockIdx.x, (int32_t)gridDim.x);
}

// Several batches in one launch, so that blocks of later batches start
// wherever blocks of earlier ones end: batch i < n1 takes blocks
// [i per, (i + 1) per); the batches after them take per2 blocks each (the
// launch's last batches, which can be cut into smaller chunks than the
// others, so that the launch's last blocks are short ones).
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5)))
fit_kernel_multi(const FitArgs *__restrict__ args, int32_t per, int32_t n1, int32_t per2)
{
    const int32_t b = (int32_t)blockIdx.x, head = n1 * per;
    int32_t i, lb, nb;
    if (b < head) {
        i = b / per;
        lb = b - i * per;
        nb = per;
    } else {
        const int32_t t = (b - head) / per2;
        i = n1 + t;
        lb = b - head - t * per2;
        nb = per2;
    }
    // read through the constant address space: the argument loads can then be
    // repeated where they are used instead of holding every field in registers
    ConstArgs *ca = (ConstArgs *)args;
    fit_block(*(const FitArgs *)&ca[i], lb, nb);
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
        const int64_t ex = (int64_t)block_excl_scan64((uint64_t)v, warp, tot);
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
        const int64_t ex = (int64_t)block_excl_scan64((uint64_t)v, warp, tot);
        if (g < n) out[g] = carry + ex;
        carry += (int64_t)tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_sum[gridDim.x];
}

__global__ void zero_i64(int64_t *p)
{
    if (threadIdx.x == 0) p[0] = 0;
}

}  // namespace

hipError_t launch_fit_multi(const FitArgs *args, int n1, int per, int n2, int per2, hipStream_t stream)
{
    hipLaunchKernelGGL(fit_kernel_multi, dim3(n1 * per + n2 * per2), dim3(kBlock), 0, stream, args,
                       (int32_t)per, (int32_t)n1, (int32_t)(per2 > 0 ? per2 : 1));
    return hipGetLastError();
}

hipError_t launch_fit(const FitArgs &a, int grid, hipStream_t stream, hipEvent_t start, hipEvent_t stop)
{
    if (start != nullptr || stop != nullptr)
        hipExtLaunchKernelGGL(fit_kernel, dim3(grid), dim3(kBlock), 0u, stream, start, stop, 0u, a);
    else
        hipLaunchKernelGGL(fit_kernel, dim3(grid), dim3(kBlock), 0, stream, a);
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
