// Unpack of a packed input word stream into the CSR batch (arXiv:1311.0380,
// Sec. 2.1: the first of the three stages fills the data structures from
// the input).  The word format is this library's own (include/svt.h): tagged
// 32-bit words -- event header, road header (sector, hit counts), XFT word,
// hit words of two hits.
//
// Every word's place in the batch follows from counts over the words before
// it, so the unpack is two data-parallel passes instead of a sequential
// parse:
//   tile_reduce  per tile of kTile words: event headers, road headers, hits
//                declared by road headers, last road header, last event
//                header (and a copy of the words into device memory when
//                they are read from host-mapped memory);
//   tile_apply   per tile, the same quantities before it (the block adds up
//                the earlier tiles' sums itself); per word, its event / road
//                / hit index from that plus a block scan, the checks that a
//                sequential parser would make at that word, and the writes.
//                The block of the last tile also checks the stream's end and
//                writes the totals and the final offsets.
// The first word that breaks the format is the smallest flagged word: up to
// it the stream is well formed, so every count there equals the parser's.
#include "svt_unpack.h"

namespace svt {
namespace {

#ifndef SVT_UNPACK_PER
#define SVT_UNPACK_PER 8
#endif
constexpr int kPer = SVT_UNPACK_PER;           // words per thread (16-byte loads of 4)
constexpr int kTile = kBlock * kPer;           // words per tile
constexpr uint32_t kNone = 0xFFFFFFFFu;

// sums and last positions (-1 if none) over a range of words
using Agg = UnpackAgg;

__device__ __forceinline__ uint32_t tag_of(uint32_t w) { return w >> 30; }
__device__ __forceinline__ uint32_t road_hits(uint32_t w)
{
    const uint32_t c = w & 0xFFFFFu;
    return (c & 31u) + ((c >> 5) & 31u) + ((c >> 10) & 31u) + ((c >> 15) & 31u);
}
// words of a road: header, XFT word, ceil(hits / 2) hit words
__device__ __forceinline__ int32_t road_len(uint32_t header) { return 2 + (int32_t)(road_hits(header) + 1) / 2; }

constexpr Agg kZero{0, 0, 0, -1, -1, 0u, 0u};

__device__ __forceinline__ Agg agg_word(uint32_t w, int32_t pos)
{
    const uint32_t t = tag_of(w);
    Agg a;
    a.ev = t == 3u;
    a.rd = t == 2u;
    a.hits = t == 2u ? road_hits(w) : 0;
    a.last_road = t == 2u ? pos : -1;
    a.last_ev = t == 3u ? pos : -1;
    a.last_hdr = t == 2u ? w : 0u;
    a.pad_ = 0u;
    return a;
}

// (positions are distinct, so the later road header's word goes with the
// larger position whichever side it is on)
__device__ __forceinline__ Agg agg_add(const Agg &x, const Agg &y)
{
    return Agg{x.hits + y.hits, x.ev + y.ev, x.rd + y.rd, max(x.last_road, y.last_road),
               max(x.last_ev, y.last_ev), y.last_road > x.last_road ? y.last_hdr : x.last_hdr, 0u};
}

// Cross-lane moves by DPP for a wavefront inclusive scan: row shifts by 1,
// 2, 4 and 8 within rows of 16 lanes, then the last lane of row 0 (2) into
// row 1 (3) and the last lane of row 1 into rows 2 and 3; and wave_shr:1
// (0x138), each lane's predecessor.  A lane with no source, or outside the
// move's rows, receives the identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ Agg dpp_move(const Agg &v)
{
    Agg o;
    const uint64_t h = (uint64_t)v.hits;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)h, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(h >> 32), CTRL, ROWS, 0xf, false);
    o.hits = (int64_t)((uint64_t)hi << 32 | lo);
    o.ev = __builtin_amdgcn_update_dpp(0, v.ev, CTRL, ROWS, 0xf, false);
    o.rd = __builtin_amdgcn_update_dpp(0, v.rd, CTRL, ROWS, 0xf, false);
    o.last_road = __builtin_amdgcn_update_dpp(-1, v.last_road, CTRL, ROWS, 0xf, false);
    o.last_ev = __builtin_amdgcn_update_dpp(-1, v.last_ev, CTRL, ROWS, 0xf, false);
    o.last_hdr = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v.last_hdr, CTRL, ROWS, 0xf, false);
    o.pad_ = 0u;
    return o;
}

__device__ __forceinline__ Agg wave_incl(Agg v)
{
    v = agg_add(dpp_move<0x111, 0xf>(v), v);   // row_shr:1
    v = agg_add(dpp_move<0x112, 0xf>(v), v);   // row_shr:2
    v = agg_add(dpp_move<0x114, 0xf>(v), v);   // row_shr:4
    v = agg_add(dpp_move<0x118, 0xf>(v), v);   // row_shr:8
    v = agg_add(dpp_move<0x142, 0xa>(v), v);   // row_bcast:15 into rows 1, 3
    v = agg_add(dpp_move<0x143, 0xc>(v), v);   // row_bcast:31 into rows 2, 3
    return v;
}

// the kPer words of a thread: 16-byte loads when aligned and whole
__device__ __forceinline__ void load_words(const uint32_t *src, int64_t base, int64_t n, bool vec,
                                           uint32_t (&w)[kPer])
{
    if (vec && base + kPer <= n) {
#pragma unroll
        for (int v = 0; v < kPer / 4; ++v) {
            const uint4 q = *reinterpret_cast<const uint4 *>(src + base + 4 * v);
            w[4 * v + 0] = q.x;
            w[4 * v + 1] = q.y;
            w[4 * v + 2] = q.z;
            w[4 * v + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i) w[i] = base + i < n ? src[base + i] : 0u;
    }
}
static_assert(kPer % 4 == 0, "16-byte loads");

// Exclusive scan of v (thread order) with the block total, and the block sum
// of u, in one round of LDS and barriers.
__device__ Agg block_excl_and_sum(const Agg &v, const Agg &u, Agg *s_w, Agg *s_u, Agg &total,
                                  Agg &usum)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const Agg incl = wave_incl(v);
    const Agg uincl = wave_incl(u);
    if (lane == 63) {
        s_w[wid] = incl;
        s_u[wid] = uincl;
    }
    __syncthreads();
    Agg before = kZero, tot = kZero, us = kZero;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) before = agg_add(before, s_w[w]);
        tot = agg_add(tot, s_w[w]);
        us = agg_add(us, s_u[w]);
    }
    __syncthreads();
    total = tot;
    usum = us;
    return agg_add(before, dpp_move<0x138, 0xf>(incl));
}

// Sum of one Agg per thread across the block (the wavefront scan's last
// lane, then the wavefront sums in LDS); the same in every thread.
__device__ Agg block_total(const Agg &v, Agg *s_w)
{
    const Agg incl = wave_incl(v);
    if ((threadIdx.x & 63) == 63) s_w[threadIdx.x >> 6] = incl;
    __syncthreads();
    Agg tot = kZero;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) tot = agg_add(tot, s_w[w]);
    return tot;
}

__global__ void __launch_bounds__(kBlock) tile_reduce(UnpackArgs a)
{
    __shared__ Agg s_w[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPer;
    uint32_t w[kPer];
    load_words(a.src, base, a.n_words, a.src_vec != 0, w);
    if (a.copy) {
        if (a.words_vec && base + kPer <= a.n_words) {
#pragma unroll
            for (int v = 0; v < kPer / 4; ++v)
                *reinterpret_cast<uint4 *>(a.words + base + 4 * v) =
                    make_uint4(w[4 * v], w[4 * v + 1], w[4 * v + 2], w[4 * v + 3]);
        } else {
#pragma unroll
            for (int i = 0; i < kPer; ++i)
                if (base + i < a.n_words) a.words[base + i] = w[i];
        }
    }
    Agg acc = kZero;
#pragma unroll
    for (int i = 0; i < kPer; ++i)
        if (base + i < a.n_words) acc = agg_add(acc, agg_word(w[i], (int32_t)(base + i)));
    const Agg tot = block_total(acc, s_w);
    if (threadIdx.x == 0) a.tiles[blockIdx.x] = tot;
}

// After the last tile (totals over the whole stream): the stream must end
// where its last road ends (or right after an event header that has no
// road); the final offsets and the totals (in the partial after the apply
// blocks').  One thread.
__device__ void finish_stream(const UnpackArgs &a, const Agg &tot)
{
    uint32_t bad = kNone;
    const int64_t W = a.n_words;
    if (W > 0) {
        const int64_t end = tot.last_road > tot.last_ev
                                ? (int64_t)tot.last_road + road_len(tot.last_hdr)
                                : (int64_t)tot.last_ev + 1;
        if (end != W) bad = (uint32_t)W;
    }
    if (tot.ev <= a.max_events) a.road_offsets[tot.ev] = (int32_t)tot.rd;
    if (tot.rd <= a.max_roads) a.hit_offsets[tot.rd] = (int32_t)tot.hits;
    a.partials[a.n_apply] = BlockPartial{(uint64_t)tot.rd, (uint64_t)tot.hits, (uint32_t)tot.ev, bad,
                                         kNone, a.seq};
}

// An empty stream: its totals and final offsets.
__global__ void __launch_bounds__(64) stream_empty(UnpackArgs a)
{
    if (threadIdx.x == 0) finish_stream(a, kZero);
}

__global__ void __launch_bounds__(kBlock) tile_apply(UnpackArgs a, int64_t n_tiles)
{
    __shared__ Agg s_w[kBlock / 64];
    __shared__ Agg s_u[kBlock / 64];
    __shared__ uint32_t s_bad[kBlock / 64];
    uint32_t bad = kNone;
    // the sums before a tile: the earlier tiles' sums, which the block adds
    // up itself (from its previous tile on)
    Agg carry = kZero;
    int64_t tdone = 0;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t base = tile * kTile + (int64_t)threadIdx.x * kPer;
    uint32_t w[kPer];
    load_words(a.words, base, a.n_words, a.words_vec != 0, w);
    Agg part = kZero;
    for (int64_t t = tdone + threadIdx.x; t < tile; t += kBlock) part = agg_add(part, a.tiles[t]);
    tdone = tile;
    Agg acc = kZero;
#pragma unroll
    for (int i = 0; i < kPer; ++i)
        if (base + i < a.n_words) acc = agg_add(acc, agg_word(w[i], (int32_t)(base + i)));
    Agg tot, psum;
    const Agg ex = block_excl_and_sum(acc, part, s_w, s_u, tot, psum);
    carry = agg_add(carry, psum);
    const Agg tile_pre = carry;
    Agg pre = agg_add(tile_pre, ex);
    if (tile == n_tiles - 1 && threadIdx.x == 0) finish_stream(a, agg_add(tile_pre, tot));
    // the header of the last road before the thread's words (the thread's
    // own road headers replace it as they come)
    uint32_t hdr = pre.last_hdr;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int64_t p = base + i;
        if (p >= a.n_words) break;
        const uint32_t v = w[i], t = tag_of(v);
        // pre holds the counts over the words before p
        const int32_t P = pre.last_road, Q = pre.last_ev;
        bool ok = true;
        if (t == 3u || t == 2u) {
            // a header: the previous road of this event ends here, or the
            // event header that opens it is the word before
            const int64_t expect = P > Q ? (int64_t)P + road_len(hdr) : (int64_t)Q + 1;
            ok = (p == 0 && t == 3u) || (Q >= 0 && p == expect);
        }
        if (t == 3u) {
            ok = ok && (v & 0x3FFFFFFFu) == 0u;
            if (pre.ev < a.max_events) a.road_offsets[pre.ev] = (int32_t)pre.rd;
        } else if (t == 2u) {
            const uint32_t c = v & 0xFFFFFu;
            ok = ok && (v & 0x300000u) == 0u && (c & 31u) <= 16u && ((c >> 5) & 31u) <= 16u &&
                 ((c >> 10) & 31u) <= 16u && ((c >> 15) & 31u) <= 16u;
            if (pre.rd < a.max_roads) {
                const int64_t r = pre.rd;
                a.sector[r] = (uint8_t)((v >> 22) & 255u);
                a.nhits4[r] = (c & 31u) | (((c >> 5) & 31u) << 8) | (((c >> 10) & 31u) << 16) |
                              (((c >> 15) & 31u) << 24);
                a.hit_offsets[r] = (int32_t)pre.hits;
            }
        } else {
            // XFT or hit word of the road whose header is at P
            ok = P > Q && (v & 0x3F000000u) == 0u;
            if (ok) {
                const int64_t r = pre.rd - 1;
                if (t == 1u) {
                    ok = p == P + 1;
                    if (ok && r < a.max_roads) a.xft2[r] = (v & 0xFFFu) | (((v >> 12) & 0xFFFu) << 16);
                } else {
                    const int64_t S = road_hits(hdr);
                    const int64_t j = 2 * (p - P - 2);
                    ok = p >= P + 2 && p < (int64_t)P + road_len(hdr) && (j + 1 < S || (v & 0xFFF000u) == 0u);
                    if (ok) {
                        const int64_t h = pre.hits - S + j;   // pre.hits counts this road's hits
                        if (h < a.max_hits) a.hits[h] = (int16_t)(v & 0xFFFu);
                        if (j + 1 < S && h + 1 < a.max_hits) a.hits[h + 1] = (int16_t)((v >> 12) & 0xFFFu);
                    }
                }
            }
        }
        if (!ok) bad = min(bad, (uint32_t)p);
        if (t == 2u) hdr = v;
        pre = agg_add(pre, agg_word(v, (int32_t)p));
    }
    }
    // lowest flagged word of the block -> host-mapped partials
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bad = min(bad, (uint32_t)__shfl_xor((int)bad, off, 64));
    if ((threadIdx.x & 63) == 0) s_bad[threadIdx.x >> 6] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = s_bad[0];
        for (int i = 1; i < kBlock / 64; ++i) b = min(b, s_bad[i]);
        a.partials[blockIdx.x] = BlockPartial{0, 0, 0, b, kNone, a.seq};
    }
}

}  // namespace

int64_t unpack_tiles(int64_t n_words) { return (n_words + kTile - 1) / kTile; }

size_t unpack_scratch_bytes(int64_t n_words) { return (size_t)(unpack_tiles(n_words) + 1) * sizeof(Agg); }

int64_t unpack_max_words() { return 0x7FFFFFFF; }   // word positions fit 31 bits

int32_t unpack_apply_blocks(int64_t n_words, int max_partials)
{
    const int64_t t = unpack_tiles(n_words);
    return (int32_t)(t < max_partials - 1 ? t : max_partials - 1);
}

hipError_t launch_unpack(UnpackArgs a, hipStream_t stream)
{
    const int64_t tiles = unpack_tiles(a.n_words);
    if (tiles > 0 && a.n_apply > 0) {
        hipLaunchKernelGGL(tile_reduce, dim3((unsigned)tiles), dim3(kBlock), 0, stream, a);
        hipLaunchKernelGGL(tile_apply, dim3((unsigned)a.n_apply), dim3(kBlock), 0, stream, a, tiles);
    } else {
        hipLaunchKernelGGL(stream_empty, dim3(1), dim3(64), 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace svt
