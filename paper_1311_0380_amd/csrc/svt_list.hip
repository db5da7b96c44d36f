// Every passing combination of a batch (arXiv:1311.0380, Sec. 2: the fit
// runs on every combination of one hit per layer; this kernel keeps each one
// within the chi2 cut, with its fit rows, instead of only the best of its
// road).
//
// Two kernels on the request's stream:
// - list_tile_sums: npass summed over tiles of kListTile roads;
// - list_kernel: a block takes a tile of 256 roads at a time (the running
//   sum of npass before it is the tile sums before it, which the block adds
//   up itself), in sub-chunks whose hits and row pieces fit in LDS, one
//   thread per road in phase A and one per row piece in phase B, as the fit
//   kernel does:
//   A  each road is loaded and validated as the fit does; its list offset is
//      the running sum before the tile plus the npass of the tile's earlier
//      roads, and is written out (and the list's length after the last
//      road).  A road to evaluate (valid, npass > 0) is cut into row pieces:
//      (i0, i1) and a run of at most 32 / n3 values of i2, so that a piece
//      has at most 32 combinations.  The pieces get places in road order
//      (their combinations then come in combination order) and in a list
//      binned by (n3, piece length), largest first, which gives the lanes of
//      a wavefront the same trip counts and leaves the smallest pieces to the
//      last, partial pass over the list; the sub-chunk's hits are staged in
//      LDS.
//   B  one lane per piece (two pieces per thread at a time, so that their
//      loads overlap): its combinations' constraint rows and chi2 in fp64,
//      exact as in the fit (every value is an integer below 2^53 whenever
//      chi2 <= cut < 2^48), and a 32-bit mask of the passing ones in
//      combination order, stored at the piece's place in road order.
//   S  the masks' counts are scanned in road order: a piece's passing
//      combinations come after those of every piece before it, so entry e of
//      the sub-chunk is a piece (a binary search over the scan) and a bit of
//      its mask (a select over popcounts); each road's count is checked
//      against its npass.
//   W  thread t writes entries t, t + 256, ... (four at a time): the
//      combination index, chi2 and fit rows 0..2, exact in integers;
//      consecutive entries go to consecutive places in the list.
// A road whose count of passing combinations differs from its npass, or
// whose npass is negative, is reported as a bad road; its entries past its
// npass are not written.
#include "svt_list.h"
#include "svt_rows.h"
#include <stddef.h>

namespace svt {
namespace {

constexpr int kWaves = kBlock / 64;

// A 64-bit value from another lane by DPP: CTRL is row_shr:n (0x110 + n),
// row_bcast:15 (0x142) or row_bcast:31 (0x143); lanes with no source, or
// outside the rows in ROWS, receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ int64_t dpp64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, false);
    return (int64_t)((uint64_t)hi << 32 | lo);
}

// Inclusive running sum across the wavefront (all lanes active), by DPP.
__device__ __forceinline__ int64_t wave_incl64(int64_t v)
{
    v += dpp64<0x111, 0xf>(v);
    v += dpp64<0x112, 0xf>(v);
    v += dpp64<0x114, 0xf>(v);
    v += dpp64<0x118, 0xf>(v);
    v += dpp64<0x142, 0xa>(v);
    v += dpp64<0x143, 0xc>(v);
    return v;
}

// Sum across the wavefront (all lanes active), as a uniform value.
__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
    const uint64_t u = (uint64_t)wave_incl64(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return (int64_t)((uint64_t)hi << 32 | lo);
}

__global__ void __launch_bounds__(kBlock) list_tile_sums(const int32_t *npass, int32_t n, int64_t *tsum)
{
    __shared__ int64_t s_w[kWaves];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t * kListTile < n; t += gridDim.x) {
        int64_t v = 0;
        for (int i = threadIdx.x; i < kListTile; i += kBlock) {
            const int64_t r = t * kListTile + i;
            if (r < n) v += npass[r];
        }
        v = wave_sum64(v);
        if (lane == 0) s_w[wid] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t s = 0;
            for (int w = 0; w < kWaves; ++w) s += s_w[w];
            tsum[t] = s;
        }
        __syncthreads();
    }
}

// Row pieces and staged hits of one sub-chunk.
constexpr int kLHitCap = 4096;                     // hits staged per sub-chunk
constexpr int kLPieceCap = 2048;                   // row pieces per sub-chunk (>= one road's)
constexpr int kLHitVecs = kLHitCap / 8 / kBlock;   // 16-byte hit groups per thread
constexpr int kLBins = 256;                        // (n3 - 1) * 16 + (piece length - 1)
static_assert(kLPieceCap == 8 * kBlock, "eight places per thread in the scan");
static_assert(kLBins == kBlock, "one bin per thread");

struct ListShared {
    __align__(16) int16_t hit[kLHitCap];
    uint32_t row[kLPieceCap];      // binned: j | i0 << 8 | i1 << 12 | i2s << 16 | place << 20
    uint32_t pinfo[kLPieceCap];    // at its place: j | i0 << 8 | i1 << 12 | i2s << 16
    uint32_t mask[kLPieceCap];     // passing combinations of the piece, in combination order
    uint32_t excl[kLPieceCap + 1]; // counts of the masks, then their running sum
    int64_t o0[kBlock];            // list offset of each road
    uint32_t rfirst[kBlock + 1];   // first place of each road's pieces
    int32_t np[kBlock];
    uint32_t n4[kBlock];           // hit counts (zero for a road not evaluated)
    uint32_t info[kBlock];         // window position of its first hit | sector << 16 | i2 run << 24
    uint32_t x2[kBlock];
    int32_t base[3][kBlock];       // constraint rows 3..5 at zero hits (offset and XFT columns)
    __align__(16) uint32_t bin[kLBins];   // read four at a time
    uint32_t w[4][kBlock / 64];    // per-wavefront sums of the scans
    int64_t wt[kBlock / 64];       // per-wavefront sums of tile sums
};

static_assert(offsetof(ListShared, bin) % 16 == 0 && offsetof(ListShared, hit) % 16 == 0,
              "16-byte LDS accesses");

// The first lane where p holds (64 if none); every lane must be active.
__device__ __forceinline__ int32_t wave_first(bool p)
{
    const uint64_t m = __ballot(p);
    return m ? __ffsll((unsigned long long)m) - 1 : 64;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
    return ~wave_min(~x);
}

// Position of the n-th set bit (from 0) of m, which has more than n set bits.
__device__ __forceinline__ uint32_t select_bit(uint32_t m, uint32_t n)
{
    uint32_t b = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const uint32_t low = m & ((1u << w) - 1u);
        const uint32_t c = (uint32_t)__popc(low);
        const bool up = n >= c;
        n = up ? n - c : n;
        m = up ? m >> w : low;
        b += up ? (uint32_t)w : 0u;
    }
    return b;
}

// One row piece of phase B: its place, the rows at its (i0, i1), the columns
// of inner layers 2 and 3, and where its hits lie in LDS.
struct Piece {
    double z[3], av[3], cv[3];
    const int16_t *h2, *h3;
    uint32_t place, p, n3;
    bool act;
};

__device__ __forceinline__ Piece piece_setup(const ListShared &S, const double *cst, int idx, int P)
{
    Piece q;
    q.act = idx < P;
    const uint32_t e = S.row[q.act ? idx : P - 1];
    const uint32_t j = e & 255u, i0 = (e >> 8) & 15u, i1 = (e >> 12) & 15u, i2s = (e >> 16) & 15u;
    q.place = e >> 20;
    const uint32_t c4 = S.n4[j], inf = S.info[j];
    const uint32_t m0 = c4 & 255u, m1 = (c4 >> 8) & 255u, m2 = (c4 >> 16) & 255u;
    q.n3 = c4 >> 24;
    q.p = min(inf >> 24, m2 - i2s);   // this piece's run of i2
    const int16_t *hh = S.hit + (inf & 0xFFFFu);
    const double *c = cst + ((inf >> 16) & 255u) * kCstStride;
    const double x0 = (double)hh[i0], x1 = (double)hh[m0 + i1];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        q.z[k] = fma(c[3 + k], x1, fma(c[k], x0, (double)S.base[k][j]));
        q.av[k] = c[6 + k];
        q.cv[k] = c[9 + k];
    }
    q.h2 = hh + m0 + m1 + i2s;
    q.h3 = hh + m0 + m1 + m2;
    return q;
}

// The piece's passing combinations as a mask in combination order, and its
// count, at its place.  Every lane of the wavefront takes part.
__device__ __forceinline__ void piece_mask(ListShared &S, const Piece &q, double cut)
{
    const uint32_t pm = wave_max(q.act ? q.p : 0u), n3m = wave_max(q.act ? q.n3 : 0u);
    uint32_t m = 0;
    for (uint32_t i2 = 0; i2 < pm; ++i2) {
        const double x2v = (double)q.h2[min(i2, q.p - 1u)];
        const double q3 = fma(q.av[0], x2v, q.z[0]);
        const double q4 = fma(q.av[1], x2v, q.z[1]);
        const double q5 = fma(q.av[2], x2v, q.z[2]);
        const uint32_t rowbit = i2 * q.n3;
        for (uint32_t i3 = 0; i3 < n3m; ++i3) {
            const double x3v = (double)q.h3[min(i3, q.n3 - 1u)];
            const double y3 = fma(q.cv[0], x3v, q3);
            const double y4 = fma(q.cv[1], x3v, q4);
            const double y5 = fma(q.cv[2], x3v, q5);
            const double v = fma(y5, y5, fma(y4, y4, y3 * y3));
            const bool in = v <= cut && i2 < q.p && i3 < q.n3;
            m |= in ? 1u << ((rowbit + i3) & 31u) : 0u;
        }
    }
    if (q.act) {
        S.mask[q.place] = m;
        S.excl[q.place] = (uint32_t)__popc(m);
    }
}

__global__ void __launch_bounds__(kBlock) list_kernel(ListArgs a)
{
    __shared__ __align__(16) ListShared S;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = (int)(__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6);
    const double *cst = a.cst;
    const double cut = (double)a.cut;   // exact: below 2^48
    uint64_t comb = 0, pass = 0;
    uint32_t err_road = 0xFFFFFFFFu;
    // 16-byte hit loads need a 16-byte aligned hits array
    const bool vec = (reinterpret_cast<uintptr_t>(a.hits) & 15u) == 0u;

    S.bin[tid] = 0;
    if (a.n_roads == 0 && blockIdx.x == 0 && tid == 0) a.offsets[0] = 0;
    // the running sum of npass before a tile: the tile sums before it, which
    // the block adds up itself (from its previous tile on)
    int64_t carry = 0, tdone = 0;
    for (int64_t tile = blockIdx.x; tile * kListTile < a.n_roads; tile += gridDim.x) {
        const int32_t t0 = (int32_t)(tile * kListTile);
        const int32_t rb = (int32_t)min((int64_t)a.n_roads, tile * kListTile + kListTile);
        int64_t tp = 0;
        for (int64_t t = tdone + tid; t < tile; t += kBlock) tp += a.tile_sum[t];
        tdone = tile;
        int64_t obase = carry;   // the tile sums are added at the first sub-chunk
        bool first = true;
        for (int32_t s = t0; s < rb;) {
            // ---- A: roads, window, pieces ----
            const int32_t r = s + tid;
            const bool inr = r < rb;
            int32_t np = 0, h0 = 0, h1 = 0;
            uint32_t sec = 0, nh4 = 0, x2 = 0;
            if (inr) {
                np = a.npass[r];
                sec = a.sector[r];
                nh4 = a.nhits4[r];
                h0 = a.hit_offsets[r];
                h1 = a.hit_offsets[r + 1];
                x2 = a.xft2[r];
            }
            // the window: from road s's first hit to the end of the last road
            // the sub-chunk can hold (at least road s's own end, so that road
            // s always fits), rounded down to a 16-byte boundary
            const int32_t hs = clampi(a.hit_offsets[s], 0, a.n_hits);
            const int32_t he = clampi(max(a.hit_offsets[rb], a.hit_offsets[s + 1]), hs, a.n_hits);
            const int32_t hw = hs & ~7;
            const int32_t W = min(he - hw, kLHitCap);
            uint4 hv[kLHitVecs];
#pragma unroll
            for (int q = 0; q < kLHitVecs; ++q) {
                const int32_t t = 8 * (tid + q * kBlock);
                hv[q] = make_uint4(0u, 0u, 0u, 0u);
                if (t < W) {
                    if (vec && hw + t + 8 <= a.n_hits) {
                        hv[q] = *reinterpret_cast<const uint4 *>(a.hits + hw + t);
                    } else {
                        uint32_t u[4];
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            const int32_t i = hw + t + 2 * d;
                            const uint32_t lo = i < a.n_hits ? (uint16_t)a.hits[i] : 0u;
                            const uint32_t hi = i + 1 < a.n_hits ? (uint16_t)a.hits[i + 1] : 0u;
                            u[d] = lo | hi << 16;
                        }
                        hv[q] = make_uint4(u[0], u[1], u[2], u[3]);
                    }
                }
            }

            const uint32_t n0 = nh4 & 255u, n1 = (nh4 >> 8) & 255u, n2 = (nh4 >> 16) & 255u,
                           n3 = nh4 >> 24;
            const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
            bool ok = inr && sec < (uint32_t)a.n_sectors && n0 <= 16 && n1 <= 16 && n2 <= 16 && n3 <= 16;
            ok = ok && h0 >= 0 && h1 <= a.n_hits && (int64_t)h1 - h0 == (int64_t)(n0 + n1 + n2 + n3);
            ok = ok && xa >= 0 && xa < 4096 && xb >= 0 && xb < 4096;
            const bool walk = ok && np > 0;
            // pieces: (i0, i1) x runs of at most P2 = 32 / n3 values of i2
            const uint32_t P2 = n3 > 0 ? max(1u, 32u / n3) : 32u;
            const uint32_t npc = (n2 + P2 - 1u) / P2;
            const uint32_t pieces = walk ? n0 * n1 * npc : 0u;
            const int32_t pos = h0 - hw;
            const bool in_window = !walk || (pos >= 0 && pos + (h1 - h0) <= W);

            // running sums over the sub-chunk's roads: pieces and npass; the
            // tile sums before the tile
            const int64_t tpw = wave_sum64(first ? tp : 0);
            if (lane == 0) S.wt[wid] = tpw;
            const uint32_t pincl = wave_incl_scan(pieces);
            const uint64_t nincl = (uint64_t)wave_incl64((int64_t)np);
            if (lane == 63) {
                S.w[0][wid] = pincl;
                S.w[1][wid] = (uint32_t)nincl;
                S.w[2][wid] = (uint32_t)(nincl >> 32);
            }
            // (ballots with every lane active, then one lane writes)
            const uint32_t out_w = (uint32_t)wave_first(inr && !in_window);
            if (lane == 0) S.w[3][wid] = out_w;
#pragma unroll
            for (int q = 0; q < kLHitVecs; ++q) {
                const int32_t t = 8 * (tid + q * kBlock);
                if (t < W) *reinterpret_cast<uint4 *>(&S.hit[t]) = hv[q];
            }
            __syncthreads();
            uint32_t pbefore = 0, ptotal = 0, first_out = kBlock;
            uint64_t nbefore = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) obase += S.wt[w];
            if (first) carry = obase;
            first = false;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) {
                const uint32_t pw = S.w[0][w];
                const uint64_t nw = (uint64_t)S.w[1][w] | (uint64_t)S.w[2][w] << 32;
                pbefore += w < wid ? pw : 0u;
                nbefore += w < wid ? nw : 0u;
                ptotal += pw;
                const uint32_t o = S.w[3][w];
                first_out = (first_out == (uint32_t)kBlock && o < 64u) ? (uint32_t)(w * 64) + o : first_out;
            }
            const uint32_t rfirst = pbefore + pincl - pieces;
            const int64_t o0 = obase + (int64_t)(nbefore + nincl) - np;
            // the roads that fit (hits inside the window, pieces inside the
            // list) are a prefix [0, L) of the sub-chunk; road s always fits
            int L = min(kBlock, rb - s);
            if (ptotal > (uint32_t)kLPieceCap || first_out < (uint32_t)kBlock) {
                __syncthreads();
                const bool fit = inr && in_window && rfirst + pieces <= (uint32_t)kLPieceCap;
                const uint32_t nofit_w = (uint32_t)wave_first(!fit);
                if (lane == 0) S.w[3][wid] = nofit_w;
                __syncthreads();
                L = kBlock;
#pragma unroll
                for (int w = kBlock / 64 - 1; w >= 0; --w) {
                    const uint32_t f = S.w[3][w];
                    L = f < 64u ? w * 64 + (int)f : L;
                }
            }
            const bool active = tid < L;
            if (active) {
                a.offsets[r] = o0;
                if (!ok || np < 0) err_road = min(err_road, (uint32_t)r);
                if (walk) comb += (uint64_t)n0 * n1 * n2 * n3;
                S.o0[tid] = o0;
                S.np[tid] = np;
                S.rfirst[tid] = rfirst;
                S.n4[tid] = walk ? nh4 : 0u;
                S.info[tid] = ((uint32_t)pos & 0xFFFFu) | (sec << 16) | (min(P2, 16u) << 24);
                S.x2[tid] = x2;
                if (tid == L - 1) S.rfirst[L] = rfirst + pieces;
            }
            uint32_t boff_full = 0, boff_last = 0;
            const uint32_t plast = n2 - (npc - 1u) * P2;   // length of the last run of i2
            // bin keys in descending (n3, run length): the largest pieces first
            const uint32_t kfull = 255u - ((n3 - 1u) * 16u + (min(P2, n2) - 1u));
            const uint32_t klast = 255u - ((n3 - 1u) * 16u + (plast - 1u));
            const bool split = plast != min(P2, n2);        // the last run is shorter
            if (active && pieces) {
                // (a road with pieces has hit counts in 1..16: both keys < 256)
                const uint32_t nfull = n0 * n1 * (split ? npc - 1u : npc);
                if (nfull) boff_full = atomicAdd(&S.bin[kfull & 255u], nfull);
                if (split) boff_last = atomicAdd(&S.bin[klast & 255u], n0 * n1);
                // constraint rows 3..5 at zero hits, exact in int32
                const double *cs = cst + sec * kCstStride;
                const int32_t *cbi = reinterpret_cast<const int32_t *>(cs) + kCstIntB;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    S.base[k][tid] =
                        (int32_t)fma(cs[15 + k], (double)xb, fma(cs[12 + k], (double)xa, (double)cbi[k]));
            }
            __syncthreads();
            const uint32_t P = S.rfirst[L];
            // bin starts (lane l of every wavefront scans bins 4l .. 4l + 3)
            uint32_t bs_full = 0, bs_last = 0;
            {
                const uint4 vb = *reinterpret_cast<const uint4 *>(&S.bin[4 * lane]);
                const uint32_t loc = vb.x + vb.y + vb.z + vb.w;
                const uint32_t run = wave_incl_scan(loc) - loc;
                auto start = [&](uint32_t key) {
                    const int o = (int)(key >> 2);
                    const uint32_t i = key & 3u;
                    const uint32_t r0 = (uint32_t)__shfl((int)run, o, 64);
                    const uint32_t b0 = (uint32_t)__shfl((int)vb.x, o, 64);
                    const uint32_t b1 = (uint32_t)__shfl((int)vb.y, o, 64);
                    const uint32_t b2 = (uint32_t)__shfl((int)vb.z, o, 64);
                    return r0 + (i > 0 ? b0 : 0u) + (i > 1 ? b1 : 0u) + (i > 2 ? b2 : 0u);
                };
                bs_full = start(kfull & 255u);
                bs_last = start(klast & 255u);
            }
            // the road's pieces, at their places (road order) and in the bins
            if (active && pieces) {
                uint32_t place = rfirst, f = bs_full + boff_full, l = bs_last + boff_last;
                for (uint32_t i0 = 0; i0 < n0; ++i0)
                    for (uint32_t i1 = 0; i1 < n1; ++i1)
                        for (uint32_t pc = 0; pc < npc; ++pc, ++place) {
                            const uint32_t e = (uint32_t)tid | i0 << 8 | i1 << 12 | (pc * P2) << 16;
                            S.pinfo[place] = e;
                            const bool last = split && pc == npc - 1u;
                            S.row[last ? l++ : f++] = e | place << 20;
                        }
            }
            __syncthreads();
            S.bin[tid] = 0;   // ready for the next sub-chunk

            // ---- B: the pieces' masks ----
            // (two pieces per thread at a time: their loads overlap)
            for (int idx0 = 0; idx0 < (int)P; idx0 += 2 * kBlock) {
                if (idx0 + (tid & ~63) >= (int)P) continue;   // whole wavefront idle
                Piece pc[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) pc[u] = piece_setup(S, cst, idx0 + u * kBlock + tid, (int)P);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    // (the second piece's wavefront may have nothing left)
                    if (idx0 + u * kBlock + (tid & ~63) < (int)P) piece_mask(S, pc[u], cut);
                }
            }
            __syncthreads();

            // ---- S: running sum of the counts, in road order ----
            {
                uint32_t v[8], sum = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t idx = (uint32_t)tid * 8u + (uint32_t)i;
                    v[i] = idx < P ? S.excl[idx] : 0u;
                    sum += v[i];
                }
                const uint32_t incl = wave_incl_scan(sum);
                if (lane == 63) S.w[0][wid] = incl;
                __syncthreads();
                uint32_t before = 0, total = 0;
#pragma unroll
                for (int w = 0; w < kBlock / 64; ++w) {
                    before += w < wid ? S.w[0][w] : 0u;
                    total += S.w[0][w];
                }
                uint32_t run = before + incl - sum;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t idx = (uint32_t)tid * 8u + (uint32_t)i;
                    if (idx < P) S.excl[idx] = run;
                    run += v[i];
                }
                if (tid == 0) S.excl[P] = total;
            }
            __syncthreads();
            const uint32_t T = S.excl[P];
            if (active && walk) {
                const uint32_t cnt = S.excl[rfirst + pieces] - S.excl[rfirst];
                if (cnt != (uint32_t)np) err_road = min(err_road, (uint32_t)r);
            }
            pass += T;

            // ---- W: entries, thread t taking entries t, t + 256, ... ----
            // (four entries per thread at a time: their searches and loads
            // overlap)
            const uint32_t top = P ? 1u << (31 - __builtin_clz(P)) : 0u;
            for (uint32_t e0 = (uint32_t)tid; e0 < T; e0 += 4u * kBlock) {
                uint32_t lo[4], ee[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    ee[u] = min(e0 + (uint32_t)u * kBlock, T - 1u);
                    lo[u] = 0;
                }
                // the piece of each entry: the last place with excl <= e
                // (excl[P] = T exceeds every entry)
                for (uint32_t step = top; step; step >>= 1) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t c = lo[u] + step;
                        lo[u] = S.excl[min(c, P)] <= ee[u] ? c : lo[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t e = ee[u], pl = lo[u];
                    const uint32_t pi = S.pinfo[pl];
                    const uint32_t j = pi & 255u, i0 = (pi >> 8) & 15u, i1 = (pi >> 12) & 15u,
                                   i2s = (pi >> 16) & 15u;
                    const uint32_t b = select_bit(S.mask[pl], e - S.excl[pl]);
                    const uint32_t c4 = S.n4[j];
                    const uint32_t m0 = c4 & 255u, m1 = (c4 >> 8) & 255u, m2 = (c4 >> 16) & 255u,
                                   m3 = c4 >> 24;
                    // b = (i2 - i2s) n3 + i3 with b < 32: b / n3 as b ceil(1024 / n3) / 1024
                    const uint32_t q = (b * ((1024u + m3 - 1u) / m3)) >> 10;
                    const uint32_t i2 = i2s + q, i3 = b - q * m3;
                    const uint32_t k = ((i0 * m1 + i1) * m2 + i2) * m3 + i3;
                    const uint32_t rank = e - S.excl[S.rfirst[j]];
                    const int64_t at = S.o0[j] + (int64_t)rank;
                    const uint32_t inf = S.info[j];
                    const int16_t *hh = S.hit + (inf & 0xFFFFu);
                    const uint32_t xw = S.x2[j];
                    const int32_t x[6] = {hh[i0], hh[m0 + i1], hh[m0 + m1 + i2], hh[m0 + m1 + m2 + i3],
                                          (int16_t)(xw & 0xFFFFu), (int16_t)(xw >> 16)};
                    const double *c = cst + ((inf >> 16) & 255u) * kCstStride;
                    const int32_t *ci = reinterpret_cast<const int32_t *>(c);
                    // constraint rows 3..5 (exact in fp64) and chi2 (exact: at most the cut)
                    double y[3];
#pragma unroll
                    for (int t = 0; t < 3; ++t) {
                        double v = (double)S.base[t][j];
#pragma unroll
                        for (int col = 0; col < 4; ++col) v = fma(c[3 * col + t], (double)x[col], v);
                        y[t] = v;
                    }
                    const double c2 = fma(y[2], y[2], fma(y[1], y[1], y[0] * y[0]));
                    int32_t par[3];
#pragma unroll
                    for (int t = 0; t < 3; ++t) {
                        uint32_t acc32 = (uint32_t)ci[kCstIntPB + t];
#pragma unroll
                        for (int col = 0; col < 6; ++col)
                            acc32 += (uint32_t)__mul24(ci[kCstIntP + col * 3 + t], x[col]);
                        par[t] = (int32_t)acc32;
                    }
                    if (e0 + (uint32_t)u * kBlock < T && rank < (uint32_t)S.np[j] && at >= 0 &&
                        at < a.capacity) {
                        a.k[at] = (int32_t)k;
                        a.chi2[at] = (uint64_t)c2;
                        a.params[3 * at + 0] = par[0];
                        a.params[3 * at + 1] = par[1];
                        a.params[3 * at + 2] = par[2];
                    }
                }
            }
            // the next sub-chunk starts at road s + L, its list offset after
            // this one's roads
            obase = S.o0[L - 1] + S.np[L - 1];
            s += L;
            __syncthreads();
        }
        if (rb == a.n_roads && tid == 0) a.offsets[a.n_roads] = obase;   // the list's length
    }

    // block sums -> host-mapped partials (the host reduces them)
    __shared__ BlockPartial s_part[kBlock / 64];
    const uint64_t wcomb = wave_sum64((int64_t)comb), wpass = pass;   // pass is block-uniform
    uint32_t werr = wave_min(err_road);
    if (lane == 0) s_part[wid] = BlockPartial{wcomb, wpass, 0u, werr, 0xFFFFFFFFu, 0u};
    __syncthreads();
    if (threadIdx.x == 0) {
        BlockPartial p = s_part[0];
        for (int w = 1; w < kBlock / 64; ++w) {
            p.comb += s_part[w].comb;
            p.err_road = min(p.err_road, s_part[w].err_road);
        }
        p.seq = a.seq;
        a.partials[blockIdx.x] = p;
    }
}

}  // namespace

size_t list_scratch_bytes(int32_t n_roads)
{
    const int64_t tiles = ((int64_t)n_roads + kListTile - 1) / kListTile;
    return (size_t)(tiles + 1) * sizeof(int64_t);
}

hipError_t launch_list(const ListArgs &a, int grid, int64_t *scratch, hipStream_t stream)
{
    const int64_t tiles = ((int64_t)a.n_roads + kListTile - 1) / kListTile;
    if (tiles > 0) {
        const int tgrid = (int)min(tiles, (int64_t)4096);
        hipLaunchKernelGGL(list_tile_sums, dim3(tgrid), dim3(kBlock), 0, stream, a.npass, a.n_roads,
                           scratch);
    }
    ListArgs b = a;
    b.tile_sum = scratch;
    hipLaunchKernelGGL(list_kernel, dim3(grid), dim3(kBlock), 0, stream, b);
    return hipGetLastError();
}

}  // namespace svt
