// Every passing combination of a batch (arXiv:1311.0380, Sec. 2: the fit
// runs on every combination of one hit per layer; this kernel keeps each one
// within the chi2 cut, with its fit rows, instead of only the best of its
// road).
//
// Three kernels on the request's stream:
// - list_tile_sums: npass summed over tiles of kListTile roads;
// - list_tile_scan: one block turns the tile sums into a running sum;
// - list_kernel: each wavefront takes 16 consecutive roads at a time (blocks
//   of four wavefronts step over groups of 64 roads).  Its lanes 0..15 load
//   and validate one road each, as the fit does; the road's offset in the
//   list is the running sum before its tile plus the npass of the tile's
//   earlier roads, and is written out.  Each road to evaluate (valid,
//   npass > 0) gets a record in the wavefront's part of LDS: the sector's rows
//   with the XFT columns folded into each row's constant part, the hit counts
//   and the constants of the division by them, and its first slot in the
//   wavefront's run of combinations, which puts those roads' combinations one
//   after the other in road order and index order; the group's hits are
//   staged in LDS beside the records (the group's hit range at once, or road
//   by road when a road's hits lie outside it).  The wavefront then walks the run 64 slots per
//   round, whatever roads they belong to: each lane finds its road by a
//   binary search over the roads' first slots, decodes its combination index
//   k into (i0, i1, i2, i3) by multiply-high division, and evaluates the
//   constraint rows exactly in int32 and chi2 in 64-bit integers.  A passing
//   lane's place in the list is the road's offset plus the count of passing
//   slots between the road's first slot and its own (a running count, a
//   ballot and a lane count; the count at each road's first slot is kept in
//   its record), so a road's entries come out in combination order.  Fit
//   rows 0..2 are evaluated for passing lanes only.  A road whose count of
//   passing combinations differs from its npass, or whose npass is negative,
//   is reported as a bad road.
#include "svt_list.h"

namespace svt {
namespace {

constexpr int kRoadsPerWave = 16;                        // lanes 0..15 hold the roads
constexpr int kRoadHitCap = 64;                          // 4 layers of at most 16 hits
constexpr int kWaves = kBlock / 64;
static_assert(kListRoads == kRoadsPerWave * kWaves, "roads per block pass");
static_assert(kListTile % kRoadsPerWave == 0 && kListTile <= 4 * 64, "tile of the offsets scan");

// One road of a wavefront, as its lanes read it.
struct alignas(16) RoadRec {
    int4 chi[3];   // constraint rows 3..5, hit columns 0..3
    int4 zc;       // constant parts of rows 3..5; hit counts (4 x 5 bits) | first hit in LDS << 20
    int4 dec;      // first slot, division constants of n1, n2, n3
    int4 pos;      // passing slots before the first slot, npass, list offset (low, high)
    int4 par[3];   // parameter rows 0..2, hit columns 0..3
    int4 zp;       // constant parts of rows 0..2, unused
};

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Division by n in 1..16 of t < 2^16: with m = ceil(2^20 / n) = (2^20 + d) / n,
// 0 <= d < n, t m / 2^20 = t / n + t d / (n 2^20), and t d < 2^20 keeps the
// excess below 1 / n, so the integer part is the quotient.  (t << 12) < 2^28
// and m <= 2^20 fit 32 bits; the product's high word is t m / 2^20.
__device__ __forceinline__ uint32_t div_small(uint32_t t, uint32_t m)
{
    return __umulhi(t << 12, m);
}

__device__ __forceinline__ uint32_t magic(uint32_t n)
{
    return n > 0 ? ((1u << 20) + n - 1u) / n : 0u;
}

__device__ __forceinline__ int32_t row(int32_t z, const int4 &c, const int32_t (&x)[4])
{
    return z + __mul24(c.x, x[0]) + __mul24(c.y, x[1]) + __mul24(c.z, x[2]) + __mul24(c.w, x[3]);
}

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

template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
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

// One block: tile sums -> exclusive running sum in place, the total after the
// last tile and at offsets[n] (the list's length by npass).
__global__ void __launch_bounds__(kBlock) list_tile_scan(int64_t *tsum, int32_t n_tiles, int64_t *offsets,
                                                         int32_t n)
{
    __shared__ int64_t s_w[kWaves];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t carry = 0;
    for (int32_t b0 = 0; b0 < n_tiles; b0 += kBlock) {
        const int32_t b = b0 + threadIdx.x;
        const int64_t v = b < n_tiles ? tsum[b] : 0;
        const int64_t incl = wave_incl64(v);
        if (lane == 63) s_w[wid] = incl;
        __syncthreads();
        int64_t before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            before += w < wid ? s_w[w] : 0;
            tot += s_w[w];
        }
        if (b < n_tiles) tsum[b] = carry + before + incl - v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tsum[n_tiles] = carry;
        offsets[n] = carry;
    }
}

__global__ void __launch_bounds__(kBlock) list_kernel(ListArgs a)
{
    __shared__ RoadRec s_rec[kWaves][kRoadsPerWave];
    __shared__ uint32_t s_first[kWaves][kRoadsPerWave];
    __shared__ int16_t s_hit[kWaves][kRoadsPerWave * kRoadHitCap];
    __shared__ BlockPartial s_part[kWaves];
    const uint32_t lane = lane_id();
    const int wid = (int)(__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6);
    RoadRec *rec = s_rec[wid];
    uint32_t *first = s_first[wid];
    int16_t *sh = s_hit[wid];
    uint64_t comb = 0, pass = 0;
    uint32_t err_road = 0xFFFFFFFFu;

    for (int64_t g0 = (int64_t)blockIdx.x * kListRoads + wid * kRoadsPerWave; g0 < a.n_roads;
         g0 += (int64_t)gridDim.x * kListRoads) {
        const int32_t r0 = (int32_t)g0, r1 = (int32_t)min((int64_t)a.n_roads, g0 + kRoadsPerWave);
        const int32_t r = r0 + (int32_t)lane;
        const bool inr = lane < (uint32_t)kRoadsPerWave && r < r1;
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
        // npass of the tile's roads before this group (at most four loads per lane)
        const int32_t ts = r0 - r0 % kListTile;
        int64_t before = 0;
#pragma unroll
        for (int u = 0; u < kListTile / 64; ++u) {
            const int32_t i = ts + (int32_t)lane + 64 * u;
            if (i < r0) before += a.npass[i];
        }
        before = wave_sum64(before) + a.tile_excl[r0 / kListTile];

        const uint32_t n0 = nh4 & 255u, n1 = (nh4 >> 8) & 255u, n2 = (nh4 >> 16) & 255u, n3 = nh4 >> 24;
        const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
        bool ok = inr && sec < (uint32_t)a.n_sectors && n0 <= 16 && n1 <= 16 && n2 <= 16 && n3 <= 16;
        ok = ok && h0 >= 0 && h1 <= a.n_hits && (int64_t)h1 - h0 == (int64_t)(n0 + n1 + n2 + n3);
        ok = ok && xa >= 0 && xa < 4096 && xb >= 0 && xb < 4096;
        if (inr && (!ok || np < 0)) err_road = min(err_road, (uint32_t)r);
        const bool walk = ok && np > 0;
        const uint32_t nc = walk ? n0 * n1 * n2 * n3 : 0u;

        // list offsets and first slots: running sums of npass and nc over
        // lanes 0..15 (DPP row shifts within the first row of 16 lanes)
        static_assert(kRoadsPerWave == 16, "one DPP row");
        int64_t po = np;
        uint32_t incl = nc;
        po += dpp64<0x111, 0xf>(po);
        incl += dpp32<0x111>(incl);
        po += dpp64<0x112, 0xf>(po);
        incl += dpp32<0x112>(incl);
        po += dpp64<0x114, 0xf>(po);
        incl += dpp32<0x114>(incl);
        po += dpp64<0x118, 0xf>(po);
        incl += dpp32<0x118>(incl);
        const int64_t o0 = before + po - np;
        if (inr) a.offsets[r] = o0;
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kRoadsPerWave - 1);
        const uint32_t start = lane < (uint32_t)kRoadsPerWave ? incl - nc : total;
        if (lane < (uint32_t)kRoadsPerWave) first[lane] = start;

        // the group's hits in LDS: its hit range when every road to evaluate
        // lies inside it (then a road's hits start at h0 - hs), else road by
        // road at 64 places each
        const int32_t hs = __builtin_amdgcn_readfirstlane(h0);
        const int32_t he = __builtin_amdgcn_readlane(h1, r1 - r0 - 1);
        const bool range = hs >= 0 && hs <= he && he <= a.n_hits &&
                           he - hs <= kRoadsPerWave * kRoadHitCap &&
                           __ballot(walk && (h0 < hs || h1 > he)) == 0;
        uint32_t hbase;
        if (range) {
            const int32_t cnt = he - hs;
            for (int32_t i0 = 0; i0 < cnt; i0 += 4 * 64) {
                int16_t v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t i = i0 + (int32_t)lane + 64 * u;
                    v[u] = i < cnt ? a.hits[hs + i] : (int16_t)0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t i = i0 + (int32_t)lane + 64 * u;
                    if (i < cnt) sh[i] = v[u];
                }
            }
            hbase = (uint32_t)(h0 - hs);
        } else {
            int16_t v[kRoadsPerWave];
#pragma unroll
            for (int u = 0; u < kRoadsPerWave; ++u) {
                const int32_t hb = __builtin_amdgcn_readlane(h0, u);
                const uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane(walk ? h1 - h0 : 0, u);
                v[u] = lane < cnt ? a.hits[hb + (int32_t)lane] : (int16_t)0;
            }
#pragma unroll
            for (int u = 0; u < kRoadsPerWave; ++u) {
                const uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane(walk ? h1 - h0 : 0, u);
                if (lane < cnt) sh[u * kRoadHitCap + (int32_t)lane] = v[u];
            }
            hbase = lane * (uint32_t)kRoadHitCap;
        }

        if (walk) {
            // the sector's rows, with the XFT columns folded into each row's
            // constant part
            const int2 *cf = reinterpret_cast<const int2 *>(a.coef + sec * 36);
            const int2 *of = reinterpret_cast<const int2 *>(a.offset + sec * 6);
            int32_t A[6][6], b[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    const int2 t = cf[k * 3 + l];
                    A[k][2 * l] = t.x;
                    A[k][2 * l + 1] = t.y;
                }
            }
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int2 t = of[l];
                b[2 * l] = t.x;
                b[2 * l + 1] = t.y;
            }
            int32_t z[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) z[k] = b[k] + __mul24(A[k][4], xa) + __mul24(A[k][5], xb);
            RoadRec &q = rec[lane];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                q.chi[k] = make_int4(A[k + 3][0], A[k + 3][1], A[k + 3][2], A[k + 3][3]);
                q.par[k] = make_int4(A[k][0], A[k][1], A[k][2], A[k][3]);
            }
            q.zc = make_int4(z[3], z[4], z[5], (int32_t)(n0 | n1 << 5 | n2 << 10 | n3 << 15 | hbase << 20));
            q.dec = make_int4((int32_t)start, (int32_t)magic(n1), (int32_t)magic(n2), (int32_t)magic(n3));
            q.pos = make_int4(0, np, (int32_t)(uint32_t)o0, (int32_t)(o0 >> 32));
            q.zp = make_int4(z[0], z[1], z[2], 0);
        }

        // the run, 64 slots per round
        uint32_t run = 0, rb = 0;
        for (uint32_t f0 = 0; f0 < total; f0 += 64) {
            const uint32_t f = f0 + lane;
            const bool live = f < total;
            // the last road whose first slot is at or before f
            uint32_t j = 0;
#pragma unroll
            for (uint32_t step = kRoadsPerWave / 2; step > 0; step >>= 1)
                j += first[j + step] <= f ? step : 0u;
            uint64_t c2 = 0;
            int32_t x[4] = {0, 0, 0, 0};
            uint32_t k = 0;
            if (live) {
                const RoadRec &q = rec[j];
                const int4 zc = q.zc, dec = q.dec;
                k = f - (uint32_t)dec.x;
                const uint32_t w = (uint32_t)zc.w;
                const uint32_t m0 = w & 31u, m1 = (w >> 5) & 31u, m2 = (w >> 10) & 31u, m3 = (w >> 15) & 31u;
                const uint32_t q3 = div_small(k, (uint32_t)dec.w), i3 = k - q3 * m3;
                const uint32_t q2 = div_small(q3, (uint32_t)dec.z), i2 = q3 - q2 * m2;
                const uint32_t i0 = div_small(q2, (uint32_t)dec.y), i1 = q2 - i0 * m1;
                const int16_t *hr = sh + (w >> 20);
                x[0] = hr[i0];
                x[1] = hr[m0 + i1];
                x[2] = hr[m0 + m1 + i2];
                x[3] = hr[m0 + m1 + m2 + i3];
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const int32_t y = row(t == 0 ? zc.x : t == 1 ? zc.y : zc.z, q.chi[t], x);
                    c2 += (uint64_t)((int64_t)y * y);
                }
            }
            const bool ps = live && c2 <= a.cut;
            const uint64_t m = __ballot(ps);
            // roads whose first slot is in this round: passing slots before it
            if (start >= f0 && start < f0 + 64 && lane < (uint32_t)kRoadsPerWave) {
                rb = run + (uint32_t)__popcll(m & ((1ull << (start - f0)) - 1ull));
                rec[lane].pos.x = (int32_t)rb;
            }
            if (ps) {
                const RoadRec &q = rec[j];
                const int4 pos = q.pos, zp = q.zp;
                const uint32_t rank = run +
                                      __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) -
                                      (uint32_t)pos.x;
                const int64_t at = (((int64_t)pos.w) << 32 | (uint32_t)pos.z) + rank;
                if (at >= 0 && rank < (uint32_t)pos.y && at < a.capacity) {
                    a.k[at] = (int32_t)k;
                    a.chi2[at] = c2;
                    a.params[3 * at + 0] = row(zp.x, q.par[0], x);
                    a.params[3 * at + 1] = row(zp.y, q.par[1], x);
                    a.params[3 * at + 2] = row(zp.z, q.par[2], x);
                }
            }
            run += (uint32_t)__popcll(m);
        }
        // each road's count of passing combinations: the next road's base
        // minus its own (roads that start at the run's end have all of it)
        if (start >= total) rb = run;
        const uint32_t nxt = (uint32_t)__shfl_down((int)rb, 1, 64);
        if (walk && nxt - rb != (uint32_t)np) err_road = min(err_road, (uint32_t)r);
        comb += total;
        pass += run;
    }

    // block sums -> host-mapped partials (the host reduces them)
    const uint64_t wcomb = comb, wpass = pass;   // wave-uniform
    uint32_t werr = err_road;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) werr = min(werr, (uint32_t)__shfl_xor((int)werr, off, 64));
    if (lane == 0) s_part[wid] = BlockPartial{wcomb, wpass, 0u, werr, 0xFFFFFFFFu, 0u};
    __syncthreads();
    if (threadIdx.x == 0) {
        BlockPartial p = s_part[0];
        for (int w = 1; w < kWaves; ++w) {
            p.comb += s_part[w].comb;
            p.pass += s_part[w].pass;
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
    hipLaunchKernelGGL(list_tile_scan, dim3(1), dim3(kBlock), 0, stream, scratch, (int32_t)tiles,
                       a.offsets, a.n_roads);
    ListArgs b = a;
    b.tile_excl = scratch;
    hipLaunchKernelGGL(list_kernel, dim3(grid), dim3(kBlock), 0, stream, b);
    return hipGetLastError();
}

}  // namespace svt
