// Every passing combination of a batch (arXiv:1311.0380, Sec. 2: the fit
// runs on every combination of one hit per layer; this kernel keeps each one
// within the chi2 cut, with its fit rows, instead of only the best of its
// road).
//
// One block per 64 roads (a grid-stride loop over such groups), with the
// sector constants in LDS.  Lanes 0..15 of each wavefront load one road each
// and validate it as the fit does; the block stages the group's hits in LDS
// when they fit.  Each wavefront then walks those of its 16 roads that have
// passing combinations (npass > 0, from the fit), one road at a time: its
// lanes take the combination indices k = lane, lane + 64, ..., decode
// (i0, i1, i2, i3), evaluate the constraint rows exactly in int32 and chi2
// in 64-bit integers, and the passing lanes write their entries at the
// road's offset plus their rank among the road's passing combinations so
// far (a ballot and a lane count), so the entries come out in combination
// order.  Fit rows 0..2 are evaluated for passing
// lanes only.  A road whose count of passing combinations differs from its
// npass is reported as a bad road.
#include "svt_internal.h"

namespace svt {
namespace {

constexpr int kListHitCap = 4096;
constexpr int kRoadsPerWave = 16;                        // lanes 0..15 hold the roads
static_assert(kListRoads == kRoadsPerWave * kBlock / 64, "roads per block pass");

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// t / n for t < 2^16 and 1 <= n <= 16, with m = floor((2^32 - 1) / n) + 1
// (n > 1): t m / 2^32 exceeds t / n by less than t n / 2^32 < 1 / n, so its
// integer part is the quotient.
__device__ __forceinline__ uint32_t div_small(uint32_t t, uint32_t n, uint32_t m)
{
    return n == 1 ? t : __umulhi(t, m);
}

__device__ __forceinline__ uint32_t magic(uint32_t n)
{
    return n > 1 ? 0xFFFFFFFFu / n + 1u : 0u;
}

// Every combination of one road, 64 at a time in index order; the passing
// ones are written at base + their rank.  Returns how many pass.  Hits come
// from LDS (LDS) or global memory; hb is the road's first hit there.
template <bool LDS>
__device__ __forceinline__ uint32_t list_road(const ListArgs &a, const int16_t *s_hit, int32_t hb,
                                              uint32_t m0, uint32_t m1, uint32_t m2, uint32_t m3,
                                              const int32_t (&A)[6][4], const int32_t (&z)[6],
                                              int64_t base, int64_t end, uint32_t lane)
{
    const uint32_t ncomb = m0 * m1 * m2 * m3;
    const uint32_t q1m = magic(m1), q2m = magic(m2), q3m = magic(m3);
    const int32_t p1 = hb + (int32_t)m0, p2 = p1 + (int32_t)m1, p3 = p2 + (int32_t)m2;
    uint32_t count = 0;
    for (uint32_t t0 = 0; t0 < ncomb; t0 += 64) {
        const uint32_t t = t0 + lane;
        const bool live = t < ncomb;
        const uint32_t q3 = div_small(t, m3, q3m), i3 = t - q3 * m3;
        const uint32_t q2 = div_small(q3, m2, q2m), i2 = q3 - q2 * m2;
        const uint32_t i0 = div_small(q2, m1, q1m), i1 = q2 - i0 * m1;
        int32_t x[4] = {0, 0, 0, 0};
        if (live) {
            const int16_t *h = LDS ? s_hit : a.hits;
            x[0] = h[hb + (int32_t)i0];
            x[1] = h[p1 + (int32_t)i1];
            x[2] = h[p2 + (int32_t)i2];
            x[3] = h[p3 + (int32_t)i3];
        }
        int64_t c2 = 0;
#pragma unroll
        for (int k = 3; k < 6; ++k) {
            int32_t y = z[k];
#pragma unroll
            for (int l = 0; l < 4; ++l) y += __mul24(A[k][l], x[l]);
            c2 += (int64_t)y * y;
        }
        const bool ps = live && (uint64_t)c2 <= a.cut;
        const uint64_t m = __ballot(ps);
        if (ps) {
            const int64_t at = base + count +
                               __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (at >= 0 && at < end && at < a.capacity) {
                int32_t p[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    int32_t y = z[k];
#pragma unroll
                    for (int l = 0; l < 4; ++l) y += __mul24(A[k][l], x[l]);
                    p[k] = y;
                }
                a.k[at] = (int32_t)t;
                a.chi2[at] = (uint64_t)c2;
                a.params[3 * at + 0] = p[0];
                a.params[3 * at + 1] = p[1];
                a.params[3 * at + 2] = p[2];
            }
        }
        count += (uint32_t)__popcll(m);
    }
    return count;
}

__global__ void __launch_bounds__(kBlock) list_kernel(ListArgs a)
{
    extern __shared__ int32_t s_cst[];   // per sector: rows 0..5 x 6 columns, then the 6 offsets
    __shared__ int16_t s_hit[kListHitCap];
    __shared__ BlockPartial s_part[kBlock / 64];
    const int tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const int wid = (int)(__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6);
    uint64_t comb = 0, pass = 0;
    uint32_t err_road = 0xFFFFFFFFu;

    // the sector constants, once per block
    for (int i = tid; i < a.n_sectors * 42; i += kBlock) {
        const int sct = i / 42, j = i - sct * 42;
        s_cst[i] = j < 36 ? a.coef[sct * 36 + j] : a.offset[sct * 6 + (j - 36)];
    }

    for (int64_t g0 = (int64_t)blockIdx.x * kListRoads; g0 < a.n_roads;
         g0 += (int64_t)gridDim.x * kListRoads) {
        const int32_t r0 = (int32_t)g0, r1 = (int32_t)min((int64_t)a.n_roads, g0 + kListRoads);
        // a few roads per wavefront, so that many wavefronts walk roads at once
        const int32_t r = r0 + wid * kRoadsPerWave + (int32_t)lane;
        const bool inr = lane < (uint32_t)kRoadsPerWave && r < r1;
        // the group's hit range, staged when it is well formed and fits
        const int32_t hs = a.hit_offsets[r0], he = a.hit_offsets[r1];
        const bool stage = hs >= 0 && he >= hs && he <= a.n_hits && he - hs <= kListHitCap;
        uint32_t sec = 0, nh4 = 0, x2 = 0, np = 0;
        int32_t h0 = 0, h1 = 0;
        int64_t o0 = 0, o1 = 0;
        if (inr) {
            np = (uint32_t)a.npass[r];
            sec = a.sector[r];
            nh4 = a.nhits4[r];
            h0 = a.hit_offsets[r];
            h1 = a.hit_offsets[r + 1];
            x2 = a.xft2[r];
            o0 = a.offsets[r];
            o1 = a.offsets[r + 1];
        }
        if (stage)
            for (int i = tid; i < he - hs; i += kBlock) s_hit[i] = a.hits[hs + i];
        const uint32_t n0 = nh4 & 255u, n1 = (nh4 >> 8) & 255u, n2 = (nh4 >> 16) & 255u, n3 = nh4 >> 24;
        const int32_t xa = (int16_t)(x2 & 0xFFFFu), xb = (int16_t)(x2 >> 16);
        bool ok = inr && sec < (uint32_t)a.n_sectors && n0 <= 16 && n1 <= 16 && n2 <= 16 && n3 <= 16;
        ok = ok && h0 >= 0 && h1 <= a.n_hits && (int64_t)h1 - h0 == (int64_t)(n0 + n1 + n2 + n3);
        ok = ok && xa >= 0 && xa < 4096 && xb >= 0 && xb < 4096;
        if (inr && !ok) err_road = min(err_road, (uint32_t)r);
        const bool local = stage && h0 >= hs && h1 <= he;
        __syncthreads();   // staged hits and constants visible

        // this wavefront's roads with passing combinations, one at a time
        uint64_t todo = __ballot(ok && np > 0);
        while (todo) {
            const int j = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int32_t rr = __builtin_amdgcn_readlane(r, j);
            const uint32_t s = __builtin_amdgcn_readlane(sec, j);
            const uint32_t c4 = __builtin_amdgcn_readlane(nh4, j);
            const uint32_t m0 = c4 & 255u, m1 = (c4 >> 8) & 255u, m2 = (c4 >> 16) & 255u, m3 = c4 >> 24;
            const uint32_t want = __builtin_amdgcn_readlane(np, j);
            const int32_t ya = __builtin_amdgcn_readlane(xa, j), yb = __builtin_amdgcn_readlane(xb, j);
            const int32_t hbase = __builtin_amdgcn_readlane(local ? h0 - hs : h0, j);
            const bool in_lds = __builtin_amdgcn_readlane(local ? 1 : 0, j) != 0;
            const int64_t base = ((int64_t)__builtin_amdgcn_readlane((int32_t)(o0 >> 32), j) << 32) |
                                 (uint32_t)__builtin_amdgcn_readlane((int32_t)o0, j);
            const int64_t end = ((int64_t)__builtin_amdgcn_readlane((int32_t)(o1 >> 32), j) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int32_t)o1, j);
            // the sector's rows from LDS, with the XFT columns folded into
            // each row's constant part
            const int32_t *cs = s_cst + s * 42;
            int32_t A[6][4], z[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
#pragma unroll
                for (int l = 0; l < 4; ++l) A[k][l] = cs[k * 6 + l];
                z[k] = cs[36 + k] + cs[k * 6 + 4] * ya + cs[k * 6 + 5] * yb;
            }
            const uint32_t count = in_lds
                ? list_road<true>(a, s_hit, hbase, m0, m1, m2, m3, A, z, base, end, lane)
                : list_road<false>(a, s_hit, hbase, m0, m1, m2, m3, A, z, base, end, lane);
            comb += m0 * m1 * m2 * m3;
            pass += count;
            if (count != want) err_road = min(err_road, (uint32_t)rr);
        }
        __syncthreads();   // the staged hits are reused by the next group
    }

    // block sums -> host-mapped partials (the host reduces them)
    const uint64_t wcomb = comb, wpass = pass;   // wave-uniform
    uint32_t werr = err_road;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) werr = min(werr, (uint32_t)__shfl_xor((int)werr, off, 64));
    if (lane == 0) s_part[wid] = BlockPartial{wcomb, wpass, 0u, werr, 0xFFFFFFFFu, 0u};
    __syncthreads();
    if (tid == 0) {
        BlockPartial p = s_part[0];
        for (int w = 1; w < kBlock / 64; ++w) {
            p.comb += s_part[w].comb;
            p.pass += s_part[w].pass;
            p.err_road = min(p.err_road, s_part[w].err_road);
        }
        p.seq = a.seq;
        a.partials[blockIdx.x] = p;
    }
}

}  // namespace

hipError_t launch_list(const ListArgs &a, int grid, hipStream_t stream)
{
    const size_t dyn = (size_t)a.n_sectors * 42 * sizeof(int32_t);
    hipLaunchKernelGGL(list_kernel, dim3(grid), dim3(kBlock), dyn, stream, a);
    return hipGetLastError();
}

}  // namespace svt
