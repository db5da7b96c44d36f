// Block partials of a ring run reduced on the device, so that the host reads
// one summary instead of every block's (a 100-pass run over the 3000-event
// batch has 76,800 of them).  The same sums, minima and sequence check as
// the host's reduction of a single request's partials.
#include "svt_partials.h"

namespace svt {
namespace {

constexpr int kWaves = kBlock / 64;

// The partials in[lo, hi) -> *out, by the whole block.
__device__ void reduce_range(const BlockPartial *in, int64_t lo, int64_t hi, uint32_t seq,
                             BlockPartial *out)
{
    __shared__ uint64_t s_comb[kWaves], s_pass[kWaves];
    __shared__ uint32_t s_tr[kWaves], s_er[kWaves], s_ee[kWaves], s_bad[kWaves];
    uint64_t comb = 0, pass = 0;
    uint32_t tr = 0, er = 0xFFFFFFFFu, ee = 0xFFFFFFFFu, bad = 0;
    for (int64_t i = lo + (int64_t)threadIdx.x; i < hi; i += kBlock) {
        const BlockPartial p = in[i];
        comb += p.comb;
        pass += p.pass;
        tr += p.tracks;
        er = min(er, p.err_road);
        ee = min(ee, p.err_event);
        bad |= p.seq != seq ? 1u : 0u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        comb += __shfl_xor(comb, off, 64);
        pass += __shfl_xor(pass, off, 64);
        tr += (uint32_t)__shfl_xor((int)tr, off, 64);
        er = min(er, (uint32_t)__shfl_xor((int)er, off, 64));
        ee = min(ee, (uint32_t)__shfl_xor((int)ee, off, 64));
        bad |= (uint32_t)__shfl_xor((int)bad, off, 64);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_comb[wid] = comb;
        s_pass[wid] = pass;
        s_tr[wid] = tr;
        s_er[wid] = er;
        s_ee[wid] = ee;
        s_bad[wid] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        BlockPartial r{0, 0, 0, 0xFFFFFFFFu, 0xFFFFFFFFu, 0};
        uint32_t b = 0;
        for (int w = 0; w < kWaves; ++w) {
            r.comb += s_comb[w];
            r.pass += s_pass[w];
            r.tracks += s_tr[w];
            r.err_road = min(r.err_road, s_er[w]);
            r.err_event = min(r.err_event, s_ee[w]);
            b |= s_bad[w];
        }
        r.seq = b ? seq + 1u : seq;
        *out = r;
    }
}

__global__ void __launch_bounds__(kBlock) reduce_partials_a(const BlockPartial *in, int64_t n,
                                                            BlockPartial *mid, const uint32_t *seq_dev)
{
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = min(n, (int64_t)blockIdx.x * per), hi = min(n, lo + per);
    reduce_range(in, lo, hi, *seq_dev, mid + blockIdx.x);
}

__global__ void __launch_bounds__(kBlock) reduce_partials_b(const BlockPartial *mid, int32_t n,
                                                            BlockPartial *out, const uint32_t *seq_dev)
{
    reduce_range(mid, 0, n, *seq_dev, out);
}

}  // namespace

hipError_t launch_reduce_partials(const BlockPartial *in, int64_t n, BlockPartial *mid,
                                  BlockPartial *out, const uint32_t *seq_dev, hipStream_t stream)
{
    hipLaunchKernelGGL(reduce_partials_a, dim3(kPartialRedBlocks), dim3(kBlock), 0, stream, in, n, mid,
                       seq_dev);
    hipLaunchKernelGGL(reduce_partials_b, dim3(1), dim3(kBlock), 0, stream, mid,
                       (int32_t)kPartialRedBlocks, out, seq_dev);
    return hipGetLastError();
}

}  // namespace svt
