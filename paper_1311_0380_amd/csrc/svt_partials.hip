// Block partials of a ring run reduced on the device, so that the host reads
// one summary instead of every block's (a 100-pass run over the 3000-event
// batch has 75,000 of them).  The same sums, minima and sequence check as
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

// One launch: every block reduces its share of in[0, n) into mid[block];
// the block that finishes last (a counter, released and acquired at device
// scope, so that the other blocks' mid entries are visible to it) reduces
// mid into *out, resets the counter and advances the run's sequence number.
__global__ void __launch_bounds__(kBlock) reduce_partials(const BlockPartial *in, int64_t n,
                                                          BlockPartial *mid, BlockPartial *out,
                                                          uint32_t *seq_dev, uint32_t *counter)
{
    __shared__ uint32_t s_last;
    const uint32_t seq = *seq_dev;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = min(n, (int64_t)blockIdx.x * per), hi = min(n, lo + per);
    reduce_range(in, lo, hi, seq, mid + blockIdx.x);
    if (threadIdx.x == 0) {
        // (thread 0 wrote mid[block]; the release orders that write first)
        const uint32_t done =
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = done == gridDim.x - 1u ? 1u : 0u;
    }
    __syncthreads();
    if (s_last == 0u) return;
    // every thread of the last block acquires before it reads mid
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    reduce_range(mid, 0, gridDim.x, seq, out);
    if (threadIdx.x == 0) {
        *counter = 0u;          // ready for the next run (stream order)
        *seq_dev = seq + 1u;    // the next run's sequence number
    }
}

}  // namespace

hipError_t launch_reduce_partials(const BlockPartial *in, int64_t n, BlockPartial *mid,
                                  BlockPartial *out, uint32_t *seq_dev, uint32_t *counter,
                                  hipStream_t stream)
{
    hipLaunchKernelGGL(reduce_partials, dim3(kPartialRedBlocks), dim3(kBlock), 0, stream, in, n, mid,
                       out, seq_dev, counter);
    return hipGetLastError();
}

}  // namespace svt
