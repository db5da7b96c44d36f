// Transfer probe for the I/O study: host <-> device latency and bandwidth for
// pageable, pinned and mapped host memory on one GPU (the one-GPU analog of
// the paper's comparison of copy strategies, Sec. 4.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "svt.h"

namespace svt {
namespace {

// In-place access of mapped host memory by the GPU (zero copy).
__global__ void __launch_bounds__(256) zero_copy(const uint4 *src, uint4 *dst, size_t n16,
                                                 const uint8_t *src_tail, uint8_t *dst_tail,
                                                 size_t tail)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
    if (blockIdx.x == 0 && threadIdx.x < tail) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
}

}  // namespace

hipError_t launch_zero_copy(const void *src, void *dst, size_t bytes, int cus, hipStream_t st)
{
    const size_t n16 = bytes / 16, tail = bytes - n16 * 16;
    size_t blocks = (n16 + 255) / 256;
    const size_t cap = (size_t)cus * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_copy, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16,
                       static_cast<const uint8_t *>(src) + n16 * 16,
                       static_cast<uint8_t *>(dst) + n16 * 16, tail);
    return hipGetLastError();
}

}  // namespace svt
