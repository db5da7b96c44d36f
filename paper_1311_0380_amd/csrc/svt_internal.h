// Internal declarations shared by the host runtime and the kernels of libsvt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svt {

// Launch geometry of the fused fit kernel.
constexpr int kBlock = 256;        // threads per block (4 wave64)
constexpr int kSubRoads = 256;     // roads per sub-chunk: one thread per road
constexpr int kHitCap = 4096;      // hits staged in LDS per sub-chunk
constexpr int kRowCap = 1536;      // rows per sub-chunk (the block kernel's row list)
constexpr int kMaxEventsPerChunk = 256;
constexpr int kMaxBlocksPerCu = 16;
constexpr int kTargetRoadsPerChunk = 256;
// Per sector, in device memory, read by the fit kernel through the caches
// (stride kCstStride doubles = 272 bytes):
//   doubles [0, 18)   constraint rows 3..5, 6 columns x 3 rows ([col * 3 + row])
//   int32   [36, 39)  offsets of rows 3..5
//   int32   [40, 58)  parameter rows 0..2, 6 columns x 3 rows ([col * 3 + row])
//   int32   [58, 61)  offsets of rows 0..2
constexpr int kCstStride = 34;
constexpr int kCstBytesPerSector = kCstStride * 8;
constexpr int kCstIntB = 36;      // int32 index of the constraint offsets
constexpr int kCstIntP = 40;      // int32 index of the parameter columns
constexpr int kCstIntPB = 58;     // int32 index of the parameter offsets

// Sizes of a batch when they are read from device memory (graph replay).
struct Sizes {
    int32_t n_events, n_roads, n_hits;
    uint32_t seq;   // request sequence number (graph replays)
};

// Partial sums of one block, written by the block into host-mapped memory and
// reduced by the host when the request completes (no device-wide atomics or
// fences: contended atomics serialize and device-scope fences write back and
// invalidate an XCD's whole L2).
struct BlockPartial {
    uint64_t comb;
    uint64_t pass;
    uint32_t tracks;
    uint32_t err_road;    // lowest bad road, 0xFFFFFFFF if none
    uint32_t err_event;   // lowest bad event, 0xFFFFFFFF if none
    uint32_t seq;         // request sequence number
};

struct FitArgs {
    // batch (device-visible pointers)
    const int32_t *road_offsets;
    const uint8_t *sector;
    const uint32_t *nhits4;     // 4 x uint8 per road
    const int32_t *hit_offsets;
    const int16_t *hits;
    const uint32_t *xft2;       // 2 x int16 per road
    int32_t n_events, n_roads, n_hits;
    int32_t n_sectors;
    const Sizes *sizes;         // non-NULL: sizes are read from here instead
    const uint32_t *seq_dev;    // non-NULL: the request's sequence number is read here
    // constants (device)
    const int32_t *coef;        // [n_sectors][6][6]
    const int32_t *offset;      // [n_sectors][6]
    double cut_d;               // chi2 cut as a double (exact: < 2^48)
    // results (device-visible pointers)
    int32_t *ncomb;
    int32_t *npass;
    int32_t *best;
    uint64_t *chi2;
    int32_t *params;
    uint32_t *hit_index4;       // 4 x uint8 per road
    int32_t *ntracks;
    const double *cst_block;    // the kernel's table of the constants: [n_sectors][kCstStride]
    int32_t frac_key;           // 1: cut < 2^44, minimise chi2 + index / 256
    // launch shape
    int32_t events_per_chunk;
    int32_t schedule;           // 1 cyclic, 2 blocked
    // request bookkeeping
    BlockPartial *partials;     // host-mapped, one per block the batch is spread over
    uint32_t seq;
};

// start/stop non-NULL: the dispatch itself records them around the kernel
// (no separate event packets on the stream).
hipError_t launch_fit(const FitArgs &a, int grid, hipStream_t stream, hipEvent_t start = nullptr,
                      hipEvent_t stop = nullptr);
// n1 + n2 batches in one launch of the block kernel: args is device memory
// holding one FitArgs per batch; batch i < n1 is spread over blocks
// [i per, (i+1) per), and batch n1 + j over the per2 blocks after the first
// n1 per and j per2.
hipError_t launch_fit_multi(const FitArgs *args, int n1, int per, int n2, int per2, hipStream_t stream);
hipError_t launch_comb_offsets(const int32_t *ncomb, int64_t *comb_offsets, int32_t n_roads,
                               int64_t *scratch, hipStream_t stream);
size_t comb_offsets_scratch_bytes(int32_t n_roads);

}  // namespace svt
