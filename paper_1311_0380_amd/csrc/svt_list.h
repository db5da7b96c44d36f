// Declarations of the passing-combination list (svt_list.hip), shared with
// the host runtime.
#pragma once
#include "svt_internal.h"

namespace svt {

// The list of every passing combination (svt_list.hip).
struct ListArgs {
    const uint8_t *sector;
    const uint32_t *nhits4;
    const int32_t *hit_offsets;
    const int16_t *hits;
    const uint32_t *xft2;
    const int32_t *npass;       // pass counts of the fit, [n_roads]
    int64_t *offsets;           // out: exclusive running sum of npass, [n_roads + 1]
    const int64_t *tile_sum;    // npass summed over each tile of kListTile roads
    int32_t n_roads, n_hits, n_sectors;
    const double *cst;          // the fit kernel's table of the constants: [n_sectors][kCstStride]
    uint64_t cut;               // < 2^48
    int32_t *k;                 // entries: combination index, chi2, fit rows 0..2
    uint64_t *chi2;
    int32_t *params;
    int64_t capacity;
    BlockPartial *partials;     // host-mapped, [gridDim.x]
    uint32_t seq;
};
constexpr int kListTile = 256;   // roads per tile of the offsets scan and per block pass of the list kernel
size_t list_scratch_bytes(int32_t n_roads);
// The offsets scan and the list kernel; scratch holds list_scratch_bytes.
hipError_t launch_list(const ListArgs &a, int grid, int64_t *scratch, hipStream_t stream);

}  // namespace svt
