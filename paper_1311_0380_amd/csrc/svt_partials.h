// The reduction of a ring run's block partials on the device
// (svt_partials.hip), shared with the host runtime.
#pragma once
#include "svt_internal.h"

namespace svt {

constexpr int kPartialRedBlocks = 64;   // blocks of the reduction

// in[0, n) -> *out in one launch (mid holds kPartialRedBlocks partials, the
// last block to finish reduces them): the sums of comb, pass and tracks, the
// lowest err_road and err_event, and seq = *seq_dev when every input carries
// the run's sequence number *seq_dev (*seq_dev + 1 otherwise, so that the
// host sees an incomplete run).  Then *seq_dev is advanced by one for the
// next run, and *counter (zero before the launch) is zero again.
hipError_t launch_reduce_partials(const BlockPartial *in, int64_t n, BlockPartial *mid,
                                  BlockPartial *out, uint32_t *seq_dev, uint32_t *counter,
                                  hipStream_t stream);

}  // namespace svt
