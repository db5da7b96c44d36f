// Declarations of the packed-word-stream unpack (svt_unpack.hip), shared
// with the host runtime.
#pragma once
#include "svt_internal.h"

namespace svt {

// The unpack of a packed word stream (svt_unpack.hip).
struct UnpackAgg {              // over a range of words (positions < 2^31)
    int64_t hits;               // hits the road headers declare
    int32_t ev, rd;             // event headers, road headers
    int32_t last_road, last_ev; // last road / event header, -1 if none
    uint32_t last_hdr, pad_;    // the last road header's word (0 if none)
};
struct UnpackArgs {
    const uint32_t *src;        // the words as given (device-visible)
    uint32_t *words;            // the words in device memory (== src if already there)
    int32_t copy;               // 1: the first pass copies src into words
    int32_t src_vec, words_vec; // 1: src / words 16-byte aligned (4-word loads)
    int64_t n_words;
    UnpackAgg *tiles;           // [tiles]: the sums over each tile
    int32_t *road_offsets;      // outputs, [max_events + 1] ...
    uint8_t *sector;
    uint32_t *nhits4;
    int32_t *hit_offsets;
    int16_t *hits;
    uint32_t *xft2;
    int32_t max_events, max_roads, max_hits;
    int32_t n_apply;            // blocks of the last pass (a grid-stride loop over the
                                // tiles); the totals' partial follows theirs
    BlockPartial *partials;     // host-mapped, [n_apply + 1]
    uint32_t seq;
};
int64_t unpack_tiles(int64_t n_words);
size_t unpack_scratch_bytes(int64_t n_words);
int64_t unpack_max_words();
int32_t unpack_apply_blocks(int64_t n_words, int max_partials);
hipError_t launch_unpack(UnpackArgs a, hipStream_t stream);

}  // namespace svt
