/*
 * svt.h -- C ABI of libsvt.so, the MI355X (gfx950) SVT linearized track fit.
 *
 * The operation (arXiv:1311.0380, Sec. 2 and Sec. 2.1): for every event and
 * every road of the event, enumerate every combination of one hit per
 * silicon layer, evaluate the per-sector linearized fit
 *     p_i = f_i . x + q_i            (Sec. 2, the fit equation)
 * for six rows -- rows 0..2 the track words (d0, phi, curvature), rows 3..5
 * the chi2 constraint components -- form chi2 = y3^2 + y4^2 + y5^2 with
 * integer additions and multiplications (Sec. 2), apply the chi2 cut and
 * keep the best passing combination of each road.
 *
 * Conventions fixed by this library where the paper is silent:
 *   - fit input of a combination: x = (h0[i0], h1[i1], h2[i2], h3[i3], xft0, xft1),
 *     every word in [0, 4096);
 *   - combination index k = ((i0*n1 + i1)*n2 + i2)*n3 + i3 (layer 0 most
 *     significant: the order of the nested loops of Sec. 2.1);
 *   - arithmetic is exact: y_k in int32 (guaranteed by the constant bound
 *     checked at load), chi2 in uint64, no shift and no rounding;
 *   - a combination passes when chi2 <= cut; the best is the passing
 *     combination with the smallest chi2, ties to the smallest k.
 *
 * All functions return svt_status (SVT_OK = 0, negative = error), never throw,
 * and may be called from several threads as long as calls on one context are
 * serialized by the caller.
 */
#ifndef SVT_H
#define SVT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t svt_status;
typedef int64_t svt_ticket;
typedef struct svt_ctx svt_ctx;
typedef struct svt_plan svt_plan;

enum {
    SVT_OK = 0,
    SVT_E_INVAL = -1,   /* malformed call: NULL pointer, negative count, bad kind  */
    SVT_E_RANGE = -2,   /* malformed data: see svt_summary.err_road / err_event    */
    SVT_E_NOMEM = -3,   /* the request exceeds the context's device-memory budget  */
    SVT_E_STATE = -4,   /* wrong state: no constants loaded, tickets in flight ... */
    SVT_E_AGAIN = -5,   /* not finished yet (poll) / no free ticket slot          */
    SVT_E_DEVICE = -6   /* a HIP runtime error; svt_last_error() has its text      */
};

/* Where a buffer lives. */
enum {
    SVT_MEM_PAGEABLE = 0,  /* ordinary host memory: copied through the DMA engine     */
    SVT_MEM_PINNED = 1,    /* page-locked host memory (hipHostMalloc): async DMA copy  */
    SVT_MEM_MAPPED = 2,    /* page-locked host memory mapped into the GPU address
                              space: kernels read / write it in place (zero copy)      */
    SVT_MEM_DEVICE = 3     /* device memory (hipMalloc, torch CUDA tensors)            */
};

/*
 * One batch of events (Sec. 2: events contain roads; a road holds the hits of
 * each layer and selects a sector constant set).  CSR layout:
 *   road_offsets [n_events+1] int32   roads of event e: [road_offsets[e], road_offsets[e+1]);
 *                                     road_offsets[0] = 0, nondecreasing, last = n_roads
 *   sector       [n_roads]    uint8   constant set of the road, < n_sectors
 *   nhits        [n_roads*4]  uint8   hits in layers 0..3, each 0..16 (0 = no combination)
 *   hit_offsets  [n_roads+1]  int32   hits of road r: [hit_offsets[r], hit_offsets[r+1]),
 *                                     difference = sum of nhits; first 0, last = n_hits
 *   hits         [n_hits]     int16   hit words, layer-major inside a road, in [0, 4096)
 *   xft          [n_roads*2]  int16   the road's two XFT words (curvature, phi), in [0, 4096)
 * All pointers share mem_kind.  nhits and xft must be 4-byte aligned.
 */
typedef struct {
    int32_t n_events, n_roads, n_hits, mem_kind;
    const int32_t *road_offsets;
    const uint8_t *sector;
    const uint8_t *nhits;
    const int32_t *hit_offsets;
    const int16_t *hits;
    const int16_t *xft;
} svt_event_batch;

/*
 * Per-road and per-event results (Sec. 2: d0, phi, p_T word and chi2 of the
 * fitted track).  Sizes are those of the batch they answer.
 *   ncomb     [n_roads]   int32   n0*n1*n2*n3
 *   npass     [n_roads]   int32   combinations with chi2 <= cut
 *   best      [n_roads]   int32   k of the best passing combination, -1 if none
 *   chi2      [n_roads]   uint64  its chi2, UINT64_MAX if none
 *   params    [n_roads*3] int32   its fit rows 0..2, 0 if none
 *   hit_index [n_roads*4] uint8   its (i0, i1, i2, i3), 0xFF if none (4-byte aligned)
 *   ntracks   [n_events]  int32   roads of the event with a best combination
 *   comb_offsets [n_roads+1] int64, may be NULL: exclusive prefix sum of ncomb
 * All pointers share mem_kind.  On any error status the contents are unspecified.
 */
typedef struct {
    int32_t *ncomb;
    int32_t *npass;
    int32_t *best;
    uint64_t *chi2;
    int32_t *params;
    uint8_t *hit_index;
    int32_t *ntracks;
    int64_t *comb_offsets;
    int32_t mem_kind;
    int32_t pad_;
} svt_results;

typedef struct {
    int64_t total_comb;     /* sum of ncomb                                       */
    int64_t total_pass;     /* sum of npass                                       */
    int32_t total_tracks;   /* sum of ntracks                                     */
    int32_t err_road;       /* lowest malformed road, -1 if none                  */
    int32_t err_event;      /* lowest malformed event, -1 if none                 */
    int32_t status;         /* status of the request (same as svt_result returns) */
    int64_t device_ns;      /* device time of the request: the fit kernel's own
                               dispatch when the request is that kernel alone
                               (device or mapped buffers, no comb_offsets);
                               otherwise from the first to the last command,
                               copies included; 0 for a fit request that
                               svt_set_timing left untimed                          */
} svt_summary;

/* Launch shape of the fit: each block takes a chunk of events (by default
 * sized for about 256 roads).  Results are the same bit for bit whatever the
 * shape. */
typedef struct {
    int32_t events_per_chunk;  /* events per work item (1..256); 0 = automatic    */
    int32_t blocks_per_cu;     /* grid = CUs * blocks_per_cu (1..16), fewer when
                                  there are fewer chunks; 0 = automatic           */
    int32_t schedule;          /* 1 = cyclic (item w -> worker w mod workers),
                                  2 = blocked, 3 = balanced by roads (each block
                                  takes the events whose first road falls in its
                                  equal share of the roads); 0 keeps the current
                                  value                                           */
    int32_t kernel;            /* 0 or 1: the block-per-chunk kernel (the only
                                  one; other values are SVT_E_INVAL)              */
} svt_tuning;

/*
 * Context: one device, its resident constants, a device-memory budget for
 * staging buffers and scratch, a stream and a ring of ticket slots.
 * device: HIP device ordinal.  hbm_budget_bytes: upper bound on the device
 * memory the context may allocate (0 = no bound).  *out receives the context.
 * Errors: SVT_E_INVAL (out NULL, bad device), SVT_E_DEVICE, SVT_E_NOMEM.
 */
svt_status svt_create(svt_ctx **out, int32_t device, size_t hbm_budget_bytes);
/* Waits for all requests of the context, then frees everything it owns. */
svt_status svt_destroy(svt_ctx *ctx);

/*
 * Per-sector constant sets f_i, q_i of the linearized fit (Sec. 2) and the
 * chi2 cut.  coef [n_sectors][6][6] int32 row-major (coef[s][k][j] multiplies
 * input j in row k); offset [n_sectors][6] int32; host memory, copied -- the
 * caller may free it on return.  n_sectors in 1..256; chi2_cut < 2^48.
 * Every row must satisfy sum_j |coef[s][k][j]|*4095 + |offset[s][k]| <= 2^31-1
 * (then every fit row is exact in int32).  Errors: SVT_E_INVAL (NULL,
 * n_sectors out of range), SVT_E_RANGE (bound or cut violated), SVT_E_STATE
 * (requests in flight), SVT_E_DEVICE.
 */
svt_status svt_load_constants(svt_ctx *ctx, int32_t n_sectors, const int32_t *coef,
                              const int32_t *offset, uint64_t chi2_cut);

/*
 * Fit every road of a batch (asynchronous).  Copies host inputs to device
 * staging (PAGEABLE, PINNED), or reads them in place (MAPPED, DEVICE), runs
 * the fit, and copies results back when they are host memory.  hip_stream is
 * a hipStream_t (NULL = the null stream, as everywhere in HIP).  The caller keeps every
 * buffer alive and unmodified until svt_result() has returned something other
 * than SVT_E_AGAIN for *ticket.  Errors returned here: SVT_E_INVAL,
 * SVT_E_STATE (no constants), SVT_E_NOMEM (staging over budget), SVT_E_AGAIN
 * (all ticket slots in flight), SVT_E_DEVICE.  Data errors (SVT_E_RANGE) are
 * found on the device and reported by svt_result().
 */
svt_status svt_fit_events(svt_ctx *ctx, const svt_event_batch *batch, const svt_results *res,
                          void *hip_stream, svt_ticket *ticket);

/*
 * Completion of a request.  wait_us: -1 blocks, 0 polls, > 0 waits at most
 * that long.  Returns SVT_E_AGAIN while running; otherwise the request's
 * status (SVT_OK, SVT_E_RANGE with err_road / err_event set, SVT_E_DEVICE),
 * fills *out (may be NULL) and releases the ticket.  Unknown or released
 * tickets: SVT_E_INVAL.
 */
svt_status svt_result(svt_ctx *ctx, svt_ticket ticket, int32_t wait_us, svt_summary *out);

/*
 * Every passing combination of a batch, road by road in combination-index
 * order (Sec. 2: the fit runs on all combinations; this keeps each one
 * within the cut with its fit words, not only the best of its road).
 * Device memory (SVT_MEM_DEVICE) only:
 *   offsets [n_roads+1] int64   written: road r's entries are
 *                               [offsets[r], offsets[r+1]) (running sum of npass)
 *   k       [capacity]  int32   combination index in its road (layer 0 most significant)
 *   chi2    [capacity]  uint64  its chi2 (<= cut)
 *   params  [capacity*3] int32  its fit rows 0..2
 */
typedef struct {
    int64_t *offsets;
    int32_t *k;
    uint64_t *chi2;
    int32_t *params;
    int64_t capacity;       /* entries k, chi2 and params hold (>= 0)              */
} svt_pass_list;

/*
 * List every passing combination of `batch` (asynchronous; batch, npass and
 * list in device memory).  npass [n_roads] int32 are the pass counts of the
 * same batch under the loaded constants, as svt_fit_events wrote them: they
 * place each road's entries, and roads with npass 0 are not evaluated again.
 * Events are not read.  svt_result() then gives total_pass = entries listed
 * (offsets[n_roads]) and total_comb = combinations evaluated; it returns
 * SVT_E_RANGE when a road is malformed, its npass is negative or its passing
 * combinations differ in number from its npass (err_road = the lowest such
 * road), or when the list
 * exceeds capacity (err_road = -1; entries past capacity are not written).
 * Errors returned here: SVT_E_INVAL, SVT_E_STATE (no constants), SVT_E_AGAIN,
 * SVT_E_NOMEM, SVT_E_DEVICE.
 */
svt_status svt_list_passing(svt_ctx *ctx, const svt_event_batch *batch, const int32_t *npass,
                            const svt_pass_list *list, void *hip_stream, svt_ticket *ticket);

/*
 * svt_list_passing for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same contracts, results and errors, but the running sums
 * of the pass counts go to a fixed 512 KiB scratch array that the library
 * holds on each device until the process ends, so the call allocates
 * nothing.  At most 2^24 roads: a larger batch returns SVT_E_NOMEM, and
 * svt_last_error() names the limit.  Every call on one device shares that
 * array, whatever its context or stream: calls that overlap on one device
 * race, and the caller must not let them overlap (wait for one with
 * svt_result before submitting the next).  SVT_E_STATE when the device has
 * no scratch (device ordinals above 63).
 */
svt_status svt_list_passing_noalloc(svt_ctx *ctx, const svt_event_batch *batch,
                                    const int32_t *npass, const svt_pass_list *list,
                                    void *hip_stream, svt_ticket *ticket);

/*
 * Packed input word stream (this library's own format; the paper's unpack
 * stage, Sec. 2.1, reads the experiment's raw words, whose format is not
 * given).  32-bit words, the top two bits a tag:
 *   3 event header  bits 29..0 zero; the roads up to the next event header
 *                   belong to it
 *   2 road header   bits 29..22 sector, bits 19..0 the hit counts of layers
 *                   0..3 (5 bits each, layer 0 lowest, each <= 16), 21..20 zero
 *   1 XFT word      bits 11..0 first XFT word, 23..12 second, 29..24 zero
 *   0 hit word      two hits in layer-major order, bits 11..0 the first and
 *                   23..12 the second (zero in a road's last word when its
 *                   hit count is odd), bits 29..24 zero
 * A road is its header, its XFT word and ceil(hits / 2) hit words; the
 * stream starts with an event header.
 */
typedef struct {
    int32_t *road_offsets;  /* [max_events+1]  as in svt_event_batch           */
    uint8_t *sector;        /* [max_roads]                                      */
    uint8_t *nhits;         /* [max_roads*4], 4-byte aligned                    */
    int32_t *hit_offsets;   /* [max_roads+1]                                    */
    int16_t *hits;          /* [max_hits]                                       */
    int16_t *xft;           /* [max_roads*2], 4-byte aligned                    */
    int32_t max_events, max_roads, max_hits, pad_;
} svt_unpack_out;

/*
 * Unpack a word stream into the batch arrays of `out` (device memory), ready
 * for svt_fit_events (asynchronous).  mem_kind says where `words` lives:
 * SVT_MEM_DEVICE (read in place), SVT_MEM_MAPPED (read in place over the
 * bus: zero copy), SVT_MEM_PINNED or SVT_MEM_PAGEABLE (copied to device
 * staging first).  n_words < 2^31.
 * svt_result() then gives the batch's size in the summary -- total_tracks =
 * events, total_comb = roads, total_pass = hits -- and returns SVT_E_RANGE
 * when the stream breaks the format (err_road = the index of the first word
 * out of place, n_words if it ends inside a road; the arrays are then
 * unspecified) or when the batch exceeds a capacity (err_road = -1).
 * Errors returned here: SVT_E_INVAL, SVT_E_AGAIN, SVT_E_NOMEM, SVT_E_DEVICE.
 */
svt_status svt_unpack_stream(svt_ctx *ctx, const uint32_t *words, int64_t n_words, int32_t mem_kind,
                             const svt_unpack_out *out, void *hip_stream, svt_ticket *ticket);

/* Static text for a status; svt_last_error() is the last HIP error text of
 * the calling thread (empty if none). */
const char *svt_status_string(svt_status status);
const char *svt_last_error(void);

/* Launch shape used by later requests (affects speed only, never results). */
svt_status svt_set_tuning(svt_ctx *ctx, const svt_tuning *tuning);
svt_status svt_get_tuning(svt_ctx *ctx, svt_tuning *tuning);

/* Which later fit requests (svt_fit_events, svt_plan_fit) measure their
 * device time: every = 1
 * (the default) all of them, every = N > 1 those whose ticket is a multiple
 * of N, every = 0 none.  An untimed request records only its completion on
 * the stream, which costs the host far less per launch than a start
 * timestamp as well (on ROCm 7, about 3 us against 14 us); its summary
 * reports device_ns = 0.  Results never change.  Other requests are always
 * timed.  Errors: SVT_E_INVAL (every < 0). */
svt_status svt_set_timing(svt_ctx *ctx, int32_t every);

/* Device facts used for reporting: compute units, clock (kHz), HBM bytes. */
typedef struct {
    int32_t compute_units;
    int32_t clock_khz;
    int64_t hbm_bytes;
    int64_t budget_bytes;
    int64_t used_bytes;
    char arch[32];
} svt_device_info;
svt_status svt_get_device_info(svt_ctx *ctx, svt_device_info *info);

/* Transfer probe for the I/O study (the one-GPU analog of the paper's
 * comparison of copy strategies, Sec. 4.2): reps transfers of `bytes` between
 * a fresh host buffer of the given kind and device memory, timed one by one
 * with events on the context's stream; *median_us receives the median.
 * kind: SVT_MEM_PAGEABLE or SVT_MEM_PINNED (DMA copies), SVT_MEM_MAPPED (a
 * kernel reading / writing the mapped host buffer in place).  direction:
 * 0 = host to device, 1 = device to host.  Allocates and frees its buffers
 * (device memory counts against the context's budget). */
svt_status svt_io_probe(svt_ctx *ctx, int32_t kind, int32_t direction, size_t bytes,
                        int32_t reps, double *median_us);

/* ------------------------------------------------------------------------
 * Plans: uneven batches fitted by one persistent, graph-captured launch.
 * A plan owns device buffers for a batch of up to max_events / max_roads /
 * max_hits and a captured graph [copy of the batch sizes from pinned host
 * memory -> fit kernel over a fixed persistent grid reading those sizes], so
 * one graph replays any batch within capacity.  The launch shape comes from
 * tuning (NULL or 0 fields: the context's).  Constants are captured: after
 * svt_load_constants the plan must be recreated (svt_plan_fit returns
 * SVT_E_STATE).  One request per plan may be in flight.
 * ------------------------------------------------------------------------ */
svt_status svt_plan_create(svt_ctx *ctx, int32_t max_events, int32_t max_roads, int32_t max_hits,
                           const svt_tuning *tuning, svt_plan **out);
svt_status svt_plan_destroy(svt_plan *plan);

/* Device views of the plan's own input and result buffers (capacities in the
 * counts).  A batch whose pointers are these buffers is fitted in place, and
 * results requested into these buffers are not copied. */
svt_status svt_plan_buffers(svt_plan *plan, svt_event_batch *in, svt_results *out);

/* Like svt_fit_events (same contracts and errors; completion through
 * svt_result on the plan's context), replaying the plan's graph.  Inputs
 * and results of any memory kind are copied into / out of the plan's
 * buffers unless they are those buffers.  Batches above capacity:
 * SVT_E_INVAL.  comb_offsets, if requested, must be device memory. */
svt_status svt_plan_fit(svt_plan *plan, const svt_event_batch *batch, const svt_results *res,
                        void *hip_stream, svt_ticket *ticket);

/* ------------------------------------------------------------------------
 * Rings: device-resident batches fitted back to back in one graph launch.
 * A read-out that fills a ring of device buffers while the GPU fits them in
 * order is the steady state of the fit; the paper times 100 repetitions of
 * each sample back to back (Sec. 4.1), which a ring of 100 passes gives
 * without host launch gaps between them.  svt_ring_create prepares the
 * launches of n_passes fit passes and the reduction of their block sums,
 * captured as one graph when there are more than four launches, and
 * enqueued one by one at each run otherwise (a graph launch adds some 20 us
 * from the host call to its first kernel): pass p fits batches[p % n_batches] into
 * results[p % n_batches] (a later pass over the same batch rewrites the same
 * results).  Every batch and results must be device memory (SVT_MEM_DEVICE),
 * without comb_offsets, and follows the svt_fit_events layout; the arrays
 * are copied, the buffers they point to are not, and must stay alive and
 * unmodified while the ring exists.  n_batches in 1..n_passes, n_passes in
 * 1..1024.  The launch shape is the context's tuning at creation.  Constants
 * are captured: after svt_load_constants the ring must be recreated
 * (svt_ring_run returns SVT_E_STATE).  Destroy rings before their context.
 * ------------------------------------------------------------------------ */
typedef struct svt_ring svt_ring;
/* passes_per_launch: passes one kernel launch covers (each of its batches
 * spread over the same number of blocks), 1..128, or 0 for automatic (at
 * most 128, the passes split evenly over the launches).  Results do not
 * depend on it. */
svt_status svt_ring_create(svt_ctx *ctx, int32_t n_batches, const svt_event_batch *batches,
                           const svt_results *results, int32_t n_passes, int32_t passes_per_launch,
                           svt_ring **out);
/* Run the ring's passes on hip_stream (asynchronous; one run per ring in
 * flight, else SVT_E_AGAIN).  svt_result on the ring's context then gives the
 * sums over all passes (total_comb = sum over passes of each pass's
 * combinations, and so on), the lowest err_road / err_event any pass
 * reported (each the index within that pass's batch) and device_ns from the
 * first pass to the last. */
svt_status svt_ring_run(svt_ring *ring, void *hip_stream, svt_ticket *ticket);
/* The ring's shape: its passes, the passes one kernel launch covers and the
 * launches per run (any pointer may be NULL). */
svt_status svt_ring_info(const svt_ring *ring, int32_t *n_passes, int32_t *passes_per_launch,
                         int32_t *n_launches);
/* Waits for the ring's run in flight, if any, then frees it. */
svt_status svt_ring_destroy(svt_ring *ring);

/* ------------------------------------------------------------------------
 * Float shadow of the fit, for calibrating the constants before they are
 * quantized.  The same linearized fit (Sec. 2: each row a scalar product of
 * per-sector constants with the inputs plus an offset) evaluated in fp32 on
 * unquantized input words, with every sum over tracks accumulated in fp64 in
 * a fixed order (bit-reproducible).  Loss of N tracks:
 *   L = (1/N) sum_t [ sum_{k<3} w_k (y_k - tau_k)^2 + sum_{k>=3} y_k^2 ]
 *       + lambda sum_s || C_s C_s^T - I ||_F^2       (C_s: rows 3..5 of sector s)
 * All pointers below are device memory; calls are asynchronous on hip_stream
 * (NULL = the null stream).  Shadow calls on one context must not run
 * concurrently on different streams (they share the context's scratch).
 * Errors: SVT_E_INVAL (NULL, counts out of range), SVT_E_NOMEM, SVT_E_DEVICE.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_tracks, n_sectors;     /* n_sectors in 1..256                      */
    const float *x;                  /* [n_tracks][6] input words                */
    const float *tau;                /* [n_tracks][3] truth of rows 0..2         */
    const int32_t *sector_offsets;   /* [n_sectors+1] tracks of sector s are
                                        [off[s], off[s+1]); off[0] = 0,
                                        nondecreasing, last = n_tracks (other
                                        values are clamped, never read out of
                                        bounds, and give unspecified results)   */
    float w[3];                      /* weights of the row 0..2 residuals        */
    int32_t pad_;
} svt_shadow_tracks;

/* Blocks per sector the forward and backward run over (slices of about 2048
 * tracks of one sector each, at least 1 and at most 64; the partial sums of a
 * sector's slices are then reduced in slice order).  Reporting only: results
 * never depend on it beyond fp64 rounding order, which is fixed for given
 * counts.  Errors: SVT_E_INVAL (slices NULL, n_tracks < 0, n_sectors out of
 * 1..256). */
svt_status svt_shadow_slices(int32_t n_tracks, int32_t n_sectors, int32_t *slices);

/* Fit rows y (optional [n_tracks][6], may be NULL) and the data term of L
 * (double, written to loss[0]).  coef [n_sectors][6][6], offset [n_sectors][6]. */
svt_status svt_shadow_forward(svt_ctx *ctx, const svt_shadow_tracks *tracks, const float *coef,
                              const float *offset, float *y, double *loss, void *hip_stream);

/* scale * dL_data/dcoef and scale * dL_data/doffset (hand-written backward:
 * (2/N) sum_t w_k r_tk x_tj and (2/N) sum_t w_k r_tk), written in fp64, and
 * also in fp32 where the _f32 pointers are not NULL.  scale is a device
 * double (the incoming gradient of the loss), NULL meaning 1. */
svt_status svt_shadow_backward(svt_ctx *ctx, const svt_shadow_tracks *tracks, const float *coef,
                               const float *offset, const double *scale, double *grad_coef,
                               double *grad_offset, float *grad_coef_f32,
                               float *grad_offset_f32, void *hip_stream);

/* value[0] = lambda sum_s ||C_s C_s^T - I||^2; its gradient 4 lambda (C C^T - I) C
 * is ADDED to grad_coef (fp64; rows 3..5) and the sum copied to grad_coef_f32
 * when not NULL. */
svt_status svt_shadow_penalty(svt_ctx *ctx, int32_t n_sectors, const float *coef, double lambda,
                              double *value, double *grad_coef, float *grad_coef_f32,
                              void *hip_stream);

/* One Adam step on n fp32 parameters from fp64 gradients (step counts from 1). */
svt_status svt_shadow_adam(svt_ctx *ctx, int32_t n, float *param, const double *grad, float *m,
                           float *v, float lr, float beta1, float beta2, float eps, int32_t step,
                           void *hip_stream);

/* Integer constants from fp32 ones, per sector: the largest shift S in
 * [-30, 30] such that every |rint(A 2^S)| < max_abs and every row satisfies
 * the svt_load_constants bound; rint rounds half to even.  Writes coef_int
 * [S][6][6], offset_int [S][6], shift [S]; sets *status (device int) to 1 if
 * a sector has no valid shift (its shift is then INT32_MIN). */
svt_status svt_requantize(svt_ctx *ctx, int32_t n_sectors, const float *coef, const float *offset,
                          int32_t max_abs, int32_t *coef_int, int32_t *offset_int, int32_t *shift,
                          int32_t *status, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SVT_H */
