// Host runtime of libsvt: contexts, resident constants, staging, tickets.
// Implements the C ABI declared in include/svt.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "svt.h"
#include "svt_internal.h"
#include "svt_list.h"
#include "svt_unpack.h"
#include "svt_partials.h"
#include "svt_shadow.h"
#include "svt_submit_guard.h"

namespace svt {
hipError_t launch_zero_copy(const void *src, void *dst, size_t bytes, int cus, hipStream_t st);
}

namespace {

thread_local std::string g_last_error;

svt_status hip_fail(hipError_t e, const char *what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_last_error = buf;
    return SVT_E_DEVICE;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

constexpr int kSlots = 64;
// Rings of at most this many fit launches enqueue their kernels on the
// caller's stream at each run instead of launching a captured graph: a graph
// launch took some 20 us longer from the host call to its first kernel.
#ifndef SVT_RING_DIRECT_MAX
#define SVT_RING_DIRECT_MAX 4
#endif
constexpr int kRingDirectMax = SVT_RING_DIRECT_MAX;
constexpr int kRingCounter = 32;   // a ring's reduction counter: seq_dev[32], 128 bytes on

// Scratch of svt_list_passing_noalloc: the running sums of the pass counts
// (one int64 per tile of svt::kListTile roads, plus the total) for at most
// kNoAllocRoads roads, 512 KiB.  Every device holds its own copy until the
// process ends.  Host code never uses the array's name as an address: it
// uses the device address svt_create takes for each device.
constexpr int32_t kNoAllocRoads = 1 << 24;
constexpr int64_t kNoAllocWords = ((int64_t)kNoAllocRoads + svt::kListTile - 1) / svt::kListTile + 1;
static __device__ __align__(256) int64_t scratch[(kNoAllocWords + 31) / 32 * 32];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t *g_scratch_dev[kMaxDevices] = {};   // device address of `scratch` on each device

// Once per device, with that device current: the device address of its copy
// of the scratch array.
svt_status scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return SVT_OK;   // no allocation-free calls there
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device] != nullptr) return SVT_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[device] = static_cast<int64_t *>(p);
    return SVT_OK;
}

struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
};

struct Slot {
    bool busy = false;
    svt_ticket ticket = -1;
    hipEvent_t ev_start = nullptr, ev_end = nullptr;
    svt::BlockPartial *partials = nullptr;   // host-mapped [max grid]
    svt::BlockPartial *parts = nullptr;      // partials the request in flight writes
    int grid = 0;                            // blocks of the request in flight
    svt_plan *plan = nullptr;                // plan of the request, if any
    svt_ring *ring = nullptr;                // ring of the request, if any
    uint32_t ring_seq = 0;                   // a ring run's sequence number
    DevBuf stage;                            // device staging for host inputs / results
    DevBuf scan;                             // scratch of the running sums (offsets scans)
    svt_status host_status = SVT_OK;
    int64_t list_capacity = -1;              // a passing-combination list: its capacity
    bool timed = true;                       // ev_start was recorded (device_ns valid)
    bool unpack = false;                     // a stream unpack: its capacities
    int64_t unpack_cap[3] = {0, 0, 0};
};

}  // namespace

struct svt_ctx {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    int clock_khz = 0;
    size_t hbm_bytes = 0;
    char arch[32] = {0};
    int max_grid = 0;
    // constants
    int32_t *coef = nullptr;
    int32_t *offset = nullptr;
    void *cst_block = nullptr;               // the fit kernel's table of the constants
    int32_t n_sectors = 0;
    uint64_t cut = 0;
    bool loaded = false;
    // requests
    Slot slots[kSlots];
    svt_ticket next_ticket = 1;
    DevBuf shadow_scratch;                   // float-shadow partial sums
    std::vector<DevBuf> pool;                // idle staging buffers
    uint64_t const_gen = 0;                  // bumped by every svt_load_constants
    svt_tuning tuning{0, 0, 1, 0};  // automatic chunk, occupancy and kernel; cyclic
    int32_t timing_every = 1;                // fit requests that record their start
};

// A captured fit of any batch up to a fixed capacity (see svt_plan_create).
struct svt_plan {
    svt_ctx *ctx = nullptr;
    int32_t max_events = 0, max_roads = 0, max_hits = 0;
    void *buf = nullptr;                    // device: inputs + results at capacity
    size_t buf_bytes = 0;
    svt_event_batch in{};                   // device views of the input buffers
    svt_results out{};                      // device views of the result buffers
    // the batch's sizes: host-mapped, written by svt_plan_fit and read by the
    // captured kernel through sizes_dev (its device view), so the graph needs
    // no copy node
    svt::Sizes *sizes_host = nullptr;
    const svt::Sizes *sizes_dev = nullptr;
    svt::BlockPartial *partials = nullptr;  // host-mapped [grid]
    int grid = 0;
    svt_tuning tuning{};
    uint64_t const_gen = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool busy = false;
};

// A captured sequence of fit passes over resident batches (see svt_ring_create).
struct svt_ring {
    svt_ctx *ctx = nullptr;
    int32_t n_batches = 0, n_passes = 0;
    int32_t per_launch = 1;                 // passes per kernel launch
    int total_parts = 0;                    // block partials of all passes
    svt::BlockPartial *parts_dev = nullptr; // device [total_parts], pass after pass
    svt::BlockPartial *mid_dev = nullptr;   // device: the reduction blocks' partials
    svt::BlockPartial *summary = nullptr;   // host-mapped: the run's reduced partial
    // device: [0] the run's sequence number, which the fit kernels read and
    // the reduction advances at the end of each run; [kRingCounter] the
    // reduction's block counter
    uint32_t *seq_dev = nullptr;
    uint32_t runs = 0;                      // runs enqueued (the next run's sequence number)
    svt::FitArgs *args_dev = nullptr;       // device: the launch arguments of every pass
    size_t args_bytes = 0;
    uint64_t const_gen = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // a ring of few launches enqueues its kernels itself (no graph): the
    // first pass of each launch, its passes and its grid; the passes'
    // arguments on the host for one-pass launches
    struct Launch {
        int32_t p0, np, grid;        // first pass, head passes, blocks per head pass
        int32_t n_tail, tail_grid;   // then n_tail passes of tail_grid blocks each
    };
    std::vector<Launch> launches;
    std::vector<svt::FitArgs> args_host;
    svt::BlockPartial *summary_dev = nullptr;
    bool direct = false;
    bool busy = false;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

svt_status dev_alloc(svt_ctx *c, void **p, size_t bytes)
{
    if (c->budget && c->used + bytes > c->budget) return SVT_E_NOMEM;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return SVT_E_NOMEM;
    }
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    c->used += bytes;
    return SVT_OK;
}

void dev_free(svt_ctx *c, void *p, size_t bytes)
{
    if (p) {
        (void)hipFree(p);
        c->used -= bytes;
    }
}

svt_status ensure(svt_ctx *c, DevBuf &b, size_t bytes)
{
    if (b.cap >= bytes) return SVT_OK;
    size_t want = bytes + bytes / 4;
    if (c->budget && c->used - b.cap + want > c->budget) want = bytes;
    if (c->budget && c->used - b.cap + want > c->budget) return SVT_E_NOMEM;
    dev_free(c, b.ptr, b.cap);
    b.ptr = nullptr;
    b.cap = 0;
    void *p = nullptr;
    svt_status st = dev_alloc(c, &p, want);
    if (st != SVT_OK) return st;
    b.ptr = p;
    b.cap = want;
    return SVT_OK;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Staging buffers of requests in flight come from a pool: best fit among the
// idle buffers, else a new allocation, first releasing idle buffers when the
// budget requires it.  SVT_E_NOMEM means the in-flight requests leave no
// room for this one now.
svt_status stage_acquire(svt_ctx *c, DevBuf &out, size_t bytes)
{
    int best = -1;
    for (int i = 0; i < (int)c->pool.size(); ++i)
        if (c->pool[i].cap >= bytes && (best < 0 || c->pool[i].cap < c->pool[best].cap)) best = i;
    if (best >= 0) {
        out = c->pool[best];
        c->pool.erase(c->pool.begin() + best);
        return SVT_OK;
    }
    const size_t want = align_up(bytes, (size_t)1 << 20);
    while (c->budget && c->used + want > c->budget && !c->pool.empty()) {
        int big = 0;
        for (int i = 1; i < (int)c->pool.size(); ++i)
            if (c->pool[i].cap > c->pool[big].cap) big = i;
        dev_free(c, c->pool[big].ptr, c->pool[big].cap);
        c->pool.erase(c->pool.begin() + big);
    }
    void *p = nullptr;
    svt_status st = dev_alloc(c, &p, want);
    if (st != SVT_OK) return st;
    out.ptr = p;
    out.cap = want;
    return SVT_OK;
}

void stage_release(svt_ctx *c, DevBuf &b)
{
    if (b.ptr) c->pool.push_back(b);
    b.ptr = nullptr;
    b.cap = 0;
}

bool kind_ok(int32_t k) { return k >= SVT_MEM_PAGEABLE && k <= SVT_MEM_DEVICE; }

// Device-visible address of a caller buffer of the given kind.
const void *device_view(const void *p, int32_t kind)
{
    if (p == nullptr || kind != SVT_MEM_MAPPED) return p;
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, const_cast<void *>(p), 0) != hipSuccess) {
        (void)hipGetLastError();
        return p;   // on ROCm host pointers of pinned memory are valid device addresses
    }
    return d;
}

int auto_events_per_chunk(int32_t n_events, int32_t n_roads, int target, int max_events)
{
    if (n_events <= 0) return 1;
    const double rpe = (double)n_roads / (double)n_events;
    int e = rpe > 0 ? (int)((double)target / rpe + 0.5) : max_events;
    if (e < 1) e = 1;
    if (e > max_events) e = max_events;
    return e;
}

// Roads per chunk of the block kernel, from the work a road is expected to
// hold.  With m hits per road on average, a road of four equal layers has
// about (m / 4)^4 combinations (never fewer than that for unequal means).
// A chunk aims at the batch's combinations spread over the grid's slots,
// kept between 2048 and 10000 combinations, and at 16 to 256 roads:
// 256-road chunks of 256-combination roads would leave most of the grid idle.
int block_roads_per_chunk(int32_t n_roads, int32_t n_hits, int64_t slots)
{
    if (n_roads <= 0) return svt::kTargetRoadsPerChunk;
    const double m = (double)n_hits / (double)n_roads / 4.0;
    const double per_road = m * m * m * m > 1.0 ? m * m * m * m : 1.0;
    double target = per_road * (double)n_roads / (double)(slots > 0 ? slots : 1);
    target = target < 2048.0 ? 2048.0 : (target > 10000.0 ? 10000.0 : target);
    int roads = (int)(target / per_road + 0.5);
    if (roads < 16) roads = 16;
    if (roads > svt::kTargetRoadsPerChunk) roads = svt::kTargetRoadsPerChunk;
    return roads;
}

// Chunking and grid of a launch of the fit kernel (a chunk per block).  A
// persistent grid (graph plans) keeps the full size; otherwise the grid
// shrinks to the number of chunks.  Five blocks are resident per CU, but the
// chunks are sized for three: fuller sub-chunks cost less per road, and the
// other slots are filled by the blocks of the next pass or request (with
// four resident blocks, one 3000 x 64-road pass alone: 15.9 us against 15.5
// with chunks sized for four; back to back: 10.0 us against 11.4).
struct LaunchShape {
    int epc;      // events per chunk
    int grid;
};

LaunchShape launch_shape(const svt_ctx *c, const svt_tuning &t, int32_t ne, int32_t nr, int32_t nh,
                         bool persistent, int chunk_mult = 1)
{
    LaunchShape ls;
    const int bpc = t.blocks_per_cu > 0 ? t.blocks_per_cu : 5;
    const int sizing = t.blocks_per_cu > 0 ? t.blocks_per_cu : 3;
    ls.epc = t.events_per_chunk > 0
                 ? t.events_per_chunk
                 : auto_events_per_chunk(
                       ne, nr, block_roads_per_chunk(nr, nh, (int64_t)c->cu_count * sizing) * chunk_mult,
                       svt::kMaxEventsPerChunk);
    int64_t grid = (int64_t)c->cu_count * bpc;
    if (!persistent && t.schedule == 3) {
        // balanced by roads: at least 64 roads per block
        const int64_t need = ((int64_t)nr + 63) / 64;
        if (grid > need) grid = need;
    } else if (!persistent) {
        const int64_t n_chunks = ne > 0 ? ((int64_t)ne + ls.epc - 1) / ls.epc : 0;
        if (grid > n_chunks) grid = n_chunks;
    }
    if (grid < 1) grid = 1;
    ls.grid = (int)grid;
    return ls;
}

// The launch arguments that follow from the context's tables and the shape.
void set_shape_args(const svt_ctx *c, svt::FitArgs &a, const LaunchShape &ls)
{
    a.frac_key = c->cut < (1ull << 44) ? 1 : 0;
    a.cst_block = static_cast<const double *>(c->cst_block);
    a.events_per_chunk = ls.epc;
}

hipError_t launch_shaped(const svt_ctx *c, svt::FitArgs &a, const LaunchShape &ls,
                         hipStream_t st, hipEvent_t start = nullptr, hipEvent_t stop = nullptr)
{
    set_shape_args(c, a, ls);
    return svt::launch_fit(a, ls.grid, st, start, stop);
}

// Call-level validation shared by the fit entry points.
svt_status check_call(const svt_event_batch *b, const svt_results *res)
{
    if (!kind_ok(b->mem_kind) || !kind_ok(res->mem_kind)) return SVT_E_INVAL;
    const int32_t ne = b->n_events, nr = b->n_roads, nh = b->n_hits;
    if (ne < 0 || nr < 0 || nh < 0) return SVT_E_INVAL;
    if (ne == 0 && nr != 0) return SVT_E_INVAL;
    if (nr == 0 && nh != 0) return SVT_E_INVAL;
    if (ne == INT32_MAX || nr == INT32_MAX) return SVT_E_INVAL;
    if (b->road_offsets == nullptr) return SVT_E_INVAL;
    if (nr > 0 && (b->sector == nullptr || b->nhits == nullptr || b->hit_offsets == nullptr ||
                   b->xft == nullptr))
        return SVT_E_INVAL;
    if (nh > 0 && b->hits == nullptr) return SVT_E_INVAL;
    if (nr > 0 && (res->ncomb == nullptr || res->npass == nullptr || res->best == nullptr ||
                   res->chi2 == nullptr || res->params == nullptr || res->hit_index == nullptr))
        return SVT_E_INVAL;
    if (ne > 0 && res->ntracks == nullptr) return SVT_E_INVAL;
    if ((reinterpret_cast<uintptr_t>(b->nhits) | reinterpret_cast<uintptr_t>(b->xft) |
         reinterpret_cast<uintptr_t>(res->hit_index)) & 3u)
        return SVT_E_INVAL;
    return SVT_OK;
}

}  // namespace

extern "C" {

const char *svt_status_string(svt_status s)
{
    switch (s) {
    case SVT_OK: return "SVT_OK";
    case SVT_E_INVAL: return "SVT_E_INVAL: malformed call";
    case SVT_E_RANGE: return "SVT_E_RANGE: malformed data";
    case SVT_E_NOMEM: return "SVT_E_NOMEM: over the device-memory budget";
    case SVT_E_STATE: return "SVT_E_STATE: wrong state";
    case SVT_E_AGAIN: return "SVT_E_AGAIN: not finished / no free slot";
    case SVT_E_DEVICE: return "SVT_E_DEVICE: HIP runtime error";
    default: return "unknown status";
    }
}

const char *svt_last_error(void) { return g_last_error.c_str(); }

svt_status svt_create(svt_ctx **out, int32_t device, size_t hbm_budget_bytes)
{
    if (out == nullptr) return SVT_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return SVT_E_INVAL;
    DeviceGuard g(device);
    svt_ctx *c = new (std::nothrow) svt_ctx();
    if (c == nullptr) return SVT_E_NOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    c->cu_count = prop.multiProcessorCount;
    c->clock_khz = prop.clockRate;
    c->hbm_bytes = prop.totalGlobalMem;
    snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
    c->max_grid = c->cu_count * svt::kMaxBlocksPerCu;
    {
        const svt_status ss = scratch_setup(device);
        if (ss != SVT_OK) {
            delete c;
            return ss;
        }
    }
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipStreamCreate");
    }
    for (int i = 0; i < kSlots; ++i) {
        Slot &s = c->slots[i];
        svt_status st = SVT_OK;
        if (hipEventCreate(&s.ev_start) != hipSuccess || hipEventCreate(&s.ev_end) != hipSuccess)
            st = hip_fail(hipGetLastError(), "hipEventCreate");
        if (st == SVT_OK &&
            hipHostMalloc(reinterpret_cast<void **>(&s.partials),
                          sizeof(svt::BlockPartial) * c->max_grid,
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
            st = hip_fail(hipGetLastError(), "hipHostMalloc");
        if (st != SVT_OK) {
            *out = c;
            svt_destroy(c);
            *out = nullptr;
            return st;
        }
        memset(s.partials, 0, sizeof(svt::BlockPartial) * c->max_grid);
    }
    *out = c;
    return SVT_OK;
}

svt_status svt_destroy(svt_ctx *c)
{
    if (c == nullptr) return SVT_E_INVAL;
    DeviceGuard g(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i < kSlots; ++i) {
        Slot &s = c->slots[i];
        if (s.busy && s.ev_end) (void)hipEventSynchronize(s.ev_end);
        if (s.ev_start) (void)hipEventDestroy(s.ev_start);
        if (s.ev_end) (void)hipEventDestroy(s.ev_end);
        if (s.partials) (void)hipHostFree(s.partials);
        if (s.stage.ptr) (void)hipFree(s.stage.ptr);
        if (s.scan.ptr) (void)hipFree(s.scan.ptr);
    }
    if (c->coef) (void)hipFree(c->coef);
    if (c->cst_block) (void)hipFree(c->cst_block);
    if (c->shadow_scratch.ptr) (void)hipFree(c->shadow_scratch.ptr);
    for (DevBuf &b : c->pool) (void)hipFree(b.ptr);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return SVT_OK;
}

svt_status svt_load_constants(svt_ctx *c, int32_t n_sectors, const int32_t *coef,
                              const int32_t *offset, uint64_t chi2_cut)
{
    if (c == nullptr || coef == nullptr || offset == nullptr) return SVT_E_INVAL;
    if (n_sectors < 1 || n_sectors > 256) return SVT_E_INVAL;
    if (chi2_cut >= (1ull << 48)) return SVT_E_RANGE;
    for (int s = 0; s < n_sectors; ++s)
        for (int k = 0; k < 6; ++k) {
            int64_t bound = llabs((long long)offset[s * 6 + k]);
            for (int j = 0; j < 6; ++j) bound += llabs((long long)coef[(s * 6 + k) * 6 + j]) * 4095;
            if (bound > 2147483647LL) return SVT_E_RANGE;
        }
    for (int i = 0; i < kSlots; ++i)
        if (c->slots[i].busy) return SVT_E_STATE;
    DeviceGuard g(c->device);
    if (c->coef == nullptr) {
        void *p = nullptr;
        svt_status st = dev_alloc(c, &p, 256 * 42 * sizeof(int32_t));
        if (st != SVT_OK) return st;
        c->coef = static_cast<int32_t *>(p);
        c->offset = c->coef + 256 * 36;
    }
    if (c->cst_block == nullptr) {
        svt_status st = dev_alloc(c, &c->cst_block, (size_t)256 * svt::kCstBytesPerSector);
        if (st != SVT_OK) return st;
    }
    HIP_TRY(hipMemcpy(c->coef, coef, sizeof(int32_t) * 36 * n_sectors, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->offset, offset, sizeof(int32_t) * 6 * n_sectors, hipMemcpyHostToDevice));
    {
        // the fit kernel's table (see svt_internal.h for the layout)
        std::vector<double> img((size_t)n_sectors * svt::kCstStride, 0.0);
        for (int s = 0; s < n_sectors; ++s) {
            const int32_t *A = coef + s * 36, *b = offset + s * 6;
            double *d = img.data() + (size_t)s * svt::kCstStride;
            int32_t *ci = reinterpret_cast<int32_t *>(d);
            for (int col = 0; col < 6; ++col)
                for (int k = 0; k < 3; ++k) {
                    d[col * 3 + k] = (double)A[(3 + k) * 6 + col];
                    ci[svt::kCstIntP + col * 3 + k] = A[k * 6 + col];
                }
            for (int k = 0; k < 3; ++k) {
                ci[svt::kCstIntB + k] = b[3 + k];
                ci[svt::kCstIntPB + k] = b[k];
            }
        }
        HIP_TRY(hipMemcpy(c->cst_block, img.data(), img.size() * 8, hipMemcpyHostToDevice));
    }
    c->n_sectors = n_sectors;
    c->cut = chi2_cut;
    c->loaded = true;
    ++c->const_gen;
    return SVT_OK;
}

svt_status svt_set_tuning(svt_ctx *c, const svt_tuning *t)
{
    if (c == nullptr || t == nullptr) return SVT_E_INVAL;
    if (t->events_per_chunk < 0 || t->events_per_chunk > svt::kMaxEventsPerChunk) return SVT_E_INVAL;
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > svt::kMaxBlocksPerCu) return SVT_E_INVAL;
    if (t->schedule < 0 || t->schedule > 3) return SVT_E_INVAL;
    if (t->kernel < 0 || t->kernel > 1) return SVT_E_INVAL;
    c->tuning.events_per_chunk = t->events_per_chunk;   // 0 = automatic
    c->tuning.blocks_per_cu = t->blocks_per_cu;         // 0 = automatic
    if (t->schedule) c->tuning.schedule = t->schedule;
    c->tuning.kernel = t->kernel;
    return SVT_OK;
}

svt_status svt_set_timing(svt_ctx *c, int32_t every)
{
    if (c == nullptr || every < 0) return SVT_E_INVAL;
    c->timing_every = every;
    return SVT_OK;
}

svt_status svt_get_tuning(svt_ctx *c, svt_tuning *t)
{
    if (c == nullptr || t == nullptr) return SVT_E_INVAL;
    *t = c->tuning;
    return SVT_OK;
}

svt_status svt_get_device_info(svt_ctx *c, svt_device_info *info)
{
    if (c == nullptr || info == nullptr) return SVT_E_INVAL;
    memset(info, 0, sizeof *info);
    info->compute_units = c->cu_count;
    info->clock_khz = c->clock_khz;
    info->hbm_bytes = (int64_t)c->hbm_bytes;
    info->budget_bytes = (int64_t)c->budget;
    info->used_bytes = (int64_t)c->used;
    snprintf(info->arch, sizeof info->arch, "%s", c->arch);
    return SVT_OK;
}

svt_status svt_fit_events(svt_ctx *c, const svt_event_batch *b, const svt_results *res,
                          void *hip_stream, svt_ticket *ticket)
{
    if (c == nullptr || b == nullptr || res == nullptr || ticket == nullptr) return SVT_E_INVAL;
    const svt_status vs = check_call(b, res);
    if (vs != SVT_OK) return vs;
    const int32_t ne = b->n_events, nr = b->n_roads, nh = b->n_hits;
    if (!c->loaded) return SVT_E_STATE;

    // a free ticket slot
    const int si = (int)(c->next_ticket % kSlots);
    Slot &s = c->slots[si];
    if (s.busy) return SVT_E_AGAIN;

    DeviceGuard g(c->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream

    // byte layout of inputs and results
    const size_t b_ro = sizeof(int32_t) * ((size_t)ne + 1), b_sec = (size_t)nr,
                 b_nh = 4 * (size_t)nr, b_ho = sizeof(int32_t) * ((size_t)nr + 1),
                 b_hits = sizeof(int16_t) * (size_t)nh, b_xft = 4 * (size_t)nr;
    const size_t b_ncomb = 4 * (size_t)nr, b_np = 4 * (size_t)nr, b_best = 4 * (size_t)nr,
                 b_chi2 = 8 * (size_t)nr, b_par = 12 * (size_t)nr, b_hi = 4 * (size_t)nr,
                 b_ntr = 4 * (size_t)ne, b_co = res->comb_offsets ? 8 * ((size_t)nr + 1) : 0;
    const bool stage_in = b->mem_kind == SVT_MEM_PAGEABLE || b->mem_kind == SVT_MEM_PINNED;
    const bool stage_out = res->mem_kind == SVT_MEM_PAGEABLE || res->mem_kind == SVT_MEM_PINNED;
    size_t off = 0;
    size_t o_ro = 0, o_sec = 0, o_nh = 0, o_ho = 0, o_hits = 0, o_xft = 0;
    if (stage_in) {
        o_ro = off; off = align_up(off + b_ro, 256);
        o_sec = off; off = align_up(off + b_sec, 256);
        o_nh = off; off = align_up(off + b_nh, 256);
        o_ho = off; off = align_up(off + b_ho, 256);
        o_hits = off; off = align_up(off + b_hits, 256);
        o_xft = off; off = align_up(off + b_xft, 256);
    }
    size_t o_ncomb = 0, o_np = 0, o_best = 0, o_chi2 = 0, o_par = 0, o_hi = 0, o_ntr = 0, o_co = 0;
    if (stage_out) {
        o_ncomb = off; off = align_up(off + b_ncomb, 256);
        o_np = off; off = align_up(off + b_np, 256);
        o_best = off; off = align_up(off + b_best, 256);
        o_chi2 = off; off = align_up(off + b_chi2, 256);
        o_par = off; off = align_up(off + b_par, 256);
        o_hi = off; off = align_up(off + b_hi, 256);
        o_ntr = off; off = align_up(off + b_ntr, 256);
        o_co = off; off = align_up(off + b_co, 256);
    }
    if (res->comb_offsets) {
        svt_status r = ensure(c, s.scan, svt::comb_offsets_scratch_bytes(nr));
        if (r != SVT_OK) return r;
    }
    if (off) {
        svt_status r = stage_acquire(c, s.stage, off);
        if (r != SVT_OK) return r;
    }
    // the staging buffer goes back to the pool unless the request is
    // submitted; once something is enqueued, only after the stream is idle
    auto guard = svt::make_submit_guard([st] { (void)hipStreamSynchronize(st); },
                                        [c, &s] { stage_release(c, s.stage); });
    char *base = static_cast<char *>(s.stage.ptr);

    svt::FitArgs a;
    memset(&a, 0, sizeof a);
    a.n_events = ne;
    a.n_roads = nr;
    a.n_hits = nh;
    a.n_sectors = c->n_sectors;
    a.coef = c->coef;
    a.offset = c->offset;
    a.cut_d = (double)c->cut;

    // a request that is the kernel alone is timed by its dispatch (no event
    // packets of its own on the stream); copies or the offsets scan need
    // events around the whole request
    const bool kernel_only = !stage_in && !stage_out && res->comb_offsets == nullptr;
    const int32_t every = c->timing_every;
    const bool timed = every == 1 || (every > 1 && c->next_ticket % every == 0);
    guard.enqueuing();
    if (!kernel_only && timed) HIP_TRY(hipEventRecord(s.ev_start, st));
    if (stage_in) {
        const hipMemcpyKind k = hipMemcpyHostToDevice;
        HIP_TRY(hipMemcpyAsync(base + o_ro, b->road_offsets, b_ro, k, st));
        if (nr) {
            HIP_TRY(hipMemcpyAsync(base + o_sec, b->sector, b_sec, k, st));
            HIP_TRY(hipMemcpyAsync(base + o_nh, b->nhits, b_nh, k, st));
            HIP_TRY(hipMemcpyAsync(base + o_ho, b->hit_offsets, b_ho, k, st));
            HIP_TRY(hipMemcpyAsync(base + o_xft, b->xft, b_xft, k, st));
        }
        if (nh) HIP_TRY(hipMemcpyAsync(base + o_hits, b->hits, b_hits, k, st));
        a.road_offsets = reinterpret_cast<const int32_t *>(base + o_ro);
        a.sector = reinterpret_cast<const uint8_t *>(base + o_sec);
        a.nhits4 = reinterpret_cast<const uint32_t *>(base + o_nh);
        a.hit_offsets = reinterpret_cast<const int32_t *>(base + o_ho);
        a.hits = reinterpret_cast<const int16_t *>(base + o_hits);
        a.xft2 = reinterpret_cast<const uint32_t *>(base + o_xft);
    } else {
        a.road_offsets = static_cast<const int32_t *>(device_view(b->road_offsets, b->mem_kind));
        a.sector = static_cast<const uint8_t *>(device_view(b->sector, b->mem_kind));
        a.nhits4 = static_cast<const uint32_t *>(device_view(b->nhits, b->mem_kind));
        a.hit_offsets = static_cast<const int32_t *>(device_view(b->hit_offsets, b->mem_kind));
        a.hits = static_cast<const int16_t *>(device_view(b->hits, b->mem_kind));
        a.xft2 = static_cast<const uint32_t *>(device_view(b->xft, b->mem_kind));
    }
    int64_t *co_dev = nullptr;
    if (stage_out) {
        a.ncomb = reinterpret_cast<int32_t *>(base + o_ncomb);
        a.npass = reinterpret_cast<int32_t *>(base + o_np);
        a.best = reinterpret_cast<int32_t *>(base + o_best);
        a.chi2 = reinterpret_cast<uint64_t *>(base + o_chi2);
        a.params = reinterpret_cast<int32_t *>(base + o_par);
        a.hit_index4 = reinterpret_cast<uint32_t *>(base + o_hi);
        a.ntracks = reinterpret_cast<int32_t *>(base + o_ntr);
        co_dev = res->comb_offsets ? reinterpret_cast<int64_t *>(base + o_co) : nullptr;
    } else {
        const int32_t k = res->mem_kind;
        a.ncomb = static_cast<int32_t *>(const_cast<void *>(device_view(res->ncomb, k)));
        a.npass = static_cast<int32_t *>(const_cast<void *>(device_view(res->npass, k)));
        a.best = static_cast<int32_t *>(const_cast<void *>(device_view(res->best, k)));
        a.chi2 = static_cast<uint64_t *>(const_cast<void *>(device_view(res->chi2, k)));
        a.params = static_cast<int32_t *>(const_cast<void *>(device_view(res->params, k)));
        a.hit_index4 = static_cast<uint32_t *>(const_cast<void *>(device_view(res->hit_index, k)));
        a.ntracks = static_cast<int32_t *>(const_cast<void *>(device_view(res->ntracks, k)));
        co_dev = static_cast<int64_t *>(const_cast<void *>(device_view(res->comb_offsets, k)));
    }

    const LaunchShape ls = launch_shape(c, c->tuning, ne, nr, nh, false);
    const int64_t grid = ls.grid;
    a.schedule = c->tuning.schedule;
    a.partials = static_cast<svt::BlockPartial *>(
        const_cast<void *>(device_view(s.partials, SVT_MEM_MAPPED)));
    a.seq = (uint32_t)c->next_ticket;
    s.grid = (int)grid;
    s.parts = s.partials;
    s.plan = nullptr;
    s.ring = nullptr;

    // a kernel-only request: the dispatch itself records the events (only
    // the completion when untimed)
    hipError_t e = kernel_only ? launch_shaped(c, a, ls, st, timed ? s.ev_start : nullptr, s.ev_end)
                               : launch_shaped(c, a, ls, st);
    if (e != hipSuccess) return hip_fail(e, "fit kernel launch");
    if (co_dev) {
        e = svt::launch_comb_offsets(a.ncomb, co_dev, nr, static_cast<int64_t *>(s.scan.ptr), st);
        if (e != hipSuccess) return hip_fail(e, "comb_offsets launch");
    }
    if (stage_out) {
        const hipMemcpyKind k = hipMemcpyDeviceToHost;
        if (nr) {
            HIP_TRY(hipMemcpyAsync(res->ncomb, a.ncomb, b_ncomb, k, st));
            HIP_TRY(hipMemcpyAsync(res->npass, a.npass, b_np, k, st));
            HIP_TRY(hipMemcpyAsync(res->best, a.best, b_best, k, st));
            HIP_TRY(hipMemcpyAsync(res->chi2, a.chi2, b_chi2, k, st));
            HIP_TRY(hipMemcpyAsync(res->params, a.params, b_par, k, st));
            HIP_TRY(hipMemcpyAsync(res->hit_index, a.hit_index4, b_hi, k, st));
        }
        if (ne) HIP_TRY(hipMemcpyAsync(res->ntracks, a.ntracks, b_ntr, k, st));
        if (co_dev) HIP_TRY(hipMemcpyAsync(res->comb_offsets, co_dev, b_co, k, st));
    }
    if (!kernel_only) HIP_TRY(hipEventRecord(s.ev_end, st));
    guard.submitted();
    s.timed = timed;
    s.busy = true;
    s.ticket = c->next_ticket++;
    *ticket = s.ticket;
    return SVT_OK;
}

}  // extern "C"

namespace {

// Both list entry points: with fixed == NULL the running sums go to the
// slot's scratch (allocated or grown here); otherwise to `fixed`, which
// holds at least list_scratch_bytes(n_roads) (no allocation at all).
svt_status list_submit(svt_ctx *c, const svt_event_batch *b, const int32_t *npass,
                       const svt_pass_list *list, void *hip_stream, svt_ticket *ticket,
                       int64_t *fixed)
{
    if (c == nullptr || b == nullptr || list == nullptr || ticket == nullptr) return SVT_E_INVAL;
    const int32_t nr = b->n_roads, nh = b->n_hits;
    if (b->mem_kind != SVT_MEM_DEVICE || nr < 0 || nh < 0 || nr == INT32_MAX) return SVT_E_INVAL;
    if (nr == 0 && nh != 0) return SVT_E_INVAL;
    if (nr > 0 && (b->sector == nullptr || b->nhits == nullptr || b->hit_offsets == nullptr ||
                   b->xft == nullptr || npass == nullptr))
        return SVT_E_INVAL;
    if (nh > 0 && b->hits == nullptr) return SVT_E_INVAL;
    if ((reinterpret_cast<uintptr_t>(b->nhits) | reinterpret_cast<uintptr_t>(b->xft)) & 3u)
        return SVT_E_INVAL;
    if (list->offsets == nullptr || list->capacity < 0) return SVT_E_INVAL;
    if (list->capacity > 0 && (list->k == nullptr || list->chi2 == nullptr || list->params == nullptr))
        return SVT_E_INVAL;
    if (!c->loaded) return SVT_E_STATE;
    const int si = (int)(c->next_ticket % kSlots);
    Slot &s = c->slots[si];
    if (s.busy) return SVT_E_AGAIN;
    DeviceGuard g(c->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream
    int64_t *scan = fixed;
    if (scan == nullptr) {
        const svt_status r = ensure(c, s.scan, svt::list_scratch_bytes(nr));
        if (r != SVT_OK) return r;
        scan = static_cast<int64_t *>(s.scan.ptr);
    }

    svt::ListArgs a;
    memset(&a, 0, sizeof a);
    a.sector = b->sector;
    a.nhits4 = reinterpret_cast<const uint32_t *>(b->nhits);
    a.hit_offsets = b->hit_offsets;
    a.hits = b->hits;
    a.xft2 = reinterpret_cast<const uint32_t *>(b->xft);
    a.npass = npass;
    a.offsets = list->offsets;
    a.n_roads = nr;
    a.n_hits = nh;
    a.n_sectors = c->n_sectors;
    a.cst = static_cast<const double *>(c->cst_block);
    a.cut = c->cut;
    a.k = list->k;
    a.chi2 = list->chi2;
    a.params = list->params;
    a.capacity = list->capacity;
    a.partials = static_cast<svt::BlockPartial *>(
        const_cast<void *>(device_view(s.partials, SVT_MEM_MAPPED)));
    a.seq = (uint32_t)c->next_ticket;
    // one block per tile of svt::kListTile roads, at most the partials' capacity
    int64_t grid = ((int64_t)nr + svt::kListTile - 1) / svt::kListTile;
    if (grid > c->max_grid) grid = c->max_grid;
    if (grid < 1) grid = 1;

    // nothing to give back on failure, but the scan scratch and the partials
    // stay with this slot until enqueued work is done
    auto guard = svt::make_submit_guard([st] { (void)hipStreamSynchronize(st); }, [] {});
    guard.enqueuing();
    HIP_TRY(hipEventRecord(s.ev_start, st));
    hipError_t e = svt::launch_list(a, (int)grid, scan, st);
    if (e != hipSuccess) return hip_fail(e, "list kernel launch");
    HIP_TRY(hipEventRecord(s.ev_end, st));
    guard.submitted();
    s.grid = (int)grid;
    s.parts = s.partials;
    s.plan = nullptr;
    s.ring = nullptr;
    s.list_capacity = list->capacity;
    s.busy = true;
    s.ticket = c->next_ticket++;
    *ticket = s.ticket;
    return SVT_OK;
}

}  // namespace

extern "C" {

svt_status svt_list_passing(svt_ctx *c, const svt_event_batch *b, const int32_t *npass,
                            const svt_pass_list *list, void *hip_stream, svt_ticket *ticket)
{
    return list_submit(c, b, npass, list, hip_stream, ticket, nullptr);
}

svt_status svt_list_passing_noalloc(svt_ctx *c, const svt_event_batch *b, const int32_t *npass,
                                    const svt_pass_list *list, void *hip_stream, svt_ticket *ticket)
{
    if (c == nullptr || b == nullptr) return SVT_E_INVAL;
    if (b->n_roads > kNoAllocRoads) {
        g_last_error = "svt_list_passing_noalloc: more than 2^24 roads (its scratch holds the "
                       "running sums of at most 2^24 roads)";
        return SVT_E_NOMEM;
    }
    int64_t *p = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_dev[c->device] : nullptr;
    if (p == nullptr) {
        g_last_error = "svt_list_passing_noalloc: no scratch on this device";
        return SVT_E_STATE;
    }
    return list_submit(c, b, npass, list, hip_stream, ticket, p);
}

svt_status svt_unpack_stream(svt_ctx *c, const uint32_t *words, int64_t n_words, int32_t mem_kind,
                             const svt_unpack_out *out, void *hip_stream, svt_ticket *ticket)
{
    if (c == nullptr || out == nullptr || ticket == nullptr || !kind_ok(mem_kind)) return SVT_E_INVAL;
    if (n_words < 0 || (n_words > 0 && words == nullptr)) return SVT_E_INVAL;
    if (n_words > svt::unpack_max_words()) return SVT_E_INVAL;
    if (out->max_events < 0 || out->max_roads < 0 || out->max_hits < 0) return SVT_E_INVAL;
    if (out->road_offsets == nullptr || out->hit_offsets == nullptr) return SVT_E_INVAL;
    if (out->max_roads > 0 && (out->sector == nullptr || out->nhits == nullptr || out->xft == nullptr))
        return SVT_E_INVAL;
    if (out->max_hits > 0 && out->hits == nullptr) return SVT_E_INVAL;
    if ((reinterpret_cast<uintptr_t>(out->nhits) | reinterpret_cast<uintptr_t>(out->xft)) & 3u)
        return SVT_E_INVAL;
    const int si = (int)(c->next_ticket % kSlots);
    Slot &s = c->slots[si];
    if (s.busy) return SVT_E_AGAIN;
    DeviceGuard g(c->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream

    // staging: the tile sums, then the words when they are not in device memory
    const bool in_device = mem_kind == SVT_MEM_DEVICE;
    const size_t b_tiles = align_up(svt::unpack_scratch_bytes(n_words), 256);
    const size_t need = b_tiles + (in_device ? 0 : align_up(4 * (size_t)n_words, 256));
    svt_status r = stage_acquire(c, s.stage, need);
    if (r != SVT_OK) return r;
    auto guard = svt::make_submit_guard([st] { (void)hipStreamSynchronize(st); },
                                        [c, &s] { stage_release(c, s.stage); });
    char *base = static_cast<char *>(s.stage.ptr);

    svt::UnpackArgs a;
    memset(&a, 0, sizeof a);
    a.n_words = n_words;
    a.tiles = reinterpret_cast<svt::UnpackAgg *>(base);
    uint32_t *dev_words = in_device ? const_cast<uint32_t *>(words)
                                    : reinterpret_cast<uint32_t *>(base + b_tiles);
    a.words = dev_words;
    a.src = dev_words;
    a.copy = 0;
    a.road_offsets = out->road_offsets;
    a.sector = out->sector;
    a.nhits4 = reinterpret_cast<uint32_t *>(out->nhits);
    a.hit_offsets = out->hit_offsets;
    a.hits = out->hits;
    a.xft2 = reinterpret_cast<uint32_t *>(out->xft);
    a.max_events = out->max_events;
    a.max_roads = out->max_roads;
    a.max_hits = out->max_hits;
    a.n_apply = svt::unpack_apply_blocks(n_words, c->max_grid);
    a.partials = static_cast<svt::BlockPartial *>(
        const_cast<void *>(device_view(s.partials, SVT_MEM_MAPPED)));
    a.seq = (uint32_t)c->next_ticket;

    guard.enqueuing();
    HIP_TRY(hipEventRecord(s.ev_start, st));
    if (mem_kind == SVT_MEM_MAPPED) {
        // zero copy: the first pass reads the host words in place and leaves
        // a device copy for the others
        a.src = static_cast<const uint32_t *>(device_view(words, mem_kind));
        a.copy = 1;
    } else if (!in_device && n_words > 0) {
        HIP_TRY(hipMemcpyAsync(dev_words, words, 4 * (size_t)n_words, hipMemcpyHostToDevice, st));
    }
    // host-mapped words are read four bytes per lane: 16-byte reads over
    // the bus were slower
    a.src_vec = a.copy == 0 && (reinterpret_cast<uintptr_t>(a.src) & 15u) == 0;
    a.words_vec = (reinterpret_cast<uintptr_t>(a.words) & 15u) == 0;
    hipError_t e = svt::launch_unpack(a, st);
    if (e != hipSuccess) return hip_fail(e, "unpack launch");
    HIP_TRY(hipEventRecord(s.ev_end, st));
    guard.submitted();
    s.grid = a.n_apply + 1;
    s.parts = s.partials;
    s.plan = nullptr;
    s.ring = nullptr;
    s.unpack = true;
    s.unpack_cap[0] = out->max_events;
    s.unpack_cap[1] = out->max_roads;
    s.unpack_cap[2] = out->max_hits;
    s.busy = true;
    s.ticket = c->next_ticket++;
    *ticket = s.ticket;
    return SVT_OK;
}

svt_status svt_result(svt_ctx *c, svt_ticket t, int32_t wait_us, svt_summary *out)
{
    if (c == nullptr || t <= 0) return SVT_E_INVAL;
    Slot &s = c->slots[t % kSlots];
    if (!s.busy || s.ticket != t) return SVT_E_INVAL;
    DeviceGuard g(c->device);
    if (wait_us < 0) {
        HIP_TRY(hipEventSynchronize(s.ev_end));
    } else {
        const auto t0 = std::chrono::steady_clock::now();
        for (;;) {
            hipError_t q = hipEventQuery(s.ev_end);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) return hip_fail(q, "hipEventQuery");
            const auto dt = std::chrono::duration_cast<std::chrono::microseconds>(
                                std::chrono::steady_clock::now() - t0)
                                .count();
            if (dt >= wait_us) return SVT_E_AGAIN;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    // reduce the blocks' partial sums
    uint64_t comb = 0, pass = 0;
    uint32_t trk = 0, er = 0xFFFFFFFFu, ee = 0xFFFFFFFFu;
    bool complete = true;
    for (int b = 0; b < s.grid; ++b) {
        const svt::BlockPartial p = s.parts[b];
        complete = complete && p.seq == (s.ring ? s.ring_seq : (uint32_t)t);
        comb += p.comb;
        pass += p.pass;
        trk += p.tracks;
        er = p.err_road < er ? p.err_road : er;
        ee = p.err_event < ee ? p.err_event : ee;
    }
    svt_status status = SVT_OK;
    if (!complete) {
        g_last_error = "fit kernel did not report every block";
        status = SVT_E_DEVICE;
    } else if (er != 0xFFFFFFFFu || ee != 0xFFFFFFFFu) {
        status = SVT_E_RANGE;
    } else if (s.list_capacity >= 0 && (int64_t)pass > s.list_capacity) {
        status = SVT_E_RANGE;   // the list did not fit
    } else if (s.unpack && ((int64_t)trk > s.unpack_cap[0] || (int64_t)comb > s.unpack_cap[1] ||
                            (int64_t)pass > s.unpack_cap[2])) {
        status = SVT_E_RANGE;   // the batch did not fit
    }
    if (out) {
        memset(out, 0, sizeof *out);
        out->total_comb = (int64_t)comb;
        out->total_pass = (int64_t)pass;
        out->total_tracks = (int32_t)trk;
        out->err_road = er == 0xFFFFFFFFu ? -1 : (int32_t)er;
        out->err_event = ee == 0xFFFFFFFFu ? -1 : (int32_t)ee;
        out->status = status;
        float ms = 0.f;
        if (!s.timed)
            out->device_ns = 0;
        else if (hipEventElapsedTime(&ms, s.ev_start, s.ev_end) == hipSuccess)
            out->device_ns = (int64_t)((double)ms * 1e6);
        else
            (void)hipGetLastError();
    }
    if (s.plan) s.plan->busy = false;
    s.plan = nullptr;
    if (s.ring) s.ring->busy = false;
    s.ring = nullptr;
    stage_release(c, s.stage);
    s.list_capacity = -1;
    s.unpack = false;
    s.timed = true;
    s.busy = false;
    s.ticket = -1;
    return status;
}

// ---------------------------------------------------------------------------
// float shadow
// ---------------------------------------------------------------------------
static bool shadow_ok(const svt_shadow_tracks *t)
{
    return t && t->n_tracks >= 0 && t->n_sectors >= 1 && t->n_sectors <= 256 &&
           t->sector_offsets && (t->n_tracks == 0 || (t->x && t->tau));
}

svt_status svt_shadow_slices(int32_t n_tracks, int32_t n_sectors, int32_t *slices)
{
    if (slices == nullptr || n_tracks < 0 || n_sectors < 1 || n_sectors > 256) return SVT_E_INVAL;
    *slices = svt::shadow_slices(n_tracks, n_sectors);
    return SVT_OK;
}

svt_status svt_shadow_forward(svt_ctx *c, const svt_shadow_tracks *t, const float *coef,
                              const float *offset, float *y, double *loss, void *hip_stream)
{
    if (c == nullptr || !shadow_ok(t) || coef == nullptr || offset == nullptr || loss == nullptr)
        return SVT_E_INVAL;
    DeviceGuard g(c->device);
    svt_status r = ensure(c, c->shadow_scratch, svt::shadow_scratch_bytes(t->n_tracks, t->n_sectors));
    if (r != SVT_OK) return r;
    svt::ShadowCall sc{t->x, t->tau, t->sector_offsets, t->n_tracks, t->n_sectors,
                       {t->w[0], t->w[1], t->w[2]}, coef, offset, y, loss,
                       nullptr, nullptr, nullptr, nullptr};
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream
    hipError_t e = svt::launch_shadow_forward(sc, static_cast<double *>(c->shadow_scratch.ptr), st);
    return e == hipSuccess ? SVT_OK : hip_fail(e, "shadow forward launch");
}

svt_status svt_shadow_backward(svt_ctx *c, const svt_shadow_tracks *t, const float *coef,
                               const float *offset, const double *scale, double *grad_coef,
                               double *grad_offset, float *grad_coef_f32, float *grad_offset_f32,
                               void *hip_stream)
{
    if (c == nullptr || !shadow_ok(t) || coef == nullptr || offset == nullptr ||
        grad_coef == nullptr || grad_offset == nullptr)
        return SVT_E_INVAL;
    DeviceGuard g(c->device);
    svt_status r = ensure(c, c->shadow_scratch, svt::shadow_scratch_bytes(t->n_tracks, t->n_sectors));
    if (r != SVT_OK) return r;
    svt::ShadowCall sc{t->x, t->tau, t->sector_offsets, t->n_tracks, t->n_sectors,
                       {t->w[0], t->w[1], t->w[2]}, coef, offset, nullptr, nullptr,
                       grad_coef, grad_offset, grad_coef_f32, grad_offset_f32};
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream
    hipError_t e = svt::launch_shadow_backward(sc, scale, static_cast<double *>(c->shadow_scratch.ptr), st);
    return e == hipSuccess ? SVT_OK : hip_fail(e, "shadow backward launch");
}

svt_status svt_shadow_penalty(svt_ctx *c, int32_t n_sectors, const float *coef, double lambda,
                              double *value, double *grad_coef, float *grad_coef_f32,
                              void *hip_stream)
{
    if (c == nullptr || n_sectors < 1 || n_sectors > 256 || coef == nullptr || value == nullptr ||
        grad_coef == nullptr)
        return SVT_E_INVAL;
    DeviceGuard g(c->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream
    hipError_t e = svt::launch_shadow_penalty(coef, n_sectors, lambda, value, grad_coef, grad_coef_f32, st);
    return e == hipSuccess ? SVT_OK : hip_fail(e, "shadow penalty launch");
}

svt_status svt_shadow_adam(svt_ctx *c, int32_t n, float *param, const double *grad, float *m,
                           float *v, float lr, float beta1, float beta2, float eps, int32_t step,
                           void *hip_stream)
{
    if (c == nullptr || n < 0 || step < 1 || (n > 0 && (!param || !grad || !m || !v)))
        return SVT_E_INVAL;
    if (n == 0) return SVT_OK;
    DeviceGuard g(c->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream
    hipError_t e = svt::launch_adam(n, param, grad, m, v, lr, beta1, beta2, eps, step, st);
    return e == hipSuccess ? SVT_OK : hip_fail(e, "adam launch");
}

svt_status svt_requantize(svt_ctx *c, int32_t n_sectors, const float *coef, const float *offset,
                          int32_t max_abs, int32_t *coef_int, int32_t *offset_int, int32_t *shift,
                          int32_t *status, void *hip_stream)
{
    if (c == nullptr || n_sectors < 1 || n_sectors > 256 || !coef || !offset || !coef_int ||
        !offset_int || !shift || !status || max_abs < 1)
        return SVT_E_INVAL;
    DeviceGuard g(c->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream
    hipError_t e = svt::launch_requantize(coef, offset, n_sectors, max_abs, coef_int, offset_int,
                                          shift, status, st);
    return e == hipSuccess ? SVT_OK : hip_fail(e, "requantize launch");
}

// ---------------------------------------------------------------------------
// plans: one persistent, graph-captured fit of any batch within a capacity
// ---------------------------------------------------------------------------
static void plan_free(svt_plan *p)
{
    if (p == nullptr) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->buf) dev_free(p->ctx, p->buf, p->buf_bytes);
    if (p->sizes_host) (void)hipHostFree(p->sizes_host);
    if (p->partials) (void)hipHostFree(p->partials);
    delete p;
}

svt_status svt_plan_create(svt_ctx *c, int32_t max_events, int32_t max_roads, int32_t max_hits,
                           const svt_tuning *tuning, svt_plan **out)
{
    if (c == nullptr || out == nullptr || max_events < 1 || max_roads < 0 || max_hits < 0 ||
        max_events == INT32_MAX || max_roads == INT32_MAX)
        return SVT_E_INVAL;
    *out = nullptr;
    if (!c->loaded) return SVT_E_STATE;
    DeviceGuard g(c->device);
    svt_plan *p = new (std::nothrow) svt_plan();
    if (p == nullptr) return SVT_E_NOMEM;
    p->ctx = c;
    p->max_events = max_events;
    p->max_roads = max_roads;
    p->max_hits = max_hits;
    p->tuning = c->tuning;
    if (tuning) {
        if (tuning->events_per_chunk < 0 || tuning->events_per_chunk > svt::kMaxEventsPerChunk ||
            tuning->blocks_per_cu < 0 || tuning->blocks_per_cu > svt::kMaxBlocksPerCu ||
            tuning->schedule < 0 || tuning->schedule > 3 || tuning->kernel < 0 ||
            tuning->kernel > 1) {
            delete p;
            return SVT_E_INVAL;
        }
        if (tuning->events_per_chunk) p->tuning.events_per_chunk = tuning->events_per_chunk;
        if (tuning->blocks_per_cu) p->tuning.blocks_per_cu = tuning->blocks_per_cu;
        if (tuning->schedule) p->tuning.schedule = tuning->schedule;
        p->tuning.kernel = tuning->kernel;
    }
    const LaunchShape ls = launch_shape(c, p->tuning, max_events, max_roads, max_hits, true);
    p->const_gen = c->const_gen;

    // buffer layout: inputs, then results, then the size descriptor
    const size_t ne = (size_t)max_events, nr = (size_t)max_roads, nh = (size_t)max_hits;
    size_t off = 0;
    const size_t o_ro = off; off = align_up(off + 4 * (ne + 1), 256);
    const size_t o_sec = off; off = align_up(off + nr, 256);
    const size_t o_nh = off; off = align_up(off + 4 * nr, 256);
    const size_t o_ho = off; off = align_up(off + 4 * (nr + 1), 256);
    const size_t o_hits = off; off = align_up(off + 2 * nh, 256);
    const size_t o_xft = off; off = align_up(off + 4 * nr, 256);
    const size_t o_ncomb = off; off = align_up(off + 4 * nr, 256);
    const size_t o_np = off; off = align_up(off + 4 * nr, 256);
    const size_t o_best = off; off = align_up(off + 4 * nr, 256);
    const size_t o_chi2 = off; off = align_up(off + 8 * nr, 256);
    const size_t o_par = off; off = align_up(off + 12 * nr, 256);
    const size_t o_hi = off; off = align_up(off + 4 * nr, 256);
    const size_t o_ntr = off; off = align_up(off + 4 * ne, 256);
    svt_status st = dev_alloc(c, &p->buf, off);
    if (st != SVT_OK) {
        delete p;
        return st;
    }
    p->buf_bytes = off;
    char *base = static_cast<char *>(p->buf);
    p->in = svt_event_batch{0, 0, 0, SVT_MEM_DEVICE,
                            reinterpret_cast<const int32_t *>(base + o_ro),
                            reinterpret_cast<const uint8_t *>(base + o_sec),
                            reinterpret_cast<const uint8_t *>(base + o_nh),
                            reinterpret_cast<const int32_t *>(base + o_ho),
                            reinterpret_cast<const int16_t *>(base + o_hits),
                            reinterpret_cast<const int16_t *>(base + o_xft)};
    p->out = svt_results{reinterpret_cast<int32_t *>(base + o_ncomb),
                         reinterpret_cast<int32_t *>(base + o_np),
                         reinterpret_cast<int32_t *>(base + o_best),
                         reinterpret_cast<uint64_t *>(base + o_chi2),
                         reinterpret_cast<int32_t *>(base + o_par),
                         reinterpret_cast<uint8_t *>(base + o_hi),
                         reinterpret_cast<int32_t *>(base + o_ntr), nullptr, SVT_MEM_DEVICE, 0};
    p->grid = ls.grid;
    if (hipHostMalloc(reinterpret_cast<void **>(&p->sizes_host), sizeof(svt::Sizes),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&p->partials),
                      sizeof(svt::BlockPartial) * p->grid,
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        st = hip_fail(hipGetLastError(), "hipHostMalloc");
        plan_free(p);
        return st;
    }
    memset(p->sizes_host, 0, sizeof(svt::Sizes));
    p->sizes_dev = static_cast<const svt::Sizes *>(device_view(p->sizes_host, SVT_MEM_MAPPED));
    memset(p->partials, 0, sizeof(svt::BlockPartial) * p->grid);

    svt::FitArgs a;
    memset(&a, 0, sizeof a);
    a.road_offsets = p->in.road_offsets;
    a.sector = p->in.sector;
    a.nhits4 = reinterpret_cast<const uint32_t *>(p->in.nhits);
    a.hit_offsets = p->in.hit_offsets;
    a.hits = p->in.hits;
    a.xft2 = reinterpret_cast<const uint32_t *>(p->in.xft);
    a.sizes = p->sizes_dev;
    a.n_sectors = c->n_sectors;
    a.coef = c->coef;
    a.offset = c->offset;
    a.cut_d = (double)c->cut;
    a.ncomb = p->out.ncomb;
    a.npass = p->out.npass;
    a.best = p->out.best;
    a.chi2 = p->out.chi2;
    a.params = p->out.params;
    a.hit_index4 = reinterpret_cast<uint32_t *>(p->out.hit_index);
    a.ntracks = p->out.ntracks;
    a.schedule = p->tuning.schedule;
    a.partials = static_cast<svt::BlockPartial *>(const_cast<void *>(device_view(p->partials, SVT_MEM_MAPPED)));

    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = launch_shaped(c, a, ls, cs);
        e = hipStreamEndCapture(cs, &p->graph);
        if (e == hipSuccess && e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    // uploaded now, so that the first run does not pay for it
    if (e == hipSuccess) e = hipGraphUpload(p->exec, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        st = hip_fail(e, "plan capture");
        plan_free(p);
        return st;
    }
    *out = p;
    return SVT_OK;
}

svt_status svt_plan_destroy(svt_plan *p)
{
    if (p == nullptr) return SVT_E_INVAL;
    DeviceGuard g(p->ctx->device);
    if (p->busy) {
        for (int i = 0; i < kSlots; ++i) {
            Slot &s = p->ctx->slots[i];
            if (s.busy && s.plan == p) {
                (void)hipEventSynchronize(s.ev_end);
                s.plan = nullptr;
                s.busy = false;
            }
        }
    }
    plan_free(p);
    return SVT_OK;
}

svt_status svt_plan_buffers(svt_plan *p, svt_event_batch *in, svt_results *out)
{
    if (p == nullptr) return SVT_E_INVAL;
    if (in) {
        *in = p->in;
        in->n_events = p->max_events;
        in->n_roads = p->max_roads;
        in->n_hits = p->max_hits;
    }
    if (out) *out = p->out;
    return SVT_OK;
}

svt_status svt_plan_fit(svt_plan *p, const svt_event_batch *b, const svt_results *res,
                        void *hip_stream, svt_ticket *ticket)
{
    if (p == nullptr || b == nullptr || res == nullptr || ticket == nullptr) return SVT_E_INVAL;
    svt_ctx *c = p->ctx;
    const svt_status vs = check_call(b, res);
    if (vs != SVT_OK) return vs;
    const int32_t ne = b->n_events, nr = b->n_roads, nh = b->n_hits;
    if (ne > p->max_events || nr > p->max_roads || nh > p->max_hits) return SVT_E_INVAL;
    if (res->comb_offsets && res->mem_kind != SVT_MEM_DEVICE) return SVT_E_INVAL;
    if (!c->loaded || c->const_gen != p->const_gen) return SVT_E_STATE;
    if (p->busy) return SVT_E_AGAIN;
    const int si = (int)(c->next_ticket % kSlots);
    Slot &s = c->slots[si];
    if (s.busy) return SVT_E_AGAIN;
    DeviceGuard g(c->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream
    if (res->comb_offsets) {
        svt_status r = ensure(c, s.scan, svt::comb_offsets_scratch_bytes(nr));
        if (r != SVT_OK) return r;
    }

    const int32_t every = c->timing_every;
    const bool timed = every == 1 || (every > 1 && c->next_ticket % every == 0);
    // the plan's buffers and partials stay unused until enqueued work is done
    auto guard = svt::make_submit_guard([st] { (void)hipStreamSynchronize(st); }, [] {});
    guard.enqueuing();
    if (timed) HIP_TRY(hipEventRecord(s.ev_start, st));
    // inputs into the plan's buffers (skipped when the caller filled them in place)
    const void *src[6] = {b->road_offsets, b->sector, b->nhits, b->hit_offsets, b->hits, b->xft};
    const void *dst[6] = {p->in.road_offsets, p->in.sector, p->in.nhits, p->in.hit_offsets,
                          p->in.hits, p->in.xft};
    const size_t bytes[6] = {4 * ((size_t)ne + 1), (size_t)nr, 4 * (size_t)nr,
                             4 * ((size_t)nr + 1), 2 * (size_t)nh, 4 * (size_t)nr};
    for (int i = 0; i < 6; ++i)
        if (bytes[i] && src[i] != dst[i])
            HIP_TRY(hipMemcpyAsync(const_cast<void *>(dst[i]), src[i], bytes[i], hipMemcpyDefault, st));
    p->sizes_host->n_events = ne;
    p->sizes_host->n_roads = nr;
    p->sizes_host->n_hits = nh;
    p->sizes_host->seq = (uint32_t)c->next_ticket;
    HIP_TRY(hipGraphLaunch(p->exec, st));
    if (res->comb_offsets) {
        hipError_t e = svt::launch_comb_offsets(p->out.ncomb, res->comb_offsets, nr,
                                                static_cast<int64_t *>(s.scan.ptr), st);
        if (e != hipSuccess) return hip_fail(e, "comb_offsets launch");
    }
    // results out of the plan's buffers (skipped when the caller reads them in place)
    const void *rs[7] = {p->out.ncomb, p->out.npass, p->out.best, p->out.chi2, p->out.params,
                         p->out.hit_index, p->out.ntracks};
    void *rd[7] = {res->ncomb, res->npass, res->best, res->chi2, res->params, res->hit_index,
                   res->ntracks};
    const size_t rb[7] = {4 * (size_t)nr, 4 * (size_t)nr, 4 * (size_t)nr, 8 * (size_t)nr,
                          12 * (size_t)nr, 4 * (size_t)nr, 4 * (size_t)ne};
    for (int i = 0; i < 7; ++i)
        if (rb[i] && rd[i] != rs[i]) HIP_TRY(hipMemcpyAsync(rd[i], rs[i], rb[i], hipMemcpyDefault, st));
    HIP_TRY(hipEventRecord(s.ev_end, st));
    guard.submitted();
    s.timed = timed;
    s.busy = true;
    s.ticket = c->next_ticket++;
    s.parts = p->partials;
    s.grid = p->grid;
    s.plan = p;
    s.ring = nullptr;
    p->busy = true;
    *ticket = s.ticket;
    return SVT_OK;
}

// ---------------------------------------------------------------------------
// rings: captured back-to-back fit passes over resident batches
// ---------------------------------------------------------------------------
static void ring_free(svt_ring *r)
{
    if (r == nullptr) return;
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    if (r->seq_dev) dev_free(r->ctx, r->seq_dev, 256);
    if (r->args_dev) dev_free(r->ctx, r->args_dev, r->args_bytes);
    if (r->parts_dev) dev_free(r->ctx, r->parts_dev, sizeof(svt::BlockPartial) * r->total_parts);
    if (r->mid_dev) dev_free(r->ctx, r->mid_dev, sizeof(svt::BlockPartial) * svt::kPartialRedBlocks);
    if (r->summary) (void)hipHostFree(r->summary);
    delete r;
}

svt_status svt_ring_create(svt_ctx *c, int32_t n_batches, const svt_event_batch *batches,
                           const svt_results *results, int32_t n_passes, int32_t passes_per_launch,
                           svt_ring **out)
{
    if (c == nullptr || out == nullptr || batches == nullptr || results == nullptr)
        return SVT_E_INVAL;
    *out = nullptr;
    if (n_passes < 1 || n_passes > 1024 || n_batches < 1 || n_batches > n_passes ||
        passes_per_launch < 0 || passes_per_launch > 128)
        return SVT_E_INVAL;
    for (int i = 0; i < n_batches; ++i) {
        const svt_status vs = check_call(&batches[i], &results[i]);
        if (vs != SVT_OK) return vs;
        if (batches[i].mem_kind != SVT_MEM_DEVICE || results[i].mem_kind != SVT_MEM_DEVICE ||
            results[i].comb_offsets != nullptr)
            return SVT_E_INVAL;
    }
    if (!c->loaded) return SVT_E_STATE;
    DeviceGuard g(c->device);
    svt_ring *r = new (std::nothrow) svt_ring();
    if (r == nullptr) return SVT_E_NOMEM;
    r->ctx = c;
    r->n_batches = n_batches;
    r->n_passes = n_passes;
    r->const_gen = c->const_gen;
    // passes per launch: several batches per launch (by default up to 128,
    // the passes split evenly over the launches) spread the launch's start
    // and its last blocks over many batches (3000 events x 64 roads, a ring
    // of 100 passes: 8.51 us per pass at 25 per launch, 8.40 at 50, 8.33 at
    // 100)
    int k = passes_per_launch;
    if (k == 0) {
        const int launches = (n_passes + 127) / 128;
        k = (n_passes + launches - 1) / launches;
    }
    if (k < 1) k = 1;
    if (k > n_passes) k = n_passes;
    r->per_launch = k;
    // chunks of a multi-pass launch: three times a lone pass's (three full
    // sub-chunks of 256 roads per block on the 3000 x 64-road batch) when the
    // launch still has at least two blocks per grid slot, since the blocks of
    // its other passes fill the grid; each block's start-up is then shared by
    // three sub-chunks (back to back: 8.30 us per pass with 4 events per
    // chunk, 7.84 with 8, 7.73 with 12 or 16, 7.81 with 32, 8.59 with 6,
    // whose 384 roads leave a half-empty sub-chunk; a 20-pass launch: 8.87
    // against 8.68 us per pass with 12)
    std::vector<LaunchShape> small(n_batches), shapes(n_batches);
    const int64_t slots = (int64_t)c->cu_count * 5;
    for (int i = 0; i < n_batches; ++i) {
        const svt_event_batch &b = batches[i];
        small[i] = shapes[i] = launch_shape(c, c->tuning, b.n_events, b.n_roads, b.n_hits, false);
        const int64_t chunks = b.n_events > 0 ? ((int64_t)b.n_events + small[i].epc - 1) / small[i].epc : 0;
        if (k > 1 && (int64_t)k * chunks >= 2 * 3 * slots)
            shapes[i] = launch_shape(c, c->tuning, b.n_events, b.n_roads, b.n_hits, false, 3);
    }
    // A launch's last blocks run on an emptying grid, so when its chunks
    // are the larger ones its last passes keep the lone pass's chunks
    // (shorter blocks): as many passes as fill the grid's slots once, at
    // most a quarter of the launch's passes.  Each launch of the block
    // kernel gives every batch of its head the same number of blocks (the
    // largest grid of those passes) and every batch of its tail the tail's
    // largest grid; block partials pass by pass.
    bool larger = false;
    for (int i = 0; i < n_batches; ++i) larger = larger || small[i].epc != shapes[i].epc;
    const int n_launch = (n_passes + k - 1) / k;
    std::vector<int> launch_per(n_launch, 1), tail_per(n_launch, 1), n_tail(n_launch, 0),
        part_off(n_passes + 1, 0);
    std::vector<char> in_tail(n_passes, 0);
    for (int l = 0; l < n_launch; ++l) {
        const int p0 = l * k, np = (p0 + k <= n_passes) ? k : n_passes - p0;
        int m = 0;
        int64_t cover = 0;
        while (larger && m < np / 4 && cover < slots) {
            cover += small[(p0 + np - 1 - m) % n_batches].grid;
            ++m;
        }
        n_tail[l] = m;
        for (int p = p0; p < p0 + np; ++p) {
            const bool t = p >= p0 + np - m;
            in_tail[p] = t ? 1 : 0;
            const int gp = t ? small[p % n_batches].grid : shapes[p % n_batches].grid;
            int &per = t ? tail_per[l] : launch_per[l];
            per = gp > per ? gp : per;
        }
    }
    for (int p = 0; p < n_passes; ++p)
        part_off[p + 1] = part_off[p] + (k > 1 ? (in_tail[p] ? tail_per[p / k] : launch_per[p / k])
                                               : shapes[p % n_batches].grid);
    r->total_parts = part_off[n_passes];
    // the blocks' partials stay in device memory and are reduced there (by
    // the last node of the graph) into one host-mapped summary
    svt_status st = dev_alloc(c, reinterpret_cast<void **>(&r->seq_dev), 256);
    if (st != SVT_OK) {
        delete r;
        return st;
    }
    // (before any capture: the first run's sequence number and the counter)
    if (hipMemset(r->seq_dev, 0, 256) != hipSuccess) {
        st = hip_fail(hipGetLastError(), "hipMemset");
        ring_free(r);
        return st;
    }
    st = dev_alloc(c, reinterpret_cast<void **>(&r->parts_dev),
                   sizeof(svt::BlockPartial) * r->total_parts);
    if (st == SVT_OK)
        st = dev_alloc(c, reinterpret_cast<void **>(&r->mid_dev),
                       sizeof(svt::BlockPartial) * svt::kPartialRedBlocks);
    if (st != SVT_OK) {
        ring_free(r);
        return st;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&r->summary), sizeof(svt::BlockPartial),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        st = hip_fail(hipGetLastError(), "hipHostMalloc");
        ring_free(r);
        return st;
    }
    memset(r->summary, 0, sizeof(svt::BlockPartial));
    r->summary->seq = 0xFFFFFFFFu;   // no run's number until a run writes it
    svt::BlockPartial *parts_dev = r->parts_dev;
    svt::BlockPartial *summary_dev = static_cast<svt::BlockPartial *>(
        const_cast<void *>(device_view(r->summary, SVT_MEM_MAPPED)));

    // the launch arguments of every pass
    std::vector<svt::FitArgs> args(n_passes);
    for (int p = 0; p < n_passes; ++p) {
        const svt_event_batch &b = batches[p % n_batches];
        const svt_results &res = results[p % n_batches];
        svt::FitArgs &a = args[p];
        memset(&a, 0, sizeof a);
        a.road_offsets = b.road_offsets;
        a.sector = b.sector;
        a.nhits4 = reinterpret_cast<const uint32_t *>(b.nhits);
        a.hit_offsets = b.hit_offsets;
        a.hits = b.hits;
        a.xft2 = reinterpret_cast<const uint32_t *>(b.xft);
        a.n_events = b.n_events;
        a.n_roads = b.n_roads;
        a.n_hits = b.n_hits;
        a.n_sectors = c->n_sectors;
        a.coef = c->coef;
        a.offset = c->offset;
        a.cut_d = (double)c->cut;
        a.ncomb = res.ncomb;
        a.npass = res.npass;
        a.best = res.best;
        a.chi2 = res.chi2;
        a.params = res.params;
        a.hit_index4 = reinterpret_cast<uint32_t *>(res.hit_index);
        a.ntracks = res.ntracks;
        a.schedule = c->tuning.schedule;
        a.partials = parts_dev + part_off[p];
        a.seq_dev = r->seq_dev;
        set_shape_args(c, a, in_tail[p] ? small[p % n_batches] : shapes[p % n_batches]);
    }
    if (k > 1) {
        r->args_bytes = sizeof(svt::FitArgs) * (size_t)n_passes;
        st = dev_alloc(c, reinterpret_cast<void **>(&r->args_dev), r->args_bytes);
        if (st == SVT_OK && hipMemcpy(r->args_dev, args.data(), r->args_bytes,
                                      hipMemcpyHostToDevice) != hipSuccess)
            st = hip_fail(hipGetLastError(), "ring arguments");
        if (st != SVT_OK) {
            ring_free(r);
            return st;
        }
    }

    r->summary_dev = summary_dev;
    for (int l = 0; l < n_launch; ++l) {
        const int p0 = l * k, np = (p0 + k <= n_passes) ? k : n_passes - p0;
        r->launches.push_back({p0, np - n_tail[l], k > 1 ? launch_per[l] : shapes[p0 % n_batches].grid,
                               n_tail[l], tail_per[l]});
    }
    if (n_launch <= kRingDirectMax) {
        r->direct = true;
        if (k == 1) r->args_host = args;
        *out = r;
        return SVT_OK;
    }
    // the graph: the launches in order, then the reduction of their partials
    // (which also advances the sequence number the next run's blocks read)
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = hipSuccess;
        for (int l = 0; l < n_launch && e2 == hipSuccess; ++l) {
            const int p0 = l * k, np = (p0 + k <= n_passes) ? k : n_passes - p0;
            if (k > 1)
                e2 = svt::launch_fit_multi(r->args_dev + p0, np - n_tail[l], launch_per[l], n_tail[l],
                                           tail_per[l], cs);
            else
                e2 = launch_shaped(c, args[p0], shapes[p0 % n_batches], cs);
        }
        if (e2 == hipSuccess)
            e2 = svt::launch_reduce_partials(parts_dev, r->total_parts, r->mid_dev, summary_dev,
                                             r->seq_dev, r->seq_dev + kRingCounter, cs);
        e = hipStreamEndCapture(cs, &r->graph);
        if (e == hipSuccess && e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0);
    // uploaded now, so that the first run does not pay for it
    if (e == hipSuccess) e = hipGraphUpload(r->exec, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        st = hip_fail(e, "ring capture");
        ring_free(r);
        return st;
    }
    *out = r;
    return SVT_OK;
}

svt_status svt_ring_run(svt_ring *r, void *hip_stream, svt_ticket *ticket)
{
    if (r == nullptr || ticket == nullptr) return SVT_E_INVAL;
    svt_ctx *c = r->ctx;
    if (!c->loaded || c->const_gen != r->const_gen) return SVT_E_STATE;
    if (r->busy) return SVT_E_AGAIN;
    const int si = (int)(c->next_ticket % kSlots);
    Slot &s = c->slots[si];
    if (s.busy) return SVT_E_AGAIN;
    DeviceGuard g(c->device);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);  // NULL: the null stream
    auto guard = svt::make_submit_guard([st] { (void)hipStreamSynchronize(st); }, [] {});
    guard.enqueuing();
    HIP_TRY(hipEventRecord(s.ev_start, st));
    if (r->direct) {
        // the same kernels, in the same order, as a captured ring's graph
        for (const svt_ring::Launch &l : r->launches) {
            if (r->per_launch > 1)
                HIP_TRY(svt::launch_fit_multi(r->args_dev + l.p0, l.np, l.grid, l.n_tail, l.tail_grid, st));
            else
                HIP_TRY(svt::launch_fit(r->args_host[l.p0], l.grid, st));
        }
        HIP_TRY(svt::launch_reduce_partials(r->parts_dev, r->total_parts, r->mid_dev, r->summary_dev,
                                            r->seq_dev, r->seq_dev + kRingCounter, st));
    } else {
        HIP_TRY(hipGraphLaunch(r->exec, st));
    }
    // the run's last kernel advances the device's sequence number, so the
    // host's count follows every run that was enqueued
    const uint32_t run_seq = r->runs++;
    HIP_TRY(hipEventRecord(s.ev_end, st));
    guard.submitted();
    s.timed = true;
    s.busy = true;
    s.ticket = c->next_ticket++;
    s.parts = r->summary;   // the graph reduced the blocks' partials into it
    s.grid = 1;
    s.ring_seq = run_seq;
    s.plan = nullptr;
    s.ring = r;
    r->busy = true;
    *ticket = s.ticket;
    return SVT_OK;
}

svt_status svt_ring_info(const svt_ring *r, int32_t *n_passes, int32_t *passes_per_launch,
                         int32_t *n_launches)
{
    if (r == nullptr) return SVT_E_INVAL;
    if (n_passes) *n_passes = r->n_passes;
    if (passes_per_launch) *passes_per_launch = r->per_launch;
    if (n_launches) *n_launches = (r->n_passes + r->per_launch - 1) / r->per_launch;
    return SVT_OK;
}

svt_status svt_ring_destroy(svt_ring *r)
{
    if (r == nullptr) return SVT_E_INVAL;
    DeviceGuard g(r->ctx->device);
    if (r->busy) {
        for (int i = 0; i < kSlots; ++i) {
            Slot &s = r->ctx->slots[i];
            if (s.busy && s.ring == r) {
                (void)hipEventSynchronize(s.ev_end);
                s.ring = nullptr;
                s.busy = false;
            }
        }
    }
    ring_free(r);
    return SVT_OK;
}

// ---------------------------------------------------------------------------
// I/O probe
// ---------------------------------------------------------------------------
svt_status svt_io_probe(svt_ctx *c, int32_t kind, int32_t direction, size_t bytes, int32_t reps,
                        double *median_us)
{
    if (c == nullptr || median_us == nullptr || reps < 1 || bytes == 0 ||
        (direction != 0 && direction != 1) ||
        (kind != SVT_MEM_PAGEABLE && kind != SVT_MEM_PINNED && kind != SVT_MEM_MAPPED))
        return SVT_E_INVAL;
    DeviceGuard g(c->device);
    void *dev = nullptr;
    svt_status st = dev_alloc(c, &dev, bytes);
    if (st != SVT_OK) return st;
    void *host = nullptr;
    hipError_t e = hipSuccess;
    if (kind == SVT_MEM_PAGEABLE) {
        host = malloc(bytes);
        if (host == nullptr) {
            dev_free(c, dev, bytes);
            return SVT_E_NOMEM;
        }
    } else {
        e = hipHostMalloc(&host, bytes,
                          kind == SVT_MEM_MAPPED ? (hipHostMallocMapped | hipHostMallocCoherent)
                                                 : hipHostMallocDefault);
        if (e != hipSuccess) {
            dev_free(c, dev, bytes);
            return hip_fail(e, "hipHostMalloc");
        }
    }
    memset(host, 1, bytes);
    std::vector<double> t;
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const void *hview = kind == SVT_MEM_MAPPED ? device_view(host, SVT_MEM_MAPPED) : host;
    for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {
        e = hipEventRecord(a, c->stream);
        if (e != hipSuccess) break;
        if (kind == SVT_MEM_MAPPED)
            e = direction == 0 ? svt::launch_zero_copy(hview, dev, bytes, c->cu_count, c->stream)
                               : svt::launch_zero_copy(dev, const_cast<void *>(hview), bytes,
                                                       c->cu_count, c->stream);
        else
            e = direction == 0 ? hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c->stream)
                               : hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) break;
        e = hipEventRecord(b, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && r > 0) t.push_back((double)ms * 1e3);   // first one warms up
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (kind == SVT_MEM_PAGEABLE) free(host); else (void)hipHostFree(host);
    dev_free(c, dev, bytes);
    if (e != hipSuccess) return hip_fail(e, "io probe");
    std::sort(t.begin(), t.end());
    *median_us = t[t.size() / 2];
    return SVT_OK;
}

}  // extern "C"
