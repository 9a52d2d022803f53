// C-ABI host layer of the melded kernel library: argument checks, plans,
// scratch and launches. Every compute step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/meld.h"
#include "kernels.h"
#include "tune.h"

using meld::SortArray;

struct meld_ctx {
    int device = 0;
    // Tail workspace backing the virtual padding of non-power-of-two sorts.
    uint32_t *tail = nullptr;
    size_t tail_words = 0;
    // Segmented sort: queue state, per-segment class and queue, and the
    // per-workgroup padding scratch of the persistent grid.
    meld::SegState *seg_state = nullptr;
    uint8_t *seg_cls = nullptr;
    uint32_t *seg_queue = nullptr;
    size_t seg_cap = 0;  // segments the two arrays above hold
    uint32_t *seg_work = nullptr;
    uint32_t seg_grid = 0;
    // Captured segmented-sort sequences (reset, classify, plan, scatter,
    // persistent sort), most recently used first, replayed on the caller's
    // stream. A graph bakes in its arguments, hence the key.
    struct SegGraph {
        const void *keys;
        const void *offsets;
        size_t nseg;
        uint32_t n_keys;
        bool lo, hi, xch;
        hipGraphExec_t exec;
    };
    std::list<SegGraph> seg_graphs;
    hipStream_t capture_stream = nullptr;
    bool use_graphs = true;
    uint32_t sort_log_tile = 0;  // 0: chosen per call
    // Phases k <= 64 of the sorts: -1 the library's choice (lane exchanges
    // under a fixed form, timed under MELD_AUTO), 0 the LDS comparator
    // network, 1 registers with DPP lane exchanges.
    int lane_exchange = -1;
    // Tuner: decisions per shape class, scratch for timed trials on copies of
    // the caller's data, and device counters for the divergence probes.
    meld::Tuner tuner;
    uint32_t *tune_buf = nullptr;
    // Merge sort: the other buffer of each merge pass.
    uint32_t *merge_buf = nullptr;
    size_t merge_words = 0;
    uint32_t *merge_cuts = nullptr;  // merge-path cut of every tile of a merge pass
    size_t merge_cut_words = 0;
    size_t tune_words = 0;
    unsigned long long *probe_buf = nullptr;  // kProbeWords counters
    double theta = 0.5;  // mixed-wave fraction from which the probe favours melding
    double tie = 0.02;   // trials within 2 % count as ties
};

namespace {
constexpr size_t kProbeWords = 64;
// Sorts whose array (padded, keys and payloads) exceeds this many bytes use
// nontemporal global accesses.
constexpr size_t kNontemporalBytes = (size_t)256 << 20;
// Tie window of the sort tuner's second round (relative): the spread of the
// medians of five or nine timed local-sort launches on one MI355X.
constexpr double kFinalTie = 0.005;

// Scratch of meld_sort_u32_noalloc: the padding of a non-power-of-two sort,
// in a device array of the library itself, so that the call allocates
// nothing. Every device holds its own copy until the process ends; host code
// reaches a device's copy only through the address hipGetSymbolAddress gives
// for it (the array's name is not a device address in host code).
constexpr size_t kNoAllocWords = MELD_NOALLOC_SCRATCH_WORDS;
__device__ __align__(256) uint32_t scratch[kNoAllocWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxDevices] = {};

// Looks up device `device`'s copy of the scratch array once; the device must
// be current.
hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device] != nullptr) return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<uint32_t *>(ptr);
    return hipSuccess;
}

uint32_t *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

namespace {

thread_local std::string g_err;

meld_status fail(meld_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

meld_status hip_fail(hipError_t e, const char *what) {
    return fail(MELD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// A device pointer on the context's device (or managed memory).
bool is_device_ptr(const meld_ctx *ctx, const void *p) {
    if (p == nullptr) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return false;
    return attr.device == ctx->device;
}

uint32_t log2_ceil(uint64_t n) {
    uint32_t l = 0;
    while ((1ull << l) < n) ++l;
    return l;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            (void)hipSetDevice(dev);
        } else {
            prev = -1;
        }
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

meld_status ensure_tail(meld_ctx *ctx, size_t words) {
    if (words <= ctx->tail_words) return MELD_OK;
    if (ctx->tail != nullptr) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(ctx->tail);
        ctx->tail = nullptr;
        ctx->tail_words = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, words * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MELD_ENOMEM, "cannot allocate %zu bytes of sort scratch", words * 4);
    }
    ctx->tail = static_cast<uint32_t *>(p);
    ctx->tail_words = words;
    return MELD_OK;
}

bool use_melded(meld_variant v) { return v != MELD_DIVERGENT; }

meld_status dev_alloc(void **p, size_t bytes, const char *what) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(MELD_ENOMEM, "cannot allocate %zu bytes of %s", bytes, what);
    }
    return MELD_OK;
}

meld_status ensure_words(uint32_t **buf, size_t *have, size_t words, const char *what) {
    if (words <= *have) return MELD_OK;
    if (*buf != nullptr) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(*buf);
        *buf = nullptr;
        *have = 0;
    }
    meld_status st = dev_alloc(reinterpret_cast<void **>(buf), words * sizeof(uint32_t), what);
    if (st == MELD_OK) *have = words;
    return st;
}

meld_status ensure_probe(meld_ctx *ctx) {
    if (ctx->probe_buf != nullptr) return MELD_OK;
    return dev_alloc(reinterpret_cast<void **>(&ctx->probe_buf),
                     kProbeWords * sizeof(unsigned long long), "probe counters");
}

// Runs a probe launcher on zeroed counters and copies `count` of them back.
template <class Launch>
meld_status run_probe(meld_ctx *ctx, hipStream_t s, size_t count, unsigned long long *host,
                      Launch launch) {
    meld_status st = ensure_probe(ctx);
    if (st != MELD_OK) return st;
    hipError_t e = meld::launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->probe_buf), 0u,
                                         kProbeWords * 2, s);
    if (e == hipSuccess) e = launch(ctx->probe_buf);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host, ctx->probe_buf, count * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "divergence probe");
    return MELD_OK;
}

// Median milliseconds of `reps` runs of run() on stream s, each preceded by
// an untimed prep().
template <class Prep, class Run>
meld_status time_median(hipStream_t s, int reps, Prep prep, Run run, double *ms_out) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return fail(MELD_EHIP, "hipEventCreate failed");
    }
    std::vector<float> t;
    meld_status st = MELD_OK;
    for (int r = 0; r < reps && st == MELD_OK; ++r) {
        st = prep();
        if (st != MELD_OK) break;
        (void)hipEventRecord(a, s);
        st = run();
        (void)hipEventRecord(b, s);
        if (st != MELD_OK) break;
        if (hipEventSynchronize(b) != hipSuccess) {
            st = fail(MELD_EHIP, "hipEventSynchronize failed");
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != MELD_OK) return st;
    std::sort(t.begin(), t.end());
    *ms_out = t.empty() ? 0.0 : t[t.size() / 2];
    return MELD_OK;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

std::string fmt(const char *f, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

constexpr size_t kMaxSegGraphs = 8;

void drop_seg_graphs(meld_ctx *ctx) {
    for (auto &g : ctx->seg_graphs) (void)hipGraphExecDestroy(g.exec);
    ctx->seg_graphs.clear();
}

// Scratch of the segmented sort for up to nseg segments.
meld_status ensure_seg(meld_ctx *ctx, size_t nseg) {
    if (ctx->seg_state == nullptr) {
        hipError_t e = meld::seg_sort_grid(ctx->device, &ctx->seg_grid);
        if (e != hipSuccess) return hip_fail(e, "segmented sort occupancy query");
        meld_status st = dev_alloc(reinterpret_cast<void **>(&ctx->seg_state),
                                   sizeof(meld::SegState), "segmented sort state");
        if (st != MELD_OK) return st;
        if (hipMemset(ctx->seg_state, 0, sizeof(meld::SegState)) != hipSuccess)
            return fail(MELD_EHIP, "hipMemset of segmented sort state failed");
        st = dev_alloc(reinterpret_cast<void **>(&ctx->seg_work),
                       (size_t)ctx->seg_grid * meld::kSegWorkWords * sizeof(uint32_t),
                       "segmented sort staging");
        if (st != MELD_OK) return st;
    }
    if (nseg > ctx->seg_cap) {
        if (ctx->seg_cls != nullptr || ctx->seg_queue != nullptr) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
            // Every captured graph holds the old arrays' addresses: none may
            // be replayed after they are freed, whichever caller grows them.
            drop_seg_graphs(ctx);
            (void)hipFree(ctx->seg_cls);
            (void)hipFree(ctx->seg_queue);
            ctx->seg_cls = nullptr;
            ctx->seg_queue = nullptr;
            ctx->seg_cap = 0;
        }
        meld_status st = dev_alloc(reinterpret_cast<void **>(&ctx->seg_cls), nseg, "segment classes");
        if (st != MELD_OK) return st;
        st = dev_alloc(reinterpret_cast<void **>(&ctx->seg_queue), nseg * sizeof(uint32_t),
                       "segment queue");
        if (st != MELD_OK) return st;
        ctx->seg_cap = nseg;
    }
    return MELD_OK;
}

// The graph of (keys, n_keys, offsets, nseg, forms), captured on first use.
meld_status seg_graph(meld_ctx *ctx, uint32_t *keys, uint32_t n_keys, const uint32_t *offsets,
                      size_t nseg, bool lo, bool hi, bool xch, hipGraphExec_t *out) {
    for (auto it = ctx->seg_graphs.begin(); it != ctx->seg_graphs.end(); ++it) {
        if (it->keys == keys && it->n_keys == n_keys && it->offsets == offsets &&
            it->nseg == nseg && it->lo == lo && it->hi == hi && it->xch == xch) {
            ctx->seg_graphs.splice(ctx->seg_graphs.begin(), ctx->seg_graphs, it);
            *out = it->exec;
            return MELD_OK;
        }
    }
    if (ctx->capture_stream == nullptr) {
        hipError_t e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    hipError_t e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = meld::launch_segmented_sort(keys, n_keys, offsets, (uint32_t)nseg,
                                                ctx->seg_state, ctx->seg_cls, ctx->seg_queue,
                                                ctx->seg_work, ctx->seg_grid, lo, hi, xch,
                                                ctx->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph != nullptr) (void)hipGraphDestroy(graph);
        return hip_fail(le != hipSuccess ? le : e, "capturing the segmented sort");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (ctx->seg_graphs.size() >= kMaxSegGraphs) {
        (void)hipGraphExecDestroy(ctx->seg_graphs.back().exec);
        ctx->seg_graphs.pop_back();
    }
    ctx->seg_graphs.push_front({keys, offsets, nseg, n_keys, lo, hi, xch, exec});
    *out = exec;
    return MELD_OK;
}

// Offsets are u32, so any key count of 2^32 - 1 or more bounds every offset.
uint32_t key_bound(size_t n_keys) {
    return n_keys >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)n_keys;
}

meld_status segmented_impl(meld_ctx *ctx, uint32_t *keys, size_t n_keys, const uint32_t *offsets,
                           size_t nseg, bool meld_lo, bool meld_hi, bool xch, hipStream_t stream,
                           const char *fn) {
    if (nseg == 0) return MELD_OK;
    if (nseg >= (1ull << 31)) return fail(MELD_EINVAL, "%s: nseg = %zu >= 2^31", fn, nseg);
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, keys) || !is_device_ptr(ctx, offsets))
        return fail(MELD_EINVAL, "%s: keys and offsets must be device pointers on device %d", fn,
                    ctx->device);
    meld_status st = ensure_seg(ctx, nseg);  // drops the graphs if the scratch moves
    if (st != MELD_OK) return st;
    // A caller that is itself capturing gets the launches in its own graph.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (!ctx->use_graphs || cs != hipStreamCaptureStatusNone) {
        e = meld::launch_segmented_sort(keys, key_bound(n_keys), offsets, (uint32_t)nseg,
                                        ctx->seg_state, ctx->seg_cls, ctx->seg_queue,
                                        ctx->seg_work, ctx->seg_grid, meld_lo, meld_hi, xch,
                                        stream);
        if (e != hipSuccess) return hip_fail(e, "segmented sort launch");
        return MELD_OK;
    }
    hipGraphExec_t exec = nullptr;
    st = seg_graph(ctx, keys, key_bound(n_keys), offsets, nseg, meld_lo, meld_hi, xch, &exec);
    if (st != MELD_OK) return st;
    e = hipGraphLaunch(exec, stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return MELD_OK;
}

// Threads per workgroup of the LDS-only tile kernel (tiles below 2^8): one
// comparator per lane per iteration.
int tile_threads(uint32_t log_t) {
    if (log_t <= 7) return 64;
    if (log_t <= 9) return 256;
    return 512;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// How a single-array sort runs: the tile size and the form per stage.
struct SortPlan {
    uint32_t log_t;
    bool lo, hi;
    bool xch;  // phases k <= 64 in registers with lane exchanges
};

constexpr uint32_t kMinLogRegsTile = 8;  // smallest tile of the register-window kernels

uint32_t max_log_tile(bool pairs) { return pairs ? meld::kMaxLogTilePairs : meld::kMaxLogTileKeys; }

// Tile size without timing, from a sweep of 2^14 .. 2^28 elements on
// gfx950: 2^11 while the array is small (more tiles spread over the chip
// and one tile's sort stays short), larger tiles (fewer streaming passes)
// from 2^20 elements on.
uint32_t default_log_tile(bool pairs, uint32_t log_n) {
    uint32_t t;
    if (log_n <= 19)
        t = 11;
    else if (log_n <= 21)
        t = 12;
    else
        t = pairs ? (log_n <= 25 ? 12 : 13) : 14;
    return std::max(kMinLogRegsTile, std::min(t, max_log_tile(pairs)));
}

// Sizes (high bits first) of the streaming passes of d global steps: the
// fewest passes of at most max_gather steps, as equal as possible (a gathered
// pass of 8 pair steps has rows of only 128 bytes and runs slower than one of
// 7, so 14 steps go as 7 + 7 rather than 8 + 6).
std::vector<uint32_t> split_passes(uint32_t d, uint32_t max_gather) {
    const uint32_t n = (d + max_gather - 1) / max_gather;
    std::vector<uint32_t> sizes;
    uint32_t left = d;
    for (uint32_t p = 0; p < n; ++p) {
        const uint32_t r = (left + (n - p) - 1) / (n - p);
        sizes.push_back(r);
        left -= r;
    }
    return sizes;
}

// Pair sorts: launch time of a streaming pass over 2^28 pairs on one MI355X
// (microseconds; median of four sorts in one process; gathered passes in
// XCD runs), by kind, steps r and lowest array bit b_lo (column b_lo - 13;
// the rows of the pass lie 2^b_lo elements apart). The time depends on where
// the pass sits, not only on its size: passes whose steps span array bits
// 19 .. 24 (rows 2 .. 64 MiB apart) run up to 70 % slower than the same pass
// on bits from 13 up. Only the ratios matter. Zero: not measured
// (b_lo + r > 28); the lookup clamps b_lo into the measured columns.
constexpr uint16_t kPairRegsUs[7][15] = {
    {0},
    {644, 636, 650, 651, 639, 647, 662, 675, 675, 720, 711, 690, 660, 663, 672},
    {652, 657, 674, 672, 675, 669, 706, 735, 779, 866, 784, 668, 680, 708, 0},
    {671, 679, 698, 698, 692, 702, 733, 786, 851, 917, 728, 702, 725, 0, 0},
    {690, 707, 724, 724, 732, 755, 784, 840, 864, 767, 728, 737, 0, 0, 0},
    {720, 736, 742, 736, 768, 847, 860, 849, 783, 766, 754, 0, 0, 0, 0},
    {724, 737, 748, 763, 801, 908, 958, 800, 796, 776, 0, 0, 0, 0, 0},
};
constexpr uint16_t kPairGatherUs[9][15] = {
    {0}, {0}, {0}, {0}, {0},
    {659, 673, 736, 725, 763, 869, 818, 1108, 764, 711, 750, 0, 0, 0, 0},
    {651, 728, 780, 813, 850, 736, 747, 930, 754, 753, 0, 0, 0, 0, 0},
    {714, 727, 736, 735, 730, 729, 736, 775, 778, 0, 0, 0, 0, 0, 0},
    {740, 790, 851, 855, 866, 842, 936, 1006, 0, 0, 0, 0, 0, 0, 0},
};

double pair_pass_us(bool gather, uint32_t r, uint32_t b_lo) {
    const uint32_t hi = 28 - r;  // last measured b_lo for this r
    const uint32_t col = std::min(std::max(b_lo, 13u), hi) - 13;
    return gather ? kPairGatherUs[r][col] : kPairRegsUs[r][col];
}

struct PassSplit {
    uint32_t r;   // steps of the pass
    bool gather;  // through a gathered LDS tile (else registers)
};

// The streaming passes (high bits first) of the d global pair steps on array
// bits log_t .. log_t + d - 1, of least total time under the tables; the
// first pass of the x lowest steps (r of them) has b_lo = log_t + x - r.
// Gathered passes only where gather_ok.
std::vector<PassSplit> split_passes_pairs(uint32_t d, uint32_t log_t, bool gather_ok) {
    std::vector<double> best(d + 1, 1e300);
    std::vector<PassSplit> first(d + 1, PassSplit{0, false});
    best[0] = 0.0;
    for (uint32_t x = 1; x <= d; ++x) {
        for (uint32_t r = 1; r <= std::min(x, meld::kMaxFusedSteps); ++r) {
            const double c = best[x - r] + pair_pass_us(false, r, log_t + x - r);
            if (c < best[x]) {
                best[x] = c;
                first[x] = PassSplit{r, false};
            }
        }
        if (!gather_ok) continue;
        for (uint32_t r = meld::kMinGatherStepsPairs; r <= std::min(x, meld::kMaxGatherStepsPairs);
             ++r) {
            const double c = best[x - r] + pair_pass_us(true, r, log_t + x - r);
            if (c < best[x]) {
                best[x] = c;
                first[x] = PassSplit{r, true};
            }
        }
    }
    std::vector<PassSplit> out;
    for (uint32_t x = d; x > 0; x -= first[x].r) out.push_back(first[x]);
    return out;
}

// One launch of a single-array sort.
enum class PassKind { kTile, kLocal, kRegs, kGather, kMerge };
struct SortPass {
    PassKind kind;
    uint32_t m;           // phase 2^m (kRegs, kGather, kMerge)
    uint32_t b_hi, b_lo;  // steps j = 2^b_hi .. 2^b_lo (kRegs, kGather)
    uint32_t steps;       // network steps the launch runs
};

const char *pass_name(PassKind k) {
    switch (k) {
        case PassKind::kTile: return "tile";
        case PassKind::kLocal: return "local";
        case PassKind::kRegs: return "regs";
        case PassKind::kGather: return "gather";
        default: return "merge";
    }
}

// The launches of the whole network of N = 2^log_n elements under a plan
// (log_n > plan.log_t: local sort of every tile, then per phase 2^m above the
// tile its streaming passes and its merge tail; otherwise a single tile).
std::vector<SortPass> sort_passes(const SortPlan &plan, bool pairs, uint32_t log_n) {
    std::vector<SortPass> out;
    if (log_n <= plan.log_t) {
        const uint32_t log_t = std::max<uint32_t>(log_n, 1);
        out.push_back({PassKind::kTile, 0, 0, 0, log_t * (log_t + 1) / 2});
        return out;
    }
    const uint32_t log_t = plan.log_t;
    out.push_back({PassKind::kLocal, 0, 0, 0, log_t * (log_t + 1) / 2});
    const uint32_t max_gather = pairs ? meld::kMaxGatherStepsPairs : meld::kMaxGatherStepsKeys;
    const uint32_t gather_log = pairs ? meld::kGatherLogPairs : meld::kGatherLogKeys;
    for (uint32_t m = log_t + 1; m <= log_n; ++m) {
        // Steps j = 2^(m-1) .. 2^log_t stream through HBM in as few passes as
        // possible: up to kMaxFusedSteps per pass in registers, more (high
        // bits first) through gathered LDS tiles where their rows fit.
        uint32_t b_hi = m - 1;
        std::vector<PassSplit> sizes;
        if (pairs) {
            sizes = split_passes_pairs(m - log_t, log_t, log_n >= gather_log);
        } else {
            for (uint32_t r : split_passes(m - log_t, max_gather))
                sizes.push_back(PassSplit{r, r > meld::kMaxFusedSteps});
        }
        for (const PassSplit &ps : sizes) {
            const uint32_t r = ps.r;
            const uint32_t b_lo = b_hi + 1 - r;
            const bool gather_fits = log_n >= gather_log && b_lo + r >= gather_log;
            if (ps.gather && gather_fits) {
                out.push_back({PassKind::kGather, m, b_hi, b_lo, r});
            } else {
                // register passes only (balanced)
                const uint32_t parts = (r + meld::kMaxFusedSteps - 1) / meld::kMaxFusedSteps;
                uint32_t hi = b_hi;
                for (uint32_t p = 0; p < parts; ++p) {
                    const uint32_t remaining = hi - b_lo + 1;
                    const uint32_t this_r = (remaining + (parts - p) - 1) / (parts - p);
                    out.push_back({PassKind::kRegs, m, hi, hi + 1 - this_r, this_r});
                    hi -= this_r;
                }
            }
            b_hi = b_lo - 1;
        }
        // Steps j = 2^(log_t-1) .. 1 of phase m: the direction is uniform per
        // tile, both forms coincide; registers with LDS transposes.
        out.push_back({PassKind::kMerge, m, 0, 0, log_t});
    }
    return out;
}

// Enqueues the whole network (or its first step_limit steps) on keys[0..n).
// marks: NULL, or one event per launch plus one, recorded on the stream
// before the first launch (and the tail fill) and after every launch.
// fixed_tail: NULL (the context's tail workspace, grown on demand), or device
// memory of fixed_tail_words words that holds the padding instead (nothing is
// allocated; MELD_EINVAL if it is too small).
meld_status sort_impl(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                      const SortPlan &plan, int64_t step_limit, hipStream_t stream,
                      const std::vector<hipEvent_t> *marks = nullptr,
                      uint32_t *fixed_tail = nullptr, size_t fixed_tail_words = 0) {
    const bool pairs = payload != nullptr;
    const uint32_t log_n = log2_ceil(n);
    const size_t big_n = (size_t)1 << log_n;

    // Nontemporal accesses once the array outgrows the caches (L2 and the
    // 256 MB Infinity Cache); below, the array stays cached between launches.
    const bool nt = big_n * (pairs ? 8 : 4) > kNontemporalBytes;
    SortArray a{keys, payload, nullptr, nullptr, (uint32_t)n, nt ? 1u : 0u};
    int64_t left = step_limit;  // < 0: unlimited
    auto take = [&left](uint64_t steps) -> int32_t {
        if (left < 0) return -1;
        const int64_t s = std::min<int64_t>(left, (int64_t)steps);
        left -= s;
        return (int32_t)s;
    };

    if (log_n > plan.log_t && (plan.log_t < kMinLogRegsTile || plan.log_t > max_log_tile(pairs)))
        return fail(MELD_EINVAL, "sort: tile 2^%u outside 2^%u .. 2^%u", plan.log_t,
                    kMinLogRegsTile, max_log_tile(pairs));
    const std::vector<SortPass> passes = sort_passes(plan, pairs, log_n);
    if (marks != nullptr && marks->size() != passes.size() + 1)
        return fail(MELD_EINVAL, "sort: %zu timing events for %zu launches", marks->size(),
                    passes.size());
    auto mark = [&](size_t i) -> hipError_t {
        return marks != nullptr ? hipEventRecord((*marks)[i], stream) : hipSuccess;
    };

    hipError_t e;
    if (passes[0].kind == PassKind::kTile) {
        // One tile holds everything; positions >= n are sentinels.
        const uint32_t log_t = std::max<uint32_t>(log_n, 1);
        const int io = big_n > n ? meld::kIoSentinel
                       : (aligned16(keys) && (!pairs || aligned16(payload))) ? meld::kIoPlainVec
                                                                             : meld::kIoPlain;
        const int32_t steps = take(passes[0].steps);
        e = mark(0);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        if (log_t >= kMinLogRegsTile)
            e = meld::launch_bitonic_sort_regs(a, log_t, 1, steps, plan.lo, plan.hi, plan.xch, io,
                                               stream);
        else
            e = meld::launch_bitonic_tile(a, log_t, 1, 1, log_t, 0, steps, plan.lo, plan.hi, io,
                                          tile_threads(log_t), stream);
        if (e == hipSuccess) e = mark(1);
        if (e != hipSuccess) return hip_fail(e, "bitonic tile launch");
        return MELD_OK;
    }

    if (big_n > n) {
        const size_t pad = big_n - n;
        const size_t words = pairs ? 2 * pad : pad;
        uint32_t *tail = fixed_tail;
        if (tail == nullptr) {
            meld_status st = ensure_tail(ctx, words);
            if (st != MELD_OK) return st;
            tail = ctx->tail;
        } else if (words > fixed_tail_words) {
            return fail(MELD_EINVAL, "sort: padding of %zu words exceeds the %zu-word scratch",
                        words, fixed_tail_words);
        }
        a.tk = tail;
        a.tv = pairs ? tail + pad : nullptr;
        e = mark(0);
        if (e == hipSuccess) e = meld::launch_fill_u32(tail, 0xFFFFFFFFu, words, stream);
        if (e != hipSuccess) return hip_fail(e, "fill launch");
    } else {
        e = mark(0);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }

    const uint32_t log_t = plan.log_t;
    const uint32_t n_tiles = (uint32_t)(big_n >> log_t);
    const int io = a.tk != nullptr ? meld::kIoTail
                   : (aligned16(keys) && (!pairs || aligned16(payload))) ? meld::kIoPlainVec
                                                                         : meld::kIoPlain;
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        const SortPass &p = passes[pi];
        const int32_t steps = take(p.steps);
        switch (p.kind) {
            case PassKind::kLocal:
                e = meld::launch_bitonic_sort_regs(a, log_t, n_tiles, steps, plan.lo, plan.hi,
                                                   plan.xch, io, stream);
                break;
            case PassKind::kGather:
                e = meld::launch_bitonic_gather(a, log_n, p.m, p.b_hi, p.b_lo, steps, io, stream);
                break;
            case PassKind::kRegs:
                e = meld::launch_bitonic_global(a, log_n, p.m, p.b_hi, p.b_lo, steps, stream);
                break;
            case PassKind::kMerge:
                e = meld::launch_bitonic_merge(a, log_t, n_tiles, p.m, steps, io, stream);
                break;
            default:
                return fail(MELD_EINVAL, "sort: unexpected pass");
        }
        if (e == hipSuccess) e = mark(pi + 1);
        if (e != hipSuccess)
            return hip_fail(e, fmt("bitonic %s launch", pass_name(p.kind)).c_str());
    }
    return MELD_OK;
}

// The tile the context fixes (MELD_OPT_SORT_LOG_TILE), else the size rule.
uint32_t plan_log_tile(const meld_ctx *ctx, bool pairs, uint32_t log_n) {
    if (ctx->sort_log_tile != 0) return std::min(ctx->sort_log_tile, max_log_tile(pairs));
    return default_log_tile(pairs, log_n);
}

// Lane exchanges unless the context asks for the LDS comparator network.
bool plan_xch(const meld_ctx *ctx) { return ctx->lane_exchange != 0; }

SortPlan fixed_plan(const meld_ctx *ctx, bool pairs, size_t n, meld_variant v) {
    const bool m = use_melded(v);
    return SortPlan{plan_log_tile(ctx, pairs, log2_ceil(n)), m, m, plan_xch(ctx)};
}

// Probe of one tile's network: mixed-wave fraction of the phases k <= 64 and
// k >= 128.
meld_status probe_network(meld_ctx *ctx, uint32_t log_t, hipStream_t s, double *mixed_lo,
                          double *mixed_hi) {
    unsigned long long c[2 * 16] = {0};
    meld_status st = run_probe(ctx, s, 2 * log_t, c, [&](unsigned long long *out) {
        return meld::launch_probe_network(log_t, log_t >= kMinLogRegsTile, out, s);
    });
    if (st != MELD_OK) return st;
    unsigned long long ml = 0, al = 0, mh = 0, ah = 0;
    for (uint32_t m = 1; m <= log_t; ++m) {
        (m <= 6 ? ml : mh) += c[2 * (m - 1)];
        (m <= 6 ? al : ah) += c[2 * (m - 1) + 1];
    }
    *mixed_lo = al ? (double)ml / (double)al : 0.0;
    *mixed_hi = ah ? (double)mh / (double)ah : 0.0;
    return MELD_OK;
}

// Tuning-cache key of a sort shape class (array size class, pairs, forced
// tile, forced low-phase path).
std::string sort_tune_key(const meld_ctx *ctx, bool pairs, uint32_t log_n) {
    const uint32_t forced =
        ctx->sort_log_tile ? std::min(ctx->sort_log_tile, max_log_tile(pairs)) : 0;
    std::string k = forced ? fmt("n=%u pairs=%d t=%u", log_n, pairs ? 1 : 0, forced)
                           : fmt("n=%u pairs=%d", log_n, pairs ? 1 : 0);
    if (ctx->lane_exchange >= 0) k += fmt(" x=%d", ctx->lane_exchange);
    return k;
}

// The tuned plan of a shape class, if the tuner holds a usable one.
bool cached_sort_plan(const meld_ctx *ctx, bool pairs, uint32_t log_n, SortPlan *out) {
    if (const meld::TuneEntry *e = ctx->tuner.find("sort", sort_tune_key(ctx, pairs, log_n))) {
        const uint32_t t = (uint32_t)e->log_t;
        if (t >= kMinLogRegsTile && t <= max_log_tile(pairs)) {
            *out = SortPlan{t, e->lo != 0, e->hi != 0, e->xch != 0};
            return true;
        }
    }
    return false;
}

// MELD_AUTO for a sort: the tuned plan of this shape class, timing the
// candidates (tile size x form per stage) on a scratch copy the first time.
meld_status auto_sort_plan(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                           hipStream_t s, SortPlan *out) {
    const bool pairs = payload != nullptr;
    const uint32_t log_n = log2_ceil(n);
    const uint32_t max_t = max_log_tile(pairs);
    const uint32_t forced = ctx->sort_log_tile ? std::min(ctx->sort_log_tile, max_t) : 0;
    const std::string key = sort_tune_key(ctx, pairs, log_n);
    if (cached_sort_plan(ctx, pairs, log_n, out)) return MELD_OK;
    *out = SortPlan{plan_log_tile(ctx, pairs, log_n), true, true, plan_xch(ctx)};
    if (capturing(s)) return MELD_OK;  // no timing inside a capture; untuned default
    // Candidate tiles: from one that leaves a few hundred tiles up to the
    // largest (a single tile when everything fits); the forced one alone.
    std::vector<uint32_t> tiles;
    if (forced) {
        tiles.push_back(forced);
    } else {
        const uint32_t hi_t = std::min(max_t, std::max(log_n, kMinLogRegsTile));
        const int lo_want = std::min<int>((int)max_t - 1, (int)log_n - 10);
        const uint32_t lo_t = std::min(hi_t, (uint32_t)std::max<int>((int)kMinLogRegsTile, lo_want));
        for (uint32_t t = lo_t; t <= hi_t; ++t) tiles.push_back(t);
    }
    const size_t words = pairs ? 2 * n : n;
    meld_status st = ensure_words(&ctx->tune_buf, &ctx->tune_words, words, "tuning scratch");
    if (st != MELD_OK) return st;
    uint32_t *tk = ctx->tune_buf;
    uint32_t *tv = pairs ? ctx->tune_buf + n : nullptr;
    auto time_plan = [&](const SortPlan &p, int64_t steps, int reps, double *t) {
        return time_median(
            s, reps,
            [&]() -> meld_status {
                hipError_t e = hipMemcpyAsync(tk, keys, n * 4, hipMemcpyDeviceToDevice, s);
                if (e == hipSuccess && pairs)
                    e = hipMemcpyAsync(tv, payload, n * 4, hipMemcpyDeviceToDevice, s);
                return e == hipSuccess ? MELD_OK : hip_fail(e, "tuning copy");
            },
            [&]() { return sort_impl(ctx, tk, tv, n, p, steps, s); }, t);
    };
    // The candidates within the tie window of the fastest, timed again with
    // more runs, interleaved; returns the index of the fastest (or, within
    // `tie`, the one the probe's rule prefers) and updates ms.
    auto final_round = [&](const std::vector<SortPlan> &c, std::vector<double> &ms, int64_t steps,
                           double mixed_lo, double mixed_hi, double tie, int *pick) {
        const double best_ms = *std::min_element(ms.begin(), ms.end());
        std::vector<int> fin;
        for (int i = 0; i < (int)c.size(); ++i)
            if (ms[i] <= best_ms * (1.0 + ctx->tie)) fin.push_back(i);
        if (fin.size() > 1) {
            const int reps2 = n >= (1u << 24) ? 5 : 9;
            std::vector<std::vector<double>> runs(fin.size());
            for (int r = 0; r < reps2; ++r)
                for (size_t f = 0; f < fin.size(); ++f) {
                    double t = 0;
                    meld_status st2 = time_plan(c[fin[f]], steps, 1, &t);
                    if (st2 != MELD_OK) return st2;
                    runs[f].push_back(t);
                }
            for (size_t f = 0; f < fin.size(); ++f) {
                std::sort(runs[f].begin(), runs[f].end());
                ms[fin[f]] = runs[f][runs[f].size() / 2];
            }
        }
        std::vector<double> m2;
        std::vector<int> lo2, hi2;
        for (int i : fin) {
            m2.push_back(ms[i]);
            lo2.push_back(c[i].lo);
            hi2.push_back(c[i].hi);
        }
        *pick = fin[meld::choose((int)fin.size(), m2.data(), lo2.data(), hi2.data(), mixed_lo,
                                 mixed_hi, ctx->theta, tie)];
        return MELD_OK;
    };
    const int reps = n >= (1u << 24) ? 2 : 3;
    // Step 1, the tile: whole sorts with the default forms (the forms change
    // only the local-sort launch, a few percent of a large sort).
    std::vector<SortPlan> tplans;
    std::vector<double> tms;
    for (uint32_t t : tiles) {
        tplans.push_back(SortPlan{t, true, true, plan_xch(ctx)});
        double ms1 = 0;
        st = time_plan(tplans.back(), -1, reps, &ms1);
        if (st != MELD_OK) return st;
        tms.push_back(ms1);
    }
    int tpick = 0;
    st = final_round(tplans, tms, -1, 0.0, 0.0, 0.0, &tpick);
    if (st != MELD_OK) return st;
    const uint32_t log_t = tplans[tpick].log_t;
    const uint32_t local_log = std::max<uint32_t>(std::min(log_t, log_n), 1);
    const int64_t local_steps = (int64_t)local_log * (local_log + 1) / 2;
    // Step 2, the forms: the local-sort launch alone (the network's first
    // local_steps steps), every form per stage on each low-phase path.
    std::vector<bool> xchs;
    if (ctx->lane_exchange >= 0)
        xchs.push_back(ctx->lane_exchange != 0);
    else
        xchs = {false, true};
    std::vector<SortPlan> cands;
    std::vector<double> ms;
    for (bool x : xchs)
        for (int f = 0; f < 4; ++f) {
            cands.push_back(SortPlan{log_t, (f & 1) != 0, (f & 2) != 0, x});
            double t = 0;
            st = time_plan(cands.back(), local_steps, reps, &t);
            if (st != MELD_OK) return st;
            ms.push_back(t);
        }
    double mixed_lo = 0, mixed_hi = 0;
    st = probe_network(ctx, std::min(log_n, max_t), s, &mixed_lo, &mixed_hi);
    if (st != MELD_OK) return st;
    int pick = 0;
    st = final_round(cands, ms, local_steps, mixed_lo, mixed_hi, kFinalTie, &pick);
    if (st != MELD_OK) return st;
    *out = cands[pick];
    meld::TuneEntry e;
    e.op = "sort";
    e.key = key;
    e.lo = out->lo;
    e.hi = out->hi;
    e.log_t = (int)out->log_t;
    e.xch = out->xch ? 1 : 0;
    e.form = out->lo ? 1 : 0;
    e.ms = tms[tpick];
    e.mixed_lo = mixed_lo;
    e.mixed_hi = mixed_hi;
    e.trials = (int)(tplans.size() + cands.size());
    ctx->tuner.put(e);
    return MELD_OK;
}

// MELD_AUTO for a segmented sort: the tuned forms of this shape class, timing
// the four per-stage combinations on a scratch copy the first time.
meld_status auto_seg_forms(meld_ctx *ctx, uint32_t *keys, size_t n_keys, const uint32_t *offsets,
                           size_t nseg, hipStream_t s, bool *lo, bool *hi, bool *xch) {
    *lo = *hi = true;
    *xch = plan_xch(ctx);
    if (capturing(s)) {
        return MELD_OK;
    }
    uint32_t total = 0;
    hipError_t e = hipMemcpyAsync(&total, offsets + nseg, sizeof total, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading offsets[nseg]");
    // the trials copy keys[0 .. offsets[nseg]): never past the caller's array
    if (total > n_keys)
        return fail(MELD_EINVAL, "meld_segmented_sort_u32: offsets[nseg] = %u > n_keys = %zu",
                    total, n_keys);
    std::string key = fmt("nseg=%u total=%u", log2_ceil(nseg), log2_ceil(total));
    if (ctx->lane_exchange >= 0) key += fmt(" x=%d", ctx->lane_exchange);
    if (const meld::TuneEntry *t = ctx->tuner.find("segsort", key)) {
        *lo = t->lo != 0;
        *hi = t->hi != 0;
        *xch = t->xch != 0;
        return MELD_OK;
    }
    if (total == 0) return MELD_OK;
    meld_status st = ensure_words(&ctx->tune_buf, &ctx->tune_words, total, "tuning scratch");
    if (st != MELD_OK) return st;
    st = ensure_seg(ctx, nseg);
    if (st != MELD_OK) return st;
    std::vector<double> ms;
    std::vector<int> flo, fhi, fx;
    const int paths = ctx->lane_exchange >= 0 ? 1 : 2;
    for (int f = 0; f < 4 * paths; ++f) {
        const bool l = (f & 1) != 0, h = (f & 2) != 0;
        const bool x = ctx->lane_exchange >= 0 ? ctx->lane_exchange != 0 : (f & 4) != 0;
        double t = 0;
        st = time_median(
            s, 3,
            [&]() -> meld_status {
                hipError_t r = hipMemcpyAsync(ctx->tune_buf, keys, (size_t)total * 4,
                                              hipMemcpyDeviceToDevice, s);
                return r == hipSuccess ? MELD_OK : hip_fail(r, "tuning copy");
            },
            [&]() -> meld_status {
                hipError_t r = meld::launch_segmented_sort(
                    ctx->tune_buf, total, offsets, (uint32_t)nseg, ctx->seg_state, ctx->seg_cls,
                    ctx->seg_queue, ctx->seg_work, ctx->seg_grid, l, h, x, s);
                return r == hipSuccess ? MELD_OK : hip_fail(r, "segmented sort launch");
            },
            &t);
        if (st != MELD_OK) return st;
        ms.push_back(t);
        flo.push_back(l);
        fhi.push_back(h);
        fx.push_back(x);
    }
    unsigned long long c[4] = {0};
    st = run_probe(ctx, s, 4, c, [&](unsigned long long *out) {
        return meld::launch_probe_segments(offsets, (uint32_t)nseg, out, s);
    });
    if (st != MELD_OK) return st;
    const double mixed_lo = c[1] ? (double)c[0] / (double)c[1] : 0.0;
    const double mixed_hi = c[3] ? (double)c[2] / (double)c[3] : 0.0;
    const int pick = meld::choose((int)ms.size(), ms.data(), flo.data(), fhi.data(), mixed_lo,
                                  mixed_hi, ctx->theta, ctx->tie);
    *lo = flo[pick] != 0;
    *hi = fhi[pick] != 0;
    *xch = fx[pick] != 0;
    meld::TuneEntry te;
    te.op = "segsort";
    te.key = key;
    te.lo = *lo;
    te.hi = *hi;
    te.xch = *xch;
    te.form = *lo ? 1 : 0;
    te.ms = ms[pick];
    te.mixed_lo = mixed_lo;
    te.mixed_hi = mixed_hi;
    te.trials = (int)ms.size();
    ctx->tuner.put(te);
    return MELD_OK;
}

meld::RegionForm region_form(meld_variant v) {
    return v == MELD_DIVERGENT        ? meld::RegionForm::kDivergent
           : v == MELD_MELDED_INPLACE ? meld::RegionForm::kMeldedInPlace
                                      : meld::RegionForm::kMelded;
}

// MELD_AUTO for the region: the tuned form of this shape class, timing the
// three forms on the caller's arrays (the final run overwrites y).
meld_status auto_region_form(meld_ctx *ctx, const float *x, float *y, size_t n, const float *tab,
                             size_t tab_len, uint64_t seed, uint64_t thr,
                             const meld::RegionSide &T, const meld::RegionSide &F, hipStream_t s,
                             meld::RegionForm *out) {
    *out = meld::RegionForm::kMelded;
    const uint32_t p10 = (uint32_t)((thr * 10 + (1ull << 31)) >> 32);
    const std::string key = fmt("n=%u tab=%u tT=%u tF=%u p10=%u", log2_ceil(n), log2_ceil(tab_len),
                                T.trips, F.trips, p10);
    if (const meld::TuneEntry *t = ctx->tuner.find("region", key)) {
        *out = t->form == 0   ? meld::RegionForm::kDivergent
               : t->form == 3 ? meld::RegionForm::kMeldedInPlace
                              : meld::RegionForm::kMelded;
        return MELD_OK;
    }
    if (capturing(s)) return MELD_OK;
    const meld::RegionForm forms[3] = {meld::RegionForm::kDivergent, meld::RegionForm::kMelded,
                                       meld::RegionForm::kMeldedInPlace};
    const int codes[3] = {0, 1, 3};
    double ms[3];
    int flo[3], fhi[3];
    for (int f = 0; f < 3; ++f) {
        const meld::RegionForm form = forms[f];
        auto run = [&]() -> meld_status {
            hipError_t r = meld::launch_region(x, y, (uint32_t)n, tab, (uint32_t)(tab_len - 1),
                                               seed, thr, T, F, form, s);
            return r == hipSuccess ? MELD_OK : hip_fail(r, "region launch");
        };
        meld_status st = run();  // warm-up
        if (st != MELD_OK) return st;
        st = time_median(s, 3, []() { return MELD_OK; }, run, &ms[f]);
        if (st != MELD_OK) return st;
        flo[f] = fhi[f] = f == 0 ? 0 : 1;
    }
    unsigned long long c[3] = {0};
    meld_status st = run_probe(ctx, s, 3, c, [&](unsigned long long *o) {
        return meld::launch_probe_region((uint32_t)n, seed, thr, o, s);
    });
    if (st != MELD_OK) return st;
    const double mixed = c[2] ? (double)c[0] / (double)c[2] : 0.0;
    const int pick = meld::choose(3, ms, flo, fhi, mixed, mixed, ctx->theta, ctx->tie);
    *out = forms[pick];
    meld::TuneEntry te;
    te.op = "region";
    te.key = key;
    te.lo = te.hi = flo[pick];
    te.form = codes[pick];
    te.ms = ms[pick];
    te.mixed_lo = te.mixed_hi = mixed;
    te.trials = 3;
    ctx->tuner.put(te);
    return MELD_OK;
}

// Checks shared by the region entry points (after which the device is set).
meld_status check_region_args(const char *name, meld_ctx *ctx, const float *x, const float *y,
                              size_t n, const float *tab, size_t tab_len, meld_variant variant) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "%s: ctx is NULL", name);
    if (n >= (1ull << 32)) return fail(MELD_EINVAL, "%s: n >= 2^32", name);
    if (tab_len == 0 || (tab_len & (tab_len - 1)) != 0 || tab_len > (1ull << 32))
        return fail(MELD_EINVAL, "%s: tab_len = %zu is not a power of two <= 2^32", name, tab_len);
    if ((unsigned)variant > MELD_MELDED_INPLACE) return fail(MELD_EINVAL, "%s: bad variant", name);
    return MELD_OK;
}

meld_status check_region_pointers(const char *name, meld_ctx *ctx, const float *x,
                                  const float *y, const float *tab) {
    if (!is_device_ptr(ctx, x) || !is_device_ptr(ctx, y) || !is_device_ptr(ctx, tab))
        return fail(MELD_EINVAL, "%s: x, y and tab must be device pointers on device %d", name,
                    ctx->device);
    if (x == y) return fail(MELD_EINVAL, "%s: y aliases x", name);
    return MELD_OK;
}

// MELD_AUTO for the region variants: times the three forms once per shape
// class on the caller's arrays (the final run overwrites y) and keeps the
// fastest, preferring the melded ones within the tie margin.
template <typename Launch>
meld_status auto_timed_form(meld_ctx *ctx, const char *op, const std::string &key, Launch launch,
                            hipStream_t s, meld::RegionForm *out) {
    *out = meld::RegionForm::kMelded;
    if (const meld::TuneEntry *t = ctx->tuner.find(op, key)) {
        *out = t->form == 0   ? meld::RegionForm::kDivergent
               : t->form == 3 ? meld::RegionForm::kMeldedInPlace
                              : meld::RegionForm::kMelded;
        return MELD_OK;
    }
    if (capturing(s)) return MELD_OK;
    const meld::RegionForm forms[3] = {meld::RegionForm::kDivergent, meld::RegionForm::kMelded,
                                       meld::RegionForm::kMeldedInPlace};
    const int codes[3] = {0, 1, 3};
    double ms[3];
    int flo[3], fhi[3];
    for (int f = 0; f < 3; ++f) {
        auto run = [&]() -> meld_status {
            hipError_t r = launch(forms[f]);
            return r == hipSuccess ? MELD_OK : hip_fail(r, "region launch");
        };
        meld_status st = run();  // warm-up
        if (st != MELD_OK) return st;
        st = time_median(s, 3, []() { return MELD_OK; }, run, &ms[f]);
        if (st != MELD_OK) return st;
        flo[f] = fhi[f] = f == 0 ? 0 : 1;
    }
    const int pick = meld::choose(3, ms, flo, fhi, 1.0, 1.0, ctx->theta, ctx->tie);
    *out = forms[pick];
    meld::TuneEntry te;
    te.op = op;
    te.key = key;
    te.lo = te.hi = flo[pick];
    te.form = codes[pick];
    te.ms = ms[pick];
    te.mixed_lo = te.mixed_hi = 1.0;
    te.trials = 3;
    ctx->tuner.put(te);
    return MELD_OK;
}

// MELD_AUTO for an in-place keys-only operation with a divergent and a
// melded form: the tuned form of this shape class, timing both on a scratch
// copy of the keys the first time. run(keys, melded) enqueues the operation.
template <typename Run>
meld_status auto_two_forms(meld_ctx *ctx, const char *op, const std::string &key,
                           const uint32_t *keys, size_t n, hipStream_t s, Run run, bool *melded) {
    *melded = true;
    if (const meld::TuneEntry *t = ctx->tuner.find(op, key)) {
        *melded = t->form != 0;
        return MELD_OK;
    }
    if (capturing(s)) return MELD_OK;
    meld_status st = ensure_words(&ctx->tune_buf, &ctx->tune_words, n, "tuning scratch");
    if (st != MELD_OK) return st;
    double ms[2];
    int flo[2], fhi[2];
    for (int f = 0; f < 2; ++f) {
        st = time_median(
            s, 3,
            [&]() -> meld_status {
                hipError_t e = hipMemcpyAsync(ctx->tune_buf, keys, n * 4, hipMemcpyDeviceToDevice,
                                              s);
                return e == hipSuccess ? MELD_OK : hip_fail(e, "tuning copy");
            },
            [&]() -> meld_status { return run(ctx->tune_buf, f == 1); }, &ms[f]);
        if (st != MELD_OK) return st;
        flo[f] = fhi[f] = f;
    }
    const int pick = meld::choose(2, ms, flo, fhi, 1.0, 1.0, ctx->theta, ctx->tie);
    *melded = pick == 1;
    meld::TuneEntry te;
    te.op = op;
    te.key = key;
    te.lo = te.hi = pick;
    te.form = pick;
    te.ms = ms[pick];
    te.mixed_lo = te.mixed_hi = 1.0;
    te.trials = 2;
    ctx->tuner.put(te);
    return MELD_OK;
}

// Bottom-up merge sort: runs of 2^10 by the odd-even network, then up to
// max_passes merge passes (negative: all) ping-ponging between keys and the
// context's merge buffer; the result ends in keys.
constexpr uint32_t kMergeRunLog = 10;

meld_status merge_sort_impl(meld_ctx *ctx, uint32_t *keys, size_t n, int64_t max_passes,
                            bool melded, hipStream_t s) {
    hipError_t e = meld::launch_oddeven_buckets(keys, (uint32_t)n, kMergeRunLog, -1, melded, s);
    if (e != hipSuccess) return hip_fail(e, "odd-even launch");
    if (n <= (1u << kMergeRunLog) || max_passes == 0) return MELD_OK;
    meld_status st = ensure_words(&ctx->merge_buf, &ctx->merge_words, n, "merge buffer");
    if (st != MELD_OK) return st;
    st = ensure_words(&ctx->merge_cuts, &ctx->merge_cut_words,
                      meld::merge_pass_cut_words((uint32_t)n), "merge cuts");
    if (st != MELD_OK) return st;
    uint32_t *src = keys, *dst = ctx->merge_buf;
    int64_t pass = 0;
    for (uint32_t lr = kMergeRunLog; ((size_t)1 << lr) < n; ++lr) {
        if (max_passes >= 0 && pass == max_passes) break;
        e = meld::launch_merge_pass(src, dst, (uint32_t)n, lr, melded, ctx->merge_cuts, s);
        if (e != hipSuccess) return hip_fail(e, "merge pass launch");
        std::swap(src, dst);
        ++pass;
    }
    if (src != keys) {
        e = hipMemcpyAsync(keys, src, n * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "merge sort copy-back");
    }
    return MELD_OK;
}

// The region call and its gathers-only probe: argument checks, MELD_AUTO,
// launch.
meld_status region_entry(meld_ctx *ctx, const float *x, float *y, size_t n, const float *tab,
                         size_t tab_len, uint64_t seed, uint64_t thr, meld_side side_true,
                         meld_side side_false, meld_variant variant, void *stream,
                         bool gathers_only, const char *name) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "%s: ctx is NULL", name);
    if (n >= (1ull << 32)) return fail(MELD_EINVAL, "%s: n >= 2^32", name);
    if (tab_len == 0 || (tab_len & (tab_len - 1)) != 0 || tab_len > (1ull << 32))
        return fail(MELD_EINVAL,
                    "%s: tab_len = %zu is not a power of two <= 2^32", name,
                    tab_len);
    if (thr > (1ull << 32))
        return fail(MELD_EINVAL, "%s: thr > 2^32", name);
    if (side_true.trips > 65536 || side_false.trips > 65536)
        return fail(MELD_EINVAL, "%s: trips > 65536", name);
    if ((unsigned)variant > MELD_MELDED_INPLACE)
        return fail(MELD_EINVAL, "%s: bad variant", name);
    if (n == 0) return MELD_OK;
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, x) || !is_device_ptr(ctx, y) || !is_device_ptr(ctx, tab))
        return fail(MELD_EINVAL,
                    "%s: x, y and tab must be device pointers on device %d", name,
                    ctx->device);
    if (x == y) return fail(MELD_EINVAL, "%s: y aliases x", name);
    const meld::RegionSide T{side_true.a, side_true.off, side_true.step, side_true.trips};
    const meld::RegionSide F{side_false.a, side_false.off, side_false.step, side_false.trips};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    meld::RegionForm form = region_form(variant);
    if (variant == MELD_AUTO) {
        meld_status st = auto_region_form(ctx, x, y, n, tab, tab_len, seed, thr, T, F, s, &form);
        if (st != MELD_OK) return st;
    }
    auto launch = gathers_only ? meld::launch_region_gathers : meld::launch_region;
    hipError_t e = launch(x, y, (uint32_t)n, tab, (uint32_t)(tab_len - 1), seed, thr, T, F, form, s);
    if (e != hipSuccess) return hip_fail(e, "region launch");
    return MELD_OK;
}

}  // namespace

extern "C" {

int meld_version(void) { return 100; }

const char *meld_last_error(void) { return g_err.c_str(); }

meld_status meld_create(int hip_device, meld_ctx **out) {
    if (out == nullptr) return fail(MELD_EINVAL, "meld_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= count)
        return fail(MELD_EINVAL, "meld_create: device %d out of range (%d devices)", hip_device,
                    count);
    {
        DeviceGuard g(hip_device);
        e = noalloc_scratch_init(hip_device);
        if (e != hipSuccess) return hip_fail(e, "meld_create: address of the device scratch");
    }
    meld_ctx *ctx = new (std::nothrow) meld_ctx();
    if (ctx == nullptr) return fail(MELD_ENOMEM, "meld_create: out of host memory");
    ctx->device = hip_device;

    hipDeviceProp_t prop;
    int runtime = 0;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess &&
        hipRuntimeGetVersion(&runtime) == hipSuccess)
        ctx->tuner.set_identity(prop.gcnArchName, runtime);
    if (const char *path = std::getenv("MELD_TUNE_CACHE")) {
        if (path[0] != '\0' && !ctx->tuner.attach(path)) {
            delete ctx;
            return fail(MELD_EINVAL, "meld_create: malformed tuning cache %s", path);
        }
    }
    *out = ctx;
    g_err.clear();
    return MELD_OK;
}

void meld_destroy(meld_ctx *ctx) {
    if (ctx == nullptr) return;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    drop_seg_graphs(ctx);
    if (ctx->capture_stream != nullptr) (void)hipStreamDestroy(ctx->capture_stream);
    for (void *p : {(void *)ctx->tail, (void *)ctx->seg_state, (void *)ctx->seg_cls,
                    (void *)ctx->seg_queue, (void *)ctx->seg_work, (void *)ctx->tune_buf,
                    (void *)ctx->merge_buf, (void *)ctx->merge_cuts, (void *)ctx->probe_buf})
        if (p != nullptr) (void)hipFree(p);
    delete ctx;
}

meld_status meld_sort_u32(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                          meld_variant variant, void *stream) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_sort_u32: ctx is NULL");
    if (n >= (1ull << 31)) return fail(MELD_EINVAL, "meld_sort_u32: n = %zu >= 2^31", n);
    if ((unsigned)variant > MELD_MELDED_INPLACE) return fail(MELD_EINVAL, "meld_sort_u32: bad variant");
    if (n <= 1) return MELD_OK;
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, keys))
        return fail(MELD_EINVAL, "meld_sort_u32: keys is not a device pointer on device %d",
                    ctx->device);
    if (payload != nullptr && !is_device_ptr(ctx, payload))
        return fail(MELD_EINVAL, "meld_sort_u32: payload is not a device pointer on device %d",
                    ctx->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    SortPlan plan = fixed_plan(ctx, payload != nullptr, n, variant);
    if (variant == MELD_AUTO) {
        meld_status st = auto_sort_plan(ctx, keys, payload, n, s, &plan);
        if (st != MELD_OK) return st;
    }
    return sort_impl(ctx, keys, payload, n, plan, -1, s);
}

meld_status meld_sort_u32_noalloc(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                                  meld_variant variant, void *stream) {
    const char *name = "meld_sort_u32_noalloc";
    if (ctx == nullptr) return fail(MELD_EINVAL, "%s: ctx is NULL", name);
    if (n >= (1ull << 31)) return fail(MELD_EINVAL, "%s: n = %zu >= 2^31", name, n);
    if ((unsigned)variant > MELD_MELDED_INPLACE) return fail(MELD_EINVAL, "%s: bad variant", name);
    if (n <= 1) return MELD_OK;
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, keys) || (payload != nullptr && !is_device_ptr(ctx, payload)))
        return fail(MELD_EINVAL, "%s: keys and payload must be device pointers on device %d",
                    name, ctx->device);
    const bool pairs = payload != nullptr;
    const uint32_t log_n = log2_ceil(n);
    SortPlan plan = fixed_plan(ctx, pairs, n, variant);
    // MELD_AUTO: a decision the tuner already holds, never a timed trial
    // (trials copy the input into allocated scratch)
    if (variant == MELD_AUTO) (void)cached_sort_plan(ctx, pairs, log_n, &plan);
    const size_t pad = ((size_t)1 << log_n) - n;
    const size_t words = pairs ? 2 * pad : pad;
    const bool one_tile = log_n <= plan.log_t;  // padded in LDS, no scratch
    if (!one_tile && words > kNoAllocWords)
        return fail(MELD_EINVAL,
                    "%s: n = %zu needs %zu words of padding, above the %zu-word scratch "
                    "(MELD_NOALLOC_SCRATCH_WORDS); use meld_sort_u32",
                    name, n, words, kNoAllocWords);
    uint32_t *tail = noalloc_scratch(ctx->device);
    if (tail == nullptr) return fail(MELD_EHIP, "%s: no device scratch on device %d", name, ctx->device);
    return sort_impl(ctx, keys, payload, n, plan, -1, static_cast<hipStream_t>(stream), nullptr,
                     tail, kNoAllocWords);
}

meld_status meld_sort_u32_timed(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                                meld_variant variant, void *stream, float *launch_ms,
                                size_t cap, size_t *n_launches) {
    const char *name = "meld_sort_u32_timed";
    if (ctx == nullptr || launch_ms == nullptr || n_launches == nullptr)
        return fail(MELD_EINVAL, "%s: ctx, launch_ms and n_launches must not be NULL", name);
    *n_launches = 0;
    if (n >= (1ull << 31)) return fail(MELD_EINVAL, "%s: n = %zu >= 2^31", name, n);
    if ((unsigned)variant > MELD_MELDED_INPLACE) return fail(MELD_EINVAL, "%s: bad variant", name);
    if (n <= 1) return MELD_OK;
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, keys) || (payload != nullptr && !is_device_ptr(ctx, payload)))
        return fail(MELD_EINVAL, "%s: keys and payload must be device pointers on device %d",
                    name, ctx->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bool pairs = payload != nullptr;
    SortPlan plan = fixed_plan(ctx, pairs, n, variant);
    if (variant == MELD_AUTO) {
        meld_status st = auto_sort_plan(ctx, keys, payload, n, s, &plan);
        if (st != MELD_OK) return st;
    }
    const size_t launches = sort_passes(plan, pairs, log2_ceil(n)).size();
    if (cap < launches)
        return fail(MELD_EINVAL, "%s: cap = %zu < %zu launches", name, cap, launches);
    std::vector<hipEvent_t> marks(launches + 1, nullptr);
    meld_status st = MELD_OK;
    for (auto &ev : marks)
        if (hipEventCreate(&ev) != hipSuccess) {
            ev = nullptr;
            st = fail(MELD_EHIP, "%s: hipEventCreate failed", name);
            break;
        }
    if (st == MELD_OK) st = sort_impl(ctx, keys, payload, n, plan, -1, s, &marks);
    if (st == MELD_OK) {
        hipError_t e = hipEventSynchronize(marks.back());
        if (e != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
    }
    if (st == MELD_OK) {
        for (size_t i = 0; i < launches; ++i) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, marks[i], marks[i + 1]);
            launch_ms[i] = ms;
        }
        *n_launches = launches;
    }
    for (hipEvent_t ev : marks)
        if (ev != nullptr) (void)hipEventDestroy(ev);
    return st;
}

meld_status meld_sort_plan_describe(meld_ctx *ctx, size_t n, int with_payload,
                                    meld_variant variant, char *buf, size_t len) {
    const char *name = "meld_sort_plan_describe";
    if (buf == nullptr) return fail(MELD_EINVAL, "%s: buf must not be NULL", name);
    if (n >= (1ull << 31)) return fail(MELD_EINVAL, "%s: n = %zu >= 2^31", name, n);
    if ((unsigned)variant > MELD_MELDED_INPLACE) return fail(MELD_EINVAL, "%s: bad variant", name);
    const bool pairs = with_payload != 0;
    const uint32_t log_n = n <= 1 ? 0 : log2_ceil(n);
    const bool m = variant == MELD_AUTO || use_melded(variant);
    SortPlan plan{default_log_tile(pairs, log_n), m, m, true};
    bool tuned = false;
    if (ctx != nullptr) {
        plan.log_t = plan_log_tile(ctx, pairs, log_n);
        plan.xch = plan_xch(ctx);
        if (variant == MELD_AUTO) tuned = cached_sort_plan(ctx, pairs, log_n, &plan);
    }
    std::string d = fmt("{\"n\": %zu, \"log_n\": %u, \"pairs\": %s, \"tuned\": %s", n, log_n,
                        pairs ? "true" : "false", tuned ? "true" : "false");
    uint32_t hbm = 0, steps = 0;
    std::string list;
    if (n > 1) {
        const std::vector<SortPass> passes = sort_passes(plan, pairs, log_n);
        const bool regs_kernel = passes[0].kind != PassKind::kTile || log_n >= kMinLogRegsTile;
        d += fmt(", \"log_tile\": %u, \"low\": \"%s\", \"high\": \"%s\", \"low_path\": \"%s\"",
                 passes[0].kind == PassKind::kTile ? std::max<uint32_t>(log_n, 1) : plan.log_t,
                 plan.lo ? "melded" : "divergent", plan.hi ? "melded" : "divergent",
                 !regs_kernel ? "lds" : plan.xch ? "lane_exchange" : "lds");
        for (const SortPass &p : passes) {
            if (!list.empty()) list += ", ";
            list += fmt("{\"kind\": \"%s\", \"steps\": %u", pass_name(p.kind), p.steps);
            if (p.kind != PassKind::kTile && p.kind != PassKind::kLocal)
                list += fmt(", \"m\": %u", p.m);
            if (p.kind == PassKind::kRegs || p.kind == PassKind::kGather)
                list += fmt(", \"b_hi\": %u, \"b_lo\": %u", p.b_hi, p.b_lo);
            list += "}";
            steps += p.steps;
        }
        hbm = (uint32_t)passes.size();
    }
    d += fmt(", \"hbm_passes\": %u, \"steps\": %u, \"passes\": [", hbm, steps) + list + "]}";
    if (d.size() + 1 > len)
        return fail(MELD_EINVAL, "%s: buffer too small (need %zu bytes)", name, d.size() + 1);
    std::memcpy(buf, d.c_str(), d.size() + 1);
    return MELD_OK;
}

meld_status meld_oddeven_sort_buckets_u32(meld_ctx *ctx, uint32_t *keys, size_t n,
                                          uint32_t log_bucket, int64_t max_steps,
                                          meld_variant variant, void *stream) {
    const char *name = "meld_oddeven_sort_buckets_u32";
    if (ctx == nullptr) return fail(MELD_EINVAL, "%s: ctx is NULL", name);
    if (n >= (1ull << 31)) return fail(MELD_EINVAL, "%s: n = %zu >= 2^31", name, n);
    if (log_bucket < 6 || log_bucket > 14)
        return fail(MELD_EINVAL, "%s: log_bucket = %u outside 6..14", name, log_bucket);
    if ((unsigned)variant > MELD_MELDED_INPLACE) return fail(MELD_EINVAL, "%s: bad variant", name);
    if (n == 0 || max_steps == 0) return MELD_OK;
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, keys))
        return fail(MELD_EINVAL, "%s: keys is not a device pointer on device %d", name,
                    ctx->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    bool melded = use_melded(variant);
    if (variant == MELD_AUTO) {
        auto run = [&](uint32_t *k, bool m) -> meld_status {
            hipError_t e = meld::launch_oddeven_buckets(k, (uint32_t)n, log_bucket, -1, m, s);
            return e == hipSuccess ? MELD_OK : hip_fail(e, "odd-even launch");
        };
        meld_status st = auto_two_forms(ctx, "oddeven", fmt("n=%u b=%u", log2_ceil(n), log_bucket),
                                        keys, n, s, run, &melded);
        if (st != MELD_OK) return st;
    }
    const int32_t limit = max_steps < 0 || max_steps > 0x7FFFFFFF ? -1 : (int32_t)max_steps;
    hipError_t e = meld::launch_oddeven_buckets(keys, (uint32_t)n, log_bucket, limit, melded, s);
    if (e != hipSuccess) return hip_fail(e, "odd-even launch");
    return MELD_OK;
}

meld_status meld_merge_sort_u32(meld_ctx *ctx, uint32_t *keys, size_t n, int64_t max_passes,
                                meld_variant variant, void *stream) {
    const char *name = "meld_merge_sort_u32";
    if (ctx == nullptr) return fail(MELD_EINVAL, "%s: ctx is NULL", name);
    if (n >= (1ull << 31)) return fail(MELD_EINVAL, "%s: n = %zu >= 2^31", name, n);
    if ((unsigned)variant > MELD_MELDED_INPLACE) return fail(MELD_EINVAL, "%s: bad variant", name);
    if (n <= 1) return MELD_OK;
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, keys))
        return fail(MELD_EINVAL, "%s: keys is not a device pointer on device %d", name,
                    ctx->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    bool melded = use_melded(variant);
    if (variant == MELD_AUTO) {
        auto run = [&](uint32_t *k, bool m) { return merge_sort_impl(ctx, k, n, -1, m, s); };
        meld_status st =
            auto_two_forms(ctx, "mergesort", fmt("n=%u", log2_ceil(n)), keys, n, s, run, &melded);
        if (st != MELD_OK) return st;
    }
    return merge_sort_impl(ctx, keys, n, max_passes, melded, s);
}

meld_status meld_sort_u32_steps(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                                int64_t max_steps, meld_variant variant, void *stream) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_sort_u32_steps: ctx is NULL");
    if (n < 2 || n >= (1ull << 31) || (n & (n - 1)) != 0)
        return fail(MELD_EINVAL, "meld_sort_u32_steps: n = %zu is not a power of two in [2, 2^30]",
                    n);
    if ((unsigned)variant > MELD_MELDED_INPLACE) return fail(MELD_EINVAL, "meld_sort_u32_steps: bad variant");
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, keys) || (payload != nullptr && !is_device_ptr(ctx, payload)))
        return fail(MELD_EINVAL, "meld_sort_u32_steps: arrays must be device pointers");
    if (max_steps < 0) max_steps = -1;
    return sort_impl(ctx, keys, payload, n, fixed_plan(ctx, payload != nullptr, n, variant),
                     max_steps, static_cast<hipStream_t>(stream));
}

meld_status meld_divergent_region_f32(meld_ctx *ctx, const float *x, float *y, size_t n,
                                      const float *tab, size_t tab_len, uint64_t seed,
                                      uint64_t thr, meld_side side_true, meld_side side_false,
                                      meld_variant variant, void *stream) {
    return region_entry(ctx, x, y, n, tab, tab_len, seed, thr, side_true, side_false, variant,
                        stream, false, "meld_divergent_region_f32");
}

meld_status meld_probe_region_gathers(meld_ctx *ctx, const float *x, float *y, size_t n,
                                      const float *tab, size_t tab_len, uint64_t seed,
                                      uint64_t thr, meld_side side_true, meld_side side_false,
                                      meld_variant variant, void *stream) {
    return region_entry(ctx, x, y, n, tab, tab_len, seed, thr, side_true, side_false, variant,
                        stream, true, "meld_probe_region_gathers");
}

meld_status meld_region3_f32(meld_ctx *ctx, const float *x, float *y, size_t n,
                             const float *tab, size_t tab_len, uint64_t seed, uint64_t thr0,
                             uint64_t thr1, meld_side way0, meld_side way1, meld_side way2,
                             meld_variant variant, void *stream) {
    const char *name = "meld_region3_f32";
    meld_status st = check_region_args(name, ctx, x, y, n, tab, tab_len, variant);
    if (st != MELD_OK) return st;
    if (thr0 > thr1 || thr1 > (1ull << 32))
        return fail(MELD_EINVAL, "%s: thresholds must satisfy thr0 <= thr1 <= 2^32", name);
    if (way0.trips > 65536 || way1.trips > 65536 || way2.trips > 65536)
        return fail(MELD_EINVAL, "%s: trips > 65536", name);
    if (n == 0) return MELD_OK;
    DeviceGuard g(ctx->device);
    st = check_region_pointers(name, ctx, x, y, tab);
    if (st != MELD_OK) return st;
    const meld::RegionSide W0{way0.a, way0.off, way0.step, way0.trips};
    const meld::RegionSide W1{way1.a, way1.off, way1.step, way1.trips};
    const meld::RegionSide W2{way2.a, way2.off, way2.step, way2.trips};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    auto launch = [&](meld::RegionForm f) {
        return meld::launch_region3(x, y, (uint32_t)n, tab, (uint32_t)(tab_len - 1), seed, thr0,
                                    thr1, W0, W1, W2, f, s);
    };
    meld::RegionForm form = region_form(variant);
    if (variant == MELD_AUTO) {
        const uint32_t p0 = (uint32_t)((thr0 * 10 + (1ull << 31)) >> 32);
        const uint32_t p1 = (uint32_t)((thr1 * 10 + (1ull << 31)) >> 32);
        const std::string key =
            fmt("n=%u tab=%u t=%u,%u,%u p10=%u,%u", log2_ceil(n), log2_ceil(tab_len), W0.trips,
                W1.trips, W2.trips, p0, p1);
        st = auto_timed_form(ctx, "region3", key, launch, s, &form);
        if (st != MELD_OK) return st;
    }
    hipError_t e = launch(form);
    if (e != hipSuccess) return hip_fail(e, "region3 launch");
    return MELD_OK;
}

meld_status meld_region_lanetrips_f32(meld_ctx *ctx, const float *x, float *y, size_t n,
                                      const float *tab, size_t tab_len, uint64_t seed,
                                      uint64_t thr, meld_side_range side_true,
                                      meld_side_range side_false, meld_variant variant,
                                      void *stream) {
    const char *name = "meld_region_lanetrips_f32";
    meld_status st = check_region_args(name, ctx, x, y, n, tab, tab_len, variant);
    if (st != MELD_OK) return st;
    if (thr > (1ull << 32)) return fail(MELD_EINVAL, "%s: thr > 2^32", name);
    for (const meld_side_range *r : {&side_true, &side_false}) {
        if (r->trips_lo > r->trips_hi)
            return fail(MELD_EINVAL, "%s: trips_lo > trips_hi", name);
        if (r->trips_hi > 65536) return fail(MELD_EINVAL, "%s: trips > 65536", name);
    }
    if (n == 0) return MELD_OK;
    DeviceGuard g(ctx->device);
    st = check_region_pointers(name, ctx, x, y, tab);
    if (st != MELD_OK) return st;
    const meld::RegionSideRange T{side_true.a, side_true.off, side_true.step, side_true.trips_lo,
                                  side_true.trips_hi - side_true.trips_lo};
    const meld::RegionSideRange F{side_false.a, side_false.off, side_false.step,
                                  side_false.trips_lo, side_false.trips_hi - side_false.trips_lo};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    auto launch = [&](meld::RegionForm f) {
        return meld::launch_region_lanetrips(x, y, (uint32_t)n, tab, (uint32_t)(tab_len - 1), seed,
                                             thr, T, F, f, s);
    };
    meld::RegionForm form = region_form(variant);
    if (variant == MELD_AUTO) {
        const uint32_t p10 = (uint32_t)((thr * 10 + (1ull << 31)) >> 32);
        const std::string key =
            fmt("n=%u tab=%u T=%u-%u F=%u-%u p10=%u", log2_ceil(n), log2_ceil(tab_len),
                side_true.trips_lo, side_true.trips_hi, side_false.trips_lo, side_false.trips_hi,
                p10);
        st = auto_timed_form(ctx, "region_lanetrips", key, launch, s, &form);
        if (st != MELD_OK) return st;
    }
    hipError_t e = launch(form);
    if (e != hipSuccess) return hip_fail(e, "region_lanetrips launch");
    return MELD_OK;
}

meld_status meld_segmented_sort_u32(meld_ctx *ctx, uint32_t *keys, size_t n_keys,
                                    const uint32_t *offsets, size_t nseg, meld_variant variant,
                                    void *stream) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_segmented_sort_u32: ctx is NULL");
    if ((unsigned)variant > MELD_MELDED_INPLACE)
        return fail(MELD_EINVAL, "meld_segmented_sort_u32: bad variant");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    bool lo = use_melded(variant), hi = lo, xch = plan_xch(ctx);
    if (variant == MELD_AUTO && nseg > 0 && nseg < (1ull << 31)) {
        DeviceGuard g(ctx->device);
        if (!is_device_ptr(ctx, keys) || !is_device_ptr(ctx, offsets))
            return fail(MELD_EINVAL,
                        "meld_segmented_sort_u32: keys and offsets must be device pointers on "
                        "device %d",
                        ctx->device);
        meld_status st = auto_seg_forms(ctx, keys, n_keys, offsets, nseg, s, &lo, &hi, &xch);
        if (st != MELD_OK) return st;
    }
    return segmented_impl(ctx, keys, n_keys, offsets, nseg, lo, hi, xch, s,
                          "meld_segmented_sort_u32");
}

meld_status meld_segmented_sort_u32_staged(meld_ctx *ctx, uint32_t *keys, size_t n_keys,
                                           const uint32_t *offsets, size_t nseg,
                                           meld_variant low_phases, meld_variant high_phases,
                                           void *stream) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_segmented_sort_u32_staged: ctx is NULL");
    if ((unsigned)low_phases > MELD_MELDED_INPLACE || (unsigned)high_phases > MELD_MELDED_INPLACE)
        return fail(MELD_EINVAL, "meld_segmented_sort_u32_staged: bad variant");
    return segmented_impl(ctx, keys, n_keys, offsets, nseg, use_melded(low_phases),
                          use_melded(high_phases), plan_xch(ctx), static_cast<hipStream_t>(stream),
                          "meld_segmented_sort_u32_staged");
}

meld_status meld_tune(meld_ctx *ctx, const char *cache_path) {
    if (ctx == nullptr || cache_path == nullptr)
        return fail(MELD_EINVAL, "meld_tune: ctx and cache_path must not be NULL");
    if (!ctx->tuner.attach(cache_path))
        return fail(MELD_EINVAL, "meld_tune: malformed tuning cache %s", cache_path);
    return MELD_OK;
}

meld_status meld_plan_describe(meld_ctx *ctx, char *buf, size_t len) {
    if (ctx == nullptr || buf == nullptr)
        return fail(MELD_EINVAL, "meld_plan_describe: ctx and buf must not be NULL");
    const std::string d = ctx->tuner.describe();
    if (d.size() + 1 > len)
        return fail(MELD_EINVAL, "meld_plan_describe: buffer too small (need %zu bytes)",
                    d.size() + 1);
    std::memcpy(buf, d.c_str(), d.size() + 1);
    return MELD_OK;
}

int meld_tune_choose(int n, const double *ms, const int *melded_lo, const int *melded_hi,
                     double mixed_lo, double mixed_hi, double theta, double tie) {
    if (n <= 0 || ms == nullptr || melded_lo == nullptr || melded_hi == nullptr) return -1;
    return meld::choose(n, ms, melded_lo, melded_hi, mixed_lo, mixed_hi, theta, tie);
}

meld_status meld_probe_region(meld_ctx *ctx, size_t n, uint64_t seed, uint64_t thr,
                              uint64_t out[3], void *stream) {
    if (ctx == nullptr || out == nullptr)
        return fail(MELD_EINVAL, "meld_probe_region: ctx and out must not be NULL");
    if (n >= (1ull << 32) || thr > (1ull << 32))
        return fail(MELD_EINVAL, "meld_probe_region: n >= 2^32 or thr > 2^32");
    DeviceGuard g(ctx->device);
    unsigned long long c[3] = {0, 0, 0};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    meld_status st = run_probe(ctx, s, 3, c, [&](unsigned long long *o) {
        return meld::launch_probe_region((uint32_t)n, seed, thr, o, s);
    });
    for (int i = 0; i < 3; ++i) out[i] = c[i];
    return st;
}

meld_status meld_probe_network(meld_ctx *ctx, uint32_t log_t, uint64_t *out, void *stream) {
    if (ctx == nullptr || out == nullptr)
        return fail(MELD_EINVAL, "meld_probe_network: ctx and out must not be NULL");
    if (log_t < 1 || log_t > 16) return fail(MELD_EINVAL, "meld_probe_network: log_t not in 1..16");
    DeviceGuard g(ctx->device);
    unsigned long long c[32] = {0};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    meld_status st = run_probe(ctx, s, 2 * log_t, c, [&](unsigned long long *o) {
        return meld::launch_probe_network(log_t, false, o, s);
    });
    for (uint32_t i = 0; i < 2 * log_t; ++i) out[i] = c[i];
    return st;
}

meld_status meld_probe_segments(meld_ctx *ctx, const uint32_t *offsets, size_t nseg,
                                uint64_t out[4], void *stream) {
    if (ctx == nullptr || out == nullptr)
        return fail(MELD_EINVAL, "meld_probe_segments: ctx and out must not be NULL");
    if (nseg >= (1ull << 31)) return fail(MELD_EINVAL, "meld_probe_segments: nseg >= 2^31");
    for (int i = 0; i < 4; ++i) out[i] = 0;
    if (nseg == 0) return MELD_OK;
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, offsets))
        return fail(MELD_EINVAL, "meld_probe_segments: offsets must be a device pointer");
    unsigned long long c[4] = {0, 0, 0, 0};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    meld_status st = run_probe(ctx, s, 4, c, [&](unsigned long long *o) {
        return meld::launch_probe_segments(offsets, (uint32_t)nseg, o, s);
    });
    for (int i = 0; i < 4; ++i) out[i] = c[i];
    return st;
}

meld_status meld_set_option(meld_ctx *ctx, meld_option option, int64_t value) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_set_option: ctx is NULL");
    switch (option) {
        case MELD_OPT_USE_GRAPHS:
            ctx->use_graphs = value != 0;
            return MELD_OK;
        case MELD_OPT_SORT_LOG_TILE:
            if (value != 0 && (value < (int64_t)kMinLogRegsTile || value > meld::kMaxLogTileKeys))
                return fail(MELD_EINVAL, "meld_set_option: sort tile 2^%lld outside 2^%u .. 2^%d",
                            (long long)value, kMinLogRegsTile, meld::kMaxLogTileKeys);
            ctx->sort_log_tile = (uint32_t)value;
            return MELD_OK;
        case MELD_OPT_LANE_EXCHANGE:
            if (value < -1 || value > 1)
                return fail(MELD_EINVAL, "meld_set_option: lane exchange %lld not in {-1, 0, 1}",
                            (long long)value);
            ctx->lane_exchange = (int)value;
            return MELD_OK;
        default:
            return fail(MELD_EINVAL, "meld_set_option: unknown option %d", (int)option);
    }
}

meld_status meld_segmented_sort_check(meld_ctx *ctx, void *stream) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_segmented_sort_check: ctx is NULL");
    if (ctx->seg_state == nullptr) return MELD_OK;
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t sticky = 0;
    e = hipMemcpy(&sticky, &ctx->seg_state->sticky, sizeof sticky, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the segmented sort flag");
    const uint32_t zero = 0;
    e = hipMemcpy(&ctx->seg_state->sticky, &zero, sizeof zero, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "clearing the segmented sort flag");
    if (sticky == 0) return MELD_OK;
    return fail(MELD_EINVAL, "segmented sort: invalid offsets (%s%s%s%s); keys left untouched",
                (sticky & meld::kSegBadFirst) ? "offsets[0] != 0 " : "",
                (sticky & meld::kSegDecreasing) ? "decreasing offsets " : "",
                (sticky & meld::kSegTooLong) ? "segment longer than 65536 " : "",
                (sticky & meld::kSegBeyondEnd) ? "offset beyond n_keys" : "");
}

}  // extern "C"
