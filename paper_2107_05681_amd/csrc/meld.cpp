// C-ABI host layer of the melded kernel library: argument checks, plans,
// scratch and launches. Every compute step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/meld.h"
#include "kernels.h"

using meld::SortArray;

struct meld_ctx {
    int device = 0;
    // Tail workspace backing the virtual padding of non-power-of-two sorts.
    uint32_t *tail = nullptr;
    size_t tail_words = 0;
};

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

// Threads per workgroup for a tile of 2^log_t elements: one comparator per
// lane per iteration, at most 512 lanes.
int tile_threads(uint32_t log_t) {
    if (log_t <= 7) return 64;
    if (log_t <= 9) return 256;
    return 512;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Enqueues the whole network (or its first step_limit steps) on keys[0..n).
meld_status sort_impl(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                      meld_variant variant, int64_t step_limit, hipStream_t stream) {
    const bool pairs = payload != nullptr;
    const uint32_t log_n = log2_ceil(n);
    const size_t big_n = (size_t)1 << log_n;
    const uint32_t max_log_t = pairs ? meld::kMaxLogTilePairs : meld::kMaxLogTileKeys;
    const bool melded = use_melded(variant);

    SortArray a{keys, payload, nullptr, nullptr, (uint32_t)n};
    int64_t left = step_limit;  // < 0: unlimited
    auto take = [&left](uint64_t steps) -> int32_t {
        if (left < 0) return -1;
        const int64_t s = std::min<int64_t>(left, (int64_t)steps);
        left -= s;
        return (int32_t)s;
    };

    hipError_t e;
    if (log_n <= max_log_t) {
        // One tile holds everything; positions >= n are sentinels in LDS.
        const uint32_t log_t = std::max<uint32_t>(log_n, 1);
        const int io = big_n > n ? meld::kIoSentinel
                       : (aligned16(keys) && (!pairs || aligned16(payload))) ? meld::kIoPlainVec
                                                                             : meld::kIoPlain;
        e = meld::launch_bitonic_tile(a, log_t, 1, 1, log_t, 0,
                                      take((uint64_t)log_t * (log_t + 1) / 2), melded, io,
                                      tile_threads(log_t), stream);
        if (e != hipSuccess) return hip_fail(e, "bitonic tile launch");
        return MELD_OK;
    }

    if (big_n > n) {
        const size_t pad = big_n - n;
        meld_status st = ensure_tail(ctx, pairs ? 2 * pad : pad);
        if (st != MELD_OK) return st;
        a.tk = ctx->tail;
        a.tv = pairs ? ctx->tail + pad : nullptr;
        e = meld::launch_fill_u32(ctx->tail, 0xFFFFFFFFu, pairs ? 2 * pad : pad, stream);
        if (e != hipSuccess) return hip_fail(e, "fill launch");
    }

    const uint32_t log_t = max_log_t;
    const uint32_t n_tiles = (uint32_t)(big_n >> log_t);
    const int threads = tile_threads(log_t);
    const int io = a.tk != nullptr ? meld::kIoTail
                   : (aligned16(keys) && (!pairs || aligned16(payload))) ? meld::kIoPlainVec
                                                                         : meld::kIoPlain;
    e = meld::launch_bitonic_tile(a, log_t, n_tiles, 1, log_t, 0,
                                  take((uint64_t)log_t * (log_t + 1) / 2), melded, io, threads,
                                  stream);
    if (e != hipSuccess) return hip_fail(e, "bitonic tile launch");

    for (uint32_t m = log_t + 1; m <= log_n; ++m) {
        // Steps j = 2^(m-1) .. 2^log_t stream through HBM, fused in balanced
        // groups of at most kMaxFusedSteps.
        const uint32_t d = m - log_t;
        const uint32_t passes = (d + meld::kMaxFusedSteps - 1) / meld::kMaxFusedSteps;
        uint32_t b_hi = m - 1;
        for (uint32_t p = 0; p < passes; ++p) {
            const uint32_t remaining = b_hi - log_t + 1;
            const uint32_t this_r = (remaining + (passes - p) - 1) / (passes - p);
            const uint32_t b_lo = b_hi + 1 - this_r;
            e = meld::launch_bitonic_global(a, log_n, m, b_hi, b_lo, take(this_r), stream);
            if (e != hipSuccess) return hip_fail(e, "bitonic global launch");
            b_hi = b_lo - 1;
        }
        // Steps j = 2^(log_t-1) .. 1 of phase m in LDS tiles.
        e = meld::launch_bitonic_tile(a, log_t, n_tiles, m, m, log_t - 1, take(log_t), melded,
                                      io, threads, stream);
        if (e != hipSuccess) return hip_fail(e, "bitonic merge launch");
    }
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
    meld_ctx *ctx = new (std::nothrow) meld_ctx();
    if (ctx == nullptr) return fail(MELD_ENOMEM, "meld_create: out of host memory");
    ctx->device = hip_device;
    *out = ctx;
    g_err.clear();
    return MELD_OK;
}

void meld_destroy(meld_ctx *ctx) {
    if (ctx == nullptr) return;
    DeviceGuard g(ctx->device);
    if (ctx->tail != nullptr) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->tail);
    }
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
    return sort_impl(ctx, keys, payload, n, variant, -1, static_cast<hipStream_t>(stream));
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
    return sort_impl(ctx, keys, payload, n, variant, max_steps, static_cast<hipStream_t>(stream));
}

meld_status meld_divergent_region_f32(meld_ctx *ctx, const float *x, float *y, size_t n,
                                      const float *tab, size_t tab_len, uint64_t seed,
                                      uint64_t thr, meld_side side_true, meld_side side_false,
                                      meld_variant variant, void *stream) {
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_divergent_region_f32: ctx is NULL");
    if (n >= (1ull << 32)) return fail(MELD_EINVAL, "meld_divergent_region_f32: n >= 2^32");
    if (tab_len == 0 || (tab_len & (tab_len - 1)) != 0 || tab_len > (1ull << 32))
        return fail(MELD_EINVAL,
                    "meld_divergent_region_f32: tab_len = %zu is not a power of two <= 2^32",
                    tab_len);
    if (thr > (1ull << 32))
        return fail(MELD_EINVAL, "meld_divergent_region_f32: thr > 2^32");
    if (side_true.trips > 65536 || side_false.trips > 65536)
        return fail(MELD_EINVAL, "meld_divergent_region_f32: trips > 65536");
    if ((unsigned)variant > MELD_MELDED_INPLACE)
        return fail(MELD_EINVAL, "meld_divergent_region_f32: bad variant");
    if (n == 0) return MELD_OK;
    DeviceGuard g(ctx->device);
    if (!is_device_ptr(ctx, x) || !is_device_ptr(ctx, y) || !is_device_ptr(ctx, tab))
        return fail(MELD_EINVAL,
                    "meld_divergent_region_f32: x, y and tab must be device pointers on device %d",
                    ctx->device);
    if (x == y) return fail(MELD_EINVAL, "meld_divergent_region_f32: y aliases x");
    const meld::RegionSide T{side_true.a, side_true.off, side_true.step, side_true.trips};
    const meld::RegionSide F{side_false.a, side_false.off, side_false.step, side_false.trips};
    const meld::RegionForm form = variant == MELD_DIVERGENT ? meld::RegionForm::kDivergent
                                  : variant == MELD_MELDED_INPLACE
                                      ? meld::RegionForm::kMeldedInPlace
                                      : meld::RegionForm::kMelded;
    hipError_t e = meld::launch_region(x, y, (uint32_t)n, tab, (uint32_t)(tab_len - 1), seed, thr,
                                       T, F, form, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "region launch");
    return MELD_OK;
}

meld_status meld_segmented_sort_u32(meld_ctx *ctx, uint32_t *keys, const uint32_t *offsets,
                                    size_t nseg, meld_variant variant, void *stream) {
    (void)keys;
    (void)offsets;
    (void)variant;
    (void)stream;
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_segmented_sort_u32: ctx is NULL");
    if (nseg == 0) return MELD_OK;
    return fail(MELD_EUNSUPPORTED, "meld_segmented_sort_u32: not built yet");
}

meld_status meld_segmented_sort_check(meld_ctx *ctx, void *stream) {
    (void)stream;
    if (ctx == nullptr) return fail(MELD_EINVAL, "meld_segmented_sort_check: ctx is NULL");
    return MELD_OK;
}

}  // extern "C"
