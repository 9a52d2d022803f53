// Segmented bitonic sort: many uneven buckets in one persistent launch.
//
// The paper's bitonic benchmark sorts one bucket per thread block
// (Evaluation section, "Bitonic Sort (BIT)"). Here thousands of buckets of
// 0..65536 keys are sorted in one launch:
//   1. reset    — clears the work-queue counters (a kernel, so the sequence
//                 can be captured in a graph);
//   2. classify — per segment: validity checks and the size class
//                 c = ceil(log2(len)) (0 for len <= 1: nothing to do);
//   3. plan     — queue layout: classes in descending order (largest first),
//                 segments of more than 128 keys are one work item each,
//                 shorter ones are bundled 16 to an item (one per wave);
//   4. scatter  — segment ids into the queue;
//   5. sort     — a persistent grid (one 1024-lane workgroup per CU, 128 KiB
//                 of LDS each) pulls items from an atomic counter until the
//                 queue is empty.
// Each segment runs the Figure 1 network on its own (padded) length with
// the segment-local index giving the direction. Per stage the caller picks
// the divergent or melded compare-exchange: MELD_LO for phases k <= 64 (the
// direction differs between the lanes of a wave) and MELD_HI for k >= 128
// (wave-uniform direction).
//
// A segment of up to 2^15 keys sorts in LDS. A longer one (up to 2^16) sorts
// its two halves in LDS (phases up to 2^15: the first ascending, the second
// descending), runs the step j = 2^15 of the last phase through global memory
// and merges each half in LDS; padding positions past the segment live in a
// per-workgroup global scratch of 2^15 words. All of it stays inside one
// workgroup, so no grid-wide synchronisation is needed.
#include "device_common.h"
#include "kernels.h"
#include "network.h"

namespace meld {

namespace {

constexpr uint32_t kPad = 0xFFFFFFFFu;
constexpr uint32_t kWavesPerBlock = kSegThreads / 64;
constexpr uint32_t kSmallMax = 128;
constexpr uint32_t kSmallClassMax = 7;  // ceil(log2(128))

__device__ __forceinline__ uint32_t ceil_log2(uint32_t v) {
    return v <= 1 ? 0u : 32u - (uint32_t)__clz(v - 1);
}

__global__ void seg_reset_kernel(SegState *st) {
    const uint32_t t = threadIdx.x;
    if (t < kSegClasses) {
        st->cnt[t] = 0;
        st->fill[t] = 0;
        st->base[t] = 0;
    }
    if (t == 0) {
        st->head = 0;
        st->flag = 0;
        st->n_big = 0;
        st->n_small = 0;
        st->n_items = 0;
    }
}

__global__ __launch_bounds__(256) void seg_classify_kernel(const uint32_t *__restrict__ off,
                                                           uint32_t nseg, SegState *st,
                                                           uint8_t *__restrict__ cls) {
    __shared__ uint32_t lcnt[kSegClasses];
    if (threadIdx.x < kSegClasses) lcnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s < nseg) {
        const uint32_t lo = off[s];
        const uint32_t hi = off[s + 1];
        uint32_t f = 0;
        if (s == 0 && lo != 0) f |= kSegBadFirst;
        if (hi < lo)
            f |= kSegDecreasing;
        else if (hi - lo > kSegMaxLen)
            f |= kSegTooLong;
        if (f != 0) {
            atomicOr(&st->flag, f);
            atomicOr(&st->sticky, f);
        }
        const uint32_t c = f != 0 ? 0u : ceil_log2(hi - lo);
        cls[s] = (uint8_t)c;
        if (c != 0) atomicAdd(&lcnt[c], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kSegClasses && threadIdx.x != 0 && lcnt[threadIdx.x] != 0)
        atomicAdd(&st->cnt[threadIdx.x], lcnt[threadIdx.x]);
}

__global__ void seg_plan_kernel(SegState *st) {
    if (threadIdx.x != 0) return;
    uint32_t pos = 0, n_big = 0, n_small = 0;
    for (int c = (int)kSegClasses - 1; c >= 1; --c) {
        st->base[c] = pos;
        pos += st->cnt[c];
        if ((uint32_t)c > kSmallClassMax)
            n_big += st->cnt[c];
        else
            n_small += st->cnt[c];
    }
    st->n_big = n_big;
    st->n_small = n_small;
    st->n_items = n_big + (n_small + kWavesPerBlock - 1) / kWavesPerBlock;
    st->head = 0;
}

__global__ __launch_bounds__(256) void seg_scatter_kernel(uint32_t nseg,
                                                          const uint8_t *__restrict__ cls,
                                                          SegState *st,
                                                          uint32_t *__restrict__ queue) {
    __shared__ uint32_t lcnt[kSegClasses];
    __shared__ uint32_t lbase[kSegClasses];
    if (threadIdx.x < kSegClasses) lcnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    const uint32_t c = s < nseg ? cls[s] : 0u;
    const uint32_t rank = c != 0 ? atomicAdd(&lcnt[c], 1u) : 0u;
    __syncthreads();
    if (threadIdx.x < kSegClasses && lcnt[threadIdx.x] != 0)
        lbase[threadIdx.x] = atomicAdd(&st->fill[threadIdx.x], lcnt[threadIdx.x]);
    __syncthreads();
    if (c != 0) queue[st->base[c] + lbase[c] + rank] = s;
}

// Sorts segment [lo, lo + len), 128 < len <= 2^15, padded to 2^m in LDS.
template <bool MELD_LO, bool MELD_HI>
__device__ void sort_in_lds(uint32_t *__restrict__ keys, uint32_t *s, uint32_t lo, uint32_t len,
                            uint32_t m) {
    const uint32_t T = 1u << m;
    const uint32_t tid = threadIdx.x;
    for (uint32_t p = tid; p < T; p += kSegThreads) s[p] = p < len ? keys[lo + p] : kPad;
    __syncthreads();
    lds_network<uint32_t, MELD_LO, MELD_HI, kSegThreads, true>(s, T, 0, 1, m, 0, -1, tid);
    __syncthreads();
    for (uint32_t p = tid; p < len; p += kSegThreads) keys[lo + p] = s[p];
    __syncthreads();
}

// Sorts segment [lo, lo + len), 2^15 < len <= 2^16, as two LDS halves.
template <bool MELD_LO, bool MELD_HI>
__device__ void sort_two_halves(uint32_t *__restrict__ keys, uint32_t *s,
                                uint32_t *__restrict__ pad, uint32_t lo, uint32_t len) {
    constexpr uint32_t T = kSegTile;
    const uint32_t tid = threadIdx.x;
    // Position q of the padded segment: the caller's keys below len, the
    // workgroup's pad scratch above (q - len < 2^16 - len < 2^15).
    auto at = [&](uint32_t q) -> uint32_t * { return q < len ? keys + lo + q : pad + (q - len); };
    // Phases 2 .. 2^15 on each half; bit 15 of the index makes the second
    // half descending.
    for (uint32_t h = 0; h < 2; ++h) {
        for (uint32_t p = tid; p < T; p += kSegThreads) {
            const uint32_t q = h * T + p;
            s[p] = q < len ? keys[lo + q] : kPad;
        }
        __syncthreads();
        lds_network<uint32_t, MELD_LO, MELD_HI, kSegThreads, true>(s, T, h * T, 1, kSegLogTile,
                                                                   0, -1, tid);
        __syncthreads();
        for (uint32_t p = tid; p < T; p += kSegThreads) *at(h * T + p) = s[p];
        __syncthreads();
    }
    // Phase 2^16, step j = 2^15: ascending (bit 16 of every index is 0).
    for (uint32_t i = tid; i < T; i += kSegThreads) {
        uint32_t *pa = at(i);
        uint32_t *pb = at(i + T);
        const uint32_t a = *pa;
        const uint32_t b = *pb;
        if (b < a) {
            *pa = b;
            *pb = a;
        }
    }
    __syncthreads();
    // Phase 2^16, steps j = 2^14 .. 1 on each half; padding stays at the end.
    for (uint32_t h = 0; h < 2; ++h) {
        for (uint32_t p = tid; p < T; p += kSegThreads) s[p] = *at(h * T + p);
        __syncthreads();
        lds_network<uint32_t, MELD_LO, MELD_HI, kSegThreads, true>(
            s, T, h * T, kSegLogTile + 1, kSegLogTile + 1, kSegLogTile - 1, -1, tid);
        __syncthreads();
        for (uint32_t p = tid; p < T && h * T + p < len; p += kSegThreads)
            keys[lo + h * T + p] = s[p];
        __syncthreads();
    }
}

// One wave sorts one segment of 2..128 keys in its own 128-word LDS slot.
template <bool MELD_LO, bool MELD_HI>
__device__ void sort_small(uint32_t *__restrict__ keys, uint32_t *ws, uint32_t lo, uint32_t len,
                           uint32_t lane) {
    const uint32_t m = ceil_log2(len);
    const uint32_t P = 1u << m;
    if (lane < P) ws[lane] = lane < len ? keys[lo + lane] : kPad;
    if (lane + 64 < P) ws[lane + 64] = lane + 64 < len ? keys[lo + lane + 64] : kPad;
    wave_lds_sync();
    lds_network<uint32_t, MELD_LO, MELD_HI, 64, false>(ws, P, 0, 1, m, 0, -1, lane);
    if (lane < len) keys[lo + lane] = ws[lane];
    if (lane + 64 < len) keys[lo + lane + 64] = ws[lane + 64];
}

template <bool MELD_LO, bool MELD_HI>
__global__ __launch_bounds__(kSegThreads) void seg_sort_kernel(uint32_t *__restrict__ keys,
                                                               const uint32_t *__restrict__ off,
                                                               const uint32_t *__restrict__ queue,
                                                               SegState *st,
                                                               uint32_t *__restrict__ pad_all) {
    extern __shared__ __align__(16) uint32_t s[];
    __shared__ uint32_t item_sh;
    if (st->flag != 0) return;  // invalid offsets: leave the keys untouched
    const uint32_t n_items = st->n_items;
    const uint32_t n_big = st->n_big;
    const uint32_t n_small = st->n_small;
    uint32_t *pad = pad_all + (size_t)blockIdx.x * kSegTile;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) item_sh = atomicAdd(&st->head, 1u);
        __syncthreads();
        const uint32_t item = item_sh;
        __syncthreads();
        if (item >= n_items) break;  // every wave of every workgroup reaches this
        if (item < n_big) {
            const uint32_t seg = queue[item];
            const uint32_t lo = off[seg];
            const uint32_t len = off[seg + 1] - lo;
            const uint32_t m = ceil_log2(len);
            if (m <= kSegLogTile)
                sort_in_lds<MELD_LO, MELD_HI>(keys, s, lo, len, m);
            else
                sort_two_halves<MELD_LO, MELD_HI>(keys, s, pad, lo, len);
        } else {
            const uint32_t w = tid >> 6;
            const uint32_t qi = n_big + (item - n_big) * kWavesPerBlock + w;
            if (qi < n_big + n_small) {
                const uint32_t seg = queue[qi];
                const uint32_t lo = off[seg];
                sort_small<MELD_LO, MELD_HI>(keys, s + w * kSmallMax, lo, off[seg + 1] - lo,
                                             tid & 63);
            }
            __syncthreads();
        }
    }
}

template <bool LO, bool HI>
hipError_t launch_sort_t(uint32_t *keys, const uint32_t *off, const uint32_t *queue, SegState *st,
                         uint32_t *pad, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL((seg_sort_kernel<LO, HI>), dim3(grid), dim3(kSegThreads),
                       kSegTile * sizeof(uint32_t), stream, keys, off, queue, st, pad);
    return hipGetLastError();
}

template <bool LO, bool HI>
hipError_t allow_big_lds() {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(seg_sort_kernel<LO, HI>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kSegTile * sizeof(uint32_t)));
}

}  // namespace

hipError_t seg_sort_grid(int device, uint32_t *grid) {
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    // The LDS limit is raised for every form up front, outside any capture.
    for (hipError_t r : {allow_big_lds<true, true>(), allow_big_lds<true, false>(),
                         allow_big_lds<false, true>(), allow_big_lds<false, false>()})
        if (r != hipSuccess) return r;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(seg_sort_kernel<true, true>), kSegThreads,
        kSegTile * sizeof(uint32_t));
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    *grid = (uint32_t)(cus * per_cu);
    return hipSuccess;
}

hipError_t launch_segmented_sort(uint32_t *keys, const uint32_t *off, uint32_t nseg,
                                 SegState *st, uint8_t *cls, uint32_t *queue, uint32_t *pad,
                                 uint32_t grid, bool meld_lo, bool meld_hi, hipStream_t stream) {
    if (nseg == 0) return hipSuccess;
    const uint32_t blocks = (nseg + 255) / 256;
    hipLaunchKernelGGL(seg_reset_kernel, dim3(1), dim3(64), 0, stream, st);
    hipLaunchKernelGGL(seg_classify_kernel, dim3(blocks), dim3(256), 0, stream, off, nseg, st,
                       cls);
    hipLaunchKernelGGL(seg_plan_kernel, dim3(1), dim3(64), 0, stream, st);
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(blocks), dim3(256), 0, stream, nseg, cls, st,
                       queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (meld_lo)
        return meld_hi ? launch_sort_t<true, true>(keys, off, queue, st, pad, grid, stream)
                       : launch_sort_t<true, false>(keys, off, queue, st, pad, grid, stream);
    return meld_hi ? launch_sort_t<false, true>(keys, off, queue, st, pad, grid, stream)
                   : launch_sort_t<false, false>(keys, off, queue, st, pad, grid, stream);
}

}  // namespace meld
