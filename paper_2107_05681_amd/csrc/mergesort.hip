// Bottom-up merge sort with a merge-path merge step, the paper's MS benchmark
// (Evaluation section, "Mergesort"): its merge step holds a data-dependent
// divergent region.
//
// A pass merges pairs of sorted runs of length L into runs of 2L (the last
// pair may be ragged or alone). A workgroup of 256 lanes produces 2048
// consecutive outputs: the merge path (Green, McColl and Bader, "GPU Merge
// Path", ICS 2012) gives how many of the first d outputs come from run A for
// the workgroup's two diagonals; the two input slices are staged in LDS; each
// lane finds its own 8-output diagonal the same way and merges sequentially.
// Ties take A first (the merge is stable).
//
// Per output the lane holds the heads of its two slices and
//   divergent: if (A's head is taken) { emit it; load the next A } else
//              { emit B's head; load the next B } — two sides, each with its
//              own LDS load; whether a lane takes A depends on the keys, so
//              waves are mixed at random;
//   melded:    the sides align: the emitted key is selected, one LDS load
//              reads from the selected slice, the heads are updated by
//              selects.
#include "device_common.h"
#include "kernels.h"

namespace meld {

namespace {

constexpr uint32_t kMsThreads = 256;
constexpr uint32_t kMsItems = 8;
constexpr uint32_t kMsTile = kMsThreads * kMsItems;

// Number of A elements among the first d outputs of merging a[0..al) and
// b[0..bl) (A first on ties).
template <typename P>
__device__ __forceinline__ uint32_t merge_path(P a, uint32_t al, P b, uint32_t bl, uint32_t d) {
    uint32_t lo = d > bl ? d - bl : 0;
    uint32_t hi = d < al ? d : al;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= b[d - 1 - mid])
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// merge_path as an 8-way search: 7 probes per round, their 14 loads issued
// together, shrink the range by a factor of 8 (the predicate is monotone,
// so the probes that hold form a prefix). Same result, a third of the
// dependent load rounds.
__device__ __forceinline__ uint32_t merge_path_8way(const uint32_t *__restrict__ a, uint32_t al,
                                                    const uint32_t *__restrict__ b, uint32_t bl,
                                                    uint32_t d) {
    uint32_t lo = d > bl ? d - bl : 0;
    uint32_t hi = d < al ? d : al;
    while (lo < hi) {
        const uint32_t r = hi - lo;
        uint32_t p[7];
        bool f[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) p[j] = lo + (uint32_t)(((uint64_t)r * (j + 1)) >> 3);
#pragma unroll
        for (int j = 0; j < 7; ++j) f[j] = a[p[j]] <= b[d - 1 - p[j]];
        uint32_t nlo = lo, nhi = hi;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            if (f[j]) nlo = p[j] + 1;
            if (!f[j] && nhi == hi) nhi = p[j];
        }
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Cut of every tile (its start diagonal), for the passes whose runs are long
// enough that a workgroup's own search would hold it up (a chain of log2(L)
// dependent global loads before any of its data moves). One lane in
// kCutSpread searches: the scattered probes of a wave go through one CU's
// address path, so few searching lanes per wave spread them over every CU.
constexpr uint32_t kCutSpread = 8;
constexpr uint32_t kCutThreads = 64;

__global__ __launch_bounds__(kCutThreads) void merge_cuts_kernel(const uint32_t *__restrict__ src,
                                                                 uint32_t n, uint32_t log_run,
                                                                 uint32_t n_tiles,
                                                                 uint32_t *__restrict__ cuts) {
    const uint32_t g = blockIdx.x * kCutThreads + threadIdx.x;
    const uint32_t w = g / kCutSpread;
    if (g % kCutSpread != 0 || w >= n_tiles) return;
    const uint32_t o0 = w * kMsTile;
    const uint32_t L = 1u << log_run;
    const uint32_t ps = o0 & ~(2 * L - 1);
    const uint32_t al = n - ps < L ? n - ps : L;
    const uint32_t bl = n - ps > L ? (n - ps - L < L ? n - ps - L : L) : 0;
    cuts[w] = merge_path_8way(src + ps, al, src + ps + al, bl, o0 - ps);
}

// cuts: NULL, or the start cut of every tile (merge_cuts_kernel).
template <bool MELDED>
__global__ __launch_bounds__(kMsThreads) void merge_pass_kernel(const uint32_t *__restrict__ src,
                                                                uint32_t *__restrict__ dst,
                                                                uint32_t n, uint32_t log_run,
                                                                const uint32_t *__restrict__ cuts) {
    __shared__ uint32_t s_in[kMsTile];
    // outputs staged with one pad word per 32: lane t stores its 8 outputs at
    // t*8 + k, which without the pad puts 16 lanes of a store on one bank
    __shared__ uint32_t s_out[kMsTile + kMsTile / 32];
    __shared__ uint32_t s_cut[2];
    const uint32_t t = threadIdx.x;
    const uint32_t o0 = blockIdx.x * kMsTile;  // tiles never straddle a pair: 2L >= kMsTile
    const uint32_t L = 1u << log_run;
    const uint32_t ps = o0 & ~(2 * L - 1);
    const uint32_t al = n - ps < L ? n - ps : L;
    const uint32_t bl = n - ps > L ? (n - ps - L < L ? n - ps - L : L) : 0;
    const uint32_t *A = src + ps;
    const uint32_t *B = src + ps + al;
    const uint32_t d0 = o0 - ps;
    const uint32_t d1 = d0 + kMsTile < al + bl ? d0 + kMsTile : al + bl;
    if (t < 2) {
        // the tile's end cut is the next tile's start cut, or all of A when
        // the tile ends its pair
        const bool last = d1 == al + bl;
        s_cut[t] = t == 1 && last ? al
                   : cuts != nullptr ? cuts[blockIdx.x + t]
                                     : merge_path(A, al, B, bl, t == 0 ? d0 : d1);
    }
    __syncthreads();
    const uint32_t a0 = s_cut[0], a1 = s_cut[1];
    const uint32_t b0 = d0 - a0, b1 = d1 - a1;
    const uint32_t tal = a1 - a0, tbl = b1 - b0;  // slices: s_in[0..tal) and s_in[tal..tal+tbl)
#pragma unroll
    for (uint32_t k = 0; k < kMsItems; ++k) {
        const uint32_t q = t + k * kMsThreads;
        if (q < tal + tbl) s_in[q] = q < tal ? A[a0 + q] : B[b0 + (q - tal)];
    }
    __syncthreads();
    const uint32_t *sa = s_in;
    const uint32_t *sb = s_in + tal;
    const uint32_t count = tal + tbl;
    const uint32_t dt = t * kMsItems < count ? t * kMsItems : count;
    uint32_t ai = merge_path(sa, tal, sb, tbl, dt);
    uint32_t bi = dt - ai;
    uint32_t ha = ai < tal ? sa[ai] : 0, hb = bi < tbl ? sb[bi] : 0;
    uint32_t out[kMsItems];
#pragma unroll
    for (uint32_t k = 0; k < kMsItems; ++k) {
        const bool take_a = ai < tal && (bi >= tbl || ha <= hb);
        if constexpr (MELDED) {
            out[k] = take_a ? ha : hb;
            const uint32_t nx = take_a ? ai + 1 : bi + 1;
            const uint32_t lim = take_a ? tal : tbl;
            const uint32_t v = nx < lim ? s_in[(take_a ? 0 : tal) + nx] : 0;
            ha = take_a ? v : ha;
            hb = take_a ? hb : v;
            ai += take_a ? 1 : 0;
            bi += take_a ? 0 : 1;
        } else {
            if (take_a) {
                MELD_SIDE_MARK("take a");
                out[k] = ha;
                ++ai;
                ha = ai < tal ? sa[ai] : 0;
            } else {
                MELD_SIDE_MARK("take b");
                out[k] = hb;
                ++bi;
                hb = bi < tbl ? sb[bi] : 0;
            }
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < kMsItems; ++k) {
        const uint32_t q = t * kMsItems + k;
        if (q < count) s_out[q + (q >> 5)] = out[k];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kMsItems; ++k) {
        const uint32_t q = t + k * kMsThreads;
        if (q < count) dst[o0 + q] = s_out[q + (q >> 5)];
    }
}

}  // namespace

uint32_t merge_pass_cut_words(uint32_t n) { return blocks_for(n, kMsTile); }

hipError_t launch_merge_pass(const uint32_t *src, uint32_t *dst, uint32_t n, uint32_t log_run,
                             bool melded, uint32_t *cuts, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    if ((2u << log_run) < kMsTile) return hipErrorInvalidValue;
    const uint32_t blocks = blocks_for(n, kMsTile);
    // A separate cut kernel pays off once the grid is several times what the
    // chip holds at once (each workgroup's own search then delays every
    // later wave of workgroups) and the runs are long (deep searches).
    if (log_run < kMergeCutLog || blocks <= kMergeCutMinTiles) cuts = nullptr;
    if (cuts != nullptr)
        hipLaunchKernelGGL(merge_cuts_kernel,
                           dim3((blocks * kCutSpread + kCutThreads - 1) / kCutThreads),
                           dim3(kCutThreads), 0, stream, src, n, log_run, blocks, cuts);
    if (melded)
        hipLaunchKernelGGL(merge_pass_kernel<true>, dim3(blocks), dim3(kMsThreads), 0, stream, src,
                           dst, n, log_run, (const uint32_t *)cuts);
    else
        hipLaunchKernelGGL(merge_pass_kernel<false>, dim3(blocks), dim3(kMsThreads), 0, stream,
                           src, dst, n, log_run, (const uint32_t *)cuts);
    return hipGetLastError();
}

}  // namespace meld
