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

template <bool MELDED>
__global__ __launch_bounds__(kMsThreads) void merge_pass_kernel(const uint32_t *__restrict__ src,
                                                                uint32_t *__restrict__ dst,
                                                                uint32_t n, uint32_t log_run) {
    __shared__ uint32_t s_in[kMsTile];
    __shared__ uint32_t s_out[kMsTile];
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
    if (t < 2) s_cut[t] = merge_path(A, al, B, bl, t == 0 ? d0 : d1);
    __syncthreads();
    const uint32_t a0 = s_cut[0], a1 = s_cut[1];
    const uint32_t b0 = d0 - a0, b1 = d1 - a1;
    const uint32_t tal = a1 - a0, tbl = b1 - b0;  // slices: s_in[0..tal) and s_in[tal..tal+tbl)
    for (uint32_t q = t; q < tal + tbl; q += kMsThreads)
        s_in[q] = q < tal ? A[a0 + q] : B[b0 + (q - tal)];
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
    for (uint32_t k = 0; k < kMsItems; ++k)
        if (t * kMsItems + k < count) s_out[t * kMsItems + k] = out[k];
    __syncthreads();
    for (uint32_t q = t; q < count; q += kMsThreads) dst[o0 + q] = s_out[q];
}

}  // namespace

hipError_t launch_merge_pass(const uint32_t *src, uint32_t *dst, uint32_t n, uint32_t log_run,
                             bool melded, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    if ((2u << log_run) < kMsTile) return hipErrorInvalidValue;
    const uint32_t blocks = (n + kMsTile - 1) / kMsTile;
    if (melded)
        hipLaunchKernelGGL(merge_pass_kernel<true>, dim3(blocks), dim3(kMsThreads), 0, stream, src,
                           dst, n, log_run);
    else
        hipLaunchKernelGGL(merge_pass_kernel<false>, dim3(blocks), dim3(kMsThreads), 0, stream,
                           src, dst, n, log_run);
    return hipGetLastError();
}

}  // namespace meld
