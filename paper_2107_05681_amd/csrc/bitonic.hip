// Bitonic sort network (the paper's running example, Motivating Example
// section, Figure 1): divergent and melded compare-exchange, LDS tiles and
// register-resident streaming passes.
//
// Network: phases k = 2, 4, ..., N; steps j = k/2, ..., 1. Step (k, j) pairs
// element lo with hi = lo + j for every lo whose bit j is clear; the pair is
// put in ascending order when bit k of lo is clear and in descending order
// otherwise, with strict compares (equal elements are never swapped). Pairs
// of u32 (key, payload) are compared as the 64-bit composite key:payload.
//
// Tile kernel: one workgroup owns a tile of T = 2^log_t consecutive
// elements in LDS and runs a range of steps on it; each lane takes one
// comparator c per iteration (lo = c with a zero bit inserted at bit j).
// The direction of a comparator is bit k of lo, i.e. bit k-1 of c; for
// k <= 64 that is one of the six lane bits, so the direction branch is
// divergent inside every wave. That is the region the two forms differ in:
//
//   divergent (Figure 1 as written): if (up) { a = s[lo]; b = s[hi];
//       if (b < a) swap } else { a = s[lo]; b = s[hi]; if (b > a) swap }
//   melded (the paper's melded bitonic, "Putting All Together"): the loads
//       of the two sides align with identical operands and become one load
//       pair; the two compares do not align and both run; the branch
//       condition of the swap is select(up, b < a, b > a); the swap stores
//       align with identical operands and become one store pair.
//
// Steps with j >= 128 exchange data between waves and end with a workgroup
// barrier. For j <= 64 the 64 comparators of a wave (one iteration) touch
// only the 128-element block [2*c0, 2*c0 + 128) of their first comparator
// c0, the same block in every such step, so those steps need only the wave's
// own LDS operations to have completed.
//
// Streaming pass: for steps whose j is at least the tile size every thread
// loads the 2^R elements that differ only in bits b_lo .. b_hi (R = b_hi -
// b_lo + 1) and runs the R steps in registers. The direction bit k lies above
// b_hi, so it is the same for all of a thread's elements and, because the
// low bits of the index come from the lane, for the whole wave: both forms
// coincide there and a single kernel serves them.
#include "device_common.h"
#include "kernels.h"
#include "network.h"

namespace meld {

namespace {

constexpr uint32_t kPadValue = 0xFFFFFFFFu;  // value of every position >= n

template <bool PAIRS>
struct ElemOf {
    using type = uint32_t;
};
template <>
struct ElemOf<true> {
    using type = uint64_t;
};

// Where the elements of a launch live:
//   kPlain     every position is below n: direct loads and stores.
//   kPlainVec  as kPlain, with 16-byte aligned arrays: tiles move 4 elements
//              per lane per access.
//   kTail      positions >= n live in the tail workspace: the address is
//              selected per element (no branch).
//   kSentinel  positions >= n read as the sentinel and are never stored
//              (a single tile padded in LDS).
enum IoMode { kPlain = kIoPlain, kPlainVec = kIoPlainVec, kTail = kIoTail, kSentinel = kIoSentinel };

template <int MODE>
__device__ __forceinline__ uint32_t ld_u32(const uint32_t *main, const uint32_t *tail, uint32_t n,
                                           uint32_t p) {
    if constexpr (MODE == kTail) {
        const uint32_t *src = p < n ? main + p : tail + (p - n);
        return *src;
    } else if constexpr (MODE == kSentinel) {
        return p < n ? main[p] : kPadValue;
    } else {
        return main[p];
    }
}

template <int MODE>
__device__ __forceinline__ void st_u32(uint32_t *main, uint32_t *tail, uint32_t n, uint32_t p,
                                       uint32_t v) {
    if constexpr (MODE == kTail) {
        uint32_t *dst = p < n ? main + p : tail + (p - n);
        *dst = v;
    } else if constexpr (MODE == kSentinel) {
        if (p < n) main[p] = v;
    } else {
        main[p] = v;
    }
}

template <bool PAIRS, int MODE>
__device__ __forceinline__ typename ElemOf<PAIRS>::type load_elem(const SortArray &a, uint32_t p) {
    const uint32_t k = ld_u32<MODE>(a.keys, a.tk, a.n, p);
    if constexpr (PAIRS) {
        const uint32_t v = ld_u32<MODE>(a.vals, a.tv, a.n, p);
        return ((uint64_t)k << 32) | v;
    } else {
        return k;
    }
}

template <bool PAIRS, int MODE>
__device__ __forceinline__ void store_elem(const SortArray &a, uint32_t p,
                                           typename ElemOf<PAIRS>::type e) {
    if constexpr (PAIRS) {
        st_u32<MODE>(a.keys, a.tk, a.n, p, (uint32_t)(e >> 32));
        st_u32<MODE>(a.vals, a.tv, a.n, p, (uint32_t)e);
    } else {
        st_u32<MODE>(a.keys, a.tk, a.n, p, e);
    }
}

// Moves tile [base, base + T) between global memory and LDS.
template <bool PAIRS, int MODE, int NT>
__device__ __forceinline__ void tile_load(const SortArray &a, typename ElemOf<PAIRS>::type *s,
                                          uint32_t base, uint32_t T) {
    using E = typename ElemOf<PAIRS>::type;
    if constexpr (MODE == kPlainVec) {
        for (uint32_t p = threadIdx.x * 4; p < T; p += NT * 4) {
            const uint4 k = *reinterpret_cast<const uint4 *>(a.keys + base + p);
            if constexpr (PAIRS) {
                const uint4 v = *reinterpret_cast<const uint4 *>(a.vals + base + p);
                s[p + 0] = ((E)k.x << 32) | v.x;
                s[p + 1] = ((E)k.y << 32) | v.y;
                s[p + 2] = ((E)k.z << 32) | v.z;
                s[p + 3] = ((E)k.w << 32) | v.w;
            } else {
                *reinterpret_cast<uint4 *>(s + p) = k;
            }
        }
    } else {
        for (uint32_t p = threadIdx.x; p < T; p += NT) s[p] = load_elem<PAIRS, MODE>(a, base + p);
    }
}

template <bool PAIRS, int MODE, int NT>
__device__ __forceinline__ void tile_store(const SortArray &a,
                                           const typename ElemOf<PAIRS>::type *s, uint32_t base,
                                           uint32_t T) {
    if constexpr (MODE == kPlainVec) {
        for (uint32_t p = threadIdx.x * 4; p < T; p += NT * 4) {
            if constexpr (PAIRS) {
                const uint64_t e0 = s[p], e1 = s[p + 1], e2 = s[p + 2], e3 = s[p + 3];
                *reinterpret_cast<uint4 *>(a.keys + base + p) =
                    make_uint4((uint32_t)(e0 >> 32), (uint32_t)(e1 >> 32), (uint32_t)(e2 >> 32),
                               (uint32_t)(e3 >> 32));
                *reinterpret_cast<uint4 *>(a.vals + base + p) =
                    make_uint4((uint32_t)e0, (uint32_t)e1, (uint32_t)e2, (uint32_t)e3);
            } else {
                *reinterpret_cast<uint4 *>(a.keys + base + p) =
                    *reinterpret_cast<const uint4 *>(s + p);
            }
        }
    } else {
        for (uint32_t p = threadIdx.x; p < T; p += NT) store_elem<PAIRS, MODE>(a, base + p, s[p]);
    }
}

template <bool PAIRS, bool MELD_LO, bool MELD_HI, int NT, int MODE>
__global__ __launch_bounds__(NT) void bitonic_tile_kernel(SortArray a, uint32_t log_t,
                                                          uint32_t m_begin, uint32_t m_end,
                                                          uint32_t j_first, int32_t step_limit) {
    using E = typename ElemOf<PAIRS>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    E *s = reinterpret_cast<E *>(smem);
    const uint32_t T = 1u << log_t;
    const uint32_t base = blockIdx.x << log_t;

    const bool below_n = MODE == kTail && base + T <= a.n;  // uniform per workgroup
    if (below_n)
        tile_load<PAIRS, kPlain, NT>(a, s, base, T);
    else
        tile_load<PAIRS, MODE, NT>(a, s, base, T);
    __syncthreads();
    lds_network<E, MELD_LO, MELD_HI, NT, true>(s, T, base, m_begin, m_end, j_first, step_limit,
                                              threadIdx.x);
    __syncthreads();
    if (below_n)
        tile_store<PAIRS, kPlain, NT>(a, s, base, T);
    else
        tile_store<PAIRS, MODE, NT>(a, s, base, T);
}

template <typename E>
__device__ __forceinline__ void cex_regs(E &x, E &y, bool up) {
    const E mn = x < y ? x : y;
    const E mx = x < y ? y : x;
    x = up ? mn : mx;
    y = up ? mx : mn;
}

constexpr int kGlobalThreads = 256;

template <bool PAIRS, int R, int MODE>
__global__ __launch_bounds__(kGlobalThreads) void bitonic_global_kernel(SortArray a,
                                                                      uint32_t n_threads,
                                                                      uint32_t m, uint32_t b_lo,
                                                                      int32_t nsteps) {
    using E = typename ElemOf<PAIRS>::type;
    const uint32_t t = blockIdx.x * kGlobalThreads + threadIdx.x;
    if (t >= n_threads) return;
    const uint32_t low = t & ((1u << b_lo) - 1);
    const uint32_t base = ((t >> b_lo) << (b_lo + R)) | low;
    const bool up = ((base >> m) & 1u) == 0;
    E e[1 << R];
#pragma unroll
    for (int q = 0; q < (1 << R); ++q)
        e[q] = load_elem<PAIRS, MODE>(a, base + ((uint32_t)q << b_lo));
#pragma unroll
    for (int s = R - 1; s >= 0; --s) {
        if (R - 1 - s < nsteps) {
#pragma unroll
            for (int q = 0; q < (1 << R); ++q)
                if ((q & (1 << s)) == 0) cex_regs(e[q], e[q | (1 << s)], up);
        }
    }
#pragma unroll
    for (int q = 0; q < (1 << R); ++q)
        store_elem<PAIRS, MODE>(a, base + ((uint32_t)q << b_lo), e[q]);
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t value, size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

template <bool PAIRS, bool LO, bool HI, int NT, int MODE>
hipError_t launch_tile_m(const SortArray &a, uint32_t log_t, uint32_t n_tiles, uint32_t m_begin,
                         uint32_t m_end, uint32_t j_first, int32_t step_limit,
                         hipStream_t stream) {
    using E = typename ElemOf<PAIRS>::type;
    const size_t lds = ((size_t)1 << log_t) * sizeof(E);
    auto kern = bitonic_tile_kernel<PAIRS, LO, HI, NT, MODE>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(NT), lds, stream, a, log_t, m_begin, m_end,
                       j_first, step_limit);
    return hipGetLastError();
}

template <bool PAIRS, bool LO, bool HI, int NT>
hipError_t launch_tile_t(const SortArray &a, uint32_t log_t, uint32_t n_tiles, uint32_t m_begin,
                         uint32_t m_end, uint32_t j_first, int32_t step_limit, int io_mode,
                         hipStream_t stream) {
#define MELD_TILE_MODE(M)                                                                    \
    case M:                                                                                  \
        return launch_tile_m<PAIRS, LO, HI, NT, M>(a, log_t, n_tiles, m_begin, m_end, j_first, \
                                                   step_limit, stream);
    switch (io_mode) {
        MELD_TILE_MODE(kPlain)
        MELD_TILE_MODE(kPlainVec)
        MELD_TILE_MODE(kTail)
        MELD_TILE_MODE(kSentinel)
        default:
            return hipErrorInvalidValue;
    }
#undef MELD_TILE_MODE
}

template <bool PAIRS, bool LO, bool HI>
hipError_t launch_tile_nt(const SortArray &a, uint32_t log_t, uint32_t n_tiles, uint32_t m_begin,
                          uint32_t m_end, uint32_t j_first, int32_t step_limit, int io_mode,
                          int threads, hipStream_t stream) {
    switch (threads) {
        case 64:
            return launch_tile_t<PAIRS, LO, HI, 64>(a, log_t, n_tiles, m_begin, m_end, j_first,
                                                    step_limit, io_mode, stream);
        case 256:
            return launch_tile_t<PAIRS, LO, HI, 256>(a, log_t, n_tiles, m_begin, m_end, j_first,
                                                     step_limit, io_mode, stream);
        case 512:
            return launch_tile_t<PAIRS, LO, HI, 512>(a, log_t, n_tiles, m_begin, m_end, j_first,
                                                     step_limit, io_mode, stream);
        default:
            return hipErrorInvalidValue;
    }
}

template <bool PAIRS>
hipError_t launch_tile_p(const SortArray &a, uint32_t log_t, uint32_t n_tiles, uint32_t m_begin,
                         uint32_t m_end, uint32_t j_first, int32_t step_limit, bool lo, bool hi,
                         int io_mode, int threads, hipStream_t stream) {
    if (lo)
        return hi ? launch_tile_nt<PAIRS, true, true>(a, log_t, n_tiles, m_begin, m_end, j_first,
                                                      step_limit, io_mode, threads, stream)
                  : launch_tile_nt<PAIRS, true, false>(a, log_t, n_tiles, m_begin, m_end,
                                                       j_first, step_limit, io_mode, threads,
                                                       stream);
    return hi ? launch_tile_nt<PAIRS, false, true>(a, log_t, n_tiles, m_begin, m_end, j_first,
                                                   step_limit, io_mode, threads, stream)
              : launch_tile_nt<PAIRS, false, false>(a, log_t, n_tiles, m_begin, m_end, j_first,
                                                    step_limit, io_mode, threads, stream);
}

template <bool PAIRS, int R, int MODE>
hipError_t launch_global_r(const SortArray &a, uint32_t log_n, uint32_t m, uint32_t b_lo,
                           int32_t step_limit, hipStream_t stream) {
    const uint32_t n_threads = 1u << (log_n - R);
    const uint32_t blocks = (n_threads + kGlobalThreads - 1) / kGlobalThreads;
    hipLaunchKernelGGL((bitonic_global_kernel<PAIRS, R, MODE>), dim3(blocks),
                       dim3(kGlobalThreads), 0, stream, a, n_threads, m, b_lo,
                       step_limit < 0 ? R : step_limit);
    return hipGetLastError();
}

template <bool PAIRS, int MODE>
hipError_t launch_global_p(const SortArray &a, uint32_t log_n, uint32_t m, uint32_t b_hi,
                           uint32_t b_lo, int32_t step_limit, hipStream_t stream) {
    switch (b_hi - b_lo + 1) {
        case 1: return launch_global_r<PAIRS, 1, MODE>(a, log_n, m, b_lo, step_limit, stream);
        case 2: return launch_global_r<PAIRS, 2, MODE>(a, log_n, m, b_lo, step_limit, stream);
        case 3: return launch_global_r<PAIRS, 3, MODE>(a, log_n, m, b_lo, step_limit, stream);
        case 4: return launch_global_r<PAIRS, 4, MODE>(a, log_n, m, b_lo, step_limit, stream);
        case 5: return launch_global_r<PAIRS, 5, MODE>(a, log_n, m, b_lo, step_limit, stream);
        case 6: return launch_global_r<PAIRS, 6, MODE>(a, log_n, m, b_lo, step_limit, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_bitonic_tile(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                               uint32_t m_begin, uint32_t m_end, uint32_t j_first,
                               int32_t step_limit, bool meld_lo, bool meld_hi, int io_mode,
                               int threads, hipStream_t stream) {
    if (n_tiles == 0 || step_limit == 0) return hipSuccess;
    if (io_mode == kPlainVec && log_t < 2) io_mode = kPlain;
    if (a.vals != nullptr)
        return launch_tile_p<true>(a, log_t, n_tiles, m_begin, m_end, j_first, step_limit, meld_lo,
                                   meld_hi, io_mode, threads, stream);
    return launch_tile_p<false>(a, log_t, n_tiles, m_begin, m_end, j_first, step_limit, meld_lo,
                                meld_hi, io_mode, threads, stream);
}

hipError_t launch_bitonic_global(const SortArray &a, uint32_t log_n, uint32_t m, uint32_t b_hi,
                                 uint32_t b_lo, int32_t step_limit, hipStream_t stream) {
    if (step_limit == 0) return hipSuccess;
    const bool tail = a.tk != nullptr;
    if (a.vals != nullptr)
        return tail ? launch_global_p<true, kTail>(a, log_n, m, b_hi, b_lo, step_limit, stream)
                    : launch_global_p<true, kPlain>(a, log_n, m, b_hi, b_lo, step_limit, stream);
    return tail ? launch_global_p<false, kTail>(a, log_n, m, b_hi, b_lo, step_limit, stream)
                : launch_global_p<false, kPlain>(a, log_n, m, b_hi, b_lo, step_limit, stream);
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    const int threads = 256;
    const size_t blocks = (count + threads - 1) / threads;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks), dim3(threads), 0, stream, p,
                       value, count);
    return hipGetLastError();
}

}  // namespace meld
