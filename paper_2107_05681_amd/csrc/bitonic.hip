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
#include "tile_regs.h"

namespace meld {

namespace {

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

// Workgroup order of the streaming passes. Consecutive workgroups go to
// the eight XCDs in turn, each with its own L2, so tiles that lie next to
// each other in the array would each go to another XCD. xcd_run_index gives
// every XCD runs of 2^RUN consecutive tile indices instead: within each group
// of 8 * 2^RUN workgroups, workgroup b's XCD (b % 8) takes 2^RUN indices in a
// row, and the group as a whole still covers one contiguous range; a
// workgroup in a last, partial group keeps its index (a bijection on
// [0, count)). Merge tails (contiguous tiles) take runs of 16 tiles; the
// tiles of consecutive middle indices of a gathered pass (array bits
// [C, b_lo)) hold neighbouring 2^C-element pieces of every row, and take runs
// of 4 (so each L2 streams 4 * 2^C contiguous elements per row). Both lengths
// were the fastest of those timed on 2^28 pairs (runs of 1 .. 1024 tiles).
constexpr uint32_t kXcdRunLogMerge = 4, kXcdRunLogGather = 2;
template <uint32_t RUN>
__device__ __forceinline__ uint32_t xcd_run_index(uint32_t b, uint32_t count) {
    constexpr uint32_t mask = (8u << RUN) - 1;
    if (b >= (count & ~mask)) return b;
    const uint32_t j = b & mask;
    return (b & ~mask) | ((j & 7u) << RUN) | (j >> 3);
}

// One pass of S steps (on element bits L-1 .. L-S of a tile of 2^L) of
// phase k = 2^m, whose direction bit m lies above the tile's bits. Tile map
// with C low bits: workgroup b's bits fill array bits [C, b_lo) and then
// [b_lo + L - C, ...). Merge tail: S = C = L (contiguous tiles, b_lo = L).
// Gathered streaming pass: C = L - S, so the steps act on array bits
// b_lo .. b_lo + S - 1 and each of the 2^S rows is 2^C contiguous elements.
// Both take their tiles in XCD runs (a gathered pass only where the middle
// index has the bits for them).
template <bool PAIRS, int L, int S, int C>
__global__ __launch_bounds__(1 << (L - 4)) void bitonic_pass_regs_kernel(SortArray a, uint32_t m,
                                                                         uint32_t b_lo, int mode,
                                                                         int32_t nsteps) {
    using E = typename ElemOf<PAIRS>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    E *s = reinterpret_cast<E *>(smem);
    const uint32_t t = threadIdx.x;
    const uint32_t spread = b_lo - C;
    uint32_t b = blockIdx.x;
    if constexpr (S == L)
        b = xcd_run_index<kXcdRunLogMerge>(b, gridDim.x);
    else if (spread >= 3 + kXcdRunLogGather)
        b = xcd_run_index<kXcdRunLogGather>(b, gridDim.x);
    const uint32_t base = ((b & ((1u << spread) - 1)) << C) | ((b >> spread) << (b_lo + L - C));
    const TileMap<L, C> map{base, b_lo};
    const bool up = ((base >> m) & 1u) == 0;

    E e[kMergeE];
    // The tile's loads go out at a raised wave priority: with two workgroups
    // per CU, a workgroup starting its tile then issues ahead of the other's
    // compare-exchange and transpose work, and HBM stays busier.
    __builtin_amdgcn_s_setprio(2);
    regs_load<PAIRS, L, C>(a, map, t, mode, e);
    __builtin_amdgcn_s_setprio(0);
    if (0 < nsteps) merge_reg_step<3>(e, up);                // element bit L-1
    if (S >= 2 && 1 < nsteps) merge_reg_step<2>(e, up);      // element bit L-2
    if constexpr (S == L && merge_uses_xch<L>()) {
        merge_windows_xch<L, L - 3, -1>(e, s, t, up, nsteps);
        regs_store<PAIRS, L, C, 0>(a, s, map, t, mode, e);
    } else {
        merge_windows<L, 1, -1, L - S>(e, s, t, up, nsteps);
        regs_store<PAIRS, L, C, last_layout<L, L - S>()>(a, s, map, t, mode, e);
    }
}

template <bool PAIRS, int L>
hipError_t launch_merge_l(const SortArray &a, uint32_t n_tiles, uint32_t m, int32_t nsteps,
                          int io_mode, hipStream_t stream) {
    const size_t lds = regs_lds_bytes<PAIRS, L>();
    auto kern = bitonic_pass_regs_kernel<PAIRS, L, L, L>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(1u << (L - 4)), lds, stream, a, m, (uint32_t)L,
                       io_mode, nsteps);
    return hipGetLastError();
}

// Gathered streaming pass of R steps over the whole array, in tiles of the
// largest size of the element type (2^13 pairs, 2^14 keys: 64 KiB).
template <bool PAIRS>
constexpr int gather_log() {
    return PAIRS ? kGatherLogPairs : kGatherLogKeys;
}

template <bool PAIRS, int R>
hipError_t launch_gather_r(const SortArray &a, uint32_t log_n, uint32_t m, uint32_t b_lo,
                           int32_t nsteps, int io_mode, hipStream_t stream) {
    constexpr int L = gather_log<PAIRS>();
    constexpr int C = L - R;
    if (log_n < (uint32_t)L || b_lo < (uint32_t)C || b_lo + R > log_n) return hipErrorInvalidValue;
    const size_t lds = regs_lds_bytes<PAIRS, L>();
    auto kern = bitonic_pass_regs_kernel<PAIRS, L, R, C>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(1u << (log_n - L)), dim3(1u << (L - 4)), lds, stream, a, m,
                       b_lo, io_mode, nsteps);
    return hipGetLastError();
}

template <bool PAIRS>
hipError_t launch_merge_p(const SortArray &a, uint32_t log_t, uint32_t n_tiles, uint32_t m,
                          int32_t nsteps, int io_mode, hipStream_t stream) {
#define MELD_CASE(L) \
    case L: return launch_merge_l<PAIRS, L>(a, n_tiles, m, nsteps, io_mode, stream);
    switch (log_t) {
        MELD_REGS_SIZES(MELD_CASE)
        default: return hipErrorInvalidValue;
    }
#undef MELD_CASE
}

constexpr int kGlobalThreads = 256;

// Start of row q (q << b_lo elements into p), computed on the scalar unit
// and kept there: the empty asm hides it from reassociation with the lane's
// offset, so each access is a scalar base plus one 32-bit lane offset. The
// stores compute their row starts again (FRESH: a volatile asm, which the
// compiler cannot merge with the loads' one), rather than keeping 2^R of
// them live across the compare-exchange steps.
// The row start is a global-memory pointer (address space 1): through a
// generic pointer the compiler would emit flat instructions.
typedef __attribute__((address_space(1))) uint32_t global_u32;
template <bool FRESH = false>
__device__ __forceinline__ global_u32 *row_ptr(uint32_t *p, int q, uint32_t b_lo) {
    uint32_t *r = p + ((size_t)q << b_lo);
    if constexpr (FRESH)
        asm volatile("" : "+s"(r));
    else
        asm("" : "+s"(r));
    return (global_u32 *)r;
}

template <bool NT>
__device__ __forceinline__ uint32_t ld4g(const global_u32 *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT>
__device__ __forceinline__ void st4g(global_u32 *p, uint32_t v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <bool PAIRS, int R, int MODE, bool NT>
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
    if constexpr (MODE == kPlain) {
        // Row q of every lane starts at the uniform address keys + (q << b_lo)
        // (a scalar base) and the lane adds its own 32-bit offset: one offset
        // register serves all 2^R rows, where per-element 64-bit addresses
        // kept live from the loads to the stores took 256 VGPRs at R = 6.
#pragma unroll
        for (int q = 0; q < (1 << R); ++q) {
            const uint32_t k = ld4g<NT>(row_ptr(a.keys, q, b_lo) + base);
            if constexpr (PAIRS)
                e[q] = ((E)k << 32) | ld4g<NT>(row_ptr(a.vals, q, b_lo) + base);
            else
                e[q] = k;
        }
    } else {
#pragma unroll
        for (int q = 0; q < (1 << R); ++q)
            e[q] = load_elem<PAIRS, MODE, NT>(a, base + ((uint32_t)q << b_lo));
    }
#pragma unroll
    for (int s = R - 1; s >= 0; --s) {
        if (R - 1 - s < nsteps) {
#pragma unroll
            for (int q = 0; q < (1 << R); ++q)
                if ((q & (1 << s)) == 0) cex_regs(e[q], e[q | (1 << s)], up);
        }
    }
    if constexpr (MODE == kPlain) {
#pragma unroll
        for (int q = 0; q < (1 << R); ++q) {
            if constexpr (PAIRS) {
                st4g<NT>(row_ptr<true>(a.keys, q, b_lo) + base, (uint32_t)(e[q] >> 32));
                st4g<NT>(row_ptr<true>(a.vals, q, b_lo) + base, (uint32_t)e[q]);
            } else {
                st4g<NT>(row_ptr<true>(a.keys, q, b_lo) + base, e[q]);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < (1 << R); ++q)
            store_elem<PAIRS, MODE, NT>(a, base + ((uint32_t)q << b_lo), e[q]);
    }
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
    const int32_t nsteps = step_limit < 0 ? R : step_limit;
    if (a.nt != 0)
        hipLaunchKernelGGL((bitonic_global_kernel<PAIRS, R, MODE, true>), dim3(blocks),
                           dim3(kGlobalThreads), 0, stream, a, n_threads, m, b_lo, nsteps);
    else
        hipLaunchKernelGGL((bitonic_global_kernel<PAIRS, R, MODE, false>), dim3(blocks),
                           dim3(kGlobalThreads), 0, stream, a, n_threads, m, b_lo, nsteps);
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

hipError_t launch_bitonic_sort_regs(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                                    int32_t step_limit, bool meld_lo, bool meld_hi, bool xch,
                                    int io_mode, hipStream_t stream) {
    return xch ? launch_bitonic_sort_regs_xch(a, log_t, n_tiles, step_limit, meld_lo, meld_hi,
                                              io_mode, stream)
               : launch_bitonic_sort_regs_lds(a, log_t, n_tiles, step_limit, meld_lo, meld_hi,
                                              io_mode, stream);
}

hipError_t launch_bitonic_gather(const SortArray &a, uint32_t log_n, uint32_t m, uint32_t b_hi,
                                 uint32_t b_lo, int32_t step_limit, int io_mode,
                                 hipStream_t stream) {
    if (step_limit == 0) return hipSuccess;
    if (io_mode == kPlain) io_mode = kTail;
    if (io_mode != kTail && io_mode != kPlainVec) return hipErrorInvalidValue;
    const int32_t r = (int32_t)(b_hi - b_lo + 1);
    const int32_t nsteps = step_limit < 0 ? r : step_limit;
    if (a.vals != nullptr) {
        switch (r) {
            case 5: return launch_gather_r<true, 5>(a, log_n, m, b_lo, nsteps, io_mode, stream);
            case 6: return launch_gather_r<true, 6>(a, log_n, m, b_lo, nsteps, io_mode, stream);
            case 7: return launch_gather_r<true, 7>(a, log_n, m, b_lo, nsteps, io_mode, stream);
            case 8: return launch_gather_r<true, 8>(a, log_n, m, b_lo, nsteps, io_mode, stream);
            default: return hipErrorInvalidValue;
        }
    }
    switch (r) {
        case 7: return launch_gather_r<false, 7>(a, log_n, m, b_lo, nsteps, io_mode, stream);
        case 8: return launch_gather_r<false, 8>(a, log_n, m, b_lo, nsteps, io_mode, stream);
        case 9: return launch_gather_r<false, 9>(a, log_n, m, b_lo, nsteps, io_mode, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bitonic_merge(const SortArray &a, uint32_t log_t, uint32_t n_tiles, uint32_t m,
                                int32_t step_limit, int io_mode, hipStream_t stream) {
    if (n_tiles == 0 || step_limit == 0) return hipSuccess;
    if (io_mode == kPlain) io_mode = kTail;
    const int32_t nsteps = step_limit < 0 ? (int32_t)log_t : step_limit;
    if (a.vals != nullptr) return launch_merge_p<true>(a, log_t, n_tiles, m, nsteps, io_mode, stream);
    return launch_merge_p<false>(a, log_t, n_tiles, m, nsteps, io_mode, stream);
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
