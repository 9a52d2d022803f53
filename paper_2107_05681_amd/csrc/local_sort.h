// Local tile sort of the bitonic network: phases k = 2 .. T of every tile of
// T = 2^L elements, 16 elements per thread in registers, in the two forms of
// the direction region and on the two low-phase paths. Each path is compiled
// in a translation unit of its own (bitonic_local_xch.hip,
// bitonic_local_lds.hip): with every window base a compile-time constant the
// kernels are long, and the two build in parallel.
#pragma once

#include "tile_regs.h"

namespace meld {

namespace {

// One register step on register bit Q in the two forms of the direction
// region. Divergent: Figure 1's if/else on the direction, each side with its
// own compare and conditional swap (the marks keep the sides apart). Melded:
// both compares, the swap chosen by a select on the direction.
template <int Q, bool MELDED, typename E>
__device__ __forceinline__ void reg_step_form(E (&e)[kMergeE], bool up) {
    if constexpr (MELDED) {
        merge_reg_step<Q>(e, up);
    } else {
        if (up) {
            MELD_SIDE_MARK("ascending regs");
#pragma unroll
            for (int r = 0; r < kMergeE; ++r)
                if ((r & (1 << Q)) == 0) {
                    const E x = e[r], y = e[r | (1 << Q)];
                    if (y < x) {
                        e[r] = y;
                        e[r | (1 << Q)] = x;
                    }
                }
        } else {
            MELD_SIDE_MARK("descending regs");
#pragma unroll
            for (int r = 0; r < kMergeE; ++r)
                if ((r & (1 << Q)) == 0) {
                    const E x = e[r], y = e[r | (1 << Q)];
                    if (y > x) {
                        e[r] = y;
                        e[r | (1 << Q)] = x;
                    }
                }
        }
    }
}

// Steps on register bits hi_q .. 0 of the current window, while steps are left.
template <bool MELDED, typename E>
__device__ __forceinline__ void reg_steps(E (&e)[kMergeE], int hi_q, bool up, int32_t &left) {
    if (hi_q >= 3 && left > 0) {
        reg_step_form<3, MELDED>(e, up);
        --left;
    }
    if (hi_q >= 2 && left > 0) {
        reg_step_form<2, MELDED>(e, up);
        --left;
    }
    if (hi_q >= 1 && left > 0) {
        reg_step_form<1, MELDED>(e, up);
        --left;
    }
    if (left > 0) {
        reg_step_form<0, MELDED>(e, up);
        --left;
    }
}

// Phases 2^M .. 2^L of the lane-exchange path with every window base known at
// compile time, so that each LDS access of a window move has an immediate
// offset (with run-time bases, every element's offset costs scalar
// arithmetic and a vector add). Phase M starts and ends in layout W0; TOP is
// the highest step bit left in the phase and PREV the layout e is in. Four-bit
// windows while TOP is at least 7, then W0, where the steps on element bits
// 6, 5 and 4 are lane exchanges (lane t ^ 4, t ^ 2, t ^ 1): phase 2^7 needs no
// transpose at all and phase 2^11 one fewer.
template <int L, bool MELD_HI, int TOP, int PREV, typename E>
__device__ __forceinline__ void xch_phase_windows(E (&e)[kMergeE], E *s, uint32_t t, bool up,
                                                  int32_t &left) {
    if constexpr (TOP >= 7) {
        constexpr int B = TOP - 3;
        merge_transpose<L, PREV, B>(e, s, t);
        reg_steps<MELD_HI>(e, 3, up, left);
        xch_phase_windows<L, MELD_HI, B - 1, B>(e, s, t, up, left);
    } else {
        if constexpr (PREV != 0) merge_transpose<L, PREV, 0>(e, s, t);
        if constexpr (TOP >= 6) {
            if (left > 0) {
                lane_step<2, MELD_HI>(e, up, ((t >> 2) & 1u) == 0);
                --left;
            }
        }
        if constexpr (TOP >= 5) {
            if (left > 0) {
                lane_step<1, MELD_HI>(e, up, ((t >> 1) & 1u) == 0);
                --left;
            }
        }
        if constexpr (TOP >= 4) {
            if (left > 0) {
                lane_step<0, MELD_HI>(e, up, (t & 1u) == 0);
                --left;
            }
        }
        reg_steps<MELD_HI>(e, TOP < 3 ? TOP : 3, up, left);
    }
}

template <int L, bool MELD_HI, int M, typename E>
__device__ __forceinline__ void xch_phases(E (&e)[kMergeE], E *s, uint32_t t, uint32_t base,
                                           int32_t &left) {
    if constexpr (M <= L) {
        const bool up = (((base >> M) | (t >> (M - 4))) & 1u) == 0;
        xch_phase_windows<L, MELD_HI, M - 1, 0>(e, s, t, up, left);
        xch_phases<L, MELD_HI, M + 1>(e, s, t, base, left);
    }
}

// The same for the LDS path's phases 2^M .. 2^L: windows with bases M-4,
// M-8, ... (clamped at 0), window W taking steps on bits M-4(W-1)-1 .. B.
template <int L, bool MELD_HI, int M, int W, int PREV, typename E>
__device__ __forceinline__ void lds_phase_windows(E (&e)[kMergeE], E *s, uint32_t t, bool up,
                                                  int32_t &left) {
    constexpr int B = M > 4 * W ? M - 4 * W : 0;
    constexpr int HI_Q = M - 4 * (W - 1) - 1 - B;
    if constexpr (PREV != B) merge_transpose<L, PREV, B>(e, s, t);
    reg_steps<MELD_HI>(e, HI_Q, up, left);
    if constexpr (B != 0) lds_phase_windows<L, MELD_HI, M, W + 1, B>(e, s, t, up, left);
}

template <int L, bool MELD_HI, int M, int PREV, typename E>
__device__ __forceinline__ void lds_phases(E (&e)[kMergeE], E *s, uint32_t t, uint32_t base,
                                           int32_t &left) {
    if constexpr (M <= L) {
        const bool up = (((base >> M) | (t >> (M - 4))) & 1u) == 0;
        lds_phase_windows<L, MELD_HI, M, 1, PREV>(e, s, t, up, left);
        lds_phases<L, MELD_HI, M + 1, 0>(e, s, t, base, left);
    }
}

// The whole network of a tile of T = 2^L elements (phases k = 2 .. T; the
// last one's direction is bit L of the tile's base).
//
// XCH = false: phases k <= 64 run as the LDS comparator network, one
// comparator per lane per iteration (Figure 1's mapping), in form MELD_LO:
// their direction is a lane bit of the comparator index. Phases k = 2^m >= 128
// run in register windows: for phase m the windows have bases m-4, m-8, ...
// (clamped at 0), each taking four of the steps on bits m-1 .. 0.
//
// XCH = true: the tile goes to layout W0 (register r of thread t holds
// element 16 t + r) and phases k <= 64 run in registers with DPP lane
// exchanges for the steps on element bits 4 and 5 (xch_network_low): no LDS
// access at all. Phases 2^1 .. 2^3 then have a direction fixed per register
// and phases 2^4 .. 2^6 one from a lane bit; form MELD_LO decides how those
// run. Phases m >= 7 take windows with bases m-4, m-8, ... while their top
// step bit is at least 7 and end in W0, where the steps on bits 6, 5 and 4
// are lane exchanges (phase 2^7 runs in W0 alone).
//
// In window B element bit m (>= B+4) is thread bit m-4, so the direction is
// the same for all of a thread's elements and, for m <= 9, differs between
// the lanes of a wave: form MELD_HI decides how that region runs.
template <bool PAIRS, int L, bool MELD_LO, bool MELD_HI, bool XCH>
__global__ __launch_bounds__(1 << (L - 4)) void bitonic_sort_regs_kernel(SortArray a, int mode,
                                                                         int32_t step_limit) {
    using E = typename ElemOf<PAIRS>::type;
    constexpr uint32_t NT = 1u << (L - 4);
    constexpr uint32_t T = 1u << L;
    extern __shared__ __align__(16) unsigned char smem[];
    E *s = reinterpret_cast<E *>(smem);
    const uint32_t t = threadIdx.x;
    const uint32_t base = blockIdx.x * T;

    const TileMap<L, L> map{base, (uint32_t)L};
    E e[kMergeE];
    regs_load<PAIRS, L, L>(a, map, t, mode, e);
    if constexpr (XCH) {
        merge_transpose<L, -1, 0>(e, s, t);
        const int32_t lo_steps = xch_network_low<MELD_LO>(e, t, step_limit);
        int32_t left = step_limit < 0 ? 0x7FFFFFFF : step_limit - lo_steps;
        xch_phases<L, MELD_HI, 7>(e, s, t, base, left);
    } else {
#pragma unroll
        for (int r = 0; r < kMergeE; ++r) s[low_swz<E, PAIRS>(merge_index<L, -1>(t, r))] = e[r];  // natural order
        __syncthreads();
        const int32_t lo_steps = lds_network_low<E, MELD_LO, 8, PAIRS>(s, base, 6, t, NT, step_limit);
        __syncthreads();
        int32_t left = step_limit < 0 ? 0x7FFFFFFF : step_limit - lo_steps;

        // Phase 2^7 starts in window 3 (element bits 3..6), read from the natural
        // order the comparator network leaves in s.
        {
            const uint32_t tb = window_tpart(t, 3);
#pragma unroll
            for (int r = 0; r < kMergeE; ++r) e[r] = s[low_swz<E, PAIRS>(tb | ((uint32_t)r << 3))];
            __syncthreads();
        }
        lds_phases<L, MELD_HI, 7, 3>(e, s, t, base, left);
    }
    regs_store<PAIRS, L, L, 0>(a, s, map, t, mode, e);
}

template <bool PAIRS, int L, bool LO, bool HI, bool XCH>
hipError_t launch_sort_regs_f(const SortArray &a, uint32_t n_tiles, int32_t step_limit,
                              int io_mode, hipStream_t stream) {
    const size_t lds = regs_lds_bytes<PAIRS, L>();
    auto kern = bitonic_sort_regs_kernel<PAIRS, L, LO, HI, XCH>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(1u << (L - 4)), lds, stream, a, io_mode,
                       step_limit);
    return hipGetLastError();
}

template <bool PAIRS, int L, bool XCH>
hipError_t launch_sort_regs_x(const SortArray &a, uint32_t n_tiles, int32_t step_limit, bool lo,
                              bool hi, int io_mode, hipStream_t stream) {
    if (lo)
        return hi ? launch_sort_regs_f<PAIRS, L, true, true, XCH>(a, n_tiles, step_limit, io_mode,
                                                                  stream)
                  : launch_sort_regs_f<PAIRS, L, true, false, XCH>(a, n_tiles, step_limit,
                                                                   io_mode, stream);
    return hi ? launch_sort_regs_f<PAIRS, L, false, true, XCH>(a, n_tiles, step_limit, io_mode,
                                                               stream)
              : launch_sort_regs_f<PAIRS, L, false, false, XCH>(a, n_tiles, step_limit, io_mode,
                                                                stream);
}

template <bool PAIRS, bool XCH>
hipError_t launch_sort_regs_p(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                              int32_t step_limit, bool lo, bool hi, int io_mode,
                              hipStream_t stream) {
#define MELD_CASE(L) \
    case L:          \
        return launch_sort_regs_x<PAIRS, L, XCH>(a, n_tiles, step_limit, lo, hi, io_mode, stream);
    switch (log_t) {
        MELD_REGS_SIZES(MELD_CASE)
        default: return hipErrorInvalidValue;
    }
#undef MELD_CASE
}

// The local sort of every tile on one low-phase path (XCH: lane exchanges).
template <bool XCH>
hipError_t launch_sort_regs_path(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                                 int32_t step_limit, bool meld_lo, bool meld_hi, int io_mode,
                                 hipStream_t stream) {
    if (n_tiles == 0 || step_limit == 0) return hipSuccess;
    if (io_mode == kPlain) io_mode = kTail;  // no tail workspace: every tile is below n
    if (a.vals != nullptr)
        return launch_sort_regs_p<true, XCH>(a, log_t, n_tiles, step_limit, meld_lo, meld_hi,
                                             io_mode, stream);
    return launch_sort_regs_p<false, XCH>(a, log_t, n_tiles, step_limit, meld_lo, meld_hi,
                                          io_mode, stream);
}

}  // namespace

}  // namespace meld
