// Bitonic compare-exchange in LDS: the divergent and melded forms of the
// direction region (Motivating Example, Figure 1; Detailed Design, "Putting
// All Together") and the loop that runs a range of network steps on a tile.
#pragma once

#include "device_common.h"

namespace meld {

// Waits for this wave's LDS operations and keeps the compiler from moving
// memory operations across the point.
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Figure 1's region as written: each side holds its own loads, compare and
// conditional swap.
template <typename E>
__device__ __forceinline__ void cex_divergent(E *s, uint32_t lo, uint32_t hi, bool up) {
    // The marks keep each side's loads and stores inside that side: without
    // them the compiler sinks the two identical swap-store blocks into one,
    // which would already be a (partial) meld.
    if (up) {
        MELD_SIDE_MARK("ascending");
        const E a = s[lo];
        const E b = s[hi];
        if (b < a) {
            s[lo] = b;
            s[hi] = a;
            MELD_SIDE_MARK("ascending swap");
        }
    } else {
        MELD_SIDE_MARK("descending");
        const E a = s[lo];
        const E b = s[hi];
        if (b > a) {
            s[lo] = b;
            s[hi] = a;
            MELD_SIDE_MARK("descending swap");
        }
    }
}

// Swap condition of the melded compare-exchange: select(up, b < a, b > a),
// the two sides' compares chosen by the direction. Written as lane-mask
// operations (the compare's mask flipped for descending lanes, equal elements
// never swap): as a select of two booleans hipcc keeps both compares as 0/1
// values in VGPRs and tests the selected one again, four VALU operations more.
template <typename E>
__device__ __forceinline__ bool melded_swap(E a, E b, bool up) {
    return ((b < a) == up) & (a != b);
}

// The melded region: one load pair, both compares, a select of the swap
// condition, one conditional store pair.
template <typename E>
__device__ __forceinline__ void cex_melded(E *s, uint32_t lo, uint32_t hi, bool up) {
    const E a = s[lo];
    const E b = s[hi];
    if (melded_swap(a, b, up)) {
        s[lo] = b;
        s[hi] = a;
    }
}

// One network step (k = 2^m, j) on the tile: each lane takes comparators
// c = lane0, lane0 + NT, ... below T/2; lo is c with a zero inserted at bit j.
// The direction is bit m of the element's index base | lo.
template <typename E, bool MELDED, int NT>
__device__ __forceinline__ void lds_step(E *s, uint32_t half, uint32_t base, uint32_t m,
                                         uint32_t j, uint32_t lane0) {
    for (uint32_t c = lane0; c < half; c += NT) {
        const uint32_t lo = ((c & ~(j - 1)) << 1) | (c & (j - 1));
        const uint32_t hi = lo + j;
        const bool up = (((base | lo) >> m) & 1u) == 0;
        if constexpr (MELDED)
            cex_melded(s, lo, hi, up);
        else
            cex_divergent(s, lo, hi, up);
    }
}

// Runs the steps of phases m_begin..m_end (phase m_begin from j = 2^j_first,
// the others from j = k/2) on the T-element LDS tile s, at most step_limit
// steps (negative: all). Returns the number of steps run.
//
// MELD_LO selects the form for phases k <= 64, whose direction bit is one of
// the six lane bits of the comparator index (divergent inside a wave);
// MELD_HI for phases k >= 128, whose direction is uniform per wave.
//
// Steps with j >= 128 exchange data between waves: a workgroup barrier
// follows them (BLOCK) — callers with T <= 128 that run one wave per tile
// pass BLOCK = false. For j <= 64, the comparators one wave takes in one
// iteration touch only the 128-element block [2*c0, 2*c0 + 128), the same in
// every such step, so only the wave's own LDS operations need to complete.
template <typename E, bool MELD_LO, bool MELD_HI, int NT, bool BLOCK>
__device__ __forceinline__ int32_t lds_network(E *s, uint32_t T, uint32_t base, uint32_t m_begin,
                                               uint32_t m_end, uint32_t j_first,
                                               int32_t step_limit, uint32_t lane0) {
    const uint32_t half = T >> 1;
    int32_t steps = 0;
    for (uint32_t m = m_begin; m <= m_end; ++m) {
        const uint32_t k = 1u << m;
        for (uint32_t j = (m == m_begin) ? (1u << j_first) : (k >> 1); j > 0; j >>= 1) {
            if (steps == step_limit) return steps;
            ++steps;
            if (k <= 64)
                lds_step<E, MELD_LO, NT>(s, half, base, m, j, lane0);
            else
                lds_step<E, MELD_HI, NT>(s, half, base, m, j, lane0);
            const bool next_crosses_waves = (j >= 128) || (j == 1 && k >= 128);
            if (BLOCK && next_crosses_waves)
                __syncthreads();
            else
                wave_lds_sync();
        }
    }
    return steps;
}

// LDS position of tile element x in the steps of phases k <= 64. With
// comparators dealt to consecutive lanes, the ends of a step j <= 32 that a
// pass of 32 (or 64) lanes touches are the elements of a 64 (128) block whose
// bit j is clear, or set: in natural order two of them share every bank. For
// 4-byte elements, flipping bits 0..4 when bit 5 is set and bit 5 when bit 6
// is set sends them to distinct banks for every j, on 32 and on 64 banks; for
// 8-byte elements the same with bits 4 and 5. A permutation inside each
// 128-element (64 for 8-byte) block; positions of the blocks are unchanged.
// SWZ = false keeps natural order: the ends of a comparator then sit a fixed
// distance apart and pair into one ds_read2 / ds_write2, which the swizzle
// gives up (more instructions, fewer conflicts; it pays for 8-byte pairs and
// for the segmented sort, not for the 2^16-key local sort).
template <typename E, bool SWZ = true>
__device__ __forceinline__ uint32_t low_swz(uint32_t x) {
    if constexpr (!SWZ) return x;
    constexpr uint32_t S = sizeof(E) == 4 ? 5u : 4u;
    return x ^ (((x >> S) & 1u) * ((1u << S) - 1u)) ^ (((x >> (S + 1)) & 1u) << S);
}

// One group of ITERS comparators of a step (k = 2^m, j) per lane: lane0,
// lane0 + nt, ... All loads of the group are issued before its first compare,
// so their LDS latency overlaps.
//   melded: one load pair per comparator, both compares, a select of the swap
//     condition on the direction, one conditional store pair;
//   divergent: Figure 1's if/else. With nt >= 64 the direction of a phase
//     k <= 64 is a bit of lane0 alone, the same for all of the lane's
//     comparators, so the branch is taken once per step (the loop is
//     unswitched) and each side holds its own batched loads, compares and
//     swap stores; with nt < 64 it stays per comparator.
template <typename E, bool MELDED, int ITERS, bool SWZ>
__device__ __forceinline__ void lds_step_group(E *s, uint32_t base, uint32_t m, uint32_t j,
                                               uint32_t lane0, uint32_t nt) {
    uint32_t lo[ITERS];
    if (nt >= 64) {
        // j <= 32 in phases k <= 64 and nt is a multiple of 64: inserting the
        // zero bit at j leaves the comparators i * nt apart as 2 i nt, so only
        // the first index is computed (the rest become immediate offsets)
        const uint32_t lo0 = ((lane0 & ~(j - 1)) << 1) | (lane0 & (j - 1));
#pragma unroll
        for (int i = 0; i < ITERS; ++i) lo[i] = lo0 + 2u * (uint32_t)i * nt;
    } else {
#pragma unroll
        for (int i = 0; i < ITERS; ++i) {
            const uint32_t c = lane0 + (uint32_t)i * nt;
            lo[i] = ((c & ~(j - 1)) << 1) | (c & (j - 1));
        }
    }
    // LDS positions of the two ends (low_swz); the direction uses lo itself
    uint32_t pl[ITERS], ph[ITERS];
    if (nt >= 64) {
        // 2 i nt is a multiple of 128: it commutes with the swizzle
        const uint32_t pl0 = low_swz<E, SWZ>(lo[0]), ph0 = low_swz<E, SWZ>(lo[0] + j);
#pragma unroll
        for (int i = 0; i < ITERS; ++i) {
            pl[i] = pl0 + 2u * (uint32_t)i * nt;
            ph[i] = ph0 + 2u * (uint32_t)i * nt;
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITERS; ++i) {
            pl[i] = low_swz<E, SWZ>(lo[i]);
            ph[i] = low_swz<E, SWZ>(lo[i] + j);
        }
    }
    if constexpr (MELDED) {
        E a[ITERS], b[ITERS];
#pragma unroll
        for (int i = 0; i < ITERS; ++i) {
            a[i] = s[pl[i]];
            b[i] = s[ph[i]];
        }
        if (nt >= 64) {
            // nt is a multiple of 64 >= 2^m: every comparator of the lane has
            // the direction of its first one
            const bool up = (((base | lo[0]) >> m) & 1u) == 0;
#pragma unroll
            for (int i = 0; i < ITERS; ++i)
                if (melded_swap(a[i], b[i], up)) {
                    s[pl[i]] = b[i];
                    s[ph[i]] = a[i];
                }
        } else {
#pragma unroll
            for (int i = 0; i < ITERS; ++i) {
                const bool up = (((base | lo[i]) >> m) & 1u) == 0;
                if (melded_swap(a[i], b[i], up)) {
                    s[pl[i]] = b[i];
                    s[ph[i]] = a[i];
                }
            }
        }
    } else if (nt >= 64) {
        const bool up = (((base | lo[0]) >> m) & 1u) == 0;
        E a[ITERS], b[ITERS];
        if (up) {
            MELD_SIDE_MARK("ascending batch");
#pragma unroll
            for (int i = 0; i < ITERS; ++i) {
                a[i] = s[pl[i]];
                b[i] = s[ph[i]];
            }
#pragma unroll
            for (int i = 0; i < ITERS; ++i)
                if (b[i] < a[i]) {
                    s[pl[i]] = b[i];
                    s[ph[i]] = a[i];
                }
            MELD_SIDE_MARK("ascending batch end");
        } else {
            MELD_SIDE_MARK("descending batch");
#pragma unroll
            for (int i = 0; i < ITERS; ++i) {
                a[i] = s[pl[i]];
                b[i] = s[ph[i]];
            }
#pragma unroll
            for (int i = 0; i < ITERS; ++i)
                if (b[i] > a[i]) {
                    s[pl[i]] = b[i];
                    s[ph[i]] = a[i];
                }
            MELD_SIDE_MARK("descending batch end");
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITERS; ++i)
            cex_divergent(s, pl[i], ph[i], (((base | lo[i]) >> m) & 1u) == 0);
    }
}

// The comparators of a step in groups of at most 4 (bounding the registers a
// group holds in flight; 4 loads per comparator pair in flight per lane
// already cover the LDS latency).
template <typename E, bool MELDED, int ITERS, bool SWZ>
__device__ __forceinline__ void lds_step_batched(E *s, uint32_t base, uint32_t m, uint32_t j,
                                                 uint32_t lane0, uint32_t nt) {
    constexpr int G = ITERS < 4 ? ITERS : 4;
    static_assert(ITERS % G == 0, "comparators per lane must split into groups");
#pragma unroll
    for (int h = 0; h < ITERS / G; ++h)
        lds_step_group<E, MELDED, G, SWZ>(s, base, m, j, lane0 + (uint32_t)(h * G) * nt, nt);
}

// Phases k = 2 .. 2^m_end (m_end <= 6) of the network on a tile of
// 2 * ITERS * nt elements whose comparators are dealt to nt lanes
// (lane0 < nt), in form MELDED, at most step_limit steps (negative: all);
// returns the number of steps run. Every step is wave-local: the nt lanes of
// a team shorter than a wave share one wave, and for nt >= 64 a wave's
// comparators of one iteration stay inside one 128-element block in every
// step j <= 32.
template <typename E, bool MELDED, int ITERS, bool SWZ>
__device__ __forceinline__ int32_t lds_network_low(E *s, uint32_t base, uint32_t m_end,
                                                   uint32_t lane0, uint32_t nt,
                                                   int32_t step_limit) {
    int32_t steps = 0;
    for (uint32_t m = 1; m <= m_end; ++m) {
        for (uint32_t j = 1u << (m - 1); j > 0; j >>= 1) {
            if (steps == step_limit) return steps;
            ++steps;
            lds_step_batched<E, MELDED, ITERS, SWZ>(s, base, m, j, lane0, nt);
            wave_lds_sync();
        }
    }
    return steps;
}

}  // namespace meld
