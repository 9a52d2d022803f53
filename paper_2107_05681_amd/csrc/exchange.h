// Wavefront lane exchanges for the bitonic network held in registers.
//
// Layout W0 of a tile held 16 elements per lane: register r of lane t holds
// element 16 t + r, so element bits 0..3 are the register index and element
// bits 4, 5, 6 are lane bits 0, 1, 2. A step on element bit 4 or 5 pairs
// every lane with lane t ^ 1 or t ^ 2, inside its quad: a DPP quad
// permutation brings the partner's value, with no LDS access and no wait. A
// step on element bit 6 pairs lane t with t ^ 4: two DPP moves.
//
// Warp-level exchanges are never part of a melded region (Detailed Design,
// "Computing Melding Profitability": such intrinsics are not melded), so in
// both forms the partner value is fetched once, before the direction branch;
// only the compare and select that follow differ between the forms:
//   divergent: if (up) { compare, select } else { compare, select } — each
//     side with its own compare (Figure 1's if/else on the direction);
//   melded: one min and one max on the full wave, the kept one chosen by a
//     select on (lower end) == up.
#pragma once

#include "device_common.h"

namespace meld {

constexpr int kXchE = 16;  // elements per lane

// DPP16 control words: quad_perm [1,0,3,2] (lane ^ 1), [2,3,0,1] (lane ^ 2).
template <int B>
constexpr int dpp_quad_xor() {
    static_assert(B == 0 || B == 1, "quad permutations reach lane bits 0 and 1");
    return B == 0 ? 0xB1 : 0x4E;
}

// Partner value for the melded form: bound_ctrl set (no lane of a quad
// permutation is out of range, so it never applies), which lets the compiler
// fold the move into the min / max that use it (v_min_u32_dpp).
template <int B>
__device__ __forceinline__ uint32_t lane_xor_fused(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, dpp_quad_xor<B>(), 0xF, 0xF, true);
}

// Partner value as a move of its own, which the compiler does not fold into
// the compares inside the two sides of the divergent form: the exchange stays
// outside the branch there.
template <int B>
__device__ __forceinline__ uint32_t lane_xor_move(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, dpp_quad_xor<B>(), 0xF, 0xF,
                                                 false);
}

// Lane t ^ 4 (lane bit 2): a half-row mirror (lane t ^ 7 within each group
// of 8), then a quad reversal (t ^ 3): (t ^ 3) ^ 7 = t ^ 4. Two DPP moves.
__device__ __forceinline__ uint32_t lane_xor4(uint32_t x) {
    const int y = __builtin_amdgcn_update_dpp((int)x, (int)x, 0x141, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_update_dpp(y, y, 0x1B, 0xF, 0xF, false);
}

template <int B, bool FUSED>
__device__ __forceinline__ uint32_t lane_xor(uint32_t x) {
    if constexpr (B == 2)
        return lane_xor4(x);
    else
        return FUSED ? lane_xor_fused<B>(x) : lane_xor_move<B>(x);
}

template <int B, bool FUSED>
__device__ __forceinline__ uint64_t lane_xor(uint64_t x) {
    const uint32_t lo = lane_xor<B, FUSED>((uint32_t)x);
    const uint32_t hi = lane_xor<B, FUSED>((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Value of a lane-step compare-exchange at one end: the end at the lower
// element index (lower) keeps the smaller value when ascending (up), the
// larger one when descending; the upper end the other way round.
__device__ __forceinline__ uint32_t keep_end(uint32_t x, uint32_t p, bool keep_min) {
    const uint32_t mn = x < p ? x : p;
    const uint32_t mx = x < p ? p : x;
    return keep_min ? mn : mx;
}

// Pairs: one 64-bit compare whose lane mask is flipped where the larger value
// is kept (a scalar operation), a select per 32-bit half; equal composites
// are the same value, so taking either is the same.
__device__ __forceinline__ uint64_t keep_end(uint64_t x, uint64_t p, bool keep_min) {
    return ((p < x) == keep_min) ? p : x;
}

// The value x as seen inside one side of a branch: an empty asm statement
// that the compiler must keep in that side, so the compare and select that
// use it stay there too (without it the compiler computes the min and max of
// both sides once before the branch, melding most of the region itself).
// Emits no instruction.
__device__ __forceinline__ uint32_t side_value(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ uint64_t side_value(uint64_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

// The divergent form of a lane step on registers R0 .. R0 + G - 1: the
// partner values first, then Figure 1's if/else on the direction, each side
// with its own compare and select (ascending: the lower end keeps the smaller
// value; descending: the larger).
template <int B, int R0, int G, typename E>
__device__ __forceinline__ void lane_step_divergent(E (&e)[kXchE], bool up, bool lower) {
    E p[G];
#pragma unroll
    for (int r = 0; r < G; ++r) p[r] = lane_xor<B, false>(e[R0 + r]);
    if (up) {
        MELD_SIDE_MARK("ascending lanes");
#pragma unroll
        for (int r = 0; r < G; ++r) e[R0 + r] = keep_end(e[R0 + r], side_value(p[r]), lower);
    } else {
        MELD_SIDE_MARK("descending lanes");
#pragma unroll
        for (int r = 0; r < G; ++r) e[R0 + r] = keep_end(e[R0 + r], side_value(p[r]), !lower);
    }
}

template <int B, int R0, int G, typename E>
__device__ __forceinline__ void lane_step_groups(E (&e)[kXchE], bool up, bool lower) {
    if constexpr (R0 < kXchE) {
        lane_step_divergent<B, R0, G>(e, up, lower);
        lane_step_groups<B, R0 + G, G>(e, up, lower);
    }
}

// The step on lane bit B (element bit 4 + B) for all 16 registers.
// up: the direction (the same for the lane's 16 elements, since the phase's
// direction bit lies above bit 4 + B); lower: lane bit B is clear. The
// divergent form runs in groups of G registers (partner values of a group,
// then its branch), which bounds the registers it holds at once.
template <int B, bool MELDED, int G = kXchE, typename E>
__device__ __forceinline__ void lane_step(E (&e)[kXchE], bool up, bool lower) {
    if constexpr (MELDED) {
        const bool keep_min = lower == up;
#pragma unroll
        for (int r = 0; r < kXchE; ++r) e[r] = keep_end(e[r], lane_xor<B, true>(e[r]), keep_min);
    } else {
        static_assert(kXchE % G == 0, "groups must tile the registers");
        lane_step_groups<B, 0, G>(e, up, lower);
    }
}

// Compare-exchange of two registers for direction up, with no branch.
__device__ __forceinline__ void xch_cex(uint32_t &x, uint32_t &y, bool up) {
    const uint32_t mn = x < y ? x : y;
    const uint32_t mx = x < y ? y : x;
    x = up ? mn : mx;
    y = up ? mx : mn;
}

__device__ __forceinline__ void xch_cex(uint64_t &x, uint64_t &y, bool up) {
    const bool swap = (y < x) == up;
    const uint64_t a = swap ? y : x;
    const uint64_t b = swap ? x : y;
    x = a;
    y = b;
}

// The step on register bit Q with a direction that varies per lane: melded
// (both orders computed, a select on the direction) or divergent (Figure 1's
// if/else, each side with its own compare and swap; the marks keep the
// compiler from merging the sides).
template <int Q, bool MELDED, typename E>
__device__ __forceinline__ void xch_reg_step(E (&e)[kXchE], bool up) {
    if constexpr (MELDED) {
#pragma unroll
        for (int r = 0; r < kXchE; ++r)
            if ((r & (1 << Q)) == 0) xch_cex(e[r], e[r | (1 << Q)], up);
    } else {
        if (up) {
            MELD_SIDE_MARK("ascending xregs");
#pragma unroll
            for (int r = 0; r < kXchE; ++r)
                if ((r & (1 << Q)) == 0) {
                    const E x = e[r], y = e[r | (1 << Q)];
                    if (y < x) {
                        e[r] = y;
                        e[r | (1 << Q)] = x;
                    }
                }
        } else {
            MELD_SIDE_MARK("descending xregs");
#pragma unroll
            for (int r = 0; r < kXchE; ++r)
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

// The step on register bit Q of phase 2^M, M <= 3: the direction is bit M of
// the register index, fixed per register pair, so there is no branch in
// either form.
template <int M, int Q, typename E>
__device__ __forceinline__ void xch_reg_step_fixed(E (&e)[kXchE]) {
#pragma unroll
    for (int r = 0; r < kXchE; ++r)
        if ((r & (1 << Q)) == 0) xch_cex(e[r], e[r | (1 << Q)], ((r >> M) & 1) == 0);
}

// Step JB (j = 2^JB) of phase 2^M (M <= 6) on a tile in layout W0; t is the
// lane's index in the tile (element 16 t + r), whose bits above bit 6 do not
// matter here. Phases 2^4 .. 2^6 take their direction from lane bits 0..2:
// the region in which the forms differ.
template <int M, int JB, bool MELDED, int G, typename E>
__device__ __forceinline__ void xch_low_step(E (&e)[kXchE], uint32_t t) {
    if constexpr (JB <= 3) {
        if constexpr (M <= 3)
            xch_reg_step_fixed<M, JB>(e);
        else
            xch_reg_step<JB, MELDED>(e, ((t >> (M - 4)) & 1u) == 0);
    } else {
        lane_step<JB - 4, MELDED, G>(e, ((t >> (M - 4)) & 1u) == 0, ((t >> (JB - 4)) & 1u) == 0);
    }
}

template <int M, int JB, bool MELDED, int G, typename E>
__device__ __forceinline__ void xch_low_steps(E (&e)[kXchE], uint32_t t, int32_t limit,
                                              int32_t &done) {
    if constexpr (M <= 6) {
        if (done == limit) return;
        xch_low_step<M, JB, MELDED, G>(e, t);
        ++done;
        if constexpr (JB > 0)
            xch_low_steps<M, JB - 1, MELDED, G>(e, t, limit, done);
        else
            xch_low_steps<M + 1, M, MELDED, G>(e, t, limit, done);
    }
}

// Phases k = 2 .. 64 (21 steps) of Figure 1's network on a tile held in
// layout W0, at most limit steps (negative: all), in registers and DPP lane
// exchanges only. Returns the number of steps run. G: register group of the
// divergent lane steps (lane_step).
template <bool MELDED, int G = kXchE, typename E>
__device__ __forceinline__ int32_t xch_network_low(E (&e)[kXchE], uint32_t t, int32_t limit) {
    int32_t done = 0;
    xch_low_steps<1, 0, MELDED, G>(e, t, limit, done);
    return done;
}

}  // namespace meld
