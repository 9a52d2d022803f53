// Register tiles of the bitonic sort, shared by the streaming passes and merge
// tails (bitonic.hip) and by the local tile sorts of the two low-phase paths
// (bitonic_local_xch.hip, bitonic_local_lds.hip): element access modes and
// nontemporal helpers, the register compare-exchange, the layouts of a tile
// held 16 elements per thread and the LDS transposes between them, tile loads
// and stores.
#pragma once

#include "device_common.h"
#include "exchange.h"
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

// Global accesses of the streaming passes, the merge tails and the tile
// sorts of a large array (SortArray::nt, set when the array is far larger
// than the caches): every element is read once and written once per launch,
// so loads and stores carry the nontemporal hint. On the 2^28-pair sort:
// register passes 775 -> 737 us, merge tails 792 -> 767 us, gathered passes
// 862 -> 836 us per launch (whole sort 33.5 -> 32.4 ms); the hint on loads or
// on stores alone gained 1 % or nothing. A small array stays in L2 between
// launches, which the hint would give up (the 2^16-key sort: 47 -> 50 us).
// The choice is made once per load or store sequence (a template argument
// below it), not per access.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ uint32_t ld4(const uint32_t *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT>
__device__ __forceinline__ void st4(uint32_t *p, uint32_t v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
template <bool NT>
__device__ __forceinline__ uint4 ld16(const uint32_t *p) {
    if constexpr (NT) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    }
    return *reinterpret_cast<const uint4 *>(p);
}
template <bool NT>
__device__ __forceinline__ void st16(uint32_t *p, uint4 v) {
    if constexpr (NT) {
        const u32x4 w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(p));
    } else {
        *reinterpret_cast<uint4 *>(p) = v;
    }
}

template <int MODE, bool NT = false>
__device__ __forceinline__ uint32_t ld_u32(const uint32_t *main, const uint32_t *tail, uint32_t n,
                                           uint32_t p) {
    if constexpr (MODE == kTail) {
        const uint32_t *src = p < n ? main + p : tail + (p - n);
        return ld4<NT>(src);
    } else if constexpr (MODE == kSentinel) {
        return p < n ? main[p] : kPadValue;
    } else {
        return ld4<NT>(main + p);
    }
}

template <int MODE, bool NT = false>
__device__ __forceinline__ void st_u32(uint32_t *main, uint32_t *tail, uint32_t n, uint32_t p,
                                       uint32_t v) {
    if constexpr (MODE == kTail) {
        uint32_t *dst = p < n ? main + p : tail + (p - n);
        st4<NT>(dst, v);
    } else if constexpr (MODE == kSentinel) {
        if (p < n) main[p] = v;
    } else {
        st4<NT>(main + p, v);
    }
}

template <bool PAIRS, int MODE, bool NT = false>
__device__ __forceinline__ typename ElemOf<PAIRS>::type load_elem(const SortArray &a, uint32_t p) {
    const uint32_t k = ld_u32<MODE, NT>(a.keys, a.tk, a.n, p);
    if constexpr (PAIRS) {
        const uint32_t v = ld_u32<MODE, NT>(a.vals, a.tv, a.n, p);
        return ((uint64_t)k << 32) | v;
    } else {
        return k;
    }
}

template <bool PAIRS, int MODE, bool NT = false>
__device__ __forceinline__ void store_elem(const SortArray &a, uint32_t p,
                                           typename ElemOf<PAIRS>::type e) {
    if constexpr (PAIRS) {
        st_u32<MODE, NT>(a.keys, a.tk, a.n, p, (uint32_t)(e >> 32));
        st_u32<MODE, NT>(a.vals, a.tv, a.n, p, (uint32_t)e);
    } else {
        st_u32<MODE, NT>(a.keys, a.tk, a.n, p, e);
    }
}

// Compare-exchange of two registers for direction up, with no branch.
// Keys: min and max, then one select per output on the direction.
// Pairs: one 64-bit compare whose lane mask is flipped for descending lanes
// (a scalar operation) decides the swap, one select per 32-bit half (5 VALU
// operations instead of 9 for min / max of the composite and the selects);
// equal pairs are the same value, so swapping them or not is the same.
__device__ __forceinline__ void cex_regs(uint32_t &x, uint32_t &y, bool up) {
    const uint32_t mn = x < y ? x : y;
    const uint32_t mx = x < y ? y : x;
    x = up ? mn : mx;
    y = up ? mx : mn;
}

__device__ __forceinline__ void cex_regs(uint64_t &x, uint64_t &y, bool up) {
    const bool swap = (y < x) == up;
    const uint64_t a = swap ? y : x;
    const uint64_t b = swap ? x : y;
    x = a;
    y = b;
}

// Merge of one tile in a phase k > tile (steps j = T/2 .. 1; the direction is
// bit k of the tile's base, the same for the whole tile, so the two forms
// coincide). Each thread holds 16 elements in registers; a layout names which
// four element bits form the register index, the remaining bits are the
// thread index. Steps on register bits run in registers; an LDS transpose
// (one padding slot per 16 elements against bank conflicts) changes layout.
//
//   layout V (B = -1): register bits 0, 1 = element bits 0, 1 and register
//     bits 2, 3 = element bits L-2, L-1; thread t holds the 16-byte groups
//     4t and 4t + 2^(L-2) k, so consecutive lanes move consecutive 16 bytes.
//   window B >= 0: element bits [B, B+4) are the register index.
//
// Sequence: load in V, steps L-1 and L-2; windows L-6, L-10, ... (the last one
// clamped at 0) take the next bits four at a time; back to V to store (vector
// modes), or to window L-4 (lane-linear elements) for per-element modes.
constexpr int kMergeE = 16;

template <int L, int B>
__device__ __forceinline__ uint32_t merge_index(uint32_t t, uint32_t r) {
    if constexpr (B < 0)
        return (r & 3u) | (t << 2) | ((r >> 2) << (L - 2));
    else
        return (t & ((1u << B) - 1)) | (r << B) | ((t >> B) << (B + 4));
}

__device__ __forceinline__ uint32_t merge_phys(uint32_t i) { return i + (i >> 4); }

// For a layout index a | b with disjoint bit fields a (lane bits) and b
// (register bits), (a | b) >> 4 = (a >> 4) + (b >> 4), so
// merge_phys(a | b) = merge_phys(a) + merge_phys(b): the lane part is computed
// once per transpose and the register part is a constant, an immediate offset
// of the LDS access (a scalar for a window known only at run time).

// Windows of a pass whose steps stop at element bit SLO: base bit and top
// step bit of window w >= 1; the last layout is the last window that holds a
// step (-1, layout V, when V's two steps are all).
template <int L, int SLO>
constexpr int window_base(int w) {
    return L - 2 - 4 * w > SLO ? L - 2 - 4 * w : SLO;
}

template <int L, int SLO>
constexpr int window_top(int w) {
    return w == 1 ? L - 3 : window_base<L, SLO>(w - 1) - 1;
}

template <int L, int SLO>
constexpr int last_layout() {
    int last = -1;
    for (int w = 1; window_top<L, SLO>(w) >= SLO; ++w) last = window_base<L, SLO>(w);
    return last;
}

template <int L, int FROM, int TO, typename E>
__device__ __forceinline__ void merge_transpose(E (&e)[kMergeE], E *s, uint32_t t) {
#pragma unroll
    for (int r = 0; r < kMergeE; ++r)
        s[merge_phys(merge_index<L, FROM>(t, 0u)) + merge_phys(merge_index<L, FROM>(0u, r))] = e[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kMergeE; ++r)
        e[r] = s[merge_phys(merge_index<L, TO>(t, 0u)) + merge_phys(merge_index<L, TO>(0u, r))];
    __syncthreads();
}

// The step on register bit Q for all 16 registers.
template <int Q, typename E>
__device__ __forceinline__ void merge_reg_step(E (&e)[kMergeE], bool up) {
#pragma unroll
    for (int r = 0; r < kMergeE; ++r)
        if ((r & (1 << Q)) == 0) cex_regs(e[r], e[r | (1 << Q)], up);
}

// Steps on element bits TOP .. B of window B (register bit = element bit - B);
// the step on element bit i is number L-1-i of the pass (0-based).
template <int L, int B, int BIT, typename E>
__device__ __forceinline__ void merge_window_steps(E (&e)[kMergeE], bool up, int32_t nsteps) {
    if constexpr (BIT >= B) {
        if (L - 1 - BIT < nsteps) merge_reg_step<BIT - B>(e, up);
        merge_window_steps<L, B, BIT - 1>(e, up, nsteps);
    }
}

// Window w (w >= 1) and the ones after it, down to step bit SLO; PREV is the
// layout e is in.
template <int L, int W, int PREV, int SLO, typename E>
__device__ __forceinline__ void merge_windows(E (&e)[kMergeE], E *s, uint32_t t, bool up,
                                              int32_t nsteps) {
    constexpr int B = window_base<L, SLO>(W);
    constexpr int TOP = window_top<L, SLO>(W);
    if constexpr (TOP >= SLO) {
        merge_transpose<L, PREV, B>(e, s, t);
        merge_window_steps<L, B, TOP>(e, up, nsteps);
        merge_windows<L, W + 1, B, SLO>(e, s, t, up, nsteps);
    }
}

// Steps on element bits TOP .. 0 of a merge (layout PREV on entry) that end
// in layout W0 (window 0) instead of a last four-bit window: windows with
// bases TOP-3, TOP-7, ... while the top step bit is at least 7, then W0,
// where the steps on element bits 6, 5 and 4 are DPP lane exchanges (lane
// bits 2, 1 and 0; bit 2 takes two DPP moves, bits 1 and 0 one) and bits
// 3 .. 0 registers. The direction is uniform per tile, so the lane steps take
// the melded compare-select. For a tile of 2^13 this is one LDS transpose
// fewer than four-bit windows down to bit 0 (the 2^28-pair merge tail: 756 ->
// 734 us per launch).
template <int L, int TOP, int PREV, typename E>
__device__ __forceinline__ void merge_windows_xch(E (&e)[kMergeE], E *s, uint32_t t, bool up,
                                                  int32_t nsteps) {
    if constexpr (TOP >= 7) {
        constexpr int B = TOP - 3;
        merge_transpose<L, PREV, B>(e, s, t);
        merge_window_steps<L, B, TOP>(e, up, nsteps);
        merge_windows_xch<L, B - 1, B>(e, s, t, up, nsteps);
    } else if constexpr (TOP >= 0) {
        merge_transpose<L, PREV, 0>(e, s, t);
        if constexpr (TOP >= 6)
            if (L - 1 - 6 < nsteps) lane_step<2, true>(e, up, ((t >> 2) & 1u) == 0);
        if constexpr (TOP >= 5)
            if (L - 1 - 5 < nsteps) lane_step<1, true>(e, up, ((t >> 1) & 1u) == 0);
        if constexpr (TOP >= 4)
            if (L - 1 - 4 < nsteps) lane_step<0, true>(e, up, (t & 1u) == 0);
        merge_window_steps<L, 0, (TOP < 3 ? TOP : 3)>(e, up, nsteps);
    }
}

// Windows (LDS transposes) a merge tail of 2^L needs after layout V's two
// steps: four-bit windows all the way, or ending in W0 with lane exchanges.
constexpr int merge_windows_plain(int L) { return (L - 2 + 3) / 4; }
constexpr int merge_windows_with_xch(int L) {
    int n = 0, top = L - 3;
    for (; top >= 7; top -= 4) ++n;
    return top >= 0 ? n + 1 : n;
}
// The merge tail takes the lane-exchange ending where it saves a transpose
// (tiles of 2^8, 2^9 and 2^11 .. 2^13; for 2^10 and 2^14 both need as many).
template <int L>
constexpr bool merge_uses_xch() {
    return merge_windows_with_xch(L) < merge_windows_plain(L);
}

// Where element i of a tile lives in the array: its low C bits stay, the
// bits above C move up to start at bit b_lo, and base holds the workgroup's
// other bits. C = L is a contiguous tile at base.
template <int L, int C>
struct TileMap {
    uint32_t base, b_lo;
    __device__ __forceinline__ uint32_t operator()(uint32_t i) const {
        if constexpr (C >= L)
            return base | i;
        else
            return base | (i & ((1u << C) - 1)) | ((i >> C) << b_lo);
    }
};

// Runtime layout index: window B (element bits [B, B+4) are the register
// index) for a B known only at run time.
__device__ __forceinline__ uint32_t window_tpart(uint32_t t, uint32_t B) {
    return (t & ((1u << B) - 1)) | ((t >> B) << (B + 4));
}

// Thread t's 16 elements of a tile in layout V (C >= 2, so each 16-byte
// group is contiguous in the array). Modes: vector (16-byte groups),
// sentinel (positions >= n read as the pad value), plain or tail (positions
// >= n from the tail workspace; a tile wholly below n loads directly).
template <bool PAIRS, int L, int C, bool NT>
__device__ __forceinline__ void regs_load_t(const SortArray &a, const TileMap<L, C> &map,
                                            uint32_t t, int mode,
                                            typename ElemOf<PAIRS>::type (&e)[kMergeE]) {
    using E = typename ElemOf<PAIRS>::type;
    if (mode == kPlainVec) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t p = map(merge_index<L, -1>(t, 4 * c));
            const uint4 k = ld16<NT>(a.keys + p);
            if constexpr (PAIRS) {
                const uint4 v = ld16<NT>(a.vals + p);
                e[4 * c + 0] = ((E)k.x << 32) | v.x;
                e[4 * c + 1] = ((E)k.y << 32) | v.y;
                e[4 * c + 2] = ((E)k.z << 32) | v.z;
                e[4 * c + 3] = ((E)k.w << 32) | v.w;
            } else {
                e[4 * c + 0] = k.x;
                e[4 * c + 1] = k.y;
                e[4 * c + 2] = k.z;
                e[4 * c + 3] = k.w;
            }
        }
    } else if (mode == kSentinel) {
#pragma unroll
        for (int r = 0; r < kMergeE; ++r)
            e[r] = load_elem<PAIRS, kSentinel>(a, map(merge_index<L, -1>(t, r)));
    } else {
        const bool below_n = map((1u << L) - 1) < a.n;  // the map is increasing
#pragma unroll
        for (int r = 0; r < kMergeE; ++r) {
            const uint32_t p = map(merge_index<L, -1>(t, r));
            e[r] = below_n ? load_elem<PAIRS, kPlain, NT>(a, p) : load_elem<PAIRS, kTail, NT>(a, p);
        }
    }
}

template <bool PAIRS, int L, int C>
__device__ __forceinline__ void regs_load(const SortArray &a, const TileMap<L, C> &map, uint32_t t,
                                          int mode, typename ElemOf<PAIRS>::type (&e)[kMergeE]) {
    if (a.nt != 0)
        regs_load_t<PAIRS, L, C, true>(a, map, t, mode, e);
    else
        regs_load_t<PAIRS, L, C, false>(a, map, t, mode, e);
}

// The global stores of a tile held in layout V (vector modes) or window L-4.
template <bool PAIRS, int L, int C, bool NT>
__device__ __forceinline__ void regs_store_t(const SortArray &a, const TileMap<L, C> &map,
                                             uint32_t t, int mode,
                                             typename ElemOf<PAIRS>::type (&e)[kMergeE]) {
    if (mode == kPlainVec) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t p = map(merge_index<L, -1>(t, 4 * c));
            if constexpr (PAIRS) {
                st16<NT>(a.keys + p, make_uint4((uint32_t)(e[4 * c] >> 32),
                                                (uint32_t)(e[4 * c + 1] >> 32),
                                                (uint32_t)(e[4 * c + 2] >> 32),
                                                (uint32_t)(e[4 * c + 3] >> 32)));
                st16<NT>(a.vals + p, make_uint4((uint32_t)e[4 * c], (uint32_t)e[4 * c + 1],
                                                (uint32_t)e[4 * c + 2], (uint32_t)e[4 * c + 3]));
            } else {
                st16<NT>(a.keys + p, make_uint4(e[4 * c], e[4 * c + 1], e[4 * c + 2], e[4 * c + 3]));
            }
        }
        return;
    }
    if (mode == kSentinel) {
#pragma unroll
        for (int r = 0; r < kMergeE; ++r)
            store_elem<PAIRS, kSentinel>(a, map(merge_index<L, L - 4>(t, r)), e[r]);
    } else {
        const bool below_n = map((1u << L) - 1) < a.n;
#pragma unroll
        for (int r = 0; r < kMergeE; ++r) {
            const uint32_t p = map(merge_index<L, L - 4>(t, r));
            if (below_n)
                store_elem<PAIRS, kPlain, NT>(a, p, e[r]);
            else
                store_elem<PAIRS, kTail, NT>(a, p, e[r]);
        }
    }
}

// Stores a tile held in layout FROM: through layout V with 16-byte stores,
// or through window L-4 (consecutive lanes, consecutive elements) per element.
template <bool PAIRS, int L, int C, int FROM>
__device__ __forceinline__ void regs_store(const SortArray &a, typename ElemOf<PAIRS>::type *s,
                                           const TileMap<L, C> &map, uint32_t t, int mode,
                                           typename ElemOf<PAIRS>::type (&e)[kMergeE]) {
    if (mode == kPlainVec) {
        if constexpr (FROM != -1) merge_transpose<L, FROM, -1>(e, s, t);
    } else {
        merge_transpose<L, FROM, L - 4>(e, s, t);
    }
    if (a.nt != 0)
        regs_store_t<PAIRS, L, C, true>(a, map, t, mode, e);
    else
        regs_store_t<PAIRS, L, C, false>(a, map, t, mode, e);
}

template <bool PAIRS, int L>
size_t regs_lds_bytes() {
    using E = typename ElemOf<PAIRS>::type;
    return (size_t)((1u << L) + (1u << L) / 16) * sizeof(E);
}

template <typename K>
hipError_t allow_lds(K kern, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// Tile sizes (log2) the register-tile kernels are instantiated for; a build
// that inspects the code of a few sizes only may narrow the list.
#ifndef MELD_REGS_SIZES
#define MELD_REGS_SIZES(X) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#endif

}  // namespace

}  // namespace meld
