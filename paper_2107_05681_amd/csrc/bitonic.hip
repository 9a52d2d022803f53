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
// bases TOP-3, TOP-7, ... while the top step bit is at least 6, then W0,
// where the steps on element bits 5 and 4 are DPP lane exchanges (lane bits
// 1 and 0) and bits 3 .. 0 registers. The direction is uniform per tile, so
// the lane steps take the melded compare-select.
template <int L, int TOP, int PREV, typename E>
__device__ __forceinline__ void merge_windows_xch(E (&e)[kMergeE], E *s, uint32_t t, bool up,
                                                  int32_t nsteps) {
    if constexpr (TOP >= 6) {
        constexpr int B = TOP - 3;
        merge_transpose<L, PREV, B>(e, s, t);
        merge_window_steps<L, B, TOP>(e, up, nsteps);
        merge_windows_xch<L, B - 1, B>(e, s, t, up, nsteps);
    } else if constexpr (TOP >= 0) {
        merge_transpose<L, PREV, 0>(e, s, t);
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
    for (; top >= 6; top -= 4) ++n;
    return top >= 0 ? n + 1 : n;
}
// The merge tail takes the lane-exchange ending where it saves a transpose
// (tiles of 2^8, 2^11 and 2^12; for 2^13 and 2^14 both need three).
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

// The 16 elements of window W at p[merge_phys(r << W)] (p: the lane's part,
// already through merge_phys). With W fixed at compile time every position is
// an immediate offset of the LDS instruction (at most merge_phys(15 << 10)
// elements = 65280 bytes for keys, merge_phys(15 << 9) for pairs); a run-time
// W costs scalar arithmetic and a vector add per element.
template <int W, typename E>
__device__ __forceinline__ void window_store_w(const E (&e)[kMergeE], E *p) {
#pragma unroll
    for (int r = 0; r < kMergeE; ++r) p[merge_phys((uint32_t)r << W)] = e[r];
}
template <int W, typename E>
__device__ __forceinline__ void window_load_w(E (&e)[kMergeE], const E *p) {
#pragma unroll
    for (int r = 0; r < kMergeE; ++r) e[r] = p[merge_phys((uint32_t)r << W)];
}

// Run-time window bases are 0 .. 10 (tiles of at most 2^14 elements); each
// case ends in its own mark so that the compiler keeps the cases apart
// instead of merging them back into one block with computed offsets.
#define WINDOW_CASE(W, CALL, TAG) \
    case W:                       \
        CALL;                     \
        asm volatile("; window " TAG " " #W ::: "memory"); \
        break;

template <typename E>
__device__ __forceinline__ void window_store(const E (&e)[kMergeE], E *p, uint32_t W) {
    switch (W) {
        WINDOW_CASE(0, (window_store_w<0, E>(e, p)), "store")
        WINDOW_CASE(1, (window_store_w<1, E>(e, p)), "store")
        WINDOW_CASE(2, (window_store_w<2, E>(e, p)), "store")
        WINDOW_CASE(3, (window_store_w<3, E>(e, p)), "store")
        WINDOW_CASE(4, (window_store_w<4, E>(e, p)), "store")
        WINDOW_CASE(5, (window_store_w<5, E>(e, p)), "store")
        WINDOW_CASE(6, (window_store_w<6, E>(e, p)), "store")
        WINDOW_CASE(7, (window_store_w<7, E>(e, p)), "store")
        WINDOW_CASE(8, (window_store_w<8, E>(e, p)), "store")
        WINDOW_CASE(9, (window_store_w<9, E>(e, p)), "store")
        default: window_store_w<10, E>(e, p); break;
    }
}

template <typename E>
__device__ __forceinline__ void window_load(E (&e)[kMergeE], const E *p, uint32_t W) {
    switch (W) {
        WINDOW_CASE(0, (window_load_w<0, E>(e, p)), "load")
        WINDOW_CASE(1, (window_load_w<1, E>(e, p)), "load")
        WINDOW_CASE(2, (window_load_w<2, E>(e, p)), "load")
        WINDOW_CASE(3, (window_load_w<3, E>(e, p)), "load")
        WINDOW_CASE(4, (window_load_w<4, E>(e, p)), "load")
        WINDOW_CASE(5, (window_load_w<5, E>(e, p)), "load")
        WINDOW_CASE(6, (window_load_w<6, E>(e, p)), "load")
        WINDOW_CASE(7, (window_load_w<7, E>(e, p)), "load")
        WINDOW_CASE(8, (window_load_w<8, E>(e, p)), "load")
        WINDOW_CASE(9, (window_load_w<9, E>(e, p)), "load")
        default: window_load_w<10, E>(e, p); break;
    }
}
#undef WINDOW_CASE

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

// One pass of S steps (on element bits L-1 .. L-S of a tile of 2^L) of
// phase k = 2^m, whose direction bit m lies above the tile's bits. Tile map
// with C low bits: workgroup b's bits fill array bits [C, b_lo) and then
// [b_lo + L - C, ...). Merge tail: S = C = L (contiguous tiles, b_lo = L).
// Gathered streaming pass: C = L - S, so the steps act on array bits
// b_lo .. b_lo + S - 1 and each of the 2^S rows is 2^C contiguous elements.
template <bool PAIRS, int L, int S, int C>
__global__ __launch_bounds__(1 << (L - 4)) void bitonic_pass_regs_kernel(SortArray a, uint32_t m,
                                                                         uint32_t b_lo, int mode,
                                                                         int32_t nsteps) {
    using E = typename ElemOf<PAIRS>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    E *s = reinterpret_cast<E *>(smem);
    const uint32_t t = threadIdx.x;
    const uint32_t b = blockIdx.x;
    const uint32_t spread = b_lo - C;
    const uint32_t base = ((b & ((1u << spread) - 1)) << C) | ((b >> spread) << (b_lo + L - C));
    const TileMap<L, C> map{base, b_lo};
    const bool up = ((base >> m) & 1u) == 0;

    E e[kMergeE];
    regs_load<PAIRS, L, C>(a, map, t, mode, e);
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

// Moves a tile held in window prev to window B (run-time bases) through LDS.
template <bool PAIRS, typename E>
__device__ __forceinline__ void window_move(E (&e)[kMergeE], E *s, uint32_t t, uint32_t prev,
                                            uint32_t B) {
    if (B == prev) return;
    if constexpr (PAIRS) {
        // 8-byte elements: the per-case copies that the compile-time
        // windows leave behind cost more than the scalar offsets
        // (2^28 pairs: local sort 5.73 -> 5.97 ms melded)
        const uint32_t tp = merge_phys(window_tpart(t, prev));
        const uint32_t tb = merge_phys(window_tpart(t, B));
#pragma unroll
        for (int r = 0; r < kMergeE; ++r) s[tp + merge_phys((uint32_t)r << prev)] = e[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kMergeE; ++r) e[r] = s[tb + merge_phys((uint32_t)r << B)];
        __syncthreads();
    } else {
        window_store(e, s + merge_phys(window_tpart(t, prev)), prev);
        __syncthreads();
        window_load(e, s + merge_phys(window_tpart(t, B)), B);
        __syncthreads();
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
// step bit is at least 6 and end in W0, where the steps on bits 5 and 4 are
// lane exchanges: a window fewer for m = 9, 10, 13, 14.
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
        uint32_t prev = 0;
        for (uint32_t m = 7; m <= (uint32_t)L; ++m) {
            const bool up = (((base >> m) | (t >> (m - 4))) & 1u) == 0;
            int top = (int)m - 1;
            while (top >= 6) {
                const uint32_t B = (uint32_t)top - 3;
                window_move<PAIRS>(e, s, t, prev, B);
                reg_steps<MELD_HI>(e, 3, up, left);
                prev = B;
                top = (int)B - 1;
            }
            window_move<PAIRS>(e, s, t, prev, 0);
            prev = 0;
            if (top >= 5 && left > 0) {
                lane_step<1, MELD_HI>(e, up, ((t >> 1) & 1u) == 0);
                --left;
            }
            if (top >= 4 && left > 0) {
                lane_step<0, MELD_HI>(e, up, (t & 1u) == 0);
                --left;
            }
            reg_steps<MELD_HI>(e, top < 3 ? top : 3, up, left);
        }
    } else {
#pragma unroll
        for (int r = 0; r < kMergeE; ++r) s[low_swz<E, PAIRS>(merge_index<L, -1>(t, r))] = e[r];  // natural order
        __syncthreads();
        const int32_t lo_steps = lds_network_low<E, MELD_LO, 8, PAIRS>(s, base, 6, t, NT, step_limit);
        __syncthreads();
        int32_t left = step_limit < 0 ? 0x7FFFFFFF : step_limit - lo_steps;

        // Phase 2^7 starts in window 3 (element bits 3..6), read from the natural
        // order the comparator network leaves in s.
        uint32_t prev = 3;
        {
            const uint32_t tb = window_tpart(t, prev);
#pragma unroll
            for (int r = 0; r < kMergeE; ++r) e[r] = s[low_swz<E, PAIRS>(tb | ((uint32_t)r << prev))];
            __syncthreads();
        }
        for (uint32_t m = 7; m <= (uint32_t)L; ++m) {
            const bool up = (((base >> m) | (t >> (m - 4))) & 1u) == 0;
            for (uint32_t w = 1;; ++w) {
                const uint32_t B = m > 4 * w ? m - 4 * w : 0;
                const int hi_q = (int)(m - 4 * (w - 1) - 1 - B);
                window_move<PAIRS>(e, s, t, prev, B);
                reg_steps<MELD_HI>(e, hi_q, up, left);
                prev = B;
                if (B == 0) break;
            }
        }
    }
    regs_store<PAIRS, L, L, 0>(a, s, map, t, mode, e);
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

template <bool PAIRS, int L>
hipError_t launch_sort_regs_l(const SortArray &a, uint32_t n_tiles, int32_t step_limit, bool lo,
                              bool hi, bool xch, int io_mode, hipStream_t stream) {
    return xch ? launch_sort_regs_x<PAIRS, L, true>(a, n_tiles, step_limit, lo, hi, io_mode, stream)
               : launch_sort_regs_x<PAIRS, L, false>(a, n_tiles, step_limit, lo, hi, io_mode,
                                                     stream);
}

#define MELD_REGS_SIZES(X) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

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

template <bool PAIRS>
hipError_t launch_sort_regs_p(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                              int32_t step_limit, bool lo, bool hi, bool xch, int io_mode,
                              hipStream_t stream) {
#define MELD_CASE(L) \
    case L:          \
        return launch_sort_regs_l<PAIRS, L>(a, n_tiles, step_limit, lo, hi, xch, io_mode, stream);
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
    if (n_tiles == 0 || step_limit == 0) return hipSuccess;
    if (io_mode == kPlain) io_mode = kTail;  // no tail workspace: every tile is below n
    if (a.vals != nullptr)
        return launch_sort_regs_p<true>(a, log_t, n_tiles, step_limit, meld_lo, meld_hi, xch,
                                        io_mode, stream);
    return launch_sort_regs_p<false>(a, log_t, n_tiles, step_limit, meld_lo, meld_hi, xch,
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
