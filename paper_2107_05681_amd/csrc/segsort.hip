// Segmented bitonic sort: many uneven buckets in one persistent launch.
//
// The paper's bitonic benchmark sorts one bucket per thread block
// (Evaluation section, "Bitonic Sort (BIT)"). Here thousands of buckets of
// 0..65536 keys are sorted in one launch:
//   1. reset    — clears the work-queue counters (a kernel, so the sequence
//                 can be captured in a graph);
//   2. classify — per segment: validity checks and the size class
//                 c = ceil(log2(len)) (0 for len <= 1: nothing to do);
//   3. plan     — queue layout: classes in descending order (largest first);
//                 work items: one per segment of class 15..16, 2^(14-c)
//                 segments of class c = 8..14 per item, 16 segments of
//                 class <= 7 per item;
//   4. scatter  — segment ids into the queue;
//   5. sort     — a persistent grid of 1024-lane workgroups (68 KiB of LDS
//                 each) pulls items from an atomic counter until the queue
//                 is empty.
// Each segment runs the Figure 1 network on its own (padded) length with
// the segment-local index giving the direction. Per stage the caller picks
// the divergent or melded compare-exchange: MELD_LO for phases k <= 64 and
// MELD_HI for k >= 128.
//
// Class <= 7 (up to 128 keys): one wave per segment, the comparator network
// in LDS. Class c = 8..14: a team of 2^(c-4) lanes per segment holding 16
// keys per lane; phases k <= 64 run as the LDS comparator network (team
// lanes take comparators in turn), phases k >= 128 in register windows with
// LDS transposes (the direction is a lane bit for k <= 512). Class 15..16: the
// whole workgroup sorts the segment's 2^14-key chunks as class 14 (odd chunks
// descending), runs the steps j >= 2^14 through global memory inside the
// workgroup and merges each chunk in registers, the segment staged (with its
// padding) in a per-workgroup scratch of 2^16 words. All of it stays inside
// one workgroup, so no grid-wide synchronisation is needed.
#include "device_common.h"
#include "exchange.h"
#include "kernels.h"
#include "network.h"

namespace meld {

namespace {

constexpr uint32_t kPad = 0xFFFFFFFFu;
constexpr uint32_t kWavesPerBlock = kSegThreads / 64;
constexpr uint32_t kSmallMax = 128;
constexpr uint32_t kSmallClassMax = kSegSmallClassMax;

constexpr int kSegE = 16;  // keys per lane in the register phases
// Registers per branch of a divergent lane step: the partner values of 8
// registers at a time keep the kernel within its 64 VGPRs without spills.
constexpr int kSegLaneGroup = 8;

// Hides v's value from the optimiser at this point: the LDS and global
// addresses derived from it are then computed where they are used instead of
// being hoisted out of the persistent loop (which held ~40 of them live
// across the whole kernel and forced spills).
__device__ __forceinline__ void opaque(uint32_t &v) { asm volatile("" : "+v"(v)); }

__device__ __forceinline__ uint32_t padded(uint32_t i) { return i + (i >> 4); }

// For a window index tp | (r << B) the lane bits tp and the register bits are
// disjoint fields, and then padded(tp | b) = padded(tp) + padded(b) (no shifted
// bit of one field meets the other): the lane part is computed once per
// transpose, the register part is a scalar (the window is the workgroup's).

// Window B: element bits [B, B+4) are the register index, the others the lane.
__device__ __forceinline__ uint32_t window_tpart(uint32_t t, uint32_t B) {
    return (t & ((1u << B) - 1)) | ((t >> B) << (B + 4));
}

// Compare-exchange of two registers for direction up, with no branch: min
// and max, then one select per output on the direction.
__device__ __forceinline__ void cex_regs(uint32_t &x, uint32_t &y, bool up) {
    const uint32_t mn = x < y ? x : y;
    const uint32_t mx = x < y ? y : x;
    x = up ? mn : mx;
    y = up ? mx : mn;
}

// One register step on register bit Q: divergent (Figure 1's if/else on the
// direction, the marks keep the two sides apart) or melded (both compares,
// the swap chosen by a select).
template <int Q, bool MELDED>
__device__ __forceinline__ void seg_reg_step(uint32_t (&e)[kSegE], bool up) {
    if constexpr (MELDED) {
#pragma unroll
        for (int r = 0; r < kSegE; ++r)
            if ((r & (1 << Q)) == 0) cex_regs(e[r], e[r | (1 << Q)], up);
    } else {
        if (up) {
            MELD_SIDE_MARK("ascending regs");
#pragma unroll
            for (int r = 0; r < kSegE; ++r)
                if ((r & (1 << Q)) == 0) {
                    const uint32_t x = e[r], y = e[r | (1 << Q)];
                    if (y < x) {
                        e[r] = y;
                        e[r | (1 << Q)] = x;
                    }
                }
        } else {
            MELD_SIDE_MARK("descending regs");
#pragma unroll
            for (int r = 0; r < kSegE; ++r)
                if ((r & (1 << Q)) == 0) {
                    const uint32_t x = e[r], y = e[r | (1 << Q)];
                    if (y > x) {
                        e[r] = y;
                        e[r | (1 << Q)] = x;
                    }
                }
        }
    }
}

template <bool MELDED>
__device__ __forceinline__ void seg_reg_steps(uint32_t (&e)[kSegE], int hi_q, bool up,
                                              int32_t &left) {
    if (hi_q >= 3 && left > 0) {
        seg_reg_step<3, MELDED>(e, up);
        --left;
    }
    if (hi_q >= 2 && left > 0) {
        seg_reg_step<2, MELDED>(e, up);
        --left;
    }
    if (hi_q >= 1 && left > 0) {
        seg_reg_step<1, MELDED>(e, up);
        --left;
    }
    if (left > 0) {
        seg_reg_step<0, MELDED>(e, up);
        --left;
    }
}

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
                                                           uint32_t nseg, uint32_t n_keys,
                                                           SegState *st,
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
        if (hi > n_keys) f |= kSegBeyondEnd;
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

// Work items of class c >= 8: one per segment above 2^14 keys, otherwise
// one per 2^(14-c) segments (one team each).
__device__ __forceinline__ uint32_t class_items(uint32_t c, uint32_t cnt) {
    if (c > kSegLogChunk) return cnt;
    const uint32_t per = 1u << (kSegLogChunk - c);
    return (cnt + per - 1) / per;
}

__global__ void seg_plan_kernel(SegState *st) {
    if (threadIdx.x != 0) return;
    uint32_t pos = 0, items = 0, n_small = 0;
    for (int c = (int)kSegClasses - 1; c >= 1; --c) {
        st->base[c] = pos;
        pos += st->cnt[c];
        if ((uint32_t)c > kSmallClassMax) {
            st->item_base[c] = items;
            items += class_items((uint32_t)c, st->cnt[c]);
        } else {
            n_small += st->cnt[c];
        }
    }
    st->n_big = items;
    st->n_small = n_small;
    st->n_items = items + (n_small + kWavesPerBlock - 1) / kWavesPerBlock;
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

// The 16 registers of window W at their padded LDS positions p[padded(r << W)]
// (p: the lane's part of the index, already padded). With W fixed at compile
// time every position is an immediate offset of the LDS instruction; a window
// base known only at run time would cost three scalar instructions and a
// vector add per register.
template <int W>
__device__ __forceinline__ void window_store_w(const uint32_t (&e)[kSegE], uint32_t *p) {
#pragma unroll
    for (int r = 0; r < kSegE; ++r) p[((uint32_t)r << W) + (((uint32_t)r << W) >> 4)] = e[r];
}
template <int W>
__device__ __forceinline__ void window_load_w(uint32_t (&e)[kSegE], const uint32_t *p) {
#pragma unroll
    for (int r = 0; r < kSegE; ++r) e[r] = p[((uint32_t)r << W) + (((uint32_t)r << W) >> 4)];
}

// Window bases are 0 .. 10 (element bits [W, W + 4) of a tile of at most 2^14
// keys). Each case ends in its own mark so that the compiler keeps the cases
// apart instead of merging them back into one block with computed offsets.
#define SEG_WINDOW_CASE(W, CALL, TAG) \
    case W:                           \
        CALL;                         \
        asm volatile("; window " TAG " " #W ::: "memory"); \
        break;

__device__ __forceinline__ void window_store(const uint32_t (&e)[kSegE], uint32_t *p, uint32_t W) {
    switch (W) {
        SEG_WINDOW_CASE(0, window_store_w<0>(e, p), "store")
        SEG_WINDOW_CASE(1, window_store_w<1>(e, p), "store")
        SEG_WINDOW_CASE(2, window_store_w<2>(e, p), "store")
        SEG_WINDOW_CASE(3, window_store_w<3>(e, p), "store")
        SEG_WINDOW_CASE(4, window_store_w<4>(e, p), "store")
        SEG_WINDOW_CASE(5, window_store_w<5>(e, p), "store")
        SEG_WINDOW_CASE(6, window_store_w<6>(e, p), "store")
        SEG_WINDOW_CASE(7, window_store_w<7>(e, p), "store")
        SEG_WINDOW_CASE(8, window_store_w<8>(e, p), "store")
        SEG_WINDOW_CASE(9, window_store_w<9>(e, p), "store")
        default: window_store_w<10>(e, p); break;
    }
}

__device__ __forceinline__ void window_load(uint32_t (&e)[kSegE], const uint32_t *p, uint32_t W) {
    switch (W) {
        SEG_WINDOW_CASE(0, window_load_w<0>(e, p), "load")
        SEG_WINDOW_CASE(1, window_load_w<1>(e, p), "load")
        SEG_WINDOW_CASE(2, window_load_w<2>(e, p), "load")
        SEG_WINDOW_CASE(3, window_load_w<3>(e, p), "load")
        SEG_WINDOW_CASE(4, window_load_w<4>(e, p), "load")
        SEG_WINDOW_CASE(5, window_load_w<5>(e, p), "load")
        SEG_WINDOW_CASE(6, window_load_w<6>(e, p), "load")
        SEG_WINDOW_CASE(7, window_load_w<7>(e, p), "load")
        SEG_WINDOW_CASE(8, window_load_w<8>(e, p), "load")
        SEG_WINDOW_CASE(9, window_load_w<9>(e, p), "load")
        default: window_load_w<10>(e, p); break;
    }
}
#undef SEG_WINDOW_CASE

// Moves e from window cur to window B through the padded LDS tile.
__device__ __forceinline__ void to_window(uint32_t (&e)[kSegE], uint32_t *s, uint32_t t,
                                          uint32_t &cur, uint32_t B) {
    if (B == cur) return;
    window_store(e, s + padded(window_tpart(t, cur)), cur);
    __syncthreads();
    window_load(e, s + padded(window_tpart(t, B)), B);
    __syncthreads();
    cur = B;
}

// Steps of phase k = 2^p on element bits hi_bit .. 0 of a tile held in
// registers, 16 per lane (lane t of the tile's nt lanes): windows with bases
// hi_bit-3, hi_bit-7, ... (clamped at 0). cur is the window e is in.
template <bool MELDED>
__device__ __forceinline__ void phase_windows(uint32_t (&e)[kSegE], uint32_t *s, uint32_t t,
                                              uint32_t &cur, int hi_bit, bool up) {
    int32_t unlimited = 0x7FFFFFFF;
#pragma unroll 1
    for (int top = hi_bit; top >= 0;) {
        const uint32_t B = top >= 3 ? (uint32_t)(top - 3) : 0u;
        to_window(e, s, t, cur, B);
        seg_reg_steps<MELDED>(e, top - (int)B, up, unlimited);
        top = (int)B - 1;
    }
}

// Phase steps on element bits hi_bit .. 0 ending in layout W0 (register r of
// lane t holds element 16 t + r): four-bit windows with bases hi_bit-3,
// hi_bit-7, ... while the top bit is at least 6, then W0, where the steps on
// element bits 5 and 4 are DPP exchanges with lane t ^ 2 and t ^ 1 and bits
// 3 .. 0 registers. One LDS transpose fewer than phase_windows when hi_bit is
// 8, 9, 12 or 13.
template <bool MELDED>
__device__ __forceinline__ void phase_windows_xch(uint32_t (&e)[kSegE], uint32_t *s, uint32_t t,
                                                  uint32_t &cur, int hi_bit, bool up) {
    int32_t unlimited = 0x7FFFFFFF;
    int top = hi_bit;
#pragma unroll 1
    while (top >= 6) {
        const uint32_t B = (uint32_t)(top - 3);
        to_window(e, s, t, cur, B);
        seg_reg_steps<MELDED>(e, 3, up, unlimited);
        top = (int)B - 1;
    }
    to_window(e, s, t, cur, 0);
    if (top >= 5) lane_step<1, MELDED, kSegLaneGroup>(e, up, ((t >> 1) & 1u) == 0);
    if (top >= 4) lane_step<0, MELDED, kSegLaneGroup>(e, up, (t & 1u) == 0);
    seg_reg_steps<MELDED>(e, top < 3 ? top : 3, up, unlimited);
}

// to_window and phase_windows_xch with every window base known at compile
// time (CUR: the window e is in; TOP: the highest step bit left), for the
// sizes that dominate the work: 2^14-key chunks and their merges.
template <int CUR, int B>
__device__ __forceinline__ void to_window_c(uint32_t (&e)[kSegE], uint32_t *s, uint32_t t) {
    if constexpr (CUR != B) {
        window_store_w<CUR>(e, s + padded(window_tpart(t, CUR)));
        __syncthreads();
        window_load_w<B>(e, s + padded(window_tpart(t, B)));
        __syncthreads();
    }
}

template <bool MELDED, int TOP, int CUR>
__device__ __forceinline__ void phase_windows_xch_c(uint32_t (&e)[kSegE], uint32_t *s, uint32_t t,
                                                    bool up) {
    int32_t unlimited = 0x7FFFFFFF;
    if constexpr (TOP >= 6) {
        constexpr int B = TOP - 3;
        to_window_c<CUR, B>(e, s, t);
        seg_reg_steps<MELDED>(e, 3, up, unlimited);
        phase_windows_xch_c<MELDED, B - 1, B>(e, s, t, up);
    } else {
        to_window_c<CUR, 0>(e, s, t);
        if constexpr (TOP >= 5) lane_step<1, MELDED, kSegLaneGroup>(e, up, ((t >> 1) & 1u) == 0);
        if constexpr (TOP >= 4) lane_step<0, MELDED, kSegLaneGroup>(e, up, (t & 1u) == 0);
        seg_reg_steps<MELDED>(e, TOP < 3 ? TOP : 3, up, unlimited);
    }
}

// Phases 2^P .. 2^M of a team sort on the lane-exchange path, each starting
// and ending in W0.
template <bool MELDED, int P, int M>
__device__ __forceinline__ void team_phases_xch_c(uint32_t (&e)[kSegE], uint32_t *s, uint32_t t,
                                                  uint32_t cbase) {
    if constexpr (P <= M) {
        const bool up = (((cbase >> P) | (t >> (P - 4))) & 1u) == 0;
        phase_windows_xch_c<MELDED, P - 1, 0>(e, s, t, up);
        team_phases_xch_c<MELDED, P + 1, M>(e, s, t, cbase);
    }
}

// A team of 2^(m-4) lanes (lane t) sorts the 2^m positions cbase + i of a
// segment (8 <= m <= 14): positions below len come from keys[lo + q], the
// others are padding. s is the team's own LDS region of 17 * 2^(m-4) words.
// With work != nullptr every result goes to work[q]; otherwise results
// below len go to keys and the padding is dropped. The direction of phase p
// is bit p of cbase + i, so a chunk with bit m of cbase set ends descending.
// XCH: phases k <= 64 in registers with lane exchanges (the tile moved to
// layout W0 first) and the later phases ending each in W0; otherwise the LDS
// comparator network and four-bit windows.
template <bool MELD_LO, bool MELD_HI, bool XCH>
__device__ __forceinline__ void team_sort(uint32_t *__restrict__ keys,
                                          uint32_t *__restrict__ work, uint32_t *s, uint32_t lo,
                                          uint32_t len, uint32_t m, uint32_t cbase, uint32_t t) {
    opaque(t);
    // Global accesses as a uniform base (chunk and register row, scalar
    // arithmetic) plus the lane's 32-bit offset; the mask gives t's range back
    // after opaque, which that addressing form needs.
    const uint32_t tl = t & (kSegThreads - 1);
    const uint32_t lt = m - 4;
    uint32_t e[kSegE];
#pragma unroll
    for (int r = 0; r < kSegE; ++r) {
        const uint32_t rb = cbase + ((uint32_t)r << lt);
        e[r] = rb + tl < len ? (keys + lo + rb)[tl] : kPad;
    }
    uint32_t cur;
    if constexpr (XCH) {
        cur = lt;
        to_window(e, s, t, cur, 0);
        xch_network_low<MELD_LO, kSegLaneGroup>(e, t, -1);
        if (MELD_HI && m == kSegLogChunk) {
            team_phases_xch_c<MELD_HI, 7, (int)kSegLogChunk>(e, s, t, cbase);
        } else {
#pragma unroll 1
            for (uint32_t p = 7; p <= m; ++p) {
                const bool up = (((cbase >> p) | (t >> (p - 4))) & 1u) == 0;
                phase_windows_xch<MELD_HI>(e, s, t, cur, (int)p - 1, up);
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < kSegE; ++r) s[low_swz<uint32_t>(t | ((uint32_t)r << lt))] = e[r];
        __syncthreads();
        lds_network_low<uint32_t, MELD_LO, 8, true>(s, cbase, 6, t, 1u << lt, -1);
        __syncthreads();
        // Phase 2^7 starts in window 3 (element bits 3..6), read from the natural
        // order the comparator network leaves in s.
        cur = 3;
        {
            const uint32_t tb = window_tpart(t, cur);
#pragma unroll
            for (int r = 0; r < kSegE; ++r) e[r] = s[low_swz<uint32_t>(tb | ((uint32_t)r << cur))];
            __syncthreads();
        }
#pragma unroll 1
        for (uint32_t p = 7; p <= m; ++p) {
            const bool up = (((cbase >> p) | (t >> (p - 4))) & 1u) == 0;
            phase_windows<MELD_HI>(e, s, t, cur, (int)p - 1, up);
        }
    }
    to_window(e, s, t, cur, lt);
    if (work != nullptr) {
#pragma unroll
        for (int r = 0; r < kSegE; ++r) (work + cbase + ((uint32_t)r << lt))[tl] = e[r];
    } else {
#pragma unroll
        for (int r = 0; r < kSegE; ++r) {
            const uint32_t rb = cbase + ((uint32_t)r << lt);
            if (rb + tl < len) (keys + lo + rb)[tl] = e[r];
        }
    }
}

// Steps j = 2^(p-1) .. 2^14 of phase 2^p over the 2^m positions of a
// segment held in the workgroup's scratch (p <= m <= 16, so one or two
// steps), in registers.
__device__ void seg_global_steps(uint32_t *__restrict__ work, uint32_t m, uint32_t p,
                                 uint32_t tid) {
    __syncthreads();  // the chunks' stores are visible to the workgroup
    const uint32_t d = p - kSegLogChunk;  // 1 or 2
    const uint32_t groups = 1u << (m - d);
#pragma unroll 1
    for (uint32_t g = tid; g < groups; g += kSegThreads) {
        const uint32_t base = (g & (kSegChunk - 1)) | ((g >> kSegLogChunk) << p);
        const bool up = ((base >> p) & 1u) == 0;
        uint32_t *w = work + base;
        uint32_t v0 = w[0], v1 = w[kSegChunk];
        if (d == 1) {
            cex_regs(v0, v1, up);
        } else {
            uint32_t v2 = w[2 * kSegChunk], v3 = w[3 * kSegChunk];
            cex_regs(v0, v2, up);  // j = 2^15
            cex_regs(v1, v3, up);
            cex_regs(v0, v1, up);  // j = 2^14
            cex_regs(v2, v3, up);
            w[2 * kSegChunk] = v2;
            w[3 * kSegChunk] = v3;
        }
        w[0] = v0;
        w[kSegChunk] = v1;
    }
    __syncthreads();
}

// Steps j = 2^13 .. 1 of a phase on chunk cbase of a segment in the
// workgroup's scratch; the direction is the same for the whole chunk, so
// both forms coincide. The last phase writes the positions below len to the
// caller's keys, earlier ones write back to the scratch. XCH: the steps end
// in layout W0 with lane exchanges (three transposes instead of four).
template <bool XCH>
__device__ void chunk_merge(uint32_t *__restrict__ keys, uint32_t *__restrict__ work, uint32_t *s,
                            uint32_t lo, uint32_t len, uint32_t cbase, uint32_t t, bool up,
                            bool last) {
    opaque(t);
    const uint32_t tl = t & (kSegThreads - 1);  // as in team_sort
    constexpr uint32_t lt = kSegLogChunk - 4;
    uint32_t e[kSegE];
#pragma unroll
    for (int r = 0; r < kSegE; ++r) e[r] = (work + cbase + ((uint32_t)r << lt))[tl];
    uint32_t cur = lt;
    if constexpr (XCH) {
        phase_windows_xch_c<true, (int)kSegLogChunk - 1, (int)lt>(e, s, t, up);
        cur = 0;
    } else {
        phase_windows<true>(e, s, t, cur, (int)kSegLogChunk - 1, up);
    }
    to_window(e, s, t, cur, lt);
    if (last) {
#pragma unroll
        for (int r = 0; r < kSegE; ++r) {
            const uint32_t rb = cbase + ((uint32_t)r << lt);
            if (rb + tl < len) (keys + lo + rb)[tl] = e[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < kSegE; ++r) (work + cbase + ((uint32_t)r << lt))[tl] = e[r];
    }
}

// A segment of class 15..16 in 2^14-key chunks (the whole workgroup),
// staged in the workgroup's scratch of 2^16 words.
template <bool MELD_LO, bool MELD_HI, bool XCH>
__device__ void sort_chunked(uint32_t *__restrict__ keys, uint32_t *s, uint32_t *__restrict__ work,
                             uint32_t lo, uint32_t len, uint32_t m, uint32_t tid) {
    const uint32_t chunks = 1u << (m - kSegLogChunk);
#pragma unroll 1
    for (uint32_t h = 0; h < chunks; ++h)
        team_sort<MELD_LO, MELD_HI, XCH>(keys, work, s, lo, len, kSegLogChunk, h << kSegLogChunk,
                                         tid);
#pragma unroll 1
    for (uint32_t p = kSegLogChunk + 1; p <= m; ++p) {
        seg_global_steps(work, m, p, tid);
#pragma unroll 1
        for (uint32_t h = 0; h < chunks; ++h) {
            const uint32_t cbase = h << kSegLogChunk;
            chunk_merge<XCH>(keys, work, s, lo, len, cbase, tid, ((cbase >> p) & 1u) == 0,
                             p == m);
        }
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

template <bool MELD_LO, bool MELD_HI, bool XCH>
// At most 64 VGPRs (8 waves per SIMD): two 1024-lane workgroups fit on a CU
// (2 x 68 KiB of LDS), which hides the barriers and LDS latency of the
// network steps better than one (measured on the 4096-segment workload: 19 %
// faster than at 87 VGPRs with one workgroup per CU). The global accesses of
// a lane's 16 keys take a uniform base plus a 32-bit lane offset, which
// keeps the kernel at 61 VGPRs without spills.
__global__ __launch_bounds__(kSegThreads, 8) void seg_sort_kernel(uint32_t *__restrict__ keys,
                                                               const uint32_t *__restrict__ off,
                                                               const uint32_t *__restrict__ queue,
                                                               SegState *st,
                                                               uint32_t *__restrict__ work_all) {
    extern __shared__ __align__(16) uint32_t s[];
    __shared__ uint32_t item_sh;
    if (st->flag != 0) return;  // invalid offsets: leave the keys untouched
    const uint32_t n_items = st->n_items;
    const uint32_t n_big = st->n_big;
    const uint32_t n_small = st->n_small;
    uint32_t *work = work_all + (size_t)blockIdx.x * kSegWorkWords;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) item_sh = atomicAdd(&st->head, 1u);
        __syncthreads();
        const uint32_t item = item_sh;
        __syncthreads();
        if (item >= n_items) break;  // every wave of every workgroup reaches this
        if (item < n_big) {
            // the class whose items hold this one (classes 16 .. 8 in order)
            uint32_t c = kSmallClassMax + 1;
            for (uint32_t k = kSegClasses - 1; k > kSmallClassMax; --k) {
                const uint32_t first = st->item_base[k];
                if (item >= first && item < first + class_items(k, st->cnt[k])) {
                    c = k;
                    break;
                }
            }
            const uint32_t k = item - st->item_base[c];
            if (c > kSegLogChunk) {
                const uint32_t seg = queue[st->base[c] + k];
                const uint32_t lo = off[seg];
                sort_chunked<MELD_LO, MELD_HI, XCH>(keys, s, work, lo, off[seg + 1] - lo, c, tid);
            } else {
                const uint32_t lt = c - 4;
                const uint32_t team = tid >> lt, t = tid & ((1u << lt) - 1);
                const uint32_t qi = (k << (kSegLogChunk - c)) + team;
                uint32_t lo = 0, len = 0;  // a team past the class's last segment idles
                if (qi < st->cnt[c]) {
                    const uint32_t seg = queue[st->base[c] + qi];
                    lo = off[seg];
                    len = off[seg + 1] - lo;
                }
                team_sort<MELD_LO, MELD_HI, XCH>(keys, nullptr, s + team * (17u << lt), lo, len, c,
                                                 0, t);
            }
        } else {
            const uint32_t w = tid >> 6;
            const uint32_t qi = st->base[kSmallClassMax] + (item - n_big) * kWavesPerBlock + w;
            if (qi < st->base[kSmallClassMax] + n_small) {
                const uint32_t seg = queue[qi];
                const uint32_t lo = off[seg];
                sort_small<MELD_LO, MELD_HI>(keys, s + w * kSmallMax, lo, off[seg + 1] - lo,
                                             tid & 63);
            }
            __syncthreads();
        }
    }
}

template <bool LO, bool HI, bool XCH>
hipError_t launch_sort_t(uint32_t *keys, const uint32_t *off, const uint32_t *queue, SegState *st,
                         uint32_t *work, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL((seg_sort_kernel<LO, HI, XCH>), dim3(grid), dim3(kSegThreads),
                       kSegLdsWords * sizeof(uint32_t), stream, keys, off, queue, st, work);
    return hipGetLastError();
}

template <bool XCH>
hipError_t launch_sort_x(uint32_t *keys, const uint32_t *off, const uint32_t *queue, SegState *st,
                         uint32_t *work, uint32_t grid, bool lo, bool hi, hipStream_t stream) {
    if (lo)
        return hi ? launch_sort_t<true, true, XCH>(keys, off, queue, st, work, grid, stream)
                  : launch_sort_t<true, false, XCH>(keys, off, queue, st, work, grid, stream);
    return hi ? launch_sort_t<false, true, XCH>(keys, off, queue, st, work, grid, stream)
              : launch_sort_t<false, false, XCH>(keys, off, queue, st, work, grid, stream);
}

template <bool LO, bool HI, bool XCH>
hipError_t allow_big_lds() {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(seg_sort_kernel<LO, HI, XCH>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kSegLdsWords * sizeof(uint32_t)));
}

}  // namespace

hipError_t seg_sort_grid(int device, uint32_t *grid) {
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    // The LDS limit is raised for every form up front, outside any capture.
    for (hipError_t r :
         {allow_big_lds<true, true, false>(), allow_big_lds<true, false, false>(),
          allow_big_lds<false, true, false>(), allow_big_lds<false, false, false>(),
          allow_big_lds<true, true, true>(), allow_big_lds<true, false, true>(),
          allow_big_lds<false, true, true>(), allow_big_lds<false, false, true>()})
        if (r != hipSuccess) return r;
    // The grid is sized for the form with the fewest resident workgroups.
    per_cu = 1 << 30;
    for (const void *k : {reinterpret_cast<const void *>(seg_sort_kernel<true, true, false>),
                          reinterpret_cast<const void *>(seg_sort_kernel<false, false, false>),
                          reinterpret_cast<const void *>(seg_sort_kernel<true, true, true>),
                          reinterpret_cast<const void *>(seg_sort_kernel<false, false, true>)}) {
        int b = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, kSegThreads,
                                                         kSegLdsWords * sizeof(uint32_t));
        if (e != hipSuccess) return e;
        if (b < per_cu) per_cu = b;
    }
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    *grid = (uint32_t)(cus * per_cu);
    return hipSuccess;
}

hipError_t launch_segmented_sort(uint32_t *keys, uint32_t n_keys, const uint32_t *off,
                                 uint32_t nseg, SegState *st, uint8_t *cls, uint32_t *queue,
                                 uint32_t *work, uint32_t grid, bool meld_lo, bool meld_hi,
                                 bool xch, hipStream_t stream) {
    if (nseg == 0) return hipSuccess;
    const uint32_t blocks = (nseg + 255) / 256;
    hipLaunchKernelGGL(seg_reset_kernel, dim3(1), dim3(64), 0, stream, st);
    hipLaunchKernelGGL(seg_classify_kernel, dim3(blocks), dim3(256), 0, stream, off, nseg, n_keys,
                       st, cls);
    hipLaunchKernelGGL(seg_plan_kernel, dim3(1), dim3(64), 0, stream, st);
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(blocks), dim3(256), 0, stream, nseg, cls, st,
                       queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return xch ? launch_sort_x<true>(keys, off, queue, st, work, grid, meld_lo, meld_hi, stream)
               : launch_sort_x<false>(keys, off, queue, st, work, grid, meld_lo, meld_hi, stream);
}

}  // namespace meld
