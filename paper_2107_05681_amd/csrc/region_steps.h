// Loop steps of the region kernels (shared by the two-sided, three-way and
// per-lane-trip regions): one step is acc = fma(acc, a, tab[idx & mask]) with
// idx advancing by the side's stride. Gathers are issued ahead of the fmas
// that consume them; the fma order is the definition's, so every form
// computes the same values.
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace meld {

namespace {

constexpr int kRegionThreads = 256;
// Lanes per launch: HIP caps a grid dimension at 2^32 - 1 work-items, so a
// call on more lanes runs as several launches, each told its first lane.
constexpr uint64_t kRegionLaunchLanes = 1ull << 31;

// Branch of lane i: the upper 32 bits of stream (seed, 4) at i against thr.
__device__ __forceinline__ bool branch_taken(uint64_t bkey, uint32_t i, uint64_t thr) {
    return (mix64(bkey + i) >> 32) < thr;
}

// Gathers of G consecutive steps of one side, issued back to back (they do
// not depend on acc); the fmas that consume them run afterwards.
template <int G>
__device__ __forceinline__ void gather_group(float (&g)[G], uint32_t idx, uint32_t step,
                                             const float *__restrict__ tab, uint32_t mask) {
#pragma unroll
    for (int u = 0; u < G; ++u) g[u] = tab[(idx + (uint32_t)u * step) & mask];
}

// One step's arithmetic: the region's fma, or (ONLY_GATHERS, for measuring
// what the gathers alone cost) an integer xor of the gathered bits.
template <bool ONLY_GATHERS>
__device__ __forceinline__ float step_op(float acc, float a, float g) {
    if constexpr (ONLY_GATHERS)
        return __uint_as_float(__float_as_uint(acc) ^ __float_as_uint(g));
    else
        return __builtin_fmaf(acc, a, g);
}

template <int G, bool ONLY_GATHERS = false>
__device__ __forceinline__ float fma_group(float acc, float a, const float (&g)[G]) {
#pragma unroll
    for (int u = 0; u < G; ++u) acc = step_op<ONLY_GATHERS>(acc, a, g[u]);
    return acc;
}

// The gathers of a final chunk of c < 16 steps, in groups of 8, 4, 2 and 1 on
// the bits of c (uniform branches), all issued before any of its fmas.
struct Chunk {
    float g8[8], g4[4], g2[2], g1[1];
};

__device__ __forceinline__ void gather_chunk(Chunk &ch, uint32_t c, uint32_t idx, uint32_t step,
                                             const float *__restrict__ tab, uint32_t mask) {
    if (c & 8) {
        gather_group(ch.g8, idx, step, tab, mask);
        idx += 8 * step;
    }
    if (c & 4) {
        gather_group(ch.g4, idx, step, tab, mask);
        idx += 4 * step;
    }
    if (c & 2) {
        gather_group(ch.g2, idx, step, tab, mask);
        idx += 2 * step;
    }
    if (c & 1) gather_group(ch.g1, idx, step, tab, mask);
}

template <bool ONLY_GATHERS = false>
__device__ __forceinline__ float fma_chunk(float acc, float a, const Chunk &ch, uint32_t c) {
    if (c & 8) acc = fma_group<8, ONLY_GATHERS>(acc, a, ch.g8);
    if (c & 4) acc = fma_group<4, ONLY_GATHERS>(acc, a, ch.g4);
    if (c & 2) acc = fma_group<2, ONLY_GATHERS>(acc, a, ch.g2);
    if (c & 1) acc = fma_group<1, ONLY_GATHERS>(acc, a, ch.g1);
    return acc;
}

// Batches of 8 steps while at least 16 remain, then the last c < 16 steps as
// one chunk with all its gathers in flight. From a sweep over trip counts
// 8..32 on gfx950: batches of 8 beat longer ones for long loops, and a final
// chunk issued whole beats a guarded remainder (10 trips: 8 + 2 in one chunk
// ran 1.1-1.2x faster than a batch of 8 followed by a guarded tail).
constexpr uint32_t kBatch = 8;
constexpr uint32_t kChunkMax = 2 * kBatch;

// Steps of one side.
template <bool ONLY_GATHERS = false>
__device__ __forceinline__ float side_steps(float acc, uint32_t idx, uint32_t steps, float a,
                                            uint32_t step, const float *__restrict__ tab,
                                            uint32_t mask) {
    uint32_t k = 0;
    for (; k + kChunkMax <= steps; k += kBatch) {
        float g[kBatch];
        gather_group(g, idx, step, tab, mask);
        acc = fma_group<kBatch, ONLY_GATHERS>(acc, a, g);
        idx += kBatch * step;
    }
    const uint32_t c = steps - k;
    if (c != 0) {
        Chunk ch;
        gather_chunk(ch, c, idx, step, tab, mask);
        acc = fma_chunk<ONLY_GATHERS>(acc, a, ch, c);
    }
    return acc;
}

// Melded loop over the steps both sides have, with the gathers left
// unaligned: the side-specific gathers of a batch sit in one conditional
// block per side (what unpredication makes of consecutive unaligned
// instructions), while the index arithmetic, the fma chain and the loop
// control run once on the whole wave with the multiplier selected per lane.
// Same batching as side_steps.
template <bool ONLY_GATHERS = false>
__device__ __forceinline__ float melded_common_steps(float acc, bool taken, uint32_t idx_t,
                                                     uint32_t idx_f, uint32_t steps, float a,
                                                     uint32_t step_t, uint32_t step_f,
                                                     const float *__restrict__ tab,
                                                     uint32_t mask) {
    uint32_t k = 0;
    for (; k + kChunkMax <= steps; k += kBatch) {
        // The end marks keep every gather inside its side's block: without
        // them the compiler sinks the two blocks' last gathers into one gather
        // after the join, whose address is selected per lane, the costly
        // mixed-stream form. Each side loads into registers of its own (the
        // fma operand is selected per lane): loads into the same registers
        // make the compiler wait for one side's gathers before issuing the
        // other's.
        float gt[kBatch], gf[kBatch];
        if (taken) {
            MELD_SIDE_MARK("gathers true");
            gather_group(gt, idx_t, step_t, tab, mask);
            MELD_SIDE_MARK("gathers true end");
        } else {
            MELD_SIDE_MARK("gathers false");
            gather_group(gf, idx_f, step_f, tab, mask);
            MELD_SIDE_MARK("gathers false end");
        }
        float g[kBatch];
#pragma unroll
        for (int u = 0; u < (int)kBatch; ++u) g[u] = taken ? gt[u] : gf[u];
        acc = fma_group<kBatch, ONLY_GATHERS>(acc, a, g);
        idx_t += kBatch * step_t;
        idx_f += kBatch * step_f;
    }
    const uint32_t c = steps - k;
    if (c != 0) {
        Chunk ch;
        if (taken) {
            MELD_SIDE_MARK("gathers true");
            gather_chunk(ch, c, idx_t, step_t, tab, mask);
            MELD_SIDE_MARK("gathers true end");
        } else {
            MELD_SIDE_MARK("gathers false");
            gather_chunk(ch, c, idx_f, step_f, tab, mask);
            MELD_SIDE_MARK("gathers false end");
        }
        acc = fma_chunk<ONLY_GATHERS>(acc, a, ch, c);
    }
    return acc;
}

}  // namespace

}  // namespace meld
