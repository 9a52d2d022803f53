// Two-sided loop region: divergent (IPDOM) and melded forms.
//
// Per lane i the region computes (Evaluation section, "Synthetic Benchmarks":
// a divergent region inside a loop whose two sides hold the same instruction
// sequence on different data):
//   taken = (mix64(bkey + i) >> 32) < thr
//   s     = taken ? T : F
//   acc   = x[i];  for k < s.trips: acc = fma(acc, s.a, tab[(i + s.off + k*s.step) & mask])
//   y[i]  = acc
//
// Divergent form: `if (taken) loop_T else loop_F`. In a wave holding both
// kinds of lanes the two loops run one after the other under exec masks.
//
// Melded form (Detailed Design section, Algorithm 2 and "Unpredication"):
// the two loops are isomorphic subgraphs and become one loop whose exit runs
// to min(T.trips, F.trips), which both sides share; the |T.trips - F.trips|
// steps only the longer side has are unaligned and run in a conditional block
// entered by that side's lanes only, with that side's own (uniform) operands.
// Inside the melded loop the fma is aligned (its multiplier selected once per
// lane, a v_cndmask). The gathers read different addresses on the two sides;
// the library leaves them unaligned, each side's batch of gathers in one
// conditional block, because on gfx950 one gather serving two address
// streams costs more than two single-stream gathers (the paper notes the same
// for global memory: melded accesses to different cache lines gain little).
// The form with the gathers aligned too is kept as MELD_MELDED_INPLACE.
//
// Both forms issue the gathers of a batch of consecutive steps before the
// dependent fmas (the gathers do not depend on acc), and both keep the fma
// order of the definition, so their results are bit-identical. Lanes are
// numbered so that each XCD runs one contiguous range of them: a table entry
// read by lane i at step k is read again by lane i + step at step k - 1, and
// with the hardware's round-robin placement such lanes would sit in another
// XCD's L2 (table traffic 250 -> 135 MB per 2^24 lanes).
#include "device_common.h"
#include "kernels.h"

namespace meld {

namespace {

constexpr int kRegionThreads = 256;

// Gathers of G consecutive steps of one side, issued back to back (they do
// not depend on acc); the fmas that consume them run afterwards.
template <int G>
__device__ __forceinline__ void gather_group(float (&g)[G], uint32_t idx, uint32_t step,
                                             const float *__restrict__ tab, uint32_t mask) {
#pragma unroll
    for (int u = 0; u < G; ++u) g[u] = tab[(idx + (uint32_t)u * step) & mask];
}

template <int G>
__device__ __forceinline__ float fma_group(float acc, float a, const float (&g)[G]) {
#pragma unroll
    for (int u = 0; u < G; ++u) acc = __builtin_fmaf(acc, a, g[u]);
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

__device__ __forceinline__ float fma_chunk(float acc, float a, const Chunk &ch, uint32_t c) {
    if (c & 8) acc = fma_group(acc, a, ch.g8);
    if (c & 4) acc = fma_group(acc, a, ch.g4);
    if (c & 2) acc = fma_group(acc, a, ch.g2);
    if (c & 1) acc = fma_group(acc, a, ch.g1);
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
__device__ __forceinline__ float side_steps(float acc, uint32_t idx, uint32_t steps, float a,
                                            uint32_t step, const float *__restrict__ tab,
                                            uint32_t mask) {
    uint32_t k = 0;
    for (; k + kChunkMax <= steps; k += kBatch) {
        float g[kBatch];
        gather_group(g, idx, step, tab, mask);
        acc = fma_group(acc, a, g);
        idx += kBatch * step;
    }
    const uint32_t c = steps - k;
    if (c != 0) {
        Chunk ch;
        gather_chunk(ch, c, idx, step, tab, mask);
        acc = fma_chunk(acc, a, ch, c);
    }
    return acc;
}

__device__ __forceinline__ bool branch_taken(uint64_t bkey, uint32_t i, uint64_t thr) {
    return (mix64(bkey + i) >> 32) < thr;
}

__global__ __launch_bounds__(kRegionThreads) void region_divergent_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr, RegionSide T, RegionSide F) {
    const uint32_t i =
        xcd_contiguous_block(blockIdx.x, gridDim.x) * kRegionThreads + threadIdx.x;
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    float acc = x[i];
    if (taken) {
        MELD_SIDE_MARK("true");
        acc = side_steps(acc, i + T.off, T.trips, T.a, T.step, tab, mask);
    } else {
        MELD_SIDE_MARK("false");
        acc = side_steps(acc, i + F.off, F.trips, F.a, F.step, tab, mask);
    }
    y[i] = acc;
}

// Melded loop over the steps both sides have, with the gathers left
// unaligned: the side-specific gathers of a batch sit in one conditional
// block per side (what unpredication makes of consecutive unaligned
// instructions), while the index arithmetic, the fma chain and the loop
// control run once on the whole wave with the multiplier selected per lane.
// Same batching as side_steps.
__device__ __forceinline__ float melded_common_steps(float acc, bool taken, uint32_t idx_t,
                                                     uint32_t idx_f, uint32_t steps, float a,
                                                     uint32_t step_t, uint32_t step_f,
                                                     const float *__restrict__ tab,
                                                     uint32_t mask) {
    uint32_t k = 0;
    for (; k + kChunkMax <= steps; k += kBatch) {
        float g[kBatch];
        if (taken) {
            MELD_SIDE_MARK("gathers true");
            gather_group(g, idx_t, step_t, tab, mask);
        } else {
            MELD_SIDE_MARK("gathers false");
            gather_group(g, idx_f, step_f, tab, mask);
        }
        acc = fma_group(acc, a, g);
        idx_t += kBatch * step_t;
        idx_f += kBatch * step_f;
    }
    const uint32_t c = steps - k;
    if (c != 0) {
        Chunk ch;
        if (taken) {
            MELD_SIDE_MARK("gathers true");
            gather_chunk(ch, c, idx_t, step_t, tab, mask);
        } else {
            MELD_SIDE_MARK("gathers false");
            gather_chunk(ch, c, idx_f, step_f, tab, mask);
        }
        acc = fma_chunk(acc, a, ch, c);
    }
    return acc;
}

// Steps only the longer side has: unaligned, run by that side's lanes with
// that side's own operands.
__device__ __forceinline__ float longer_side_steps(float acc, uint32_t i, bool taken,
                                                   const float *__restrict__ tab, uint32_t mask,
                                                   const RegionSide &T, const RegionSide &F,
                                                   uint32_t common) {
    const bool true_longer = T.trips > F.trips;
    const uint32_t extra = true_longer ? T.trips - common : F.trips - common;
    if (extra != 0 && taken == true_longer) {
        const RegionSide L = true_longer ? T : F;
        acc = side_steps(acc, i + L.off + common * L.step, extra, L.a, L.step, tab, mask);
    }
    return acc;
}

// The melded form used by the library.
__global__ __launch_bounds__(kRegionThreads) void region_melded_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr, RegionSide T, RegionSide F) {
    const uint32_t i =
        xcd_contiguous_block(blockIdx.x, gridDim.x) * kRegionThreads + threadIdx.x;
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    const float a = taken ? T.a : F.a;  // differing operand of the aligned fma: a select
    const uint32_t common = T.trips < F.trips ? T.trips : F.trips;
    float acc = x[i];
    acc = melded_common_steps(acc, taken, i + T.off, i + F.off, common, a, T.step, F.step, tab,
                              mask);
    y[i] = longer_side_steps(acc, i, taken, tab, mask, T, F, common);
}

// The melded form with the gathers aligned as well: one gather instruction per
// step serves both sides, its address selected per lane. This is the melded
// code as the transformation emits it when it pairs the two loads; on gfx950
// a gather whose lanes mix two address streams costs several times the
// vector-memory work of one lane-linear stream, which makes this form slower
// than the divergent one whenever the sides read different data.
__global__ __launch_bounds__(kRegionThreads) void region_melded_inplace_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr, RegionSide T, RegionSide F) {
    const uint32_t i =
        xcd_contiguous_block(blockIdx.x, gridDim.x) * kRegionThreads + threadIdx.x;
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    const float a = taken ? T.a : F.a;
    const uint32_t off = taken ? T.off : F.off;
    const uint32_t step = taken ? T.step : F.step;
    const uint32_t common = T.trips < F.trips ? T.trips : F.trips;
    float acc = side_steps(x[i], i + off, common, a, step, tab, mask);
    y[i] = longer_side_steps(acc, i, taken, tab, mask, T, F, common);
}

}  // namespace

hipError_t launch_region(const float *x, float *y, uint32_t n, const float *tab, uint32_t mask,
                         uint64_t seed, uint64_t thr, RegionSide T, RegionSide F, RegionForm form,
                         hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint64_t bkey = stream_key(seed, 4);
    const dim3 grid((n + kRegionThreads - 1) / kRegionThreads);
    if (form == RegionForm::kMelded)
        hipLaunchKernelGGL(region_melded_kernel, grid, dim3(kRegionThreads), 0, stream, x, y, n,
                           tab, mask, bkey, thr, T, F);
    else if (form == RegionForm::kMeldedInPlace)
        hipLaunchKernelGGL(region_melded_inplace_kernel, grid, dim3(kRegionThreads), 0, stream, x,
                           y, n, tab, mask, bkey, thr, T, F);
    else
        hipLaunchKernelGGL(region_divergent_kernel, grid, dim3(kRegionThreads), 0, stream, x, y,
                           n, tab, mask, bkey, thr, T, F);
    return hipGetLastError();
}

}  // namespace meld
