// Variants of the divergent loop region (Evaluation section, synthetic
// benchmarks): a three-way if / else-if / else region whose three blocks
// compute alike on different data (SB4), and the two-sided region with a
// trip count drawn per lane.
//
// Three-way, per lane i: h = mix64(bkey + i) >> 32; way = h < thr0 ? 0 :
// h < thr1 ? 1 : 2; the way's loop as in the two-sided region.
//   divergent: the if / else-if / else chain as written; a wave holding all
//     three kinds of lanes runs the three loops one after another.
//   melded (region replication, Detailed Design, "Basic block-Region
//     Melding", then Algorithm 2 and unpredication): the chain becomes one
//     loop. With the ways' trip counts sorted as b1 <= b2 <= b3, the first b1
//     steps are melded across all three ways, steps b1..b2 across the two
//     longest ways (lanes of the shortest way are masked off), steps b2..b3
//     run by the longest way alone. The multiplier is selected per lane (one
//     aligned fma); the gathers stay unaligned, one conditional block per way.
//   melded in place: the gathers aligned too, their address operands
//     selected per lane.
//
// Per-lane trips: lane i of side s runs lo_s + ((H(seed, 11, i) >> 32) mod
// (hi_s - lo_s + 1)) steps, so the loop exit itself diverges inside a wave.
//   divergent: if (taken) loop_T else loop_F, each loop exiting per lane.
//   melded: one loop for both sides, each lane leaving after its own trip
//     count; gathers in per-side blocks, the fma aligned.
//   melded in place: the same with aligned gathers.
#include "device_common.h"
#include "kernels.h"
#include "region_steps.h"

namespace meld {

namespace {

__device__ __forceinline__ uint32_t lane_index(uint32_t lane0) {
    return lane0 + xcd_contiguous_block(blockIdx.x, gridDim.x) * kRegionThreads + threadIdx.x;
}

__device__ __forceinline__ uint32_t way_of(uint64_t bkey, uint32_t i, uint64_t thr0,
                                           uint64_t thr1) {
    const uint64_t h = mix64(bkey + i) >> 32;
    return h < thr0 ? 0u : (h < thr1 ? 1u : 2u);
}

__device__ __forceinline__ const RegionSide &pick_way(uint32_t w, const RegionSide &W0,
                                                      const RegionSide &W1, const RegionSide &W2) {
    return w == 0 ? W0 : (w == 1 ? W1 : W2);
}

__global__ __launch_bounds__(kRegionThreads) void region3_divergent_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr0, uint64_t thr1, RegionSide W0, RegionSide W1,
    RegionSide W2) {
    const uint32_t i = lane_index(lane0);
    if (i >= n) return;
    const uint64_t h = mix64(bkey + i) >> 32;
    float acc = x[i];
    if (h < thr0) {
        MELD_SIDE_MARK("way 0");
        acc = side_steps(acc, i + W0.off, W0.trips, W0.a, W0.step, tab, mask);
    } else if (h < thr1) {
        MELD_SIDE_MARK("way 1");
        acc = side_steps(acc, i + W1.off, W1.trips, W1.a, W1.step, tab, mask);
    } else {
        MELD_SIDE_MARK("way 2");
        acc = side_steps(acc, i + W2.off, W2.trips, W2.a, W2.step, tab, mask);
    }
    y[i] = acc;
}

// Gathers of G steps for the lane's way, one conditional block per way.
template <int G>
__device__ __forceinline__ void gather_group_way(float (&g)[G], uint32_t way, uint32_t i0,
                                                 uint32_t i1, uint32_t i2, const RegionSide &W0,
                                                 const RegionSide &W1, const RegionSide &W2,
                                                 const float *__restrict__ tab, uint32_t mask) {
    // The end marks keep all of a way's gathers in its block: without them the
    // compiler sinks most of them past the join as gathers whose address is
    // selected per lane among the three ways (the costly mixed-stream form).
    if (way == 0) {
        MELD_SIDE_MARK("gathers way 0");
        gather_group(g, i0, W0.step, tab, mask);
        MELD_SIDE_MARK("gathers way 0 end");
    } else if (way == 1) {
        MELD_SIDE_MARK("gathers way 1");
        gather_group(g, i1, W1.step, tab, mask);
        MELD_SIDE_MARK("gathers way 1 end");
    } else {
        MELD_SIDE_MARK("gathers way 2");
        gather_group(g, i2, W2.step, tab, mask);
        MELD_SIDE_MARK("gathers way 2 end");
    }
}

// `steps` melded steps (uniform count) from the ways' current indices.
__device__ __forceinline__ float melded3_steps(float acc, uint32_t way, uint32_t i0, uint32_t i1,
                                               uint32_t i2, uint32_t steps, float a,
                                               const RegionSide &W0, const RegionSide &W1,
                                               const RegionSide &W2,
                                               const float *__restrict__ tab, uint32_t mask) {
    uint32_t k = 0;
    for (; k + kChunkMax <= steps; k += kBatch) {
        float g[kBatch];
        gather_group_way(g, way, i0, i1, i2, W0, W1, W2, tab, mask);
        acc = fma_group(acc, a, g);
        i0 += kBatch * W0.step;
        i1 += kBatch * W1.step;
        i2 += kBatch * W2.step;
    }
    const uint32_t c = steps - k;
    if (c != 0) {
        Chunk ch;
        if (way == 0) {
            MELD_SIDE_MARK("gathers way 0");
            gather_chunk(ch, c, i0, W0.step, tab, mask);
            MELD_SIDE_MARK("gathers way 0 end");
        } else if (way == 1) {
            MELD_SIDE_MARK("gathers way 1");
            gather_chunk(ch, c, i1, W1.step, tab, mask);
            MELD_SIDE_MARK("gathers way 1 end");
        } else {
            MELD_SIDE_MARK("gathers way 2");
            gather_chunk(ch, c, i2, W2.step, tab, mask);
            MELD_SIDE_MARK("gathers way 2 end");
        }
        acc = fma_chunk(acc, a, ch, c);
    }
    return acc;
}

__global__ __launch_bounds__(kRegionThreads) void region3_melded_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr0, uint64_t thr1, RegionSide W0, RegionSide W1,
    RegionSide W2) {
    const uint32_t i = lane_index(lane0);
    if (i >= n) return;
    const uint32_t way = way_of(bkey, i, thr0, thr1);
    const RegionSide &Me = pick_way(way, W0, W1, W2);
    const float a = Me.a;  // differing operand of the aligned fma: selected per lane
    const uint32_t my_trips = Me.trips;
    // stage boundaries: the ways' trip counts in ascending order (uniform)
    const uint32_t lo01 = W0.trips < W1.trips ? W0.trips : W1.trips;
    const uint32_t hi01 = W0.trips < W1.trips ? W1.trips : W0.trips;
    const uint32_t b1 = lo01 < W2.trips ? lo01 : W2.trips;
    const uint32_t b3 = hi01 > W2.trips ? hi01 : W2.trips;
    const uint32_t b2 = W0.trips + W1.trips + W2.trips - b1 - b3;
    float acc = melded3_steps(x[i], way, i + W0.off, i + W1.off, i + W2.off, b1, a, W0, W1, W2,
                              tab, mask);
    if (b2 > b1 && my_trips >= b2)  // the two longest ways
        acc = melded3_steps(acc, way, i + W0.off + b1 * W0.step, i + W1.off + b1 * W1.step,
                            i + W2.off + b1 * W2.step, b2 - b1, a, W0, W1, W2, tab, mask);
    if (b3 > b2 && my_trips >= b3)  // the longest way alone, with its own operands
        acc = side_steps(acc, i + Me.off + b2 * Me.step, b3 - b2, a, Me.step, tab, mask);
    y[i] = acc;
}

__global__ __launch_bounds__(kRegionThreads) void region3_melded_inplace_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr0, uint64_t thr1, RegionSide W0, RegionSide W1,
    RegionSide W2) {
    const uint32_t i = lane_index(lane0);
    if (i >= n) return;
    const uint32_t way = way_of(bkey, i, thr0, thr1);
    const RegionSide &Me = pick_way(way, W0, W1, W2);
    const uint32_t lo01 = W0.trips < W1.trips ? W0.trips : W1.trips;
    const uint32_t hi01 = W0.trips < W1.trips ? W1.trips : W0.trips;
    const uint32_t b1 = lo01 < W2.trips ? lo01 : W2.trips;
    const uint32_t b3 = hi01 > W2.trips ? hi01 : W2.trips;
    const uint32_t b2 = W0.trips + W1.trips + W2.trips - b1 - b3;
    // every operand selected per lane, so each stage is one aligned loop
    float acc = side_steps(x[i], i + Me.off, b1, Me.a, Me.step, tab, mask);
    if (b2 > b1 && Me.trips >= b2)
        acc = side_steps(acc, i + Me.off + b1 * Me.step, b2 - b1, Me.a, Me.step, tab, mask);
    if (b3 > b2 && Me.trips >= b3)
        acc = side_steps(acc, i + Me.off + b2 * Me.step, b3 - b2, Me.a, Me.step, tab, mask);
    y[i] = acc;
}

// Per-lane trip count of lane i for a side with range [lo, lo + span].
__device__ __forceinline__ uint32_t lane_trips(uint64_t tkey, uint32_t i, uint32_t lo,
                                               uint32_t span) {
    const uint64_t h = mix64(tkey + i) >> 32;
    return lo + (uint32_t)(h % ((uint64_t)span + 1));
}

__global__ __launch_bounds__(kRegionThreads) void region_lt_divergent_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t tkey, uint64_t thr, RegionSideRange T,
    RegionSideRange F) {
    const uint32_t i = lane_index(lane0);
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    float acc = x[i];
    if (taken) {
        MELD_SIDE_MARK("true");
        const uint32_t t = lane_trips(tkey, i, T.lo, T.span);
        acc = side_steps(acc, i + T.off, t, T.a, T.step, tab, mask);
    } else {
        MELD_SIDE_MARK("false");
        const uint32_t t = lane_trips(tkey, i, F.lo, F.span);
        acc = side_steps(acc, i + F.off, t, F.a, F.step, tab, mask);
    }
    y[i] = acc;
}

__global__ __launch_bounds__(kRegionThreads) void region_lt_melded_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t tkey, uint64_t thr, RegionSideRange T,
    RegionSideRange F) {
    const uint32_t i = lane_index(lane0);
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    const float a = taken ? T.a : F.a;
    const uint32_t t = taken ? lane_trips(tkey, i, T.lo, T.span) : lane_trips(tkey, i, F.lo, F.span);
    y[i] = melded_common_steps(x[i], taken, i + T.off, i + F.off, t, a, T.step, F.step, tab, mask);
}

__global__ __launch_bounds__(kRegionThreads) void region_lt_melded_inplace_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t tkey, uint64_t thr, RegionSideRange T,
    RegionSideRange F) {
    const uint32_t i = lane_index(lane0);
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    const RegionSideRange &S = taken ? T : F;
    const uint32_t t = lane_trips(tkey, i, S.lo, S.span);
    y[i] = side_steps(x[i], i + S.off, t, S.a, S.step, tab, mask);
}

}  // namespace

hipError_t launch_region3(const float *x, float *y, uint32_t n, const float *tab, uint32_t mask,
                          uint64_t seed, uint64_t thr0, uint64_t thr1, RegionSide W0,
                          RegionSide W1, RegionSide W2, RegionForm form, hipStream_t stream) {
    const uint64_t bkey = stream_key(seed, 4);
    auto kern = form == RegionForm::kMelded          ? region3_melded_kernel
                : form == RegionForm::kMeldedInPlace ? region3_melded_inplace_kernel
                                                     : region3_divergent_kernel;
    for (uint64_t i0 = 0; i0 < n; i0 += kRegionLaunchLanes) {
        const uint32_t len = (uint32_t)(n - i0 < kRegionLaunchLanes ? n - i0 : kRegionLaunchLanes);
        hipLaunchKernelGGL(kern, dim3(blocks_for(len, kRegionThreads)), dim3(kRegionThreads), 0,
                           stream, x, y, n, (uint32_t)i0, tab, mask, bkey, thr0, thr1, W0, W1, W2);
    }
    return hipGetLastError();
}

hipError_t launch_region_lanetrips(const float *x, float *y, uint32_t n, const float *tab,
                                   uint32_t mask, uint64_t seed, uint64_t thr, RegionSideRange T,
                                   RegionSideRange F, RegionForm form, hipStream_t stream) {
    const uint64_t bkey = stream_key(seed, 4);
    const uint64_t tkey = stream_key(seed, 11);
    auto kern = form == RegionForm::kMelded          ? region_lt_melded_kernel
                : form == RegionForm::kMeldedInPlace ? region_lt_melded_inplace_kernel
                                                     : region_lt_divergent_kernel;
    for (uint64_t i0 = 0; i0 < n; i0 += kRegionLaunchLanes) {
        const uint32_t len = (uint32_t)(n - i0 < kRegionLaunchLanes ? n - i0 : kRegionLaunchLanes);
        hipLaunchKernelGGL(kern, dim3(blocks_for(len, kRegionThreads)), dim3(kRegionThreads), 0,
                           stream, x, y, n, (uint32_t)i0, tab, mask, bkey, tkey, thr, T, F);
    }
    return hipGetLastError();
}

}  // namespace meld
