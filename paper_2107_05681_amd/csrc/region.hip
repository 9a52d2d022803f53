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
//
// Each kernel also exists with ONLY_GATHERS set: the same lanes, branch,
// addresses, exec masks and batching, with the fma replaced by an xor of the
// gathered bits. It measures what the form's memory path alone costs (the
// ceiling the fma chain runs under); its y is not the region's value.
#include "device_common.h"
#include "kernels.h"
#include "region_steps.h"

namespace meld {

namespace {

template <bool ONLY_GATHERS>
__global__ __launch_bounds__(kRegionThreads) void region_divergent_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr, RegionSide T, RegionSide F) {
    const uint32_t i =
        lane0 + xcd_contiguous_block(blockIdx.x, gridDim.x) * kRegionThreads + threadIdx.x;
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    float acc = x[i];
    if (taken) {
        MELD_SIDE_MARK("true");
        acc = side_steps<ONLY_GATHERS>(acc, i + T.off, T.trips, T.a, T.step, tab, mask);
    } else {
        MELD_SIDE_MARK("false");
        acc = side_steps<ONLY_GATHERS>(acc, i + F.off, F.trips, F.a, F.step, tab, mask);
    }
    y[i] = acc;
}

// Steps only the longer side has: unaligned, run by that side's lanes with
// that side's own operands.
template <bool ONLY_GATHERS>
__device__ __forceinline__ float longer_side_steps(float acc, uint32_t i, bool taken,
                                                   const float *__restrict__ tab, uint32_t mask,
                                                   const RegionSide &T, const RegionSide &F,
                                                   uint32_t common) {
    const bool true_longer = T.trips > F.trips;
    const uint32_t extra = true_longer ? T.trips - common : F.trips - common;
    if (extra != 0 && taken == true_longer) {
        const RegionSide L = true_longer ? T : F;
        acc = side_steps<ONLY_GATHERS>(acc, i + L.off + common * L.step, extra, L.a, L.step, tab,
                                       mask);
    }
    return acc;
}

// The melded form used by the library.
template <bool ONLY_GATHERS>
__global__ __launch_bounds__(kRegionThreads) void region_melded_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr, RegionSide T, RegionSide F) {
    const uint32_t i =
        lane0 + xcd_contiguous_block(blockIdx.x, gridDim.x) * kRegionThreads + threadIdx.x;
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    const float a = taken ? T.a : F.a;  // differing operand of the aligned fma: a select
    const uint32_t common = T.trips < F.trips ? T.trips : F.trips;
    float acc = x[i];
    acc = melded_common_steps<ONLY_GATHERS>(acc, taken, i + T.off, i + F.off, common, a, T.step,
                                            F.step, tab, mask);
    y[i] = longer_side_steps<ONLY_GATHERS>(acc, i, taken, tab, mask, T, F, common);
}

// The melded form with the gathers aligned as well: one gather instruction per
// step serves both sides, its address selected per lane. This is the melded
// code as the transformation emits it when it pairs the two loads; on gfx950
// a gather whose lanes mix two address streams costs several times the
// vector-memory work of one lane-linear stream, which makes this form slower
// than the divergent one whenever the sides read different data.
template <bool ONLY_GATHERS>
__global__ __launch_bounds__(kRegionThreads) void region_melded_inplace_kernel(
    const float *__restrict__ x, float *__restrict__ y, uint32_t n, uint32_t lane0,
    const float *__restrict__ tab,
    uint32_t mask, uint64_t bkey, uint64_t thr, RegionSide T, RegionSide F) {
    const uint32_t i =
        lane0 + xcd_contiguous_block(blockIdx.x, gridDim.x) * kRegionThreads + threadIdx.x;
    if (i >= n) return;
    const bool taken = branch_taken(bkey, i, thr);
    const float a = taken ? T.a : F.a;
    const uint32_t off = taken ? T.off : F.off;
    const uint32_t step = taken ? T.step : F.step;
    const uint32_t common = T.trips < F.trips ? T.trips : F.trips;
    float acc = side_steps<ONLY_GATHERS>(x[i], i + off, common, a, step, tab, mask);
    y[i] = longer_side_steps<ONLY_GATHERS>(acc, i, taken, tab, mask, T, F, common);
}

template <bool ONLY_GATHERS>
hipError_t launch_region_t(const float *x, float *y, uint32_t n, const float *tab, uint32_t mask,
                           uint64_t seed, uint64_t thr, RegionSide T, RegionSide F,
                           RegionForm form, hipStream_t stream) {
    const uint64_t bkey = stream_key(seed, 4);
    auto kern = form == RegionForm::kMelded          ? region_melded_kernel<ONLY_GATHERS>
                : form == RegionForm::kMeldedInPlace ? region_melded_inplace_kernel<ONLY_GATHERS>
                                                     : region_divergent_kernel<ONLY_GATHERS>;
    for (uint64_t i0 = 0; i0 < n; i0 += kRegionLaunchLanes) {
        const uint32_t len = (uint32_t)(n - i0 < kRegionLaunchLanes ? n - i0 : kRegionLaunchLanes);
        hipLaunchKernelGGL(kern, dim3(blocks_for(len, kRegionThreads)), dim3(kRegionThreads), 0,
                           stream, x, y, n, (uint32_t)i0, tab, mask, bkey, thr, T, F);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_region(const float *x, float *y, uint32_t n, const float *tab, uint32_t mask,
                         uint64_t seed, uint64_t thr, RegionSide T, RegionSide F, RegionForm form,
                         hipStream_t stream) {
    return launch_region_t<false>(x, y, n, tab, mask, seed, thr, T, F, form, stream);
}

hipError_t launch_region_gathers(const float *x, float *y, uint32_t n, const float *tab,
                                 uint32_t mask, uint64_t seed, uint64_t thr, RegionSide T,
                                 RegionSide F, RegionForm form, hipStream_t stream) {
    return launch_region_t<true>(x, y, n, tab, mask, seed, thr, T, F, form, stream);
}

}  // namespace meld
