// Divergence probes: how many 64-lane waves see both outcomes of a branch.
//
// Only waves whose lanes disagree pay the IPDOM serialisation of a divergent
// branch (Background section, "GPGPU Architecture"), so the tuner reads the
// mixed-wave fraction of each stage before choosing a form. The probes
// evaluate exactly the predicate the kernels branch on, under the kernels'
// own lane mapping, with a ballot per wave.
#include "device_common.h"
#include "kernels.h"

namespace meld {

namespace {

// Region: waves are lanes [64w, 64w + 64) of [0, n).
// out[0] += waves whose branch mask is mixed, out[1] += lanes taking the true
// side, out[2] += waves. Each wave walks the lane range with a grid stride and
// adds its totals once (one atomic per wave and counter).
__global__ __launch_bounds__(256) void probe_region_kernel(uint32_t n, uint64_t bkey,
                                                           uint64_t thr,
                                                           unsigned long long *out) {
    unsigned long long mixed = 0, ones = 0, waves = 0;
    // 64-bit walk: with n close to 2^32 a 32-bit base would wrap below n
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < n; base += stride) {
        const uint32_t i = (uint32_t)base + __lane_id();
        const bool valid = i < n;
        const bool taken = valid && (mix64(bkey + i) >> 32) < thr;
        const uint64_t mt = __ballot(taken);
        const uint64_t mv = __ballot(valid);
        mixed += (mt != 0 && mt != mv) ? 1ull : 0ull;
        ones += (unsigned long long)__popcll(mt);
        waves += 1;
    }
    if (__lane_id() == 0 && waves != 0) {
        atomicAdd(&out[0], mixed);
        atomicAdd(&out[1], ones);
        atomicAdd(&out[2], waves);
    }
}

// Sort network on one tile of 2^log_t elements whose comparators are dealt
// to lanes in waves of 64 consecutive comparator indices (the tile kernels'
// mapping). One wave per (phase m, step j): lane l takes comparator
// c = 64 * wave + l for every comparator-wave of the step, evaluates the
// direction bit m of lo = c with a zero inserted at bit j, and counts the
// comparator-waves whose direction mask is mixed.
// With regs set, phases m >= 7 follow the register-window mapping instead:
// 2^(log_t-4) threads, thread t's direction is its bit m-4, and every step of
// the phase counts each wave of threads once.
// out[2*(m-1)] += mixed comparator-waves, out[2*(m-1)+1] += comparator-waves.
__global__ __launch_bounds__(64) void probe_network_kernel(uint32_t log_t, int regs,
                                                           unsigned long long *out) {
    const uint32_t m = blockIdx.x + 1;     // phase k = 2^m, m = 1 .. log_t
    const uint32_t jb = blockIdx.y;        // step j = 2^jb, jb < m
    if (m > log_t || jb >= m) return;
    const uint32_t j = 1u << jb;
    const uint32_t half = 1u << (log_t - 1);
    const uint32_t lane = __lane_id();
    unsigned long long mixed = 0, waves = 0;
    if (regs && m >= 7) {
        const uint32_t nt = 1u << (log_t - 4);
        for (uint32_t t0 = 0; t0 < nt; t0 += 64) {
            const uint32_t t = t0 + lane;
            const bool active = t < nt;
            const bool up = active && ((t >> (m - 4)) & 1u) == 0;
            const uint64_t mu = __ballot(up);
            const uint64_t ma = __ballot(active);
            mixed += (mu != 0 && mu != ma) ? 1 : 0;
            waves += 1;
        }
        if (lane == 0) {
            atomicAdd(&out[2 * (m - 1)], mixed);
            atomicAdd(&out[2 * (m - 1) + 1], waves);
        }
        return;
    }
    for (uint32_t c0 = 0; c0 < half; c0 += 64) {
        const uint32_t c = c0 + lane;
        const bool active = c < half;
        const uint32_t lo = ((c & ~(j - 1)) << 1) | (c & (j - 1));
        const bool up = active && ((lo >> m) & 1u) == 0;
        const uint64_t mu = __ballot(up);
        const uint64_t ma = __ballot(active);
        mixed += (mu != 0 && mu != ma) ? 1 : 0;
        waves += 1;
    }
    if (lane == 0) {
        atomicAdd(&out[2 * (m - 1)], mixed);
        atomicAdd(&out[2 * (m - 1) + 1], waves);
    }
}

// Segmented sort: per segment, the comparator-steps of each stage (phases
// k <= 64 and k >= 128) and how many of them fall in mixed waves, under the
// segmented kernel's mapping: one wave per segment of <= 128 keys (64
// consecutive comparators per wave); for a segment of class c >= 8 (chunks
// of 2^cm keys, cm = min(c, 14)) a team of nt = 2^(cm-4) lanes, which takes
// comparators t, t + nt, ... in the phases k <= 64 and holds 16 keys per lane
// (8 comparators per step, direction = lane bit p-4 in phase 2^p) in the
// register phases; the steps across chunks are wave-uniform. A team shorter
// than a wave shares it with teams of the same pattern, so its own nt lanes
// decide the wave.
// out[0] += mixed comparator-steps (low stage), out[1] += all (low stage),
// out[2], out[3]: the same for the high stage.
__global__ __launch_bounds__(64) void probe_segments_kernel(const uint32_t *__restrict__ off,
                                                            uint32_t nseg,
                                                            unsigned long long *out) {
    const uint32_t s = blockIdx.x;
    if (s >= nseg) return;
    const uint32_t lo_off = off[s], hi_off = off[s + 1];
    if (hi_off <= lo_off + 1 || hi_off - lo_off > kSegMaxLen) return;
    const uint32_t len = hi_off - lo_off;
    const uint32_t log_p = 32u - (uint32_t)__clz(len - 1);
    const uint32_t half = 1u << (log_p - 1);
    const uint32_t lane = __lane_id();
    unsigned long long acc[4] = {0, 0, 0, 0};
    const uint32_t cm = log_p < kSegLogChunk ? log_p : kSegLogChunk;
    const uint32_t nt = 1u << (cm - 4);
    const uint32_t chunks = 1u << (log_p - cm);
    for (uint32_t m = 1; m <= log_p; ++m) {
        // mixed comparators of one step of phase 2^m (whole segment)
        unsigned long long mixed_cmp = 0;
        if (log_p <= kSegSmallClassMax) {
            // The direction is bit m-1 of the comparator index in every step
            // of the phase.
            for (uint32_t w = 0; w < (half + 63) / 64; ++w) {
                const uint32_t c = w * 64 + lane;
                const bool active = c < half;
                const bool up = active && ((c >> (m - 1)) & 1u) == 0;
                const uint64_t mu = __ballot(up);
                const uint64_t ma = __ballot(active);
                if (mu != 0 && mu != ma) mixed_cmp += (unsigned long long)__popcll(ma);
            }
        } else if (m <= cm) {
            const bool low = m <= 6;
            const uint32_t waves = nt >= 64 ? nt / 64 : 1;
            const uint32_t iters = low ? (1u << (cm - 1)) / nt : 1;
            for (uint32_t w = 0; w < waves; ++w) {
                const uint32_t t = nt >= 64 ? w * 64 + lane : lane;
                const bool active = t < nt;
                for (uint32_t i = 0; i < iters; ++i) {
                    const uint32_t bit = low ? (((t + i * nt) >> (m - 1)) & 1u)
                                             : ((t >> (m - 4)) & 1u);
                    const bool up = active && bit == 0;
                    const uint64_t mu = __ballot(up);
                    const uint64_t ma = __ballot(active);
                    if (mu != 0 && mu != ma)
                        mixed_cmp += (unsigned long long)__popcll(ma) * (low ? 1u : 8u);
                }
            }
            mixed_cmp *= chunks;
        }
        const unsigned long long steps_all = (unsigned long long)m * half;
        const unsigned long long steps_mixed = (unsigned long long)m * mixed_cmp;
        const int stage = (1u << m) <= 64 ? 0 : 2;
        acc[stage] += steps_mixed;
        acc[stage + 1] += steps_all;
    }
    if (lane == 0)
        for (int q = 0; q < 4; ++q)
            if (acc[q] != 0) atomicAdd(&out[q], acc[q]);
}

}  // namespace

hipError_t launch_probe_region(uint32_t n, uint64_t seed, uint64_t thr, unsigned long long *out,
                               hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = blocks_for(n, 256);
    hipLaunchKernelGGL(probe_region_kernel, dim3(blocks < 2048 ? blocks : 2048), dim3(256), 0,
                       stream, n, stream_key(seed, 4), thr, out);
    return hipGetLastError();
}

hipError_t launch_probe_network(uint32_t log_t, bool regs, unsigned long long *out,
                                hipStream_t stream) {
    if (log_t == 0) return hipSuccess;
    hipLaunchKernelGGL(probe_network_kernel, dim3(log_t, log_t), dim3(64), 0, stream, log_t,
                       regs ? 1 : 0, out);
    return hipGetLastError();
}

hipError_t launch_probe_segments(const uint32_t *off, uint32_t nseg, unsigned long long *out,
                                 hipStream_t stream) {
    if (nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(probe_segments_kernel, dim3(nseg), dim3(64), 0, stream, off, nseg, out);
    return hipGetLastError();
}

}  // namespace meld
