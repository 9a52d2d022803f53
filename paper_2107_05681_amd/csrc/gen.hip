// Seeded inputs generated on the device (serving jobs carry a seed, not
// data): the SplitMix64 counter streams of the workload definitions, written
// from the generator's published definition (Steele, Lea and Flood, OOPSLA
// 2014): value i of stream (seed, tag) is mix64(mix64(seed + tag * golden) + i).
#include "device_common.h"
#include "kernels.h"

namespace meld {

namespace {

// keys[i] = stream(seed, 1)[i] >> 32
__global__ __launch_bounds__(256) void gen_keys_kernel(uint32_t *keys, uint32_t n, uint32_t i0,
                                                       uint64_t key) {
    const uint32_t i = i0 + blockIdx.x * 256 + threadIdx.x;
    if (i < n) keys[i] = (uint32_t)(mix64(key + i) >> 32);
}

// Segment s of keys[offsets[s] .. offsets[s+1]) gets the key stream of seeds[s].
__global__ __launch_bounds__(256) void gen_keys_segments_kernel(uint32_t *keys,
                                                                const uint32_t *offsets,
                                                                const uint64_t *seeds,
                                                                uint32_t nseg) {
    const uint32_t s = blockIdx.y;
    if (s >= nseg) return;
    const uint32_t lo = offsets[s], len = offsets[s + 1] - lo;
    const uint64_t key = stream_key(seeds[s], 1);
    for (uint64_t i = blockIdx.x * 256 + threadIdx.x; i < len; i += (uint64_t)gridDim.x * 256)
        keys[lo + (uint32_t)i] = (uint32_t)(mix64(key + i) >> 32);
}

// x[i] = (stream(seed, 2)[i] >> 40) * 2^-24
__global__ __launch_bounds__(256) void gen_x_kernel(float *x, uint32_t n, uint32_t i0,
                                                    uint64_t key) {
    const uint32_t i = i0 + blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = (float)(mix64(key + i) >> 40) * 0x1p-24f;
}

// tab[m] = 0.5 + (stream(seed, 3)[m] >> 41) * 2^-24
__global__ __launch_bounds__(256) void gen_tab_kernel(float *tab, uint32_t m, uint32_t i0,
                                                      uint64_t key) {
    const uint32_t i = i0 + blockIdx.x * 256 + threadIdx.x;
    if (i < m) tab[i] = 0.5f + (float)(mix64(key + i) >> 41) * 0x1p-24f;
}

// Launches cover at most 2^31 items each (HIP caps a grid dimension at
// 2^32 - 1 work-items); i0 is the launch's first item.
constexpr uint64_t kGenLaunchItems = 1ull << 31;

template <typename Kern, typename T>
void launch_items(Kern kern, T *out, uint32_t n, uint64_t key, hipStream_t s) {
    for (uint64_t i0 = 0; i0 < n; i0 += kGenLaunchItems) {
        const uint32_t len = (uint32_t)(n - i0 < kGenLaunchItems ? n - i0 : kGenLaunchItems);
        hipLaunchKernelGGL(kern, dim3(blocks_for(len, 256)), dim3(256), 0, s, out, n,
                           (uint32_t)i0, key);
    }
}

}  // namespace

hipError_t launch_gen_keys(uint32_t *keys, uint32_t n, uint64_t seed, hipStream_t s) {
    if (n == 0) return hipSuccess;
    launch_items(gen_keys_kernel, keys, n, stream_key(seed, 1), s);
    return hipGetLastError();
}

hipError_t launch_gen_keys_segments(uint32_t *keys, const uint32_t *offsets,
                                    const uint64_t *seeds, uint32_t nseg, uint32_t max_len,
                                    hipStream_t s) {
    if (nseg == 0 || max_len == 0) return hipSuccess;
    const uint32_t bx = blocks_for(max_len, 256);
    hipLaunchKernelGGL(gen_keys_segments_kernel, dim3(bx < 64 ? bx : 64, nseg), dim3(256), 0, s,
                       keys, offsets, seeds, nseg);
    return hipGetLastError();
}

hipError_t launch_gen_x(float *x, uint32_t n, uint64_t seed, hipStream_t s) {
    if (n == 0) return hipSuccess;
    launch_items(gen_x_kernel, x, n, stream_key(seed, 2), s);
    return hipGetLastError();
}

hipError_t launch_gen_tab(float *tab, uint32_t m, uint64_t seed, hipStream_t s) {
    if (m == 0) return hipSuccess;
    launch_items(gen_tab_kernel, tab, m, stream_key(seed, 3), s);
    return hipGetLastError();
}

}  // namespace meld
