// Shared device-side helpers of the melded kernel library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace meld {

constexpr int kWave = 64;
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// SplitMix64 output mixer (Steele, Lea and Flood, OOPSLA 2014).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// Key of stream `tag` for `seed`: counter i of that stream is mix64(key + i).
__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t tag) {
    return mix64(seed + tag * kGolden);
}

// Compiler-only fence: keeps the compiler from moving memory operations
// across it and, because the text differs per call site, from treating two
// sides of a branch as identical code (no hoisting or sinking of common
// instructions out of the sides). Emits no instruction.
#define MELD_SIDE_MARK(tag) asm volatile("; side " tag ::: "memory")

// Workgroups of `per` items that cover n items; the sum is formed in 64 bits
// so that n close to 2^32 does not wrap to an empty grid.
constexpr uint32_t blocks_for(uint32_t n, uint32_t per) {
    return (uint32_t)(((uint64_t)n + per - 1) / per);
}

// MI355X deals the workgroups of a launch to its 8 XCDs in turn (workgroup w
// runs on XCD w mod 8), and each XCD has its own L2. This renumbering gives
// every XCD one contiguous range of logical workgroups, so data that
// neighbouring workgroups share stays in one L2. A bijection on [0, nb).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_contiguous_block(uint32_t w, uint32_t nb) {
    const uint32_t q = nb / kXcds, r = nb % kXcds, x = w % kXcds;
    return x * q + (x < r ? x : r) + w / kXcds;
}

}  // namespace meld
