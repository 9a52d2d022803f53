// Batcher's odd-even merge sorting network on buckets of 2^L keys, the
// network of the paper's PCM benchmark (Evaluation section, "Partition and
// Concurrent Merge"): divergent and melded forms of its per-element region.
//
// Network: steps (p, k) for p = 1, 2, ..., T/2 and k = p, p/2, ..., 1; the
// comparators of a step are (a, a + k) for a = j + i with j running over
// k mod p, k mod p + 2k, ... and i over 0 .. k-1, whenever a and a + k lie in
// the same block of 2p keys; the smaller key goes to a. Per element e of a
// step that means (bit_k(e) is bit log2 k of e):
//   k = p:  lower when bit_k(e) = 0 (partner e + k), upper otherwise (e - k);
//   k < p:  lower when bit_k(e) = 1 and e mod 2p + k < 2p (partner e + k),
//           upper when bit_k(e) = 0 and e mod 2p >= k (partner e - k),
//           idle otherwise.
// Each lane holds E keys of the bucket (elements t, t + NT, ...) in
// registers; a step reads partners from the LDS copy of the bucket, then
// writes its new keys. Workgroups of 512 lanes and more keep two copies: a
// step reads one and writes the other, so one barrier per step orders both
// (every read of a step precedes its barrier, the next write to that copy
// follows it); smaller ones, whose barriers are cheap, keep one copy and
// separate the reads from the writes with a second barrier.
//
//   divergent: the element's region as written, an if / else-if on its
//     role: the lower side loads the partner above and keeps the minimum, the
//     upper side loads the partner below and keeps the maximum; an idle
//     element keeps its key. In a wave holding several roles the sides run
//     one after the other, each with its own LDS load.
//   melded: the two sides align (region-region melding) and the idle path is
//     replicated into them (region replication, partner = the element
//     itself): one LDS load from a selected address, then min, max or the
//     key itself selected by role.
#include "device_common.h"
#include "kernels.h"

namespace meld {

namespace {

constexpr uint32_t kOePad = 0xFFFFFFFFu;

// Role of element e at step (p, k): +1 lower, -1 upper, 0 idle.
__device__ __forceinline__ int oe_role(uint32_t e, uint32_t p, uint32_t k) {
    const bool bit = (e & k) != 0;
    if (k == p) return bit ? -1 : 1;
    const uint32_t pos = e & (2 * p - 1);
    if (bit) return pos + k < 2 * p ? 1 : 0;
    return pos >= k ? -1 : 0;
}

template <int E, int NT, bool MELDED>
__global__ __launch_bounds__(NT) void oddeven_bucket_kernel(uint32_t *__restrict__ keys, uint32_t n,
                                                            uint32_t log_t, int32_t max_steps) {
    extern __shared__ __align__(16) uint32_t s[];
    const uint32_t T = 1u << log_t;
    const uint32_t t = threadIdx.x;
    const uint32_t base = xcd_contiguous_block(blockIdx.x, gridDim.x) << log_t;
    uint32_t v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t q = base + t + (uint32_t)r * NT;
        v[r] = q < n ? keys[q] : kOePad;
        s[t + (uint32_t)r * NT] = v[r];
    }
    __syncthreads();
    constexpr bool kTwoCopies = NT >= 512;
    int32_t steps = 0;
    uint32_t *cur = s, *nxt = kTwoCopies ? s + T : s;
    for (uint32_t p = 1; p < T; p <<= 1) {
        for (uint32_t k = p; k >= 1; k >>= 1) {
            if (steps == max_steps) goto done;
            ++steps;
            const uint32_t *sc = cur;
            uint32_t nv[E];
            if (2 * p <= (uint32_t)NT) {
                // r * NT is a multiple of 2p: every element of the lane has the
                // role of element t, so the role, and the partner offset, are
                // computed once per step (the divergent form branches once per
                // step, each side with its own loads).
                const int role = oe_role(t, p, k);
                if constexpr (MELDED) {
                    const int32_t d = role > 0 ? (int32_t)k : (role < 0 ? -(int32_t)k : 0);
                    const uint32_t *pp = sc + ((int32_t)t + d);
#pragma unroll
                    for (int r = 0; r < E; ++r) {
                        const uint32_t b = pp[(uint32_t)r * NT];
                        const uint32_t mn = v[r] < b ? v[r] : b;
                        const uint32_t mx = v[r] < b ? b : v[r];
                        nv[r] = role > 0 ? mn : (role < 0 ? mx : v[r]);
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < E; ++r) nv[r] = v[r];
                    if (role > 0) {
                        MELD_SIDE_MARK("lower");
#pragma unroll
                        for (int r = 0; r < E; ++r) {
                            const uint32_t b = sc[t + (uint32_t)r * NT + k];
                            if (b < v[r]) nv[r] = b;
                        }
                    } else if (role < 0) {
                        MELD_SIDE_MARK("upper");
#pragma unroll
                        for (int r = 0; r < E; ++r) {
                            const uint32_t b = sc[t + (uint32_t)r * NT - k];
                            if (b > v[r]) nv[r] = b;
                        }
                    }
                }
            } else {
                // 2p > NT: element r is t + r NT with rr = r NT mod 2p a
                // multiple of NT. For k >= NT bit k of the element is a bit of
                // r and the role depends on r alone (scalar); for k < NT bit k
                // is t's and the block-edge tests compare t with scalars.
                const bool tbit = (t & k) != 0;
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const uint32_t e = t + (uint32_t)r * NT;
                    const uint32_t rr = ((uint32_t)r * NT) & (2 * p - 1);
                    int role;
                    if (k >= (uint32_t)NT) {
                        const bool rbit = (((uint32_t)r * NT) & k) != 0;
                        role = k == p ? (rbit ? -1 : 1)
                                      : (rbit ? (rr + k < 2 * p ? 1 : 0) : (rr >= k ? -1 : 0));
                    } else {
                        role = tbit ? (t + rr + k < 2 * p ? 1 : 0) : (t + rr >= k ? -1 : 0);
                    }
                    if constexpr (MELDED) {
                        const uint32_t partner = role > 0 ? e + k : (role < 0 ? e - k : e);
                        const uint32_t b = sc[partner];
                        const uint32_t mn = v[r] < b ? v[r] : b;
                        const uint32_t mx = v[r] < b ? b : v[r];
                        nv[r] = role > 0 ? mn : (role < 0 ? mx : v[r]);
                    } else {
                        nv[r] = v[r];
                        if (role > 0) {
                            MELD_SIDE_MARK("lower");
                            const uint32_t b = sc[e + k];
                            if (b < v[r]) nv[r] = b;
                        } else if (role < 0) {
                            MELD_SIDE_MARK("upper");
                            const uint32_t b = sc[e - k];
                            if (b > v[r]) nv[r] = b;
                        }
                    }
                }
            }
            if constexpr (!kTwoCopies) __syncthreads();  // every partner read before any write
#pragma unroll
            for (int r = 0; r < E; ++r) {
                v[r] = nv[r];
                nxt[t + (uint32_t)r * NT] = v[r];
            }
            __syncthreads();
            uint32_t *w = cur;
            cur = nxt;
            nxt = w;
        }
    }
done:
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t q = base + t + (uint32_t)r * NT;
        if (q < n) keys[q] = v[r];
    }
}

template <int E, int NT>
hipError_t launch_oe(uint32_t *keys, uint32_t n, uint32_t log_t, int32_t max_steps, bool melded,
                     hipStream_t stream) {
    const uint32_t buckets = (uint32_t)(((uint64_t)n + (1u << log_t) - 1) >> log_t);
    const size_t lds = ((size_t)(NT >= 512 ? 2 : 1) << log_t) * sizeof(uint32_t);
    auto kern = melded ? oddeven_bucket_kernel<E, NT, true> : oddeven_bucket_kernel<E, NT, false>;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(buckets), dim3(NT), lds, stream, keys, n, log_t, max_steps);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_oddeven_buckets(uint32_t *keys, uint32_t n, uint32_t log_t, int32_t max_steps,
                                  bool melded, hipStream_t stream) {
    if (n == 0 || max_steps == 0) return hipSuccess;
    switch (log_t) {
        case 6: return launch_oe<1, 64>(keys, n, log_t, max_steps, melded, stream);
        case 7: return launch_oe<2, 64>(keys, n, log_t, max_steps, melded, stream);
        case 8: return launch_oe<4, 64>(keys, n, log_t, max_steps, melded, stream);
        case 9: return launch_oe<8, 64>(keys, n, log_t, max_steps, melded, stream);
        case 10: return launch_oe<8, 128>(keys, n, log_t, max_steps, melded, stream);
        case 11: return launch_oe<8, 256>(keys, n, log_t, max_steps, melded, stream);
        case 12: return launch_oe<8, 512>(keys, n, log_t, max_steps, melded, stream);
        case 13: return launch_oe<8, 1024>(keys, n, log_t, max_steps, melded, stream);
        case 14: return launch_oe<16, 1024>(keys, n, log_t, max_steps, melded, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace meld
