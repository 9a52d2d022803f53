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
// registers; a step with k < NT reads partners from the LDS copy of the
// bucket, then writes its new keys. A step with k >= NT finds every partner
// in the lane's own registers with a role shared by all lanes, so it runs as
// register compare-exchanges without LDS traffic (the LDS copy is refreshed
// before the next LDS step). Workgroups of 512 lanes and more keep two copies: a
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

// Partner offset of element e at step (p, k): +k at the lower end of a
// comparator, -k at the upper end, 0 when idle; and whether a lower end keeps
// the minimum (the side, meaningful when the offset is not 0). Branch-free.
struct OeRole {
    int32_t d;
    bool lower;
};
__device__ __forceinline__ OeRole oe_role(uint32_t e, uint32_t p, uint32_t k) {
    const bool bit = (e & k) != 0;
    const uint32_t pos = e & (2 * p - 1);
    const bool lower = k == p ? !bit : bit;
    const bool active = k == p || (bit ? pos + k < 2 * p : pos >= k);
    const int32_t kk = (int32_t)k;
    return {active ? (lower ? kk : -kk) : 0, lower};
}

// The melded update of an element with key v and partner key b: the lower end
// keeps the minimum, the upper end the maximum. The partner is taken when
// (b < v) equals the side, one compare, one mask operation on the scalar unit
// and one select (ties: b equals v, either is right; an idle element reads
// itself).
__device__ __forceinline__ uint32_t oe_keep_side(uint32_t v, uint32_t b, bool lower) {
    return (b < v) == lower ? b : v;
}

// Steps with k >= NT (so 2p > NT): element r of the lane (t + r NT) has its
// partner r +- q, q = k / NT, in the lane's own registers, and its role is
// the same for every lane: bit k of the element is bit q of r and the
// block-of-2p tests reduce to r mod Q, Q = 2p / NT. With Q and q fixed at
// compile time the step is a set of register compare-exchanges (r, r + q),
// the lower end keeping the minimum, in both forms (no lane diverges).
template <int E, int Q, int q>
__device__ __forceinline__ void oe_register_step(uint32_t (&v)[E]) {
#pragma unroll
    for (int r = 0; r + q < E; ++r) {
        const bool bit = (r & q) != 0;
        const bool lower = q == Q / 2 ? !bit : (bit && (r % Q) + q < Q);
        if (lower) {
            const uint32_t a = v[r], b = v[r + q];
            v[r] = a < b ? a : b;
            v[r + q] = a < b ? b : a;
        }
    }
}

// Steps with k < NT < 2p: element r of lane t sits at position t + (r mod Q) NT
// of its block of 2p = Q NT, and bit k is t's. Its side is the lane's (lower
// when bit k of t is set) except at the block edges: rows with r mod Q = 0
// are idle on lanes t < k of the upper side, rows with r mod Q = Q - 1 on
// lanes t + k >= NT of the lower side. With Q fixed at compile time each row
// knows its class, so the lane computes three partner offsets once per step.
//   divergent: the side branch as written (lower: load the partner above,
//     keep the minimum; upper: load the partner below, keep the maximum),
//     each side with its own LDS loads and the idle test on its edge rows;
//   melded: the sides aligned and the idle path replicated into them with
//     partner = the element itself (min and max of a key with itself are the
//     key): one LDS load per element from the row class's address, then the
//     minimum or maximum selected by side.
template <int E, int NT, int Q, bool MELDED>
__device__ __forceinline__ void oe_edge_step(const uint32_t (&v)[E], uint32_t (&nv)[E],
                                             const uint32_t *sc, uint32_t t, uint32_t k) {
    const bool lower = (t & k) != 0;
    if constexpr (MELDED) {
        const int32_t kk = (int32_t)k;
        const int32_t d_mid = lower ? kk : -kk;
        const int32_t d_first = lower ? kk : (t < k ? 0 : -kk);
        const int32_t d_last = lower ? (t + k >= (uint32_t)NT ? 0 : kk) : -kk;
        const uint32_t *p_mid = sc + ((int32_t)t + d_mid);
        const uint32_t *p_first = sc + ((int32_t)t + d_first);
        const uint32_t *p_last = sc + ((int32_t)t + d_last);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t *pp = r % Q == 0 ? p_first : (r % Q == Q - 1 ? p_last : p_mid);
            const uint32_t b = pp[(uint32_t)r * NT];
            nv[r] = oe_keep_side(v[r], b, lower);
        }
    } else {
#pragma unroll
        for (int r = 0; r < E; ++r) nv[r] = v[r];
        if (lower) {
            MELD_SIDE_MARK("lower");
            const bool edge_idle = t + k >= (uint32_t)NT;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                if (r % Q == Q - 1 && edge_idle) continue;
                const uint32_t b = sc[t + (uint32_t)r * NT + k];
                if (b < v[r]) nv[r] = b;
            }
        } else {
            MELD_SIDE_MARK("upper");
            const bool edge_idle = t < k;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                if (r % Q == 0 && edge_idle) continue;
                const uint32_t b = sc[t + (uint32_t)r * NT - k];
                if (b > v[r]) nv[r] = b;
            }
        }
    }
}

struct OeState {
    uint32_t *cur, *nxt;  // LDS copy holding the current keys, copy written next
    int32_t steps;        // steps run so far
    bool lds_current;     // cur holds the lane's registers (register steps leave it behind)
};

// One step through LDS (k < NT). Q = 0: 2p <= NT; otherwise Q = 2p / NT.
template <int E, int NT, bool MELDED, int Q>
__device__ __forceinline__ void oe_lds_step(uint32_t (&v)[E], OeState &st, uint32_t t,
                                            uint32_t p, uint32_t k) {
    constexpr bool kTwoCopies = NT >= 512;
    if (!st.lds_current) {
        // nobody reads cur until the barrier below: every read of the last
        // LDS step preceded that step's barrier
#pragma unroll
        for (int r = 0; r < E; ++r) st.cur[t + (uint32_t)r * NT] = v[r];
        __syncthreads();
        st.lds_current = true;
    }
    const uint32_t *sc = st.cur;
    uint32_t nv[E];
    if constexpr (Q == 0) {
        // r * NT is a multiple of 2p: every element of the lane has the role
        // of element t, so the role, and the partner offset, are computed once
        // per step (the divergent form branches once per step, each side with
        // its own loads).
        const OeRole role = oe_role(t, p, k);
        if constexpr (MELDED) {
            // idle: partner = the element itself, whose min and max are the key
            const uint32_t *pp = sc + ((int32_t)t + role.d);
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const uint32_t b = pp[(uint32_t)r * NT];
                nv[r] = oe_keep_side(v[r], b, role.lower);
            }
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) nv[r] = v[r];
            if (role.d > 0) {
                MELD_SIDE_MARK("lower");
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const uint32_t b = sc[t + (uint32_t)r * NT + k];
                    if (b < v[r]) nv[r] = b;
                }
            } else if (role.d < 0) {
                MELD_SIDE_MARK("upper");
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const uint32_t b = sc[t + (uint32_t)r * NT - k];
                    if (b > v[r]) nv[r] = b;
                }
            }
        }
    } else {
        oe_edge_step<E, NT, Q, MELDED>(v, nv, sc, t, k);
    }
    if constexpr (!kTwoCopies) __syncthreads();  // every partner read before any write
#pragma unroll
    for (int r = 0; r < E; ++r) {
        v[r] = nv[r];
        st.nxt[t + (uint32_t)r * NT] = v[r];
    }
    __syncthreads();
    uint32_t *w = st.cur;
    st.cur = st.nxt;
    st.nxt = w;
}

// Register steps k = q NT for q = Q/2 .. 1 of phase p = Q NT / 2; false once
// max_steps steps have run.
template <int E, int Q, int q>
__device__ __forceinline__ bool oe_register_steps(uint32_t (&v)[E], OeState &st,
                                                  int32_t max_steps) {
    if (st.steps == max_steps) return false;
    ++st.steps;
    oe_register_step<E, Q, q>(v);
    st.lds_current = false;
    if constexpr (q > 1) return oe_register_steps<E, Q, q / 2>(v, st, max_steps);
    return true;
}

// Phases p = Q NT / 2 for Q = Q0, 2 Q0, ..., E (2p > NT): the register steps
// k >= NT, then the steps k = NT/2 .. 1 through LDS; false once max_steps
// steps have run.
template <int E, int NT, bool MELDED, int Q>
__device__ __forceinline__ bool oe_high_phases(uint32_t (&v)[E], OeState &st, uint32_t t,
                                               int32_t max_steps) {
    if constexpr (Q <= E) {
        constexpr uint32_t p = (uint32_t)Q * NT / 2;
        if (!oe_register_steps<E, Q, Q / 2>(v, st, max_steps)) return false;
        for (uint32_t k = NT / 2; k >= 1; k >>= 1) {
            if (st.steps == max_steps) return false;
            ++st.steps;
            oe_lds_step<E, NT, MELDED, Q>(v, st, t, p, k);
        }
        return oe_high_phases<E, NT, MELDED, 2 * Q>(v, st, t, max_steps);
    }
    return true;
}

// Buckets of T = E NT keys (log_t = log2 T).
template <int E, int NT, bool MELDED>
__global__ __launch_bounds__(NT) void oddeven_bucket_kernel(uint32_t *__restrict__ keys, uint32_t n,
                                                            uint32_t log_t, int32_t max_steps) {
    extern __shared__ __align__(16) uint32_t s[];
    constexpr uint32_t T = (uint32_t)E * NT;
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
    OeState st{s, NT >= 512 ? s + T : s, 0, true};
    for (uint32_t p = 1; p < T && 2 * p <= (uint32_t)NT; p <<= 1) {
        for (uint32_t k = p; k >= 1; k >>= 1) {
            if (st.steps == max_steps) goto done;
            ++st.steps;
            oe_lds_step<E, NT, MELDED, 0>(v, st, t, p, k);
        }
    }
    if constexpr (E >= 2) {
        if (!oe_high_phases<E, NT, MELDED, 2>(v, st, t, max_steps)) goto done;
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
    if ((1u << log_t) != (uint32_t)E * NT) return hipErrorInvalidValue;  // bucket = E NT keys
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
