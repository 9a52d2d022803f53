/*
 * CPU oracle — TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * What each function follows:
 *  - oracle_sort_u32 / oracle_sort_pairs_u32 / oracle_segmented_sort_u32:
 *    the plain definition of an ascending sort, which the bitonic network of
 *    the paper's running example (Motivating Example section, Figure 1)
 *    reaches exactly. Pairs use the lexicographic (key, payload) order so
 *    that exactly one output is correct. Segments follow the BIT benchmark's
 *    per-bucket sort (Evaluation section, "Bitonic Sort (BIT)").
 *    oracle_sort_pairs_u32_threads computes the same order on several host
 *    threads (chunk sorts, then pairwise merges): it exists to time the
 *    oracle on all host cores.
 *  - oracle_bitonic_emulate: the Figure 1 network itself, executed one
 *    (k, j) step at a time on a power-of-two array: for each thread index
 *    t with partner p = t xor j and p > t, keep ascending order when
 *    (t & k) == 0 and descending order otherwise, using strict compares.
 *  - oracle_region_f32: the two-sided loop region evaluated lane by lane in
 *    the order its two source sides run (Detailed Design section: a
 *    divergent branch whose sides hold similar instruction sequences; the
 *    melded form must compute the same values). One fused multiply-add per
 *    step, correctly rounded (std::fma).
 *  - oracle_region3_f32: the three-way variant (Evaluation section,
 *    synthetic benchmark SB4, an if / else-if / else whose three blocks
 *    compute alike), lane by lane in the source order.
 *  - oracle_region_lanetrips_f32: the two-sided region with a trip count
 *    drawn per lane (a loop whose exit itself diverges inside a wave).
 *  - oracle_oddeven_emulate: Batcher's odd-even merge sorting network, the
 *    network of the paper's PCM benchmark (Evaluation section), written from
 *    its definition: for p = 1, 2, 4, ... and k = p, p/2, ..., 1, compare
 *    a with a + k for every a = j + i, j running over k mod p, k mod p + 2k,
 *    ... and i over 0 .. k-1, whenever a and a + k lie in the same block of
 *    2p elements.
 *  - oracle_mixed_waves: the share of 64-lane waves whose branch mask is
 *    neither all-true nor all-false (Background section: only such waves
 *    pay the IPDOM serialisation).
 *
 * Built with g++ -O2 -ffp-contract=off and without fast-math.
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// SplitMix64 output mixer, from its published definition (Steele, Lea and
// Flood, OOPSLA 2014).
uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// Branch-bit stream of the region: tag 4.
uint64_t branch_hash(uint64_t seed, uint64_t i) { return mix64(mix64(seed + 4 * kGolden) + i); }

bool branch_true(uint64_t seed, uint64_t thr, uint64_t i) { return (branch_hash(seed, i) >> 32) < thr; }

inline uint64_t composite(uint32_t k, uint32_t v) { return ((uint64_t)k << 32) | v; }

bool is_pow2(size_t n) { return n != 0 && (n & (n - 1)) == 0; }

// Batcher's odd-even merge network, step by step. Calls visit(a, a + k) for
// every comparator of the first max_steps steps (negative: all).
template <typename Visit>
void oddeven_network(size_t n, int64_t max_steps, Visit visit) {
    int64_t steps = 0;
    for (size_t p = 1; p < n; p <<= 1) {
        for (size_t k = p; k >= 1; k >>= 1) {
            if (steps == max_steps) return;
            ++steps;
            for (size_t j = k % p; j + k < n; j += 2 * k) {
                for (size_t i = 0; i < k && i + j + k < n; ++i) {
                    const size_t a = i + j, b = i + j + k;
                    if (a / (2 * p) == b / (2 * p)) visit(a, b);
                }
            }
        }
    }
}


}  // namespace

extern "C" {

uint64_t oracle_mix64(uint64_t z) { return mix64(z); }

uint64_t oracle_branch_hash(uint64_t seed, uint64_t i) { return branch_hash(seed, i); }

void oracle_sort_u32(uint32_t *keys, size_t n) { std::sort(keys, keys + n); }

void oracle_sort_pairs_u32(uint32_t *keys, uint32_t *vals, size_t n) {
    std::vector<uint64_t> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = composite(keys[i], vals[i]);
    std::sort(tmp.begin(), tmp.end());
    for (size_t i = 0; i < n; ++i) {
        keys[i] = (uint32_t)(tmp[i] >> 32);
        vals[i] = (uint32_t)tmp[i];
    }
}

int oracle_sort_pairs_u32_threads(uint32_t *keys, uint32_t *vals, size_t n, unsigned threads) {
    if (threads == 0) return -1;
    // Runs fn(0 .. parts-1), one host thread each.
    auto parallel = [](size_t parts, const auto &fn) {
        std::vector<std::thread> ts;
        for (size_t p = 0; p < parts; ++p) ts.emplace_back(fn, p);
        for (auto &t : ts) t.join();
    };
    const size_t chunks = std::max<size_t>(1, std::min<size_t>(threads, n));
    std::vector<uint64_t> a(n), b(n);
    std::vector<size_t> bounds(chunks + 1);
    for (size_t c = 0; c <= chunks; ++c) bounds[c] = n * c / chunks;
    // each chunk sorted on its own thread
    parallel(chunks, [&](size_t c) {
        for (size_t i = bounds[c]; i < bounds[c + 1]; ++i) a[i] = composite(keys[i], vals[i]);
        std::sort(a.begin() + bounds[c], a.begin() + bounds[c + 1]);
    });
    // sorted runs merged two at a time, the merges of a round in parallel
    while (bounds.size() > 2) {
        const size_t runs = bounds.size() - 1;
        std::vector<size_t> next;
        for (size_t r = 0; r < runs; r += 2) next.push_back(bounds[r]);
        next.push_back(n);
        parallel((runs + 1) / 2, [&](size_t q) {
            const size_t r = 2 * q;
            if (r + 1 < runs)
                std::merge(a.begin() + bounds[r], a.begin() + bounds[r + 1],
                           a.begin() + bounds[r + 1], a.begin() + bounds[r + 2],
                           b.begin() + bounds[r]);
            else
                std::copy(a.begin() + bounds[r], a.begin() + bounds[r + 1], b.begin() + bounds[r]);
        });
        std::swap(a, b);
        bounds.swap(next);
    }
    parallel(chunks, [&](size_t c) {
        for (size_t i = n * c / chunks; i < n * (c + 1) / chunks; ++i) {
            keys[i] = (uint32_t)(a[i] >> 32);
            vals[i] = (uint32_t)a[i];
        }
    });
    return 0;
}

int oracle_segmented_sort_u32(uint32_t *keys, const uint32_t *offsets, size_t nseg) {
    if (nseg == 0) return 0;
    if (offsets[0] != 0) return -1;
    for (size_t s = 0; s < nseg; ++s)
        if (offsets[s + 1] < offsets[s]) return -1;
    for (size_t s = 0; s < nseg; ++s) std::sort(keys + offsets[s], keys + offsets[s + 1]);
    return 0;
}

// Number of (k, j) steps of the network on n_pow2 elements: sum over phases
// k = 2, 4, ..., n of log2(k).
uint64_t oracle_bitonic_num_steps(size_t n_pow2) {
    uint64_t steps = 0;
    for (size_t k = 2; k <= n_pow2; k *= 2)
        for (size_t j = k / 2; j > 0; j /= 2) ++steps;
    return steps;
}

// Runs the first max_steps steps (all of them when max_steps < 0) of the
// Figure 1 network. vals may be NULL (keys only); with vals the compare is on
// the composite (key, payload). The array length must be a power of two;
// callers pad with 0xFFFFFFFF themselves.
int oracle_bitonic_emulate(uint32_t *keys, uint32_t *vals, size_t n_pow2, int64_t max_steps) {
    if (n_pow2 == 0) return 0;
    if (!is_pow2(n_pow2)) return -1;
    int64_t done = 0;
    for (size_t k = 2; k <= n_pow2; k *= 2) {
        for (size_t j = k / 2; j > 0; j /= 2) {
            if (max_steps >= 0 && done == max_steps) return 0;
            for (size_t tid = 0; tid < n_pow2; ++tid) {
                size_t ixj = tid ^ j;
                if (ixj <= tid) continue;
                uint64_t a = composite(keys[tid], vals ? vals[tid] : 0);
                uint64_t b = composite(keys[ixj], vals ? vals[ixj] : 0);
                bool do_swap = ((tid & k) == 0) ? (b < a) : (b > a);
                if (do_swap) {
                    std::swap(keys[tid], keys[ixj]);
                    if (vals) std::swap(vals[tid], vals[ixj]);
                }
            }
            ++done;
        }
    }
    return 0;
}

// Lanes i0 .. i0+n-1 of the two-sided loop region:
//   side  = branch bit of lane i (true when (H(seed,4,i) >> 32) < thr)
//   acc   = x[i]
//   step k = 0 .. trips-1 of that side:
//           idx = (i + off + k * step) mod 2^32, masked to the table length
//           acc = fma(acc, a, tab[idx])
//   y[i]  = acc
// x and y are indexed from 0 (they hold lanes i0 .. i0+n-1).
int oracle_region_f32(const float *x, float *y, uint64_t i0, size_t n, const float *tab,
                      size_t tab_len, uint64_t seed, uint64_t thr, oracle_side side_true,
                      oracle_side side_false) {
    if (!is_pow2(tab_len) || thr > (1ull << 32)) return -1;
    const uint32_t mask = (uint32_t)(tab_len - 1);
    for (size_t j = 0; j < n; ++j) {
        const uint64_t i = i0 + j;
        const bool taken = branch_true(seed, thr, i);
        float acc = x[j];
        if (taken) {
            for (uint32_t k = 0; k < side_true.trips; ++k) {
                uint32_t idx = ((uint32_t)i + side_true.off + k * side_true.step) & mask;
                acc = std::fma(acc, side_true.a, tab[idx]);
            }
        } else {
            for (uint32_t k = 0; k < side_false.trips; ++k) {
                uint32_t idx = ((uint32_t)i + side_false.off + k * side_false.step) & mask;
                acc = std::fma(acc, side_false.a, tab[idx]);
            }
        }
        y[j] = acc;
    }
    return 0;
}

// One side's loop, as written in the region's definition.
static float run_side(float acc, uint64_t i, float a, uint32_t off, uint32_t step,
                      uint32_t trips, const float *tab, uint32_t mask) {
    for (uint32_t k = 0; k < trips; ++k) {
        const uint32_t idx = ((uint32_t)i + off + k * step) & mask;
        acc = std::fma(acc, a, tab[idx]);
    }
    return acc;
}

// Three-way region: lane i compares h = branch_hash(seed, i) >> 32 with the
// two thresholds in the order of the if / else-if / else chain.
int oracle_region3_f32(const float *x, float *y, uint64_t i0, size_t n, const float *tab,
                       size_t tab_len, uint64_t seed, uint64_t thr0, uint64_t thr1,
                       oracle_side s0, oracle_side s1, oracle_side s2) {
    if (!is_pow2(tab_len) || thr0 > thr1 || thr1 > (1ull << 32)) return -1;
    const uint32_t mask = (uint32_t)(tab_len - 1);
    for (size_t j = 0; j < n; ++j) {
        const uint64_t i = i0 + j;
        const uint64_t h = branch_hash(seed, i) >> 32;
        float acc = x[j];
        if (h < thr0)
            acc = run_side(acc, i, s0.a, s0.off, s0.step, s0.trips, tab, mask);
        else if (h < thr1)
            acc = run_side(acc, i, s1.a, s1.off, s1.step, s1.trips, tab, mask);
        else
            acc = run_side(acc, i, s2.a, s2.off, s2.step, s2.trips, tab, mask);
        y[j] = acc;
    }
    return 0;
}

// Per-lane trip count: stream (seed, 11) of the counter generator.
uint32_t oracle_lane_trips(uint64_t seed, uint64_t i, uint32_t lo, uint32_t hi) {
    const uint64_t h = mix64(mix64(seed + 11 * kGolden) + i) >> 32;
    return lo + (uint32_t)(h % ((uint64_t)hi - lo + 1));
}

int oracle_region_lanetrips_f32(const float *x, float *y, uint64_t i0, size_t n,
                                const float *tab, size_t tab_len, uint64_t seed, uint64_t thr,
                                oracle_side_range side_true, oracle_side_range side_false) {
    if (!is_pow2(tab_len) || thr > (1ull << 32) || side_true.trips_lo > side_true.trips_hi ||
        side_false.trips_lo > side_false.trips_hi)
        return -1;
    const uint32_t mask = (uint32_t)(tab_len - 1);
    for (size_t j = 0; j < n; ++j) {
        const uint64_t i = i0 + j;
        const oracle_side_range &s = branch_true(seed, thr, i) ? side_true : side_false;
        const uint32_t t = oracle_lane_trips(seed, i, s.trips_lo, s.trips_hi);
        y[j] = run_side(x[j], i, s.a, s.off, s.step, t, tab, mask);
    }
    return 0;
}

int oracle_oddeven_emulate(uint32_t *keys, size_t n_pow2, int64_t max_steps) {
    if (!is_pow2(n_pow2)) return -1;
    oddeven_network(n_pow2, max_steps, [&](size_t a, size_t b) {
        if (keys[b] < keys[a]) std::swap(keys[a], keys[b]);
    });
    return 0;
}

uint64_t oracle_oddeven_num_comparators(size_t n_pow2) {
    uint64_t c = 0;
    if (!is_pow2(n_pow2)) return 0;
    oddeven_network(n_pow2, -1, [&](size_t, size_t) { ++c; });
    return c;
}

uint64_t oracle_count_true(uint64_t seed, uint64_t thr, uint64_t i0, size_t n) {
    uint64_t c = 0;
    for (size_t j = 0; j < n; ++j) c += branch_true(seed, thr, i0 + j) ? 1 : 0;
    return c;
}

// Waves are the lanes [w*wave, (w+1)*wave) intersected with [0, n).
uint64_t oracle_mixed_waves(uint64_t seed, uint64_t thr, size_t n, uint32_t wave) {
    uint64_t mixed = 0;
    for (size_t base = 0; base < n; base += wave) {
        size_t end = std::min(n, base + (size_t)wave);
        size_t ones = 0;
        for (size_t i = base; i < end; ++i) ones += branch_true(seed, thr, i) ? 1 : 0;
        if (ones != 0 && ones != end - base) ++mixed;
    }
    return mixed;
}

// For independent lanes with P(true) = p: 1 - p^W - (1-p)^W.
double oracle_mixed_fraction_closed_form(double p, uint32_t wave) {
    return 1.0 - std::pow(p, (double)wave) - std::pow(1.0 - p, (double)wave);
}

}  // extern "C"
