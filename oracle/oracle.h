/*
 * CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct host implementations of what the melded
 * kernel library computes. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The GPU library never
 * links it, and the two share no source, header or helper.
 *
 * All pointers are host pointers owned by the caller. Functions that can
 * reject their arguments return 0 on success and a negative value on error.
 */
#ifndef MELD_ORACLE_H
#define MELD_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One side of the two-sided loop region: multiplier, table offset, index
 * stride and trip count. */
typedef struct {
    float a;
    uint32_t off;
    uint32_t step;
    uint32_t trips;
} oracle_side;

uint64_t oracle_mix64(uint64_t z);
uint64_t oracle_branch_hash(uint64_t seed, uint64_t i);

void oracle_sort_u32(uint32_t *keys, size_t n);
void oracle_sort_pairs_u32(uint32_t *keys, uint32_t *vals, size_t n);
/* oracle_sort_pairs_u32's result on `threads` host threads: contiguous chunks
 * sorted one per thread, then merged two at a time. -1 for threads == 0. */
int oracle_sort_pairs_u32_threads(uint32_t *keys, uint32_t *vals, size_t n, unsigned threads);
int oracle_segmented_sort_u32(uint32_t *keys, const uint32_t *offsets, size_t nseg);

uint64_t oracle_bitonic_num_steps(size_t n_pow2);
int oracle_bitonic_emulate(uint32_t *keys, uint32_t *vals, size_t n_pow2, int64_t max_steps);

int oracle_region_f32(const float *x, float *y, uint64_t i0, size_t n, const float *tab,
                      size_t tab_len, uint64_t seed, uint64_t thr, oracle_side side_true,
                      oracle_side side_false);

/* Three-way region (Evaluation section, synthetic benchmark SB4: an
 * if / else-if / else whose three blocks compute alike on different data).
 * Lane i takes side 0 when (branch_hash >> 32) < thr0, side 1 when it is
 * below thr1, side 2 otherwise (thr0 <= thr1 <= 2^32), then runs that side's
 * loop as oracle_region_f32 does. */
int oracle_region3_f32(const float *x, float *y, uint64_t i0, size_t n, const float *tab,
                       size_t tab_len, uint64_t seed, uint64_t thr0, uint64_t thr1,
                       oracle_side s0, oracle_side s1, oracle_side s2);

/* A side whose trip count varies per lane within [trips_lo, trips_hi]. */
typedef struct {
    float a;
    uint32_t off;
    uint32_t step;
    uint32_t trips_lo;
    uint32_t trips_hi;
} oracle_side_range;

/* Trip count of lane i for a side with range [lo, hi]:
 * lo + ((H(seed, 11, i) >> 32) mod (hi - lo + 1)). */
uint32_t oracle_lane_trips(uint64_t seed, uint64_t i, uint32_t lo, uint32_t hi);

/* Two-sided loop region whose loops run a per-lane trip count
 * (oracle_lane_trips with the lane's side range); otherwise as
 * oracle_region_f32. */
int oracle_region_lanetrips_f32(const float *x, float *y, uint64_t i0, size_t n,
                                const float *tab, size_t tab_len, uint64_t seed, uint64_t thr,
                                oracle_side_range side_true, oracle_side_range side_false);

/* Batcher's odd-even merge sorting network on a power-of-two array (the
 * network behind the paper's PCM benchmark, Evaluation section), its first
 * max_steps steps (negative: all). A step is one (p, k) pair: p = 1, 2, 4, ...
 * < n, then k = p, p/2, ..., 1; each comparator (a, a + k) of the step keeps
 * the smaller key at a. Returns -1 if n is not a power of two. */
int oracle_oddeven_emulate(uint32_t *keys, size_t n_pow2, int64_t max_steps);
/* Comparators of the whole network on n = 2^t elements. */
uint64_t oracle_oddeven_num_comparators(size_t n_pow2);

uint64_t oracle_count_true(uint64_t seed, uint64_t thr, uint64_t i0, size_t n);
uint64_t oracle_mixed_waves(uint64_t seed, uint64_t thr, size_t n, uint32_t wave);
double oracle_mixed_fraction_closed_form(double p, uint32_t wave);

#ifdef __cplusplus
}
#endif
#endif
