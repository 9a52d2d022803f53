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
int oracle_segmented_sort_u32(uint32_t *keys, const uint32_t *offsets, size_t nseg);

uint64_t oracle_bitonic_num_steps(size_t n_pow2);
int oracle_bitonic_emulate(uint32_t *keys, uint32_t *vals, size_t n_pow2, int64_t max_steps);

int oracle_region_f32(const float *x, float *y, uint64_t i0, size_t n, const float *tab,
                      size_t tab_len, uint64_t seed, uint64_t thr, oracle_side side_true,
                      oracle_side side_false);

uint64_t oracle_count_true(uint64_t seed, uint64_t thr, uint64_t i0, size_t n);
uint64_t oracle_mixed_waves(uint64_t seed, uint64_t thr, size_t n, uint32_t wave);
double oracle_mixed_fraction_closed_form(double p, uint32_t wave);

#ifdef __cplusplus
}
#endif
#endif
