/*
 * Seeded synthetic input generators.
 *
 * This module produces the inputs that both the CPU oracle and the GPU
 * library consume. It contains none of the method's arithmetic (no sort, no
 * compare-exchange, no region evaluation): only counter-based random numbers
 * and the fixed recipes that turn them into keys, table entries, trip counts
 * and segment lengths.
 *
 * Generator: the SplitMix64 output mixer (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014), used in counter
 * mode:
 *     mix64(z)      = z ^= z>>30; z *= 0xBF58476D1CE4E5B9;
 *                     z ^= z>>27; z *= 0x94D049BB133111EB; z ^= z>>31
 *     H(seed,tag,i) = mix64(mix64(seed + tag * 0x9E3779B97F4A7C15) + i)
 * All arithmetic is unsigned 64-bit with wraparound. Tags name the stream:
 *     1 sort keys, 2 region inputs x, 3 region table, 4 region branch bits,
 *     5 trip counts, 6 segment lengths, 7 arrival gaps, 8 job kind, 9 job size.
 *
 * Every float produced here is an integer below 2^24 scaled by a power of two,
 * so the conversion is exact on any IEEE machine.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define GOLDEN 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

static inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
    return mix64(seed + tag * GOLDEN);
}

uint64_t gen_hash(uint64_t seed, uint64_t tag, uint64_t i) {
    return mix64(stream_key(seed, tag) + i);
}

uint64_t gen_mix64(uint64_t z) { return mix64(z); }

/* keys[j] = H(seed, 1, i0 + j) >> 32 */
void gen_keys_u32(uint64_t seed, uint64_t i0, uint32_t *out, size_t n) {
    const uint64_t k = stream_key(seed, 1);
    for (size_t j = 0; j < n; ++j) out[j] = (uint32_t)(mix64(k + i0 + j) >> 32);
}

/* out[j] = i0 + j (payload = original index) */
void gen_iota_u32(uint64_t i0, uint32_t *out, size_t n) {
    for (size_t j = 0; j < n; ++j) out[j] = (uint32_t)(i0 + j);
}

/* x[j] = (H(seed, 2, i0 + j) >> 40) * 2^-24, in [0, 1) */
void gen_x_f32(uint64_t seed, uint64_t i0, float *out, size_t n) {
    const uint64_t k = stream_key(seed, 2);
    for (size_t j = 0; j < n; ++j)
        out[j] = (float)(mix64(k + i0 + j) >> 40) * 0x1p-24f;
}

/* tab[m] = 0.5 + (H(seed, 3, m) >> 41) * 2^-24, in [0.5, 1) */
void gen_tab_f32(uint64_t seed, float *out, size_t m) {
    const uint64_t k = stream_key(seed, 3);
    for (size_t j = 0; j < m; ++j)
        out[j] = 0.5f + (float)(mix64(k + j) >> 41) * 0x1p-24f;
}

/* Trip counts of the two sides: 8 + H(seed, 5, s) % 25, s = 0 (true), 1 (false). */
void gen_trips(uint64_t seed, uint32_t *t_true, uint32_t *t_false) {
    *t_true = 8u + (uint32_t)(gen_hash(seed, 5, 0) % 25u);
    *t_false = 8u + (uint32_t)(gen_hash(seed, 5, 1) % 25u);
}

/* Trip count of way s of a multi-way region: 8 + H(seed, 5, s) % 25 (ways 0
 * and 1 are the two sides of gen_trips). */
uint32_t gen_way_trips(uint64_t seed, uint32_t s) {
    return 8u + (uint32_t)(gen_hash(seed, 5, s) % 25u);
}

/* Segment s has length clamp(floor(2^(lo + (hi - lo) * u)), 2^lo, 2^hi) with
 * u = (H(seed, 6, s) >> 11) * 2^-53 in [0, 1) (log-uniform lengths).
 * offsets has nseg + 1 entries, offsets[0] = 0. Returns the total length. */
uint64_t gen_segment_offsets(uint64_t seed, uint32_t nseg, uint32_t lo_log2, uint32_t hi_log2,
                             uint32_t *offsets) {
    const uint64_t k = stream_key(seed, 6);
    const double lo = (double)(1ull << lo_log2), hi = (double)(1ull << hi_log2);
    uint64_t acc = 0;
    offsets[0] = 0;
    for (uint32_t s = 0; s < nseg; ++s) {
        double u = (double)(mix64(k + s) >> 11) * 0x1p-53;
        double len = floor(exp2((double)lo_log2 + (double)(hi_log2 - lo_log2) * u));
        if (len < lo) len = lo;
        if (len > hi) len = hi;
        acc += (uint64_t)len;
        offsets[s + 1] = (uint32_t)acc;
    }
    return acc;
}

/* Uniform double in [0, 1) from stream `tag` at counter i. */
double gen_uniform(uint64_t seed, uint64_t tag, uint64_t i) {
    return (double)(gen_hash(seed, tag, i) >> 11) * 0x1p-53;
}
