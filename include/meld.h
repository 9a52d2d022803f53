/*
 * meld — hand-melded SIMT kernels for MI355X (gfx950), C ABI.
 *
 * Every compute entry point exists in two forms selected by meld_variant:
 *   MELD_DIVERGENT  the divergent if/else region runs as written: the two
 *                   sides execute one after the other under exec masks and
 *                   the wave reconverges at the immediate post-dominator
 *                   (Background section, "GPGPU Architecture").
 *   MELD_MELDED     the two sides are melded as the paper's subgraph melding
 *                   does (Detailed Design section, "DARM Code Generation",
 *                   Algorithm 2): aligned instructions run once on the whole
 *                   wave, operands that differ are chosen by a select on the
 *                   branch condition, memory operations with identical
 *                   operands become one access, and only unaligned work stays
 *                   under a branch (the "Unpredication" subsection).
 *   MELD_AUTO       the library picks per stage (measured divergence and the
 *                   tuned plan).
 *   MELD_MELDED_INPLACE  for the region: the melded form with the two sides'
 *                   gathers aligned too (one gather instruction per step,
 *                   address selected per lane). MELD_MELDED leaves those
 *                   gathers unaligned (one conditional block per side and
 *                   batch), which is faster on gfx950 when the sides read
 *                   different addresses. For the sorts it is MELD_MELDED.
 * Both forms return bit-identical results.
 *
 * Conventions for every call below:
 *   - Array arguments are DEVICE pointers on the context's device, owned by
 *     the caller; the library never frees or keeps them.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Calls are
 *     asynchronous on it; results are ready once the stream has reached the
 *     call. Kernel faults surface at the caller's next synchronisation.
 *     Exception: a call that needs more context scratch than the context
 *     holds (the first non-power-of-two sort at a larger padding, a
 *     segmented sort over more segments than before, the first MELD_AUTO
 *     trials of a shape) waits for the device (hipDeviceSynchronize) before it
 *     frees the smaller buffer and allocates the larger one; later calls of
 *     that size or less are asynchronous. meld_sort_u32_noalloc never
 *     allocates or waits.
 *   - Argument errors are detected before anything is enqueued and return
 *     MELD_EINVAL with a message in meld_last_error(); the arrays are then
 *     untouched. A failed launch returns MELD_EHIP.
 *   - A context's scratch (sort tail, segmented-sort queues, merge and tuning
 *     buffers) is shared by every call on it. Calls on one context must not
 *     overlap from several host threads, and must all be enqueued on one
 *     stream (or on streams ordered by events): two calls on one context on
 *     streams that run concurrently race on that scratch. Use one context per
 *     stream.
 *   - The library never calls exit() or abort().
 */
#ifndef MELD_H
#define MELD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct meld_ctx meld_ctx;

typedef enum {
    MELD_OK = 0,
    MELD_EINVAL = 1,
    MELD_ENOMEM = 2,
    MELD_EHIP = 3,
    MELD_EUNSUPPORTED = 4
} meld_status;

typedef enum {
    MELD_DIVERGENT = 0,
    MELD_MELDED = 1,
    MELD_AUTO = 2,
    MELD_MELDED_INPLACE = 3
} meld_variant;

/* Library version as major*10000 + minor*100 + patch. */
int meld_version(void);

/* Creates a context on HIP device `hip_device`. The context owns the
 * library's scratch memory (tail padding for non-power-of-two sorts, work
 * queues, counters), which grows on demand and is freed by meld_destroy. */
meld_status meld_create(int hip_device, meld_ctx **out);

/* Waits for the context's pending work and frees its scratch. NULL is a no-op. */
void meld_destroy(meld_ctx *ctx);

typedef enum {
    /* 1 (default): segmented sorts replay a captured hipGraph of their five
     * launches (captured once per keys/offsets/nseg/forms, at most 8 kept);
     * 0: launch them one by one. A stream that is itself being captured
     * always gets the launches directly. */
    MELD_OPT_USE_GRAPHS = 0,
    /* log2 of the tile of meld_sort_u32 and meld_sort_u32_steps: 0 (default)
     * lets the library choose (timed under MELD_AUTO, from n otherwise);
     * 8..14 for keys, 8..13 for pairs, fixes it (a larger value applies to
     * key-only sorts and is clamped to 13 for pairs). MELD_EINVAL outside
     * {0} and 8..14. */
    MELD_OPT_SORT_LOG_TILE = 1,
    /* How the phases k <= 64 of the sorts (tile sorts of meld_sort_u32 and
     * meld_sort_u32_steps, and the segments of meld_segmented_sort_u32 above
     * 128 keys) run, on top of the form meld_variant selects:
     *   1  in registers, 16 elements per lane (element 16 t + r in register
     *      r of lane t), the steps on element bits 4 and 5 as DPP exchanges
     *      with lane t ^ 1 / t ^ 2. The exchange is taken before the
     *      direction branch in both forms (warp-level intrinsics are never
     *      melded, Detailed Design, "Computing Melding Profitability"); only
     *      the compare and select differ between them.
     *   0  as the LDS comparator network of Figure 1's mapping (one
     *      comparator per lane per step).
     *  -1  (default) the library's choice: 1 under MELD_DIVERGENT and
     *      MELD_MELDED, timed against 0 by the tuner under MELD_AUTO.
     * Both give the same network, step for step. MELD_EINVAL outside -1..1. */
    MELD_OPT_LANE_EXCHANGE = 2
} meld_option;

/* Sets a context option. MELD_EINVAL for an unknown option. */
meld_status meld_set_option(meld_ctx *ctx, meld_option option, int64_t value);

/* Message of the last failed call on this host thread ("" if none). The
 * pointer stays valid until the next library call on the same thread. */
const char *meld_last_error(void);

/* In-place ascending sort of keys[0..n) with the bitonic network of the
 * paper's running example (Motivating Example section, Figure 1): phases
 * k = 2, 4, ..., N and steps j = k/2, ..., 1 over N = the next power of two
 * >= n; element i is kept in ascending order when (i & k) == 0 and in
 * descending order otherwise, with strict compares. Positions n..N-1 hold
 * the value 0xFFFFFFFF (for pairs (0xFFFFFFFF, 0xFFFFFFFF)) in library
 * scratch; nothing past n is read or written in the caller's arrays.
 *
 * keys:    device u32[n], sorted in place (unsigned order).
 * payload: NULL, or device u32[n] moved with its key. With a payload the
 *          order is the lexicographic (key, payload) order, so the output is
 *          unique; with payload = original index this is a stable sort.
 * n:       number of elements, n < 2^31; n <= 1 is a no-op.
 * Errors:  MELD_EINVAL for NULL/host pointers when n > 1 or n >= 2^31;
 *          MELD_ENOMEM when scratch for a non-power-of-two n cannot be
 *          allocated.
 */
meld_status meld_sort_u32(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                          meld_variant variant, void *stream);

/* Words of the device scratch behind meld_sort_u32_noalloc: 2^22 (16 MiB). */
#define MELD_NOALLOC_SCRATCH_WORDS (1u << 22)

/* meld_sort_u32 for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It allocates nothing (no hipMalloc, hipFree or allocating library call):
 * the padding of a non-power-of-two n lives in a device array of the library
 * (MELD_NOALLOC_SCRATCH_WORDS u32, one copy per device, held until the
 * process ends, its address looked up by meld_create), filled with the
 * sentinel by a kernel on every call. The same network, forms and result as
 * meld_sort_u32; MELD_AUTO takes the tuner's decision for the shape if it
 * holds one and the melded default otherwise (it never times trials).
 * The array is shared by every call on the device, whatever the context:
 * calls that overlap on one GPU (other host threads, or streams that run
 * concurrently) race on it and must be ordered by the caller.
 * Arguments and errors: as meld_sort_u32, plus MELD_EINVAL when the padding
 * (N - n words for keys, 2 (N - n) for pairs, N the next power of two >= n)
 * exceeds MELD_NOALLOC_SCRATCH_WORDS and n is above one tile (every n up to
 * 2^22 keys or 2^21 pairs fits, as does every power of two). */
meld_status meld_sort_u32_noalloc(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                                  meld_variant variant, void *stream);

/* meld_sort_u32 with the duration of every launch: a HIP event is recorded
 * on `stream` before the first launch and after each one, the call waits for
 * the last, and launch_ms[i] receives the time between events i and i+1 in
 * milliseconds (launch i of the plan meld_sort_plan_describe lists; for a
 * non-power-of-two n the first also holds the fill of the padding). Used to
 * measure each kernel against its roofline. Synchronous.
 * launch_ms: host float[cap]; *n_launches receives the number of launches
 * (0 for n <= 1).
 * Errors: as meld_sort_u32, plus MELD_EINVAL for NULL launch_ms or
 * n_launches and for cap below the number of launches. */
meld_status meld_sort_u32_timed(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                                meld_variant variant, void *stream, float *launch_ms,
                                size_t cap, size_t *n_launches);

/* Runs only the first max_steps (k, j) steps of the same network (all of
 * them when max_steps < 0), in the same order, for stage-by-stage checks and
 * tracing. n must be a power of two in [2, 2^30]; nothing is padded.
 * Errors: as meld_sort_u32, plus MELD_EINVAL when n is not a power of two. */
meld_status meld_sort_u32_steps(meld_ctx *ctx, uint32_t *keys, uint32_t *payload, size_t n,
                                int64_t max_steps, meld_variant variant, void *stream);

/* The launches meld_sort_u32 would enqueue for n elements (the network of
 * the Motivating Example section, Figure 1, split into on-chip and HBM
 * passes), as JSON in buf (NUL-terminated), without launching anything:
 *   {"n", "log_n", "pairs", "tuned", "log_tile", "low", "high",
 *    "hbm_passes", "steps", "passes": [{"kind", "steps", "m", "b_hi", "b_lo"}]}
 * kind "tile" (everything in one tile), "local" (every tile's phases up to
 * the tile), "regs" / "gather" (steps j = 2^b_hi .. 2^b_lo of phase 2^m
 * streamed through HBM in registers / a gathered LDS tile), "merge" (the
 * steps below the tile of phase 2^m). Every pass reads and writes the whole
 * array once, so hbm_passes is the number of HBM round trips; steps totals
 * log_n (log_n + 1) / 2. "tuned" is true when MELD_AUTO found a decision of
 * the tuner (without timing anything here); an untuned MELD_AUTO describes
 * the melded default. with_payload: nonzero for (key, payload) pairs.
 * n <= 1 gives an empty pass list. Host-only: touches no device memory.
 * ctx may be NULL: the default tile rule, no tuner (a context adds its
 * MELD_OPT_SORT_LOG_TILE and, for MELD_AUTO, its tuned decisions).
 * Errors: MELD_EINVAL for NULL buf, n >= 2^31, a bad variant, or len too
 * small (the message gives the size needed). */
meld_status meld_sort_plan_describe(meld_ctx *ctx, size_t n, int with_payload,
                                    meld_variant variant, char *buf, size_t len);

/* Sorts each segment keys[offsets[s] .. offsets[s+1]) ascending in place;
 * no key crosses a segment boundary. This is the per-bucket sort of the
 * paper's bitonic benchmark (Evaluation section, "Bitonic Sort (BIT)": each
 * thread block sorts one bucket), batched over many uneven buckets.
 *
 * keys:    device u32[n_keys]; the segments cover keys[0 .. offsets[nseg]).
 * n_keys:  length of the keys array; every offset must be <= n_keys.
 * offsets: device u32[nseg + 1], offsets[0] = 0, non-decreasing. Segments
 *          may be empty. Segment length <= 65536.
 * nseg:    number of segments, < 2^31; 0 is a no-op.
 * Runs as one persistent launch after three small planning kernels that
 * build a largest-first work queue on the device; nothing is read back to
 * the host. Scratch: 5 bytes per segment plus 256 KiB per resident
 * workgroup (one per CU) for staging segments of more than 2^14 keys, owned
 * by the context.
 * Errors:  MELD_EINVAL for NULL/host pointers. Offsets live on the device
 *          and are not inspected on the host: a segment longer than 65536,
 *          decreasing offsets, offsets[0] != 0 or an offset above n_keys
 *          leave the keys untouched and set the context's device error flag,
 *          read by meld_segmented_sort_check(). MELD_AUTO reads offsets[nseg]
 *          to size its trials and returns MELD_EINVAL at once if it exceeds
 *          n_keys.
 */
meld_status meld_segmented_sort_u32(meld_ctx *ctx, uint32_t *keys, size_t n_keys,
                                    const uint32_t *offsets, size_t nseg, meld_variant variant,
                                    void *stream);

/* Sorts each bucket keys[b 2^log_bucket .. min(n, (b+1) 2^log_bucket))
 * ascending in place with Batcher's odd-even merge network (the network of
 * the paper's PCM benchmark, Evaluation section, "Partition and Concurrent
 * Merge"), running at most max_steps of its log_bucket (log_bucket + 1) / 2
 * steps per bucket (negative: all). Per element and step the network has a
 * three-way region (lower end of a comparator, upper end, idle): the
 * divergent form runs it as an if / else-if with one LDS load per side, the
 * melded form replicates the idle path into the two aligned sides and runs
 * one load from a selected address. MELD_AUTO times both forms once per shape
 * class on a scratch copy.
 *
 * keys:       device u32[n], n < 2^31; the last bucket may be ragged (its
 *             missing positions act as 0xFFFFFFFF and are never written).
 * log_bucket: 6..14.
 * Errors:     MELD_EINVAL for NULL/host pointers, log_bucket outside 6..14,
 *             n >= 2^31. */
meld_status meld_oddeven_sort_buckets_u32(meld_ctx *ctx, uint32_t *keys, size_t n,
                                          uint32_t log_bucket, int64_t max_steps,
                                          meld_variant variant, void *stream);

/* Ascending bottom-up merge sort of keys[0..n) in place (the paper's MS
 * benchmark, Evaluation section, "Mergesort"): runs of 1024 keys sorted by
 * the odd-even network, then merge passes that double the run length, at
 * most max_passes of them (negative: all). A pass merges along the merge path
 * (Green, McColl and Bader, ICS 2012); per output each lane takes the head of
 * run A or of run B, a data-dependent branch: the divergent form runs its two
 * sides (emit, advance, load the next key of that run) as written, the melded
 * form selects the emitted key and issues one load from a selected address.
 * Ties take run A first. MELD_AUTO times both forms once per shape class.
 *
 * keys:    device u32[n], n < 2^31.
 * Scratch: a second buffer of n keys, owned by the context.
 * Errors:  MELD_EINVAL for NULL/host pointers or n >= 2^31. */
meld_status meld_merge_sort_u32(meld_ctx *ctx, uint32_t *keys, size_t n, int64_t max_passes,
                                meld_variant variant, void *stream);

/* As meld_segmented_sort_u32, with the form chosen per stage: low_phases for
 * the phases k <= 64, run one comparator per lane in LDS, whose direction
 * bit is one of the lane bits (the direction branch is divergent inside a
 * wave); high_phases for the phases k >= 128, run 16 keys per lane in
 * registers, whose direction is a lane bit for k <= 512 and uniform per wave
 * above. Used by the tuner and for per-stage measurements. MELD_AUTO counts
 * as MELD_MELDED here. */
meld_status meld_segmented_sort_u32_staged(meld_ctx *ctx, uint32_t *keys, size_t n_keys,
                                           const uint32_t *offsets, size_t nseg,
                                           meld_variant low_phases, meld_variant high_phases,
                                           void *stream);

/* Synchronises `stream` and reports whether any segmented sort on the context
 * since the last check found invalid offsets (MELD_EINVAL, with the reason)
 * or not (MELD_OK). Clears the flag. */
meld_status meld_segmented_sort_check(meld_ctx *ctx, void *stream);

/* One side of the two-sided loop region: multiplier, table offset, index
 * stride and trip count. */
typedef struct {
    float a;
    uint32_t off;
    uint32_t step;
    uint32_t trips;
} meld_side;

/* The two-sided loop region, lane by lane (the paper's synthetic benchmarks:
 * a divergent region whose two sides hold the same instruction sequence on
 * different data, Evaluation section, "Synthetic Benchmarks"):
 *   taken = (mix64(mix64(seed + 4*0x9E3779B97F4A7C15) + i) >> 32) < thr
 *           (SplitMix64 output mixer, Steele, Lea and Flood, OOPSLA 2014)
 *   s     = taken ? side_true : side_false
 *   acc   = x[i]
 *   for k in 0 .. s.trips-1:
 *       idx = (uint32)(i + s.off + k*s.step) & (tab_len - 1)
 *       acc = fmaf(acc, s.a, tab[idx])      (one rounding per step)
 *   y[i]  = acc
 * The melded form runs one loop of min(trips) steps on the whole wave (the
 * fma multiplier selected per lane; each side's gathers of a batch in one
 * conditional block) and leaves the remaining steps of the longer side under
 * an exec mask.
 *
 * x, y:    device f32[n]; y may not alias x.
 * tab:     device f32[tab_len], tab_len a power of two <= 2^32.
 * thr:     threshold in [0, 2^32]; P(taken) = thr / 2^32.
 * trips:   each side's trip count <= 65536.
 * n:       lanes, n < 2^32; 0 is a no-op.
 * Errors:  MELD_EINVAL for NULL/host pointers, tab_len not a power of two,
 *          thr > 2^32, trips > 65536, n >= 2^32.
 */
meld_status meld_divergent_region_f32(meld_ctx *ctx, const float *x, float *y, size_t n,
                                      const float *tab, size_t tab_len, uint64_t seed,
                                      uint64_t thr, meld_side side_true, meld_side side_false,
                                      meld_variant variant, void *stream);

/* The memory path of meld_divergent_region_f32 alone, for measuring the
 * ceiling a form's fma chain runs under: the same lanes, branch, gather
 * addresses, exec masks and batching as that call in form `variant`, with
 * each step's fma replaced by an xor of the gathered bits:
 *   bits(y[i]) = bits(x[i]) ^ bits(tab[idx_0]) ^ ... ^ bits(tab[idx_{t-1}])
 * over the lane's side (y is not the region's value). Arguments and errors as
 * meld_divergent_region_f32. */
meld_status meld_probe_region_gathers(meld_ctx *ctx, const float *x, float *y, size_t n,
                                      const float *tab, size_t tab_len, uint64_t seed,
                                      uint64_t thr, meld_side side_true, meld_side side_false,
                                      meld_variant variant, void *stream);

/* Three-way region (the paper's synthetic benchmark SB4, Evaluation section:
 * an if / else-if / else whose three blocks compute alike on different data;
 * its melding is region replication, Detailed Design, "Basic block-Region
 * Melding"). Lane i:
 *   h   = mix64(mix64(seed + 4*0x9E3779B97F4A7C15) + i) >> 32
 *   way = h < thr0 ? way0 : (h < thr1 ? way1 : way2)
 * then the way's loop exactly as meld_divergent_region_f32 runs a side.
 * The divergent form runs the chain as written; the melded form runs one
 * loop whose first min(trips) steps are melded across the three ways, the
 * next ones across the two longest, the rest by the longest way alone
 * (multiplier selected per lane, each way's gathers in one conditional
 * block); MELD_MELDED_INPLACE aligns the gathers as well. MELD_AUTO times the
 * three forms once per shape class.
 *
 * Arguments as for meld_divergent_region_f32; thr0 <= thr1 <= 2^32.
 * Errors:  as meld_divergent_region_f32, plus MELD_EINVAL for thr0 > thr1.
 */
meld_status meld_region3_f32(meld_ctx *ctx, const float *x, float *y, size_t n,
                             const float *tab, size_t tab_len, uint64_t seed, uint64_t thr0,
                             uint64_t thr1, meld_side way0, meld_side way1, meld_side way2,
                             meld_variant variant, void *stream);

/* A side whose trip count is drawn per lane in [trips_lo, trips_hi]. */
typedef struct {
    float a;
    uint32_t off;
    uint32_t step;
    uint32_t trips_lo;
    uint32_t trips_hi;
} meld_side_range;

/* The two-sided loop region with a trip count per lane (the loop exit itself
 * diverges inside a wave): lane i on side s runs
 *   s.trips_lo + ((mix64(mix64(seed + 11*0x9E3779B97F4A7C15) + i) >> 32)
 *                 mod (s.trips_hi - s.trips_lo + 1))
 * steps, otherwise as meld_divergent_region_f32. The melded form runs one
 * loop for both sides, each lane leaving after its own count; the divergent
 * one runs each side's loop in turn. MELD_AUTO times the three forms once per
 * shape class.
 *
 * Arguments as for meld_divergent_region_f32; trips_lo <= trips_hi <= 65536.
 * Errors:  as meld_divergent_region_f32, plus MELD_EINVAL for a range with
 *          trips_lo > trips_hi.
 */
meld_status meld_region_lanetrips_f32(meld_ctx *ctx, const float *x, float *y, size_t n,
                                      const float *tab, size_t tab_len, uint64_t seed,
                                      uint64_t thr, meld_side_range side_true,
                                      meld_side_range side_false, meld_variant variant,
                                      void *stream);

/* ---- Divergence probes (synchronous: they wait for `stream`) -----------
 * Only waves whose lanes take both outcomes of a branch pay the IPDOM
 * serialisation (Background section, "GPGPU Architecture"). The probes
 * evaluate the exact predicate a kernel branches on, under that kernel's
 * lane mapping, with one ballot per 64-lane wave, and return host counts. */

/* Region branch over lanes [0, n): out[0] = waves whose mask is mixed,
 * out[1] = lanes taking the true side, out[2] = waves (64 consecutive lanes,
 * the last one ragged). Errors: MELD_EINVAL for NULL ctx/out, n >= 2^32 or
 * thr > 2^32. */
meld_status meld_probe_region(meld_ctx *ctx, size_t n, uint64_t seed, uint64_t thr,
                              uint64_t out[3], void *stream);

/* Sort network on one LDS tile of 2^log_t elements, comparators dealt to
 * lanes in waves of 64 consecutive indices: out[2(m-1)] = mixed
 * comparator-waves of phase k = 2^m summed over its steps, out[2(m-1)+1] =
 * all comparator-waves of that phase, m = 1..log_t (out holds 2*log_t
 * words). Errors: MELD_EINVAL for NULL ctx/out or log_t outside 1..16. */
meld_status meld_probe_network(meld_ctx *ctx, uint32_t log_t, uint64_t *out, void *stream);

/* Segmented sort on device offsets[nseg+1]: out[0] / out[1] = comparator-
 * steps in mixed waves / all comparator-steps of the phases k <= 64, out[2] /
 * out[3] the same for k >= 128, under the segmented kernel's mapping.
 * Invalid segments are skipped. */
meld_status meld_probe_segments(meld_ctx *ctx, const uint32_t *offsets, size_t nseg,
                                uint64_t out[4], void *stream);

/* ---- Autotuner -------------------------------------------------------------
 * MELD_AUTO resolves per shape class (sort: log2 n and pairs; segmented:
 * log2 nseg and log2 of the key count; region: log2 n, log2 tab_len, the
 * trip counts and p in tenths). The first call of a class times the
 * candidates on the caller's stream — sorts on a scratch copy of the input
 * (tile size x divergent/melded per stage), the region on the caller's own
 * arrays (its three forms) — runs the matching divergence probe, and keeps
 * the decision (see meld_tune_choose). Later calls reuse it. A stream that is
 * being captured gets the untuned default (melded) without timing. */

/* Loads decisions from the JSON file cache_path (if it exists and was
 * written on the same GPU architecture and HIP runtime) and saves every new
 * decision there. The environment variable MELD_TUNE_CACHE does the same at
 * meld_create. Errors: MELD_EINVAL for a malformed file. */
meld_status meld_tune(meld_ctx *ctx, const char *cache_path);

/* Writes the context's decisions as JSON into buf (NUL-terminated).
 * Errors: MELD_EINVAL when len is too small (the message gives the size). */
meld_status meld_plan_describe(meld_ctx *ctx, char *buf, size_t len);

/* The tuner's decision rule over n timed candidates: the fastest, unless
 * others are within `tie` (relative) of it; among those the candidate whose
 * per-stage forms agree most with the probe wins (melded for a stage whose
 * mixed-wave fraction is at least theta, divergent otherwise). Returns the
 * index, or -1 for n <= 0 or NULL arrays. Pure host function. */
int meld_tune_choose(int n, const double *ms, const int *melded_lo, const int *melded_hi,
                     double mixed_lo, double mixed_hi, double theta, double tie);

/* ---- Serving ---------------------------------------------------------------
 * A request loop for sort and region jobs of mixed sizes on one GPU. Jobs
 * are submitted at any time (non-blocking) and wait in a FIFO. A dispatcher
 * thread admits the head of the queue as soon as a slot (a stream with its
 * own library context, so concurrent jobs never share scratch) and enough of
 * the device-memory budget are free: strict FIFO, a job larger than the
 * budget is rejected at submit. Continuous batching: the small sort jobs
 * (<= 65536 keys) standing one after the other at the head of the queue are
 * packed into one segmented-sort launch; larger sorts and region jobs run one
 * per slot, and the slots overlap on the device. Inputs are generated on the
 * device from each job's seed (sort keys H(seed,1,i) >> 32; region x
 * (H(seed,2,i) >> 40) * 2^-24, over one resident table). A job's result stays
 * in the budget until meld_server_release. Every result is bit-identical to
 * the same job run alone. */

typedef struct meld_server meld_server;

typedef enum { MELD_JOB_SORT = 0, MELD_JOB_REGION = 1 } meld_job_kind;

typedef struct {
    int kind;                 /* meld_job_kind */
    size_t n;                 /* keys (sort) or lanes (region), 1 .. 2^31 - 1 */
    uint64_t seed;            /* input stream seed (and the region's branch seed) */
    uint64_t thr;             /* region: branch threshold in [0, 2^32] */
    meld_side side_true;      /* region sides */
    meld_side side_false;
    double arrival_s;         /* scheduled arrival on the server's clock (meld_server_now):
                                 a job submitted ahead waits until then; <= 0, or a time
                                 already past, queues it at once. Latency is measured
                                 from it (from the submit time when <= 0). NaN or
                                 infinite: MELD_EINVAL. */
} meld_job;

typedef struct {
    uint64_t job_id;
    meld_status status;       /* MELD_EHIP if its launch failed */
    int kind;
    size_t n;
    double arrival_s;         /* the job's arrival (its submit time if it gave none) */
    double submit_s, start_s, done_s;  /* seconds since the server was created */
    const void *result_dev;   /* device u32[n] sorted keys or f32[n] y; NULL on failure;
                                 valid until meld_server_release(job_id) */
    int batched;              /* jobs in the launch this one ran in */
} meld_completion;

typedef struct {
    uint64_t submitted, rejected, completed, failed, launches, batched_jobs;
    size_t budget_bytes, inflight_bytes, max_inflight_bytes, pending;
    int slots, max_concurrent;
} meld_server_stats;

/* Creates a server on HIP device hip_device: an arena of mem_budget_bytes for
 * job buffers, `slots` streams (1..64), the forms to run (variant), and a
 * resident region table of 2^table_log2 entries generated from table_seed.
 * Errors: MELD_EINVAL for bad arguments, MELD_ENOMEM if the arena or table
 * cannot be allocated (message in meld_server_last_error()). */
meld_status meld_server_create(int hip_device, size_t mem_budget_bytes, int slots,
                               meld_variant variant, uint64_t table_seed, uint32_t table_log2,
                               meld_server **out);

/* The same scheduler over a simulated device (host only, no GPU calls): a
 * unit finishes ns_per_item nanoseconds per key or lane after its launch;
 * jobs whose ids are listed in fail_ids complete with MELD_EHIP. For tests of
 * admission, batching, fairness and failure isolation. */
meld_status meld_server_create_simulated(size_t mem_budget_bytes, int slots, double ns_per_item,
                                         const uint64_t *fail_ids, size_t n_fail,
                                         meld_server **out);

/* Queues a job (or schedules it for its arrival_s); returns its id.
 * MELD_ENOMEM if it needs more than the whole budget (sort: 4n bytes; region:
 * 8n bytes, each rounded up to 256). */
meld_status meld_server_submit(meld_server *srv, const meld_job *job, uint64_t *job_id);

/* Moves up to cap completions into out (completion order). */
meld_status meld_server_poll(meld_server *srv, meld_completion *out, size_t cap, size_t *n_out);

/* Frees a completed job's result (its budget share returns to the pool). */
meld_status meld_server_release(meld_server *srv, uint64_t job_id);

/* Copies the first `bytes` of a completed job's result to host memory
 * (synchronous). MELD_EUNSUPPORTED on a simulated server. */
meld_status meld_server_read(meld_server *srv, uint64_t job_id, void *host_dst, size_t bytes);

/* Waits until no job is queued or running (completed results stay). */
meld_status meld_server_drain(meld_server *srv, double timeout_s);

meld_status meld_server_stats_get(meld_server *srv, meld_server_stats *out);

/* Seconds since the server was created: the clock of arrival_s, submit_s,
 * start_s and done_s. */
double meld_server_now(meld_server *srv);

/* Message of the last failed server call on this host thread. */
const char *meld_server_last_error(void);

/* Stops the dispatcher (running work is waited for) and frees everything. */
void meld_server_destroy(meld_server *srv);

#ifdef __cplusplus
}
#endif
#endif
