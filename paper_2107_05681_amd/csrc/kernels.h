// Internal launch interface between the C-ABI host layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace meld {

struct RegionSide {
    float a;
    uint32_t off;
    uint32_t step;
    uint32_t trips;
};

enum class RegionForm { kDivergent, kMelded, kMeldedInPlace };

hipError_t launch_region(const float *x, float *y, uint32_t n, const float *tab, uint32_t mask,
                         uint64_t seed, uint64_t thr, RegionSide T, RegionSide F, RegionForm form,
                         hipStream_t stream);

// The region's memory path alone: launch_region's lanes, branch, addresses,
// exec masks and batching with the fma replaced by an xor of the gathered
// bits (y is not the region's value). For measuring a form's ceiling.
hipError_t launch_region_gathers(const float *x, float *y, uint32_t n, const float *tab,
                                 uint32_t mask, uint64_t seed, uint64_t thr, RegionSide T,
                                 RegionSide F, RegionForm form, hipStream_t stream);

// Three-way region (region_variants.hip): way 0 below thr0, way 1 below thr1,
// way 2 otherwise (thr0 <= thr1 <= 2^32).
hipError_t launch_region3(const float *x, float *y, uint32_t n, const float *tab, uint32_t mask,
                          uint64_t seed, uint64_t thr0, uint64_t thr1, RegionSide W0,
                          RegionSide W1, RegionSide W2, RegionForm form, hipStream_t stream);

// A side whose trip count is drawn per lane in [lo, lo + span].
struct RegionSideRange {
    float a;
    uint32_t off;
    uint32_t step;
    uint32_t lo;
    uint32_t span;
};

hipError_t launch_region_lanetrips(const float *x, float *y, uint32_t n, const float *tab,
                                   uint32_t mask, uint64_t seed, uint64_t thr, RegionSideRange T,
                                   RegionSideRange F, RegionForm form, hipStream_t stream);

// Array with virtual padding: position p < n lives in keys/vals[p], position
// n <= p < N in the tail workspace tk/tv[p - n] (pre-filled with the
// sentinel); without a workspace, positions >= n read as the sentinel and
// are not written.
struct SortArray {
    uint32_t *keys;
    uint32_t *vals;  // NULL for keys-only
    uint32_t *tk;    // tail workspace for keys (may be NULL)
    uint32_t *tv;    // tail workspace for vals (may be NULL)
    uint32_t n;
    uint32_t nt;     // nonzero: global accesses carry the nontemporal hint
};

// Runs, on every tile of 2^log_t elements, the network steps of phases
// k = 2^m for m in [m_begin, m_end], starting phase m_begin at j = 2^j_first
// (later phases start at j = k/2). At most step_limit steps run (negative:
// all). Tiles: n_tiles. Threads per workgroup: 64, 256 or 512.
// io_mode: 0 plain, 1 plain with 16-byte aligned arrays (vector I/O),
// 2 tail workspace, 3 sentinel padding of a single tile.
constexpr int kIoPlain = 0, kIoPlainVec = 1, kIoTail = 2, kIoSentinel = 3;
// meld_lo / meld_hi: melded (true) or divergent compare-exchange for the
// phases k <= 64 / k >= 128.
hipError_t launch_bitonic_tile(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                               uint32_t m_begin, uint32_t m_end, uint32_t j_first,
                               int32_t step_limit, bool meld_lo, bool meld_hi, int io_mode,
                               int threads, hipStream_t stream);

// The whole network of every tile of 2^log_t elements (log_t in 8..14):
// phases k <= 64 in form meld_lo, as the LDS comparator network (xch false)
// or in registers with DPP lane exchanges (xch true); phases k >= 128 in
// register windows in form meld_hi (with lane exchanges for the steps on
// element bits 4 and 5 of a phase when xch). io_mode: plain, vector, tail or
// sentinel. At most step_limit steps run (negative: all).
hipError_t launch_bitonic_sort_regs(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                                    int32_t step_limit, bool meld_lo, bool meld_hi, bool xch,
                                    int io_mode, hipStream_t stream);
// The same on one path each (xch true and false), one translation unit each.
hipError_t launch_bitonic_sort_regs_xch(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                                        int32_t step_limit, bool meld_lo, bool meld_hi,
                                        int io_mode, hipStream_t stream);
hipError_t launch_bitonic_sort_regs_lds(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                                        int32_t step_limit, bool meld_lo, bool meld_hi,
                                        int io_mode, hipStream_t stream);

// Steps j = 2^b_hi .. 2^b_lo of phase k = 2^m over all N = 2^log_n elements
// in one pass through LDS: each workgroup gathers 2^(b_hi-b_lo+1) rows of
// contiguous elements (b_hi - b_lo + 1 in 5..8 for pairs, 7..9 for keys;
// rows of at least 32 elements). io_mode plain, vector or tail.
hipError_t launch_bitonic_gather(const SortArray &a, uint32_t log_n, uint32_t m, uint32_t b_hi,
                                 uint32_t b_lo, int32_t step_limit, int io_mode,
                                 hipStream_t stream);
constexpr uint32_t kMaxGatherStepsPairs = 8, kMaxGatherStepsKeys = 9;
constexpr uint32_t kMinGatherStepsPairs = 5;

// Steps j = 2^(log_t-1) .. 1 of phase k = 2^m > 2^log_t on every tile, in
// registers with LDS transposes (log_t in 8..14; io_mode plain, vector or
// tail). At most step_limit steps run (negative: all).
hipError_t launch_bitonic_merge(const SortArray &a, uint32_t log_t, uint32_t n_tiles, uint32_t m,
                                int32_t step_limit, int io_mode, hipStream_t stream);

// One streaming pass over all N = 2^log_n elements for the steps
// j = 2^b_hi .. 2^b_lo of phase k = 2^m (b_hi - b_lo + 1 <= kMaxFusedSteps),
// all in registers. At most step_limit steps run (negative: all).
constexpr uint32_t kMaxFusedSteps = 6;
hipError_t launch_bitonic_global(const SortArray &a, uint32_t log_n, uint32_t m, uint32_t b_hi,
                                 uint32_t b_lo, int32_t step_limit, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t count, hipStream_t stream);

// Seeded inputs generated on the device (gen.hip).
hipError_t launch_gen_keys(uint32_t *keys, uint32_t n, uint64_t seed, hipStream_t s);
hipError_t launch_gen_keys_segments(uint32_t *keys, const uint32_t *offsets,
                                    const uint64_t *seeds, uint32_t nseg, uint32_t max_len,
                                    hipStream_t s);
hipError_t launch_gen_x(float *x, uint32_t n, uint64_t seed, hipStream_t s);
hipError_t launch_gen_tab(float *tab, uint32_t m, uint64_t seed, hipStream_t s);

// Divergence probes (probe.hip). Counters are accumulated into out.
// Region: out[0] mixed waves, out[1] true lanes, out[2] waves.
hipError_t launch_probe_region(uint32_t n, uint64_t seed, uint64_t thr, unsigned long long *out,
                               hipStream_t stream);
// One tile of 2^log_t: out[2(m-1)] mixed comparator-waves of phase 2^m,
// out[2(m-1)+1] comparator-waves of that phase (over all its steps); regs:
// phases k >= 128 under the register-window mapping (2^(log_t-4) threads,
// direction = thread bit m-4).
hipError_t launch_probe_network(uint32_t log_t, bool regs, unsigned long long *out,
                                hipStream_t stream);
// Segments: out[0..1] mixed / all comparator-steps of the phases k <= 64,
// out[2..3] the same for k >= 128.
hipError_t launch_probe_segments(const uint32_t *off, uint32_t nseg, unsigned long long *out,
                                 hipStream_t stream);

// Segmented sort (segsort.hip).
constexpr uint32_t kSegThreads = 1024;
constexpr uint32_t kSegLogChunk = 14;  // 2^14 keys: 16 per lane of a workgroup
constexpr uint32_t kSegChunk = 1u << kSegLogChunk;
constexpr uint32_t kSegLdsWords = kSegChunk + kSegChunk / 16;  // padded tile, 68 KiB
constexpr uint32_t kSegWorkWords = 1u << 16;  // staging of a segment of up to 2^16 keys
constexpr uint32_t kSegMaxLen = 1u << 16;
constexpr uint32_t kSegClasses = 17;  // size class ceil(log2(len)) in 0..16
constexpr uint32_t kSegSmallClassMax = 7;  // up to 128 keys: one wave per segment
constexpr uint32_t kSegBadFirst = 1, kSegDecreasing = 2, kSegTooLong = 4, kSegBeyondEnd = 8;

// Device-side work-queue state of one segmented sort.
struct SegState {
    uint32_t cnt[kSegClasses];        // segments per size class
    uint32_t fill[kSegClasses];       // scatter cursors
    uint32_t base[kSegClasses];       // queue start of each class (largest class first)
    uint32_t item_base[kSegClasses];  // first work item of each class >= 8
    uint32_t head;                    // next work item
    uint32_t flag;                    // invalid-offset bits of this call
    uint32_t sticky;                  // invalid-offset bits since the last check
    uint32_t n_big;                   // work items of the classes >= 8
    uint32_t n_small;                 // segments of 2..128 keys (16 per item)
    uint32_t n_items;
};

// Persistent grid size: CUs x resident 1024-lane workgroups (68 KiB of LDS).
hipError_t seg_sort_grid(int device, uint32_t *grid);

// Enqueues reset, classify, plan, scatter and the persistent sort (segments
// above 128 keys: phases k <= 64 as the LDS comparator network, or with xch in
// registers with DPP lane exchanges). keys holds
// n_keys words (an offset above n_keys flags the call invalid), cls nseg
// bytes, queue nseg words, work grid * kSegWorkWords words.
hipError_t launch_segmented_sort(uint32_t *keys, uint32_t n_keys, const uint32_t *off,
                                 uint32_t nseg, SegState *st, uint8_t *cls, uint32_t *queue,
                                 uint32_t *work, uint32_t grid, bool meld_lo, bool meld_hi,
                                 bool xch, hipStream_t stream);

// Batcher's odd-even merge network on each bucket of 2^log_t keys
// (oddeven.hip; log_t in 6..14, the last bucket ragged), at most max_steps
// steps per bucket (negative: all), divergent or melded.
hipError_t launch_oddeven_buckets(uint32_t *keys, uint32_t n, uint32_t log_t, int32_t max_steps,
                                  bool melded, hipStream_t stream);

// One merge pass (mergesort.hip): the sorted runs of 2^log_run keys of src
// merged in pairs into runs of twice that length in dst (the last pair may be
// ragged); log_run >= 10. cuts: NULL, or scratch of merge_pass_cut_words(n)
// words; with it, passes of runs of at least 2^kMergeCutLog keys over more
// than kMergeCutMinTiles tiles of 2048 keys find the tiles' merge-path cuts
// in a kernel of their own first.
constexpr uint32_t kMergeCutLog = 11;
constexpr uint32_t kMergeCutMinTiles = 2048;
uint32_t merge_pass_cut_words(uint32_t n);
hipError_t launch_merge_pass(const uint32_t *src, uint32_t *dst, uint32_t n, uint32_t log_run,
                             bool melded, uint32_t *cuts, hipStream_t stream);

// Largest tile (log2 elements) the tile kernel supports for keys / pairs.
constexpr uint32_t kMaxLogTileKeys = 14;
constexpr uint32_t kMaxLogTilePairs = 13;
// Tile of the gathered streaming passes: 64 KiB of elements.
constexpr uint32_t kGatherLogKeys = 14;
constexpr uint32_t kGatherLogPairs = 13;

}  // namespace meld
