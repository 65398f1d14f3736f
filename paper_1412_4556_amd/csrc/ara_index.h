// Index arithmetic of the trial passes' YET loads and of the fused table
// build's entry lists.  The kernels call these functions, and a CPU test
// (tests/index_model.cpp) runs the same functions: over every trial length
// and start, to check that each 16-byte load stays inside the YET's last
// granule and that every event is taken exactly once; over catalogue sizes,
// to check that every list entry and count lands inside its range's part of
// the table and of the block filter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ara {

// Events of a chunk: 64 lanes x 4 consecutive events.
constexpr int64_t kChunkEvents = 256;

// Position of the first chunk of a trial that starts at event b: with
// 16-byte aligned IDs, the 16-byte granule holding b.
__host__ __device__ inline int64_t chunk_start(bool aligned16, int64_t b) { return aligned16 ? (b & ~3LL) : b; }

// Highest granule a lane may load for trial [b, e): the trial's last
// granule, or the YET's last one (last_granule = (n_events - 1) & ~3) for an
// empty trial and for fixed-length passes, whose trials end on a granule.
__host__ __device__ inline int64_t load_limit(bool fixed, int64_t b, int64_t e, int64_t last_granule) {
    return (fixed || e <= b) ? last_granule : ((e - 1) & ~3LL);
}

// Granule a lane loads for its chunk position p (a multiple of 4): p itself,
// or the limit for a lane past the trial's end (a line the wave reads anyway).
__host__ __device__ inline int64_t clamped_granule(int64_t p, int64_t lim) { return p < lim ? p : lim; }

// Bit v is set iff element p + v lies in the trial [b, e).  Fixed-length
// passes: a lane's four elements are all inside or all past the trial.
__host__ __device__ inline uint32_t granule_valid(bool fixed, int64_t p, int64_t b, int64_t e) {
    if (fixed) return p < e ? 0xfu : 0u;
    const int64_t lo64 = b - p, hi64 = e - p;
    const int lo = lo64 < 0 ? 0 : (int)(lo64 > 4 ? 4 : lo64);
    const int hi = hi64 < 0 ? 0 : (int)(hi64 > 4 ? 4 : hi64);
    uint32_t m = 0;
    for (int v = 0; v < 4; ++v) m |= (((v >= lo) & (v < hi)) ? 1u : 0u) << v;
    return m;
}

// ---- fused table build (k_build_lists, k_fused_build)
// The catalogue events [0, catalog] (catalog: the zero slot) fall into
// ranges of kBuildRange events; work-group g of the table kernel owns range
// g.  Range g's entry list is kept in range g's part of the table, its count
// in range g's first block-filter word (a filter word covers 2^(fshift + 5)
// events, and a range whole words).
constexpr int kBuildRangeShift = 13;
constexpr int kBuildRange = 1 << kBuildRangeShift;
constexpr int kBuildThreads = 1024;
// Entries of a range the build lists before adding them (a range with more
// reads every ID of the layer instead, taking the ELTs one at a time); a
// multiple of kBuildThreads.
constexpr int kBuildList = 4 * kBuildThreads;
// Ranges up to which the listing kernel counts a work-group's entries per
// range in LDS before reserving their places (beyond: one atomic per entry).
constexpr int kListHist = 4096;

// Whether a range covers whole block-filter words (the count word and the
// words the table kernel writes for the range are the range's own).
__host__ __device__ inline bool build_ranges_cover_words(int32_t fshift) {
    const int ws = 5 + fshift;
    return (kBuildRange >> ws) >= 1 && ((kBuildRange >> ws) << ws) == kBuildRange;
}

// Ranges of a catalogue (the last may hold only the zero slot).
__host__ __device__ inline int64_t build_ranges(int32_t catalog) {
    return ((int64_t)catalog + kBuildRange) >> kBuildRangeShift;
}

// Range of catalogue event e, and e's offset in it.
__host__ __device__ inline int64_t build_range_of(int32_t e) { return (int64_t)(e >> kBuildRangeShift); }
__host__ __device__ inline uint32_t build_range_offset(int32_t e) { return (uint32_t)e & (kBuildRange - 1); }

// Table entries of range g: [g R, g R + range_events).
__host__ __device__ inline int64_t range_events(int64_t g, int32_t catalog) {
    const int64_t left = (int64_t)catalog + 1 - g * kBuildRange;
    return left < kBuildRange ? left : kBuildRange;
}

// 8-byte list entries that range g's part of the table holds (value_bytes:
// the table's value size), at most kBuildList.
__host__ __device__ inline int range_capacity(int64_t g, int32_t catalog, int value_bytes) {
    const int64_t cap = range_events(g, catalog) * value_bytes / 8;
    return cap < kBuildList ? (int)cap : kBuildList;
}

// Block-filter word that holds range g's count: the range's first word.
__host__ __device__ inline int64_t range_count_word(int64_t g, int32_t fshift) {
    return (g << kBuildRangeShift) >> (5 + fshift);
}

}  // namespace ara
