// Index arithmetic of the trial passes' YET loads.  The kernels call these
// functions, and a CPU test (tests/index_model.cpp) runs the same functions
// over every trial length and start to check that each 16-byte load stays
// inside the YET's last granule and that every event is taken exactly once.
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

}  // namespace ara
