// Internal types shared by the host side of libara and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ara.h"
#include "ara_index.h"

namespace ara {

constexpr int kMaxElts = ARA_MAX_ELTS;
constexpr int kWave = 64;

// A device-resident YET as the kernels see it.
struct YetView {
    const int32_t *ids;      // [n_events]
    const int64_t *offsets;  // [n_trials + 1] or nullptr (fixed length)
    int64_t n_trials;
    int64_t events_per_trial;  // used when offsets == nullptr
    int64_t n_events;
    int32_t aligned16;  // ids pointer is 16-byte aligned (vector loads allowed)
};

// Per-layer terms, in the arithmetic of the pass (T = double or float).
template <typename T>
struct Terms {
    T ret[kMaxElts];
    T lim[kMaxElts];
    T occ_ret, occ_lim;
    double agg_ret, agg_lim;  // aggregate terms are always binary64
    int32_t n_elts;
};

// Device pointers of a layer's tables (only those of its layout are set).
struct TablesView {
    // DIRECT: [n_elts][catalog] losses
    const void *direct;
    // SPARSE: ELT j holds sp_ids/sp_loss[sp_off[j] .. sp_off[j+1]), ids ascending
    const int32_t *sp_ids;
    const void *sp_loss;
    const int64_t *sp_off;
    // COMPACT: bm[w] = {presence bits of events 32w..32w+31, number of present
    // events below 32w}; rows[rank][n_elts] losses of present events
    const uint2 *bm;
    const void *rows;
    // FUSED: occ[catalog + 1] occurrence loss of every event (occ[catalog] = 0);
    // event E maps to bit E mod 32 of filt[E >> (fshift + 5)], which is set
    // iff one of the 2^fshift events sharing it (E + 32 t inside the word's
    // 2^(fshift + 5) events) has a non-zero occurrence loss.  When fshift > 0
    // a second, hashed filter follows in filt[n_fwords .. n_fwords +
    // n_hwords): bit E mod 32 of word ((E mod 2^24) * kHashMul24 mod 2^32)
    // >> (hshift + 5) is set for every event E with a non-zero occurrence
    // loss (n_hwords = 0: none).  A probe is one LDS word and a bit-field
    // extract at the ID's own low five bits.
    const void *occ;
    const uint32_t *filt;
    int32_t n_fwords;
    int32_t fshift;
    int32_t n_hwords;
    int32_t hshift;
    int32_t catalog;
    int32_t n_words;
};

// Largest block filter the fused pass keeps in LDS (bits): 128 KiB.
constexpr int64_t kFilterBits = 1 << 20;
// LDS of the fused pass for both filters (bytes), and the multiplier of the
// hashed filter: odd and below 2^24, so that the hash is one full-rate
// 24 x 24-bit multiply (IDs above 2^24 hash by their low 24 bits: more
// collisions, never a missed event).  Its filters let through as few events
// as a 32-bit multiplicative hash (checked on random, clustered and
// paper-shaped key sets); the golden-ratio fraction 0x9E3779 does not (its
// products' top bits vary slowly over IDs below 2^21: twice the false hits).
constexpr int64_t kFusedLdsBytes = 160 * 1024;
constexpr uint32_t kHashMul24 = 0xEBCA6Bu;

// LDS filters of the fused pass: a block filter of n_fwords words (blocks of
// 2^fshift events) and, when blocks hold more than one event, a hashed filter
// of n_hwords words (a power of two) in the LDS the block filter leaves free.
inline void filter_geometry(int32_t C, int32_t &fshift, int32_t &n_fwords, int32_t &n_hwords, int32_t &hshift) {
    fshift = 0;
    while ((((int64_t)C + (1LL << fshift) - 1) >> fshift) > kFilterBits) ++fshift;
    const int64_t n_blocks = ((int64_t)C + (1LL << fshift) - 1) >> fshift;
    n_fwords = (int32_t)((n_blocks + 31) / 32);
    n_hwords = 0;
    hshift = 0;
    const int64_t room = kFusedLdsBytes / 4 - n_fwords;
    if (fshift > 0 && room >= 1) {
        int64_t w = 1;
        int log2_bits = 5;
        while (w * 2 <= room) {
            w *= 2;
            ++log2_bits;
        }
        n_hwords = (int32_t)w;
        hshift = 32 - log2_bits;
    }
}

enum Layout : int32_t {
    kDirect = ARA_LAYOUT_DIRECT,
    kSparse = ARA_LAYOUT_SPARSE,
    kCompact = ARA_LAYOUT_COMPACT,
    kFused = ARA_LAYOUT_FUSED
};

struct LayerHost {
    int32_t n_elts = 0;
    int32_t catalog = 0;
    int32_t precision = 0;
    int32_t layout = 0;
    Terms<double> t64{};
    Terms<float> t32{};
    TablesView tab{};
    int64_t n_present = 0;  // COMPACT: events present in at least one ELT
    size_t bytes = 0;
    // device allocations owned by the layer
    void *alloc[6] = {};
};

// A non-blocking stream of the library for its own set-up work (one per
// device, created on first use; safe to call from several host threads).
hipStream_t internal_stream();
// Compute units of the current device (cached per device; 256 if unknown).
constexpr int kMaxDevices = 64;
int cu_count();
// Raises the dynamic LDS limit of a kernel to bytes on the current device,
// once per (device, kernel, bytes); safe to call from several host threads.
hipError_t allow_dynamic_lds(const void *kern, int bytes);

// Launchers (ara_kernels.hip).  Return a hipError_t.
hipError_t launch_validate_yet(const YetView &y, int32_t catalog, int32_t *d_flags, hipStream_t s);
// d_omax (optional, [n_trials]): the largest occurrence loss of each trial.
hipError_t launch_trial_pass(const YetView &y, const LayerHost &L, double *d_ylt, double *d_omax, hipStream_t s);
hipError_t launch_trial_pass_events(const YetView &y, const LayerHost &L, double *d_ylt, double *d_cum,
                                    double *d_net, hipStream_t s);

// Batched pass (ara_kernels.hip).  Records: one per catalogue event, bytes
// 0..7 the layer indices of its entries (kNoLayer = empty), then kRecVals
// values.  An event with more entries than fit keeps kRecVals - 1 inline,
// marks byte 7 with kOverflowMark, holds the number of further entries in
// byte kRecVals - 1 and their start in the overflow arrays in value slot
// kRecVals - 1 (as a uint32).  Each event's overflow entries start on a
// multiple of four and fill whole blocks of four (padding: kNoLayer, 0).
constexpr uint8_t kNoLayer = 0xff, kOverflowMark = 0xfe;
template <typename T>
struct RecFormat;
template <>
struct RecFormat<double> {
    static constexpr int kVals = 7, kBytes = 64;
};
template <>
struct RecFormat<float> {
    static constexpr int kVals = 6, kBytes = 32;
};

struct BatchTables {
    const void *rec;          // [catalog] records
    const uint8_t *ovf_lid;   // overflow layer indices
    const void *ovf_val;      // overflow values
    double *const *ylts;      // device array [n_layers] of YLT pointers
    const double *agg_ret;    // [n_layers]
    const double *agg_lim;    // [n_layers]
    int32_t n_layers;
};

// Dense form of a batch of at most kDenseMax layers, in sub-tables of at
// most kDenseWidth layers each (one pass over the YET per sub-table).  A
// sub-table holds one record of nl values per catalogue event (its
// occurrence losses in the sub-table's layers, in layer order, zeros past
// n_layers; the record of event `catalog` is all zeros), event-major, and
// the fused layers' two LDS filters built over the events with any non-zero
// value (same geometry as a fused layer's).
constexpr int kDenseMax = 16;
constexpr int kDenseWidth = 4;
struct DenseTables {
    const void *rec;          // [(catalog + 1) * nl]
    const uint32_t *filt;     // [n_fwords + n_hwords]
    int32_t n_fwords;
    int32_t fshift;
    int32_t n_hwords;
    int32_t hshift;
    int32_t catalog;
    int32_t nl;               // record width: 1, 2 or 4
    double *const *ylts;      // device array [n_layers] of YLT pointers
    const double *agg_ret;    // [n_layers]
    const double *agg_lim;    // [n_layers]
    int32_t n_layers;
};

struct BatchLaunch {
    int threads;     // work-group size (multiple of 64)
    int wg_per_cu;   // work-groups per CU requested (clamped by LDS)
    int group;       // 256-event chunks of a trial loaded per step (2, 4 or 8),
                     // or 1: the pipelined pass (one chunk per step, loads
                     // staged over three steps)
};
// Largest work-group of the pipelined batched pass.
constexpr int kMaxStreamThreads = 256;

// occ pointers of the layers -> records.  Returns the total number of
// overflow entries through *d_ovf_total (device) in the counting phase.
hipError_t launch_batch_count(const void *const *occ, int32_t n_layers, int32_t catalog, bool fp64, int32_t *d_count,
                              unsigned long long *d_ovf_total, hipStream_t s);
hipError_t launch_batch_fill(const void *const *occ, int32_t n_layers, int32_t catalog, bool fp64,
                             const int32_t *d_count, void *d_rec, uint8_t *d_ovf_lid, void *d_ovf_val,
                             unsigned long long *d_ovf_cursor, hipStream_t s);
hipError_t launch_batch_pass(const YetView &y, const BatchTables &b, bool fp64, const BatchLaunch &cfg, hipStream_t s);
// Dense form: records and filters from the layers' fused tables (filter
// words cleared first; *d_union_count, cleared by the caller, receives the
// number of events with any non-zero value), then the pass.
hipError_t launch_dense_fill(const void *const *occ, int32_t n_layers, bool fp64, const DenseTables &d,
                             unsigned long long *d_union_count, hipStream_t s);
// group: 256-event chunks loaded per step, 2 or 4 (2 only for 4-wide records)
hipError_t launch_dense_pass(const YetView &y, const DenseTables &d, bool fp64, int group, hipStream_t s);
size_t batch_lds_bytes(int32_t n_layers, int threads);
// Fused table of a layer, built on the GPU: the ELTs idx[0..n) of device
// arrays d_ids / d_loss (ELT k at host offsets off[k] .. off[k + 1]) added
// in that order, then the occurrence terms and the LDS filters; enqueued on
// s.  Used for pool layers and for layers from host ELTs alike.  d_lo:
// binary32 scratch [catalog] for FP32C, else unused.
hipError_t launch_pool_layer(LayerHost &L, const int32_t *d_ids, const void *d_loss, const int64_t *h_off,
                             const int32_t *h_idx, int32_t n, float *d_lo, hipStream_t s);
// The same table in three launches when fused_build_fits: the filter words
// cleared, each range's entries listed (one read of every ID), and the table
// with one work-group per kBuildRange catalogue events.
// host_losses: d_loss holds the ELTs' binary64 losses as given by the host,
// and the kernel validates every entry into *d_flags (bit 1 ID out of range,
// 2 duplicate ID in one ELT, 4 bad loss; cleared by the caller); else
// d_loss holds the pool's values (the layer's precision) and d_flags is
// unused.  Returns hipErrorNotSupported when the layer does not fit.
// (kBuildRange, kBuildThreads, kBuildList and the build's index arithmetic:
// ara_index.h)
constexpr int kBuildUnroll = 16;
// IDs read over all work-groups if every range overflowed its list
constexpr int64_t kBuildReadBudget = (int64_t)1 << 30;
struct BuildSegs {
    int64_t begin[kMaxElts];  // ELT j of the layer: entries begin[j] .. begin[j] + count[j]
    int64_t count[kMaxElts];
    double ret[kMaxElts];     // FT1 terms (binary64; converted like the layer's terms)
    double lim[kMaxElts];
    int32_t n;
};
bool fused_build_fits(int64_t catalog, int32_t fshift, int64_t n_entries);
hipError_t launch_fused_build(LayerHost &L, const int32_t *d_ids, const void *d_loss, bool host_losses,
                              const int64_t *h_off, const int32_t *h_idx, int32_t n, int *d_flags, hipStream_t s);
// d[0 .. n) = 0 with a kernel (no memset node if the caller captures a graph)
hipError_t launch_fill_zero(double *d, int64_t n, hipStream_t s);

// Roll-up (ara_rollup.hip): out[g][i] = sum of in[q][i] for q in
// first[g] .. first[g+1), added in that order from 0, for every group g.
struct RollupTables {
    const double *in[ARA_MAX_BATCH];
    double *out[ARA_MAX_BATCH];
    int32_t first[ARA_MAX_BATCH + 1];
    int32_t n_groups;
};
hipError_t launch_rollup(const RollupTables &a, int64_t n, hipStream_t s);

// Selection (ara_select.hip): PML / TVaR of n_ylt YLTs of length n for n_rp
// tail sizes k[r]; h_out[2 * (y * n_rp + r)] = PML, [... + 1] = TVaR.
hipError_t pml_tvar_device(const double *const *d_ylts, int32_t n_ylt, int64_t n, const int64_t *h_k, int32_t n_rp,
                           double *h_out, int32_t *h_nan, hipStream_t s);
// The same selection over the library's static device scratch, results into
// device arrays; asynchronous, allocates nothing.
hipError_t pml_tvar_noalloc(const double *const *d_ylts, int32_t n_ylt, int64_t n, const int64_t *h_k, int32_t n_rp,
                            double *d_pml, double *d_tvar, hipStream_t s);

}  // namespace ara
