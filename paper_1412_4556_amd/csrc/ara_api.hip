// C ABI of libara: argument checks, layer table construction, handles and
// errors.  The operations themselves run in the HIP kernels of
// ara_kernels.hip and ara_select.hip.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "ara_internal.h"

struct ara_yet_s {
    ara::YetView v{};
    int32_t catalog = 0;
    int device = 0;
};

struct ara_pool_s;

struct ara_layer_s {
    ara::LayerHost h;
    int device = 0;
    ara_pool_s *pool = nullptr;   // layer built from a pool slot (not owned)
    int slot = -1;
    hipEvent_t ready = nullptr;   // recorded after the device build of a pool layer
};

// A device-resident set of ELTs from which layers are built on the GPU, and
// a fixed number of table slots for such layers (the admission budget).
struct ara_pool_s {
    int32_t n_elts = 0;
    int32_t precision = 0;
    int32_t catalog = 0;
    int32_t max_layers = 0;
    int32_t fshift = 0;
    int32_t n_fwords = 0;
    int32_t n_hwords = 0;
    int32_t hshift = 0;
    int device = 0;
    void *d_ids = nullptr;
    void *d_loss = nullptr;
    std::vector<int64_t> off;  // host [n_elts + 1]
    std::vector<void *> occ, filt, lo;
    std::vector<hipEvent_t> ready;
    std::vector<int> free_slots;
    std::mutex mu;
    size_t slot_bytes = 0;
    size_t bytes = 0;
};

struct ara_batch_s {
    ara::YetView yv{};
    int32_t n = 0;
    int32_t precision = 0;
    int32_t catalog = 0;
    // form of the current layers: dense (at most ara::kDenseMax layers) or
    // sparse records; each form's buffers are allocated when first needed
    // and kept (grown, never shrunk) for later rebuilds
    bool dense = false;
    void *d_dense = nullptr;      // dense records: sub-table s at s * dense_stride bytes
    size_t dense_cap = 0;         // bytes
    size_t dense_stride = 0;      // bytes of one sub-table ((catalog + 1) * kDenseWidth values)
    uint32_t *d_dfilt = nullptr;  // dense filters: sub-table s at s * (n_fwords + n_hwords) words
    int32_t dfilt_subs = 0;       // sub-tables the filter allocation holds
    int32_t fshift = 0, n_fwords = 0, n_hwords = 0, hshift = 0;
    void *d_rec = nullptr;        // sparse records
    void *d_ovf_lid = nullptr;
    void *d_ovf_val = nullptr;
    int32_t *d_count = nullptr; // [catalog] entries per event (record build scratch)
    unsigned long long *d_ctr = nullptr;  // overflow total, fill cursor
    unsigned long long ovf_cap = 0;
    unsigned long long *d_ucount = nullptr;  // [kDenseMax / kDenseWidth] events in each dense sub-table's union
    double **d_ylts = nullptr;  // device array of the YLT pointers of the last run
    double *d_agg = nullptr;    // [2 * ARA_MAX_BATCH]: aggregate retentions, then limits
    std::vector<double *> h_ylts;
    ara::BatchLaunch cfg{256, 1, 4};
    // dense form: tuned chunk-group size per record width (1, 2, 4: index 0..2)
    int dgroup[3] = {0, 0, 0};
    bool tuned = false;
    bool use_graph = true;
    int capture_failures = 0;  // in a row; the batch stops capturing after kMaxCaptureFailures
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // what the captured graph's kernel arguments hold: it is replayed only
    // while the batch's form, tables and launch shape are still these
    bool graph_dense = false;
    ara::BatchTables graph_tables{};
    const void *graph_drec = nullptr;
    const uint32_t *graph_dfilt = nullptr;
    ara::BatchLaunch graph_cfg{0, 0, 0};
    // recorded on the caller's stream after every run: a rebuild, and a run
    // on another stream, wait for it before they overwrite what the last
    // run reads (records, overflow entries, terms, YLT pointers)
    hipEvent_t last_run = nullptr;
    hipStream_t last_stream = nullptr;
    bool ran = false;
    bool valid = false;  // records match the layers (false after a failed rebuild)
    size_t bytes = 0;
    int device = 0;
};

namespace {

// Message of the last failing call, per host thread, in a fixed buffer (so
// that reporting an error allocates nothing).
thread_local char g_err[512];

ara_status fail(ara_status code, const char *msg) {
    std::snprintf(g_err, sizeof(g_err), "%s", msg);
    return code;
}

ara_status fail(ara_status code, const std::string &msg) { return fail(code, msg.c_str()); }

ara_status hip_fail(hipError_t e, const char *what) {
    std::snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ARA_ERR_OOM : ARA_ERR_DEVICE;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }
bool limit_ok(double x) { return !std::isnan(x) && x >= 0.0; }

// Optional allocation-failure injection for tests of the error paths:
// ARA_FAULT_ALLOC_AFTER=n makes the (n+1)-th device allocation fail.
long long fault_budget() {
    static long long v = [] {
        const char *s = std::getenv("ARA_FAULT_ALLOC_AFTER");
        return s ? std::atoll(s) : -1LL;
    }();
    return v;
}
std::atomic<long long> g_alloc_count{0};

// Optional capture-failure injection for tests of the fallback:
// ARA_FAULT_CAPTURE=1 makes every batch graph capture fail as an
// invalidated capture does.
bool fault_capture() {
    static bool v = [] {
        const char *s = std::getenv("ARA_FAULT_CAPTURE");
        return s && std::atoi(s) != 0;
    }();
    return v;
}

// Device staging of the ELTs of fused layers built from host memory: one
// buffer per device, grown on demand and kept until the process ends, used
// under its lock (a build is synchronous).
struct Staging {
    std::mutex mu;
    void *d = nullptr;
    size_t cap = 0;
};
// dev in 0 .. kMaxDevices - 1 (checked by the caller)
Staging &staging_for(int dev) {
    static Staging s[ara::kMaxDevices];
    return s[dev];
}

hipError_t dev_alloc(void **p, size_t bytes) {
    long long fb = fault_budget();
    if (fb >= 0 && g_alloc_count++ >= fb) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    if (bytes == 0) bytes = 16;
    return hipMalloc(p, bytes);
}

void free_layer_memory(ara::LayerHost &h) {
    for (void *&p : h.alloc)
        if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
}

template <typename T>
ara_status upload(ara::LayerHost &h, int slot, const T *src, size_t count, const void **dst) {
    void *d = nullptr;
    hipError_t e = dev_alloc(&d, count * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "device allocation of layer tables");
    h.alloc[slot] = d;
    h.bytes += count * sizeof(T);
    if (count) {
        hipStream_t s = ara::internal_stream();
        e = hipMemcpyAsync(d, src, count * sizeof(T), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "copy of layer tables");
    }
    *dst = d;
    return ARA_OK;
}

// ELT sizes -> start offsets of the ELTs in the concatenated arrays.
ara_status elt_starts(int32_t C, int32_t n_elts, const int32_t *h_elt_ids, const double *h_elt_losses,
                      const int64_t *h_elt_sizes, std::vector<int64_t> &start) {
    start.assign(n_elts + 1, 0);
    for (int j = 0; j < n_elts; ++j) {
        if (h_elt_sizes[j] < 0) return fail(ARA_ERR_INVALID_ARG, "negative ELT size");
        if (h_elt_sizes[j] > C) return fail(ARA_ERR_DUP_EVENT, "ELT larger than the catalogue");
        start[j + 1] = start[j] + h_elt_sizes[j];
    }
    if (start[n_elts] > 0 && (!h_elt_ids || !h_elt_losses)) return fail(ARA_ERR_INVALID_ARG, "NULL ELT arrays");
    return ARA_OK;
}

// Every entry: ID in range, unique within its ELT, loss finite and >= 0.
ara_status validate_elts(int32_t C, int32_t n_elts, const int32_t *h_elt_ids, const double *h_elt_losses,
                         const int64_t *h_elt_sizes, std::vector<int64_t> &start) {
    ara_status st = elt_starts(C, n_elts, h_elt_ids, h_elt_losses, h_elt_sizes, start);
    if (st != ARA_OK) return st;
    // one bit per catalogue event (C / 8 bytes, cache-resident at the paper's
    // sizes), set by an ELT's IDs and cleared again before the next ELT
    std::vector<uint64_t> seen;
    try {
        seen.assign(((size_t)C + 63) / 64, 0);
    } catch (const std::bad_alloc &) {
        return fail(ARA_ERR_OOM, "host allocation");
    }
    for (int j = 0; j < n_elts; ++j) {
        for (int64_t n = start[j]; n < start[j + 1]; ++n) {
            const int32_t e = h_elt_ids[n];
            if (e < 0 || e >= C) return fail(ARA_ERR_EVENT_RANGE, "ELT event ID outside [0, catalog_size)");
            const uint64_t bit = 1ULL << (e & 63);
            if (seen[(size_t)e >> 6] & bit) return fail(ARA_ERR_DUP_EVENT, "duplicate event ID in one ELT");
            seen[(size_t)e >> 6] |= bit;
            if (!finite_nonneg(h_elt_losses[n])) return fail(ARA_ERR_VALUE, "ELT loss must be finite and >= 0");
        }
        for (int64_t n = start[j]; n < start[j + 1]; ++n) seen[(size_t)h_elt_ids[n] >> 6] = 0;
    }
    return ARA_OK;
}

ara_status validate_terms(int32_t n_elts, const double *h_ret, const double *h_lim, double occ_ret, double occ_lim,
                          double agg_ret, double agg_lim) {
    for (int j = 0; j < n_elts; ++j) {
        if (!finite_nonneg(h_ret[j])) return fail(ARA_ERR_VALUE, "ELT retention must be finite and >= 0");
        if (!limit_ok(h_lim[j])) return fail(ARA_ERR_VALUE, "ELT limit must be >= 0");
    }
    if (!finite_nonneg(occ_ret) || !limit_ok(occ_lim)) return fail(ARA_ERR_VALUE, "bad occurrence terms");
    if (!finite_nonneg(agg_ret) || !limit_ok(agg_lim)) return fail(ARA_ERR_VALUE, "bad aggregate terms");
    return ARA_OK;
}

void set_terms(ara::LayerHost &h, int32_t n_elts, const double *h_ret, const double *h_lim, double occ_ret,
               double occ_lim, double agg_ret, double agg_lim) {
    for (int j = 0; j < n_elts; ++j) {
        h.t64.ret[j] = h_ret[j];
        h.t64.lim[j] = h_lim[j];
        h.t32.ret[j] = (float)h_ret[j];
        h.t32.lim[j] = (float)h_lim[j];
    }
    h.t64.occ_ret = occ_ret;
    h.t64.occ_lim = occ_lim;
    h.t32.occ_ret = (float)occ_ret;
    h.t32.occ_lim = (float)occ_lim;
    h.t64.agg_ret = h.t32.agg_ret = agg_ret;
    h.t64.agg_lim = h.t32.agg_lim = agg_lim;
    h.t64.n_elts = h.t32.n_elts = n_elts;
}

template <typename T>
ara_status build_tables(ara::LayerHost &h, const int32_t *ids, const double *loss, const std::vector<int64_t> &start,
                        const int64_t *sizes) {
    const int J = h.n_elts;
    const int64_t C = h.catalog;
    ara_status st = ARA_OK;
    if (h.layout == ara::kDirect) {
        std::vector<T> tab;
        try {
            tab.assign((size_t)J * (size_t)C, T(0));
        } catch (const std::bad_alloc &) {
            return fail(ARA_ERR_OOM, "host allocation of the direct-access tables");
        }
        for (int j = 0; j < J; ++j)
            for (int64_t n = 0; n < sizes[j]; ++n) tab[(size_t)j * C + ids[start[j] + n]] = (T)loss[start[j] + n];
        const void *d;
        if ((st = upload(h, 0, tab.data(), tab.size(), &d)) != ARA_OK) return st;
        h.tab.direct = d;
    } else if (h.layout == ara::kSparse) {
        std::vector<int32_t> sid;
        std::vector<T> sl;
        std::vector<int64_t> off(J + 1, 0);
        sid.reserve(start[J]);
        sl.reserve(start[J]);
        for (int j = 0; j < J; ++j) {
            std::vector<int64_t> perm(sizes[j]);
            std::iota(perm.begin(), perm.end(), (int64_t)0);
            const int32_t *e = ids + start[j];
            std::sort(perm.begin(), perm.end(), [e](int64_t a, int64_t b) { return e[a] < e[b]; });
            for (int64_t p : perm) {
                sid.push_back(e[p]);
                sl.push_back((T)loss[start[j] + p]);
            }
            off[j + 1] = (int64_t)sid.size();
        }
        const void *d0, *d1, *d2;
        if ((st = upload(h, 0, sid.data(), sid.size(), &d0)) != ARA_OK) return st;
        if ((st = upload(h, 1, sl.data(), sl.size(), &d1)) != ARA_OK) return st;
        if ((st = upload(h, 2, off.data(), off.size(), &d2)) != ARA_OK) return st;
        h.tab.sp_ids = static_cast<const int32_t *>(d0);
        h.tab.sp_loss = d1;
        h.tab.sp_off = static_cast<const int64_t *>(d2);
    } else if (h.layout == ara::kFused) {
        // occurrence loss per catalogue event, built on the GPU from the
        // layer's ELTs in layer order (the kernels of pool layers), then the
        // LDS filters; the ELTs are staged in the device's build buffer, so
        // the build allocates nothing but the layer's own tables
        const size_t n = (size_t)start[J];
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "current device");
        if (dev < 0 || dev >= ara::kMaxDevices) return fail(ARA_ERR_UNSUPPORTED, "device id beyond the library's tables");
        int32_t fshift = 0, n_fwords = 0, n_hwords = 0, hshift = 0;
        ara::filter_geometry((int32_t)C, fshift, n_fwords, n_hwords, hshift);
        void *d_occ = nullptr, *d_filt = nullptr;
        // catalogue + 1 entries: occ[C] stays 0 for the pass's unmarked lanes
        e = dev_alloc(&d_occ, ((size_t)C + 1) * sizeof(T));
        if (e != hipSuccess) return hip_fail(e, "device allocation of the fused table");
        h.alloc[2] = d_occ;
        h.bytes += ((size_t)C + 1) * sizeof(T);
        e = dev_alloc(&d_filt, (size_t)(n_fwords + n_hwords) * sizeof(uint32_t));
        if (e != hipSuccess) return hip_fail(e, "device allocation of the fused filter");
        h.alloc[3] = d_filt;
        h.bytes += (size_t)(n_fwords + n_hwords) * sizeof(uint32_t);
        h.tab.occ = d_occ;
        h.tab.filt = static_cast<const uint32_t *>(d_filt);
        h.tab.fshift = fshift;
        h.tab.n_fwords = (int32_t)n_fwords;
        h.tab.n_hwords = n_hwords;
        h.tab.hshift = hshift;
        const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
        if (ara::fused_build_fits(C, fshift, (int64_t)n)) {
            // the GPU build makes the table from the ELTs as given (binary64
            // losses) and checks every entry on the way
            const size_t b_ids = up(n * sizeof(int32_t)), b_loss = up(n * sizeof(double));
            const size_t need = b_ids + b_loss + 256;
            Staging &sg = staging_for(dev);
            std::lock_guard<std::mutex> g(sg.mu);
            if (sg.cap < need) {
                if (sg.d) (void)hipFree(sg.d);
                sg.d = nullptr;
                sg.cap = 0;
                e = dev_alloc(&sg.d, need);
                if (e != hipSuccess) {
                    sg.d = nullptr;
                    return hip_fail(e, "device allocation of the build staging");
                }
                sg.cap = need;
            }
            char *base = static_cast<char *>(sg.d);
            int32_t *d_ids = reinterpret_cast<int32_t *>(base);
            double *d_loss = reinterpret_cast<double *>(base + b_ids);
            int *d_flags = reinterpret_cast<int *>(base + b_ids + b_loss);
            hipStream_t s = ara::internal_stream();
            if (!s) return fail(ARA_ERR_DEVICE, "no set-up stream");
            e = hipMemsetAsync(d_flags, 0, sizeof(int), s);
            if (e == hipSuccess && n) e = hipMemcpyAsync(d_ids, ids, n * sizeof(int32_t), hipMemcpyHostToDevice, s);
            if (e == hipSuccess && n) e = hipMemcpyAsync(d_loss, loss, n * sizeof(double), hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "copy of the layer's ELTs");
            std::vector<int32_t> order(J);
            for (int j = 0; j < J; ++j) order[j] = j;
            e = ara::launch_fused_build(h, d_ids, d_loss, true, start.data(), order.data(), J, d_flags, s);
            int flags = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(&flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, s);
            // the staging is reused by the next build only after this wait
            const hipError_t se = hipStreamSynchronize(s);
            if (e == hipSuccess) e = se;
            if (e != hipSuccess) return hip_fail(e, "building the fused table");
            if (flags & 1) return fail(ARA_ERR_EVENT_RANGE, "ELT event ID outside [0, catalog_size)");
            if (flags & 2) return fail(ARA_ERR_DUP_EVENT, "duplicate event ID in one ELT");
            if (flags & 4) return fail(ARA_ERR_VALUE, "ELT loss must be finite and >= 0");
            return ARA_OK;
        }
        // staging: IDs, losses in the layer's arithmetic and, for FP32C, the
        // compensation terms of the binary32 sums (256-byte aligned parts)
        const size_t b_ids = up(n * sizeof(int32_t)), b_loss = up(n * sizeof(T));
        const size_t b_lo = sizeof(T) == sizeof(float) ? up((size_t)C * sizeof(float)) : 0;
        const size_t need = b_ids + b_loss + b_lo > 256 ? b_ids + b_loss + b_lo : 256;
        std::vector<T> lt;
        if (sizeof(T) != sizeof(double)) {
            lt.resize(n);
            for (size_t i = 0; i < n; ++i) lt[i] = (T)loss[i];
        }
        const void *h_loss = sizeof(T) == sizeof(double) ? static_cast<const void *>(loss) : lt.data();
        Staging &sg = staging_for(dev);
        std::lock_guard<std::mutex> g(sg.mu);
        if (sg.cap < need) {
            if (sg.d) (void)hipFree(sg.d);
            sg.d = nullptr;
            sg.cap = 0;
            e = dev_alloc(&sg.d, need);
            if (e != hipSuccess) {
                sg.d = nullptr;
                return hip_fail(e, "device allocation of the build staging");
            }
            sg.cap = need;
        }
        char *base = static_cast<char *>(sg.d);
        int32_t *d_ids = reinterpret_cast<int32_t *>(base);
        void *d_loss = base + b_ids;
        float *d_lo = b_lo ? reinterpret_cast<float *>(base + b_ids + b_loss) : nullptr;
        hipStream_t s = ara::internal_stream();
        if (!s) return fail(ARA_ERR_DEVICE, "no set-up stream");
        if (n) e = hipMemcpyAsync(d_ids, ids, n * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && n) e = hipMemcpyAsync(d_loss, h_loss, n * sizeof(T), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "copy of the layer's ELTs");
        std::vector<int32_t> order(J);
        for (int j = 0; j < J; ++j) order[j] = j;
        e = ara::launch_pool_layer(h, d_ids, d_loss, start.data(), order.data(), J, d_lo, s);
        // the staging is reused by the next build only after this wait
        const hipError_t se = hipStreamSynchronize(s);
        if (e == hipSuccess) e = se;
        if (e != hipSuccess) return hip_fail(e, "building the fused table");
    } else {
        const int64_t n_words = (C + 31) / 32;
        std::vector<uint2> bm((size_t)n_words, uint2{0u, 0u});
        for (int j = 0; j < J; ++j)
            for (int64_t n = 0; n < sizes[j]; ++n) {
                int32_t e = ids[start[j] + n];
                bm[e >> 5].x |= 1u << (e & 31);
            }
        uint32_t rank = 0;
        for (int64_t w = 0; w < n_words; ++w) {
            bm[w].y = rank;
            rank += (uint32_t)__builtin_popcount(bm[w].x);
        }
        h.n_present = rank;
        std::vector<T> rows;
        try {
            rows.assign((size_t)rank * (size_t)J, T(0));
        } catch (const std::bad_alloc &) {
            return fail(ARA_ERR_OOM, "host allocation of the compact rows");
        }
        for (int j = 0; j < J; ++j)
            for (int64_t n = 0; n < sizes[j]; ++n) {
                int32_t e = ids[start[j] + n];
                uint2 w = bm[e >> 5];
                uint32_t bit = 1u << (e & 31);
                size_t idx = (size_t)w.y + (size_t)__builtin_popcount(w.x & (bit - 1u));
                rows[idx * J + j] = (T)loss[start[j] + n];
            }
        const void *d0, *d1;
        if ((st = upload(h, 0, bm.data(), bm.size(), &d0)) != ARA_OK) return st;
        if ((st = upload(h, 1, rows.data(), rows.size(), &d1)) != ARA_OK) return st;
        h.tab.bm = static_cast<const uint2 *>(d0);
        h.tab.rows = d1;
        h.tab.n_words = (int32_t)n_words;
    }
    return ARA_OK;
}

}  // namespace

extern "C" {

const char *ara_last_error(void) { return g_err; }

int32_t ara_abi_version(void) { return 1; }

ara_status ara_create_yet(const int32_t *d_event_ids, const int64_t *d_offsets, int64_t n_trials,
                          int64_t events_per_trial, int32_t catalog_size, void *hip_stream, ara_yet *out) {
    if (!out) return fail(ARA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_trials < 0) return fail(ARA_ERR_INVALID_ARG, "n_trials < 0");
    if (catalog_size < 1) return fail(ARA_ERR_INVALID_ARG, "catalog_size < 1");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    ara::YetView v{};
    v.ids = d_event_ids;
    v.offsets = d_offsets;
    v.n_trials = n_trials;
    if (!d_offsets) {
        if (events_per_trial < 0) return fail(ARA_ERR_INVALID_ARG, "events_per_trial < 0");
        if (events_per_trial > 0 && n_trials > std::numeric_limits<int64_t>::max() / events_per_trial)
            return fail(ARA_ERR_INVALID_ARG, "n_trials * events_per_trial overflows");
        v.events_per_trial = events_per_trial;
        v.n_events = n_trials * events_per_trial;
    } else {
        int64_t last = 0;
        hipError_t e = hipMemcpyAsync(&last, d_offsets + n_trials, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "reading offsets[n_trials]");
        if (last < 0) return fail(ARA_ERR_INVALID_ARG, "offsets[n_trials] < 0");
        v.n_events = last;
    }
    if (v.n_events > 0 && !d_event_ids) return fail(ARA_ERR_INVALID_ARG, "d_event_ids is NULL");
    v.aligned16 = ((reinterpret_cast<uintptr_t>(d_event_ids) & 15u) == 0u) ? 1 : 0;

    if (v.n_events > 0 || d_offsets) {
        int32_t *d_flags = nullptr;
        hipError_t e = dev_alloc(reinterpret_cast<void **>(&d_flags), 2 * sizeof(int32_t));
        if (e != hipSuccess) return hip_fail(e, "validation flags");
        int32_t hf[2] = {0, 0};
        e = hipMemcpyAsync(d_flags, hf, sizeof(hf), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = ara::launch_validate_yet(v, catalog_size, d_flags, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hf, d_flags, sizeof(hf), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(d_flags);
        if (e != hipSuccess) return hip_fail(e, "YET validation");
        if (hf[1]) return fail(ARA_ERR_INVALID_ARG, "offsets must start at 0 and be non-decreasing");
        if (hf[0]) return fail(ARA_ERR_EVENT_RANGE, "an event ID lies outside [0, catalog_size)");
    }
    ara_yet_s *y = new (std::nothrow) ara_yet_s;
    if (!y) return fail(ARA_ERR_OOM, "host allocation");
    y->v = v;
    y->catalog = catalog_size;
    (void)hipGetDevice(&y->device);
    *out = y;
    return ARA_OK;
}

void ara_destroy_yet(ara_yet yet) {
    if (!yet) return;
    (void)hipDeviceSynchronize();
    delete yet;
}

ara_status ara_create_layer(ara_yet yet, int32_t n_elts, const int32_t *h_elt_ids, const double *h_elt_losses,
                            const int64_t *h_elt_sizes, const double *h_ret, const double *h_lim, double occ_ret,
                            double occ_lim, double agg_ret, double agg_lim, int32_t precision, int32_t layout,
                            ara_layer *out) {
    if (!out) return fail(ARA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!yet) return fail(ARA_ERR_INVALID_ARG, "yet is NULL");
    if (n_elts < 1) return fail(ARA_ERR_INVALID_ARG, "n_elts < 1");
    if (n_elts > ARA_MAX_ELTS) return fail(ARA_ERR_UNSUPPORTED, "n_elts exceeds ARA_MAX_ELTS");
    if (precision != ARA_FP64 && precision != ARA_FP32C) return fail(ARA_ERR_INVALID_ARG, "unknown precision");
    if (layout < ARA_LAYOUT_AUTO || layout > ARA_LAYOUT_FUSED) return fail(ARA_ERR_INVALID_ARG, "unknown layout");
    if (!h_elt_sizes || !h_ret || !h_lim) return fail(ARA_ERR_INVALID_ARG, "NULL term or size array");
    const int32_t C = yet->catalog;
    std::vector<int64_t> start;
    ara_status vst = elt_starts(C, n_elts, h_elt_ids, h_elt_losses, h_elt_sizes, start);
    if (vst != ARA_OK) return vst;
    // a fused layer built on the GPU has its entries checked by the build's
    // kernels; every other layer checks them here
    int32_t fshift = 0, n_fwords = 0, n_hwords = 0, hshift = 0;
    ara::filter_geometry(C, fshift, n_fwords, n_hwords, hshift);
    const bool fused = layout == ARA_LAYOUT_AUTO || layout == ARA_LAYOUT_FUSED;
    const bool gpu_checked = fused && ara::fused_build_fits(C, fshift, start[n_elts]);
    if (!gpu_checked) {
        vst = validate_elts(C, n_elts, h_elt_ids, h_elt_losses, h_elt_sizes, start);
        if (vst != ARA_OK) return vst;
    }
    vst = validate_terms(n_elts, h_ret, h_lim, occ_ret, occ_lim, agg_ret, agg_lim);
    if (vst != ARA_OK) return vst;

    ara_layer_s *L = new (std::nothrow) ara_layer_s;
    if (!L) return fail(ARA_ERR_OOM, "host allocation");
    ara::LayerHost &h = L->h;
    h.n_elts = n_elts;
    h.catalog = C;
    h.precision = precision;
    h.layout = layout == ARA_LAYOUT_AUTO ? ARA_LAYOUT_FUSED : layout;
    h.tab.catalog = C;
    set_terms(h, n_elts, h_ret, h_lim, occ_ret, occ_lim, agg_ret, agg_lim);
    (void)hipGetDevice(&L->device);

    ara_status st = precision == ARA_FP32C ? build_tables<float>(h, h_elt_ids, h_elt_losses, start, h_elt_sizes)
                                           : build_tables<double>(h, h_elt_ids, h_elt_losses, start, h_elt_sizes);
    if (st != ARA_OK) {
        free_layer_memory(h);
        delete L;
        return st;
    }
    *out = L;
    return ARA_OK;
}

void ara_destroy_layer(ara_layer layer) {
    if (!layer) return;
    if (layer->pool) {
        // the slot returns to its pool without a device-wide wait; its next
        // build is ordered after this layer's build and the caller's use of it
        std::lock_guard<std::mutex> g(layer->pool->mu);
        layer->pool->free_slots.push_back(layer->slot);
        delete layer;
        return;
    }
    (void)hipDeviceSynchronize();
    free_layer_memory(layer->h);
    delete layer;
}

size_t ara_layer_device_bytes(ara_layer layer) { return layer ? layer->h.bytes : 0; }
int32_t ara_layer_layout(ara_layer layer) { return layer ? layer->h.layout : -1; }
int32_t ara_layer_precision(ara_layer layer) { return layer ? layer->h.precision : -1; }
int32_t ara_layer_n_elts(ara_layer layer) { return layer ? layer->h.n_elts : -1; }

ara_status ara_run_layer(ara_yet yet, ara_layer layer, double *d_ylt, void *hip_stream) {
    if (!yet || !layer) return fail(ARA_ERR_INVALID_ARG, "NULL handle");
    if (layer->h.catalog != yet->catalog) return fail(ARA_ERR_INVALID_ARG, "layer built for another catalogue");
    if (yet->v.n_trials > 0 && !d_ylt) return fail(ARA_ERR_INVALID_ARG, "d_ylt is NULL");
    if (layer->ready) {
        hipError_t we = hipStreamWaitEvent(static_cast<hipStream_t>(hip_stream), layer->ready, 0);
        if (we != hipSuccess) return hip_fail(we, "waiting for the layer build");
    }
    hipError_t e = ara::launch_trial_pass(yet->v, layer->h, d_ylt, nullptr, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "trial pass launch");
    return ARA_OK;
}

ara_status ara_run_layer_max_occurrence(ara_yet yet, ara_layer layer, double *d_ylt, double *d_max_occ,
                                        void *hip_stream) {
    if (!yet || !layer) return fail(ARA_ERR_INVALID_ARG, "NULL handle");
    if (layer->h.catalog != yet->catalog) return fail(ARA_ERR_INVALID_ARG, "layer built for another catalogue");
    if (yet->v.n_trials > 0 && (!d_ylt || !d_max_occ)) return fail(ARA_ERR_INVALID_ARG, "d_ylt or d_max_occ is NULL");
    if (layer->ready) {
        hipError_t we = hipStreamWaitEvent(static_cast<hipStream_t>(hip_stream), layer->ready, 0);
        if (we != hipSuccess) return hip_fail(we, "waiting for the layer build");
    }
    hipError_t e = ara::launch_trial_pass(yet->v, layer->h, d_ylt, d_max_occ, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "trial pass launch");
    return ARA_OK;
}

ara_status ara_run_layer_events(ara_yet yet, ara_layer layer, double *d_ylt, double *d_event_cum, double *d_event_net,
                                void *hip_stream) {
    if (!yet || !layer) return fail(ARA_ERR_INVALID_ARG, "NULL handle");
    if (layer->h.catalog != yet->catalog) return fail(ARA_ERR_INVALID_ARG, "layer built for another catalogue");
    if (yet->v.n_trials > 0 && !d_ylt) return fail(ARA_ERR_INVALID_ARG, "d_ylt is NULL");
    if (layer->ready) {
        hipError_t we = hipStreamWaitEvent(static_cast<hipStream_t>(hip_stream), layer->ready, 0);
        if (we != hipSuccess) return hip_fail(we, "waiting for the layer build");
    }
    hipError_t e = ara::launch_trial_pass_events(yet->v, layer->h, d_ylt, d_event_cum, d_event_net,
                                                 static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "per-event trial pass launch");
    return ARA_OK;
}

static void free_pool(ara_pool p) {
    for (void *q : p->occ)
        if (q) (void)hipFree(q);
    for (void *q : p->filt)
        if (q) (void)hipFree(q);
    for (void *q : p->lo)
        if (q) (void)hipFree(q);
    for (hipEvent_t ev : p->ready)
        if (ev) (void)hipEventDestroy(ev);
    if (p->d_ids) (void)hipFree(p->d_ids);
    if (p->d_loss) (void)hipFree(p->d_loss);
    delete p;
}

static ara_status upload_pool_losses(ara_pool p, const double *h_losses, size_t n, bool fp32) {
    const size_t vb = fp32 ? sizeof(float) : sizeof(double);
    std::vector<float> f;
    if (fp32) {
        f.resize(n);
        for (size_t i = 0; i < n; ++i) f[i] = (float)h_losses[i];
    }
    const void *src = fp32 ? static_cast<const void *>(f.data()) : static_cast<const void *>(h_losses);
    hipError_t e = dev_alloc(&p->d_loss, n * vb);
    hipStream_t s = ara::internal_stream();
    if (e == hipSuccess && n) e = hipMemcpyAsync(p->d_loss, src, n * vb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pool upload");
    p->bytes += n * vb;
    return ARA_OK;
}

ara_status ara_create_pool(ara_yet yet, int32_t n_elts, const int32_t *h_elt_ids, const double *h_elt_losses,
                           const int64_t *h_elt_sizes, int32_t precision, int32_t max_layers, ara_pool *out) {
    if (!out) return fail(ARA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!yet || !h_elt_sizes) return fail(ARA_ERR_INVALID_ARG, "NULL yet or sizes");
    if (n_elts < 1) return fail(ARA_ERR_INVALID_ARG, "n_elts < 1");
    if (max_layers < 1) return fail(ARA_ERR_INVALID_ARG, "max_layers < 1");
    if (precision != ARA_FP64 && precision != ARA_FP32C) return fail(ARA_ERR_INVALID_ARG, "unknown precision");
    std::vector<int64_t> start;
    ara_status st = validate_elts(yet->catalog, n_elts, h_elt_ids, h_elt_losses, h_elt_sizes, start);
    if (st != ARA_OK) return st;
    ara_pool_s *p = new (std::nothrow) ara_pool_s;
    if (!p) return fail(ARA_ERR_OOM, "host allocation");
    p->n_elts = n_elts;
    p->precision = precision;
    p->catalog = yet->catalog;
    p->max_layers = max_layers;
    p->off = start;
    (void)hipGetDevice(&p->device);
    ara::filter_geometry(yet->catalog, p->fshift, p->n_fwords, p->n_hwords, p->hshift);
    const size_t total = (size_t)start[n_elts];
    hipStream_t s = ara::internal_stream();
    hipError_t e = dev_alloc(&p->d_ids, total * sizeof(int32_t));
    if (e == hipSuccess && total)
        e = hipMemcpyAsync(p->d_ids, h_elt_ids, total * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_pool(p);
        return hip_fail(e, "pool upload");
    }
    p->bytes += total * sizeof(int32_t);
    st = upload_pool_losses(p, h_elt_losses, total, precision == ARA_FP32C);
    if (st != ARA_OK) {
        free_pool(p);
        return st;
    }
    const size_t C = (size_t)yet->catalog;
    const size_t occ_bytes = (C + 1) * (precision == ARA_FP32C ? sizeof(float) : sizeof(double));
    const size_t filt_bytes = (size_t)(p->n_fwords + p->n_hwords) * sizeof(uint32_t);
    const size_t lo_bytes = precision == ARA_FP32C ? C * sizeof(float) : 0;
    p->slot_bytes = occ_bytes + filt_bytes + lo_bytes;
    p->occ.assign(max_layers, nullptr);
    p->filt.assign(max_layers, nullptr);
    p->lo.assign(max_layers, nullptr);
    p->ready.assign(max_layers, nullptr);
    for (int i = 0; i < max_layers && e == hipSuccess; ++i) {
        e = dev_alloc(&p->occ[i], occ_bytes);
        if (e == hipSuccess) e = dev_alloc(&p->filt[i], filt_bytes);
        if (e == hipSuccess && lo_bytes) e = dev_alloc(&p->lo[i], lo_bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ready[i], hipEventDisableTiming);
        p->free_slots.push_back(max_layers - 1 - i);
    }
    if (e != hipSuccess) {
        free_pool(p);
        return hip_fail(e, "pool layer slots");
    }
    p->bytes += p->slot_bytes * (size_t)max_layers;
    *out = p;
    return ARA_OK;
}

void ara_destroy_pool(ara_pool pool) {
    if (!pool) return;
    (void)hipDeviceSynchronize();
    free_pool(pool);
}

size_t ara_pool_device_bytes(ara_pool pool) { return pool ? pool->bytes : 0; }

int32_t ara_pool_free_slots(ara_pool pool) {
    if (!pool) return -1;
    std::lock_guard<std::mutex> g(pool->mu);
    return (int32_t)pool->free_slots.size();
}

ara_status ara_create_layer_from_pool(ara_pool pool, int32_t n_elts, const int32_t *h_elt_index, const double *h_ret,
                                      const double *h_lim, double occ_ret, double occ_lim, double agg_ret,
                                      double agg_lim, void *hip_stream, ara_layer *out) {
    if (!out) return fail(ARA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!pool || !h_elt_index || !h_ret || !h_lim) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (n_elts < 1) return fail(ARA_ERR_INVALID_ARG, "n_elts < 1");
    if (n_elts > ARA_MAX_ELTS) return fail(ARA_ERR_UNSUPPORTED, "n_elts exceeds ARA_MAX_ELTS");
    for (int j = 0; j < n_elts; ++j)
        if (h_elt_index[j] < 0 || h_elt_index[j] >= pool->n_elts) return fail(ARA_ERR_INVALID_ARG, "ELT index outside the pool");
    ara_status st = validate_terms(n_elts, h_ret, h_lim, occ_ret, occ_lim, agg_ret, agg_lim);
    if (st != ARA_OK) return st;
    int slot = -1;
    {
        std::lock_guard<std::mutex> g(pool->mu);
        if (pool->free_slots.empty()) return fail(ARA_ERR_OOM, "no free layer slot in the pool");
        slot = pool->free_slots.back();
        pool->free_slots.pop_back();
    }
    ara_layer_s *L = new (std::nothrow) ara_layer_s;
    if (!L) {
        std::lock_guard<std::mutex> g(pool->mu);
        pool->free_slots.push_back(slot);
        return fail(ARA_ERR_OOM, "host allocation");
    }
    L->pool = pool;
    L->slot = slot;
    L->ready = pool->ready[slot];
    L->device = pool->device;
    ara::LayerHost &h = L->h;
    h.n_elts = n_elts;
    h.catalog = pool->catalog;
    h.precision = pool->precision;
    h.layout = ara::kFused;
    h.tab.catalog = pool->catalog;
    h.tab.occ = pool->occ[slot];
    h.tab.filt = static_cast<const uint32_t *>(pool->filt[slot]);
    h.tab.fshift = pool->fshift;
    h.tab.n_fwords = pool->n_fwords;
    h.tab.n_hwords = pool->n_hwords;
    h.tab.hshift = pool->hshift;
    h.bytes = pool->slot_bytes;
    set_terms(h, n_elts, h_ret, h_lim, occ_ret, occ_lim, agg_ret, agg_lim);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = ara::launch_fused_build(h, static_cast<const int32_t *>(pool->d_ids), pool->d_loss, false,
                                           pool->off.data(), h_elt_index, n_elts, nullptr, s);
    if (e == hipErrorNotSupported)
        e = ara::launch_pool_layer(h, static_cast<const int32_t *>(pool->d_ids), pool->d_loss, pool->off.data(),
                                   h_elt_index, n_elts, static_cast<float *>(pool->lo[slot]), s);
    if (e == hipSuccess) e = hipEventRecord(L->ready, s);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> g(pool->mu);
        pool->free_slots.push_back(slot);
        delete L;
        return hip_fail(e, "building the layer from the pool");
    }
    *out = L;
    return ARA_OK;
}

static void drop_graph(ara_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

static void free_batch(ara_batch b) {
    drop_graph(b);
    if (b->last_run) (void)hipEventDestroy(b->last_run);
    for (void *p : {b->d_rec, b->d_ovf_lid, b->d_ovf_val, (void *)b->d_ylts, (void *)b->d_agg, (void *)b->d_count,
                     (void *)b->d_ctr, b->d_dense, (void *)b->d_dfilt, (void *)b->d_ucount})
        if (p) (void)hipFree(p);
    delete b;
}

static ara_status check_batch_layers(int32_t catalog, const ara_layer *layers, int32_t n_layers, int32_t *prec,
                                     const void **occ) {
    if (!layers) return fail(ARA_ERR_INVALID_ARG, "NULL layers");
    if (n_layers < 1) return fail(ARA_ERR_INVALID_ARG, "n_layers < 1");
    if (n_layers > ARA_MAX_BATCH) return fail(ARA_ERR_UNSUPPORTED, "n_layers exceeds ARA_MAX_BATCH");
    for (int l = 0; l < n_layers; ++l) {
        if (!layers[l]) return fail(ARA_ERR_INVALID_ARG, "NULL layer handle");
        const ara::LayerHost &h = layers[l]->h;
        if (h.catalog != catalog) return fail(ARA_ERR_INVALID_ARG, "layer built for another catalogue");
        if (h.layout != ara::kFused) return fail(ARA_ERR_UNSUPPORTED, "batched layers must use the fused layout");
        if (*prec >= 0 && h.precision != *prec) return fail(ARA_ERR_INVALID_ARG, "layers of different precisions");
        *prec = h.precision;
        occ[l] = h.tab.occ;
    }
    return ARA_OK;
}

namespace {

// Sub-tables of the dense form: sub-table s takes layers
// [kDenseWidth s, kDenseWidth s + width), records of the next power of two
// of its width.
int dense_subs(int32_t n) { return (n + ara::kDenseWidth - 1) / ara::kDenseWidth; }

ara::DenseTables dense_tables(ara_batch b, int sub) {
    const int first = sub * ara::kDenseWidth;
    const int cnt = b->n - first < ara::kDenseWidth ? b->n - first : ara::kDenseWidth;
    int nl = 1;
    while (nl < cnt) nl <<= 1;
    ara::DenseTables t{};
    t.rec = static_cast<const char *>(b->d_dense) + (size_t)sub * b->dense_stride;
    t.filt = b->d_dfilt + (size_t)sub * (size_t)(b->n_fwords + b->n_hwords);
    t.n_fwords = b->n_fwords;
    t.fshift = b->fshift;
    t.n_hwords = b->n_hwords;
    t.hshift = b->hshift;
    t.catalog = b->catalog;
    t.nl = nl;
    t.ylts = b->d_ylts + first;
    t.agg_ret = b->d_agg + first;
    t.agg_lim = b->d_agg + ARA_MAX_BATCH + first;
    t.n_layers = cnt;
    return t;
}

// Dense records and filters of up to ara::kDenseMax layers (on s, after the
// waits the caller queued).  Sets b->n to n_layers (the sub-table geometry
// follows from it) and *union_frac to the sum over sub-tables of the
// fraction of catalogue events with any non-zero value (the events whose
// record a dense pass gathers).
ara_status rebuild_dense(ara_batch b, const void *const *occ, int32_t n_layers, bool fp64, hipStream_t s,
                         double *union_frac) {
    const int subs = dense_subs(n_layers);
    const size_t val_bytes = fp64 ? 8 : 4;
    const size_t stride = (((size_t)b->catalog + 1) * ara::kDenseWidth * val_bytes + 255) & ~(size_t)255;
    const size_t need = stride * (size_t)subs;
    const size_t fwords = (size_t)(b->n_fwords + b->n_hwords);
    hipError_t e = hipSuccess;
    if (need > b->dense_cap || subs > b->dfilt_subs) {
        // grows only; the wait for the last run is queued on s, so finish it
        // before the frees
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "waiting for the batch's last run");
    }
    if (subs > b->dfilt_subs) {
        if (b->d_dfilt) (void)hipFree(b->d_dfilt);
        b->bytes -= (size_t)b->dfilt_subs * fwords * sizeof(uint32_t);
        b->d_dfilt = nullptr;
        b->dfilt_subs = 0;
        e = dev_alloc(reinterpret_cast<void **>(&b->d_dfilt), (size_t)subs * fwords * sizeof(uint32_t));
        if (e != hipSuccess) {
            b->d_dfilt = nullptr;
            return hip_fail(e, "batch filter allocation");
        }
        b->dfilt_subs = subs;
        b->bytes += (size_t)subs * fwords * sizeof(uint32_t);
    }
    if (need > b->dense_cap) {
        if (b->d_dense) (void)hipFree(b->d_dense);
        b->bytes -= b->dense_cap;
        b->d_dense = nullptr;
        b->dense_cap = 0;
        e = dev_alloc(&b->d_dense, need);
        if (e != hipSuccess) {
            b->d_dense = nullptr;
            return hip_fail(e, "batch record allocation");
        }
        b->dense_cap = need;
        b->bytes += need;
    }
    b->dense_stride = stride;
    b->n = n_layers;
    const size_t ucount_bytes = sizeof(unsigned long long) * (ara::kDenseMax / ara::kDenseWidth);
    e = hipMemsetAsync(b->d_ucount, 0, ucount_bytes, s);
    for (int sub = 0; sub < subs && e == hipSuccess; ++sub) {
        const ara::DenseTables t = dense_tables(b, sub);
        e = ara::launch_dense_fill(occ + sub * ara::kDenseWidth, t.n_layers, fp64, t, b->d_ucount + sub, s);
    }
    unsigned long long cnt[ara::kDenseMax / ara::kDenseWidth] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, b->d_ucount, ucount_bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "building the batch records");
    double f = 0.0;
    for (int sub = 0; sub < subs; ++sub) f += (double)cnt[sub] / (double)b->catalog;
    *union_frac = f;
    return ARA_OK;
}

// Whether the dense form is expected to beat the sparse one.  Per trial-
// event the sparse pass fills one 64-byte record line (most catalogue
// events are non-zero in some layer of a large batch), the dense passes
// fill one 32-byte record line per sub-table whose union holds the event,
// and each dense pass streams the YET once.  Measured on MI355X over 1M
// Poisson(1000) trials: a dense record gather costs 0.42 of a sparse one,
// and a pass's YET stream 0.03 of the sparse pass.
bool dense_wins(double union_frac, int subs) { return 0.42 * union_frac + 0.03 * subs < 1.0; }

// Sparse records (on s, after the waits the caller queued).
ara_status rebuild_sparse(ara_batch b, const void *const *occ, int32_t n_layers, bool fp64, hipStream_t s) {
    const size_t val_bytes = fp64 ? 8 : 4;
    const size_t C = (size_t)b->catalog;
    hipError_t e = hipSuccess;
    if (!b->d_rec) {
        const size_t rec_bytes = fp64 ? 64 : 32;
        e = dev_alloc(&b->d_rec, C * rec_bytes);
        if (e == hipSuccess) e = dev_alloc(reinterpret_cast<void **>(&b->d_count), C * sizeof(int32_t));
        if (e == hipSuccess) e = dev_alloc(reinterpret_cast<void **>(&b->d_ctr), 2 * sizeof(unsigned long long));
        if (e != hipSuccess) {
            for (void **p : {&b->d_rec, reinterpret_cast<void **>(&b->d_count), reinterpret_cast<void **>(&b->d_ctr)}) {
                if (*p) (void)hipFree(*p);
                *p = nullptr;
            }
            return hip_fail(e, "batch record allocation");
        }
        b->bytes += C * (rec_bytes + sizeof(int32_t)) + 16;
    }
    unsigned long long h_ctr[2] = {0, 0};
    e = hipMemcpyAsync(b->d_ctr, h_ctr, sizeof(h_ctr), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = ara::launch_batch_count(occ, n_layers, b->catalog, fp64, b->d_count, b->d_ctr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_ctr, b->d_ctr, sizeof(h_ctr), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "counting the batch records");
    // at least one block of four overflow slots: the passes prefetch
    // overflow entries of every event at clamped indices, block 0 for
    // events without any
    const unsigned long long n_ovf = h_ctr[0] > 4 ? h_ctr[0] : 4;
    if (n_ovf >= (1ULL << 32)) return fail(ARA_ERR_UNSUPPORTED, "too many overflow entries for one batch");
    if (n_ovf > b->ovf_cap) {
        // grows only; the stream is idle here, the last run finished
        if (b->d_ovf_lid) (void)hipFree(b->d_ovf_lid);
        if (b->d_ovf_val) (void)hipFree(b->d_ovf_val);
        b->d_ovf_lid = b->d_ovf_val = nullptr;
        b->bytes -= (size_t)b->ovf_cap * (1 + val_bytes);
        b->ovf_cap = 0;
        e = dev_alloc(&b->d_ovf_lid, (size_t)n_ovf);
        if (e == hipSuccess) e = dev_alloc(&b->d_ovf_val, (size_t)n_ovf * val_bytes);
        if (e != hipSuccess) return hip_fail(e, "batch overflow area");
        b->ovf_cap = n_ovf;
        b->bytes += (size_t)n_ovf * (1 + val_bytes);
    }
    e = ara::launch_batch_fill(occ, n_layers, b->catalog, fp64, b->d_count, b->d_rec,
                               static_cast<uint8_t *>(b->d_ovf_lid), b->d_ovf_val, b->d_ctr + 1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "building the batch records");
    return ARA_OK;
}

}  // namespace

ara_status ara_batch_rebuild(ara_batch b, const ara_layer *layers, int32_t n_layers) {
    if (!b) return fail(ARA_ERR_INVALID_ARG, "NULL batch");
    const void *occ[ARA_MAX_BATCH];
    int32_t prec = b->precision;
    ara_status st = check_batch_layers(b->catalog, layers, n_layers, &prec, occ);
    if (st != ARA_OK) return st;
    const bool fp64 = prec == ARA_FP64;
    hipStream_t s = ara::internal_stream();
    if (!s) return fail(ARA_ERR_DEVICE, "no set-up stream");
    hipError_t e = hipSuccess;
    // everything below overwrites what the batch's last run reads: wait for it
    if (b->ran) e = hipStreamWaitEvent(s, b->last_run, 0);
    for (int l = 0; l < n_layers && e == hipSuccess; ++l)
        if (layers[l]->ready) e = hipStreamWaitEvent(s, layers[l]->ready, 0);
    std::vector<double> agg(2 * ARA_MAX_BATCH, 0.0);
    for (int l = 0; l < n_layers; ++l) {
        agg[l] = layers[l]->h.t64.agg_ret;
        agg[ARA_MAX_BATCH + l] = layers[l]->h.t64.agg_lim;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_agg, agg.data(), sizeof(double) * agg.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "batch terms");
    bool dense = n_layers <= ara::kDenseMax;
    const int32_t n_before = b->n;
    b->valid = false;
    if (dense) {
        double union_frac = 0.0;
        st = rebuild_dense(b, occ, n_layers, fp64, s, &union_frac);
        // layers whose non-zero events cover most of the catalogue: the
        // sparse records instead
        if (st == ARA_OK && !dense_wins(union_frac, dense_subs(n_layers))) dense = false;
    }
    if (!dense) st = rebuild_sparse(b, occ, n_layers, fp64, s);
    b->n = n_before;
    if (st != ARA_OK) return st;
    if (n_layers != b->n || dense != b->dense) {
        // a batch whose size changes (a server's) launches directly from now
        // on instead of capturing a graph per size
        drop_graph(b);
        b->tuned = false;
        b->dgroup[0] = b->dgroup[1] = b->dgroup[2] = 0;
        b->use_graph = b->n == 0;
        b->n = n_layers;
        b->dense = dense;
    }
    b->h_ylts.assign(n_layers, nullptr);
    b->valid = true;
    return ARA_OK;
}

ara_status ara_create_batch(ara_yet yet, const ara_layer *layers, int32_t n_layers, ara_batch *out) {
    if (!out) return fail(ARA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!yet) return fail(ARA_ERR_INVALID_ARG, "NULL yet");
    const void *occ[ARA_MAX_BATCH];
    int32_t prec = -1;
    ara_status st = check_batch_layers(yet->catalog, layers, n_layers, &prec, occ);
    if (st != ARA_OK) return st;
    ara_batch_s *b = new (std::nothrow) ara_batch_s;
    if (!b) return fail(ARA_ERR_OOM, "host allocation");
    b->yv = yet->v;
    b->precision = prec;
    b->catalog = yet->catalog;
    (void)hipGetDevice(&b->device);
    ara::filter_geometry(yet->catalog, b->fshift, b->n_fwords, b->n_hwords, b->hshift);
    hipError_t e = hipEventCreateWithFlags(&b->last_run, hipEventDisableTiming);
    if (e != hipSuccess) b->last_run = nullptr;
    if (e == hipSuccess) e = dev_alloc(reinterpret_cast<void **>(&b->d_ylts), sizeof(double *) * ARA_MAX_BATCH);
    if (e == hipSuccess) e = dev_alloc(reinterpret_cast<void **>(&b->d_agg), sizeof(double) * 2 * ARA_MAX_BATCH);
    if (e == hipSuccess)
        e = dev_alloc(reinterpret_cast<void **>(&b->d_ucount),
                      sizeof(unsigned long long) * (ara::kDenseMax / ara::kDenseWidth));
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "batch allocation");
    }
    b->bytes = (sizeof(double *) + 2 * sizeof(double)) * ARA_MAX_BATCH;
    st = ara_batch_rebuild(b, layers, n_layers);
    if (st != ARA_OK) {
        free_batch(b);
        return st;
    }
    *out = b;
    return ARA_OK;
}

void ara_destroy_batch(ara_batch batch) {
    if (!batch) return;
    (void)hipDeviceSynchronize();
    free_batch(batch);
}

size_t ara_batch_device_bytes(ara_batch batch) { return batch ? batch->bytes : 0; }

namespace {

ara::BatchTables batch_tables(ara_batch b) {
    ara::BatchTables t{};
    t.rec = b->d_rec;
    t.ovf_lid = static_cast<const uint8_t *>(b->d_ovf_lid);
    t.ovf_val = b->d_ovf_val;
    t.ylts = b->d_ylts;
    t.agg_ret = b->d_agg;
    t.agg_lim = b->d_agg + ARA_MAX_BATCH;
    t.n_layers = b->n;
    return t;
}

// Launch shapes are chosen by timing the real pass once per (precision,
// layers, trial count, YET form) and remembered for the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t, int, int>, ara::BatchLaunch> g_tuned;

hipError_t tune_batch(ara_batch b, hipStream_t s) {
    const bool fp64 = b->precision == ARA_FP64;
    const int form = b->yv.offsets ? 1 : 0;
    int n_bucket = 1;  // layer counts share a tuned shape per power of two
    while (n_bucket < b->n) n_bucket <<= 1;
    const auto key = std::make_tuple(b->precision, n_bucket, b->yv.n_trials, form, (int)b->yv.aligned16);
    // "threads,wg_per_cu[,group]" skips the search (and is not remembered)
    const char *force = std::getenv("ARA_BATCH_LAUNCH");
    if (!force) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            // the shape was tuned for another layer count of the bucket: the
            // per-wave accumulators grow with the count, so narrow the
            // work-group until they fit the LDS
            ara::BatchLaunch c = it->second;
            while (c.threads > ara::kWave && ara::batch_lds_bytes(b->n, c.threads) > 160u * 1024u)
                c.threads -= ara::kWave;
            b->cfg = c;
            b->tuned = true;
            return hipSuccess;
        }
    }
    std::vector<ara::BatchLaunch> cands;
    if (force) {
        int t = 256, w = 1, g = 4;
        const int got = std::sscanf(force, "%d,%d,%d", &t, &w, &g);
        if (got >= 2 && t >= 64 && t <= (g == 1 ? ara::kMaxStreamThreads : 512) && t % 64 == 0 && w >= 1 &&
            (g == 1 || g == 2 || g == 4 || g == 8)) {
            while (t > ara::kWave && ara::batch_lds_bytes(b->n, t) > 160u * 1024u) t -= ara::kWave;
            cands.push_back({t, w, g});
        }
    }
    if (cands.empty())
        for (int g : {1, 2, 4, 8})
            for (int t : {256, 512})
                for (int w : {1, 2, 4})
                    if ((g != 1 || t <= ara::kMaxStreamThreads) &&
                        ara::batch_lds_bytes(b->n, t) * (size_t)w <= 160u * 1024u)
                        cands.push_back({t, w, g});
    if (cands.empty()) cands.push_back({64, 1, 4});
    const ara::BatchTables tb = batch_tables(b);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    ara::BatchLaunch best_cfg = cands[0];
    for (const auto &c : cands) {
        if (e != hipSuccess) break;
        if (cands.size() > 1) e = ara::launch_batch_pass(b->yv, tb, fp64, c, s);  // warm-up
        float tot = 0.0f;
        for (int rep = 0; rep < 2 && e == hipSuccess && cands.size() > 1; ++rep) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = ara::launch_batch_pass(b->yv, tb, fp64, c, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            tot += ms;
        }
        if (e == hipSuccess && tot < best) {
            best = tot;
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    b->cfg = best_cfg;
    b->tuned = true;
    if (cands.size() > 1) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[key] = best_cfg;
    }
    return hipSuccess;
}

int nl_index(int nl) { return nl == 1 ? 0 : (nl == 2 ? 1 : 2); }

// One launch of the batch's pass in its current form.
hipError_t pass_once(ara_batch b, hipStream_t s) {
    const bool fp64 = b->precision == ARA_FP64;
    if (b->dense) {
        hipError_t e = hipSuccess;
        for (int sub = 0; sub < dense_subs(b->n) && e == hipSuccess; ++sub) {
            const ara::DenseTables t = dense_tables(b, sub);
            e = ara::launch_dense_pass(b->yv, t, fp64, b->dgroup[nl_index(t.nl)], s);
        }
        return e;
    }
    return ara::launch_batch_pass(b->yv, batch_tables(b), fp64, b->cfg, s);
}

// Chunk-group size of the dense pass per record width, chosen by timing the
// candidates on the batch's first sub-table of that width, remembered per
// (precision, width, trial count, YET form) for the process.
std::map<std::tuple<int, int, int64_t, int, int>, int> g_dense_tuned;

hipError_t tune_dense(ara_batch b, hipStream_t s) {
    const bool fp64 = b->precision == ARA_FP64;
    const int form = b->yv.offsets ? 1 : 0;
    for (int sub = 0; sub < dense_subs(b->n); ++sub) {
        const ara::DenseTables t = dense_tables(b, sub);
        const int ix = nl_index(t.nl);
        if (b->dgroup[ix]) continue;
        const auto key = std::make_tuple(b->precision, t.nl, b->yv.n_trials, form, (int)b->yv.aligned16);
        {
            std::lock_guard<std::mutex> g(g_tune_mu);
            auto it = g_dense_tuned.find(key);
            if (it != g_dense_tuned.end()) {
                b->dgroup[ix] = it->second;
                continue;
            }
        }
        std::vector<int> cands = t.nl >= 4 ? std::vector<int>{2} : std::vector<int>{2, 4};
        int best = cands[0];
        if (cands.size() > 1) {
            hipEvent_t e0, e1;
            hipError_t e = hipEventCreate(&e0);
            if (e == hipSuccess) e = hipEventCreate(&e1);
            float best_ms = 1e30f;
            for (int g : cands) {
                if (e != hipSuccess) break;
                e = ara::launch_dense_pass(b->yv, t, fp64, g, s);  // warm-up
                float tot = 0.0f;
                for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                    e = hipEventRecord(e0, s);
                    if (e == hipSuccess) e = ara::launch_dense_pass(b->yv, t, fp64, g, s);
                    if (e == hipSuccess) e = hipEventRecord(e1, s);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.0f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    tot += ms;
                }
                if (e == hipSuccess && tot < best_ms) {
                    best_ms = tot;
                    best = g;
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (e != hipSuccess) return e;
        }
        b->dgroup[ix] = best;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_dense_tuned[key] = best;
    }
    return hipSuccess;
}

constexpr int kMaxCaptureFailures = 3;

hipError_t capture_batch(ara_batch b) {
    if (fault_capture()) return hipErrorStreamCaptureInvalidated;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = pass_once(b, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e == hipSuccess) {
            b->graph = g;
            b->graph_dense = b->dense;
            b->graph_tables = batch_tables(b);
            b->graph_drec = b->d_dense;
            b->graph_dfilt = b->d_dfilt;
            b->graph_cfg = b->cfg;
        } else {
            b->exec = nullptr;
            if (g) (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    return e;
}

// The captured graph holds the table pointers, the layer count and the launch
// shape as kernel arguments; a rebuild may have reallocated the overflow
// arrays, so the graph is replayed only while they are unchanged.
bool graph_current(const ara_batch b) {
    if (!b->exec || b->dense != b->graph_dense) return false;
    if (b->dense)  // the layer count is the graph's whenever the graph exists
        return b->d_dense == b->graph_drec && b->d_dfilt == b->graph_dfilt && b->n == b->graph_tables.n_layers;
    const ara::BatchTables now = batch_tables(b);
    const ara::BatchTables &was = b->graph_tables;
    return now.rec == was.rec && now.ovf_lid == was.ovf_lid && now.ovf_val == was.ovf_val &&
           now.ylts == was.ylts && now.agg_ret == was.agg_ret && now.agg_lim == was.agg_lim &&
           now.n_layers == was.n_layers && b->cfg.threads == b->graph_cfg.threads &&
           b->cfg.wg_per_cu == b->graph_cfg.wg_per_cu && b->cfg.group == b->graph_cfg.group;
}

// Launch the pass (graph replay or direct launch) and record the batch's
// last-run event after it.
ara_status launch_batch(ara_batch batch, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (!batch->use_graph) {
        e = pass_once(batch, s);
        if (e != hipSuccess) return hip_fail(e, "batch launch");
    } else {
        if (batch->exec && !graph_current(batch)) drop_graph(batch);
        if (!batch->exec) {
            e = capture_batch(batch);
            if (e != hipSuccess) {
                // A capture can fail for reasons outside the batch (it can be
                // invalidated from outside, e.g. by a synchronizing call --
                // a free, an allocation -- that another host thread makes
                // meanwhile).  The pass then runs as a direct launch, the same kernels with the
                // same arguments, and the next run captures again; after
                // kMaxCaptureFailures failures in a row the batch stops trying.
                (void)hipGetLastError();
                if (++batch->capture_failures >= kMaxCaptureFailures) batch->use_graph = false;
                e = pass_once(batch, s);
                if (e != hipSuccess) return hip_fail(e, "batch launch after a failed graph capture");
                return ARA_OK;
            }
            batch->capture_failures = 0;
        }
        e = hipGraphLaunch(batch->exec, s);
        if (e != hipSuccess) return hip_fail(e, "batch graph launch");
    }
    return ARA_OK;
}

}  // namespace

ara_status ara_run_batch(ara_batch batch, double *const *d_ylts, void *hip_stream) {
    if (!batch || !d_ylts) return fail(ARA_ERR_INVALID_ARG, "NULL batch or d_ylts");
    if (!batch->valid) return fail(ARA_ERR_INVALID_ARG, "the batch's last rebuild failed; rebuild it first");
    for (int l = 0; l < batch->n; ++l)
        if (!d_ylts[l] && batch->yv.n_trials > 0) return fail(ARA_ERR_INVALID_ARG, "NULL YLT pointer");
    if (batch->yv.n_trials == 0) return ARA_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipSuccess;
    // a run on another stream than the last one waits for the last run: it
    // may overwrite the YLT pointers that run reads
    if (batch->ran && s != batch->last_stream) {
        e = hipStreamWaitEvent(s, batch->last_run, 0);
        if (e != hipSuccess) return hip_fail(e, "ordering after the batch's last run");
    }
    if (!std::equal(batch->h_ylts.begin(), batch->h_ylts.end(), d_ylts)) {
        for (int l = 0; l < batch->n; ++l) batch->h_ylts[l] = d_ylts[l];
        e = hipMemcpyAsync(batch->d_ylts, batch->h_ylts.data(), sizeof(double *) * batch->n, hipMemcpyHostToDevice,
                           s);
        if (e != hipSuccess) return hip_fail(e, "copy of the YLT pointers");
    }
    if (batch->yv.n_events == 0) {
        // every trial is empty, and an empty trial's year loss is
        // min(max(0 - FT3_1, 0), FT3_2) = 0 since FT3_1 >= 0
        for (int l = 0; l < batch->n && e == hipSuccess; ++l)
            e = ara::launch_fill_zero(d_ylts[l], batch->yv.n_trials, s);
        if (e != hipSuccess) return hip_fail(e, "zero YLTs");
    } else {
        if (!batch->tuned) {
            e = batch->dense ? tune_dense(batch, s) : tune_batch(batch, s);
            if (e != hipSuccess) return hip_fail(e, "batch launch tuning");
            batch->tuned = true;
        }
        ara_status st = launch_batch(batch, s);
        if (st != ARA_OK) return st;
    }
    e = hipEventRecord(batch->last_run, s);
    if (e != hipSuccess) return hip_fail(e, "recording the batch's run");
    batch->ran = true;
    batch->last_stream = s;
    return ARA_OK;
}

ara_status ara_batch_launch_config(ara_batch batch, int32_t *threads, int32_t *wg_per_cu) {
    if (!batch || !threads || !wg_per_cu) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (batch->dense) {
        // 1024-thread groups, the LDS filters allow one per CU
        *threads = batch->tuned ? 1024 : 0;
        *wg_per_cu = batch->tuned ? 1 : 0;
        return ARA_OK;
    }
    *threads = batch->tuned ? batch->cfg.threads : 0;
    *wg_per_cu = batch->tuned ? batch->cfg.wg_per_cu : 0;
    return ARA_OK;
}

ara_status ara_batch_launch_group(ara_batch batch, int32_t *group) {
    if (!batch || !group) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (!batch->tuned) {
        *group = 0;
    } else if (batch->dense) {
        *group = batch->dgroup[nl_index(dense_tables(batch, 0).nl)];
    } else {
        *group = batch->cfg.group;
    }
    return ARA_OK;
}

ara_status ara_run_layers(ara_yet yet, const ara_layer *layers, double *const *d_ylts, int32_t n_layers,
                          void *hip_stream) {
    ara_batch b = nullptr;
    ara_status st = ara_create_batch(yet, layers, n_layers, &b);
    if (st != ARA_OK) return st;
    st = ara_run_batch(b, d_ylts, hip_stream);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
    ara_destroy_batch(b);
    if (st != ARA_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "batched pass");
    return ARA_OK;
}

ara_status ara_rollup(const double *const *d_ylts, int32_t n_inputs, const int32_t *h_group, int32_t n_groups,
                      int64_t n_trials, double *const *d_out, void *hip_stream) {
    if (!d_ylts || !h_group || !d_out) return fail(ARA_ERR_INVALID_ARG, "NULL pointer");
    if (n_inputs < 1 || n_inputs > ARA_MAX_BATCH) return fail(ARA_ERR_INVALID_ARG, "n_inputs outside 1 .. ARA_MAX_BATCH");
    if (n_groups < 1 || n_groups > ARA_MAX_BATCH) return fail(ARA_ERR_INVALID_ARG, "n_groups outside 1 .. ARA_MAX_BATCH");
    if (n_trials < 0 || n_trials > 2147483647LL) return fail(ARA_ERR_INVALID_ARG, "n_trials outside 0 .. 2^31-1");
    for (int l = 0; l < n_inputs; ++l) {
        if (!d_ylts[l] && n_trials > 0) return fail(ARA_ERR_INVALID_ARG, "NULL input table");
        if (h_group[l] < 0 || h_group[l] >= n_groups) return fail(ARA_ERR_INVALID_ARG, "group index outside 0 .. n_groups-1");
    }
    for (int g = 0; g < n_groups; ++g)
        if (!d_out[g] && n_trials > 0) return fail(ARA_ERR_INVALID_ARG, "NULL output table");
    if (n_trials == 0) return ARA_OK;
    // no output may share a byte with an input or with another output
    const uintptr_t bytes = (uintptr_t)n_trials * sizeof(double);
    auto overlap = [bytes](const void *a, const void *b) {
        const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
        return bytes > 0 && x < y + bytes && y < x + bytes;
    };
    for (int g = 0; g < n_groups; ++g) {
        for (int l = 0; l < n_inputs; ++l)
            if (overlap(d_out[g], d_ylts[l])) return fail(ARA_ERR_INVALID_ARG, "an output table overlaps an input");
        for (int h = 0; h < g; ++h)
            if (overlap(d_out[g], d_out[h])) return fail(ARA_ERR_INVALID_ARG, "two output tables overlap");
    }
    // inputs ordered by group, each group's in increasing input index
    ara::RollupTables a{};
    a.n_groups = n_groups;
    int q = 0;
    for (int g = 0; g < n_groups; ++g) {
        a.first[g] = q;
        a.out[g] = d_out[g];
        for (int l = 0; l < n_inputs; ++l)
            if (h_group[l] == g) a.in[q++] = d_ylts[l];
    }
    a.first[n_groups] = q;
    hipError_t e = ara::launch_rollup(a, n_trials, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "roll-up");
    return ARA_OK;
}

static ara_status tail_sizes(int64_t n_trials, const double *h_return_periods, int32_t n_rp, int64_t *k) {
    if (n_trials < 1 || n_trials > 2147483647LL) return fail(ARA_ERR_INVALID_ARG, "n_trials outside 1 .. 2^31-1");
    if (n_rp < 1 || n_rp > 16) return fail(ARA_ERR_INVALID_ARG, "n_rp outside 1 .. 16");
    for (int r = 0; r < n_rp; ++r) {
        const double N = h_return_periods[r];
        if (!(N > 0.0) || !std::isfinite(N)) return fail(ARA_ERR_INVALID_ARG, "return period must be finite and > 0");
        const double kk = std::floor((double)n_trials / N);
        if (kk < 1.0) return fail(ARA_ERR_RP, "return period leaves no tail trial (floor(T/N) < 1)");
        if (kk > (double)n_trials) return fail(ARA_ERR_RP, "return period shorter than one year (floor(T/N) > T)");
        k[r] = (int64_t)kk;
    }
    return ARA_OK;
}

ara_status ara_pml_tvar(const double *d_ylt, int64_t n_trials, const double *h_return_periods, int32_t n_rp,
                        double *h_pml, double *h_tvar, void *hip_stream) {
    if (!d_ylt || !h_return_periods || !h_pml || !h_tvar) return fail(ARA_ERR_INVALID_ARG, "NULL pointer");
    return ara_pml_tvar_many(&d_ylt, 1, n_trials, h_return_periods, n_rp, h_pml, h_tvar, hip_stream);
}

ara_status ara_pml_tvar_many(const double *const *d_ylts, int32_t n_ylts, int64_t n_trials,
                             const double *h_return_periods, int32_t n_rp, double *h_pml, double *h_tvar,
                             void *hip_stream) {
    if (!d_ylts || !h_return_periods || !h_pml || !h_tvar) return fail(ARA_ERR_INVALID_ARG, "NULL pointer");
    if (n_ylts < 1 || n_ylts > ARA_MAX_BATCH) return fail(ARA_ERR_INVALID_ARG, "n_ylts outside 1 .. ARA_MAX_BATCH");
    for (int i = 0; i < n_ylts; ++i)
        if (!d_ylts[i]) return fail(ARA_ERR_INVALID_ARG, "NULL YLT pointer");
    int64_t k[16];
    ara_status st = tail_sizes(n_trials, h_return_periods, n_rp, k);
    if (st != ARA_OK) return st;
    std::vector<double> out(2 * (size_t)n_ylts * n_rp);
    int32_t nan = 0;
    hipError_t e = ara::pml_tvar_device(d_ylts, n_ylts, n_trials, k, n_rp, out.data(), &nan,
                                        static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "PML/TVaR");
    if (nan) return fail(ARA_ERR_VALUE, "a YLT holds NaN");
    for (int i = 0; i < n_ylts * n_rp; ++i) {
        h_pml[i] = out[2 * i];
        h_tvar[i] = out[2 * i + 1];
    }
    return ARA_OK;
}

ara_status ara_pml_tvar_many_noalloc(const double *const *d_ylts, int32_t n_ylts, int64_t n_trials,
                                     const double *h_return_periods, int32_t n_rp, double *d_pml, double *d_tvar,
                                     void *hip_stream) {
    if (!d_ylts || !h_return_periods || !d_pml || !d_tvar) return fail(ARA_ERR_INVALID_ARG, "NULL pointer");
    if (n_ylts < 1 || n_ylts > ARA_MAX_BATCH) return fail(ARA_ERR_INVALID_ARG, "n_ylts outside 1 .. ARA_MAX_BATCH");
    for (int i = 0; i < n_ylts; ++i)
        if (!d_ylts[i]) return fail(ARA_ERR_INVALID_ARG, "NULL YLT pointer");
    int64_t k[16];
    ara_status st = tail_sizes(n_trials, h_return_periods, n_rp, k);
    if (st != ARA_OK) return st;
    if (n_ylts * n_rp > ARA_NOALLOC_MAX_SEL)
        return fail(ARA_ERR_UNSUPPORTED, "n_ylts * n_rp exceeds ARA_NOALLOC_MAX_SEL (the size of the static scratch)");
    hipError_t e = ara::pml_tvar_noalloc(d_ylts, n_ylts, n_trials, k, n_rp, d_pml, d_tvar,
                                         static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "PML/TVaR (no allocation)");
    return ARA_OK;
}

}  // extern "C"
