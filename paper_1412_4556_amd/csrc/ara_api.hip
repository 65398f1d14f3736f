// C ABI of libara: argument checks, layer table construction, handles and
// errors.  The operations themselves run in the HIP kernels of
// ara_kernels.hip and ara_select.hip.
#include <algorithm>
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

struct ara_layer_s {
    ara::LayerHost h;
    int device = 0;
};

struct ara_batch_s {
    ara::YetView yv{};
    int32_t n = 0;
    int32_t precision = 0;
    int32_t catalog = 0;
    void *d_rec = nullptr;
    void *d_ovf_lid = nullptr;
    void *d_ovf_val = nullptr;
    double **d_ylts = nullptr;  // device array of the YLT pointers of the last run
    double *d_agg = nullptr;    // [2n]: aggregate retentions, then limits
    std::vector<double *> h_ylts;
    ara::BatchLaunch cfg{256, 1};
    bool tuned = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t bytes = 0;
    int device = 0;
};

namespace {

thread_local std::string g_err;

ara_status fail(ara_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

ara_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? ARA_ERR_OOM : ARA_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
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
long long g_alloc_count = 0;

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

void release_slot(ara::LayerHost &h, int slot, size_t bytes) {
    if (h.alloc[slot]) {
        (void)hipFree(h.alloc[slot]);
        h.alloc[slot] = nullptr;
        h.bytes -= bytes;
    }
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
        if (h.layout == ara::kCompact) {
            const void *d0, *d1;
            if ((st = upload(h, 0, bm.data(), bm.size(), &d0)) != ARA_OK) return st;
            if ((st = upload(h, 1, rows.data(), rows.size(), &d1)) != ARA_OK) return st;
            h.tab.bm = static_cast<const uint2 *>(d0);
            h.tab.rows = d1;
            h.tab.n_words = (int32_t)n_words;
        } else {
            // fused: occurrence loss per catalogue event and the LDS filter
            std::vector<int32_t> present;
            present.reserve(rank);
            for (int64_t w = 0; w < n_words; ++w)
                for (uint32_t x = bm[w].x; x; x &= x - 1u) present.push_back((int32_t)(w * 32 + __builtin_ctz(x)));
            int32_t fshift = 0;
            while ((((int64_t)C + (1LL << fshift) - 1) >> fshift) > ara::kFilterBits) ++fshift;
            const int64_t n_blocks = ((int64_t)C + (1LL << fshift) - 1) >> fshift;
            const int64_t n_fwords = (n_blocks + 31) / 32;
            const void *d_rows, *d_present;
            if ((st = upload(h, 0, rows.data(), rows.size(), &d_rows)) != ARA_OK) return st;
            if ((st = upload(h, 1, present.data(), present.size(), &d_present)) != ARA_OK) return st;
            void *d_occ = nullptr, *d_filt = nullptr;
            // catalogue + 1 entries: occ[C] stays 0 for the pass's unmarked lanes
            hipError_t e = dev_alloc(&d_occ, ((size_t)C + 1) * sizeof(T));
            if (e != hipSuccess) return hip_fail(e, "device allocation of the fused table");
            h.alloc[2] = d_occ;
            h.bytes += ((size_t)C + 1) * sizeof(T);
            e = dev_alloc(&d_filt, (size_t)n_fwords * sizeof(uint32_t));
            if (e != hipSuccess) return hip_fail(e, "device allocation of the fused filter");
            h.alloc[3] = d_filt;
            h.bytes += (size_t)n_fwords * sizeof(uint32_t);
            h.tab.occ = d_occ;
            h.tab.filt = static_cast<const uint32_t *>(d_filt);
            h.tab.fshift = fshift;
            h.tab.n_fwords = (int32_t)n_fwords;
            hipStream_t s = ara::internal_stream();
            e = ara::launch_fuse(h, d_rows, static_cast<const int32_t *>(d_present), (int64_t)rank, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "building the fused table");
            release_slot(h, 0, rows.size() * sizeof(T));
            release_slot(h, 1, present.size() * sizeof(int32_t));
        }
    }
    return ARA_OK;
}

}  // namespace

extern "C" {

const char *ara_last_error(void) { return g_err.c_str(); }

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
    std::vector<int64_t> start(n_elts + 1, 0);
    for (int j = 0; j < n_elts; ++j) {
        if (h_elt_sizes[j] < 0) return fail(ARA_ERR_INVALID_ARG, "negative ELT size");
        if (h_elt_sizes[j] > C) return fail(ARA_ERR_DUP_EVENT, "ELT larger than the catalogue");
        start[j + 1] = start[j] + h_elt_sizes[j];
    }
    if (start[n_elts] > 0 && (!h_elt_ids || !h_elt_losses)) return fail(ARA_ERR_INVALID_ARG, "NULL ELT arrays");
    for (int j = 0; j < n_elts; ++j) {
        if (!finite_nonneg(h_ret[j])) return fail(ARA_ERR_VALUE, "ELT retention must be finite and >= 0");
        if (!limit_ok(h_lim[j])) return fail(ARA_ERR_VALUE, "ELT limit must be >= 0");
    }
    if (!finite_nonneg(occ_ret) || !limit_ok(occ_lim)) return fail(ARA_ERR_VALUE, "bad occurrence terms");
    if (!finite_nonneg(agg_ret) || !limit_ok(agg_lim)) return fail(ARA_ERR_VALUE, "bad aggregate terms");
    {
        std::vector<int32_t> stamp;
        try {
            stamp.assign((size_t)C, 0);
        } catch (const std::bad_alloc &) {
            return fail(ARA_ERR_OOM, "host allocation");
        }
        for (int j = 0; j < n_elts; ++j)
            for (int64_t n = start[j]; n < start[j + 1]; ++n) {
                int32_t e = h_elt_ids[n];
                if (e < 0 || e >= C) return fail(ARA_ERR_EVENT_RANGE, "ELT event ID outside [0, catalog_size)");
                if (stamp[e] == j + 1) return fail(ARA_ERR_DUP_EVENT, "duplicate event ID in one ELT");
                stamp[e] = j + 1;
                if (!finite_nonneg(h_elt_losses[n])) return fail(ARA_ERR_VALUE, "ELT loss must be finite and >= 0");
            }
    }

    ara_layer_s *L = new (std::nothrow) ara_layer_s;
    if (!L) return fail(ARA_ERR_OOM, "host allocation");
    ara::LayerHost &h = L->h;
    h.n_elts = n_elts;
    h.catalog = C;
    h.precision = precision;
    h.layout = layout == ARA_LAYOUT_AUTO ? ARA_LAYOUT_FUSED : layout;
    h.tab.catalog = C;
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
    hipError_t e = ara::launch_trial_pass(yet->v, layer->h, d_ylt, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "trial pass launch");
    return ARA_OK;
}

ara_status ara_run_layer_events(ara_yet yet, ara_layer layer, double *d_ylt, double *d_event_cum, double *d_event_net,
                                void *hip_stream) {
    if (!yet || !layer) return fail(ARA_ERR_INVALID_ARG, "NULL handle");
    if (layer->h.catalog != yet->catalog) return fail(ARA_ERR_INVALID_ARG, "layer built for another catalogue");
    if (yet->v.n_trials > 0 && !d_ylt) return fail(ARA_ERR_INVALID_ARG, "d_ylt is NULL");
    hipError_t e = ara::launch_trial_pass_events(yet->v, layer->h, d_ylt, d_event_cum, d_event_net,
                                                 static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "per-event trial pass launch");
    return ARA_OK;
}

static void free_batch(ara_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *p : {b->d_rec, b->d_ovf_lid, b->d_ovf_val, (void *)b->d_ylts, (void *)b->d_agg})
        if (p) (void)hipFree(p);
    delete b;
}

ara_status ara_create_batch(ara_yet yet, const ara_layer *layers, int32_t n_layers, ara_batch *out) {
    if (!out) return fail(ARA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!yet || !layers) return fail(ARA_ERR_INVALID_ARG, "NULL yet or layers");
    if (n_layers < 1) return fail(ARA_ERR_INVALID_ARG, "n_layers < 1");
    if (n_layers > ARA_MAX_BATCH) return fail(ARA_ERR_UNSUPPORTED, "n_layers exceeds ARA_MAX_BATCH");
    const void *occ[ARA_MAX_BATCH];
    int32_t prec = -1;
    for (int l = 0; l < n_layers; ++l) {
        if (!layers[l]) return fail(ARA_ERR_INVALID_ARG, "NULL layer handle");
        const ara::LayerHost &h = layers[l]->h;
        if (h.catalog != yet->catalog) return fail(ARA_ERR_INVALID_ARG, "layer built for another catalogue");
        if (h.layout != ara::kFused) return fail(ARA_ERR_UNSUPPORTED, "batched layers must use the fused layout");
        if (prec >= 0 && h.precision != prec) return fail(ARA_ERR_INVALID_ARG, "layers of different precisions");
        prec = h.precision;
        occ[l] = h.tab.occ;
    }
    ara_batch_s *b = new (std::nothrow) ara_batch_s;
    if (!b) return fail(ARA_ERR_OOM, "host allocation");
    b->yv = yet->v;
    b->n = n_layers;
    b->precision = prec;
    b->catalog = yet->catalog;
    (void)hipGetDevice(&b->device);
    const bool fp64 = prec == ARA_FP64;
    const size_t rec_bytes = fp64 ? 64 : 32, val_bytes = fp64 ? 8 : 4;
    const size_t C = (size_t)yet->catalog;
    hipStream_t s = ara::internal_stream();
    int32_t *d_count = nullptr;
    unsigned long long *d_ctr = nullptr;  // [0] overflow total, [1] fill cursor
    unsigned long long h_ctr[2] = {0, 0};
    hipError_t e = dev_alloc(reinterpret_cast<void **>(&d_count), C * sizeof(int32_t));
    if (e == hipSuccess) e = dev_alloc(reinterpret_cast<void **>(&d_ctr), sizeof(h_ctr));
    if (e == hipSuccess) e = hipMemcpyAsync(d_ctr, h_ctr, sizeof(h_ctr), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = ara::launch_batch_count(occ, n_layers, yet->catalog, fp64, d_count, d_ctr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_ctr, d_ctr, sizeof(h_ctr), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const unsigned long long n_ovf = h_ctr[0];
    if (e == hipSuccess && n_ovf >= (1ULL << 32)) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = dev_alloc(&b->d_rec, C * rec_bytes);
    if (e == hipSuccess) e = dev_alloc(&b->d_ovf_lid, (size_t)n_ovf);
    if (e == hipSuccess) e = dev_alloc(&b->d_ovf_val, (size_t)n_ovf * val_bytes);
    if (e == hipSuccess) e = dev_alloc(reinterpret_cast<void **>(&b->d_ylts), sizeof(double *) * n_layers);
    if (e == hipSuccess) e = dev_alloc(reinterpret_cast<void **>(&b->d_agg), sizeof(double) * 2 * n_layers);
    std::vector<double> agg(2 * n_layers);
    for (int l = 0; l < n_layers; ++l) {
        agg[l] = layers[l]->h.t64.agg_ret;
        agg[n_layers + l] = layers[l]->h.t64.agg_lim;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_agg, agg.data(), sizeof(double) * agg.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = ara::launch_batch_fill(occ, n_layers, yet->catalog, fp64, d_count, b->d_rec,
                                   static_cast<uint8_t *>(b->d_ovf_lid), b->d_ovf_val, d_ctr + 1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (d_count) (void)hipFree(d_count);
    if (d_ctr) (void)hipFree(d_ctr);
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "building the batch records");
    }
    b->bytes = C * rec_bytes + (size_t)n_ovf * (1 + val_bytes) + sizeof(double *) * n_layers +
               sizeof(double) * 2 * n_layers;
    b->h_ylts.assign(n_layers, nullptr);
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
    t.agg_lim = b->d_agg + b->n;
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
    const auto key = std::make_tuple(b->precision, b->n, b->yv.n_trials, form, (int)b->yv.aligned16);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            b->cfg = it->second;
            b->tuned = true;
            return hipSuccess;
        }
    }
    const char *force = std::getenv("ARA_BATCH_LAUNCH");  // "threads,wg_per_cu" skips the search
    std::vector<ara::BatchLaunch> cands;
    if (force) {
        int t = 256, w = 1;
        if (std::sscanf(force, "%d,%d", &t, &w) == 2 && t >= 64 && t <= 512 && t % 64 == 0 && w >= 1) cands.push_back({t, w});
    }
    if (cands.empty())
        for (int t : {128, 256, 512})
            for (int w : {1, 2, 4, 8})
                if (ara::batch_lds_bytes(b->n, t) * (size_t)w <= 160u * 1024u) cands.push_back({t, w});
    if (cands.empty()) cands.push_back({64, 1});
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
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[key] = best_cfg;
    return hipSuccess;
}

hipError_t capture_batch(ara_batch b) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = ara::launch_batch_pass(b->yv, batch_tables(b), b->precision == ARA_FP64, b->cfg, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e == hipSuccess) b->graph = g;
        else if (g) (void)hipGraphDestroy(g);
    }
    (void)hipStreamDestroy(cs);
    return e;
}

}  // namespace

ara_status ara_run_batch(ara_batch batch, double *const *d_ylts, void *hip_stream) {
    if (!batch || !d_ylts) return fail(ARA_ERR_INVALID_ARG, "NULL batch or d_ylts");
    for (int l = 0; l < batch->n; ++l)
        if (!d_ylts[l] && batch->yv.n_trials > 0) return fail(ARA_ERR_INVALID_ARG, "NULL YLT pointer");
    if (batch->yv.n_trials == 0) return ARA_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipSuccess;
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
        return ARA_OK;
    }
    if (!batch->tuned) {
        e = tune_batch(batch, s);
        if (e != hipSuccess) return hip_fail(e, "batch launch tuning");
    }
    if (!batch->exec) {
        e = capture_batch(batch);
        if (e != hipSuccess) return hip_fail(e, "batch graph capture");
    }
    e = hipGraphLaunch(batch->exec, s);
    if (e != hipSuccess) return hip_fail(e, "batch graph launch");
    return ARA_OK;
}

ara_status ara_batch_launch_config(ara_batch batch, int32_t *threads, int32_t *wg_per_cu) {
    if (!batch || !threads || !wg_per_cu) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    *threads = batch->tuned ? batch->cfg.threads : 0;
    *wg_per_cu = batch->tuned ? batch->cfg.wg_per_cu : 0;
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

ara_status ara_pml_tvar(const double *d_ylt, int64_t n_trials, const double *h_return_periods, int32_t n_rp,
                        double *h_pml, double *h_tvar, void *hip_stream) {
    if (!d_ylt || !h_return_periods || !h_pml || !h_tvar) return fail(ARA_ERR_INVALID_ARG, "NULL pointer");
    if (n_trials < 1 || n_trials > 2147483647LL) return fail(ARA_ERR_INVALID_ARG, "n_trials outside 1 .. 2^31-1");
    if (n_rp < 1 || n_rp > 16) return fail(ARA_ERR_INVALID_ARG, "n_rp outside 1 .. 16");
    int64_t k[16];
    for (int r = 0; r < n_rp; ++r) {
        double N = h_return_periods[r];
        if (!(N > 0.0) || !std::isfinite(N)) return fail(ARA_ERR_INVALID_ARG, "return period must be finite and > 0");
        double kk = std::floor((double)n_trials / N);
        if (kk < 1.0) return fail(ARA_ERR_RP, "return period leaves no tail trial (floor(T/N) < 1)");
        if (kk > (double)n_trials) return fail(ARA_ERR_RP, "return period shorter than one year (floor(T/N) > T)");
        k[r] = (int64_t)kk;
    }
    int32_t nan = 0;
    hipError_t e = ara::pml_tvar_device(d_ylt, n_trials, k, n_rp, h_pml, h_tvar, &nan,
                                        static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "PML/TVaR");
    if (nan) return fail(ARA_ERR_VALUE, "the YLT holds NaN");
    return ARA_OK;
}

}  // extern "C"
