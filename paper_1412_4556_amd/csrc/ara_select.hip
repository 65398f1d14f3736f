// PML and TVaR of Year Loss Tables on the GPU.
//
// For each (YLT, tail size k) pair -- a "selection" -- the k-th largest year
// loss is found exactly by a most-significant-digit radix selection over
// order-preserving 64-bit keys of the binary64 values (8 passes of 8 bits;
// every pass builds a 256-bin histogram of the candidates that still share
// the selected prefix, and the next launch picks the bin holding the rank).  The tail mean then adds every value strictly above
// the selected one with a deterministic tree (fixed grid, fixed order) and
// the ties at the selected value as (k - count) * value, all in binary64.
// Many YLTs of the same length are handled by the same launches (one grid
// row per YLT).
#include <atomic>
#include <mutex>
#include <vector>

#include "ara_internal.h"

namespace ara {
namespace {

constexpr int kMaxRp = 16;
constexpr int kMaxYlt = 64;
constexpr int kMaxSel = kMaxRp * kMaxYlt;
constexpr int kSumBlocks = 512;
constexpr int kThreads = 256;

struct SelState {
    unsigned long long prefix;
    unsigned long long mask;
    long long k_rem;  // rank still to find among candidates, 1-based from the top
    long long k;
};

struct YltPtrs {
    const double *p[kMaxYlt];
};

__device__ __forceinline__ unsigned long long order_key(double v) {
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ULL);
}

__device__ __forceinline__ double key_value(unsigned long long key) {
    unsigned long long u = (key >> 63) ? (key & 0x7fffffffffffffffULL) : ~key;
    return __longlong_as_double((long long)u);
}

struct TailSizes {
    long long k[kMaxRp];
};

// The selection state for pass p lives in st[p] (st[kPasses]: the final
// one) and pass p's histogram in hist[p]: each launch derives the previous
// pass's pick from its histogram itself, so no launch reads a state that a
// block of the same launch writes.  The histograms start at zero (cleared
// when the scratch is allocated) and every call leaves them at zero: the
// launch two after the last reader of hist[p] clears it (the tail sum clears
// hist[6], the finishing kernel hist[7]).  The NaN flag is set by the first
// pass and moved to the results and cleared by the second.
constexpr int kPasses = 8;

// Clears the histogram rows of YLT yi in hist[p] (block x == 0 of each row).
__device__ __forceinline__ void clear_rows(unsigned *__restrict__ hist, int p, int n_sel, int yi, int n_rp) {
    if (blockIdx.x != 0) return;
    unsigned *row = hist + ((size_t)p * n_sel + (size_t)yi * n_rp) * 256;
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x) row[i] = 0u;
}

// Results go straight to pinned host memory, with system-scope stores.
__device__ __forceinline__ void store_host(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void store_host(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// One wave applies a pass's pick: lane l holds bins 4l .. 4l+3, a shuffle
// suffix sum gives every bin the count of candidates at or above it, and the
// one bin whose range holds rank k_rem is chosen.
__device__ SelState pick_wave(SelState x, const unsigned *__restrict__ h, int shift) {
    const int lane = (int)(threadIdx.x & 63u);
    const uint4 c = *reinterpret_cast<const uint4 *>(h + 4 * lane);
    const unsigned long long tot = (unsigned long long)c.x + c.y + c.z + c.w;
    unsigned long long suf = tot;  // candidates in bins >= 4 * lane
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long u = __shfl_down(suf, d, 64);
        if (lane + d < 64) suf += u;
    }
    const unsigned cnt[4] = {c.x, c.y, c.z, c.w};
    unsigned long long at = suf;  // candidates in bins >= 4 * lane + v
    int chosen = -1;
    unsigned long long above = 0;
    const unsigned long long k_rem = (unsigned long long)x.k_rem;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const unsigned long long up = at - cnt[v];  // bins above 4 * lane + v
        if (at >= k_rem && up < k_rem) {
            chosen = 4 * lane + v;
            above = up;
        }
        at = up;
    }
    // exactly one lane holds the chosen bin (k_rem never exceeds the candidates)
    const unsigned long long owner = __ballot(chosen >= 0);
    const int src = owner ? __builtin_ctzll(owner) : 0;
    const int cb = __shfl(chosen, src, 64);
    const unsigned long long ab = __shfl(above, src, 64);
    if (cb >= 0) {
        x.k_rem -= (long long)ab;
        x.prefix |= ((unsigned long long)cb) << shift;
        x.mask |= 255ULL << shift;
    }
    return x;
}

// Loads into s[] the selections' states for pass `pass` (st[pass]): for the
// first pass the start state (tail sizes from the arguments), else the state before the previous pass with
// that pass's pick applied from its histogram.  Waves take the selections in
// turn; block 0 stores st[pass] for the finishing kernel.  A launch reads
// st[pass - 1] and writes st[pass] only, so no block reads what another
// block of the same launch writes.
__device__ void load_states(SelState *__restrict__ st, const unsigned *__restrict__ hist, const TailSizes &tk,
                            int yi, int n_rp, int n_sel, int pass, SelState *s) {
    const int wave = (int)(threadIdx.x >> 6), n_wave = (int)(blockDim.x >> 6);
    for (int r = wave; r < n_rp; r += n_wave) {
        const int sel = yi * n_rp + r;
        SelState x;
        if (pass == 0) {
            x = SelState{0ULL, 0ULL, tk.k[r], tk.k[r]};
            if (blockIdx.x == 0 && (threadIdx.x & 63u) == 0) st[sel] = x;
        } else {
            x = st[(size_t)(pass - 1) * n_sel + sel];
            x = pick_wave(x, hist + ((size_t)(pass - 1) * n_sel + sel) * 256, 64 - 8 * pass);
            if (blockIdx.x == 0 && (threadIdx.x & 63u) == 0) st[(size_t)pass * n_sel + sel] = x;
        }
        if ((threadIdx.x & 63u) == 0) s[r] = x;
    }
}

// A thread's share of a YLT per round: kPer values TH apart (TH threads per
// block), all loaded before any is used, so their latencies overlap.
constexpr int kPer = 8;
constexpr int kHistThreads = 1024;
constexpr long long kChunk = (long long)kThreads * kPer;
constexpr long long kHistChunk = (long long)kHistThreads * kPer;

template <int TH>
__device__ __forceinline__ void load_chunk(const double *__restrict__ y, long long n, long long c0, double (&v)[kPer]) {
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const long long i = c0 + (long long)j * TH + threadIdx.x;
        v[j] = i < n ? y[i] : 0.0;
    }
}

// grid: (x blocks over the trials, one row per YLT).  A thread counts a run
// of its values that fall into one bin in a register and adds the run to the
// LDS histogram when the bin changes (the first passes see few bins).
// Selections of a YLT that still share their prefix (all of them in the
// first pass) have the same histogram: it is counted once.  Blocks are
// large, so that few of them add into each global histogram (those atomics
// are slow when many blocks hit the same bins).
__global__ __launch_bounds__(kHistThreads) void k_sel_hist(YltPtrs ylts, long long n, SelState *__restrict__ st,
                                                           TailSizes tk, int n_rp, int n_sel, int pass,
                                                           unsigned *__restrict__ hist, int *nan_flags,
                                                           int *nan_seen, int *host_nan) {
    __shared__ unsigned h[kMaxRp * 256];
    __shared__ SelState s[kMaxRp];
    __shared__ int same_as[kMaxRp];  // first selection with the same prefix
    const int yi = blockIdx.y;
    const int shift = 56 - 8 * pass;
    const double *__restrict__ y = ylts.p[yi];
    const long long stride = (long long)gridDim.x * kHistChunk;
    long long c0 = (long long)blockIdx.x * kHistChunk;
    double v[kPer];
    load_chunk<kHistThreads>(y, n, c0, v);  // in flight while the previous pick is applied
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x) h[i] = 0u;
    load_states(st, hist, tk, yi, n_rp, n_sel, pass, s);
    if (pass >= 2) clear_rows(hist, pass - 2, n_sel, yi, n_rp);
    if (pass == 1 && blockIdx.x == 0 && threadIdx.x == 0) {
        // every block of pass 0 has finished: move this YLT's flag on
        const int f = nan_flags[yi];
        nan_flags[yi] = 0;
        nan_seen[yi] = f;
        if (host_nan) store_host(host_nan + yi, f);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)n_rp) {
        int f = (int)threadIdx.x;
        for (int q = 0; q < (int)threadIdx.x; ++q)
            if (s[q].mask == s[threadIdx.x].mask && s[q].prefix == s[threadIdx.x].prefix) {
                f = q;
                break;
            }
        same_as[threadIdx.x] = f;
    }
    __syncthreads();
    int saw_nan = 0;
    while (c0 < n) {
        const long long rest = n - c0 - threadIdx.x;  // values of this thread in the chunk: j * kHistThreads < rest
        double w[kPer];
        const long long c1 = c0 + stride;
        if (c1 < n) load_chunk<kHistThreads>(y, n, c1, w);  // the next chunk, in flight while this one is counted
        for (int r = 0; r < n_rp; ++r) {
            if (same_as[r] != r) continue;
            const unsigned long long mask = s[r].mask, prefix = s[r].prefix;
            unsigned run_bin = 0u, run = 0u;
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                if ((long long)j * kHistThreads >= rest) continue;
                const unsigned long long key = order_key(v[j]);
                if ((key & mask) != prefix) continue;
                const unsigned bin = (unsigned)((key >> shift) & 255ULL);
                if (run != 0u && bin != run_bin) {
                    atomicAdd(&h[r * 256 + run_bin], run);
                    run = 0u;
                }
                run_bin = bin;
                ++run;
            }
            if (run != 0u) atomicAdd(&h[r * 256 + run_bin], run);
        }
        if (pass == 0) {
#pragma unroll
            for (int j = 0; j < kPer; ++j) saw_nan |= ((long long)j * kHistThreads < rest) & (v[j] != v[j]);
        }
        c0 = c1;
        if (c0 < n) {
#pragma unroll
            for (int j = 0; j < kPer; ++j) v[j] = w[j];
        }
    }
    if (saw_nan) atomicOr(&nan_flags[yi], 1);
    __syncthreads();
    unsigned *hp = hist + ((size_t)pass * n_sel + (size_t)yi * n_rp) * 256;
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x) {
        const unsigned c = h[same_as[i >> 8] * 256 + (i & 255)];
        if (c) atomicAdd(&hp[i], c);
    }
}

// grid: (kSumBlocks, one row per YLT).  Applies the last pass's pick (the
// selected key is then exact) and sums every value strictly above it.
__global__ __launch_bounds__(kThreads) void k_tail_sum(YltPtrs ylts, long long n, SelState *__restrict__ st, TailSizes tk,
                                                       int n_rp, int n_sel, unsigned *__restrict__ hist,
                                                       double *__restrict__ psum,
                                                       unsigned long long *__restrict__ pcnt) {
    __shared__ double ssum[kThreads];
    __shared__ unsigned long long scnt[kThreads];
    __shared__ SelState s[kMaxRp];
    const int yi = blockIdx.y;
    const double *__restrict__ y = ylts.p[yi];
    const long long stride = (long long)gridDim.x * kChunk;
    double v[kPer];
    long long held = (long long)blockIdx.x * kChunk;  // the chunk in v
    load_chunk<kThreads>(y, n, held, v);
    load_states(st, hist, tk, yi, n_rp, n_sel, kPasses, s);
    clear_rows(hist, kPasses - 2, n_sel, yi, n_rp);
    __syncthreads();
    for (int r = 0; r < n_rp; ++r) {
        const int sel = yi * n_rp + r;
        const unsigned long long thr = s[r].prefix;
        double acc = 0.0;
        unsigned long long cnt = 0;
        for (long long c0 = (long long)blockIdx.x * kChunk; c0 < n; c0 += stride) {
            if (c0 != held) {
                load_chunk<kThreads>(y, n, c0, v);
                held = c0;
            }
            const long long rest = n - c0 - threadIdx.x;
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                if ((long long)j * kThreads < rest && order_key(v[j]) > thr) {
                    acc += v[j];
                    ++cnt;
                }
            }
        }
        ssum[threadIdx.x] = acc;
        scnt[threadIdx.x] = cnt;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                ssum[threadIdx.x] += ssum[threadIdx.x + w];
                scnt[threadIdx.x] += scnt[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            psum[(size_t)sel * kSumBlocks + blockIdx.x] = ssum[0];
            pcnt[(size_t)sel * kSumBlocks + blockIdx.x] = scnt[0];
        }
        __syncthreads();
    }
}

// one block per selection; the partial sums of the kSumBlocks blocks are
// added with a fixed tree, so the result does not depend on timing
// Results go to pinned host memory (host_out, pairs per selection) or, when
// dev_pml is set, to device arrays, where a YLT holding NaN gets NaN results.
__global__ __launch_bounds__(kSumBlocks) void k_tail_finish(const SelState *st, const double *psum,
                                                            const unsigned long long *pcnt,
                                                            unsigned *__restrict__ hist7, double *host_out,
                                                            int n_rp, const int *__restrict__ nan_seen,
                                                            double *__restrict__ dev_pml,
                                                            double *__restrict__ dev_tvar) {
    __shared__ double ssum[kSumBlocks];
    __shared__ unsigned long long scnt[kSumBlocks];
    const int s = blockIdx.x;
    if (threadIdx.x < 256) hist7[(size_t)s * 256 + threadIdx.x] = 0u;
    ssum[threadIdx.x] = psum[(size_t)s * kSumBlocks + threadIdx.x];
    scnt[threadIdx.x] = pcnt[(size_t)s * kSumBlocks + threadIdx.x];
    __syncthreads();
    for (int w = kSumBlocks / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
            scnt[threadIdx.x] += scnt[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double pml = key_value(st[s].prefix);
        const long long k = st[s].k;
        const double ties = (double)(k - (long long)scnt[0]) * pml;
        const double tvar = (ssum[0] + ties) / (double)k;
        if (dev_pml) {
            const bool nan = nan_seen[s / n_rp] != 0;
            dev_pml[s] = nan ? __longlong_as_double(0x7ff8000000000000LL) : pml;
            dev_tvar[s] = nan ? __longlong_as_double(0x7ff8000000000000LL) : tvar;
        } else {
            store_host(host_out + 2 * s, pml);
            store_host(host_out + 2 * s + 1, tvar);
        }
    }
}

// Zeroes n words (the histograms and NaN flags a call of the no-allocation
// form starts from).
__global__ __launch_bounds__(kThreads) void k_zero_words(unsigned *__restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Scratch layout for up to ms selections: NaN flags per YLT | flags moved on
// by pass 1 | states per pass | histograms per pass | psum | pcnt.  Every
// offset is a multiple of 16 bytes.
struct SelLayout {
    size_t seen, state, hist, psum, pcnt, total;
};
constexpr SelLayout layout_for(size_t ms) {
    return SelLayout{sizeof(int) * kMaxYlt,
                  2 * sizeof(int) * kMaxYlt,
                  2 * sizeof(int) * kMaxYlt + sizeof(SelState) * (kPasses + 1) * ms,
                  2 * sizeof(int) * kMaxYlt + sizeof(SelState) * (kPasses + 1) * ms + sizeof(unsigned) * 256 * kPasses * ms,
                  2 * sizeof(int) * kMaxYlt + sizeof(SelState) * (kPasses + 1) * ms + sizeof(unsigned) * 256 * kPasses * ms +
                      sizeof(double) * kSumBlocks * ms,
                  2 * sizeof(int) * kMaxYlt + sizeof(SelState) * (kPasses + 1) * ms + sizeof(unsigned) * 256 * kPasses * ms +
                      (sizeof(double) + sizeof(unsigned long long)) * kSumBlocks * ms};
}
static_assert(sizeof(SelState) == 32, "selection state size");

// The launches of one call over a scratch of layout lay at base.
hipError_t launch_select(char *base, const SelLayout &lay, const double *const *d_ylts, int32_t n_ylt, int64_t n,
                         const int64_t *h_k, int32_t n_rp, int *host_nan, double *host_out, double *dev_pml,
                         double *dev_tvar, hipStream_t s) {
    int *nan_flags = reinterpret_cast<int *>(base);
    int *nan_seen = reinterpret_cast<int *>(base + lay.seen);
    SelState *st = reinterpret_cast<SelState *>(base + lay.state);
    unsigned *hist = reinterpret_cast<unsigned *>(base + lay.hist);
    double *psum = reinterpret_cast<double *>(base + lay.psum);
    unsigned long long *pcnt = reinterpret_cast<unsigned long long *>(base + lay.pcnt);
    const int n_sel = n_ylt * n_rp;
    YltPtrs yp{};
    for (int i = 0; i < n_ylt; ++i) yp.p[i] = d_ylts[i];
    // tail sizes travel as a kernel argument (no host-to-device copy)
    TailSizes tk{};
    for (int r = 0; r < n_rp; ++r) tk.k[r] = (long long)h_k[r];
    long long gx = (n + kHistChunk - 1) / kHistChunk;
    const long long cap = n_ylt > 8 ? 32 : 256;
    if (gx > cap) gx = cap;
    for (int pass = 0; pass < kPasses; ++pass)
        hipLaunchKernelGGL(k_sel_hist, dim3((unsigned)gx, n_ylt), dim3(kHistThreads), 0, s, yp, (long long)n, st, tk,
                           n_rp, n_sel, pass, hist, nan_flags, nan_seen, host_nan);
    hipLaunchKernelGGL(k_tail_sum, dim3(kSumBlocks, n_ylt), dim3(kThreads), 0, s, yp, (long long)n, st, tk, n_rp, n_sel,
                       hist, psum, pcnt);
    hipLaunchKernelGGL(k_tail_finish, dim3(n_sel), dim3(kSumBlocks), 0, s, st + (size_t)kPasses * n_sel, psum, pcnt,
                       hist + (size_t)(kPasses - 1) * n_sel * 256, host_out, n_rp, nan_seen, dev_pml, dev_tvar);
    return hipGetLastError();
}

// Scratch of the no-allocation form: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code uses only the address that
// hipGetSymbolAddress returns for the current device.
constexpr int kNoAllocSel = ARA_NOALLOC_MAX_SEL;
constexpr SelLayout kNoAllocLayout = layout_for(kNoAllocSel);
static __device__ __align__(256) unsigned char scratch[kNoAllocLayout.total];

// Library-owned scratch per device: device memory and a pinned host buffer
// that the finishing kernels write the results into.  ara_pml_tvar is
// synchronous and holds the device's lock for the duration of a call.  A
// call that fails after its first launch marks the scratch dirty, and the
// next call waits for the device, then clears the histograms and the flag
// before it starts.
struct Scratch {
    std::mutex mu;
    void *d = nullptr;
    void *h = nullptr;   // host address
    void *hd = nullptr;  // its device address
    bool dirty = false;
};

// dev in 0 .. kMaxDevices - 1 (checked by the caller)
Scratch &scratch_for(int dev) {
    static Scratch s[kMaxDevices];
    return s[dev];
}

}  // namespace

hipError_t pml_tvar_device(const double *const *d_ylts, int32_t n_ylt, int64_t n, const int64_t *h_k, int32_t n_rp,
                           double *h_out, int32_t *h_nan, hipStream_t s) {
    if (n_ylt < 1 || n_ylt > kMaxYlt || n_rp < 1 || n_rp > kMaxRp) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    Scratch &sc = scratch_for(dev);
    std::lock_guard<std::mutex> g(sc.mu);
    // host layout: NaN flag per YLT | PML/TVaR pairs
    constexpr SelLayout lay = layout_for(kMaxSel);
    const size_t res_off = sizeof(int) * kMaxYlt;
    const size_t res_bytes = res_off + sizeof(double) * 2 * kMaxSel;
    if (!sc.d) {
        e = hipMalloc(&sc.d, lay.total);
        if (e != hipSuccess) {
            sc.d = nullptr;
            return e;
        }
        e = hipMemset(sc.d, 0, lay.psum);  // flags, states and histograms start at zero
        if (e != hipSuccess) {
            (void)hipFree(sc.d);
            sc.d = nullptr;
            return e;
        }
    }
    if (!sc.h) {
        e = hipHostMalloc(&sc.h, res_bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            sc.h = nullptr;
            return e;
        }
        e = hipHostGetDevicePointer(&sc.hd, sc.h, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(sc.h);
            sc.h = nullptr;
            return e;
        }
    }
    char *base = static_cast<char *>(sc.d);
    if (sc.dirty) {
        // the failed call's kernels may still run, on another stream
        if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
        if ((e = hipMemsetAsync(base, 0, lay.seen, s)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(base + lay.hist, 0, lay.psum - lay.hist, s)) != hipSuccess) return e;
        sc.dirty = false;
    }
    int *host_nan = static_cast<int *>(sc.hd);
    double *host_out = reinterpret_cast<double *>(static_cast<char *>(sc.hd) + res_off);
    sc.dirty = true;  // until the call has run to its end
    e = launch_select(base, lay, d_ylts, n_ylt, n, h_k, n_rp, host_nan, host_out, nullptr, nullptr, s);
    if (e != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    sc.dirty = false;
    const char *hb = static_cast<const char *>(sc.h);
    const volatile int *hn = reinterpret_cast<const volatile int *>(hb);
    int any = 0;
    for (int i = 0; i < n_ylt; ++i) any |= hn[i];
    *h_nan = any;
    const volatile double *ho = reinterpret_cast<const volatile double *>(hb + res_off);
    for (int i = 0; i < 2 * n_ylt * n_rp; ++i) h_out[i] = ho[i];
    return hipSuccess;
}

hipError_t pml_tvar_noalloc(const double *const *d_ylts, int32_t n_ylt, int64_t n, const int64_t *h_k, int32_t n_rp,
                            double *d_pml, double *d_tvar, hipStream_t s) {
    if (n_ylt < 1 || n_ylt > kMaxYlt || n_rp < 1 || n_rp > kMaxRp || n_ylt * n_rp > kNoAllocSel)
        return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    // the array's address on this device, looked up once per device with the
    // device current
    static std::atomic<char *> addr[kMaxDevices];
    static std::atomic<bool> dirty[kMaxDevices];
    static std::mutex mu;
    const SelLayout &lay = kNoAllocLayout;
    char *base = addr[dev].load(std::memory_order_acquire);
    if (!base) {
        std::lock_guard<std::mutex> g(mu);
        base = addr[dev].load(std::memory_order_relaxed);
        if (!base) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (!p) return hipErrorInvalidSymbol;
            base = static_cast<char *>(p);
            dirty[dev].store(true);
            addr[dev].store(base, std::memory_order_release);
        }
    }
    // Every call that runs to its end leaves the flags and every histogram
    // row it used at zero (each row is cleared two launches after its last
    // reader).  The first call on a device, and a call after one that failed
    // between its launches, clears them first with a kernel (not a memset
    // node, so that the call can be captured).
    if (dirty[dev].exchange(false)) {
        hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(kThreads), 0, s, reinterpret_cast<unsigned *>(base),
                           (long long)(lay.state / sizeof(unsigned)));
        hipLaunchKernelGGL(k_zero_words, dim3(256), dim3(kThreads), 0, s,
                           reinterpret_cast<unsigned *>(base + lay.hist),
                           (long long)((lay.psum - lay.hist) / sizeof(unsigned)));
        if ((e = hipGetLastError()) != hipSuccess) {
            dirty[dev].store(true);
            return e;
        }
    }
    e = launch_select(base, lay, d_ylts, n_ylt, n, h_k, n_rp, nullptr, nullptr, d_pml, d_tvar, s);
    if (e != hipSuccess) dirty[dev].store(true);
    return e;
}

}  // namespace ara
