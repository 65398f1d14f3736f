// PML and TVaR of Year Loss Tables on the GPU.
//
// For each (YLT, tail size k) pair -- a "selection" -- the k-th largest year
// loss is found exactly by a most-significant-digit radix selection over
// order-preserving 64-bit keys of the binary64 values (8 passes of 8 bits;
// every pass builds a 256-bin histogram of the candidates that still share
// the selected prefix).  The tail mean then adds every value strictly above
// the selected one with a deterministic tree (fixed grid, fixed order) and
// the ties at the selected value as (k - count) * value, all in binary64.
// Many YLTs of the same length are handled by the same launches (one grid
// row per YLT).
#include <mutex>
#include <vector>

#include "ara_internal.h"

namespace ara {
namespace {

constexpr int kMaxRp = 16;
constexpr int kMaxYlt = 64;
constexpr int kMaxSel = kMaxRp * kMaxYlt;
constexpr int kSumBlocks = 64;
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

// selection s = y * n_rp + r
__global__ void k_sel_init(SelState *st, TailSizes k, int n_rp, int n_sel, unsigned *hist, int *nan_flag) {
    for (int s = threadIdx.x; s < n_sel; s += blockDim.x) st[s] = SelState{0ULL, 0ULL, k.k[s % n_rp], k.k[s % n_rp]};
    for (int i = threadIdx.x; i < n_sel * 256; i += blockDim.x) hist[i] = 0u;
    if (threadIdx.x == 0) *nan_flag = 0;
}

// grid: (x blocks over the trials, one row per YLT)
__global__ __launch_bounds__(kThreads) void k_sel_hist(YltPtrs ylts, long long n, const SelState *__restrict__ st,
                                                       int n_rp, int shift, unsigned *__restrict__ hist, int *nan_flag) {
    __shared__ unsigned h[kMaxRp * 256];
    __shared__ SelState s[kMaxRp];
    const int yi = blockIdx.y;
    const double *__restrict__ y = ylts.p[yi];
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x) h[i] = 0u;
    if (threadIdx.x < n_rp) s[threadIdx.x] = st[yi * n_rp + threadIdx.x];
    __syncthreads();
    int saw_nan = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double v = y[i];
        saw_nan |= (v != v);
        const unsigned long long key = order_key(v);
        const unsigned bin = (unsigned)((key >> shift) & 255ULL);
        for (int r = 0; r < n_rp; ++r)
            if ((key & s[r].mask) == s[r].prefix) atomicAdd(&h[r * 256 + bin], 1u);
    }
    if (saw_nan) atomicOr(nan_flag, 1);
    __syncthreads();
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[(yi * n_rp) * 256 + i], h[i]);
}

// one block per selection: the 256 bins are summed from the top in LDS and
// the bin holding the selection's rank is picked; the histogram row is then
// cleared for the next pass
__global__ __launch_bounds__(256) void k_sel_pick(SelState *st, int shift, unsigned *hist) {
    __shared__ long long suf[256];  // suf[b] = count of bins b..255
    __shared__ int chosen;
    const int s = blockIdx.x;
    const int b = threadIdx.x;
    unsigned *h = hist + (size_t)s * 256;
    suf[b] = h[b];
    if (b == 0) chosen = 0;  // unreachable fallback: k_rem never exceeds the candidates
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {  // inclusive suffix sum, Hillis-Steele
        const long long add = b + d < 256 ? suf[b + d] : 0;
        __syncthreads();
        suf[b] += add;
        __syncthreads();
    }
    const long long k_rem = st[s].k_rem;
    const long long above = b < 255 ? suf[b + 1] : 0;  // candidates in bins above b
    if (suf[b] >= k_rem && above < k_rem) chosen = b;  // exactly one bin satisfies this
    __syncthreads();
    if (b == 0) {
        SelState x = st[s];
        const int c = chosen;
        x.k_rem -= c < 255 ? suf[c + 1] : 0;
        x.prefix |= ((unsigned long long)c) << shift;
        x.mask |= 255ULL << shift;
        st[s] = x;
    }
    h[b] = 0u;
}

// grid: (kSumBlocks, one row per YLT)
__global__ __launch_bounds__(kThreads) void k_tail_sum(YltPtrs ylts, long long n, const SelState *__restrict__ st,
                                                       int n_rp, double *__restrict__ psum,
                                                       unsigned long long *__restrict__ pcnt) {
    __shared__ double ssum[kThreads];
    __shared__ unsigned long long scnt[kThreads];
    const int yi = blockIdx.y;
    const double *__restrict__ y = ylts.p[yi];
    for (int r = 0; r < n_rp; ++r) {
        const int sel = yi * n_rp + r;
        const unsigned long long thr = st[sel].prefix;
        double acc = 0.0;
        unsigned long long cnt = 0;
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
            const double v = y[i];
            if (order_key(v) > thr) {
                acc += v;
                ++cnt;
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
__global__ __launch_bounds__(kSumBlocks) void k_tail_finish(const SelState *st, const double *psum,
                                                            const unsigned long long *pcnt, double *out) {
    __shared__ double ssum[kSumBlocks];
    __shared__ unsigned long long scnt[kSumBlocks];
    const int s = blockIdx.x;
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
        out[2 * s] = pml;
        out[2 * s + 1] = (ssum[0] + ties) / (double)k;
    }
}

// Library-owned scratch per device (device memory and a pinned host buffer
// for the results); ara_pml_tvar is synchronous and holds the device's lock
// for the duration of a call.
struct Scratch {
    std::mutex mu;
    void *d = nullptr;
    void *h = nullptr;
};

Scratch &scratch_for(int dev) {
    static Scratch s[64];
    return s[dev & 63];
}

}  // namespace

hipError_t pml_tvar_device(const double *const *d_ylts, int32_t n_ylt, int64_t n, const int64_t *h_k, int32_t n_rp,
                           double *h_out, int32_t *h_nan, hipStream_t s) {
    if (n_ylt < 1 || n_ylt > kMaxYlt || n_rp < 1 || n_rp > kMaxRp) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    Scratch &sc = scratch_for(dev);
    std::lock_guard<std::mutex> g(sc.mu);
    // layout: result (nan flag, then PML/TVaR pairs) | state | hist | psum | pcnt
    const size_t res_bytes = 16 + sizeof(double) * 2 * kMaxSel;
    const size_t off_state = res_bytes;
    const size_t off_hist = off_state + sizeof(SelState) * kMaxSel;
    const size_t off_psum = off_hist + sizeof(unsigned) * 256 * kMaxSel;
    const size_t off_pcnt = off_psum + sizeof(double) * kSumBlocks * kMaxSel;
    const size_t total = off_pcnt + sizeof(unsigned long long) * kSumBlocks * kMaxSel;
    if (!sc.d) {
        e = hipMalloc(&sc.d, total);
        if (e != hipSuccess) {
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
    }
    char *base = static_cast<char *>(sc.d);
    int *nan_flag = reinterpret_cast<int *>(base);
    double *out = reinterpret_cast<double *>(base + 16);
    SelState *st = reinterpret_cast<SelState *>(base + off_state);
    unsigned *hist = reinterpret_cast<unsigned *>(base + off_hist);
    double *psum = reinterpret_cast<double *>(base + off_psum);
    unsigned long long *pcnt = reinterpret_cast<unsigned long long *>(base + off_pcnt);
    const int n_sel = n_ylt * n_rp;

    YltPtrs yp{};
    for (int i = 0; i < n_ylt; ++i) yp.p[i] = d_ylts[i];
    // tail sizes travel as a kernel argument (no host-to-device copy)
    TailSizes tk{};
    for (int r = 0; r < n_rp; ++r) tk.k[r] = (long long)h_k[r];
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1024), 0, s, st, tk, n_rp, n_sel, hist, nan_flag);
    long long gx = (n + kThreads - 1) / kThreads;
    const long long cap = n_ylt > 8 ? 64 : 512;
    if (gx > cap) gx = cap;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        hipLaunchKernelGGL(k_sel_hist, dim3((unsigned)gx, n_ylt), dim3(kThreads), 0, s, yp, (long long)n, st, n_rp, shift,
                           hist, nan_flag);
        hipLaunchKernelGGL(k_sel_pick, dim3(n_sel), dim3(256), 0, s, st, shift, hist);
    }
    hipLaunchKernelGGL(k_tail_sum, dim3(kSumBlocks, n_ylt), dim3(kThreads), 0, s, yp, (long long)n, st, n_rp, psum, pcnt);
    hipLaunchKernelGGL(k_tail_finish, dim3(n_sel), dim3(kSumBlocks), 0, s, st, psum, pcnt, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // one copy of the flag and the results into pinned memory
    const size_t got = 16 + sizeof(double) * 2 * (size_t)n_sel;
    if ((e = hipMemcpyAsync(sc.h, sc.d, got, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const char *hb = static_cast<const char *>(sc.h);
    *h_nan = *reinterpret_cast<const int *>(hb);
    const double *ho = reinterpret_cast<const double *>(hb + 16);
    for (int i = 0; i < 2 * n_sel; ++i) h_out[i] = ho[i];
    return hipSuccess;
}

}  // namespace ara
