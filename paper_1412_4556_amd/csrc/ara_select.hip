// PML and TVaR of a Year Loss Table on the GPU.
//
// For each tail size k the k-th largest year loss is found exactly by a
// most-significant-digit radix selection over order-preserving 64-bit keys
// of the binary64 values (8 passes of 8 bits; every pass builds a 256-bin
// histogram of the candidates that still share the selected prefix).  The
// tail mean then adds every value strictly above the selected one with a
// deterministic tree (fixed grid, fixed order) and the ties at the selected
// value as (k - count) * value, all in binary64.
#include <mutex>
#include <vector>

#include "ara_internal.h"

namespace ara {
namespace {

constexpr int kMaxRp = 16;
constexpr int kSumBlocks = 256;
constexpr int kThreads = 256;

struct SelState {
    unsigned long long prefix;
    unsigned long long mask;
    long long k_rem;  // rank still to find among candidates, 1-based from the top
    long long k;
};

__device__ __forceinline__ unsigned long long order_key(double v) {
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ULL);
}

__device__ __forceinline__ double key_value(unsigned long long key) {
    unsigned long long u = (key >> 63) ? (key & 0x7fffffffffffffffULL) : ~key;
    return __longlong_as_double((long long)u);
}

__global__ void k_sel_init(SelState *st, const long long *k, int n_rp, unsigned *hist, int *nan_flag) {
    int t = threadIdx.x;
    if (t < n_rp) st[t] = SelState{0ULL, 0ULL, k[t], k[t]};
    for (int i = t; i < n_rp * 256; i += blockDim.x) hist[i] = 0u;
    if (t == 0) *nan_flag = 0;
}

__global__ __launch_bounds__(kThreads) void k_sel_hist(const double *__restrict__ y, long long n,
                                                       const SelState *__restrict__ st, int n_rp, int shift,
                                                       unsigned *__restrict__ hist, int *nan_flag) {
    __shared__ unsigned h[kMaxRp * 256];
    __shared__ SelState s[kMaxRp];
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x) h[i] = 0u;
    if (threadIdx.x < n_rp) s[threadIdx.x] = st[threadIdx.x];
    __syncthreads();
    int saw_nan = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double v = y[i];
        saw_nan |= (v != v);
        unsigned long long key = order_key(v);
        unsigned bin = (unsigned)((key >> shift) & 255ULL);
        for (int r = 0; r < n_rp; ++r)
            if ((key & s[r].mask) == s[r].prefix) atomicAdd(&h[r * 256 + bin], 1u);
    }
    if (saw_nan) atomicOr(nan_flag, 1);
    __syncthreads();
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void k_sel_pick(SelState *st, int n_rp, int shift, unsigned *hist) {
    int r = threadIdx.x;
    if (r < n_rp) {
        SelState s = st[r];
        long long cum = 0;
        int chosen = 0;
        for (int b = 255; b >= 0; --b) {
            long long c = hist[r * 256 + b];
            if (cum + c >= s.k_rem) {
                chosen = b;
                s.k_rem -= cum;
                break;
            }
            cum += c;
        }
        s.prefix |= ((unsigned long long)chosen) << shift;
        s.mask |= 255ULL << shift;
        st[r] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x) hist[i] = 0u;
}

__global__ __launch_bounds__(kThreads) void k_tail_sum(const double *__restrict__ y, long long n,
                                                       const SelState *__restrict__ st, int n_rp,
                                                       double *__restrict__ psum, unsigned long long *__restrict__ pcnt) {
    __shared__ double ssum[kThreads];
    __shared__ unsigned long long scnt[kThreads];
    for (int r = 0; r < n_rp; ++r) {
        const unsigned long long thr = st[r].prefix;
        double acc = 0.0;
        unsigned long long cnt = 0;
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
            double v = y[i];
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
            psum[r * kSumBlocks + blockIdx.x] = ssum[0];
            pcnt[r * kSumBlocks + blockIdx.x] = scnt[0];
        }
        __syncthreads();
    }
}

__global__ void k_tail_finish(const SelState *st, int n_rp, const double *psum, const unsigned long long *pcnt,
                              double *out) {
    int r = threadIdx.x;
    if (r >= n_rp) return;
    double s = 0.0;
    unsigned long long c = 0;
    for (int b = 0; b < kSumBlocks; ++b) {
        s += psum[r * kSumBlocks + b];
        c += pcnt[r * kSumBlocks + b];
    }
    const double pml = key_value(st[r].prefix);
    const long long k = st[r].k;
    const double ties = (double)(k - (long long)c) * pml;
    out[r] = pml;
    out[kMaxRp + r] = (s + ties) / (double)k;
}

struct Scratch {
    std::mutex mu;
    void *d = nullptr;
    int device = -1;
};

Scratch &scratch_for(int dev) {
    static Scratch s[64];
    return s[dev & 63];
}

}  // namespace

hipError_t pml_tvar_device(const double *d_ylt, int64_t n, const int64_t *h_k, int32_t n_rp, double *h_pml,
                           double *h_tvar, int32_t *h_nan, hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    Scratch &sc = scratch_for(dev);
    std::lock_guard<std::mutex> g(sc.mu);
    // layout: state | k | hist | psum | pcnt | out | nan
    const size_t off_state = 0;
    const size_t off_k = off_state + sizeof(SelState) * kMaxRp;
    const size_t off_hist = off_k + sizeof(long long) * kMaxRp;
    const size_t off_psum = off_hist + sizeof(unsigned) * 256 * kMaxRp;
    const size_t off_pcnt = off_psum + sizeof(double) * kSumBlocks * kMaxRp;
    const size_t off_out = off_pcnt + sizeof(unsigned long long) * kSumBlocks * kMaxRp;
    const size_t off_nan = off_out + sizeof(double) * 2 * kMaxRp;
    const size_t total = off_nan + 256;
    if (!sc.d) {
        e = hipMalloc(&sc.d, total);
        if (e != hipSuccess) {
            sc.d = nullptr;
            return e;
        }
    }
    char *base = static_cast<char *>(sc.d);
    SelState *st = reinterpret_cast<SelState *>(base + off_state);
    long long *dk = reinterpret_cast<long long *>(base + off_k);
    unsigned *hist = reinterpret_cast<unsigned *>(base + off_hist);
    double *psum = reinterpret_cast<double *>(base + off_psum);
    unsigned long long *pcnt = reinterpret_cast<unsigned long long *>(base + off_pcnt);
    double *out = reinterpret_cast<double *>(base + off_out);
    int *nan_flag = reinterpret_cast<int *>(base + off_nan);

    long long hk[kMaxRp];
    for (int r = 0; r < n_rp; ++r) hk[r] = (long long)h_k[r];
    if ((e = hipMemcpyAsync(dk, hk, sizeof(long long) * n_rp, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, st, dk, n_rp, hist, nan_flag);
    int grid = (int)((n + kThreads - 1) / kThreads);
    if (grid > 1024) grid = 1024;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        hipLaunchKernelGGL(k_sel_hist, dim3(grid), dim3(kThreads), 0, s, d_ylt, (long long)n, st, n_rp, shift, hist,
                           nan_flag);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, st, n_rp, shift, hist);
    }
    hipLaunchKernelGGL(k_tail_sum, dim3(kSumBlocks), dim3(kThreads), 0, s, d_ylt, (long long)n, st, n_rp, psum, pcnt);
    hipLaunchKernelGGL(k_tail_finish, dim3(1), dim3(64), 0, s, st, n_rp, psum, pcnt, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double hout[2 * kMaxRp];
    int hn = 0;
    if ((e = hipMemcpyAsync(hout, out, sizeof(double) * 2 * kMaxRp, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&hn, nan_flag, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    for (int r = 0; r < n_rp; ++r) {
        h_pml[r] = hout[r];
        h_tvar[r] = hout[kMaxRp + r];
    }
    *h_nan = hn;
    return hipSuccess;
}

}  // namespace ara
