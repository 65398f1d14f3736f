// HIP kernels of the trial pass for gfx950 (CDNA4, wave64).
//
// Mapping: one wavefront owns one trial at a time (grid-stride over trials).
// Lane l of the wave takes events [c + 4l, c + 4l + 4) of each 256-event
// chunk c of the trial, read with one 16-byte load per lane, so a wave's
// loads of the Year Event Table are fully coalesced.  Each lane turns its
// events into occurrence losses (lookup, FT1, cross-ELT sum, FT2; Section
// III steps 1-3) and keeps a private running sum; the trial total is a wave
// reduction, and the aggregate terms FT3 (step 4) are applied in binary64.
//
// The per-event variant replaces the private sums by an inclusive scan over
// the wave (DPP row shifts and row broadcasts) with a carry between chunks,
// which yields the cumulative loss S_k after every event.
#include "ara_internal.h"
#include "ara_index.h"

#include <atomic>
#include <map>
#include <mutex>
#include <set>
#include <tuple>

namespace ara {
namespace {

// --------------------------------------------------------------------------------------------
// arithmetic
template <typename T>
__device__ __forceinline__ T clamp_excess(T x, T r, T u) {
    // min(max(x - r, 0), u)
    T v = x - r;
    v = v < T(0) ? T(0) : v;
    return v > u ? u : v;
}

// Knuth's TwoSum: s + err == a + b exactly (round-to-nearest, no overflow).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &err) {
    s = a + b;
    float bb = s - a;
    err = (a - (s - bb)) + (b - bb);
}

// Running sums.  Acc<double> is plain binary64; Acc<float> is a compensated
// binary32 pair (sum, accumulated TwoSum errors).
template <typename T>
struct Acc;

template <>
struct Acc<double> {
    double s;
    __device__ __forceinline__ static Acc zero() { return Acc{0.0}; }
    __device__ __forceinline__ void add(double o) { s += o; }
    __device__ __forceinline__ static Acc combine(const Acc &a, const Acc &b) { return Acc{a.s + b.s}; }
    __device__ __forceinline__ double value() const { return s; }
};

template <>
struct Acc<float> {
    float s, c;
    __device__ __forceinline__ static Acc zero() { return Acc{0.0f, 0.0f}; }
    __device__ __forceinline__ void add(float o) {
        float t;
        two_sum(s, o, s, t);
        c += t;
    }
    __device__ __forceinline__ static Acc combine(const Acc &a, const Acc &b) {
        Acc r;
        float t;
        two_sum(a.s, b.s, r.s, t);
        r.c = (a.c + b.c) + t;
        return r;
    }
    __device__ __forceinline__ double value() const { return (double)s + (double)c; }
};

// Combined event loss over the ELTs of a layer, in layer order.
template <typename T>
struct EventSum;

template <>
struct EventSum<double> {
    double e = 0.0;
    __device__ __forceinline__ void add(double x) { e += x; }
    __device__ __forceinline__ double value() const { return e; }
};

template <>
struct EventSum<float> {
    float hi = 0.0f, lo = 0.0f;
    __device__ __forceinline__ void add(float x) {
        float t;
        two_sum(hi, x, hi, t);
        lo += t;
    }
    __device__ __forceinline__ float value() const { return hi + lo; }
};

// --------------------------------------------------------------------------------------------
// cross-lane moves
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Word of the hashed filter for an event ID: the top 27 - hshift bits of the
// low 32 bits of a full-rate 24 x 24-bit product (the event's bit in that
// word is ID mod 32).  __umul24 returns a signed int: the product is taken
// as unsigned before the shift, so the word stays below 2^(27 - hshift),
// the filter's size in words.
__device__ __forceinline__ uint32_t hash_word(uint32_t id, int32_t hshift) {
    return (uint32_t)__umul24(id, kHashMul24) >> (hshift + 5);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i(int v) {
    // lanes of rows outside ROW_MASK, and lanes whose source is outside the
    // row, receive 0
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, true);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ Acc<double> dpp_acc(const Acc<double> &a) {
    long long b = __double_as_longlong(a.s);
    int lo = dpp_i<CTRL, ROW_MASK>((int)(b & 0xffffffffLL));
    int hi = dpp_i<CTRL, ROW_MASK>((int)(b >> 32));
    long long r = ((long long)(unsigned)lo) | ((long long)hi << 32);
    return Acc<double>{__longlong_as_double(r)};
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ Acc<float> dpp_acc(const Acc<float> &a) {
    return Acc<float>{__int_as_float(dpp_i<CTRL, ROW_MASK>(__float_as_int(a.s))),
                      __int_as_float(dpp_i<CTRL, ROW_MASK>(__float_as_int(a.c)))};
}

// DPP controls (GFX9 encoding)
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

// Inclusive scan of a over the 64 lanes: shifts by 1, 2, 4, 8 inside each
// 16-lane row, then row 0's total into row 1 and row 2's into row 3, then the
// total of rows 0-1 into rows 2-3.  The combine order is fixed, so the result
// is deterministic.
template <typename T>
__device__ __forceinline__ Acc<T> wave_inclusive_scan(Acc<T> a) {
    a = Acc<T>::combine(dpp_acc<kRowShr1, 0xf>(a), a);
    a = Acc<T>::combine(dpp_acc<kRowShr2, 0xf>(a), a);
    a = Acc<T>::combine(dpp_acc<kRowShr4, 0xf>(a), a);
    a = Acc<T>::combine(dpp_acc<kRowShr8, 0xf>(a), a);
    a = Acc<T>::combine(dpp_acc<kRowBcast15, 0xa>(a), a);
    a = Acc<T>::combine(dpp_acc<kRowBcast31, 0xc>(a), a);
    return a;
}

__device__ __forceinline__ Acc<double> shfl_acc(const Acc<double> &a, int src) {
    return Acc<double>{__shfl(a.s, src)};
}
__device__ __forceinline__ Acc<float> shfl_acc(const Acc<float> &a, int src) {
    return Acc<float>{__shfl(a.s, src), __shfl(a.c, src)};
}

// Partner of the butterfly step that pairs lane i with lane i ^ M, without
// the LDS: M = 32 and 16 by the lane-half / row swaps of gfx950, M = 2 and 1
// by quad permutes; M = 8 and 4 by row rotations, which reach a lane whose
// value is bitwise that of lane i ^ M at those steps (after the steps 32 and
// 16 every lane holds the value of all lanes equal to it mod 16, after step 8
// mod 8, since every combine is commutative).
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kRowRor4 = 0x124, kRowRor8 = 0x128;

template <int M>
__device__ __forceinline__ int butterfly_partner(int v) {
    if (M == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32u) ? r[0] : r[1];
    } else if (M == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16u) ? r[0] : r[1];
    } else if (M == 8) {
        return dpp_i<kRowRor8, 0xf>(v);
    } else if (M == 4) {
        return dpp_i<kRowRor4, 0xf>(v);
    } else if (M == 2) {
        return dpp_i<kQuadXor2, 0xf>(v);
    } else {
        return dpp_i<kQuadXor1, 0xf>(v);
    }
}

template <int M>
__device__ __forceinline__ double butterfly_partner(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = butterfly_partner<M>((int)(b & 0xffffffffLL));
    const int hi = butterfly_partner<M>((int)(b >> 32));
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}
template <int M>
__device__ __forceinline__ float butterfly_partner(float x) {
    return __int_as_float(butterfly_partner<M>(__float_as_int(x)));
}
template <int M>
__device__ __forceinline__ Acc<double> butterfly_partner(const Acc<double> &a) {
    return Acc<double>{butterfly_partner<M>(a.s)};
}
template <int M>
__device__ __forceinline__ Acc<float> butterfly_partner(const Acc<float> &a) {
    return Acc<float>{butterfly_partner<M>(a.s), butterfly_partner<M>(a.c)};
}

// Butterfly all-reduce (partners lane ^ 32, ^ 16, ..., ^ 1, in that order);
// every combine is commutative, so all lanes end with the same bits.
template <typename T>
__device__ __forceinline__ Acc<T> wave_allreduce(Acc<T> a) {
    a = Acc<T>::combine(a, butterfly_partner<32>(a));
    a = Acc<T>::combine(a, butterfly_partner<16>(a));
    a = Acc<T>::combine(a, butterfly_partner<8>(a));
    a = Acc<T>::combine(a, butterfly_partner<4>(a));
    a = Acc<T>::combine(a, butterfly_partner<2>(a));
    a = Acc<T>::combine(a, butterfly_partner<1>(a));
    return a;
}

// Largest value over the wave (exact; every lane ends with it).
template <typename T>
__device__ __forceinline__ T wave_max(T x) {
    T o = butterfly_partner<32>(x);
    x = o > x ? o : x;
    o = butterfly_partner<16>(x);
    x = o > x ? o : x;
    o = butterfly_partner<8>(x);
    x = o > x ? o : x;
    o = butterfly_partner<4>(x);
    x = o > x ? o : x;
    o = butterfly_partner<2>(x);
    x = o > x ? o : x;
    o = butterfly_partner<1>(x);
    return o > x ? o : x;
}

// --------------------------------------------------------------------------------------------
// occurrence loss of one event (Section III steps 1-3) for each layout
template <typename T, int LAYOUT>
struct Lookup;

template <typename T>
struct Lookup<T, kDirect> {
    __device__ __forceinline__ static T occ(int32_t E, const TablesView &tb, const Terms<T> &t) {
        const T *tab = static_cast<const T *>(tb.direct);
        EventSum<T> s;
        for (int j = 0; j < t.n_elts; ++j) {
            T l = tab[(size_t)j * (size_t)tb.catalog + (size_t)E];
            s.add(clamp_excess(l, t.ret[j], t.lim[j]));
        }
        return clamp_excess(s.value(), t.occ_ret, t.occ_lim);
    }
};

template <typename T>
struct Lookup<T, kSparse> {
    __device__ __forceinline__ static T occ(int32_t E, const TablesView &tb, const Terms<T> &t) {
        const T *loss = static_cast<const T *>(tb.sp_loss);
        EventSum<T> s;
        for (int j = 0; j < t.n_elts; ++j) {
            int64_t lo = tb.sp_off[j], n = tb.sp_off[j + 1] - lo;
            T l = T(0);
            if (n > 0) {
                // branch-free lower search: last index with id <= E
                int64_t base = lo;
                while (n > 1) {
                    int64_t half = n >> 1;
                    base = (tb.sp_ids[base + half] <= E) ? base + half : base;
                    n -= half;
                }
                if (tb.sp_ids[base] == E) l = loss[base];
            }
            s.add(clamp_excess(l, t.ret[j], t.lim[j]));
        }
        return clamp_excess(s.value(), t.occ_ret, t.occ_lim);
    }
};

template <typename T>
struct Lookup<T, kCompact> {
    __device__ __forceinline__ static T occ(int32_t E, const TablesView &tb, const Terms<T> &t) {
        uint2 w = tb.bm[E >> 5];
        uint32_t bit = 1u << (E & 31);
        if (!(w.x & bit)) return T(0);  // in no ELT: every x_j and o are 0
        int64_t idx = (int64_t)w.y + __popc(w.x & (bit - 1u));
        const T *row = static_cast<const T *>(tb.rows) + idx * t.n_elts;
        EventSum<T> s;
        for (int j = 0; j < t.n_elts; ++j) s.add(clamp_excess(row[j], t.ret[j], t.lim[j]));
        return clamp_excess(s.value(), t.occ_ret, t.occ_lim);
    }
};

template <typename T>
struct Lookup<T, kFused> {
    __device__ __forceinline__ static T occ(int32_t E, const TablesView &tb, const Terms<T> &) {
        return static_cast<const T *>(tb.occ)[E];
    }
};

// --------------------------------------------------------------------------------------------
// trial geometry
struct TrialRange {
    int64_t b, e;
};

__device__ __forceinline__ TrialRange trial_range(const YetView &y, int64_t i) {
    if (y.offsets) return TrialRange{y.offsets[i], y.offsets[i + 1]};
    return TrialRange{i * y.events_per_trial, (i + 1) * y.events_per_trial};
}

// Four consecutive event IDs from a 16-byte aligned address.  The YET is
// read once per pass, so its loads are marked non-temporal: they do not
// displace the layer's tables, which every trial reads again, from the caches.
__device__ __forceinline__ int4 stream_ids4(const int32_t *p) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(p));
    return make_int4(v.x, v.y, v.z, v.w);
}

// Four event IDs at positions p..p+3; positions outside [b, e) read as -1.
__device__ __forceinline__ void load4(const YetView &y, int64_t p, const TrialRange &r, int32_t id[4]) {
    if (p >= r.e) {
        id[0] = id[1] = id[2] = id[3] = -1;
    } else if (y.aligned16 && p >= r.b && p + 3 < r.e) {
        int4 v = stream_ids4(y.ids + p);
        id[0] = v.x; id[1] = v.y; id[2] = v.z; id[3] = v.w;
    } else if (y.aligned16 && p + 3 < y.n_events) {
        int4 v = stream_ids4(y.ids + p);
        id[0] = v.x; id[1] = v.y; id[2] = v.z; id[3] = v.w;
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4)
            if (p + v4 < r.b || p + v4 >= r.e) id[v4] = -1;
    } else {
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) {
            int64_t q = p + v4;
            id[v4] = (q >= r.b && q < r.e) ? y.ids[q] : -1;
        }
    }
}

__device__ __forceinline__ int64_t chunk_start(const YetView &y, int64_t b) { return ara::chunk_start(y.aligned16 != 0, b); }

// --------------------------------------------------------------------------------------------
// kernels
template <typename T, int LAYOUT>
// omax (optional): the largest occurrence loss of each trial.
__global__ __launch_bounds__(256) void k_trial_pass(YetView y, TablesView tb, Terms<T> t, double *__restrict__ ylt,
                                                    double *__restrict__ omax) {
    const int lane = lane_id();
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t trial = wave; trial < y.n_trials; trial += n_waves) {
        const TrialRange r = trial_range(y, trial);
        Acc<T> acc = Acc<T>::zero();
        T m = T(0);
        for (int64_t p = chunk_start(y, r.b) + 4 * lane; p < r.e; p += 4 * kWave) {
            int32_t id[4];
            load4(y, p, r, id);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (id[v] >= 0) {
                    const T o = Lookup<T, LAYOUT>::occ(id[v], tb, t);
                    acc.add(o);
                    m = o > m ? o : m;
                }
        }
        const double S = wave_allreduce(acc).value();
        if (lane == 0) ylt[trial] = clamp_excess(S, t.agg_ret, t.agg_lim);
        if (omax) {
            m = wave_max(m);
            if (lane == 0) omax[trial] = (double)m;
        }
    }
}

template <typename T, int LAYOUT>
__global__ __launch_bounds__(256) void k_trial_pass_events(YetView y, TablesView tb, Terms<T> t,
                                                           double *__restrict__ ylt, double *__restrict__ cum,
                                                           double *__restrict__ net) {
    const int lane = lane_id();
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t trial = wave; trial < y.n_trials; trial += n_waves) {
        const TrialRange r = trial_range(y, trial);
        Acc<T> carry = Acc<T>::zero();  // S after the previous chunk
        double carry_net = 0.0;          // A after the previous chunk
        for (int64_t c = chunk_start(y, r.b); c < r.e; c += 4 * kWave) {
            const int64_t p = c + 4 * lane;
            int32_t id[4];
            load4(y, p, r, id);
            Acc<T> pre[4];
            Acc<T> run = Acc<T>::zero();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (id[v] >= 0) run.add(Lookup<T, LAYOUT>::occ(id[v], tb, t));
                pre[v] = run;
            }
            const Acc<T> incl = wave_inclusive_scan(run);
            Acc<T> excl = shfl_acc(incl, lane > 0 ? lane - 1 : 0);
            if (lane == 0) excl = Acc<T>::zero();
            const Acc<T> base = Acc<T>::combine(carry, excl);
            double Sv[4], Av[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Sv[v] = Acc<T>::combine(base, pre[v]).value();
                Av[v] = clamp_excess(Sv[v], t.agg_ret, t.agg_lim);
            }
            // A before this lane's first event: the previous lane's last A
            double a_prev = __shfl(Av[3], lane > 0 ? lane - 1 : 0);
            if (lane == 0) a_prev = carry_net;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (id[v] >= 0) {
                    if (cum) cum[p + v] = Sv[v];
                    if (net) net[p + v] = Av[v] - a_prev;
                }
                a_prev = Av[v];
            }
            carry = Acc<T>::combine(base, pre[3]);
            carry = shfl_acc(carry, kWave - 1);
            carry_net = __shfl(Av[3], kWave - 1);
        }
        if (lane == 0) ylt[trial] = clamp_excess(carry.value(), t.agg_ret, t.agg_lim);
    }
}

// Fused layout: the pass needs one LDS filter probe per event and one gather
// of the precomputed occurrence loss only for events whose block is marked.
// A wave loads a whole group of kGroup chunks (kGroup * 256 events) of a
// trial at once and, before it works on the current trial, already issues the
// loads of its next trial, so every lane keeps 2 * kGroup 16-byte loads in
// flight.  Each lane still adds its events in the order of k_trial_pass (chunk
// by chunk, four consecutive events per chunk) and skipped events would add
// exactly zero, so the YLT is bitwise the one of the other layouts.
// kGroup is a build-time choice (-DARA_FUSED_GROUP=2|4|8, the same YLT
// bits): on MI355X four chunks are the fastest for fixed-length and ragged
// YETs in both precisions (two: 7 % and 25 % slower; eight: the fixed-length
// pass spills at the 128 VGPRs of 1024-thread groups and takes twice as long).
#ifndef ARA_FUSED_GROUP
#define ARA_FUSED_GROUP 4
#endif
constexpr int kGroup = ARA_FUSED_GROUP;

template <int G>
struct IdGroupT {
    int32_t id[G][4];
};
using IdGroup = IdGroupT<kGroup>;

// ID loads of the fused pass.  With a 16-byte aligned YET every lane issues
// its G 16-byte loads unconditionally (a conditional load makes the compiler
// wait for it inside the branch, which serialises the loads): the address is
// clamped to the trial's last 16-byte granule (for an empty trial and for
// FIXED, the YET's last one), so a lane past the end of its trial reads a
// line the wave has read already instead of the next trial's IDs, and
// positions outside the trial are masked afterwards (their IDs replaced by 0).
//   FIXED: every trial holds the same non-zero multiple of 4 events, so a
//          lane's four IDs are wholly inside or wholly past the trial.
//   !ALIGNED: element loads with bounds checks (slow path, any alignment).
template <bool FIXED, bool ALIGNED, int G = kGroup>
__device__ __forceinline__ uint32_t load_group(const YetView &y, const TrialRange &r, int64_t base, int lane,
                                               int64_t last_granule, IdGroupT<G> &g) {
    uint32_t valid = 0;  // bit 4c+v: element v of chunk c lies in the trial
    // (FIXED: a trial ends on a granule boundary; the YET-wide clamp costs
    // at most one granule per lane and no extra registers)
    const int64_t lim = load_limit(FIXED, r.b, r.e, last_granule);
#pragma unroll
    for (int c = 0; c < G; ++c) {
        const int64_t p = base + c * kChunkEvents + 4 * lane;
        if (ALIGNED) {
            const int4 v = stream_ids4(y.ids + clamped_granule(p, lim));
            g.id[c][0] = v.x; g.id[c][1] = v.y; g.id[c][2] = v.z; g.id[c][3] = v.w;
            const uint32_t m = granule_valid(FIXED, p, r.b, r.e);
            if (!FIXED) {
#pragma unroll
                for (int v4 = 0; v4 < 4; ++v4) g.id[c][v4] = ((m >> v4) & 1u) ? g.id[c][v4] : 0;
            }
            valid |= m << (4 * c);
        } else {
            load4(y, p, r, g.id[c]);
#pragma unroll
            for (int v4 = 0; v4 < 4; ++v4) {
                valid |= (g.id[c][v4] >= 0 ? 1u : 0u) << (4 * c + v4);
                g.id[c][v4] = g.id[c][v4] >= 0 ? g.id[c][v4] : 0;
            }
        }
    }
    return valid;
}

// The fused layout's LDS filters (see TablesView): block filter words, then
// hashed filter words.
struct FusedFilter {
    const uint32_t *filt;
    int32_t n_fwords;
    int32_t fshift;
    int32_t n_hwords;
    int32_t hshift;
};

__device__ __forceinline__ void load_filters(const FusedFilter &f, uint32_t *sfilt) {
    const int n = f.n_fwords + f.n_hwords;
    for (int i = threadIdx.x; i < n; i += blockDim.x) sfilt[i] = f.filt[i];
    __syncthreads();
}

// Lane mask of bit b of w: all ones if set, else 0 (one signed bit-field
// extract; only the low five bits of b count).
__device__ __forceinline__ uint32_t bit_mask(uint32_t w, uint32_t b) {
    return (uint32_t)__builtin_amdgcn_sbfe((int)w, b, 1u);
}

// Occurrence losses of a group: LDS filter probes per event, then a gather
// for every event -- of occ[E] where E passes the filters, else of the zero
// at occ[catalog] -- so no load sits under a branch.  The block filter has
// no false negatives, and neither has the hashed one (HASH), so an event
// that fails either has occ[E] = 0.  Each probe and the in-trial bit give a
// lane mask; the gathered index is the ID under their conjunction, else the
// zero slot.  WHOLE: the in-trial bits of a chunk are all set or all clear
// (fixed-length trials).  OFF32: every byte offset into the table fits in
// 32 bits (a gather is then the table's base plus a 32-bit offset).
template <typename T, bool HASH, bool WHOLE, int G = kGroup, bool OFF32 = false>
__device__ __forceinline__ void gather_group(const IdGroupT<G> &g, uint32_t valid, const uint32_t *sfilt,
                                             const FusedFilter &f, int32_t zero_slot, const T *__restrict__ occ,
                                             T (&o)[G][4]) {
    const uint32_t *shash = sfilt + f.n_fwords;
    uint32_t idx[G][4];
#pragma unroll
    for (int c = 0; c < G; ++c) {
        const uint32_t cm = bit_mask(valid, 4u * c);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint32_t id = (uint32_t)g.id[c][v];
            uint32_t m = bit_mask(sfilt[id >> (f.fshift + 5)], id) & (WHOLE ? cm : bit_mask(valid, 4u * c + v));
            if (HASH) m &= bit_mask(shash[hash_word(id, f.hshift)], id);
            idx[c][v] = (id & m) | ((uint32_t)zero_slot & ~m);
        }
    }
#pragma unroll
    for (int c = 0; c < G; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (OFF32)
                o[c][v] = *reinterpret_cast<const T *>(reinterpret_cast<const char *>(occ) +
                                                       (idx[c][v] * (uint32_t)sizeof(T)));
            else
                o[c][v] = occ[idx[c][v]];
        }
}

// The i-th of a lane's 4G IDs (i < 4G; chunk i / 4, element i % 4), chosen
// by a binary tree of selects on the bits of i.
template <int G>
__device__ __forceinline__ uint32_t select_id(const IdGroupT<G> &g, uint32_t i) {
    constexpr int N = 4 * G;
    uint32_t s[N];
#pragma unroll
    for (int k = 0; k < N; ++k) s[k] = (uint32_t)g.id[k >> 2][k & 3];
#pragma unroll
    for (int n = N / 2, b = 0; n >= 1; n >>= 1, ++b) {
        const bool hi = ((i >> b) & 1u) != 0u;
#pragma unroll
        for (int k = 0; k < n; ++k) s[k] = hi ? s[2 * k + 1] : s[2 * k];
    }
    return s[0];
}

// Gathers of a group, compacted per lane: the filter probes give each lane a
// mask of its events that pass (bit 4c + v, the lane's event order); the
// lane then gathers only those, its first kHits of them in kHits gather
// instructions (the zero slot where it has fewer), the rest one at a time
// while any lane of the wave has some left.  They are added to acc in the
// lane's event order, as the uncompacted form adds every event (the events
// skipped would add exact zeros), so the sums are bitwise the same.  OMAX:
// their largest into mx.
template <int G>
struct CompactHits;
template <>
struct CompactHits<1> {
    static constexpr int k = 2;
};
template <>
struct CompactHits<2> {
    static constexpr int k = 3;
};
template <>
struct CompactHits<4> {
    static constexpr int k = 4;
};
template <>
struct CompactHits<8> {
    static constexpr int k = 6;
};

template <typename T, bool OFF32>
__device__ __forceinline__ T gather_one(const T *__restrict__ occ, uint32_t idx) {
    if (OFF32) return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(occ) + idx * (uint32_t)sizeof(T));
    return occ[idx];
}

// Phase one: the probes, the lane's mask of passing events and its first
// kHits gathers (issued, not waited for).
template <typename T, int G>
struct HitGathers {
    T x[CompactHits<G>::k];
    uint32_t pass;  // passing events not yet gathered
};

// A lane's events of a group that lie in the trial and pass the LDS
// filters: bit 4c + v for element v of chunk c.
template <bool HASH, bool WHOLE, int G>
__device__ __forceinline__ uint32_t pass_mask(const IdGroupT<G> &g, uint32_t valid, const uint32_t *sfilt,
                                              const FusedFilter &f) {
    static_assert(4 * G <= 32, "one mask bit per event of a lane");
    const uint32_t *shash = sfilt + f.n_fwords;
    uint32_t pass = 0;
#pragma unroll
    for (int c = 0; c < G; ++c) {
        const uint32_t cm = bit_mask(valid, 4u * c);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint32_t id = (uint32_t)g.id[c][v];
            uint32_t m = bit_mask(sfilt[id >> (f.fshift + 5)], id) & (WHOLE ? cm : bit_mask(valid, 4u * c + v));
            if (HASH) m &= bit_mask(shash[hash_word(id, f.hshift)], id);
            pass |= m & (1u << (4 * c + v));
        }
    }
    return pass;
}

// Position (0 .. 4G - 1) of the lowest set bit of a non-empty mask (some
// position below 4G for an empty one; its lanes gather the zero slot).
template <int G>
__device__ __forceinline__ uint32_t first_pass(uint32_t pass) {
    static_assert(4 * G <= 32, "one mask bit per event of a lane");
    return (uint32_t)__builtin_ctz(pass | 0x80000000u) & (4 * G - 1);
}

template <typename T, bool HASH, bool WHOLE, int G, bool OFF32>
__device__ __forceinline__ void gather_hits(const IdGroupT<G> &g, uint32_t valid, const uint32_t *sfilt,
                                            const FusedFilter &f, int32_t zero_slot, const T *__restrict__ occ,
                                            HitGathers<T, G> &h) {
    uint32_t pass = pass_mask<HASH, WHOLE, G>(g, valid, sfilt, f);
#pragma unroll
    for (int k = 0; k < CompactHits<G>::k; ++k) {
        h.x[k] = gather_one<T, OFF32>(occ, pass ? select_id<G>(g, first_pass<G>(pass)) : (uint32_t)zero_slot);
        pass &= pass - 1u;
    }
    h.pass = pass;
}

template <typename T, bool OMAX>
__device__ __forceinline__ void add_hit(T x, Acc<T> &acc, T &mx) {
    if (sizeof(T) == 8) {
        acc.add(x);
    } else if (x != T(0)) {
        acc.add(x);
    }
    if (OMAX) mx = x > mx ? x : mx;
}

// Phase two: the sums in the lane's event order, then the lane's remaining
// passing events one gather at a time while any lane of the wave has some.
template <typename T, int G, bool OFF32, bool OMAX>
__device__ __forceinline__ void sum_hits(const IdGroupT<G> &g, HitGathers<T, G> &h, int32_t zero_slot,
                                         const T *__restrict__ occ, Acc<T> &acc, T &mx) {
#pragma unroll
    for (int k = 0; k < CompactHits<G>::k; ++k) add_hit<T, OMAX>(h.x[k], acc, mx);
    uint32_t pass = h.pass;
    while (__builtin_amdgcn_ballot_w64(pass != 0u)) {
        const T x = gather_one<T, OFF32>(occ, pass ? select_id<G>(g, first_pass<G>(pass)) : (uint32_t)zero_slot);
        pass &= pass - 1u;
        add_hit<T, OMAX>(x, acc, mx);
    }
}

// Adds in k_trial_pass order; adding an exact zero changes no bit of the sum.
template <typename T, int G = kGroup>
__device__ __forceinline__ void accumulate_group(const T (&o)[G][4], Acc<T> &acc) {
#pragma unroll
    for (int c = 0; c < G; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (sizeof(T) == 8) {
                acc.add(o[c][v]);
            } else if (o[c][v] != T(0)) {
                acc.add(o[c][v]);
            }
        }
}

// Largest of a group's occurrence losses (skipped events hold exact zeros,
// and every occurrence loss is >= 0).
template <typename T, int G = kGroup>
__device__ __forceinline__ void max_group(const T (&o)[G][4], T &m) {
#pragma unroll
    for (int c = 0; c < G; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) m = o[c][v] > m ? o[c][v] : m;
}

// Trial bounds; fixed-length trials (off == nullptr) need not be FIXED: their
// length may not be a multiple of 4 or the IDs may be unaligned.
template <bool FIXED>
__device__ __forceinline__ TrialRange fused_range(const YetView &y, const int64_t *__restrict__ off, int64_t i) {
    if (FIXED || off == nullptr) return TrialRange{i * y.events_per_trial, (i + 1) * y.events_per_trial};
    return TrialRange{off[i], off[i + 1]};
}

// One trial of k_trial_pass_fused: its first group's IDs are in cur; the
// next trial's range and first group are loaded into rn / nxt on the way.
// Returns the next trial.
template <typename T, bool FIXED, bool ALIGNED, bool HASH, int G, bool OMAX, bool OFF32>
__device__ __forceinline__ int64_t fused_trial(const YetView &y, const int64_t *__restrict__ off, const FusedFilter &f,
                                               const uint32_t *sfilt, int32_t zero_slot, const T *__restrict__ occ,
                                               double agg_ret, double agg_lim, double *__restrict__ ylt,
                                               double *__restrict__ omax, int64_t trial, int64_t n_waves, int lane,
                                               int64_t last_granule, const TrialRange &r, const IdGroupT<G> &cur,
                                               uint32_t cur_valid, TrialRange &rn, IdGroupT<G> &nxt,
                                               uint32_t &nxt_valid) {
    constexpr int64_t kSpan = (int64_t)G * 4 * kWave;
    // gathers of this trial first, then the IDs of the next trial, so
    // that waiting for the gathers does not wait for the prefetch
    HitGathers<T, G> hits;
    gather_hits<T, HASH, FIXED, G, OFF32>(cur, cur_valid, sfilt, f, zero_slot, occ, hits);
    // the last round of a wave loads its own last trial again (unused)
    const int64_t next = trial + n_waves;
    const int64_t pre = next < y.n_trials ? next : trial;
    rn = fused_range<FIXED>(y, off, pre);
    nxt_valid = load_group<FIXED, ALIGNED, G>(y, rn, chunk_start(y, rn.b), lane, last_granule, nxt);
    Acc<T> acc = Acc<T>::zero();
    T m = T(0);
    sum_hits<T, G, OFF32, OMAX>(cur, hits, zero_slot, occ, acc, m);
    // the rest of a longer trial: whole groups for fixed-length trials,
    // single chunks for variable-length ones (a Poisson(1000) trial
    // exceeds a group by less than a chunk or two; a second group of
    // registers would also cost occupancy-relevant VGPRs); each lane
    // still adds its chunks in increasing order
    constexpr int TG = FIXED ? G : 1;
    for (int64_t base = chunk_start(y, r.b) + kSpan; base < r.e; base += (int64_t)TG * 4 * kWave) {
        IdGroupT<TG> more;
        const uint32_t mv = load_group<FIXED, ALIGNED, TG>(y, r, base, lane, last_granule, more);
        HitGathers<T, TG> mh;
        gather_hits<T, HASH, FIXED, TG, OFF32>(more, mv, sfilt, f, zero_slot, occ, mh);
        sum_hits<T, TG, OFF32, OMAX>(more, mh, zero_slot, occ, acc, m);
    }
    const double S = wave_allreduce(acc).value();
    if (lane == 0) ylt[trial] = clamp_excess(S, agg_ret, agg_lim);
    if (OMAX) {
        m = wave_max(m);
        if (lane == 0) omax[trial] = (double)m;
    }
    return next;
}

// OMAX: also the largest occurrence loss of each trial, into omax.  A
// wave's trials alternate between two sets of ID registers (the one being
// summed, the one being prefetched), so no IDs are copied between trials.
// OFF32: (catalog + 1) * sizeof(T) <= 2^32.
template <typename T, bool FIXED, bool ALIGNED, bool HASH, int G, bool OMAX, bool OFF32>
__global__ __launch_bounds__(1024) void k_trial_pass_fused(YetView y, const int64_t *__restrict__ off, FusedFilter f,
                                                           int32_t zero_slot, const T *__restrict__ occ,
                                                           double agg_ret, double agg_lim,
                                                           double *__restrict__ ylt, double *__restrict__ omax) {
    extern __shared__ uint32_t sfilt[];
    load_filters(f, sfilt);
    const int lane = lane_id();
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t last_granule = (y.n_events - 1) & ~3LL;  // launched only with n_events >= 1
    int64_t trial = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    TrialRange r0{0, 0}, r1{0, 0};
    IdGroupT<G> g0, g1;
    uint32_t v0 = 0, v1 = 0;
    if (trial < y.n_trials) {
        r0 = fused_range<FIXED>(y, off, trial);
        v0 = load_group<FIXED, ALIGNED, G>(y, r0, chunk_start(y, r0.b), lane, last_granule, g0);
    }
    while (trial < y.n_trials) {
        trial = fused_trial<T, FIXED, ALIGNED, HASH, G, OMAX, OFF32>(y, off, f, sfilt, zero_slot, occ, agg_ret, agg_lim, ylt,
                                                              omax, trial, n_waves, lane, last_granule, r0, g0, v0,
                                                              r1, g1, v1);
        if (trial >= y.n_trials) break;
        trial = fused_trial<T, FIXED, ALIGNED, HASH, G, OMAX, OFF32>(y, off, f, sfilt, zero_slot, occ, agg_ret, agg_lim, ylt,
                                                              omax, trial, n_waves, lane, last_granule, r1, g1, v1,
                                                              r0, g0, v0);
    }
}

// Per-event outputs with the fused layout: the loads, LDS filter and gathers
// of k_trial_pass_fused, then, chunk by chunk, the scan of k_trial_pass_events
// (same chunks, same lane order, same combine tree), so the outputs are
// bitwise those of the generic per-event pass.
template <typename T, bool FIXED, bool ALIGNED, bool HASH, int G>
__global__ __launch_bounds__(1024) void k_trial_pass_events_fused(
    YetView y, const int64_t *__restrict__ off, FusedFilter f, int32_t zero_slot, const T *__restrict__ occ,
    double agg_ret, double agg_lim, double *__restrict__ ylt, double *__restrict__ cum, double *__restrict__ net) {
    extern __shared__ uint32_t sfilt[];
    load_filters(f, sfilt);
    const int lane = lane_id();
    // both outputs 32-byte aligned (a missing one counts as aligned)
    const bool out32 = ((reinterpret_cast<uintptr_t>(cum) | reinterpret_cast<uintptr_t>(net)) & 31u) == 0;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    constexpr int64_t kSpan = (int64_t)G * 4 * kWave;
    const int64_t last_granule = (y.n_events - 1) & ~3LL;  // launched only with n_events >= 1
    int64_t trial = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    TrialRange r{0, 0};
    IdGroupT<G> cur;
    uint32_t cur_valid = 0;
    if (trial < y.n_trials) {
        r = fused_range<FIXED>(y, off, trial);
        cur_valid = load_group<FIXED, ALIGNED, G>(y, r, chunk_start(y, r.b), lane, last_granule, cur);
    }
    while (trial < y.n_trials) {
        T o[G][4];
        gather_group<T, HASH, FIXED, G>(cur, cur_valid, sfilt, f, zero_slot, occ, o);
        const int64_t next = trial + n_waves;
        const TrialRange rn = fused_range<FIXED>(y, off, next < y.n_trials ? next : trial);
        IdGroupT<G> nxt;
        const uint32_t nxt_valid = load_group<FIXED, ALIGNED, G>(y, rn, chunk_start(y, rn.b), lane, last_granule, nxt);
        Acc<T> carry = Acc<T>::zero();
        double carry_net = 0.0;
        int64_t base = chunk_start(y, r.b);
        uint32_t valid = cur_valid;
        while (true) {
#pragma unroll
            for (int c = 0; c < G; ++c) {
                const int64_t p = base + c * 4 * kWave + 4 * lane;
                Acc<T> pre[4];
                Acc<T> run = Acc<T>::zero();
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if ((valid >> (4 * c + v)) & 1u) run.add(o[c][v]);
                    pre[v] = run;
                }
                const Acc<T> incl = wave_inclusive_scan(run);
                Acc<T> excl = shfl_acc(incl, lane > 0 ? lane - 1 : 0);
                if (lane == 0) excl = Acc<T>::zero();
                const Acc<T> sbase = Acc<T>::combine(carry, excl);
                double Sv[4], Av[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    Sv[v] = Acc<T>::combine(sbase, pre[v]).value();
                    Av[v] = clamp_excess(Sv[v], agg_ret, agg_lim);
                }
                double a_prev = __shfl(Av[3], lane > 0 ? lane - 1 : 0);
                if (lane == 0) a_prev = carry_net;
                double nv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    nv[v] = Av[v] - a_prev;
                    a_prev = Av[v];
                }
                // a lane's four events in one 32-byte piece of each output:
                // two 16-byte stores, else one store per event in the trial
                const uint32_t nib = (valid >> (4 * c)) & 0xfu;
                if (out32 && nib == 0xfu && (p & 3) == 0) {
                    if (cum) {
                        reinterpret_cast<double2 *>(cum + p)[0] = make_double2(Sv[0], Sv[1]);
                        reinterpret_cast<double2 *>(cum + p)[1] = make_double2(Sv[2], Sv[3]);
                    }
                    if (net) {
                        reinterpret_cast<double2 *>(net + p)[0] = make_double2(nv[0], nv[1]);
                        reinterpret_cast<double2 *>(net + p)[1] = make_double2(nv[2], nv[3]);
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if ((nib >> v) & 1u) {
                            if (cum) cum[p + v] = Sv[v];
                            if (net) net[p + v] = nv[v];
                        }
                    }
                }
                carry = shfl_acc(Acc<T>::combine(sbase, pre[3]), kWave - 1);
                carry_net = __shfl(Av[3], kWave - 1);
            }
            base += kSpan;
            if (base >= r.e) break;
            IdGroupT<G> more;
            valid = load_group<FIXED, ALIGNED, G>(y, r, base, lane, last_granule, more);
            gather_group<T, HASH, FIXED, G>(more, valid, sfilt, f, zero_slot, occ, o);
        }
        if (lane == 0) ylt[trial] = clamp_excess(carry.value(), agg_ret, agg_lim);
        trial = next;
        r = rn;
        cur = nxt;
        cur_valid = nxt_valid;
    }
}

// --------------------------------------------------------------------------------------------
// batched pass: many layers, one read of the YET

template <typename T>
struct alignas(RecFormat<T>::kBytes) Record {
    uint8_t lid[8];
    T val[RecFormat<T>::kVals];
};
static_assert(sizeof(Record<double>) == 64 && sizeof(Record<float>) == 32, "record size");

struct OccPtrs {
    const void *p[ARA_MAX_BATCH];
};

// An event's overflow entries start on a multiple of four in the overflow
// arrays and take whole blocks of four (the pipelined pass reads a block's
// four layer indices as one 32-bit word and its values as 16-byte loads).
__device__ __forceinline__ int ovf_span(int n) { return (n + 3) & ~3; }

template <typename T>
__global__ void k_batch_count(OccPtrs occ, int32_t n_layers, int32_t catalog, int32_t *__restrict__ count,
                              unsigned long long *ovf_total) {
    constexpr int KV = RecFormat<T>::kVals;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < catalog; e += (int64_t)gridDim.x * blockDim.x) {
        int n = 0;
        for (int l = 0; l < n_layers; ++l) n += static_cast<const T *>(occ.p[l])[e] != T(0);
        count[e] = n;
        if (n > KV) atomicAdd(ovf_total, (unsigned long long)ovf_span(n - (KV - 1)));
    }
}

template <typename T>
__global__ void k_batch_fill(OccPtrs occ, int32_t n_layers, int32_t catalog, const int32_t *__restrict__ count,
                             Record<T> *__restrict__ rec, uint8_t *__restrict__ ovf_lid, T *__restrict__ ovf_val,
                             unsigned long long *cursor) {
    constexpr int KV = RecFormat<T>::kVals;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < catalog; e += (int64_t)gridDim.x * blockDim.x) {
        Record<T> r;
#pragma unroll
        for (int k = 0; k < 8; ++k) r.lid[k] = kNoLayer;
#pragma unroll
        for (int k = 0; k < KV; ++k) r.val[k] = T(0);
        const int n = count[e];
        const bool ovf = n > KV;
        const int n_in = ovf ? KV - 1 : KV;
        unsigned long long pos = 0;
        if (ovf) pos = atomicAdd(cursor, (unsigned long long)ovf_span(n - n_in));
        int k = 0;
        for (int l = 0; l < n_layers; ++l) {
            const T v = static_cast<const T *>(occ.p[l])[e];
            if (v == T(0)) continue;
            if (k < n_in) {
                r.lid[k] = (uint8_t)l;
                r.val[k] = v;
            } else {
                ovf_lid[pos + (k - n_in)] = (uint8_t)l;
                ovf_val[pos + (k - n_in)] = v;
            }
            ++k;
        }
        if (ovf) {
            // the padding of the event's last block of four
            for (int q = k - n_in; q < ovf_span(n - n_in); ++q) {
                ovf_lid[pos + q] = kNoLayer;
                ovf_val[pos + q] = T(0);
            }
            r.lid[7] = kOverflowMark;
            r.lid[KV - 1] = (uint8_t)(n - n_in);
            const uint32_t p32 = (uint32_t)pos;
            __builtin_memcpy(&r.val[KV - 1], &p32, sizeof(p32));
        }
        rec[e] = r;
    }
}

// Row stride of the per-wave accumulator table acc[layer][lane] (one spare
// slot per row keeps the epilogue's row reads off a single LDS bank).
constexpr int kAccStride = kWave + 1;

template <typename T>
__device__ __forceinline__ void acc_add(Acc<T> *acc, uint32_t l, int lane, T v) {
    Acc<T> a = acc[l * kAccStride + lane];
    a.add(v);
    acc[l * kAccStride + lane] = a;
}

// The overflow entries of the four events a lane holds in one chunk: the
// first kOvPre of each are requested together (at clamped indices, slot 0
// for events without overflow), so a chunk waits for one round trip rather
// than one per entry.
constexpr int kOvPre = 4;

template <typename T>
struct OvHeads {
    uint32_t pos[4];
    int cnt[4];
    int32_t lid[4][kOvPre];
    T val[4][kOvPre];
};

template <typename T>
__device__ __forceinline__ void load_ov_heads(const Record<T> (&rr)[4], uint32_t valid4, const BatchTables &b,
                                              OvHeads<T> &h) {
    constexpr int KV = RecFormat<T>::kVals;
    const T *ov = static_cast<const T *>(b.ovf_val);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const bool ovf = ((valid4 >> v) & 1u) && rr[v].lid[7] == kOverflowMark;
        uint32_t pos;
        __builtin_memcpy(&pos, &rr[v].val[KV - 1], sizeof(pos));
        h.pos[v] = ovf ? pos : 0u;
        h.cnt[v] = ovf ? (int)rr[v].lid[KV - 1] : 0;
#pragma unroll
        for (int j = 0; j < kOvPre; ++j) {
            const uint32_t i = h.pos[v] + (j < h.cnt[v] ? (uint32_t)j : 0u);
            h.lid[v][j] = b.ovf_lid[i];
            h.val[v][j] = ov[i];
        }
    }
}

// Adds one event's entries: the inline ones, then its overflow entries in
// order (the prefetched heads, then any further ones).
template <typename T>
__device__ __forceinline__ void add_event(const Record<T> &r, bool valid, const OvHeads<T> &h, int v, Acc<T> *acc,
                                          int lane, const BatchTables &b) {
    constexpr int KV = RecFormat<T>::kVals;
    if (!valid) return;
    const bool ovf = r.lid[7] == kOverflowMark;
    const int n_in = ovf ? KV - 1 : KV;
#pragma unroll
    for (int k = 0; k < KV; ++k)
        if (k < n_in && r.lid[k] != kNoLayer) acc_add(acc, r.lid[k], lane, r.val[k]);
#pragma unroll
    for (int j = 0; j < kOvPre; ++j)
        if (j < h.cnt[v]) acc_add(acc, (uint32_t)h.lid[v][j], lane, h.val[v][j]);
    // further entries, kOvPre at a time (requested together, added in order)
    const T *ov = static_cast<const T *>(b.ovf_val);
    for (int i0 = kOvPre; i0 < h.cnt[v]; i0 += kOvPre) {
        int32_t lid[kOvPre];
        T val[kOvPre];
#pragma unroll
        for (int j = 0; j < kOvPre; ++j) {
            const uint32_t i = h.pos[v] + (uint32_t)(i0 + j < h.cnt[v] ? i0 + j : i0);
            lid[j] = b.ovf_lid[i];
            val[j] = ov[i];
        }
#pragma unroll
        for (int j = 0; j < kOvPre; ++j)
            if (i0 + j < h.cnt[v]) acc_add(acc, (uint32_t)lid[j], lane, val[j]);
    }
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per trial (same lane-to-event mapping and per-lane order as the
// single-layer passes).  Every record entry (layer l, loss o) of an event
// handled by lane i is added to acc[l][i]; at the end of the trial lane l
// folds row l with the butterfly order of wave_allreduce, so layer l's YLT is
// bitwise the one of its own pass.
template <typename T, bool FIXED, bool ALIGNED, int G>
__global__ __launch_bounds__(512) void k_trial_pass_batch(YetView y, const int64_t *__restrict__ off, BatchTables b) {
    extern __shared__ uint64_t lds_raw[];
    const int lane = lane_id();
    const int n_layers = b.n_layers;
    Acc<T> *acc = reinterpret_cast<Acc<T> *>(lds_raw) + (size_t)(threadIdx.x >> 6) * n_layers * kAccStride;
    const Record<T> *__restrict__ rec = static_cast<const Record<T> *>(b.rec);
    double *my_ylt = nullptr;
    double my_ret = 0.0, my_lim = 0.0;
    if (lane < n_layers) {
        my_ylt = b.ylts[lane];
        my_ret = b.agg_ret[lane];
        my_lim = b.agg_lim[lane];
    }
    for (int l = 0; l < n_layers; ++l) acc[l * kAccStride + lane] = Acc<T>::zero();
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    constexpr int64_t kSpan = (int64_t)G * kChunkEvents;
    const int64_t last_granule = (y.n_events - 1) & ~3LL;  // launched only with n_events >= 1
    int64_t trial = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    TrialRange r{0, 0};
    IdGroupT<G> cur;
    uint32_t cur_valid = 0;
    if (trial < y.n_trials) {
        r = fused_range<FIXED>(y, off, trial);
        cur_valid = load_group<FIXED, ALIGNED, G>(y, r, chunk_start(y, r.b), lane, last_granule, cur);
    }
    while (trial < y.n_trials) {
        const int64_t next = trial + n_waves;
        const TrialRange rn = fused_range<FIXED>(y, off, next < y.n_trials ? next : trial);
        IdGroupT<G> nxt;
        const uint32_t nxt_valid = load_group<FIXED, ALIGNED, G>(y, rn, chunk_start(y, rn.b), lane, last_granule, nxt);
        // records double-buffered across chunks: the loads of chunk c + 1 are
        // in flight while chunk c is added to the accumulators
        int64_t base = chunk_start(y, r.b);
        IdGroupT<G> g = cur;
        uint32_t valid = cur_valid;
        Record<T> rr[2][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) rr[0][v] = rec[g.id[0][v]];
        while (true) {
#pragma unroll
            for (int c = 0; c < G; ++c) {
                // chunks that start past the trial's end hold no event (a
                // variable-length trial's last group is mostly such padding)
                if (c > 0 && base + (int64_t)c * 4 * kWave >= r.e) break;
                OvHeads<T> oh;
                load_ov_heads(rr[c & 1], (valid >> (4 * c)) & 0xfu, b, oh);
                if (c + 1 < G) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) rr[(c + 1) & 1][v] = rec[g.id[c + 1][v]];
                }
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    add_event(rr[c & 1][v], ((valid >> (4 * c + v)) & 1u) != 0u, oh, v, acc, lane, b);
            }
            base += kSpan;
            if (base >= r.e) break;
            valid = load_group<FIXED, ALIGNED, G>(y, r, base, lane, last_granule, g);
#pragma unroll
            for (int v = 0; v < 4; ++v) rr[0][v] = rec[g.id[0][v]];
        }
        wave_lds_fence();
        if (lane < n_layers) {
            const Acc<T> *row = acc + lane * kAccStride;
            Acc<T> v[kWave / 2];
#pragma unroll
            for (int i = 0; i < kWave / 2; ++i) v[i] = Acc<T>::combine(row[i], row[i + kWave / 2]);
#pragma unroll
            for (int m = kWave / 4; m >= 1; m >>= 1)
#pragma unroll
                for (int i = 0; i < m; ++i) v[i] = Acc<T>::combine(v[i], v[i + m]);
            my_ylt[trial] = clamp_excess(v[0].value(), my_ret, my_lim);
        }
        wave_lds_fence();
        for (int l = 0; l < n_layers; ++l) acc[l * kAccStride + lane] = Acc<T>::zero();
        trial = next;
        r = rn;
        cur = nxt;
        cur_valid = nxt_valid;
    }
}

// --------------------------------------------------------------------------------------------
// pipelined batched pass: the same records, sums and lane order as
// k_trial_pass_batch, with the loads of a wave's chunks staged so that no
// step waits for a load issued in the same step.  A wave walks the chunks
// of its trials as one sequence (an empty trial counts as one chunk without
// events); at step k it
//   1. requests the first overflow block of every event of chunk k + 1
//      (whose records arrived),
//   2. requests the records of chunk k + 2 (whose IDs arrived),
//   3. requests the IDs of chunk k + 3,
//   4. adds chunk k's entries to the per-lane accumulators and, after a
//      trial's last chunk, writes its year losses.
// Every load is consumed one step after it was issued, so the step's LDS
// work hides its latency.  Three rotating slots hold a chunk each.

// First block of four overflow entries of an event.
template <typename T>
struct OvBlock {
    uint32_t lid4;  // layer index of entry j in bits 8j .. 8j + 7
    T val[4];
};

template <typename T>
__device__ __forceinline__ void load_ov_block(const BatchTables &b, uint32_t pos, OvBlock<T> &o) {
    o.lid4 = *reinterpret_cast<const uint32_t *>(b.ovf_lid + pos);
    if (sizeof(T) == 8) {
        const double2 *v = reinterpret_cast<const double2 *>(static_cast<const double *>(b.ovf_val) + pos);
        const double2 a = v[0], c = v[1];
        o.val[0] = (T)a.x; o.val[1] = (T)a.y; o.val[2] = (T)c.x; o.val[3] = (T)c.y;
    } else {
        const float4 a = *reinterpret_cast<const float4 *>(static_cast<const float *>(b.ovf_val) + pos);
        o.val[0] = (T)a.x; o.val[1] = (T)a.y; o.val[2] = (T)a.z; o.val[3] = (T)a.w;
    }
}

// Overflow start and count of an event's record (0, 0 without overflow).
template <typename T>
__device__ __forceinline__ void ov_of(const Record<T> &r, uint32_t &pos, int &cnt) {
    constexpr int KV = RecFormat<T>::kVals;
    const bool ovf = r.lid[7] == kOverflowMark;
    uint32_t p;
    __builtin_memcpy(&p, &r.val[KV - 1], sizeof(p));
    pos = ovf ? p : 0u;
    cnt = ovf ? (int)r.lid[KV - 1] : 0;
}

template <typename T>
struct StreamSlot {
    int32_t id[4];      // IDs of the chunk whose records are requested next
    uint32_t nvalid;    // their in-trial mask
    uint32_t valid;     // mask of the chunk whose records are in rr
    Record<T> rr[4];
    OvBlock<T> ob[4];
    int64_t ntrial, trial;  // trial of the chunk of id / of rr (-1: no chunk)
    int nlast, last;        // that chunk ends its trial
};

// A wave's walk over the chunks of its trials.
struct ChunkCursor {
    int64_t trial;  // trial of the next chunk (>= n_trials: done)
    int64_t base;   // its first position
    TrialRange r;
};

template <bool FIXED>
__device__ __forceinline__ void cursor_enter(const YetView &y, const int64_t *__restrict__ off, ChunkCursor &cc) {
    if (cc.trial < y.n_trials) {
        cc.r = fused_range<FIXED>(y, off, cc.trial);
        cc.base = chunk_start(y, cc.r.b);
    }
}

// Step 3: the next chunk's IDs into s (raw: masked when its records are
// requested), its mask and trial; advances the cursor.
template <typename T, bool FIXED, bool ALIGNED>
__device__ __forceinline__ void stream_next(const YetView &y, const int64_t *__restrict__ off, ChunkCursor &cc,
                                            int64_t n_waves, int lane, int64_t last_granule, StreamSlot<T> &s) {
    if (cc.trial >= y.n_trials) {
        s.ntrial = -1;
        s.nlast = 0;
        s.nvalid = 0;
        return;
    }
    const int64_t p = cc.base + 4 * lane;
    if (ALIGNED) {
        const int64_t lim = load_limit(FIXED, cc.r.b, cc.r.e, last_granule);
        const int4 v = stream_ids4(y.ids + clamped_granule(p, lim));
        s.id[0] = v.x; s.id[1] = v.y; s.id[2] = v.z; s.id[3] = v.w;
        s.nvalid = granule_valid(FIXED, p, cc.r.b, cc.r.e);
    } else {
        // element loads at in-trial positions (else the trial's first, or
        // the YET's first element for an empty trial), masked afterwards
        const int64_t safe = cc.r.e > cc.r.b ? cc.r.b : 0;
        uint32_t m = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t q = p + v;
            const bool in = q >= cc.r.b && q < cc.r.e;
            s.id[v] = y.ids[in ? q : safe];
            m |= (in ? 1u : 0u) << v;
        }
        s.nvalid = m;
    }
    s.ntrial = cc.trial;
    cc.base += kChunkEvents;
    s.nlast = cc.base >= cc.r.e ? 1 : 0;
    if (s.nlast) {
        cc.trial += n_waves;
        cursor_enter<FIXED>(y, off, cc);
    }
}

// Step 2: records of the slot's chunk (events outside the trial read the
// record of event 0 and are never added).
template <typename T>
__device__ __forceinline__ void stream_records(const Record<T> *__restrict__ rec, StreamSlot<T> &s) {
    s.valid = s.nvalid;
    s.trial = s.ntrial;
    s.last = s.nlast;
#pragma unroll
    for (int v = 0; v < 4; ++v) s.rr[v] = rec[((s.valid >> v) & 1u) ? s.id[v] : 0];
}

// Step 1: first overflow block of each event (block 0 for events without).
template <typename T>
__device__ __forceinline__ void stream_heads(const BatchTables &b, StreamSlot<T> &s) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        uint32_t pos;
        int cnt;
        ov_of(s.rr[v], pos, cnt);
        load_ov_block(b, ((s.valid >> v) & 1u) ? pos : 0u, s.ob[v]);
    }
}

// Adds a batch of entries with distinct layers: every accumulator is read
// before any is written, so the reads are in flight together.
template <typename T, int N>
__device__ __forceinline__ void add_distinct(Acc<T> *acc, int lane, const bool (&act)[N], const uint32_t (&lid)[N],
                                             const T (&val)[N]) {
    Acc<T> a[N];
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (act[k]) a[k] = acc[lid[k] * kAccStride + lane];
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (act[k]) {
            a[k].add(val[k]);
            acc[lid[k] * kAccStride + lane] = a[k];
        }
}

// Step 4: the chunk's events in lane order; an event's entries (inline,
// first overflow block, further blocks) hold distinct layers.
template <typename T>
__device__ __forceinline__ void stream_add(const BatchTables &b, const StreamSlot<T> &s, Acc<T> *acc, int lane) {
    constexpr int KV = RecFormat<T>::kVals;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const Record<T> &r = s.rr[v];
        const bool in = ((s.valid >> v) & 1u) != 0u;
        uint32_t pos;
        int cnt;
        ov_of(r, pos, cnt);
        const int n_in = cnt > 0 ? KV - 1 : KV;
        bool act[KV + 4];
        uint32_t lid[KV + 4];
        T val[KV + 4];
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            act[k] = in && k < n_in && r.lid[k] != kNoLayer;
            lid[k] = r.lid[k];
            val[k] = r.val[k];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            act[KV + j] = in && j < cnt;
            lid[KV + j] = (s.ob[v].lid4 >> (8 * j)) & 0xffu;
            val[KV + j] = s.ob[v].val[j];
        }
        add_distinct<T, KV + 4>(acc, lane, act, lid, val);
        // further blocks (an event in more than KV + 3 layers)
        for (int i0 = 4; i0 < (in ? cnt : 0); i0 += 4) {
            OvBlock<T> o;
            load_ov_block(b, pos + (uint32_t)i0, o);
            bool a2[4];
            uint32_t l2[4];
            T v2[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a2[j] = i0 + j < cnt;
                l2[j] = (o.lid4 >> (8 * j)) & 0xffu;
                v2[j] = o.val[j];
            }
            add_distinct<T, 4>(acc, lane, a2, l2, v2);
        }
    }
}

// Year losses of the trial in the accumulators (lane l: layer l, folded in
// the butterfly order of wave_allreduce), then the accumulators cleared.
template <typename T>
__device__ __forceinline__ void batch_finish_trial(Acc<T> *acc, int lane, int n_layers, int64_t trial, double *my_ylt,
                                                   double my_ret, double my_lim) {
    wave_lds_fence();
    if (lane < n_layers) {
        const Acc<T> *row = acc + lane * kAccStride;
        Acc<T> v[kWave / 2];
#pragma unroll
        for (int i = 0; i < kWave / 2; ++i) v[i] = Acc<T>::combine(row[i], row[i + kWave / 2]);
#pragma unroll
        for (int m = kWave / 4; m >= 1; m >>= 1)
#pragma unroll
            for (int i = 0; i < m; ++i) v[i] = Acc<T>::combine(v[i], v[i + m]);
        my_ylt[trial] = clamp_excess(v[0].value(), my_ret, my_lim);
    }
    wave_lds_fence();
    for (int l = 0; l < n_layers; ++l) acc[l * kAccStride + lane] = Acc<T>::zero();
}

template <typename T, bool FIXED, bool ALIGNED>
__device__ __forceinline__ void stream_step(const YetView &y, const int64_t *__restrict__ off, const BatchTables &b,
                                            const Record<T> *__restrict__ rec, ChunkCursor &cc, int64_t n_waves,
                                            int lane, int64_t last_granule, Acc<T> *acc, double *my_ylt,
                                            double my_ret, double my_lim, StreamSlot<T> &s0, StreamSlot<T> &s1,
                                            StreamSlot<T> &s2) {
    stream_heads(b, s1);
    stream_records(rec, s2);
    stream_next<T, FIXED, ALIGNED>(y, off, cc, n_waves, lane, last_granule, s0);
    stream_add(b, s0, acc, lane);
    if (s0.last) batch_finish_trial(acc, lane, b.n_layers, s0.trial, my_ylt, my_ret, my_lim);
}

template <typename T, bool FIXED, bool ALIGNED>
__global__ __launch_bounds__(256) void k_trial_pass_batch_stream(YetView y, const int64_t *__restrict__ off,
                                                                 BatchTables b) {
    extern __shared__ uint64_t lds_raw[];
    const int lane = lane_id();
    const int n_layers = b.n_layers;
    Acc<T> *acc = reinterpret_cast<Acc<T> *>(lds_raw) + (size_t)(threadIdx.x >> 6) * n_layers * kAccStride;
    const Record<T> *__restrict__ rec = static_cast<const Record<T> *>(b.rec);
    double *my_ylt = nullptr;
    double my_ret = 0.0, my_lim = 0.0;
    if (lane < n_layers) {
        my_ylt = b.ylts[lane];
        my_ret = b.agg_ret[lane];
        my_lim = b.agg_lim[lane];
    }
    for (int l = 0; l < n_layers; ++l) acc[l * kAccStride + lane] = Acc<T>::zero();
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t last_granule = (y.n_events - 1) & ~3LL;  // launched only with n_events >= 1
    ChunkCursor cc;
    cc.trial = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    cc.base = 0;
    cc.r = TrialRange{0, 0};
    cursor_enter<FIXED>(y, off, cc);
    StreamSlot<T> A, B, C;
    // prologue: chunk 0 in A up to its overflow blocks, chunk 1 in B up to
    // its records, chunk 2's IDs in C
    stream_next<T, FIXED, ALIGNED>(y, off, cc, n_waves, lane, last_granule, A);
    stream_next<T, FIXED, ALIGNED>(y, off, cc, n_waves, lane, last_granule, B);
    stream_records(rec, A);
    stream_next<T, FIXED, ALIGNED>(y, off, cc, n_waves, lane, last_granule, C);
    stream_records(rec, B);
    stream_heads(b, A);
    while (true) {
        if (A.trial < 0) break;
        stream_step<T, FIXED, ALIGNED>(y, off, b, rec, cc, n_waves, lane, last_granule, acc, my_ylt, my_ret, my_lim, A, B, C);
        if (B.trial < 0) break;
        stream_step<T, FIXED, ALIGNED>(y, off, b, rec, cc, n_waves, lane, last_granule, acc, my_ylt, my_ret, my_lim, B, C, A);
        if (C.trial < 0) break;
        stream_step<T, FIXED, ALIGNED>(y, off, b, rec, cc, n_waves, lane, last_granule, acc, my_ylt, my_ret, my_lim, C, A, B);
    }
}

// --------------------------------------------------------------------------------------------
// dense batched pass: at most kDenseWidth layers per pass, one record of
// all their occurrence losses per event, the union of their non-zero events
// as LDS filters

template <typename T, int NL>
struct alignas(sizeof(T) * NL <= 16 ? sizeof(T) * NL : 16) DenseRec {
    T v[NL];
};

// Records and filters of the dense form.  A wave takes 64 consecutive
// events: every lane writes its event's record, the lanes' block-filter
// bits are OR-ed over the wave per filter word (a wave's events fall into
// one word, or two when blocks are single events) and set with one atomic
// OR per word; the hashed filter gets one atomic OR per non-zero event.
// Filter words are cleared beforehand.
// *union_count receives the number of events with any non-zero value.
template <typename T, int NL>
__global__ __launch_bounds__(256) void k_dense_fill(OccPtrs occ, int32_t n_layers, int32_t catalog,
                                                    DenseRec<T, NL> *__restrict__ rec, uint32_t *__restrict__ filt,
                                                    int32_t fshift, uint32_t *__restrict__ hwords, int32_t n_hwords,
                                                    int32_t hshift, unsigned long long *union_count) {
    const int lane = lane_id();
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    for (int64_t base = wave * kWave; base <= (int64_t)catalog; base += n_waves * kWave) {
        const int64_t e = base + lane;
        DenseRec<T, NL> r;
        uint32_t any = 0;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const T v = (l < n_layers && e < catalog) ? static_cast<const T *>(occ.p[l])[e] : T(0);
            r.v[l] = v;
            any |= v != T(0) ? 1u : 0u;
        }
        if (e <= catalog) rec[e] = r;
        const int64_t w = e >> (fshift + 5);
        const int64_t w_first = base >> (fshift + 5);
        const uint32_t bit = any ? 1u << (uint32_t)(e & 31) : 0u;
        uint32_t lo = w == w_first ? bit : 0u, hi = w == w_first ? 0u : bit;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            lo |= (uint32_t)__shfl_xor((int)lo, m, kWave);
            hi |= (uint32_t)__shfl_xor((int)hi, m, kWave);
        }
        if (lane == 0 && lo) atomicOr(&filt[w_first], lo);
        if (lane == 0 && hi) atomicOr(&filt[w_first + 1], hi);
        const unsigned long long members = __ballot(any != 0u);
        if (lane == 0 && members) atomicAdd(union_count, (unsigned long long)__popcll(members));
        if (n_hwords > 0 && any) atomicOr(&hwords[hash_word((uint32_t)e, hshift)], 1u << (uint32_t)(e & 31));
    }
}

// Records of a group's passing events, compacted per lane as in the fused
// pass (gather_hits / sum_hits): the first kDenseHits in as many gathers
// (the all-zero record where a lane has fewer), then the rest one at a
// time while any lane has some.  Every layer's losses are added in the
// lane's event order, as the single-layer pass adds them (skipped events
// add exact zeros there; FP32C skips zeros as there).
template <int G>
struct DenseHits;
template <>
struct DenseHits<1> {
    static constexpr int k = 3;
};
template <>
struct DenseHits<2> {
    static constexpr int k = 4;
};
template <>
struct DenseHits<4> {
    static constexpr int k = 6;
};

template <typename T, int NL, int G>
struct HitRecs {
    DenseRec<T, NL> x[DenseHits<G>::k];
    uint32_t pass;
};

template <typename T, int NL, bool HASH, int G>
__device__ __forceinline__ void gather_recs(const IdGroupT<G> &g, uint32_t valid, const uint32_t *sfilt,
                                            const FusedFilter &f, int32_t zero_slot,
                                            const DenseRec<T, NL> *__restrict__ rec, HitRecs<T, NL, G> &h) {
    uint32_t pass = pass_mask<HASH, false, G>(g, valid, sfilt, f);
#pragma unroll
    for (int k = 0; k < DenseHits<G>::k; ++k) {
        h.x[k] = rec[pass ? select_id<G>(g, first_pass<G>(pass)) : (uint32_t)zero_slot];
        pass &= pass - 1u;
    }
    h.pass = pass;
}

template <typename T, int NL>
__device__ __forceinline__ void add_rec(const DenseRec<T, NL> &r, Acc<T> (&acc)[NL]) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        if (sizeof(T) == 8) {
            acc[l].add(r.v[l]);
        } else if (r.v[l] != T(0)) {
            acc[l].add(r.v[l]);
        }
    }
}

template <typename T, int NL, int G>
__device__ __forceinline__ void sum_recs(const IdGroupT<G> &g, HitRecs<T, NL, G> &h, int32_t zero_slot,
                                         const DenseRec<T, NL> *__restrict__ rec, Acc<T> (&acc)[NL]) {
#pragma unroll
    for (int k = 0; k < DenseHits<G>::k; ++k) add_rec<T, NL>(h.x[k], acc);
    uint32_t pass = h.pass;
    while (__builtin_amdgcn_ballot_w64(pass != 0u)) {
        const DenseRec<T, NL> r = rec[pass ? select_id<G>(g, first_pass<G>(pass)) : (uint32_t)zero_slot];
        pass &= pass - 1u;
        add_rec<T, NL>(r, acc);
    }
}

// One wave per trial, the loads, filters and lane order of
// k_trial_pass_fused; every event adds its record to NL running sums, so
// each layer's YLT is bitwise the one of its own fused pass.  Lane l < n
// writes layer l's year loss.
template <typename T, int NL, bool FIXED, bool ALIGNED, bool HASH, int G>
__global__ __launch_bounds__(1024) void k_trial_pass_dense(YetView y, const int64_t *__restrict__ off, FusedFilter f,
                                                           int32_t zero_slot,
                                                           const DenseRec<T, NL> *__restrict__ rec,
                                                           double *const *__restrict__ ylts,
                                                           const double *__restrict__ agg_ret,
                                                           const double *__restrict__ agg_lim, int32_t n_layers) {
    extern __shared__ uint32_t sfilt[];
    load_filters(f, sfilt);
    const int lane = lane_id();
    double *my_ylt = nullptr;
    double my_ret = 0.0, my_lim = 0.0;
    if (lane < n_layers) {
        my_ylt = ylts[lane];
        my_ret = agg_ret[lane];
        my_lim = agg_lim[lane];
    }
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    constexpr int64_t kSpan = (int64_t)G * kChunkEvents;
    const int64_t last_granule = (y.n_events - 1) & ~3LL;  // launched only with n_events >= 1
    int64_t trial = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    TrialRange r{0, 0};
    IdGroupT<G> cur;
    uint32_t cur_valid = 0;
    if (trial < y.n_trials) {
        r = fused_range<FIXED>(y, off, trial);
        cur_valid = load_group<FIXED, ALIGNED, G>(y, r, chunk_start(y, r.b), lane, last_granule, cur);
    }
    while (trial < y.n_trials) {
        HitRecs<T, NL, G> hits;
        gather_recs<T, NL, HASH, G>(cur, cur_valid, sfilt, f, zero_slot, rec, hits);
        const int64_t next = trial + n_waves;
        const TrialRange rn = fused_range<FIXED>(y, off, next < y.n_trials ? next : trial);
        IdGroupT<G> nxt;
        const uint32_t nxt_valid = load_group<FIXED, ALIGNED, G>(y, rn, chunk_start(y, rn.b), lane, last_granule, nxt);
        Acc<T> acc[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) acc[l] = Acc<T>::zero();
        sum_recs<T, NL, G>(cur, hits, zero_slot, rec, acc);
        constexpr int TG = FIXED ? G : 1;
        for (int64_t base = chunk_start(y, r.b) + kSpan; base < r.e; base += (int64_t)TG * kChunkEvents) {
            IdGroupT<TG> more;
            const uint32_t mv = load_group<FIXED, ALIGNED, TG>(y, r, base, lane, last_granule, more);
            HitRecs<T, NL, TG> mh;
            gather_recs<T, NL, HASH, TG>(more, mv, sfilt, f, zero_slot, rec, mh);
            sum_recs<T, NL, TG>(more, mh, zero_slot, rec, acc);
        }
        double mine = 0.0;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const double S = wave_allreduce(acc[l]).value();
            mine = lane == l ? S : mine;
        }
        if (lane < n_layers) my_ylt[trial] = clamp_excess(mine, my_ret, my_lim);
        trial = next;
        r = rn;
        cur = nxt;
        cur_valid = nxt_valid;
    }
}

// --------------------------------------------------------------------------------------------
// layers built on the device from a resident ELT pool: the fused table is
// accumulated ELT by ELT in layer order (one kernel per ELT, an ELT holding
// each event at most once), which is the order of the per-event sum of the
// host-built layouts, then the occurrence terms are applied in place.

template <typename T>
__global__ void k_pool_zero(T *__restrict__ occ, float *__restrict__ lo, int64_t catalog) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e <= catalog; e += (int64_t)gridDim.x * blockDim.x) {
        occ[e] = T(0);
        if (lo && e < catalog) lo[e] = 0.0f;
    }
}

template <typename T>
__global__ void k_pool_add(const int32_t *__restrict__ ids, const T *__restrict__ loss, int64_t n, T ret, T lim,
                           T *__restrict__ hi, float *__restrict__ lo) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = ids[i];
        const T x = clamp_excess(loss[i], ret, lim);
        if (sizeof(T) == 8) {
            hi[e] += x;
        } else {
            float sum, err;
            two_sum((float)hi[e], (float)x, sum, err);
            hi[e] = (T)sum;
            lo[e] += err;
        }
    }
}

template <typename T>
__global__ void k_pool_finish(T *__restrict__ occ, const float *__restrict__ lo, int64_t catalog, T occ_ret,
                              T occ_lim) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < catalog; e += (int64_t)gridDim.x * blockDim.x) {
        const T v = sizeof(T) == 8 ? occ[e] : (T)((float)occ[e] + lo[e]);
        occ[e] = clamp_excess(v, occ_ret, occ_lim);
    }
}

template <typename T>
__global__ void k_fill_zero(T *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

template <typename T>
__global__ void k_build_filter(const T *__restrict__ occ, int64_t catalog, int32_t fshift, uint32_t *__restrict__ filt,
                               int32_t n_fwords) {
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n_fwords; w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t bits = 0;
        const int64_t lo = w << (fshift + 5);
        const int64_t hi = lo + (32LL << fshift) < catalog ? lo + (32LL << fshift) : catalog;
        for (int64_t e = lo; e < hi; ++e) bits |= (occ[e] != T(0) ? 1u : 0u) << (uint32_t)(e & 31);
        filt[w] = bits;
    }
}

// Hashed filter: bit ((E mod 2^24) * kHashMul24) >> hshift for every event E
// with a non-zero occurrence loss (words cleared beforehand).
template <typename T>
__global__ void k_hash_filter(const T *__restrict__ occ, int64_t catalog, int32_t hshift, uint32_t *__restrict__ words) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < catalog; e += (int64_t)gridDim.x * blockDim.x)
        if (occ[e] != T(0)) atomicOr(&words[hash_word((uint32_t)e, hshift)], 1u << (uint32_t)(e & 31));
}

// Adds entry i of ELT j (at position b + i of the arrays) to its event's
// sum in LDS: FT1 of its loss, FP32C with a compensation term; CHECK: the
// loss's validity and a second entry of the same event in ELT j.
template <typename T, typename LT, bool CHECK>
__device__ __forceinline__ void build_add(T *hi, float *lo, int *stamp, uint32_t off, LT l, int j, T r, T u,
                                          int &bad) {
    if (CHECK) {
        if (!(l >= LT(0) && l <= __DBL_MAX__)) bad |= 4;
        if (atomicExch(&stamp[off], j) == j) bad |= 2;
    }
    const T x = clamp_excess((T)l, r, u);
    if (sizeof(T) == sizeof(double)) {
        hi[off] += x;
    } else {
        float sum, err;
        two_sum((float)hi[off], (float)x, sum, err);
        hi[off] = (T)sum;
        lo[off] += err;
    }
}

// IDs of one chunk of ELT j (kBuildUnroll per thread, entries i0 + q B +
// thread), every load unconditional: a chunk wholly inside the ELT reads
// at 32-bit offsets from the ELT's start, the ELT's last chunk at positions
// clamped to its last entry.
__device__ __forceinline__ void build_chunk_ids(const int32_t *__restrict__ ids, const BuildSegs &sg, int j,
                                                int64_t i0, int32_t (&e)[kBuildUnroll]) {
    const int64_t b = sg.begin[j], m = sg.count[j];
    const int32_t *__restrict__ seg = ids + b + i0;  // uniform
    if (i0 + (int64_t)kBuildUnroll * blockDim.x <= m) {
#pragma unroll
        for (int q = 0; q < kBuildUnroll; ++q) e[q] = seg[(uint32_t)(q * blockDim.x + threadIdx.x)];
    } else {
        const uint32_t last = (uint32_t)(m - 1 - i0);
#pragma unroll
        for (int q = 0; q < kBuildUnroll; ++q) {
            const uint32_t i = (uint32_t)(q * blockDim.x + threadIdx.x);
            e[q] = seg[i < last ? i : last];
        }
    }
}

// Range g's entry list, in range g's part of the table (range_capacity
// entries of 8 bytes).
template <typename T>
__device__ __forceinline__ uint64_t *range_list(T *occ, int64_t g) {
    return reinterpret_cast<uint64_t *>(occ + g * kBuildRange);
}

// The entry lists of a layer's ranges: one work-group per kListChunk entries
// of one ELT (blockIdx.y), each entry read once.  An entry goes to the list
// of its event's range, at a place taken from the range's count: the
// work-group first counts its entries per range in LDS and reserves each
// range's share with one atomic add on its count (one atomic per entry
// where the ranges outnumber kListHist).  The order of a list is
// arbitrary; the adds that read it keep the layer order.  Entries past a
// range's capacity are counted but not written (that range then reads the
// ELTs again).  The counts start at zero (the filter words are cleared
// beforehand).  CHECK: an ID outside [0, catalog) sets bit 1 of *flags.
constexpr int kListThreads = 256;
constexpr int kListPerThread = 8;
constexpr int kListChunk = kListThreads * kListPerThread;
template <typename T, bool CHECK>
__global__ __launch_bounds__(kListThreads) void k_build_lists(const int32_t *__restrict__ ids, BuildSegs sg,
                                                              int32_t catalog, T *__restrict__ occ,
                                                              uint32_t *__restrict__ filt, int32_t fshift,
                                                              int *flags) {
    __shared__ int hist[kListHist];
    const int j = blockIdx.y;
    const int64_t m = sg.count[j];
    const int64_t i0 = (int64_t)blockIdx.x * kListChunk;
    if (i0 >= m) return;  // uniform: the work-group has no entries
    const int n_ranges = (int)build_ranges(catalog);
    const bool local = n_ranges <= kListHist;
    if (local) {
        for (int k = threadIdx.x; k < n_ranges; k += blockDim.x) hist[k] = 0;
        __syncthreads();
    }
    const int32_t *__restrict__ seg = ids + sg.begin[j] + i0;
    const uint32_t n_here = (uint32_t)(m - i0 < kListChunk ? m - i0 : kListChunk);
    int32_t e[kListPerThread];
#pragma unroll
    for (int u = 0; u < kListPerThread; ++u) {
        const uint32_t i = (uint32_t)(u * kListThreads + threadIdx.x);
        e[u] = seg[i < n_here ? i : n_here - 1];
    }
    int bad = 0;
    int place[kListPerThread];
#pragma unroll
    for (int u = 0; u < kListPerThread; ++u) {
        const uint32_t i = (uint32_t)(u * kListThreads + threadIdx.x);
        place[u] = -1;
        if (i >= n_here) continue;
        if ((uint32_t)e[u] >= (uint32_t)catalog) {
            if (CHECK) bad |= 1;
            e[u] = -1;
            continue;
        }
        const int64_t g = build_range_of(e[u]);
        place[u] = local ? atomicAdd(&hist[g], 1) : atomicAdd(&filt[range_count_word(g, fshift)], 1u);
    }
    if (local) {
        __syncthreads();
        // each range's share of the list, from its count
        for (int k = threadIdx.x; k < n_ranges; k += blockDim.x) {
            const int c = hist[k];
            if (c) hist[k] = (int)atomicAdd(&filt[range_count_word(k, fshift)], (uint32_t)c);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kListPerThread; ++u) {
        if (place[u] < 0) continue;
        const int64_t g = build_range_of(e[u]);
        const int at = place[u] + (local ? hist[g] : 0);
        if (at < range_capacity(g, catalog, (int)sizeof(T))) {
            const uint32_t off = build_range_offset(e[u]);
            const int64_t pos = sg.begin[j] + i0 + u * kListThreads + threadIdx.x;
            range_list(occ, g)[at] = ((uint64_t)j << 53) | ((uint64_t)off << 40) | (uint64_t)pos;
        }
    }
    if (CHECK && bad) atomicOr(flags, bad);
}

// A layer's fused table from the entry lists of k_build_lists.  Work-group
// g owns the catalogue events [g R, (g + 1) R) (R = kBuildRange) and keeps
// their sums in LDS.  It reads its range's count and list, loads the listed
// losses together and adds FT1 of them to the sums one ELT after the other
// (an ELT holds an event at most once, so no two threads of one ELT add to
// the same slot; a barrier separates the ELTs), which is the order of
// k_pool_add.  A range whose list overflowed its capacity takes the ELTs one
// at a time instead, reading each ELT's IDs and losses as it goes.  It then
// applies the occurrence terms, writes its range of the table and its words
// of the block filter (a range covers whole filter words) and sets the
// hashed filter's bits of its non-zero events (words cleared beforehand).
// Bitwise the table of k_pool_zero / k_pool_add / k_pool_finish and the
// filter kernels.
// CHECK (ELTs from the host): also validates every loss and every pair of
// entries of one event in one ELT, reporting in *flags: 2 an ID twice in one
// ELT, 4 a loss that is negative, infinite or NaN (the table is then not
// used; k_build_lists reports IDs out of range).
// LT: type of the stored losses (binary64 from the host; the pool's own
// type for pool layers); the conversion to T is the one the host would do.
// A list entry: bits 0..39 the entry's position in the arrays, 40..52 its
// event's offset in the range, 53..57 its ELT.
template <typename T, typename LT, bool CHECK>
__global__ __launch_bounds__(kBuildThreads) void k_fused_build(const int32_t *__restrict__ ids,
                                                               const LT *__restrict__ loss, BuildSegs sg,
                                                               int32_t catalog, T occ_ret, T occ_lim,
                                                               T *__restrict__ occ, uint32_t *__restrict__ filt,
                                                               int32_t n_fwords, int32_t fshift,
                                                               uint32_t *__restrict__ hwords, int32_t n_hwords,
                                                               int32_t hshift, int *flags) {
    static_assert(kBuildRange <= (1 << 13) && kMaxElts <= 32, "list entry fields");
    constexpr int kPerThread = kBuildList / kBuildThreads;
    extern __shared__ uint64_t build_lds[];
    T *hi = reinterpret_cast<T *>(build_lds);
    float *lo = reinterpret_cast<float *>(hi + kBuildRange);  // FP32C: compensation terms
    int *stamp = reinterpret_cast<int *>(lo + (sizeof(T) == sizeof(float) ? kBuildRange : 0));  // CHECK
    const int64_t g = blockIdx.x;
    const int64_t base = g * kBuildRange;
    const uint32_t nloc = (uint32_t)range_events(g, catalog);
    const int wshift = 5 + fshift;
    const int64_t w0 = range_count_word(g, fshift);
    // the count (a range past the last filter word holds only the zero slot)
    const int n_list = w0 < n_fwords ? (int)filt[w0] : 0;
    const bool listed = n_list <= range_capacity(g, catalog, (int)sizeof(T));
    uint64_t le[kPerThread];
    LT lv[kPerThread];
    if (listed) {
        // the listed entries and their losses, all loads in flight together
        const uint64_t *__restrict__ list = range_list(occ, g);
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int sl = threadIdx.x + k * blockDim.x;
            le[k] = sl < n_list ? list[sl] : ~0ull;
        }
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            lv[k] = LT(0);
            if (le[k] != ~0ull) lv[k] = loss[(int64_t)(le[k] & ((1ull << 40) - 1))];
        }
    }
    for (int k = threadIdx.x; k < kBuildRange; k += blockDim.x) {
        hi[k] = T(0);
        if (sizeof(T) == sizeof(float)) lo[k] = 0.0f;
        if (CHECK) stamp[k] = -1;
    }
    __syncthreads();
    int bad = 0;
    if (listed) {
        // the sums in layer order
        for (int jj = 0; jj < sg.n; ++jj) {
            const T r = (T)sg.ret[jj], u = (T)sg.lim[jj];
#pragma unroll
            for (int k = 0; k < kPerThread; ++k)
                if ((int)(le[k] >> 53) == jj)
                    build_add<T, LT, CHECK>(hi, lo, stamp, (uint32_t)(le[k] >> 40) & 0x1fffu, lv[k], jj, r, u, bad);
            __syncthreads();
        }
    } else {
        // an overflowed range: one ELT at a time
        for (int jj = 0; jj < sg.n; ++jj) {
            const int64_t b = sg.begin[jj], m = sg.count[jj];
            const T r = (T)sg.ret[jj], u = (T)sg.lim[jj];
            for (int64_t ic = 0; ic < m; ic += (int64_t)kBuildUnroll * blockDim.x) {
                int32_t e[kBuildUnroll];
                build_chunk_ids(ids, sg, jj, ic, e);
#pragma unroll 4
                for (int q = 0; q < kBuildUnroll; ++q) {
                    const int64_t i = ic + (int64_t)q * blockDim.x + threadIdx.x;
                    if (i >= m || e[q] < 0 || e[q] >= catalog) continue;  // range errors flagged by the lists
                    const uint32_t off = (uint32_t)((int64_t)e[q] - base);
                    if (off >= nloc) continue;
                    build_add<T, LT, CHECK>(hi, lo, stamp, off, loss[b + i], jj, r, u, bad);
                }
            }
            __syncthreads();
        }
    }
    if (CHECK && bad) atomicOr(flags, bad);
    // occurrence terms; the zero slot occ[catalog] stays 0
    for (uint32_t k = threadIdx.x; k < nloc; k += blockDim.x) {
        const int64_t e = base + k;
        const T v = sizeof(T) == sizeof(double) ? hi[k] : (T)((float)hi[k] + lo[k]);
        const T o = e < catalog ? clamp_excess(v, occ_ret, occ_lim) : T(0);
        occ[e] = o;
        hi[k] = o;
    }
    __syncthreads();
    // block filter words of the range: bit b of word w is set iff one of the
    // events 2^(fshift + 5) w + 32 t + b (t < 2^fshift) has a non-zero
    // occurrence loss (the range starts on a word: kBuildRange is a multiple
    // of 2^(fshift + 5), and holds the zero slot's slot as 0)
    const int n_w = kBuildRange >> wshift;
    for (int q = threadIdx.x; q < n_w; q += blockDim.x) {
        const int64_t w = w0 + q;
        if (w >= n_fwords) continue;
        uint32_t bits = 0;
        const int k0 = q << wshift;
        const int k1 = k0 + (1 << wshift) < (int)nloc ? k0 + (1 << wshift) : (int)nloc;
        for (int k = k0; k < k1; ++k) bits |= (hi[k] != T(0) ? 1u : 0u) << (uint32_t)(k & 31);
        filt[w] = bits;
    }
    if (n_hwords > 0) {
        for (uint32_t k = threadIdx.x; k < nloc; k += blockDim.x) {
            const int64_t e = base + k;
            if (e < catalog && hi[k] != T(0))
                atomicOr(&hwords[hash_word((uint32_t)e, hshift)], 1u << (uint32_t)(e & 31));
        }
    }
}

// One read of every ID: the IDs before the first 16-byte boundary and after
// the last whole 16-byte granule one by one, the granules with non-temporal
// 16-byte loads: a wave reads 8 KiB in a row (eight loads in flight per
// lane), the granules after the last whole 8 KiB chunk one per thread.
__device__ __forceinline__ uint32_t ids_outside(const int4 v, uint32_t catalog) {
    return ((uint32_t)v.x >= catalog) | ((uint32_t)v.y >= catalog) | ((uint32_t)v.z >= catalog) |
           ((uint32_t)v.w >= catalog);
}

__global__ __launch_bounds__(256) void k_validate_yet(const int32_t *__restrict__ ids, int64_t n, int32_t catalog,
                                                      const int64_t *__restrict__ off, int64_t n_trials,
                                                      int32_t *flags) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint32_t cat = (uint32_t)catalog;
    int64_t head = (int64_t)(((16u - ((uint32_t)reinterpret_cast<uintptr_t>(ids) & 15u)) & 15u) >> 2);
    head = head < n ? head : n;
    const int64_t body = (n - head) >> 2;  // whole granules after the head
    const int32_t *g0 = ids + head;
    uint32_t bad = 0;
    // whole chunks of kRound * 64 granules (8 KiB), one wave per chunk
    constexpr int kRound = 8;
    constexpr int64_t kChunkGranules = (int64_t)kRound * kWave;
    const int64_t lane = threadIdx.x & (kWave - 1), wave = tid / kWave, n_waves = stride / kWave;
    const int64_t n_chunks = body / kChunkGranules;
    for (int64_t c = wave; c < n_chunks; c += n_waves) {
        int4 v[kRound];
#pragma unroll
        for (int r = 0; r < kRound; ++r) v[r] = stream_ids4(g0 + 4 * (c * kChunkGranules + r * kWave + lane));
#pragma unroll
        for (int r = 0; r < kRound; ++r) bad |= ids_outside(v[r], cat);
    }
    for (int64_t g = n_chunks * kChunkGranules + tid; g < body; g += stride) bad |= ids_outside(stream_ids4(g0 + 4 * g), cat);
    for (int64_t i = tid; i < head; i += stride) bad |= ((uint32_t)ids[i] >= cat);
    for (int64_t i = head + 4 * body + tid; i < n; i += stride) bad |= ((uint32_t)ids[i] >= cat);
    int bad_id = bad != 0u, bad_off = 0;
    if (off) {
        for (int64_t i = tid; i < n_trials; i += stride) bad_off |= (off[i + 1] < off[i]);
        if (tid == 0) bad_off |= (off[0] != 0);
    }
    if (bad_id) atomicOr(&flags[0], 1);
    if (bad_off) atomicOr(&flags[1], 1);
}

// --------------------------------------------------------------------------------------------
int grid_for_trials(int64_t n_trials, int waves_per_block, int blocks_per_cu) {
    int64_t need = (n_trials + waves_per_block - 1) / waves_per_block;
    int64_t cap = (int64_t)cu_count() * blocks_per_cu;
    int64_t g = need < cap ? need : cap;
    return (int)(g < 1 ? 1 : g);
}

template <typename T>
hipError_t launch_pass_t(const YetView &y, const LayerHost &L, const Terms<T> &t, double *d_ylt, double *d_cum,
                         double *d_net, double *d_omax, bool events, hipStream_t s) {
    if (y.n_trials == 0) return hipSuccess;
    const int grid = grid_for_trials(y.n_trials, 4, 8);
    const dim3 blk(256);
    if (L.layout == kFused && y.n_events > 0) {
        const FusedFilter f{L.tab.filt, L.tab.n_fwords, L.tab.fshift, L.tab.n_hwords, L.tab.hshift};
        const size_t lds = (size_t)(f.n_fwords + f.n_hwords) * sizeof(uint32_t);
        if (lds > (size_t)kFusedLdsBytes) return hipErrorInvalidValue;
        const bool fixed = y.offsets == nullptr && y.aligned16 && y.events_per_trial > 0 && (y.events_per_trial % 4) == 0;
        const bool hash = f.n_hwords > 0;
        const int variant = (fixed ? 0 : (y.aligned16 ? 1 : 2)) + (hash ? 3 : 0);
        using PassK = void (*)(YetView, const int64_t *, FusedFilter, int32_t, const T *, double, double, double *,
                               double *);
        using EventsK = void (*)(YetView, const int64_t *, FusedFilter, int32_t, const T *, double, double, double *,
                                 double *, double *);
#define ARA_FUSED_PASSES(O32)                                                                                      \
    &k_trial_pass_fused<T, true, true, false, kGroup, false, O32>, &k_trial_pass_fused<T, false, true, false, kGroup, false, O32>, \
        &k_trial_pass_fused<T, false, false, false, kGroup, false, O32>,                                                    \
        &k_trial_pass_fused<T, true, true, true, kGroup, false, O32>, &k_trial_pass_fused<T, false, true, true, kGroup, false, O32>, \
        &k_trial_pass_fused<T, false, false, true, kGroup, false, O32>,                                                     \
        &k_trial_pass_fused<T, true, true, false, kGroup, true, O32>, &k_trial_pass_fused<T, false, true, false, kGroup, true, O32>, \
        &k_trial_pass_fused<T, false, false, false, kGroup, true, O32>,                                                     \
        &k_trial_pass_fused<T, true, true, true, kGroup, true, O32>, &k_trial_pass_fused<T, false, true, true, kGroup, true, O32>,   \
        &k_trial_pass_fused<T, false, false, true, kGroup, true, O32>
        const PassK pk[24] = {ARA_FUSED_PASSES(false), ARA_FUSED_PASSES(true)};
#undef ARA_FUSED_PASSES
        // 32-bit table offsets while every byte of the table (zero slot
        // included) lies below 2^32
        const bool off32 = ((int64_t)L.catalog + 1) * (int64_t)sizeof(T) <= (1LL << 32);
        const int pv = variant + (d_omax ? 6 : 0) + (off32 ? 12 : 0);
        const EventsK ek[6] = {&k_trial_pass_events_fused<T, true, true, false, kGroup>,
                               &k_trial_pass_events_fused<T, false, true, false, kGroup>,
                               &k_trial_pass_events_fused<T, false, false, false, kGroup>,
                               &k_trial_pass_events_fused<T, true, true, true, kGroup>,
                               &k_trial_pass_events_fused<T, false, true, true, kGroup>,
                               &k_trial_pass_events_fused<T, false, false, true, kGroup>};
        const void *kern = events ? reinterpret_cast<const void *>(ek[variant]) : reinterpret_cast<const void *>(pk[pv]);
        hipError_t ae = allow_dynamic_lds(kern, (int)kFusedLdsBytes);
        if (ae != hipSuccess) return ae;
        const int per_cu = lds > (size_t)kFusedLdsBytes / 2 ? 1 : 2;
        const int fgrid = grid_for_trials(y.n_trials, 16, per_cu);
        const T *occ = static_cast<const T *>(L.tab.occ);
        if (!events) {
            hipLaunchKernelGGL(pk[pv], dim3(fgrid), dim3(1024), lds, s, y, y.offsets, f, L.catalog, occ, t.agg_ret,
                               t.agg_lim, d_ylt, d_omax);
        } else {
            hipLaunchKernelGGL(ek[variant], dim3(fgrid), dim3(1024), lds, s, y, y.offsets, f, L.catalog, occ, t.agg_ret,
                               t.agg_lim, d_ylt, d_cum, d_net);
        }
        return hipGetLastError();
    }
    if (!events) {
        switch (L.layout) {
            case kDirect: hipLaunchKernelGGL((k_trial_pass<T, kDirect>), dim3(grid), blk, 0, s, y, L.tab, t, d_ylt, d_omax); break;
            case kSparse: hipLaunchKernelGGL((k_trial_pass<T, kSparse>), dim3(grid), blk, 0, s, y, L.tab, t, d_ylt, d_omax); break;
            case kFused: hipLaunchKernelGGL((k_trial_pass<T, kFused>), dim3(grid), blk, 0, s, y, L.tab, t, d_ylt, d_omax); break;
            default: hipLaunchKernelGGL((k_trial_pass<T, kCompact>), dim3(grid), blk, 0, s, y, L.tab, t, d_ylt, d_omax); break;
        }
    } else {
        switch (L.layout) {
            case kDirect:
                hipLaunchKernelGGL((k_trial_pass_events<T, kDirect>), dim3(grid), blk, 0, s, y, L.tab, t, d_ylt, d_cum, d_net);
                break;
            case kSparse:
                hipLaunchKernelGGL((k_trial_pass_events<T, kSparse>), dim3(grid), blk, 0, s, y, L.tab, t, d_ylt, d_cum, d_net);
                break;
            case kFused:
                hipLaunchKernelGGL((k_trial_pass_events<T, kFused>), dim3(grid), blk, 0, s, y, L.tab, t, d_ylt, d_cum, d_net);
                break;
            default:
                hipLaunchKernelGGL((k_trial_pass_events<T, kCompact>), dim3(grid), blk, 0, s, y, L.tab, t, d_ylt, d_cum, d_net);
                break;
        }
    }
    return hipGetLastError();
}

}  // namespace

int cu_count() {
    static std::atomic<int> cached[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const bool cacheable = dev >= 0 && dev < kMaxDevices;
    if (cacheable) {
        const int c = cached[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int n = 0;
    if (dev < 0 || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        n = 256;
    if (cacheable) cached[dev].store(n, std::memory_order_relaxed);
    return n;
}

hipError_t allow_dynamic_lds(const void *kern, int bytes) {
    static std::mutex mu;
    static std::set<std::tuple<int, const void *, int>> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const auto key = std::make_tuple(dev, kern, bytes);
    std::lock_guard<std::mutex> g(mu);
    if (done.count(key)) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) done.insert(key);
    return e;
}

hipStream_t internal_stream() {
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[dev] = st;
    return st;
}

hipError_t launch_validate_yet(const YetView &y, int32_t catalog, int32_t *d_flags, hipStream_t s) {
    const int grid = cu_count() * 8;
    hipLaunchKernelGGL(k_validate_yet, dim3(grid), dim3(256), 0, s, y.ids, y.n_events, catalog, y.offsets, y.n_trials,
                       d_flags);
    return hipGetLastError();
}

hipError_t launch_trial_pass(const YetView &y, const LayerHost &L, double *d_ylt, double *d_omax, hipStream_t s) {
    if (L.precision == ARA_FP32C) return launch_pass_t<float>(y, L, L.t32, d_ylt, nullptr, nullptr, d_omax, false, s);
    return launch_pass_t<double>(y, L, L.t64, d_ylt, nullptr, nullptr, d_omax, false, s);
}

hipError_t launch_trial_pass_events(const YetView &y, const LayerHost &L, double *d_ylt, double *d_cum,
                                    double *d_net, hipStream_t s) {
    if (L.precision == ARA_FP32C) return launch_pass_t<float>(y, L, L.t32, d_ylt, d_cum, d_net, nullptr, true, s);
    return launch_pass_t<double>(y, L, L.t64, d_ylt, d_cum, d_net, nullptr, true, s);
}

namespace {
// One thread per catalogue event (256-thread blocks).
int event_blocks(int32_t catalog) {
    const int64_t b = ((int64_t)catalog + 255) / 256;
    return (int)(b < 1 ? 1 : (b > (1LL << 20) ? (1LL << 20) : b));
}

template <typename T>
hipError_t batch_count_t(const void *const *occ, int32_t n, int32_t catalog, int32_t *cnt, unsigned long long *tot,
                         hipStream_t s) {
    OccPtrs o{};
    for (int l = 0; l < n; ++l) o.p[l] = occ[l];
    hipLaunchKernelGGL((k_batch_count<T>), dim3(event_blocks(catalog)), dim3(256), 0, s, o, n, catalog, cnt, tot);
    return hipGetLastError();
}
template <typename T>
hipError_t batch_fill_t(const void *const *occ, int32_t n, int32_t catalog, const int32_t *cnt, void *rec,
                        uint8_t *ovf_lid, void *ovf_val, unsigned long long *cursor, hipStream_t s) {
    OccPtrs o{};
    for (int l = 0; l < n; ++l) o.p[l] = occ[l];
    hipLaunchKernelGGL((k_batch_fill<T>), dim3(event_blocks(catalog)), dim3(256), 0, s, o, n, catalog, cnt,
                       static_cast<Record<T> *>(rec), ovf_lid, static_cast<T *>(ovf_val), cursor);
    return hipGetLastError();
}
template <typename T, int G>
auto batch_kernel(bool fixed, bool aligned) {
    return fixed ? &k_trial_pass_batch<T, true, true, G>
                 : (aligned ? &k_trial_pass_batch<T, false, true, G> : &k_trial_pass_batch<T, false, false, G>);
}

template <typename T>
auto batch_stream_kernel(bool fixed, bool aligned) {
    return fixed ? &k_trial_pass_batch_stream<T, true, true>
                 : (aligned ? &k_trial_pass_batch_stream<T, false, true> : &k_trial_pass_batch_stream<T, false, false>);
}

template <typename T>
hipError_t batch_pass_t(const YetView &y, const BatchTables &b, const BatchLaunch &cfg, hipStream_t s) {
    if (y.n_trials == 0) return hipSuccess;
    const bool fixed = y.offsets == nullptr && y.aligned16 && y.events_per_trial > 0 && (y.events_per_trial % 4) == 0;
    const bool al = y.aligned16 != 0;
    if (cfg.group != 1 && cfg.group != 2 && cfg.group != 4 && cfg.group != 8) return hipErrorInvalidValue;
    // group 1: the pipelined pass (256-thread work-groups at most)
    if (cfg.group == 1 && cfg.threads > kMaxStreamThreads) return hipErrorInvalidValue;
    auto kern = cfg.group == 1 ? batch_stream_kernel<T>(fixed, al)
                               : (cfg.group == 2 ? batch_kernel<T, 2>(fixed, al)
                                                 : (cfg.group == 8 ? batch_kernel<T, 8>(fixed, al)
                                                                   : batch_kernel<T, 4>(fixed, al)));
    const size_t lds = batch_lds_bytes(b.n_layers, cfg.threads);
    if (lds > 160u * 1024u || cfg.threads < kWave || cfg.threads > 512 || cfg.threads % kWave) return hipErrorInvalidValue;
    hipError_t ae = allow_dynamic_lds(reinterpret_cast<const void *>(kern), 160 * 1024);
    if (ae != hipSuccess) return ae;
    int per_cu = (int)((160 * 1024) / (lds ? lds : 1));
    if (per_cu > cfg.wg_per_cu) per_cu = cfg.wg_per_cu;
    if (per_cu < 1) per_cu = 1;
    const int grid = grid_for_trials(y.n_trials, cfg.threads / kWave, per_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(cfg.threads), lds, s, y, y.offsets, b);
    return hipGetLastError();
}
}  // namespace

namespace {
template <typename T>
hipError_t pool_layer_t(LayerHost &L, const Terms<T> &t, const int32_t *ids, const void *loss, const int64_t *off,
                        const int32_t *idx, int32_t n, float *lo, hipStream_t s) {
    T *occ = static_cast<T *>(const_cast<void *>(L.tab.occ));
    const T *ls = static_cast<const T *>(loss);
    const int g = cu_count() * 2;
    hipLaunchKernelGGL((k_pool_zero<T>), dim3(g), dim3(256), 0, s, occ, lo, (int64_t)L.catalog);
    for (int j = 0; j < n; ++j) {
        const int64_t b = off[idx[j]], m = off[idx[j] + 1] - b;
        if (m > 0)
            hipLaunchKernelGGL((k_pool_add<T>), dim3(g), dim3(256), 0, s, ids + b, ls + b, m, t.ret[j], t.lim[j], occ, lo);
    }
    hipLaunchKernelGGL((k_pool_finish<T>), dim3(g), dim3(256), 0, s, occ, lo, (int64_t)L.catalog, t.occ_ret, t.occ_lim);
    hipLaunchKernelGGL((k_build_filter<T>), dim3(g), dim3(256), 0, s, occ, (int64_t)L.catalog, L.tab.fshift,
                       const_cast<uint32_t *>(L.tab.filt), L.tab.n_fwords);
    if (L.tab.n_hwords > 0) {
        uint32_t *hw = const_cast<uint32_t *>(L.tab.filt) + L.tab.n_fwords;
        hipLaunchKernelGGL((k_fill_zero<uint32_t>), dim3(g), dim3(256), 0, s, hw, (int64_t)L.tab.n_hwords);
        hipLaunchKernelGGL((k_hash_filter<T>), dim3(g), dim3(256), 0, s, occ, (int64_t)L.catalog, L.tab.hshift, hw);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_pool_layer(LayerHost &L, const int32_t *d_ids, const void *d_loss, const int64_t *h_off,
                             const int32_t *h_idx, int32_t n, float *d_lo, hipStream_t s) {
    if (L.precision == ARA_FP32C) return pool_layer_t<float>(L, L.t32, d_ids, d_loss, h_off, h_idx, n, d_lo, s);
    return pool_layer_t<double>(L, L.t64, d_ids, d_loss, h_off, h_idx, n, nullptr, s);
}

namespace {
template <typename T>
const Terms<T> &terms_of(const LayerHost &L);
template <>
const Terms<double> &terms_of<double>(const LayerHost &L) {
    return L.t64;
}
template <>
const Terms<float> &terms_of<float>(const LayerHost &L) {
    return L.t32;
}
}  // namespace

bool fused_build_fits(int64_t catalog, int32_t fshift, int64_t n_entries) {
    if (!build_ranges_cover_words(fshift)) return false;
    const int64_t groups = build_ranges((int32_t)catalog);
    // a work-group whose range overflows its list reads every ID of the layer
    return groups * (n_entries > 0 ? n_entries : 1) <= kBuildReadBudget;
}

namespace {
template <typename T, typename LT, bool CHECK>
hipError_t fused_build_t(LayerHost &L, const int32_t *d_ids, const void *d_loss, const int64_t *h_off,
                         const int32_t *h_idx, int32_t n, int *d_flags, hipStream_t s) {
    BuildSegs sg{};
    int64_t total = 0;
    for (int j = 0; j < n; ++j) {
        sg.begin[j] = h_off[h_idx[j]];
        sg.count[j] = h_off[h_idx[j] + 1] - h_off[h_idx[j]];
        sg.ret[j] = L.t64.ret[j];
        sg.lim[j] = L.t64.lim[j];
        total += sg.count[j];
    }
    sg.n = n;
    if (!fused_build_fits(L.catalog, L.tab.fshift, total)) return hipErrorNotSupported;
    const Terms<T> &t = terms_of<T>(L);
    auto kern = &k_fused_build<T, LT, CHECK>;
    const int lds = (int)(kBuildRange * (sizeof(T) + (sizeof(T) == sizeof(float) ? 4 : 0) + (CHECK ? 4 : 0)));
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void *>(kern), lds);
    if (e != hipSuccess) return e;
    T *occ = static_cast<T *>(const_cast<void *>(L.tab.occ));
    uint32_t *filt = const_cast<uint32_t *>(L.tab.filt);
    // the filter words hold the ranges' counts until the build writes them
    hipLaunchKernelGGL((k_fill_zero<uint32_t>), dim3(64), dim3(256), 0, s, filt,
                       (int64_t)(L.tab.n_fwords + L.tab.n_hwords));
    int64_t longest = 0;
    for (int j = 0; j < n; ++j) longest = sg.count[j] > longest ? sg.count[j] : longest;
    if (longest > 0)
        hipLaunchKernelGGL((k_build_lists<T, CHECK>), dim3((unsigned)((longest + kListChunk - 1) / kListChunk), (unsigned)n),
                           dim3(kListThreads), 0, s, d_ids, sg, L.catalog, occ, filt, L.tab.fshift, d_flags);
    const int64_t groups = build_ranges(L.catalog);
    hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(kBuildThreads), lds, s, d_ids, static_cast<const LT *>(d_loss),
                       sg, L.catalog, t.occ_ret, t.occ_lim, occ, filt, L.tab.n_fwords, L.tab.fshift,
                       filt + L.tab.n_fwords, L.tab.n_hwords, L.tab.hshift, d_flags);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_fused_build(LayerHost &L, const int32_t *d_ids, const void *d_loss, bool host_losses,
                              const int64_t *h_off, const int32_t *h_idx, int32_t n, int *d_flags, hipStream_t s) {
    if (host_losses) {
        // binary64 losses straight from the host, validated on the way
        if (L.precision == ARA_FP32C) return fused_build_t<float, double, true>(L, d_ids, d_loss, h_off, h_idx, n, d_flags, s);
        return fused_build_t<double, double, true>(L, d_ids, d_loss, h_off, h_idx, n, d_flags, s);
    }
    if (L.precision == ARA_FP32C) return fused_build_t<float, float, false>(L, d_ids, d_loss, h_off, h_idx, n, nullptr, s);
    return fused_build_t<double, double, false>(L, d_ids, d_loss, h_off, h_idx, n, nullptr, s);
}

hipError_t launch_fill_zero(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_zero<double>), dim3(cu_count() * 4), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

namespace {
template <typename T, int NL>
hipError_t dense_fill_t(const void *const *occ, int32_t n, const DenseTables &d, unsigned long long *ucount,
                        hipStream_t s) {
    OccPtrs o{};
    for (int l = 0; l < n; ++l) o.p[l] = occ[l];
    uint32_t *filt = const_cast<uint32_t *>(d.filt);
    hipLaunchKernelGGL((k_fill_zero<uint32_t>), dim3(64), dim3(256), 0, s, filt, (int64_t)(d.n_fwords + d.n_hwords));
    // one wave per 64 events: every load of the fill in flight at once
    const int64_t waves = ((int64_t)d.catalog + 1 + kWave - 1) / kWave;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > (1LL << 20)) blocks = 1LL << 20;
    hipLaunchKernelGGL((k_dense_fill<T, NL>), dim3((unsigned)blocks), dim3(256), 0, s, o, n, d.catalog,
                       static_cast<DenseRec<T, NL> *>(const_cast<void *>(d.rec)), filt, d.fshift, filt + d.n_fwords,
                       d.n_hwords, d.hshift, ucount);
    return hipGetLastError();
}

template <typename T, int NL, int G>
hipError_t dense_pass_nlg(const YetView &y, const DenseTables &d, hipStream_t s) {
    const FusedFilter f{d.filt, d.n_fwords, d.fshift, d.n_hwords, d.hshift};
    const size_t lds = (size_t)(f.n_fwords + f.n_hwords) * sizeof(uint32_t);
    if (lds > (size_t)kFusedLdsBytes) return hipErrorInvalidValue;
    const bool fixed = y.offsets == nullptr && y.aligned16 && y.events_per_trial > 0 && (y.events_per_trial % 4) == 0;
    const bool hash = f.n_hwords > 0;
    using K = void (*)(YetView, const int64_t *, FusedFilter, int32_t, const DenseRec<T, NL> *, double *const *,
                       const double *, const double *, int32_t);
    const K ks[6] = {&k_trial_pass_dense<T, NL, true, true, false, G>, &k_trial_pass_dense<T, NL, false, true, false, G>,
                     &k_trial_pass_dense<T, NL, false, false, false, G>, &k_trial_pass_dense<T, NL, true, true, true, G>,
                     &k_trial_pass_dense<T, NL, false, true, true, G>, &k_trial_pass_dense<T, NL, false, false, true, G>};
    const K k = ks[(fixed ? 0 : (y.aligned16 ? 1 : 2)) + (hash ? 3 : 0)];
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void *>(k), (int)kFusedLdsBytes);
    if (e != hipSuccess) return e;
    const int per_cu = lds > (size_t)kFusedLdsBytes / 2 ? 1 : 2;
    const int grid = grid_for_trials(y.n_trials, 16, per_cu);
    hipLaunchKernelGGL(k, dim3(grid), dim3(1024), lds, s, y, y.offsets, f, d.catalog,
                       static_cast<const DenseRec<T, NL> *>(d.rec), d.ylts, d.agg_ret, d.agg_lim, d.n_layers);
    return hipGetLastError();
}

// Groups of 2 or 4 chunks (the grouping changes when IDs are loaded, not
// the order of the adds); 4-wide records hold more registers per chunk and
// take groups of 2 only.
template <typename T>
hipError_t dense_pass_t(const YetView &y, const DenseTables &d, int group, hipStream_t s) {
    if (y.n_trials == 0) return hipSuccess;
    if (group != 2 && group != 4) return hipErrorInvalidValue;
    switch (d.nl) {
        case 1: return group == 2 ? dense_pass_nlg<T, 1, 2>(y, d, s) : dense_pass_nlg<T, 1, 4>(y, d, s);
        case 2: return group == 2 ? dense_pass_nlg<T, 2, 2>(y, d, s) : dense_pass_nlg<T, 2, 4>(y, d, s);
        case 4: return dense_pass_nlg<T, 4, 2>(y, d, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t dense_fill_w(const void *const *occ, int32_t n, const DenseTables &d, unsigned long long *ucount,
                        hipStream_t s) {
    switch (d.nl) {
        case 1: return dense_fill_t<T, 1>(occ, n, d, ucount, s);
        case 2: return dense_fill_t<T, 2>(occ, n, d, ucount, s);
        case 4: return dense_fill_t<T, 4>(occ, n, d, ucount, s);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_dense_fill(const void *const *occ, int32_t n_layers, bool fp64, const DenseTables &d,
                             unsigned long long *d_union_count, hipStream_t s) {
    if (n_layers < 1 || n_layers > d.nl) return hipErrorInvalidValue;
    return fp64 ? dense_fill_w<double>(occ, n_layers, d, d_union_count, s)
                : dense_fill_w<float>(occ, n_layers, d, d_union_count, s);
}

hipError_t launch_dense_pass(const YetView &y, const DenseTables &d, bool fp64, int group, hipStream_t s) {
    if (y.n_events == 0) return hipErrorInvalidValue;  // the caller writes zeros instead
    return fp64 ? dense_pass_t<double>(y, d, group, s) : dense_pass_t<float>(y, d, group, s);
}

size_t batch_lds_bytes(int32_t n_layers, int threads) {
    return (size_t)(threads / kWave) * (size_t)n_layers * kAccStride * 8u;
}

hipError_t launch_batch_count(const void *const *occ, int32_t n_layers, int32_t catalog, bool fp64, int32_t *d_count,
                              unsigned long long *d_ovf_total, hipStream_t s) {
    return fp64 ? batch_count_t<double>(occ, n_layers, catalog, d_count, d_ovf_total, s)
                : batch_count_t<float>(occ, n_layers, catalog, d_count, d_ovf_total, s);
}

hipError_t launch_batch_fill(const void *const *occ, int32_t n_layers, int32_t catalog, bool fp64,
                             const int32_t *d_count, void *d_rec, uint8_t *d_ovf_lid, void *d_ovf_val,
                             unsigned long long *d_ovf_cursor, hipStream_t s) {
    return fp64 ? batch_fill_t<double>(occ, n_layers, catalog, d_count, d_rec, d_ovf_lid, d_ovf_val, d_ovf_cursor, s)
                : batch_fill_t<float>(occ, n_layers, catalog, d_count, d_rec, d_ovf_lid, d_ovf_val, d_ovf_cursor, s);
}

hipError_t launch_batch_pass(const YetView &y, const BatchTables &b, bool fp64, const BatchLaunch &cfg, hipStream_t s) {
    return fp64 ? batch_pass_t<double>(y, b, cfg, s) : batch_pass_t<float>(y, b, cfg, s);
}

}  // namespace ara
