// CPU check of the kernels' index arithmetic (the functions of ara_index.h
// that the kernels call).
// - YET loads: for trials of every length 0..1001 placed at every start
//   modulo 4 in a 16-byte aligned YET, and for fixed-length YETs, it walks
//   the loads the fused and batched passes issue (a first group of G chunks,
//   then further groups or single chunks) and checks that every 16-byte load
//   starts on a granule at or below the YET's last granule, that a load
//   holding a trial element is never moved by the clamp, and that every
//   element of the trial is taken exactly once and no element outside it.
// - Fused table build: for catalogue sizes from 1 to 2^31 - 1 (the filter
//   geometry the library chooses for each), it checks that every event's
//   range and offset give back the event, that each range's count word is
//   one of the range's own block-filter words and inside the filter, and
//   that each range's list (8-byte entries, for 4- and 8-byte table values)
//   stays inside the range's part of the table.
// Prints "ok" and exits 0, else reports the first failing case and exits 1.
#include <cstdio>
#include <vector>

#include "../paper_1412_4556_amd/csrc/ara_index.h"
#include "../paper_1412_4556_amd/csrc/ara_internal.h"

using namespace ara;

namespace {

int fail(const char *what, long long b, long long e, long long n, long long p) {
    std::printf("FAIL %s: trial [%lld, %lld) of %lld events, position %lld\n", what, b, e, n, p);
    return 1;
}

// One chunk at base: lanes 0..63 each load the granule of p = base + 4 lane.
int chunk(bool fixed, long long base, long long b, long long e, long long n, std::vector<int> &seen) {
    const long long last = (n - 1) & ~3LL;
    const long long lim = load_limit(fixed, b, e, last);
    for (int lane = 0; lane < 64; ++lane) {
        const long long p = base + 4 * lane;
        const long long q = clamped_granule(p, lim);
        if (q < 0 || q % 4 != 0 || q > last) return fail("load outside the YET's granules", b, e, n, p);
        const unsigned m = granule_valid(fixed, p, b, e);
        if (m != 0 && q != p) return fail("clamp moved a load that holds trial elements", b, e, n, p);
        for (int v = 0; v < 4; ++v) {
            if (!((m >> v) & 1u)) continue;
            const long long x = p + v;
            if (x < b || x >= e) return fail("element outside the trial marked valid", b, e, n, x);
            ++seen[x - b];
        }
    }
    return 0;
}

// The fused pass (G chunks, then whole groups for fixed-length trials or
// single chunks otherwise) or the batched pass (groups of G; chunks past
// the trial's end are loaded and skipped, which changes no load).
int walk(bool fixed, bool single_tail, int G, long long b, long long e, long long n) {
    std::vector<int> seen((size_t)(e - b), 0);
    const long long base0 = chunk_start(true, b);
    for (int c = 0; c < G; ++c)
        if (chunk(fixed, base0 + c * kChunkEvents, b, e, n, seen)) return 1;
    const long long span = G * kChunkEvents;
    const int tg = single_tail ? 1 : G;
    for (long long base = base0 + span; base < e; base += tg * kChunkEvents)
        for (int c = 0; c < tg; ++c)
            if (chunk(fixed, base + c * kChunkEvents, b, e, n, seen)) return 1;
    for (long long i = 0; i < e - b; ++i)
        if (seen[(size_t)i] != 1) return fail("element not taken exactly once", b, e, n, b + i);
    return 0;
}

int build_fail(const char *what, long long C, long long g, long long e) {
    std::printf("FAIL %s: catalogue %lld, range %lld, event %lld\n", what, C, g, e);
    return 1;
}

int build_event(int32_t C, int32_t fshift, int32_t n_fwords, int64_t groups, int32_t e) {
    const int64_t g = build_range_of(e);
    const uint32_t off = build_range_offset(e);
    if (g < 0 || g >= groups) return build_fail("event's range outside the ranges", C, g, e);
    if (g * kBuildRange + off != (int64_t)e) return build_fail("range and offset do not give the event", C, g, e);
    if ((int64_t)off >= range_events(g, C)) return build_fail("offset past the range's table entries", C, g, e);
    if (range_count_word(g, fshift) >= n_fwords) return build_fail("count word outside the block filter", C, g, e);
    return 0;
}

// One catalogue size: every range, and the events at every range boundary
// (every event up to 2^20 events).
int build_catalogue(int32_t C, long long &cases) {
    int32_t fshift = 0, n_fwords = 0, n_hwords = 0, hshift = 0;
    filter_geometry(C, fshift, n_fwords, n_hwords, hshift);
    if (!build_ranges_cover_words(fshift)) return 0;  // built by the pool-layer kernels instead
    const int ws = 5 + fshift;
    const int64_t groups = build_ranges(C);
    if (groups * kBuildRange < (int64_t)C + 1 || (groups - 1) * kBuildRange > (int64_t)C)
        return build_fail("ranges do not cover the table exactly", C, groups, -1);
    int64_t prev = -1;
    for (int64_t g = 0; g < groups; ++g) {
        const int64_t n = range_events(g, C);
        if (n < 1 || n > kBuildRange) return build_fail("range size", C, g, -1);
        if (g * kBuildRange + n > (int64_t)C + 1) return build_fail("range past the table's end", C, g, -1);
        const int64_t w = range_count_word(g, fshift);
        if (w != (g * kBuildRange) >> ws || w <= prev) return build_fail("count word not the range's first", C, g, -1);
        if ((((g + 1) * kBuildRange) >> ws) - w != (kBuildRange >> ws))
            return build_fail("range does not cover whole filter words", C, g, -1);
        prev = w;
        if (w >= n_fwords && g * kBuildRange < (int64_t)C)
            return build_fail("a range with catalogue events has its count past the filter", C, g, -1);
        for (int vb : {4, 8}) {
            const int cap = range_capacity(g, C, vb);
            if (cap < 0 || cap > kBuildList) return build_fail("list capacity", C, g, -1);
            if ((int64_t)cap * 8 > n * vb) return build_fail("list past the range's part of the table", C, g, -1);
            if (g * kBuildRange * vb + (int64_t)cap * 8 > ((int64_t)C + 1) * vb)
                return build_fail("list past the table's end", C, g, -1);
        }
        ++cases;
    }
    if (C <= (1 << 20)) {
        for (int32_t e = 0; e < C; ++e)
            if (build_event(C, fshift, n_fwords, groups, e)) return 1;
    } else {
        for (int64_t g = 0; g < groups; ++g)
            for (long long d : {-1LL, 0LL, 1LL, (long long)kBuildRange - 1}) {
                const int64_t e = g * kBuildRange + d;
                if (e >= 0 && e < (int64_t)C && build_event(C, fshift, n_fwords, groups, (int32_t)e)) return 1;
            }
    }
    return 0;
}

}  // namespace

int main() {
    long long cases = 0;
    // variable-length trials (offsets), 16-byte aligned YET, every start mod 4
    for (long long len = 0; len <= 1001; ++len)
        for (long long pre = 0; pre < 8; ++pre)
            for (long long post : {0LL, 1LL, 2LL, 3LL, 4LL, 5LL, 300LL}) {
                const long long b = pre, e = pre + len, n = e + post;
                if (n < 1) continue;  // the passes run only on a YET with events
                for (int G : {1, 2, 4, 8}) {
                    if (walk(false, true, G, b, e, n)) return 1;   // fused pass, single-chunk tails
                    if (walk(false, false, G, b, e, n)) return 1;  // batched pass, whole groups
                    ++cases;
                }
            }
    // fixed-length trials: every trial a non-zero multiple of 4 events
    for (long long K = 4; K <= 1004; K += 4)
        for (long long T : {1LL, 2LL, 3LL})
            for (long long i = 0; i < T; ++i)
                for (int G : {1, 2, 4, 8}) {
                    if (walk(true, false, G, i * K, (i + 1) * K, T * K)) return 1;
                    ++cases;
                }
    // the fused table build's lists and counts
    for (long long C : {1LL, 2LL, 31LL, 32LL, 33LL, 63LL, 64LL, 8191LL, 8192LL, 8193LL, 16383LL, 16384LL, 100000LL,
                        (1LL << 20) - 1, 1LL << 20, (1LL << 20) + 1, 2000000LL, 2000000LL + 8191, 1LL << 21,
                        (1LL << 21) + 1, 33554431LL, 33554432LL, 33562624LL, 40000000LL, (1LL << 28) - 1, 1LL << 28,
                        (1LL << 28) + 1, 2147483647LL})
        if (build_catalogue((int32_t)C, cases)) return 1;
    std::printf("ok %lld cases\n", cases);
    return 0;
}
