// CPU check of the trial passes' YET load indexing (the functions of
// ara_index.h that the kernels call).  For trials of every length 0..1001
// placed at every start modulo 4 in a 16-byte aligned YET, and for
// fixed-length YETs, it walks the loads the fused and batched passes issue
// (a first group of G chunks, then further groups or single chunks) and
// checks that every 16-byte load starts on a granule at or below the YET's
// last granule, that a load holding a trial element is never moved by the
// clamp, and that every element of the trial is taken exactly once and no
// element outside it.  Prints "ok" and exits 0, else reports the first
// failing case and exits 1.
#include <cstdio>
#include <vector>

#include "../paper_1412_4556_amd/csrc/ara_index.h"

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
    std::printf("ok %lld cases\n", cases);
    return 0;
}
