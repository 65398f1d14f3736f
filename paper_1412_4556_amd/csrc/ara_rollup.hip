// Roll-up of year loss tables into programs (and of programs into a
// portfolio).  Section III nests layers in programs and programs in a
// portfolio without stating how their results combine; the reading here: a
// group's year loss in a trial is the binary64 sum of its inputs' year losses
// in that trial, added in increasing input order starting from 0.
//
// One thread per trial walks the groups; every load of a wave reads 64
// consecutive doubles of one input table, and each table is read once.
#include "ara_internal.h"

namespace ara {
namespace {

__global__ __launch_bounds__(256) void k_rollup(RollupTables a, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        for (int g = 0; g < a.n_groups; ++g) {
            double s = 0.0;
            for (int q = a.first[g]; q < a.first[g + 1]; ++q) s += a.in[q][i];
            a.out[g][i] = s;
        }
    }
}

}  // namespace

hipError_t launch_rollup(const RollupTables &a, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    const int64_t cap = (int64_t)cu_count() * 16;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_rollup, dim3((unsigned)blocks), dim3(256), 0, s, a, n);
    return hipGetLastError();
}

}  // namespace ara
