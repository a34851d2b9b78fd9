// k_work.hip -- work counts of the interaction lists (for rooflines and
// cost records): sum over the list of n_t * n_s (particle pairs) or n_t
// (target particles), where n = particles of the cell.  Integer sums, so the
// result does not depend on the order of the atomic additions.
#include "fmm_internal.h"

namespace fmm {
namespace {

__global__ void k_pair_work(const uint32_t* __restrict__ tgt, const uint32_t* __restrict__ src, int64_t n,
                            CellArrays c, int both, unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[256];
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint32_t t = tgt[i];
        const unsigned long long nt = (unsigned long long)(c.end[t] - c.begin[t]);
        if (both) {
            const uint32_t s = src[i];
            acc += nt * (unsigned long long)(c.end[s] - c.begin[s]);
        } else {
            acc += nt;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

}  // namespace

void pair_work(const uint32_t* tgt, const uint32_t* src, int64_t n, CellArrays cells, int both, uint64_t* out,
               hipStream_t s) {
    (void)hipMemsetAsync(out, 0, sizeof(uint64_t), s);
    if (n <= 0) return;
    int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    k_pair_work<<<nb, 256, 0, s>>>(tgt, src, n, cells, both, (unsigned long long*)out);
}

}  // namespace fmm
