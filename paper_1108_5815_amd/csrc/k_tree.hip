// k_tree.hip -- bounding cube, Morton keys, particle permutation and the
// level-by-level adaptive octree.
//
// Tree (paper: "Hierarchical N-body algorithms" clustering into cells;
// "Results": N_crit is the maximum number of particles per cell, the tree is
// adaptive): a cell at level L < 21 holding more than ncrit particles splits
// into its non-empty octants.  Because particles are sorted by Morton key, the
// octants of a cell are contiguous runs; their boundaries are found by binary
// search for the 8 child key prefixes, so one thread handles one cell.
// Cells are numbered level by level in key order (breadth-first).
#include "fmm_internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace fmm {
namespace {

constexpr int BB = 256;

// Instance k of a batch owns input particles [seg[k], seg[k+1]) (a single
// problem is the batch of one); the same ranges hold its particles after the
// sort, which orders by (instance, key, input index).
// Largest k in [0, nseg) with seg[k] <= i: the non-empty instance holding i.
__device__ inline int seg_of(const int64_t* __restrict__ seg, int nseg, int64_t i) {
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (seg[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Block b reduces particles [bt[2b], bt[2b+1]) (one instance) to part[6b..6b+6).
template <class F>
__global__ void k_bbox(const F* __restrict__ x, const F* __restrict__ y, const F* __restrict__ z,
                       const int64_t* __restrict__ bt, double* __restrict__ part, uint32_t* __restrict__ bad) {
    __shared__ double red[6][BB];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t nb = 0;
    const int64_t i1 = bt[2 * blockIdx.x + 1];
    for (int64_t i = bt[2 * blockIdx.x] + threadIdx.x; i < i1; i += BB) {
        double v[3] = {(double)x[i], (double)y[i], (double)z[i]};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (!isfinite(v[d])) {
                nb++;
                continue;
            }
            lo[d] = fmin(lo[d], v[d]);
            hi[d] = fmax(hi[d], v[d]);
        }
    }
    if (nb) atomicAdd(bad, nb);
    for (int d = 0; d < 3; d++) {
        red[d][threadIdx.x] = lo[d];
        red[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int st = BB / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int d = 0; d < 3; d++) {
                red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + st]);
                red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + st]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Instance k (one workgroup each): min / max over its blocks [pb[k], pb[k+1]) into out[6k..6k+6).
__global__ void k_bbox_final(const double* __restrict__ part, const int32_t* __restrict__ pb, int nseg,
                             double* __restrict__ out) {
    __shared__ double red[6][BB];
    const int k = blockIdx.x;
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = pb[k] + (int)threadIdx.x; b < pb[k + 1]; b += BB)
        for (int d = 0; d < 6; d++) v[d] = d < 3 ? fmin(v[d], part[b * 6 + d]) : fmax(v[d], part[b * 6 + d]);
    for (int d = 0; d < 6; d++) red[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int st = BB / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int d = 0; d < 6; d++)
                red[d][threadIdx.x] = d < 3 ? fmin(red[d][threadIdx.x], red[d][threadIdx.x + st])
                                            : fmax(red[d][threadIdx.x], red[d][threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x < 6) out[k * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// 21-bit quantisation: one FP64 subtraction, one FP64 multiplication, floor
__device__ inline uint64_t quantise(double v, double lo, double scale) {
    double t = __dmul_rn(__dsub_rn(v, lo), scale);
    double f = floor(t);
    uint64_t q = f <= 0.0 ? 0ull : (uint64_t)f;
    return q > 2097151ull ? 2097151ull : q;
}

template <class F>
__global__ void k_morton(const F* __restrict__ x, const F* __restrict__ y, const F* __restrict__ z,
                         int64_t n, const int64_t* __restrict__ seg, int nseg, const Frame* __restrict__ fr,
                         uint64_t* __restrict__ keys, uint32_t* __restrict__ idx, uint32_t* __restrict__ inst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = nseg > 1 ? seg_of(seg, nseg, i) : 0;
    const Frame f = fr[k];
    uint64_t qx = quantise((double)x[i], f.lox, f.scale);
    uint64_t qy = quantise((double)y[i], f.loy, f.scale);
    uint64_t qz = quantise((double)z[i], f.loz, f.scale);
    keys[i] = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
    idx[i] = (uint32_t)i;
    if (inst) inst[i] = (uint32_t)k;
}

// Second, stable pass of the batch sort: (instance of the k-th key-sorted
// particle, k), sorted by instance, gives the (instance, key, index) order.
__global__ void k_inst_keys(const uint32_t* __restrict__ idx, const uint32_t* __restrict__ inst, int64_t n,
                            uint32_t* __restrict__ ik, uint32_t* __restrict__ iv) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    ik[k] = inst[idx[k]];
    iv[k] = (uint32_t)k;
}

__global__ void k_gather_sorted(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ idx,
                                const uint32_t* __restrict__ perm, int64_t n, uint64_t* __restrict__ keys2,
                                uint32_t* __restrict__ idx2) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t j = perm[k];
    keys2[k] = keys[j];
    idx2[k] = idx[j];
}

template <class F>
__global__ void k_permute(const F* __restrict__ x, const F* __restrict__ y, const F* __restrict__ z,
                          const F* __restrict__ q, int64_t n, const uint32_t* __restrict__ idx,
                          float4* __restrict__ pts) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = idx[k];
    pts[k] = make_float4((float)x[i], (float)y[i], (float)z[i], (float)q[i]);
}

// first index in [lo, hi) with keys[i] >= v
// Cells of level L that split: one wave per cell finds the 7 octant
// boundaries (bnd[o] = first index whose key is >= the smallest key of octant
// o) with 64-ary searches run side by side: each round every lane samples one
// position per open interval and a ballot per octant shrinks it 64-fold, so a
// cell of 4M keys needs 4 rounds of independent loads instead of 7 binary
// searches of 22 dependent ones.  The boundaries are kept for the emit pass.
// The level's cells are [lvl[L], lvl[L+1]) (device memory, written by the
// previous level's emit); waves stride over them.
__global__ __launch_bounds__(256) void k_tree_count(const uint64_t* __restrict__ keys, CellArrays cells,
                                                    const int32_t* __restrict__ lvl, int L, int32_t ncrit,
                                                    uint32_t* __restrict__ nsplit, int32_t* __restrict__ bounds) {
    const int lane = threadIdx.x & 63;
    const int32_t c0 = lvl[L], c1 = lvl[L + 1];
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; wv < (int64_t)c1 - c0; wv += nw) {
        const int32_t c = c0 + (int32_t)wv;  // wave-uniform
        const int32_t b = cells.begin[c], e = cells.end[c];
        uint32_t cnt = 0;
        if (e - b > ncrit && L < kMaxLevel) {
            const int sh = 3 * (20 - L);  // bit position of the level-(L+1) digit
            const uint64_t pre3 = cells.prefix[c] << 3;
            int32_t lo[7], hi[7];
#pragma unroll
            for (int o = 0; o < 7; o++) {
                lo[o] = b;
                hi[o] = e;
            }
            bool open = true;
            while (open) {
                uint64_t kv[7];
#pragma unroll
                for (int o = 0; o < 7; o++) {
                    const int64_t span = hi[o] - lo[o];
                    kv[o] = span > 0 ? keys[lo[o] + (int32_t)((span * lane) >> 6)] : 0ull;
                }
                open = false;
#pragma unroll
                for (int o = 0; o < 7; o++) {
                    const int64_t span = hi[o] - lo[o];
                    if (span <= 0) continue;
                    const uint64_t tgt = (pre3 | (uint64_t)(o + 1)) << sh;
                    const int nb = __popcll(__ballot(kv[o] < tgt));  // samples below the boundary
                    if (nb == 0) {
                        hi[o] = lo[o];  // key[lo] >= tgt
                    } else {
                        const int32_t below = lo[o] + (int32_t)((span * (nb - 1)) >> 6);
                        const int32_t above = nb < 64 ? lo[o] + (int32_t)((span * nb) >> 6) : hi[o];
                        lo[o] = below + 1;
                        hi[o] = above;
                    }
                    if (hi[o] > lo[o]) open = true;
                }
            }
            int32_t prev = b;
#pragma unroll
            for (int o = 0; o < 7; o++) {
                cnt += lo[o] > prev ? 1u : 0u;
                prev = lo[o];
            }
            cnt += e > prev ? 1u : 0u;
            if (lane < 7) {
                int32_t v = lo[0];
#pragma unroll
                for (int o = 1; o < 7; o++)
                    if (lane == o) v = lo[o];
                bounds[(int64_t)(c - c0) * 7 + lane] = v;
            }
        }
        if (lane == 0) nsplit[c - c0] = cnt;
    }
}

__device__ inline void emit_cell(CellArrays cells, int32_t c, int32_t c0, int32_t c1, int L, uint32_t cnt,
                                 const uint32_t* __restrict__ off, const int32_t* __restrict__ bounds) {
    if (cnt == 0) {
        cells.child[c] = -1;
        cells.nchild[c] = 0;
        return;
    }
    int32_t first = c1 + (int32_t)off[c - c0];
    cells.child[c] = first;
    cells.nchild[c] = (int32_t)cnt;
    int32_t bnd[9];
    bnd[0] = cells.begin[c];
    bnd[8] = cells.end[c];
#pragma unroll
    for (int o = 1; o < 8; o++) bnd[o] = bounds[(int64_t)(c - c0) * 7 + o - 1];
    const uint64_t prefix = cells.prefix[c];
    int32_t k = first;
    for (int o = 0; o < 8; o++) {
        if (bnd[o + 1] <= bnd[o]) continue;
        cells.begin[k] = bnd[o];
        cells.end[k] = bnd[o + 1];
        cells.parent[k] = c;
        cells.level[k] = L + 1;
        cells.prefix[k] = (prefix << 3) | (uint64_t)o;
        cells.child[k] = -1;
        cells.nchild[k] = 0;
        k++;
    }
}

// Children of the level's cells at lvl[L+1] + off; writes lvl[L+2].  If the
// new level would pass the cell capacity, nothing splits, lvl[L+2] = lvl[L+1]
// (the tree stops) and *ovf is set: the caller grows the arrays and builds
// again.
__global__ void k_tree_emit(CellArrays cells, int32_t* __restrict__ lvl, int L, const uint32_t* __restrict__ nsplit,
                            const uint32_t* __restrict__ off, const uint32_t* __restrict__ nnew_p,
                            const int32_t* __restrict__ bounds, int32_t cap, uint32_t* __restrict__ ovf) {
    const int32_t c0 = lvl[L], c1 = lvl[L + 1];
    const uint32_t nnew = *nnew_p;
    const bool fits = (int64_t)c1 + nnew <= (int64_t)cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        lvl[L + 2] = fits ? c1 + (int32_t)nnew : c1;
        if (!fits) *ovf = 1u;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)c1 - c0; i += stride)
        emit_cell(cells, c0 + (int32_t)i, c0, c1, L, fits ? nsplit[i] : 0u, off, bounds);
}

__global__ void k_geometry(CellArrays cells, int32_t ncell, const int64_t* __restrict__ seg, int nseg,
                           const Frame* __restrict__ fr) {
    int32_t c = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= ncell) return;
    const Frame f = fr[nseg > 1 ? seg_of(seg, nseg, cells.begin[c]) : 0];
    const double lox = f.lox, loy = f.loy, loz = f.loz, h = f.h;
    int L = cells.level[c];
    uint64_t pre = cells.prefix[c];
    int32_t a[3] = {0, 0, 0};
    for (int b = 0; b < L; b++) {
        a[0] |= (int32_t)((pre >> (3 * b)) & 1u) << b;
        a[1] |= (int32_t)((pre >> (3 * b + 1)) & 1u) << b;
        a[2] |= (int32_t)((pre >> (3 * b + 2)) & 1u) << b;
    }
    int32_t r = 1 << (kMaxLevel - L);
    int4 g = make_int4((2 * a[0] + 1) * r, (2 * a[1] + 1) * r, (2 * a[2] + 1) * r, r);
    cells.geo[c] = g;
    double4 ph;
    ph.x = __dadd_rn(lox, __dmul_rn((double)g.x, h));
    ph.y = __dadd_rn(loy, __dmul_rn((double)g.y, h));
    ph.z = __dadd_rn(loz, __dmul_rn((double)g.z, h));
    ph.w = __dmul_rn((double)r, h);
    cells.ctr[c] = ph;
}

}  // namespace

void bbox(const void* x, const void* y, const void* z, int dtype, const int64_t* bt, int nblk,
          const int32_t* pb, int nseg, double* part, double* out, uint32_t* bad, hipStream_t s) {
    hipMemsetAsync(bad, 0, sizeof(uint32_t), s);
    if (nblk > 0) {
        if (dtype == 1)
            k_bbox<double><<<nblk, BB, 0, s>>>((const double*)x, (const double*)y, (const double*)z, bt, part, bad);
        else
            k_bbox<float><<<nblk, BB, 0, s>>>((const float*)x, (const float*)y, (const float*)z, bt, part, bad);
    }
    k_bbox_final<<<nseg, BB, 0, s>>>(part, pb, nseg, out);
}

void morton_keys(const void* x, const void* y, const void* z, int dtype, int64_t n, const int64_t* seg, int nseg,
                 const Frame* fr, uint64_t* keys, uint32_t* idx, uint32_t* inst, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = (unsigned)((n + 255) / 256);
    if (dtype == 1)
        k_morton<double><<<g, 256, 0, s>>>((const double*)x, (const double*)y, (const double*)z, n, seg, nseg, fr,
                                           keys, idx, inst);
    else
        k_morton<float><<<g, 256, 0, s>>>((const float*)x, (const float*)y, (const float*)z, n, seg, nseg, fr, keys,
                                          idx, inst);
}

void inst_keys(const uint32_t* idx, const uint32_t* inst, int64_t n, uint32_t* ik, uint32_t* iv, hipStream_t s) {
    if (n <= 0) return;
    k_inst_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(idx, inst, n, ik, iv);
}

void gather_sorted(const uint64_t* keys, const uint32_t* idx, const uint32_t* perm, int64_t n, uint64_t* keys2,
                   uint32_t* idx2, hipStream_t s) {
    if (n <= 0) return;
    k_gather_sorted<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(keys, idx, perm, n, keys2, idx2);
}

void permute_points(const void* x, const void* y, const void* z, const void* q, int dtype, int64_t n,
                    const uint32_t* idx, float4* pts, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = (unsigned)((n + 255) / 256);
    if (dtype == 1)
        k_permute<double><<<g, 256, 0, s>>>((const double*)x, (const double*)y, (const double*)z,
                                            (const double*)q, n, idx, pts);
    else
        k_permute<float><<<g, 256, 0, s>>>((const float*)x, (const float*)y, (const float*)z,
                                           (const float*)q, n, idx, pts);
}

// fixed grids sized for the widest level the capacity allows
void tree_count(const uint64_t* keys, CellArrays cells, const int32_t* lvl, int L, int32_t ncrit, uint32_t* nsplit,
                int32_t* bounds, int32_t cap, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>(((int64_t)cap + 3) / 4, 2048);
    k_tree_count<<<(unsigned)blocks, 256, 0, s>>>(keys, cells, lvl, L, ncrit, nsplit, bounds);
}

void tree_emit(CellArrays cells, int32_t* lvl, int L, const uint32_t* nsplit, const uint32_t* child_off,
               const uint32_t* nnew, const int32_t* bounds, int32_t cap, uint32_t* ovf, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>(((int64_t)cap + 255) / 256, 1024);
    k_tree_emit<<<(unsigned)blocks, 256, 0, s>>>(cells, lvl, L, nsplit, child_off, nnew, bounds, cap, ovf);
}

void cell_geometry(CellArrays cells, int32_t ncell, const int64_t* seg, int nseg, const Frame* fr, hipStream_t s) {
    if (ncell <= 0) return;
    k_geometry<<<(ncell + 255) / 256, 256, 0, s>>>(cells, ncell, seg, nseg, fr);
}

}  // namespace fmm
