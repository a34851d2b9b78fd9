// k_p2p.hip -- near-field particle-particle sums.
//
// phi_i += sum_j q_j / r_ij,  E_i += sum_j q_j (x_i - x_j) / r_ij^3 over the
// source cells paired with the leaf of i or with any of its ancestors (the
// hybrid may pick particle-particle sums for non-leaf pairs, "Results").
//
// Layout: target-parallel, one wave per target leaf and no cross-wave
// reduction (the scheme the paper credits to Nyland et al., "Early
// application of GPUs").  Leaves hold fewer particles than a wave has lanes,
// so the wave is cut into G lane groups of `span` lanes; each lane holds TPL
// targets (register blocking: one source read feeds TPL interactions) and the
// groups split the sources.  The source cells of the leaf's list are
// concatenated into one stream: 64 list entries at a time are fetched
// lane-parallel, a wave prefix sum over their sizes maps stream positions to
// cells, and the wave copies the stream into an LDS chunk with all lanes
// busy.  Each group then takes a contiguous, equal share of the chunk, reads
// it from LDS (one address per group, a broadcast), accumulates in FP32 and
// adds the chunk's partial into FP64 per-target sums; the groups are summed
// in group order at the end, so results do not depend on timing.
//
// TPL (1, 2 or 4) is a tile shape chosen per leaf-size class by the
// library's autotuner; leaves are launched grouped by class.
//
// Only the leaf's own cell (or every cell for FP64 input, where distinct
// points may round to one FP32 point) needs the r = 0 guard: it is staged as
// a chunk of its own and left out of the stream.
#include "fmm_internal.h"

namespace fmm {
namespace {


template <bool GUARD>
__device__ inline void interact(const float3 P, const float4 Q, float4& f) {
    float dx = P.x - Q.x, dy = P.y - Q.y, dz = P.z - Q.z;
    float r2 = dx * dx + dy * dy + dz * dz;
    float inv = __builtin_amdgcn_rsqf(r2);
    if (GUARD) inv = r2 > 0.f ? inv : 0.f;
    float qi = Q.w * inv;
    f.w += qi;
    float qi3 = qi * inv * inv;
    f.x += qi3 * dx;
    f.y += qi3 * dy;
    f.z += qi3 * dz;
}

// Sources buf[j0, j1) against the lane's TPL targets, FP32 partials added to acc.
template <int TPL, bool GUARD>
__device__ inline void chunk_sum(const float4* buf, int j0, int j1, const float3 (&P)[TPL], double4 (&acc)[TPL]) {
    float4 f[TPL];
#pragma unroll
    for (int k = 0; k < TPL; k++) f[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    int j = j0;
    for (; j + 3 < j1; j += 4) {
        const float4 Q0 = buf[j], Q1 = buf[j + 1], Q2 = buf[j + 2], Q3 = buf[j + 3];
#pragma unroll
        for (int k = 0; k < TPL; k++) {
            interact<GUARD>(P[k], Q0, f[k]);
            interact<GUARD>(P[k], Q1, f[k]);
            interact<GUARD>(P[k], Q2, f[k]);
            interact<GUARD>(P[k], Q3, f[k]);
        }
    }
    for (; j < j1; j++) {
        const float4 Q = buf[j];
#pragma unroll
        for (int k = 0; k < TPL; k++) interact<GUARD>(P[k], Q, f[k]);
    }
#pragma unroll
    for (int k = 0; k < TPL; k++) {
        acc[k].x += f[k].x;
        acc[k].y += f[k].y;
        acc[k].z += f[k].z;
        acc[k].w += f[k].w;
    }
}

__device__ inline int wave_inclusive_scan(int v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

template <int TPL, bool GUARD_ALL>
__global__ __launch_bounds__(64) void k_p2p(const float4* __restrict__ pts, CellArrays c,
                                            const int32_t* __restrict__ leaves,
                                            const int32_t* __restrict__ off, const uint32_t* __restrict__ src,
                                            double4* __restrict__ near) {
    constexpr int CH = TPL <= 2 ? 256 : 128 * TPL;   // staged sources per chunk (8 KB of LDS at TPL = 4)
    __shared__ float4 buf[CH];
    __shared__ int s_pref[65];
    __shared__ int s_beg[64];
    static_assert(CH * sizeof(float4) >= 64 * TPL * sizeof(double4), "reduction does not fit the chunk");
    const int cell = leaves[blockIdx.x];
    const int32_t b = c.begin[cell], e = c.end[cell];
    const int lane = threadIdx.x;

    for (int32_t t0 = b; t0 < e; t0 += 64 * TPL) {
        const int ntc = min(e - t0, 64 * TPL);
        const int span = (ntc + TPL - 1) / TPL;
        const int G = 64 / span;
        const int g = lane / span, li = lane - g * span;
        const bool active = g < G;
        float3 P[TPL];
        double4 acc[TPL];
#pragma unroll
        for (int k = 0; k < TPL; k++) {
            const int t = li + k * span;
            const float4 v = pts[t0 + ((active && t < ntc) ? t : 0)];
            P[k] = make_float3(v.x, v.y, v.z);
            acc[k] = make_double4(0.0, 0.0, 0.0, 0.0);
        }
        // group g's equal share of a staged chunk of n sources
        auto share = [&](int n, int& j0, int& j1) {
            j0 = (g * n) / G;
            j1 = ((g + 1) * n) / G;
        };

        // (1) the leaf's own cell, guarded (left out of the stream below)
        if (!GUARD_ALL) {
            for (int32_t s0 = b; s0 < e; s0 += CH) {
                const int n = min(e - s0, CH);
                for (int k = lane; k < n; k += 64) buf[k] = pts[s0 + k];
                __syncthreads();
                int j0, j1;
                share(n, j0, j1);
                if (active) chunk_sum<TPL, true>(buf, j0, j1, P, acc);
                __syncthreads();
            }
        }

        // (2) every other source cell of the leaf's and its ancestors' lists
        int fill = 0;
        for (int A = cell; A >= 0; A = c.parent[A]) {
            const int32_t a1 = off[A + 1];
            for (int32_t a0 = off[A]; a0 < a1; a0 += 64) {
                const int nb = min(a1 - a0, 64);
                int sb = 0, ns = 0;
                if (lane < nb) {
                    const int s = (int)src[a0 + lane];
                    if (GUARD_ALL || s != cell) {
                        sb = c.begin[s];
                        ns = c.end[s] - sb;
                    }
                }
                const int incl = wave_inclusive_scan(ns, lane);
                const int tot = __shfl(incl, 63, 64);
                s_pref[lane + 1] = incl;
                if (lane == 0) s_pref[0] = 0;
                s_beg[lane] = sb;
                __syncthreads();
                for (int done = 0; done < tot;) {
                    const int take = min(tot - done, CH - fill);
                    for (int k = lane; k < take; k += 64) {
                        const int el = done + k;
                        // last entry whose prefix is <= el: the non-empty cell holding el
                        int lo = 0, hi = 64;
#pragma unroll
                        for (int it = 0; it < 6; it++) {
                            const int mid = (lo + hi) >> 1;
                            if (s_pref[mid] <= el) lo = mid;
                            else hi = mid;
                        }
                        buf[fill + k] = pts[s_beg[lo] + (el - s_pref[lo])];
                    }
                    fill += take;
                    done += take;
                    if (fill == CH) {
                        __syncthreads();
                        int j0, j1;
                        share(CH, j0, j1);
                        if (active) chunk_sum<TPL, GUARD_ALL>(buf, j0, j1, P, acc);
                        fill = 0;
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
        }
        if (fill > 0) {
            __syncthreads();
            int j0, j1;
            share(fill, j0, j1);
            if (active) chunk_sum<TPL, GUARD_ALL>(buf, j0, j1, P, acc);
            __syncthreads();
        }

        // (3) sum the groups in group order, through the chunk's LDS
        double4* red = reinterpret_cast<double4*>(buf);
        if (active) {
#pragma unroll
            for (int k = 0; k < TPL; k++) red[(g * span + li) * TPL + k] = acc[k];
        }
        __syncthreads();
        if (g == 0) {
#pragma unroll
            for (int k = 0; k < TPL; k++) {
                double4 s = red[li * TPL + k];
                for (int h = 1; h < G; h++) {
                    const double4 v = red[(h * span + li) * TPL + k];
                    s.x += v.x;
                    s.y += v.y;
                    s.z += v.z;
                    s.w += v.w;
                }
                const int t = li + k * span;
                if (t < ntc) near[t0 + t] = make_double4(s.w, s.x, s.y, s.z);
            }
        }
        __syncthreads();
    }
}

// P2P size class of a leaf: at most 8, 16, 32 or more targets
__global__ void k_leaf_class(CellArrays c, const int32_t* __restrict__ leaves, int32_t nleaf,
                             uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
    int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= nleaf) return;
    const int32_t cell = leaves[i];
    const int32_t nt = c.end[cell] - c.begin[cell];
    key[i] = nt <= 8 ? 0u : nt <= 16 ? 1u : nt <= 32 ? 2u : 3u;
    val[i] = (uint32_t)cell;
}

template <int TPL>
void launch(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves, const int32_t* off,
            const uint32_t* src, int guard_all, double4* near, hipStream_t s) {
    if (guard_all)
        k_p2p<TPL, true><<<nleaves, 64, 0, s>>>(pts, cells, leaves, off, src, near);
    else
        k_p2p<TPL, false><<<nleaves, 64, 0, s>>>(pts, cells, leaves, off, src, near);
}

}  // namespace

void leaf_class_keys(CellArrays cells, const int32_t* leaves, int32_t nleaf, uint32_t* key, uint32_t* val,
                     hipStream_t s) {
    if (nleaf <= 0) return;
    k_leaf_class<<<(nleaf + 255) / 256, 256, 0, s>>>(cells, leaves, nleaf, key, val);
}

void p2p(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves, const int32_t* p2p_off,
         const uint32_t* p2p_src, int guard_all, int tpl, double4* near, hipStream_t s) {
    if (nleaves <= 0) return;
    switch (tpl) {
        case 1: launch<1>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
        case 2: launch<2>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
        default: launch<4>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
    }
}

}  // namespace fmm
