// k_p2p.hip -- near-field particle-particle sums.
//
// phi_i += sum_j q_j / r_ij,  E_i += sum_j q_j (x_i - x_j) / r_ij^3 over the
// source cells paired with the leaf of i or with any of its ancestors (the
// hybrid may pick particle-particle sums for non-leaf pairs, "Results").
//
// Layout: target-parallel, one wave per target leaf and no cross-wave
// reduction (the scheme the paper credits to Nyland et al., "Early
// application of GPUs").  Leaves hold fewer particles than a wave has lanes,
// so the wave is cut into G lane groups; the groups split the sources.  The
// source cells of the leaf's list are concatenated into one stream: 64 list
// entries at a time are fetched lane-parallel, a wave prefix sum over their
// sizes maps stream positions to cells, and the wave copies the stream into
// an LDS chunk with all lanes busy.  Group g of G then takes sources g,
// g + G, g + 2G, ... of the chunk and reads them from LDS (one address per
// group, a broadcast; at each step the groups read neighbouring addresses,
// which lie in distinct banks), accumulates in FP32 and adds the chunk's
// partial into FP64 per-target sums; the groups are summed in group order at
// the end, so results do not depend on timing.
//
// Two forms of tile, chosen per leaf-size class by the library's autotuner
// (leaves are launched grouped by class):
//  - vector (shape TPL = 1, 2 or 4 targets per lane): every operation on the
//    VALU, one source read feeding TPL interactions;
//  - matrix core (shape -TPL, TPL = 1, 2 or 4 targets per lane): the VALU
//    forms only each pair's 1/r and 1/r^3, and the sums over sources run as
//    rank-1 updates on v_mfma_f32_4x4x1f32 (16 blocks of 4 targets x 4
//    columns per instruction): phi from A = 1/r against B = q, and the field from
//    A = 1/r^3 against B = (q, q x~, q y~, q z~), the source's charge and
//    charge-weighted position relative to an origin in the target leaf,
//    giving E = x~_i sum(q/r^3) - sum(q x~/r^3).  The relative origin keeps
//    the cancellation of that difference to about eps_32 (|x~_i| + |x~_j|)/r
//    of a pair's field.
//
// Only the leaf's own cell (or every cell for FP64 input, where distinct
// points may round to one FP32 point) needs the r = 0 guard: it is staged as
// a chunk of its own and left out of the stream.
#include "fmm_internal.h"

#include <type_traits>

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

// Sources g, g + G, g + 2G, ... of buf[0, n) (group g of G) against the
// lane's TPL targets, FP32 partials added to acc.
template <int TPL, bool GUARD>
__device__ inline void chunk_sum(const float4* buf, int g, int G, int n, const float3 (&P)[TPL], double4 (&acc)[TPL]) {
    float4 f[TPL];
#pragma unroll
    for (int k = 0; k < TPL; k++) f[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    int j = g;
    for (; j + 3 * G < n; j += 4 * G) {
        const float4 Q0 = buf[j], Q1 = buf[j + G], Q2 = buf[j + 2 * G], Q3 = buf[j + 3 * G];
#pragma unroll
        for (int k = 0; k < TPL; k++) {
            interact<GUARD>(P[k], Q0, f[k]);
            interact<GUARD>(P[k], Q1, f[k]);
            interact<GUARD>(P[k], Q2, f[k]);
            interact<GUARD>(P[k], Q3, f[k]);
        }
    }
    for (; j < n; j += G) {
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

        // (1) the leaf's own cell, guarded (left out of the stream below)
        if (!GUARD_ALL) {
            for (int32_t s0 = b; s0 < e; s0 += CH) {
                const int n = min(e - s0, CH);
                for (int k = lane; k < n; k += 64) buf[k] = pts[s0 + k];
                __syncthreads();
                if (active) chunk_sum<TPL, true>(buf, g, G, n, P, acc);
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
                        if (active) chunk_sum<TPL, GUARD_ALL>(buf, g, G, CH, P, acc);
                        fill = 0;
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
        }
        if (fill > 0) {
            __syncthreads();
            if (active) chunk_sum<TPL, GUARD_ALL>(buf, g, G, fill, P, acc);
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


typedef float v4f __attribute__((ext_vector_type(4)));

// 1/r of one pair (0 for coincident points when guarded; +inf padding gives 0)
template <bool GUARD>
__device__ inline float pair_inv(const float3 P, const float4 Q) {
    const float dx = P.x - Q.x, dy = P.y - Q.y, dz = P.z - Q.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float inv = __builtin_amdgcn_rsqf(r2);
    return GUARD ? (r2 > 0.f ? inv : 0.f) : inv;
}

// Sources [j0, j0 + m) of a staged chunk against the lane's TPL targets on
// the matrix cores.  Lane l is row l%4 of block l/4 for A and column l%4 for
// B; all lanes of a block walk the same sources.  Returns the FP32 partials
// per target set k (D registers: row r of the lane's block, column l%4).
// With one or two target sets, two accumulator sets alternate by source so
// that consecutive products do not wait for each other.
template <int TPL, bool GUARD>
__device__ inline void chunk_mfma(const float4* buf, const float* bq, int j0, int m, int comp, const float3 (&P)[TPL],
                                  v4f (&sp)[TPL], v4f (&se)[TPL]) {
    constexpr int NSET = TPL >= 4 ? 1 : 2;
    v4f pa[NSET][TPL], ea[NSET][TPL];
#pragma unroll
    for (int u = 0; u < NSET; u++)
#pragma unroll
        for (int k = 0; k < TPL; k++) {
            pa[u][k] = v4f{0.f, 0.f, 0.f, 0.f};
            ea[u][k] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    int jj = 0;
    for (; jj + 1 < m; jj += 2) {
        const int j = j0 + jj;
        const float4 Q0 = buf[j], Q1 = buf[j + 1];
        const float b0 = bq[4 * j + comp], b1 = bq[4 * j + 4 + comp];
#pragma unroll
        for (int k = 0; k < TPL; k++) {
            const float i0 = pair_inv<GUARD>(P[k], Q0);
            pa[0][k] = __builtin_amdgcn_mfma_f32_4x4x1f32(i0, b0, pa[0][k], 0, 0, 0);
            ea[0][k] = __builtin_amdgcn_mfma_f32_4x4x1f32(i0 * i0 * i0, b0, ea[0][k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < TPL; k++) {
            const float i1 = pair_inv<GUARD>(P[k], Q1);
            pa[NSET - 1][k] = __builtin_amdgcn_mfma_f32_4x4x1f32(i1, b1, pa[NSET - 1][k], 0, 0, 0);
            ea[NSET - 1][k] = __builtin_amdgcn_mfma_f32_4x4x1f32(i1 * i1 * i1, b1, ea[NSET - 1][k], 0, 0, 0);
        }
    }
    if (jj < m) {
        const int j = j0 + jj;
        const float4 Q0 = buf[j];
        const float b0 = bq[4 * j + comp];
#pragma unroll
        for (int k = 0; k < TPL; k++) {
            const float i0 = pair_inv<GUARD>(P[k], Q0);
            pa[0][k] = __builtin_amdgcn_mfma_f32_4x4x1f32(i0, b0, pa[0][k], 0, 0, 0);
            ea[0][k] = __builtin_amdgcn_mfma_f32_4x4x1f32(i0 * i0 * i0, b0, ea[0][k], 0, 0, 0);
        }
    }
#pragma unroll
    for (int k = 0; k < TPL; k++) {
        sp[k] = pa[0][k];
        se[k] = ea[0][k];
        if (NSET > 1) {
            sp[k] += pa[NSET - 1][k];
            se[k] += ea[NSET - 1][k];
        }
    }
}

// Matrix-core form with TPL targets per lane.  A pass covers up to 64 TPL
// targets: span4 lanes (a multiple of 4) per group, lane li of a group holds
// targets li + k span4, and G = 64 / span4 groups split the sources.  The
// FP64 per-target sums live in LDS (slot g span4 TPL + target, 5 values:
// phi, sum q/r^3, sum q x~/r^3, ...), each value owned by one lane.
template <int TPL, bool GUARD_ALL>
__global__ __launch_bounds__(64) void k_p2p_mfma(const float4* __restrict__ pts, CellArrays c,
                                                 const int32_t* __restrict__ leaves,
                                                 const int32_t* __restrict__ off, const uint32_t* __restrict__ src,
                                                 double4* __restrict__ near) {
    constexpr int CH = 256;        // staged sources per chunk
    constexpr int CHP = CH + 16;   // room for the padding that evens the group shares
    constexpr int NT = 64 * TPL;   // targets per pass
    __shared__ float4 buf[CHP];    // source (x, y, z, q)
    __shared__ float4 bqv[CHP];    // source (q, q x~, q y~, q z~)
    __shared__ double red[NT * 5];
    __shared__ int s_pref[65];
    __shared__ int s_beg[64];
    const float* bq = reinterpret_cast<const float*>(bqv);
    const int cell = leaves[blockIdx.x];
    const int32_t b = c.begin[cell], e = c.end[cell];
    const int lane = threadIdx.x;
    const int blk = lane >> 2, row = lane & 3;  // A row and B/D column within the 4x4 block
    const float4 O = pts[b];                    // origin of the relative positions
    const float INF = __builtin_inff();

    auto stage = [&](int k, const float4 v) {
        buf[k] = v;
        bqv[k] = make_float4(v.w, v.w * (v.x - O.x), v.w * (v.y - O.y), v.w * (v.z - O.z));
    };

    for (int32_t t0 = b; t0 < e; t0 += NT) {
        const int ntc = min(e - t0, NT);
        const int nbk = ((ntc + TPL - 1) / TPL + 3) >> 2;  // blocks of 4 lanes per group
        const int span4 = 4 * nbk;
        const int G = 16 / nbk;                            // groups of nbk blocks
        const int g = blk / nbk;
        const bool active = g < G;
        const int gg = active ? g : 0;  // idle blocks repeat group 0's work, results unused
        const int bb = blk - g * nbk;   // block within the group
        float3 P[TPL];
#pragma unroll
        for (int k = 0; k < TPL; k++) {
            const int t = bb * 4 + row + k * span4;
            const float4 v = pts[t0 + ((active && t < ntc) ? t : 0)];
            P[k] = make_float3(v.x, v.y, v.z);
        }
        for (int i = lane; i < G * span4 * TPL * 5; i += 64) red[i] = 0.0;

        // the group shares of a staged chunk of n sources: m each, padded with
        // zero-charge points at infinity (their 1/r is 0); the FP32 partials
        // are added into the FP64 sums in LDS
        auto flush = [&](int n, auto guard) {
            constexpr bool GD = decltype(guard)::value;
            const int m = (n + G - 1) / G;
            for (int k = n + lane; k < G * m; k += 64) {
                buf[k] = make_float4(INF, INF, INF, 0.f);
                bqv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            __syncthreads();
            v4f sp[TPL], se[TPL];
            chunk_mfma<TPL, GD>(buf, bq, gg * m, m, row, P, sp, se);
            if (active) {
#pragma unroll
                for (int k = 0; k < TPL; k++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        double* slot = red + (g * span4 * TPL + bb * 4 + r + k * span4) * 5;
                        slot[1 + row] += (double)se[k][r];
                        if (row == 0) slot[0] += (double)sp[k][r];
                    }
            }
            __syncthreads();
        };

        // (1) the leaf's own cell, guarded (left out of the stream below)
        if (!GUARD_ALL) {
            for (int32_t s0 = b; s0 < e; s0 += CH) {
                const int n = min(e - s0, CH);
                for (int k = lane; k < n; k += 64) stage(k, pts[s0 + k]);
                flush(n, std::true_type{});
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
                        int lo = 0, hi = 64;
#pragma unroll
                        for (int it = 0; it < 6; it++) {
                            const int mid = (lo + hi) >> 1;
                            if (s_pref[mid] <= el) lo = mid;
                            else hi = mid;
                        }
                        stage(fill + k, pts[s_beg[lo] + (el - s_pref[lo])]);
                    }
                    fill += take;
                    done += take;
                    if (fill == CH) {
                        flush(CH, std::integral_constant<bool, GUARD_ALL>{});
                        fill = 0;
                    }
                }
                __syncthreads();
            }
        }
        if (fill > 0) flush(fill, std::integral_constant<bool, GUARD_ALL>{});

        // (3) sum the groups in group order
        for (int t = lane; t < ntc; t += 64) {
            double sum[5];
#pragma unroll
            for (int k = 0; k < 5; k++) sum[k] = red[t * 5 + k];
            for (int h = 1; h < G; h++)
#pragma unroll
                for (int k = 0; k < 5; k++) sum[k] += red[(h * span4 * TPL + t) * 5 + k];
            const float4 T = pts[t0 + t];
            const double xt = (double)(T.x - O.x), yt = (double)(T.y - O.y), zt = (double)(T.z - O.z);
            near[t0 + t] = make_double4(sum[0], xt * sum[1] - sum[2], yt * sum[1] - sum[3], zt * sum[1] - sum[4]);
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
void launch_mfma(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves, const int32_t* off,
                 const uint32_t* src, int guard_all, double4* near, hipStream_t s) {
    if (guard_all)
        k_p2p_mfma<TPL, true><<<nleaves, 64, 0, s>>>(pts, cells, leaves, off, src, near);
    else
        k_p2p_mfma<TPL, false><<<nleaves, 64, 0, s>>>(pts, cells, leaves, off, src, near);
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
        case -1: launch_mfma<1>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
        case -2: launch_mfma<2>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
        case -4: launch_mfma<4>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
        case 1: launch<1>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
        case 2: launch<2>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
        default: launch<4>(pts, cells, leaves, nleaves, p2p_off, p2p_src, guard_all, near, s); break;
    }
}

}  // namespace fmm
