// k_p2p.hip -- near-field particle-particle sums.
//
// phi_i += sum_j q_j / r_ij,  E_i += sum_j q_j (x_i - x_j) / r_ij^3 over the
// source cells paired with the leaf of i or with any of its ancestors (the
// hybrid may pick particle-particle sums for non-leaf pairs, "Results").
// Layout: target-parallel (one wave per target leaf, no cross-wave
// reduction, the scheme credited to Nyland et al. in "Early application of
// GPUs").  Leaves hold fewer particles than a wave has lanes, so a leaf of
// at most 32 (16) targets splits every source cell across 2 (4) lane groups
// that each take every 2nd (4th) source, and the groups are summed with
// cross-lane shuffles at the end.  Sources are read as float4 (x, y, z, q)
// from the Morton-sorted array; each source cell is summed in FP32 and added
// into FP64 per-target accumulators.  Only a leaf paired with itself (or FP64
// input, where distinct points may round to one FP32 point) needs the
// r = 0 guard.
#include "fmm_internal.h"

namespace fmm {
namespace {

__device__ inline void interact(const float4 P, const float4 Q, float& fp, float& fx, float& fy, float& fz) {
    float dx = P.x - Q.x, dy = P.y - Q.y, dz = P.z - Q.z;
    float r2 = dx * dx + dy * dy + dz * dz;
    float inv = __builtin_amdgcn_rsqf(r2);
    float qi = Q.w * inv;
    fp += qi;
    float qi3 = qi * inv * inv;
    fx += qi3 * dx;
    fy += qi3 * dy;
    fz += qi3 * dz;
}

__device__ inline void interact_guarded(const float4 P, const float4 Q, float& fp, float& fx, float& fy,
                                        float& fz) {
    float dx = P.x - Q.x, dy = P.y - Q.y, dz = P.z - Q.z;
    float r2 = dx * dx + dy * dy + dz * dz;
    float inv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
    float qi = Q.w * inv;
    fp += qi;
    float qi3 = qi * inv * inv;
    fx += qi3 * dx;
    fy += qi3 * dy;
    fz += qi3 * dz;
}

__global__ __launch_bounds__(64) void k_p2p(const float4* __restrict__ pts, CellArrays c,
                                            const int32_t* __restrict__ leaves,
                                            const int32_t* __restrict__ off, const uint32_t* __restrict__ src,
                                            int guard_all, double4* __restrict__ near) {
    const int cell = leaves[blockIdx.x];
    const int32_t b = c.begin[cell], e = c.end[cell];
    const int32_t nt = e - b;
    const int G = nt <= 16 ? 4 : (nt <= 32 ? 2 : 1);
    const int span = 64 / G;
    const int lane = threadIdx.x;
    const int g = lane / span, li = lane - g * span;
    for (int32_t ch = b; ch < e; ch += span) {
        const int32_t i = ch + li;
        const bool valid = i < e;
        const float4 P = pts[valid ? i : b];
        double ap = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
        for (int A = cell; A >= 0; A = c.parent[A]) {
            const int32_t a1 = off[A + 1];
            for (int32_t a = off[A]; a < a1; a++) {
                const int s = (int)src[a];
                const int32_t sb = c.begin[s], se = c.end[s];
                float fp = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
                if (s == cell || guard_all) {
                    for (int32_t j = sb + g; j < se; j += G) interact_guarded(P, pts[j], fp, fx, fy, fz);
                } else {
                    int32_t j = sb + g;
                    for (; j + 3 * G < se; j += 4 * G) {
                        float4 Q0 = pts[j], Q1 = pts[j + G], Q2 = pts[j + 2 * G], Q3 = pts[j + 3 * G];
                        interact(P, Q0, fp, fx, fy, fz);
                        interact(P, Q1, fp, fx, fy, fz);
                        interact(P, Q2, fp, fx, fy, fz);
                        interact(P, Q3, fp, fx, fy, fz);
                    }
                    for (; j < se; j += G) interact(P, pts[j], fp, fx, fy, fz);
                }
                ap += fp;
                ax += fx;
                ay += fy;
                az += fz;
            }
        }
        for (int m = span; m < 64; m <<= 1) {
            ap += __shfl_xor(ap, m, 64);
            ax += __shfl_xor(ax, m, 64);
            ay += __shfl_xor(ay, m, 64);
            az += __shfl_xor(az, m, 64);
        }
        if (g == 0 && valid) near[i] = make_double4(ap, ax, ay, az);
    }
}

}  // namespace

void p2p(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves, const int32_t* p2p_off,
         const uint32_t* p2p_src, int guard_all, double4* near, hipStream_t s) {
    if (nleaves <= 0) return;
    k_p2p<<<nleaves, 64, 0, s>>>(pts, cells, leaves, p2p_off, p2p_src, guard_all, near);
}

}  // namespace fmm
