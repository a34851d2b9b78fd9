// k_far.hip -- P2M, and the far-field evaluation at the target particles with
// the final sum.
//
// For each target particle of a leaf: L2P of the leaf's local expansion, M2P
// of every cell-particle source paired with the leaf or one of its ancestors
// (treecode and hybrid policies, "Results"), plus the particle-particle part,
// summed in FP64 and written in the caller's particle order.
//
// Potential and gradient come from re-centring the expansion at the target
// point (Greengard & Rokhlin theorems 3.4/3.5): the potential is the degree-0
// term and the gradient the degree-1 terms, whose weights are tabulated on
// the host.  The order p is a template parameter, so every loop unrolls and
// each solid harmonic is consumed by the contraction as soon as the Cartesian
// recurrence produces it: nothing per particle goes to LDS, only the leaf's
// local expansion and the current source multipole (read as broadcasts).
#include "cart.h"
#include "fmm_internal.h"

namespace fmm {
namespace {

struct cf {
    float re, im;
};

// coefficient (n, m), any sign of m, from a real-layout array (conj for m < 0)
__device__ inline cf hat(const float* row, int n, int m) {
    if (m == 0) return {row[n * n], 0.f};
    if (m > 0) return {row[n * n + 2 * m - 1], row[n * n + 2 * m]};
    return {row[n * n - 2 * m - 1], -row[n * n - 2 * m]};
}

template <int P, class Fn>
__device__ inline void regular_walk_t(float x, float y, float z, const float* __restrict__ rc, Fn f) {
    const float r2 = x * x + y * y + z * z;
    float mre = 1.f, mim = 0.f;
#pragma unroll
    for (int m = 0; m <= P; m++) {
        if (m > 0) {
            const float c = rc[kRcC1 + m];
            const float nre = c * (x * mre - y * mim), nim = c * (x * mim + y * mre);
            mre = nre;
            mim = nim;
        }
        f(m, m, mre, mim);
        if (m < P) {
            const float c2 = rc[kRcC2 + m] * z;
            float p1re = c2 * mre, p1im = c2 * mim, p0re = mre, p0im = mim;
            f(m + 1, m, p1re, p1im);
#pragma unroll
            for (int n = m + 2; n <= P; n++) {
                const int t = n * (n + 1) / 2 + m;
                const float A = rc[kRcA + t] * z, B = rc[kRcB + t] * r2;
                const float nre = A * p1re - B * p0re, nim = A * p1im - B * p0im;
                f(n, m, nre, nim);
                p0re = p1re;
                p0im = p1im;
                p1re = nre;
                p1im = nim;
            }
        }
    }
}

template <int P, class Fn>
__device__ inline void irregular_walk_t(float x, float y, float z, const float* __restrict__ rc, Fn f) {
    const float r2 = x * x + y * y + z * z;
    const float ir2 = 1.f / r2;
    float mre = sqrtf(ir2), mim = 0.f;
#pragma unroll
    for (int m = 0; m <= P; m++) {
        if (m > 0) {
            const float c = rc[kRcC1 + m] * ir2;
            const float nre = c * (x * mre - y * mim), nim = c * (x * mim + y * mre);
            mre = nre;
            mim = nim;
        }
        f(m, m, mre, mim);
        if (m < P) {
            const float c2 = rc[kRcC2 + m] * z * ir2;
            float p1re = c2 * mre, p1im = c2 * mim, p0re = mre, p0im = mim;
            f(m + 1, m, p1re, p1im);
#pragma unroll
            for (int n = m + 2; n <= P; n++) {
                const int t = n * (n + 1) / 2 + m;
                const float A = rc[kRcA + t] * z * ir2, B = rc[kRcB + t] * ir2;
                const float nre = A * p1re - B * p0re, nim = A * p1im - B * p0im;
                f(n, m, nre, nim);
                p0re = p1re;
                p0im = p1im;
                p1re = nre;
                p1im = nim;
            }
        }
    }
}

// Local expansion Lt (scaled, real layout) at the point x-hat = (x - c)/r:
// phi-hat and the degree-1 terms of the expansion re-centred at the point.
template <int P>
__device__ inline void l2p_point(const float* Lt, const float* __restrict__ g, float x, float y, float z,
                                 const float* __restrict__ rc, float& phi, float& l10, float& l1re, float& l1im) {
    constexpr int K = (P + 1) * (P + 1);
    regular_walk_t<P>(x, y, z, rc, [&](int a, int b, float sre, float sim) {
        const cf L = hat(Lt, a, b);
        phi += (b == 0 ? 1.f : 2.f) * (L.re * sre - L.im * sim);
        if (a + 1 <= P) {
            const int n = a + 1;
            const float G0 = g[n * n + n + b] + (b > 0 ? g[n * n + n - b] : 0.f);
            const cf Ln = hat(Lt, n, b);
            l10 += G0 * (Ln.re * sre - Ln.im * sim);
            const float g1 = g[K + n * n + n + b + 1];
            const cf L1 = hat(Lt, n, b + 1);
            l1re += g1 * (L1.re * sre - L1.im * sim);
            l1im += g1 * (L1.re * sim + L1.im * sre);
            if (b >= 1) {
                const float g2 = g[K + n * n + n + 1 - b];
                const cf L2 = hat(Lt, n, 1 - b);
                l1re += g2 * (L2.re * sre + L2.im * sim);
                l1im += g2 * (L2.im * sre - L2.re * sim);
            }
        }
    });
}

// Multipole Ms (scaled, real layout) at x-hat = (x - c)/r: phi-hat and the
// degree-1 terms of its conversion into a local expansion at the point.
template <int P>
__device__ inline void m2p_point(const float* Ms, const float* __restrict__ h, float x, float y, float z,
                                 const float* __restrict__ rc, float& phi, float& l10, float& l1re, float& l1im) {
    constexpr int K = (P + 1) * (P + 1);
    irregular_walk_t<P + 1>(x, y, z, rc, [&](int a, int b, float jre, float jim) {
        if (a <= P) {
            const cf Mc = hat(Ms, a, b);
            phi += (b == 0 ? 1.f : 2.f) * (Mc.re * jre - Mc.im * jim);
        }
        if (a >= 1) {
            const int n = a - 1;
            if (b <= n) {
                const float H0 = h[n * n + n + b] + (b > 0 ? h[n * n + n - b] : 0.f);
                const cf Mn = hat(Ms, n, b);
                l10 += H0 * (Mn.re * jre - Mn.im * jim);
            }
            if (b + 1 <= n) {
                const float h1 = h[K + n * n + n + b + 1];
                const cf M1 = hat(Ms, n, b + 1);
                l1re += h1 * (M1.re * jre - M1.im * jim);
                l1im += h1 * (M1.re * jim + M1.im * jre);
            }
            if (b >= 1 && b - 1 <= n) {
                const float h2 = h[K + n * n + n + 1 - b];
                const cf M2 = hat(Ms, n, 1 - b);
                l1re += h2 * (M2.re * jre + M2.im * jim);
                l1im += h2 * (M2.im * jre - M2.re * jim);
            }
        }
    });
}

// Expansion families, each giving the per-particle pieces of the kernels
// below at x-hat = (x - c)/r: a P2M row (q times the coefficients of one
// particle, scaled), and L2P / M2P as (phi, E) of the scaled expansion:
// the particle's potential is .x / r and its field (.y, .z, .w) / r^2.
struct Sph {
    template <int P>
    static constexpr int K = (P + 1) * (P + 1);
    template <int P>
    __device__ static void p2m_row(float x, float y, float z, float qc, float* row, const float* __restrict__ rc) {
        regular_walk_t<P>(x, y, z, rc, [&](int n, int m, float re, float im) {
            if (m == 0) {
                row[n * n] = qc * re;
            } else {
                row[n * n + 2 * m - 1] = qc * re;
                row[n * n + 2 * m] = -qc * im;
            }
        });
    }
    template <int P>
    __device__ static float4 l2p(const float* Lt, float x, float y, float z, const float* __restrict__ g,
                                 const float* __restrict__ rc) {
        const float s2 = 1.41421356237309505f;
        float phi = 0.f, l10 = 0.f, l1re = 0.f, l1im = 0.f;
        l2p_point<P>(Lt, g, x, y, z, rc, phi, l10, l1re, l1im);
        return make_float4(phi, -s2 * l1re, s2 * l1im, -l10);
    }
    template <int P>
    __device__ static float4 m2p(const float* Ms, float x, float y, float z, const float* __restrict__ h,
                                 const float* __restrict__ rc) {
        const float s2 = 1.41421356237309505f;
        float phi = 0.f, l10 = 0.f, l1re = 0.f, l1im = 0.f;
        m2p_point<P>(Ms, h, x, y, z, rc, phi, l10, l1re, l1im);
        return make_float4(phi, -s2 * l1re, s2 * l1im, -l10);
    }
};

// Cartesian: M~_k = sum q (-x-hat)^k, phi-hat = sum_m L~_m x-hat^m for a local,
// sum_k a_k(x-hat) M~_k for a multipole (cart.h); E = -grad phi
struct Cart {
    template <int P>
    static constexpr int K = cart::count(P);
    template <int P>
    __device__ static void p2m_row(float x, float y, float z, float qc, float* row, const float* __restrict__) {
        float px[P + 1], py[P + 1], pz[P + 1];
        cart::powers<P>(-x, px);
        cart::powers<P>(-y, py);
        cart::powers<P>(-z, pz);
#pragma unroll
        for (int n = 0; n <= P; n++)
#pragma unroll
            for (int a = n; a >= 0; a--)
#pragma unroll
                for (int b = n - a; b >= 0; b--) row[cart::index(a, b, n - a - b)] = qc * (px[a] * py[b] * pz[n - a - b]);
    }
    template <int P>
    __device__ static float4 l2p(const float* Lt, float x, float y, float z, const float* __restrict__,
                                 const float* __restrict__) {
        float px[P + 1], py[P + 1], pz[P + 1];
        cart::powers<P>(x, px);
        cart::powers<P>(y, py);
        cart::powers<P>(z, pz);
        float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
        for (int n = 0; n <= P; n++)
#pragma unroll
            for (int a = n; a >= 0; a--)
#pragma unroll
                for (int b = n - a; b >= 0; b--) {
                    const int c = n - a - b;
                    const float L = Lt[cart::index(a, b, c)];
                    phi += L * (px[a] * py[b] * pz[c]);
                    if (a > 0) gx += (float)a * L * (px[a - 1] * py[b] * pz[c]);
                    if (b > 0) gy += (float)b * L * (px[a] * py[b - 1] * pz[c]);
                    if (c > 0) gz += (float)c * L * (px[a] * py[b] * pz[c - 1]);
                }
        return make_float4(phi, -gx, -gy, -gz);
    }
    template <int P>
    __device__ static float4 m2p(const float* Ms, float x, float y, float z, const float* __restrict__,
                                 const float* __restrict__) {
        float a[cart::count(P + 1)];
        cart::taylor<P + 1, float>(x, y, z, a);
        float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
        for (int n = 0; n <= P; n++)
#pragma unroll
            for (int i = n; i >= 0; i--)
#pragma unroll
                for (int j = n - i; j >= 0; j--) {
                    const int k = n - i - j;
                    const float M = Ms[cart::index(i, j, k)];
                    phi += a[cart::index(i, j, k)] * M;
                    gx += (float)(i + 1) * a[cart::index(i + 1, j, k)] * M;
                    gy += (float)(j + 1) * a[cart::index(i, j + 1, k)] * M;
                    gz += (float)(k + 1) * a[cart::index(i, j, k + 1)] * M;
                }
        return make_float4(phi, -gx, -gy, -gz);
    }
};

// Leaves [w LPW, w LPW + LPW) of the leaf list per 64-lane workgroup, their
// particles flattened (leaf by leaf, in particle order) and taken 64 at a
// time: leaves hold ~20 particles on average, so one leaf per wave would
// leave two lanes in three idle.  Each leaf's work stays a function of its
// own particles only (a forest gives the same per-leaf results as a single
// instance).
template <int LPW>
struct LeafPack {
    int32_t cell[LPW], beg[LPW], cnt[LPW], pre[LPW + 1];
    double4 ctr[LPW];
    int nq;
    // cooperative: lanes 0 .. LPW-1 each load one leaf, then (after a
    // barrier) lane 0 forms the prefix
    __device__ void load_lane(CellArrays c, const int32_t* __restrict__ leaves, int32_t nleaves, int lane) {
        const int32_t l = (int32_t)blockIdx.x * LPW + lane;
        if (l < nleaves) {
            const int32_t cl = leaves[l];
            cell[lane] = cl;
            beg[lane] = c.begin[cl];
            cnt[lane] = c.end[cl] - beg[lane];
            ctr[lane] = c.ctr[cl];
        } else {
            cell[lane] = -1;
            beg[lane] = 0;
            cnt[lane] = 0;
        }
    }
    __device__ void finish(int32_t nleaves) {
        nq = min(LPW, nleaves - (int32_t)blockIdx.x * LPW);
        int acc = 0;
        for (int q = 0; q < LPW; q++) {
            pre[q] = acc;
            acc += cnt[q];
        }
        pre[LPW] = acc;
    }
    // leaf (0 .. nq-1) of flattened position f < pre[LPW]
    __device__ int leaf_of(int f) const {
        int q = 0;
        while (q + 1 < nq && pre[q + 1] <= f) q++;
        return q;
    }
};

// P2M: each lane writes q * conj(S(x-c)/r) of one particle into its LDS row,
// then each leaf's rows are summed column by column in particle order,
// continuing across rounds (one sequential sum per coefficient and leaf).
template <int P, int LPW, class X>
__global__ __launch_bounds__(64) void k_p2m(const float4* __restrict__ pts, CellArrays c,
                                            const int32_t* __restrict__ leaves, int32_t nleaves, int KP,
                                            const float* __restrict__ rc, float* __restrict__ M) {
    constexpr int K = X::template K<P>;
    constexpr int CH = K <= 128 ? 64 : 32;  // rows per round
    constexpr int STR = K | 1;
    constexpr int NU = (K + 63) / 64;
    __shared__ float rows[CH * STR];
    __shared__ LeafPack<LPW> lp;
    const int lane = threadIdx.x;
    if (lane < LPW) lp.load_lane(c, leaves, nleaves, lane);
    __syncthreads();
    if (lane == 0) lp.finish(nleaves);
    __syncthreads();
    const int total = lp.pre[LPW];
    float acc[LPW][NU];
#pragma unroll
    for (int q = 0; q < LPW; q++)
#pragma unroll
        for (int u = 0; u < NU; u++) acc[q][u] = 0.f;
    for (int r0 = 0; r0 < total; r0 += CH) {
        const int nr = min(CH, total - r0);
        if (lane < nr) {
            const int f = r0 + lane;
            const int q = lp.leaf_of(f);
            const float4 Pt = pts[lp.beg[q] + (f - lp.pre[q])];
            const double4 ct = lp.ctr[q];
            const double ir = 1.0 / ct.w;
            const float x = (float)(((double)Pt.x - ct.x) * ir), y = (float)(((double)Pt.y - ct.y) * ir),
                        z = (float)(((double)Pt.z - ct.z) * ir);
            const float qc = Pt.w;
            float* row = rows + lane * STR;
            X::template p2m_row<P>(x, y, z, qc, row, rc);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < LPW; q++) {
            const int lo = max(lp.pre[q], r0) - r0, hi = min(lp.pre[q + 1], r0 + nr) - r0;
#pragma unroll
            for (int u = 0; u < NU; u++) {
                const int j = lane + 64 * u;
                if (j < K)
                    for (int r = lo; r < hi; r++) acc[q][u] += rows[r * STR + j];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < LPW; q++) {
        if (q >= lp.nq) break;
        for (int u = 0; 64 * u < KP; u++) {
            const int j = lane + 64 * u;
            float v = 0.f;
#pragma unroll
            for (int uu = 0; uu < NU; uu++)
                if (uu == u) v = acc[q][uu];
            if (j < KP) M[(size_t)lp.cell[q] * KP + j] = j < K ? v : 0.f;
        }
    }
}

// 1 where the leaf or one of its ancestors has cell-particle (M2P) sources
__global__ void k_m2p_flags(CellArrays c, const int32_t* __restrict__ leaves, int32_t nleaves,
                            const int32_t* __restrict__ m2p_off, uint8_t* __restrict__ flag) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= nleaves) return;
    uint8_t f = 0;
    for (int A = leaves[i]; A >= 0 && !f; A = c.parent[A]) f = m2p_off[A + 1] > m2p_off[A];
    flag[i] = f;
}

// Far field and final sum for every particle: near part (FP64) + L2P of its
// leaf's local + M2P of the sources paired with its leaf or an ancestor (in
// that order, as one sequential FP64 sum), written in the caller's order.
template <int P, int LPW, class X>
__global__ __launch_bounds__(64) void k_far(const float4* __restrict__ pts, const uint32_t* __restrict__ perm,
                                            CellArrays c, const int32_t* __restrict__ leaves, int32_t nleaves,
                                            const uint8_t* __restrict__ m2pflag,
                                            const int32_t* __restrict__ m2p_off, const uint32_t* __restrict__ m2p_src,
                                            int KP, const float* __restrict__ gl2p, const float* __restrict__ hm2p,
                                            const float* __restrict__ rc, const float* __restrict__ M,
                                            const float* __restrict__ L, double4* __restrict__ near,
                                            int out_dtype, void* __restrict__ ophi, void* __restrict__ oex,
                                            void* __restrict__ oey, void* __restrict__ oez) {
    constexpr int K = X::template K<P>;
    __shared__ float Lt[LPW][K];
    __shared__ LeafPack<LPW> lp;
    __shared__ uint8_t s_m2p[LPW];
    const int lane = threadIdx.x;
    if (lane < LPW) {
        lp.load_lane(c, leaves, nleaves, lane);
        const int32_t l = (int32_t)blockIdx.x * LPW + lane;
        s_m2p[lane] = l < nleaves ? m2pflag[l] : 0;
    }
    __syncthreads();
    if (lane == 0) lp.finish(nleaves);
    __syncthreads();
    for (int i = lane; i < LPW * K; i += 64) {
        const int q = i / K, k = i - q * K;
        Lt[q][k] = q < lp.nq ? L[(size_t)lp.cell[q] * KP + k] : 0.f;
    }
    __syncthreads();
    const int total = lp.pre[LPW];
    for (int r0 = 0; r0 < total; r0 += 64) {
        const int f = r0 + lane;
        const bool valid = f < total;
        const int q = valid ? lp.leaf_of(f) : 0;
        const int32_t i = lp.beg[q] + (f - lp.pre[q]);
        const float4 Pt = pts[valid ? i : lp.beg[0]];
        double4 acc = valid ? near[i] : make_double4(0, 0, 0, 0);
        {
            const double4 ct = lp.ctr[q];
            const double ir = 1.0 / ct.w;
            const float x = (float)(((double)Pt.x - ct.x) * ir), y = (float)(((double)Pt.y - ct.y) * ir),
                        z = (float)(((double)Pt.z - ct.z) * ir);
            const float4 v = X::template l2p<P>(Lt[q], x, y, z, gl2p, rc);
            const double r1 = ct.w, r2 = ct.w * ct.w;
            acc.x += (double)v.x / r1;
            acc.y += (double)v.y / r2;
            acc.z += (double)v.z / r2;
            acc.w += (double)v.w / r2;
        }
        if (valid && s_m2p[q]) {
            near[i] = acc;  // cell-particle sources follow (k_far_m2p)
        } else if (valid) {
            const uint32_t o = perm[i];
            if (out_dtype == 1) {
                ((double*)ophi)[o] = acc.x;
                ((double*)oex)[o] = acc.y;
                ((double*)oey)[o] = acc.z;
                ((double*)oez)[o] = acc.w;
            } else {
                ((float*)ophi)[o] = (float)acc.x;
                ((float*)oex)[o] = (float)acc.y;
                ((float*)oey)[o] = (float)acc.z;
                ((float*)oez)[o] = (float)acc.w;
            }
        }
    }
}

// Cell-particle (M2P) part of the leaves flagged in m2pflag.  LPW
// consecutive leaves of the leaf list share a 64-lane workgroup (unflagged
// ones take no lanes); their particles are flattened and taken 64 at a time.
// Each particle continues the FP64 sum k_far stored in near[i] with the
// sources of its leaf's list, then of its parent's, and so on to the root,
// each list in order.  The packed leaves mostly share their ancestors, so
// the lists are walked level by level: at chain depth k the distinct k-th
// ancestors of the packed leaves are the list owners, and step t stages the
// t-th source of every owner once in LDS for all the lanes under it.
template <int P, int LPW, class X>
__global__ __launch_bounds__(64) void k_far_m2p(const float4* __restrict__ pts, const uint32_t* __restrict__ perm,
                                                CellArrays c, const int32_t* __restrict__ leaves, int32_t nleaves,
                                                const uint8_t* __restrict__ m2pflag,
                                                const int32_t* __restrict__ m2p_off,
                                                const uint32_t* __restrict__ m2p_src, int KP,
                                                const float* __restrict__ hm2p, const float* __restrict__ rc,
                                                const float* __restrict__ M, const double4* __restrict__ near,
                                                int out_dtype, void* __restrict__ ophi, void* __restrict__ oex,
                                                void* __restrict__ oey, void* __restrict__ oez) {
    constexpr int K = X::template K<P>;
    constexpr int MAXD = kMaxLevel + 1;  // a leaf and its ancestors
    __shared__ LeafPack<LPW> lp;
    __shared__ int32_t anc[LPW][MAXD];   // anc[q][k]: k-th ancestor of leaf q, -1 above the root
    __shared__ int32_t chain[LPW];
    __shared__ int32_t own[LPW];         // owner index of leaf q at the current depth, -1 if none
    __shared__ int32_t dcell[LPW], dlen[LPW], doff[LPW];
    __shared__ int32_t s_nd, s_steps, s_depth;
    __shared__ int32_t aoff[LPW][MAXD], alen[LPW][MAXD];  // list of anc[q][k]: offset, length (0 if none)
    __shared__ uint32_t s_dmask;                          // depths where some packed leaf's ancestor has a list
    __shared__ float Ms[LPW][K];
    __shared__ double4 sctr[LPW];
    const int lane = threadIdx.x;
    if (lane == 0) s_dmask = 0u;
    if (lane < LPW) {
        const int32_t l = (int32_t)blockIdx.x * LPW + lane;
        const bool flagged = l < nleaves && m2pflag[l];
        lp.load_lane(c, leaves, nleaves, lane);
        if (!flagged) lp.cnt[lane] = 0;  // its particles are final already
        int d = 0;
        if (flagged)
            for (int A = lp.cell[lane]; A >= 0 && d < MAXD; A = c.parent[A]) anc[lane][d++] = A;
        chain[lane] = d;
        for (int k = d; k < MAXD; k++) anc[lane][k] = -1;
    }
    __syncthreads();
    // every (leaf, depth) list bound at once, lane-parallel
    for (int u = lane; u < LPW * MAXD; u += 64) {
        const int q = u / MAXD, k = u - q * MAXD;
        const int32_t A = anc[q][k];
        int32_t o = 0, len = 0;
        if (A >= 0) {
            o = m2p_off[A];
            len = m2p_off[A + 1] - o;
        }
        aoff[q][k] = o;
        alen[q][k] = len;
        if (len > 0) atomicOr(&s_dmask, 1u << k);
    }
    __syncthreads();
    if (lane == 0) {
        lp.finish(nleaves);
        int dm = 0;
        for (int q = 0; q < LPW; q++) dm = max(dm, chain[q]);
        s_depth = dm;
    }
    __syncthreads();
    const int total = lp.pre[LPW];
    if (total == 0) return;
    for (int r0 = 0; r0 < total; r0 += 64) {
        const int f = r0 + lane;
        const bool valid = f < total;
        const int q = valid ? lp.leaf_of(f) : 0;
        const int32_t i = lp.beg[q] + (f - lp.pre[q]);
        const float4 Pt = pts[valid ? i : lp.beg[q]];
        double4 acc = valid ? near[i] : make_double4(0, 0, 0, 0);
        for (int k = 0; k < s_depth; k++) {
            if (!((s_dmask >> k) & 1u)) continue;  // no list at this depth (uniform)
            if (lane == 0) {
                // leaves with particles in this round, in leaf order; equal
                // owners are adjacent (leaves follow the tree order)
                int nd = 0, steps = 0;
                for (int qq = 0; qq < LPW; qq++) {
                    own[qq] = -1;
                    const bool in_round = lp.cnt[qq] > 0 && lp.pre[qq] < r0 + 64 && lp.pre[qq + 1] > r0;
                    const int32_t A = in_round ? anc[qq][k] : -1;
                    if (A < 0) continue;
                    const int32_t len = alen[qq][k];
                    if (len == 0) continue;
                    if (nd == 0 || dcell[nd - 1] != A) {
                        dcell[nd] = A;
                        dlen[nd] = len;
                        doff[nd] = aoff[qq][k];
                        steps = max(steps, len);
                        nd++;
                    }
                    own[qq] = nd - 1;
                }
                s_nd = nd;
                s_steps = steps;
            }
            __syncthreads();
            const int nd = s_nd, steps = s_steps;
            const int o = valid ? own[q] : -1;
            for (int t = 0; t < steps; t++) {
                for (int u = lane; u < nd * K; u += 64) {
                    const int d = u / K, kk = u - d * K;
                    if (t < dlen[d]) {
                        const int s = (int)m2p_src[doff[d] + t];
                        Ms[d][kk] = M[(size_t)s * KP + kk];
                        if (kk == 0) sctr[d] = c.ctr[s];
                    }
                }
                __syncthreads();
                if (o >= 0 && t < dlen[o]) {
                    const double4 cs = sctr[o];
                    const double ir = 1.0 / cs.w;
                    const float x = (float)(((double)Pt.x - cs.x) * ir), y = (float)(((double)Pt.y - cs.y) * ir),
                                z = (float)(((double)Pt.z - cs.z) * ir);
                    const float4 v = X::template m2p<P>(Ms[o], x, y, z, hm2p, rc);
                    const double r1 = cs.w, r2 = cs.w * cs.w;
                    acc.x += (double)v.x / r1;
                    acc.y += (double)v.y / r2;
                    acc.z += (double)v.z / r2;
                    acc.w += (double)v.w / r2;
                }
                __syncthreads();
            }
            __syncthreads();  // own[] and the owner tables are rewritten for the next depth
        }
        if (valid) {
            const uint32_t o = perm[i];
            if (out_dtype == 1) {
                ((double*)ophi)[o] = acc.x;
                ((double*)oex)[o] = acc.y;
                ((double*)oey)[o] = acc.z;
                ((double*)oez)[o] = acc.w;
            } else {
                ((float*)ophi)[o] = (float)acc.x;
                ((float*)oex)[o] = (float)acc.y;
                ((float*)oey)[o] = (float)acc.z;
                ((float*)oez)[o] = (float)acc.w;
            }
        }
    }
}

constexpr int kLeavesPerWave = 8;
constexpr int kM2pLeavesPerWave = 16;

template <int P, class X>
void launch_far(const float4* pts, const uint32_t* perm, CellArrays cells, const int32_t* leaves, int32_t nleaves,
                uint8_t* m2pflag, const int32_t* m2p_off, const uint32_t* m2p_src, int KP, Tables t, const float* M,
                const float* L, double4* near, int out_dtype, void* phi, void* ex, void* ey, void* ez, bool any_m2p,
                hipStream_t s) {
    k_m2p_flags<<<(nleaves + 255) / 256, 256, 0, s>>>(cells, leaves, nleaves, m2p_off, m2pflag);
    constexpr int W = kLeavesPerWave;
    k_far<P, W, X><<<(nleaves + W - 1) / W, 64, 0, s>>>(pts, perm, cells, leaves, nleaves, m2pflag, m2p_off, m2p_src,
                                                        KP, t.gl2p, t.hm2p, t.rcoef, M, L, near, out_dtype, phi, ex,
                                                        ey, ez);
    if (any_m2p) {
        constexpr int W2 = kM2pLeavesPerWave;
        k_far_m2p<P, W2, X><<<(nleaves + W2 - 1) / W2, 64, 0, s>>>(pts, perm, cells, leaves, nleaves, m2pflag,
                                                                  m2p_off, m2p_src, KP, t.hm2p, t.rcoef, M, near,
                                                                  out_dtype, phi, ex, ey, ez);
    }
}

template <int P, class X>
void launch_p2m(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves, int KP, const float* rc,
                float* M, hipStream_t s) {
    constexpr int W = kLeavesPerWave;
    k_p2m<P, W, X><<<(nleaves + W - 1) / W, 64, 0, s>>>(pts, cells, leaves, nleaves, KP, rc, M);
}

}  // namespace

void far_final(const float4* pts, const uint32_t* perm, CellArrays cells, const int32_t* leaves, int32_t nleaves,
               uint8_t* m2pflag, const int32_t* m2p_off, const uint32_t* m2p_src, int64_t n_m2p, int family, int p,
               int KP, Tables t, const float* M, const float* L, double4* near, int out_dtype, void* phi, void* ex,
               void* ey, void* ez, hipStream_t s) {
    if (nleaves <= 0) return;
#define FMM_FAR_CASE(PP, XX)                                                                                      \
    case PP:                                                                                                      \
        launch_far<PP, XX>(pts, perm, cells, leaves, nleaves, m2pflag, m2p_off, m2p_src, KP, t, M, L, near,       \
                           out_dtype, phi, ex, ey, ez, n_m2p > 0, s);                                            \
        break;
    if (family == kFamilyCartesian) {
        switch (p) {
            FMM_FAR_CASE(0, Cart)
            FMM_FAR_CASE(1, Cart)
            FMM_FAR_CASE(2, Cart)
            FMM_FAR_CASE(3, Cart)
            FMM_FAR_CASE(4, Cart)
            FMM_FAR_CASE(5, Cart)
            FMM_FAR_CASE(6, Cart)
            default:
                break;
        }
        return;
    }
    switch (p) {
        FMM_FAR_CASE(0, Sph)
        FMM_FAR_CASE(1, Sph)
        FMM_FAR_CASE(2, Sph)
        FMM_FAR_CASE(3, Sph)
        FMM_FAR_CASE(4, Sph)
        FMM_FAR_CASE(5, Sph)
        FMM_FAR_CASE(6, Sph)
        FMM_FAR_CASE(7, Sph)
        FMM_FAR_CASE(8, Sph)
        FMM_FAR_CASE(9, Sph)
        FMM_FAR_CASE(10, Sph)
        FMM_FAR_CASE(11, Sph)
        FMM_FAR_CASE(12, Sph)
        FMM_FAR_CASE(13, Sph)
        FMM_FAR_CASE(14, Sph)
        FMM_FAR_CASE(15, Sph)
        FMM_FAR_CASE(16, Sph)
        default:
            break;
    }
#undef FMM_FAR_CASE
}

void p2m(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves, int family, int p, int KP,
         const float* rc, float* M, hipStream_t s) {
    if (nleaves <= 0) return;
#define FMM_P2M_CASE(PP, XX)                                              \
    case PP:                                                              \
        launch_p2m<PP, XX>(pts, cells, leaves, nleaves, KP, rc, M, s);    \
        break;
    if (family == kFamilyCartesian) {
        switch (p) {
            FMM_P2M_CASE(0, Cart)
            FMM_P2M_CASE(1, Cart)
            FMM_P2M_CASE(2, Cart)
            FMM_P2M_CASE(3, Cart)
            FMM_P2M_CASE(4, Cart)
            FMM_P2M_CASE(5, Cart)
            FMM_P2M_CASE(6, Cart)
            default:
                break;
        }
        return;
    }
    switch (p) {
        FMM_P2M_CASE(0, Sph)
        FMM_P2M_CASE(1, Sph)
        FMM_P2M_CASE(2, Sph)
        FMM_P2M_CASE(3, Sph)
        FMM_P2M_CASE(4, Sph)
        FMM_P2M_CASE(5, Sph)
        FMM_P2M_CASE(6, Sph)
        FMM_P2M_CASE(7, Sph)
        FMM_P2M_CASE(8, Sph)
        FMM_P2M_CASE(9, Sph)
        FMM_P2M_CASE(10, Sph)
        FMM_P2M_CASE(11, Sph)
        FMM_P2M_CASE(12, Sph)
        FMM_P2M_CASE(13, Sph)
        FMM_P2M_CASE(14, Sph)
        FMM_P2M_CASE(15, Sph)
        FMM_P2M_CASE(16, Sph)
        default:
            break;
    }
#undef FMM_P2M_CASE
}

}  // namespace fmm
