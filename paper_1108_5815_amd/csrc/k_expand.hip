// k_expand.hip -- P2M, M2M, L2L, the general M2L and the far-field
// evaluation (L2P + M2P + final sum) of the spherical-harmonic expansions.
//
// Expansions (paper: "Hybrid treecode/FMM algorithm" and "Results": all
// methods use spherical harmonics) follow Greengard & Rokhlin, Acta Numerica
// 1997, theorems 3.2-3.5, in radius-scaled form: a multipole of a cell of
// half side r is stored divided by r^n, a local multiplied by r^(n+1), so the
// octant M2M/L2L operators are level independent.  Harmonics come from
// Cartesian recurrences in FP32 on coordinates relative to the cell centre,
// formed in FP64 and divided by r (no trigonometry, no pole division).
// Gradients: the local (or multipole) expansion is re-centred at the target
// point, where the potential is the degree-0 term and the gradient the
// degree-1 terms; both are folded into precomputed weight tables.
#include "fmm_internal.h"
#include "host_ops.h"

namespace fmm {
namespace {

struct cf {
    float re, im;
};
__device__ inline cf cmul(cf a, cf b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

__device__ inline int idx_re(int n, int m) { return m == 0 ? n * n : n * n + 2 * m - 1; }

// coefficient (n, m), any sign of m, from a real-layout row (conj for m < 0)
__device__ inline cf hat(const float* row, int n, int m) {
    if (m == 0) return {row[n * n], 0.f};
    if (m > 0) return {row[n * n + 2 * m - 1], row[n * n + 2 * m]};
    return {row[n * n - 2 * m - 1], -row[n * n - 2 * m]};
}

// Regular solid harmonics S_n^m = rho^n Y_n^m (m >= 0, n <= P) of (x,y,z),
// each handed to f(n, m, re, im) as soon as it is formed.
template <class Fn>
__device__ inline void regular_walk(int P, float x, float y, float z, const float* __restrict__ rc, Fn f) {
    float r2 = x * x + y * y + z * z;
    float mre = 1.f, mim = 0.f;
    for (int m = 0; m <= P; m++) {
        if (m > 0) {
            float c = rc[kRcC1 + m];
            float nre = c * (x * mre - y * mim), nim = c * (x * mim + y * mre);
            mre = nre;
            mim = nim;
        }
        f(m, m, mre, mim);
        if (m == P) break;
        float c2 = rc[kRcC2 + m] * z;
        float p1re = c2 * mre, p1im = c2 * mim, p0re = mre, p0im = mim;
        f(m + 1, m, p1re, p1im);
        for (int n = m + 2; n <= P; n++) {
            int t = n * (n + 1) / 2 + m;
            float A = rc[kRcA + t] * z, B = rc[kRcB + t] * r2;
            float nre = A * p1re - B * p0re, nim = A * p1im - B * p0im;
            f(n, m, nre, nim);
            p0re = p1re;
            p0im = p1im;
            p1re = nre;
            p1im = nim;
        }
    }
}

// Irregular solid harmonics J_n^m = Y_n^m / rho^(n+1) (m >= 0, n <= P).
template <class Fn>
__device__ inline void irregular_walk(int P, float x, float y, float z, const float* __restrict__ rc, Fn f) {
    float r2 = x * x + y * y + z * z;
    float ir2 = 1.f / r2;
    float mre = sqrtf(ir2), mim = 0.f;
    for (int m = 0; m <= P; m++) {
        if (m > 0) {
            float c = rc[kRcC1 + m] * ir2;
            float nre = c * (x * mre - y * mim), nim = c * (x * mim + y * mre);
            mre = nre;
            mim = nim;
        }
        f(m, m, mre, mim);
        if (m == P) break;
        float c2 = rc[kRcC2 + m] * z * ir2;
        float p1re = c2 * mre, p1im = c2 * mim, p0re = mre, p0im = mim;
        f(m + 1, m, p1re, p1im);
        for (int n = m + 2; n <= P; n++) {
            int t = n * (n + 1) / 2 + m;
            float A = rc[kRcA + t] * z * ir2, B = rc[kRcB + t] * ir2;
            float nre = A * p1re - B * p0re, nim = A * p1im - B * p0im;
            f(n, m, nre, nim);
            p0re = p1re;
            p0im = p1im;
            p1re = nre;
            p1im = nim;
        }
    }
}

__device__ inline int degree_of(int j) {
    int d = (int)sqrtf((float)j);
    while ((d + 1) * (d + 1) <= j) d++;
    while (d * d > j) d--;
    return d;
}

// ---------------------------------------------------------------- P2M
// One workgroup of 64 lanes per leaf: each lane writes q * conj(S(x-c)/r) of
// one particle into its LDS row, then lanes sum columns (fixed order) over
// the rows that hold a particle.
__global__ __launch_bounds__(64) void k_p2m(const float4* __restrict__ pts, CellArrays c,
                                            const int32_t* __restrict__ leaves, int p, int KP,
                                            const float* __restrict__ rc, float* __restrict__ M) {
    extern __shared__ float sh[];
    const int K = (p + 1) * (p + 1);
    const int STR = K | 1;
    const int CH = K <= 128 ? 64 : 32;
    const int cell = leaves[blockIdx.x];
    const int32_t b = c.begin[cell], e = c.end[cell];
    const double4 ct = c.ctr[cell];
    const double ir = 1.0 / ct.w;
    float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    float* row = sh + (threadIdx.x < CH ? threadIdx.x : 0) * STR;
    for (int32_t ch = b; ch < e; ch += CH) {
        const int nr = min(CH, e - ch);
        if ((int)threadIdx.x < nr) {
            float4 P = pts[ch + threadIdx.x];
            float x = (float)(((double)P.x - ct.x) * ir);
            float y = (float)(((double)P.y - ct.y) * ir);
            float z = (float)(((double)P.z - ct.z) * ir);
            float q = P.w;
            regular_walk(p, x, y, z, rc, [&](int n, int m, float re, float im) {
                if (m == 0) row[n * n] = q * re;
                else {
                    row[n * n + 2 * m - 1] = q * re;
                    row[n * n + 2 * m] = -q * im;
                }
            });
        }
        __syncthreads();
        for (int u = 0; u < 5; u++) {
            int j = threadIdx.x + 64 * u;
            if (j < K) {
                float s = 0.f;
                for (int r = 0; r < nr; r++) s += sh[r * STR + j];
                acc[u] += s;
            }
        }
        __syncthreads();
    }
    for (int u = 0; u < 5; u++) {
        int j = threadIdx.x + 64 * u;
        if (j < KP) M[(size_t)cell * KP + j] = j < K ? acc[u] : 0.f;
    }
}

// ---------------------------------------------------------------- M2M / L2L
__global__ __launch_bounds__(128) void k_m2m(CellArrays c, int32_t c0, int p, int KP,
                                             const float* __restrict__ mat, float* __restrict__ M) {
    extern __shared__ float sh[];
    const int cell = c0 + blockIdx.x;
    const int nch = c.nchild[cell];
    if (nch == 0) return;
    const int K = (p + 1) * (p + 1);
    const int first = c.child[cell];
    for (int i = threadIdx.x; i < nch * K; i += blockDim.x) {
        int ch = i / K, k = i - ch * K;
        sh[ch * KP + k] = M[(size_t)(first + ch) * KP + k];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < KP; j += blockDim.x) {
        float acc = 0.f;
        if (j < K) {
            int d = degree_of(j);
            int kmax = (d + 1) * (d + 1);
            for (int ch = 0; ch < nch; ch++) {
                int oct = (int)(c.prefix[first + ch] & 7u);
                const float* A = mat + (size_t)oct * K * K;
                const float* v = sh + ch * KP;
                for (int k = 0; k < kmax; k++) acc += A[(size_t)k * K + j] * v[k];
            }
        }
        M[(size_t)cell * KP + j] = acc;
    }
}

__global__ __launch_bounds__(128) void k_l2l(CellArrays c, int32_t c0, int p, int KP,
                                             const float* __restrict__ mat, float* __restrict__ L) {
    extern __shared__ float sh[];
    const int cell = c0 + blockIdx.x;
    const int par = c.parent[cell];
    const int K = (p + 1) * (p + 1);
    for (int k = threadIdx.x; k < K; k += blockDim.x) sh[k] = L[(size_t)par * KP + k];
    __syncthreads();
    const int oct = (int)(c.prefix[cell] & 7u);
    const float* A = mat + (size_t)oct * K * K;
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        int d = degree_of(j);
        float acc = 0.f;
        for (int k = d * d; k < K; k++) acc += A[(size_t)k * K + j] * sh[k];
        L[(size_t)cell * KP + j] += acc;
    }
}

// ---------------------------------------------------------------- general M2L
// Pairs not handled by the batched GEMM (mixed levels, offsets outside the
// per-class tables), one workgroup per target cell.  Each of the 4 waves
// takes every 4th pair of the target: its lanes build the irregular harmonics
// of the offset (in units of the target half side) up to degree 2p in the
// wave's LDS area, one column m per lane, then every lane sums
// W(j,k,n,m) (rs/rt)^n O(n,m) J(j+n, m-k) over (n, m) for its outputs (j, k).
// The four partial sums are added in wave order: deterministic, no atomics.
__global__ __launch_bounds__(256) void k_m2l_general(const int32_t* __restrict__ goff,
                                                     const uint32_t* __restrict__ gsrc, CellArrays c, int p,
                                                     int KP, const float* __restrict__ W, int w_lds,
                                                     const float* __restrict__ rc, const float* __restrict__ M,
                                                     float* __restrict__ L, const uint8_t* __restrict__ skip) {
    extern __shared__ float sh[];
    const int t = blockIdx.x;
    const int32_t a0 = goff[t], a1 = goff[t + 1];
    if (a0 == a1) return;
    const int K = (p + 1) * (p + 1);
    const int P2 = 2 * p;
    const int TRI = (P2 + 1) * (P2 + 2) / 2;
    const int njk = (p + 1) * (p + 2) / 2;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* Wl = sh;
    float* base = sh + (w_lds ? njk * K : 0);
    float* Ms = base + w * (KP + 2 * TRI);
    float* Jh = Ms + KP;
    float* red = base + 4 * (KP + 2 * TRI);
    if (w_lds)
        for (int i = threadIdx.x; i < njk * K; i += 256) Wl[i] = W[i];
    __syncthreads();
    const float* Wp = w_lds ? Wl : W;
    int oj[3], ok[3];
    float are[3] = {0.f, 0.f, 0.f}, aim[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 3; u++) {
        int jk = lane + 64 * u, j = 0;
        if (jk < njk) {
            while ((j + 1) * (j + 2) / 2 <= jk) j++;
            oj[u] = j;
            ok[u] = jk - j * (j + 1) / 2;
        } else {
            oj[u] = -1;
            ok[u] = 0;
        }
    }
    const int4 gt = c.geo[t];
    const float inv = 1.f / (float)gt.w;
    for (int32_t a = a0 + w; a < a1; a += 4) {
        if (skip && skip[a]) continue;  // handled by the class-batched products
        const int s = (int)gsrc[a];
        const int4 gs = c.geo[s];
        const float qx = (float)(gs.x - gt.x) * inv, qy = (float)(gs.y - gt.y) * inv,
                    qz = (float)(gs.z - gt.z) * inv;
        const float ratio = (float)gs.w * inv;
        for (int i = lane; i < K; i += 64) Ms[i] = M[(size_t)s * KP + i];
        for (int m = lane; m <= P2; m += 64) {
            const float r2 = qx * qx + qy * qy + qz * qz, ir2 = 1.f / r2;
            float mre = sqrtf(ir2), mim = 0.f;
            for (int mm = 1; mm <= m; mm++) {
                const float cc = rc[kRcC1 + mm] * ir2;
                const float nre = cc * (qx * mre - qy * mim), nim = cc * (qx * mim + qy * mre);
                mre = nre;
                mim = nim;
            }
            int tt = m * (m + 1) / 2 + m;
            Jh[2 * tt] = mre;
            Jh[2 * tt + 1] = mim;
            if (m < P2) {
                const float c2 = rc[kRcC2 + m] * qz * ir2;
                float p1re = c2 * mre, p1im = c2 * mim, p0re = mre, p0im = mim;
                tt = (m + 1) * (m + 2) / 2 + m;
                Jh[2 * tt] = p1re;
                Jh[2 * tt + 1] = p1im;
                for (int n = m + 2; n <= P2; n++) {
                    const int uu = n * (n + 1) / 2 + m;
                    const float A = rc[kRcA + uu] * qz * ir2, B = rc[kRcB + uu] * ir2;
                    const float nre = A * p1re - B * p0re, nim = A * p1im - B * p0im;
                    Jh[2 * uu] = nre;
                    Jh[2 * uu + 1] = nim;
                    p0re = p1re;
                    p0im = p1im;
                    p1re = nre;
                    p1im = nim;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int u = 0; u < 3; u++) {
            if (oj[u] < 0) continue;
            const int j = oj[u], k = ok[u];
            const float* wr = Wp + (size_t)(j * (j + 1) / 2 + k) * K;
            float rn = 1.f, tre = 0.f, tim = 0.f;
            for (int n = 0; n <= p; n++) {
                float sre = 0.f, sim = 0.f;
                for (int m = -n; m <= n; m++) {
                    const cf O = hat(Ms, n, m);
                    const int q = j + n, mk = m - k;
                    const int uu = q * (q + 1) / 2 + (mk < 0 ? -mk : mk);
                    const float jre = Jh[2 * uu], jim = mk < 0 ? -Jh[2 * uu + 1] : Jh[2 * uu + 1];
                    const float ww = wr[n * n + n + m];
                    sre += ww * (O.re * jre - O.im * jim);
                    sim += ww * (O.re * jim + O.im * jre);
                }
                tre += rn * sre;
                tim += rn * sim;
                rn *= ratio;
            }
            are[u] += tre;
            aim[u] += tim;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int u = 0; u < 3; u++) {
        if (oj[u] < 0) continue;
        const int jk = lane + 64 * u;
        red[(w * njk + jk) * 2] = are[u];
        red[(w * njk + jk) * 2 + 1] = aim[u];
    }
    __syncthreads();
    for (int jk = threadIdx.x; jk < njk; jk += 256) {
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= jk) j++;
        const int k = jk - j * (j + 1) / 2;
        float sre = 0.f, sim = 0.f;
        for (int ww = 0; ww < 4; ww++) {
            sre += red[(ww * njk + jk) * 2];
            sim += red[(ww * njk + jk) * 2 + 1];
        }
        const int ix = idx_re(j, k);
        L[(size_t)t * KP + ix] += sre;
        if (k > 0) L[(size_t)t * KP + ix + 1] += sim;
    }
}

}  // namespace

void p2m(const float4* pts, CellArrays cells, const int32_t* leaves, int32_t nleaves, int p, int KP,
         const float* rc, float* M, hipStream_t s) {
    if (nleaves <= 0) return;
    int K = (p + 1) * (p + 1);
    size_t lds = (size_t)(K <= 128 ? 64 : 32) * (K | 1) * sizeof(float);
    k_p2m<<<nleaves, 64, lds, s>>>(pts, cells, leaves, p, KP, rc, M);
}

void m2m(CellArrays cells, int32_t c0, int32_t c1, int p, int KP, Tables t, float* M, hipStream_t s) {
    if (c1 <= c0) return;
    k_m2m<<<c1 - c0, 128, (size_t)8 * KP * sizeof(float), s>>>(cells, c0, p, KP, t.m2m, M);
}

void l2l(CellArrays cells, int32_t c0, int32_t c1, int p, int KP, Tables t, float* L, hipStream_t s) {
    if (c1 <= c0) return;
    k_l2l<<<c1 - c0, 128, (size_t)KP * sizeof(float), s>>>(cells, c0, p, KP, t.l2l, L);
}

void m2l_general(const int32_t* goff, const uint32_t* gsrc, CellArrays cells, int32_t ncell, int p, int KP,
                 Tables t, const float* M, float* L, const uint8_t* skip, hipStream_t s) {
    if (ncell <= 0) return;
    const int P2 = 2 * p;
    const int njk = (p + 1) * (p + 2) / 2, K = (p + 1) * (p + 1);
    const size_t per = 4 * ((size_t)KP + (size_t)(P2 + 1) * (P2 + 2)) + 8 * (size_t)njk;
    const int w_lds = ((size_t)njk * K + per) * sizeof(float) <= 65536 ? 1 : 0;
    const size_t lds = ((w_lds ? (size_t)njk * K : 0) + per) * sizeof(float);
    k_m2l_general<<<ncell, 256, lds, s>>>(goff, gsrc, cells, p, KP, t.wm2l, w_lds, t.rcoef, M, L, skip);
}

}  // namespace fmm
