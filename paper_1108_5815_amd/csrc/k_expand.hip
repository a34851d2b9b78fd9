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
// one particle into its LDS row, then lanes sum columns (fixed order).
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
        if (threadIdx.x < CH) {
            int32_t i = ch + threadIdx.x;
            if (i < e) {
                float4 P = pts[i];
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
            } else {
                for (int j = 0; j < K; j++) row[j] = 0.f;
            }
        }
        __syncthreads();
        for (int u = 0; u < 5; u++) {
            int j = threadIdx.x + 64 * u;
            if (j < K) {
                float s = 0.f;
                for (int r = 0; r < CH; r++) s += sh[r * STR + j];
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
// One workgroup per target cell; the pairs not handled by the batched GEMM
// (mixed levels, offsets outside the class tables) are converted one by one:
// irregular harmonics of the offset (in units of the target half side) up to
// degree 2p into LDS, then every output (j, k) sums
// W(j,k,n,m) (rs/rt)^n O(n,m) J(j+n, m-k) over (n, m).
__global__ __launch_bounds__(256) void k_m2l_general(const int32_t* __restrict__ off,
                                                     const uint32_t* __restrict__ src,
                                                     const uint32_t* __restrict__ general, CellArrays c,
                                                     int p, int KP, const float* __restrict__ W,
                                                     const float* __restrict__ rc, const float* __restrict__ M,
                                                     float* __restrict__ L) {
    extern __shared__ float sh[];
    const int t = blockIdx.x;
    const int32_t a0 = off[t], a1 = off[t + 1];
    bool any = false;
    for (int32_t a = a0; a < a1; a++) any |= general[a] != 0u;
    if (!any) return;
    const int K = (p + 1) * (p + 1);
    const int P2 = 2 * p;
    float* Ms = sh;                 // KP
    float* Jh = sh + KP;            // 2 * tri(P2)
    const int njk = (p + 1) * (p + 2) / 2;
    const int jk = threadIdx.x;
    int j = 0, k = 0;
    if (jk < njk) {
        while ((j + 1) * (j + 2) / 2 <= jk) j++;
        k = jk - j * (j + 1) / 2;
    }
    float are = 0.f, aim = 0.f;
    const int4 gt = c.geo[t];
    for (int32_t a = a0; a < a1; a++) {
        if (!general[a]) continue;
        const int s = (int)src[a];
        const int4 gs = c.geo[s];
        const float inv = 1.f / (float)gt.w;
        const float qx = (float)(gs.x - gt.x) * inv, qy = (float)(gs.y - gt.y) * inv,
                    qz = (float)(gs.z - gt.z) * inv;
        const float ratio = (float)gs.w * inv;
        __syncthreads();
        for (int i = threadIdx.x; i < K; i += blockDim.x) Ms[i] = M[(size_t)s * KP + i];
        // column m of the irregular table: thread m walks n = m .. P2
        for (int m = threadIdx.x; m <= P2; m += blockDim.x) {
            float r2 = qx * qx + qy * qy + qz * qz, ir2 = 1.f / r2;
            float mre = sqrtf(ir2), mim = 0.f;
            for (int mm = 1; mm <= m; mm++) {
                float cc = rc[kRcC1 + mm] * ir2;
                float nre = cc * (qx * mre - qy * mim), nim = cc * (qx * mim + qy * mre);
                mre = nre;
                mim = nim;
            }
            int tt = m * (m + 1) / 2 + m;
            Jh[2 * tt] = mre;
            Jh[2 * tt + 1] = mim;
            if (m < P2) {
                float c2 = rc[kRcC2 + m] * qz * ir2;
                float p1re = c2 * mre, p1im = c2 * mim, p0re = mre, p0im = mim;
                tt = (m + 1) * (m + 2) / 2 + m;
                Jh[2 * tt] = p1re;
                Jh[2 * tt + 1] = p1im;
                for (int n = m + 2; n <= P2; n++) {
                    int u = n * (n + 1) / 2 + m;
                    float A = rc[kRcA + u] * qz * ir2, B = rc[kRcB + u] * ir2;
                    float nre = A * p1re - B * p0re, nim = A * p1im - B * p0im;
                    Jh[2 * u] = nre;
                    Jh[2 * u + 1] = nim;
                    p0re = p1re;
                    p0im = p1im;
                    p1re = nre;
                    p1im = nim;
                }
            }
        }
        __syncthreads();
        if (jk < njk) {
            const float* w = W + (size_t)jk * K;
            float rn = 1.f;
            for (int n = 0; n <= p; n++) {
                float sre = 0.f, sim = 0.f;
                for (int m = -n; m <= n; m++) {
                    cf O = hat(Ms, n, m);
                    int q = j + n, mk = m - k;
                    int u = q * (q + 1) / 2 + (mk < 0 ? -mk : mk);
                    cf Jv = {Jh[2 * u], mk < 0 ? -Jh[2 * u + 1] : Jh[2 * u + 1]};
                    cf pr = cmul(O, Jv);
                    float ww = w[n * n + n + m];
                    sre += ww * pr.re;
                    sim += ww * pr.im;
                }
                are += rn * sre;
                aim += rn * sim;
                rn *= ratio;
            }
        }
    }
    if (jk < njk) {
        int ix = idx_re(j, k);
        L[(size_t)t * KP + ix] += are;
        if (k > 0) L[(size_t)t * KP + ix + 1] += aim;
    }
}

// ---------------------------------------------------------------- far field + final sum
// One workgroup per target leaf, one lane per target particle: L2P of the
// leaf's local expansion, M2P of every cell-particle source of the leaf and
// of its ancestors, plus the particle-particle part computed earlier, summed
// in FP64 and written in the caller's order.
__global__ void k_far_final(const float4* __restrict__ pts, const uint32_t* __restrict__ perm, CellArrays c,
                            const int32_t* __restrict__ leaves, const int32_t* __restrict__ m2p_off,
                            const uint32_t* __restrict__ m2p_src, int p, int KP, const float* __restrict__ gl2p,
                            const float* __restrict__ hm2p, const float* __restrict__ rc,
                            const float* __restrict__ M, const float* __restrict__ L,
                            const double4* __restrict__ near, int out_dtype, void* __restrict__ ophi,
                            void* __restrict__ oex, void* __restrict__ oey, void* __restrict__ oez) {
    extern __shared__ float sh[];
    const int K = (p + 1) * (p + 1);
    const int STR = ((p + 2) * (p + 2)) | 1;
    const int NT = blockDim.x;
    float* Lt = sh;
    float* Ms = sh + KP;
    float* row = sh + 2 * KP + threadIdx.x * STR;
    const int cell = leaves[blockIdx.x];
    const int32_t b = c.begin[cell], e = c.end[cell];
    const double4 ct = c.ctr[cell];
    for (int i = threadIdx.x; i < K; i += NT) Lt[i] = L[(size_t)cell * KP + i];
    __syncthreads();
    const float s2 = 1.41421356237309505f;
    for (int32_t ch = b; ch < e; ch += NT) {
        const int32_t i = ch + threadIdx.x;
        const bool valid = i < e;
        const float4 P = pts[valid ? i : b];
        double4 acc = valid ? near[i] : make_double4(0, 0, 0, 0);
        {
            const double ir = 1.0 / ct.w;
            float x = (float)(((double)P.x - ct.x) * ir), y = (float)(((double)P.y - ct.y) * ir),
                  z = (float)(((double)P.z - ct.z) * ir);
            regular_walk(p, x, y, z, rc, [&](int n, int m, float re, float im) {
                if (m == 0) row[n * n] = re;
                else {
                    row[n * n + 2 * m - 1] = re;
                    row[n * n + 2 * m] = im;
                }
            });
            float phi = 0.f, l10 = 0.f, l1re = 0.f, l1im = 0.f;
            for (int n = 0; n <= p; n++)
                for (int m = -n; m <= n; m++) {
                    cf Lc = hat(Lt, n, m);
                    cf Sc = hat(row, n, m);
                    phi += Lc.re * Sc.re - Lc.im * Sc.im;
                    if (n >= 1) {
                        int am = m < 0 ? -m : m;
                        if (am <= n - 1) {
                            cf S1 = hat(row, n - 1, m);
                            l10 += gl2p[n * n + n + m] * (Lc.re * S1.re - Lc.im * S1.im);
                        }
                        int m1 = m - 1, am1 = m1 < 0 ? -m1 : m1;
                        if (am1 <= n - 1) {
                            cf t = cmul(Lc, hat(row, n - 1, m1));
                            float g = gl2p[K + n * n + n + m];
                            l1re += g * t.re;
                            l1im += g * t.im;
                        }
                    }
                }
            const double r1 = ct.w, r2 = ct.w * ct.w;
            acc.x += (double)phi / r1;
            acc.y += (double)(-s2 * l1re) / r2;
            acc.z += (double)(s2 * l1im) / r2;
            acc.w += (double)(-l10) / r2;
        }
        for (int A = cell; A >= 0; A = c.parent[A]) {
            for (int32_t a = m2p_off[A]; a < m2p_off[A + 1]; a++) {
                const int s = (int)m2p_src[a];
                const double4 cs = c.ctr[s];
                __syncthreads();
                for (int u = threadIdx.x; u < K; u += NT) Ms[u] = M[(size_t)s * KP + u];
                __syncthreads();
                const double ir = 1.0 / cs.w;
                float x = (float)(((double)P.x - cs.x) * ir), y = (float)(((double)P.y - cs.y) * ir),
                      z = (float)(((double)P.z - cs.z) * ir);
                irregular_walk(p + 1, x, y, z, rc, [&](int n, int m, float re, float im) {
                    if (m == 0) row[n * n] = re;
                    else {
                        row[n * n + 2 * m - 1] = re;
                        row[n * n + 2 * m] = im;
                    }
                });
                float phi = 0.f, l10 = 0.f, l1re = 0.f, l1im = 0.f;
                for (int n = 0; n <= p; n++)
                    for (int m = -n; m <= n; m++) {
                        cf Mc = hat(Ms, n, m);
                        cf Jc = hat(row, n, m);
                        phi += Mc.re * Jc.re - Mc.im * Jc.im;
                        cf J0 = hat(row, n + 1, m);
                        l10 += hm2p[n * n + n + m] * (Mc.re * J0.re - Mc.im * J0.im);
                        cf t = cmul(Mc, hat(row, n + 1, m - 1));
                        float h = hm2p[K + n * n + n + m];
                        l1re += h * t.re;
                        l1im += h * t.im;
                    }
                const double r1 = cs.w, r2 = cs.w * cs.w;
                acc.x += (double)phi / r1;
                acc.y += (double)(-s2 * l1re) / r2;
                acc.z += (double)(s2 * l1im) / r2;
                acc.w += (double)(-l10) / r2;
            }
        }
        if (valid) {
            uint32_t o = perm[i];
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

void m2l_general(const int32_t* off, const uint32_t* src, const uint32_t* general, CellArrays cells,
                 int32_t ncell, int p, int KP, Tables t, const float* M, float* L, hipStream_t s) {
    if (ncell <= 0) return;
    int P2 = 2 * p;
    size_t lds = ((size_t)KP + 2 * (size_t)(P2 + 1) * (P2 + 2) / 2) * sizeof(float);
    k_m2l_general<<<ncell, 256, lds, s>>>(off, src, general, cells, p, KP, t.wm2l, t.rcoef, M, L);
}

void far_final(const float4* pts, const uint32_t* perm, CellArrays cells, const int32_t* leaves,
               int32_t nleaves, const int32_t* m2p_off, const uint32_t* m2p_src, int p, int KP, Tables t,
               const float* M, const float* L, const double4* near, int out_dtype, void* phi, void* ex,
               void* ey, void* ez, hipStream_t s) {
    if (nleaves <= 0) return;
    int STR = ((p + 2) * (p + 2)) | 1;
    int NT = (64 * STR + 2 * KP) * 4 <= 60000 ? 64 : 32;
    size_t lds = ((size_t)2 * KP + (size_t)NT * STR) * sizeof(float);
    k_far_final<<<nleaves, NT, lds, s>>>(pts, perm, cells, leaves, m2p_off, m2p_src, p, KP, t.gl2p, t.hm2p,
                                         t.rcoef, M, L, near, out_dtype, phi, ex, ey, ez);
}

}  // namespace fmm
