// k_expand.hip -- M2M, L2L and the general M2L of the spherical-harmonic
// expansions (P2M and the far-field evaluation are in k_far.hip).
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

// ---------------------------------------------------------------- M2M / L2L
// One level's octant translations on the VALU, NB non-leaf parents per
// workgroup.  The inputs of the batch are staged in LDS (M2M: the children of
// every octant; L2L: the parents' locals); thread j of an octant streams the
// operator column T_o[., j] from memory (coalesced over j, loads issued two
// blocks of 8 ahead) and keeps the NB dot products of output j, so each
// operator element feeds NB FMAs and each input read (an LDS broadcast) four.
// OW octants run side by side in separate waves (8 for the small levels near
// the root, where there are few parents to batch).  Per parent and octant the
// dot product runs over k ascending (terms whose degrees do not couple are
// exact zeros and the blocks holding only such terms are skipped per wave);
// M2M then adds the 8 octant products in octant order, L2L adds each into its
// child.  A parent's result therefore does not depend on NB, OW or the other
// parents of its batch.
template <bool UP, int NB, int OW, int NJ>
__global__ __launch_bounds__(OW * NJ) void k_translate(CellArrays c, const int32_t* __restrict__ inner,
                                                        const uint32_t* __restrict__ leafpos, int32_t c0,
                                                        int32_t c1, int32_t ncell, int32_t nleaf, int K, int KP,
                                                        const float* __restrict__ mat, float* __restrict__ X) {
    constexpr int NTH = OW * NJ;
    constexpr int KB = 8;  // k block of the operator stream
    extern __shared__ __attribute__((aligned(16))) float sh[];
    __shared__ int32_t sIn[8][NB];  // child of octant o of each parent, or -1
    __shared__ int32_t sPar[NB];
    const int tid = threadIdx.x;
    const int KS = (K + KB - 1) / KB * KB;  // staged input stride (zero padded)
    // this level's non-leaf cells: inner[n0 .. n1) (cells are numbered level by
    // level; leafpos[i] = leaves among cells [0, i))
    const int32_t n0 = c0 - (int32_t)leafpos[c0];
    const int32_t n1 = c1 - (c1 < ncell ? (int32_t)leafpos[c1] : nleaf);
    const int32_t b0 = n0 + (int32_t)blockIdx.x * NB;
    if (b0 >= n1) return;
    const int nb = min(NB, n1 - b0);
    for (int i = tid; i < NB; i += NTH) {
        int ch[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
        const int P = i < nb ? inner[b0 + i] : -1;
        if (P >= 0) {
            const int f = c.child[P], n = c.nchild[P];
            for (int q = 0; q < n; q++) ch[c.prefix[f + q] & 7u] = f + q;
        }
        sPar[i] = P;
#pragma unroll
        for (int o = 0; o < 8; o++) sIn[o][i] = ch[o];
    }
    __syncthreads();
    // inputs: M2M sV[o][cc][k] (children), L2L sV[cc][k] (parents)
    float* sV = sh;
    const int nin = (UP ? 8 : 1) * NB * KS;
    for (int i = tid; i < nin; i += NTH) {
        const int row = i / KS, k = i - row * KS;
        const int src = UP ? sIn[row / NB][row % NB] : sPar[row];
        sV[i] = (src >= 0 && k < K) ? X[(size_t)src * KP + k] : 0.f;
    }
    float* part = sh + nin;  // M2M with OW > 1: octant products [8][NB][NJ]
    __syncthreads();
    const int og = tid / NJ, jt = tid - og * NJ;
    const int wave = jt >> 6;
    for (int jb = 0; jb < KP; jb += NJ) {
        const int j = jb + jt;
        // inputs that can couple to this wave's outputs: [klo, khi)
        const int jlo = min(jb + 64 * wave, K - 1), jhi = min(jb + 64 * wave + 63, K - 1);
        const int dlo = degree_of(jlo), dhi = degree_of(jhi);
        const int klo = UP ? 0 : (dlo * dlo) / KB * KB;
        const int khi = UP ? min((dhi + 1) * (dhi + 1), K) : K;
        float tot[NB];
#pragma unroll
        for (int cc = 0; cc < NB; cc++) tot[cc] = 0.f;
        for (int o = og; o < 8; o += OW) {
            const float* Vo = UP ? sV + (size_t)o * NB * KS : sV;
            const float* To = mat + (size_t)o * K * K;  // wave-uniform base, 32-bit lane offsets
            const int jj = j < K ? j : 0;
            float acc[NB];
#pragma unroll
            for (int cc = 0; cc < NB; cc++) acc[cc] = 0.f;
            float t0[KB], t1[KB];
            auto load = [&](int k, float (&t)[KB]) {
#pragma unroll
                for (int i = 0; i < KB; i++) t[i] = (k + i < K && j < K) ? To[(k + i) * K + jj] : 0.f;
            };
            auto dot = [&](int k, const float (&t)[KB]) {
#pragma unroll
                for (int i = 0; i < KB; i += 4) {
#pragma unroll
                    for (int cc = 0; cc < NB; cc++) {
                        const float4 v = *reinterpret_cast<const float4*>(&Vo[cc * KS + k + i]);
                        acc[cc] = fmaf(t[i], v.x, acc[cc]);
                        acc[cc] = fmaf(t[i + 1], v.y, acc[cc]);
                        acc[cc] = fmaf(t[i + 2], v.z, acc[cc]);
                        acc[cc] = fmaf(t[i + 3], v.w, acc[cc]);
                    }
                }
            };
            // two register blocks: the loads of block k + 2 KB are issued
            // before the products of block k
            int k = klo;
            if (k < khi) load(k, t0);
            if (k + KB < khi) load(k + KB, t1);
            for (; k < khi; k += 2 * KB) {
                float u[KB];
#pragma unroll
                for (int i = 0; i < KB; i++) u[i] = t0[i];
                if (k + 2 * KB < khi) load(k + 2 * KB, t0);
                dot(k, u);
                if (k + KB < khi) {
#pragma unroll
                    for (int i = 0; i < KB; i++) u[i] = t1[i];
                    if (k + 3 * KB < khi) load(k + 3 * KB, t1);
                    dot(k + KB, u);
                }
            }
            if (UP) {
                if (OW == 1) {
#pragma unroll
                    for (int cc = 0; cc < NB; cc++) tot[cc] += acc[cc];
                } else {
#pragma unroll
                    for (int cc = 0; cc < NB; cc++) part[((size_t)o * NB + cc) * NJ + jt] = acc[cc];
                }
            } else {
#pragma unroll
                for (int cc = 0; cc < NB; cc++) {
                    const int ch = sIn[o][cc];
                    if (ch >= 0 && j < K) X[(size_t)ch * KP + j] += acc[cc];
                }
            }
        }
        if (UP) {
            if (OW > 1) {
                __syncthreads();
                if (og == 0) {
#pragma unroll
                    for (int cc = 0; cc < NB; cc++)
                        for (int o = 0; o < 8; o++) tot[cc] += part[((size_t)o * NB + cc) * NJ + jt];
                }
                __syncthreads();
            }
            if (og == 0) {
#pragma unroll
                for (int cc = 0; cc < NB; cc++)
                    if (cc < nb && j < KP) X[(size_t)sPar[cc] * KP + j] = j < K ? tot[cc] : 0.f;
            }
        }
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
    for (int32_t a = a0 + w; a < a1; a += 4) {
        if (skip && skip[a]) continue;  // handled by the class-batched products
        const int s = (int)gsrc[a];
        const int4 gs = c.geo[s];
        // The terms are (rs/rt)^n J_{j+n}(q) with q the offset in target half
        // sides.  When the source is the larger cell, q is taken in source
        // half sides instead, which turns the term into
        // (rs/rt)^-(j+1) J_{j+n}(q rt/rs) (J_l is homogeneous of degree
        // -(l+1)): every factor then stays at most of order one and the
        // products underflow towards zero instead of meeting an overflow,
        // whatever the level difference.  The half sides are powers of two,
        // so both scalings are exact.
        const bool src_larger = gs.w > gt.w;
        const float inv = 1.f / (float)(src_larger ? gs.w : gt.w);
        const float qx = (float)(gs.x - gt.x) * inv, qy = (float)(gs.y - gt.y) * inv,
                    qz = (float)(gs.z - gt.z) * inv;
        const float ratio = src_larger ? 1.f : (float)gs.w / (float)gt.w;  // per degree n of the source
        const float jfac = src_larger ? (float)gt.w / (float)gs.w : 1.f;   // per degree j of the target
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
            float rj = jfac;
            for (int jj = 0; jj < j; jj++) rj *= jfac;  // jfac^(j+1)
            float rn = rj, tre = 0.f, tim = 0.f;
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

template <bool UP, int NB, int OW, int NJ>
void translate_launch(CellArrays cells, const int32_t* inner, const uint32_t* leafpos, int32_t c0, int32_t c1,
                      int32_t ncell, int32_t nleaf, int K, int KP, const float* mat, float* X, hipStream_t s) {
    const int32_t n = c1 - c0;  // bounds the level's non-leaf cells
    const size_t KS = (size_t)(K + 7) / 8 * 8;
    const size_t lds = ((UP ? 8 : 1) * NB * KS + (UP && OW > 1 ? (size_t)8 * NB * NJ : 0)) * sizeof(float);
    k_translate<UP, NB, OW, NJ><<<(n + NB - 1) / NB, OW * NJ, lds, s>>>(cells, inner, leafpos, c0, c1, ncell, nleaf,
                                                                         K, KP, mat, X);
}

template <bool UP>
void translate_level(CellArrays cells, const int32_t* inner, const uint32_t* leafpos, int32_t c0, int32_t c1,
                     int32_t ncell, int32_t nleaf, int K, int KP, const float* mat, float* X, hipStream_t s) {
    const int32_t n = c1 - c0;
    if (n <= 0) return;
    // levels near the root: few parents, the 8 octants side by side
    if (K <= 128) {
        if (n >= 256) translate_launch<UP, 8, 8, 128>(cells, inner, leafpos, c0, c1, ncell, nleaf, K, KP, mat, X, s);
        else translate_launch<UP, 2, 8, 128>(cells, inner, leafpos, c0, c1, ncell, nleaf, K, KP, mat, X, s);
    } else {
        if (n >= 256) translate_launch<UP, 4, 1, 256>(cells, inner, leafpos, c0, c1, ncell, nleaf, K, KP, mat, X, s);
        else translate_launch<UP, 1, 2, 256>(cells, inner, leafpos, c0, c1, ncell, nleaf, K, KP, mat, X, s);
    }
}

void m2m(CellArrays cells, const int32_t* inner, const uint32_t* leafpos, int32_t c0, int32_t c1, int32_t ncell,
         int32_t nleaf, int K, int KP, Tables t, float* M, hipStream_t s) {
    translate_level<true>(cells, inner, leafpos, c0, c1, ncell, nleaf, K, KP, t.m2m, M, s);
}

void l2l(CellArrays cells, const int32_t* inner, const uint32_t* leafpos, int32_t c0, int32_t c1, int32_t ncell,
         int32_t nleaf, int K, int KP, Tables t, float* L, hipStream_t s) {
    translate_level<false>(cells, inner, leafpos, c0, c1, ncell, nleaf, K, KP, t.l2l, L, s);
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
