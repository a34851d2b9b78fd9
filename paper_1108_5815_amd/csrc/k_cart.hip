// k_cart.hip -- M2L of the Cartesian family outside the same-level GEMM:
// the operators of the (level difference, offset) classes, and the per-pair
// kernel for pairs whose offset does not fit the class key.
//
// With q the source centre minus the target centre in target half sides and
// rho = rs/rt, the scaled operator is (cart.h)
//     L~_m += sum_{|m|+|k|<=p} C(m,k) a_{m+k}(-q) rho^|k| M~_k .
#include "cart.h"
#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr int OB = 20;                              // bits per offset component of a class key
constexpr int64_t OLIM = ((int64_t)1 << (OB - 1)) - 1;

__device__ inline double binom_d(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; i++) r = r * (double)(n - k + i) / (double)i;
    return r;
}

// multi-index of position i in the graded order
__device__ inline void multi_of(int i, int& a, int& b, int& c) {
    int n = 0;
    while (cart::count(n) <= i) n++;
    int r = i - (n > 0 ? cart::count(n - 1) : 0);  // position within degree n
    // within a degree: (b + c) (b + c + 1)/2 + c, b + c = n - a
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= r) s++;
    c = r - s * (s + 1) / 2;
    b = s - c;
    a = n - s;
}

// Operator of class `cls` into T[cls] (k-major: T[k_in][m_out], KP x KP,
// zero-initialised), built once per class in FP64 and rounded to FP32 like
// the host-built operator tables.
template <int P>
__global__ __launch_bounds__(256) void k_cls_ops_cart(const uint64_t* __restrict__ key,
                                                      const int32_t* __restrict__ start, int KP,
                                                      float* __restrict__ T) {
    constexpr int K = cart::count(P);
    __shared__ double a[K];
    const int cls = blockIdx.x;
    const uint64_t kk = key[start[cls]];
    const int d = (int)(kk >> 60) - 8;
    const double ox = (double)((int64_t)((kk >> 40) & 0xFFFFFull) - OLIM);
    const double oy = (double)((int64_t)((kk >> 20) & 0xFFFFFull) - OLIM);
    const double oz = (double)((int64_t)(kk & 0xFFFFFull) - OLIM);
    const double sc = ldexp(1.0, -(d > 0 ? d : 0));
    const double ratio = ldexp(1.0, -d);
    if (threadIdx.x == 0) {
        double t[K];
        cart::taylor<P, double>(-ox * sc, -oy * sc, -oz * sc, t);
        for (int i = 0; i < K; i++) a[i] = t[i];
    }
    __syncthreads();
    float* Tc = T + (size_t)cls * KP * KP;
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
        const int im = e / K, ik = e - im * K;
        int m1, m2, m3, k1, k2, k3;
        multi_of(im, m1, m2, m3);
        multi_of(ik, k1, k2, k3);
        const int nk = k1 + k2 + k3;
        if (m1 + m2 + m3 + nk > P) continue;
        const double C = binom_d(m1 + k1, k1) * binom_d(m2 + k2, k2) * binom_d(m3 + k3, k3);
        double rk = 1.0;
        for (int u = 0; u < nk; u++) rk *= ratio;
        Tc[(size_t)ik * KP + im] = (float)(C * a[cart::index(m1 + k1, m2 + k2, m3 + k3)] * rk);
    }
}

// Per-pair M2L for the pairs the class key cannot hold (level difference
// beyond 8 or huge offsets): one workgroup per target cell, a wave per pair.
// FP32 with the offset taken in the larger cell's half sides, so that no
// factor overflows whatever the level difference: with the source larger,
// a_{m+k}(-q) rho^|k| = rho^-(|m|+1) a_{m+k}(-q / rho) (a_n is homogeneous
// of degree -(|n|+1)).  The waves' partial sums are added in wave order.
template <int P>
__global__ __launch_bounds__(256) void k_m2l_general_cart(const int32_t* __restrict__ goff,
                                                          const uint32_t* __restrict__ gsrc, CellArrays c, int KP,
                                                          const float* __restrict__ M, float* __restrict__ L,
                                                          const uint8_t* __restrict__ skip) {
    constexpr int K = cart::count(P);
    __shared__ float red[4][K];
    __shared__ float sa[4][K];  // per wave: the Taylor coefficients of its current pair
    const int t = blockIdx.x;
    const int32_t a0 = goff[t], a1 = goff[t + 1];
    if (a0 == a1) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int4 gt = c.geo[t];
    float acc[(K + 63) / 64];
#pragma unroll
    for (int u = 0; u < (K + 63) / 64; u++) acc[u] = 0.f;
    for (int32_t e = a0 + w; e < a1; e += 4) {
        if (skip && skip[e]) continue;  // handled by the class-batched products
        const int s = (int)gsrc[e];
        const int4 gs = c.geo[s];
        const bool src_larger = gs.w > gt.w;
        const float inv = 1.f / (float)(src_larger ? gs.w : gt.w);
        const float qx = (float)(gs.x - gt.x) * inv, qy = (float)(gs.y - gt.y) * inv,
                    qz = (float)(gs.z - gt.z) * inv;
        const float rk = src_larger ? 1.f : (float)gs.w / (float)gt.w;  // per degree of k
        const float rm = src_larger ? (float)gt.w / (float)gs.w : 1.f;  // per degree of m, times one
        if (lane == 0) {
            float a[K];
            cart::taylor<P, float>(-qx, -qy, -qz, a);
#pragma unroll
            for (int i = 0; i < K; i++) sa[w][i] = a[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float* a = sa[w];
        const float* Ms = M + (size_t)s * KP;
#pragma unroll
        for (int u = 0; u < (K + 63) / 64; u++) {
            const int im = lane + 64 * u;
            if (im >= K) continue;
            int m1, m2, m3;
            multi_of(im, m1, m2, m3);
            const int nm = m1 + m2 + m3;
            float fm = rm;
            for (int v = 0; v < nm; v++) fm *= rm;  // rm^(|m|+1)
            float sum = 0.f, fk = 1.f;
            for (int nk = 0; nk + nm <= P; nk++) {
                float part = 0.f;
                for (int k1 = nk; k1 >= 0; k1--)
                    for (int k2 = nk - k1; k2 >= 0; k2--) {
                        const int k3 = nk - k1 - k2;
                        const float C = (float)(binom_d(m1 + k1, k1) * binom_d(m2 + k2, k2) * binom_d(m3 + k3, k3));
                        part += C * a[cart::index(m1 + k1, m2 + k2, m3 + k3)] * Ms[cart::index(k1, k2, k3)];
                    }
                sum += fk * part;
                fk *= rk;
            }
            acc[u] += fm * sum;
        }
        // the next pair's coefficients overwrite sa[w] only after every lane read these
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int u = 0; u < (K + 63) / 64; u++) {
        const int im = lane + 64 * u;
        if (im < K) red[w][im] = acc[u];
    }
    __syncthreads();
    for (int im = threadIdx.x; im < K; im += 256)
        L[(size_t)t * KP + im] += ((red[0][im] + red[1][im]) + red[2][im]) + red[3][im];
}

}  // namespace

void cls_ops_cart(const uint64_t* key, const int32_t* start, int32_t ncls, int p, int KP, float* T, hipStream_t s) {
    if (ncls <= 0) return;
#define FMM_CLS_CART(PP)                                                  \
    case PP:                                                              \
        k_cls_ops_cart<PP><<<ncls, 256, 0, s>>>(key, start, KP, T);       \
        break;
    switch (p) {
        FMM_CLS_CART(0)
        FMM_CLS_CART(1)
        FMM_CLS_CART(2)
        FMM_CLS_CART(3)
        FMM_CLS_CART(4)
        FMM_CLS_CART(5)
        FMM_CLS_CART(6)
        default:
            break;
    }
#undef FMM_CLS_CART
}

void m2l_general_cart(const int32_t* goff, const uint32_t* gsrc, CellArrays cells, int32_t ncell, int p, int KP,
                      const float* M, float* L, const uint8_t* skip, hipStream_t s) {
    if (ncell <= 0) return;
#define FMM_GEN_CART(PP)                                                                          \
    case PP:                                                                                      \
        k_m2l_general_cart<PP><<<ncell, 256, 0, s>>>(goff, gsrc, cells, KP, M, L, skip);          \
        break;
    switch (p) {
        FMM_GEN_CART(0)
        FMM_GEN_CART(1)
        FMM_GEN_CART(2)
        FMM_GEN_CART(3)
        FMM_GEN_CART(4)
        FMM_GEN_CART(5)
        FMM_GEN_CART(6)
        default:
            break;
    }
#undef FMM_GEN_CART
}

}  // namespace fmm
