// k_m2l_cls.hip -- M2L of the pairs outside the same-level tables, batched
// by class on the matrix cores.
//
// Mixed-level pairs (and same-level pairs whose parents were at different
// levels) have no fixed slot in a target's offset table.  Their scaled
// operator depends only on the level difference d = level(s) - level(t) and
// on the integer offset o between the cube centres in units of the smaller
// half side: the offset in target half sides is q = o 2^-max(d,0) and the
// radius ratio r_s / r_t = 2^-d.  So the pairs are keyed by (d, o), sorted,
// and each class gets its operator once (built on the GPU in FP64 from the
// irregular harmonics of q, rounded to FP32, in the real layout of the
// coefficients); then every tile of up to NT pairs of a class is one dense
// product [K x K] x [K x NT] on v_mfma_f32_32x32x2f32, written to a partial
// row per pair; each target sums its pairs' partials in its list order (no
// atomics, deterministic, independent of the other pairs of a tile).
// Offsets too large for the key (never on the workloads measured) keep the
// per-pair kernel.
#include "fmm_internal.h"

namespace fmm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int OB = 20;                             // bits per offset component
constexpr int64_t OLIM = ((int64_t)1 << (OB - 1)) - 1;
constexpr uint64_t OVERSIZE = ~0ull;

__global__ void k_cls_keys(const uint32_t* __restrict__ gt, const uint32_t* __restrict__ gs, int64_t ng,
                           CellArrays c, uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    const int t = (int)gt[i], s = (int)gs[i];
    const int4 a = c.geo[t], b = c.geo[s];
    const int d = c.level[s] - c.level[t];
    const int64_t rmin = a.w < b.w ? a.w : b.w;
    const int64_t ox = ((int64_t)b.x - a.x) / rmin, oy = ((int64_t)b.y - a.y) / rmin,
                  oz = ((int64_t)b.z - a.z) / rmin;
    const bool ok = d >= -8 && d <= 7 && ox >= -OLIM && ox <= OLIM && oy >= -OLIM && oy <= OLIM &&
                    oz >= -OLIM && oz <= OLIM;
    key[i] = ok ? ((uint64_t)(d + 8) << 60) | ((uint64_t)(ox + OLIM) << 40) | ((uint64_t)(oy + OLIM) << 20) |
                      (uint64_t)(oz + OLIM)
                : OVERSIZE;
    val[i] = (uint32_t)i;
}

// head[i] = 1 where a class starts (sorted keys; the oversize group is no class)
__global__ void k_cls_heads(const uint64_t* __restrict__ key, int64_t n, uint32_t* __restrict__ head) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    head[i] = (key[i] != OVERSIZE && (i == 0 || key[i] != key[i - 1])) ? 1u : 0u;
}

// class starts, the sorted position of every pair and the source of every sorted position
__global__ void k_cls_index(const uint32_t* __restrict__ head, const uint32_t* __restrict__ hoff, int64_t n,
                            const uint32_t* __restrict__ val, const uint32_t* __restrict__ gs,
                            int32_t* __restrict__ start, int32_t* __restrict__ pos, uint32_t* __restrict__ srcs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (head[i]) start[hoff[i]] = (int32_t)i;
    pos[val[i]] = (int32_t)i;
    srcs[i] = gs[val[i]];
}

// tiles of class k: ntile[k] = ceil((start[k+1] - start[k]) / NT)
__global__ void k_cls_ntiles(const int32_t* __restrict__ start, int32_t ncls, int NT, uint32_t* __restrict__ nt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncls) return;
    nt[k] = (uint32_t)((start[k + 1] - start[k] + NT - 1) / NT);
}

__global__ void k_cls_tiles(const uint32_t* __restrict__ nt, const uint32_t* __restrict__ tbase, int32_t ncls,
                            int32_t* __restrict__ tile_cls) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncls) return;
    for (uint32_t u = 0; u < nt[k]; u++) tile_cls[tbase[k] + u] = k;
}

__device__ inline int ri(int n, int m, bool im) { return m == 0 ? n * n : n * n + 2 * m - (im ? 0 : 1); }

// Operator of class k (k-major, T[kin][row], KP x KP, zero-initialised):
// L(j,k) += sum_(n,m) W(j,k,n,m) ratio^n J_{j+n}^{m-k}(q) O_n^m with
// O_n^{-m} = conj(O_n^m), folded onto the real and imaginary parts.
__global__ __launch_bounds__(256) void k_cls_ops(const uint64_t* __restrict__ key, const int32_t* __restrict__ start,
                                                 int p, int KP, const float* __restrict__ W, float* __restrict__ T) {
    extern __shared__ double Jh[];  // (2p+1)(2p+2)/2 complex values
    const int cls = blockIdx.x;
    const uint64_t kk = key[start[cls]];
    const int d = (int)(kk >> 60) - 8;
    const double ox = (double)((int64_t)((kk >> 40) & 0xFFFFFull) - OLIM);
    const double oy = (double)((int64_t)((kk >> 20) & 0xFFFFFull) - OLIM);
    const double oz = (double)((int64_t)(kk & 0xFFFFFull) - OLIM);
    const double sc = ldexp(1.0, -(d > 0 ? d : 0));
    const double x = ox * sc, y = oy * sc, z = oz * sc;
    const double ratio = ldexp(1.0, -d);
    const int P2 = 2 * p;
    // irregular solid harmonics J_n^m(q), m >= 0, one column m per thread
    const double r2 = x * x + y * y + z * z, ir2 = 1.0 / r2;
    for (int m = threadIdx.x; m <= P2; m += blockDim.x) {
        double mre = sqrt(ir2), mim = 0.0;
        for (int mm = 1; mm <= m; mm++) {
            const double cc = sqrt((2.0 * mm - 1) / (2.0 * mm)) * ir2;
            const double nre = cc * (x * mre - y * mim), nim = cc * (x * mim + y * mre);
            mre = nre;
            mim = nim;
        }
        int t = m * (m + 1) / 2 + m;
        Jh[2 * t] = mre;
        Jh[2 * t + 1] = mim;
        if (m < P2) {
            const double c2 = sqrt(2.0 * m + 1) * z * ir2;
            double p1re = c2 * mre, p1im = c2 * mim, p0re = mre, p0im = mim;
            t = (m + 1) * (m + 2) / 2 + m;
            Jh[2 * t] = p1re;
            Jh[2 * t + 1] = p1im;
            for (int n = m + 2; n <= P2; n++) {
                const int u = n * (n + 1) / 2 + m;
                const double A = (2.0 * n - 1) * z * ir2 / sqrt((double)(n - m) * (n + m));
                const double B = sqrt((double)(n + m - 1) * (n - m - 1)) * ir2 / sqrt((double)(n - m) * (n + m));
                const double nre = A * p1re - B * p0re, nim = A * p1im - B * p0im;
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
    auto J = [&](int n, int m, double& re, double& im) {
        const int u = n * (n + 1) / 2 + (m < 0 ? -m : m);
        re = Jh[2 * u];
        im = m < 0 ? -Jh[2 * u + 1] : Jh[2 * u + 1];
    };
    const int K = (p + 1) * (p + 1);
    const int njk = (p + 1) * (p + 2) / 2;
    float* Tc = T + (size_t)cls * KP * KP;
    for (int jk = threadIdx.x; jk < njk; jk += blockDim.x) {
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= jk) j++;
        const int k = jk - j * (j + 1) / 2;
        const float* wr = W + (size_t)jk * K;
        const int rre = ri(j, k, false), rim = ri(j, k, true);
        double rn = 1.0;
        for (int n = 0; n <= p; n++) {
            for (int am = 0; am <= n; am++) {
                double jr, ji;
                J(j + n, am - k, jr, ji);
                const double wp = (double)wr[n * n + n + am] * rn;
                const double pre = wp * jr, pim = wp * ji;
                const int cre = ri(n, am, false);
                if (am == 0) {
                    Tc[(size_t)cre * KP + rre] = (float)pre;
                    if (k > 0) Tc[(size_t)cre * KP + rim] = (float)pim;
                } else {
                    J(j + n, -am - k, jr, ji);
                    const double wm = (double)wr[n * n + n - am] * rn;
                    const double mre = wm * jr, mim = wm * ji;
                    const int cim = ri(n, am, true);
                    Tc[(size_t)cre * KP + rre] = (float)(pre + mre);
                    Tc[(size_t)cim * KP + rre] = (float)(-pim + mim);
                    if (k > 0) {
                        Tc[(size_t)cre * KP + rim] = (float)(pim + mim);
                        Tc[(size_t)cim * KP + rim] = (float)(pre - mre);
                    }
                }
            }
            rn *= ratio;
        }
    }
}

// One tile of up to NT pairs of one class: part[row] = T_class M[source].
template <int KP, int NT, int RW, int CW>
__global__ __launch_bounds__(256) void k_m2l_cls(const float* __restrict__ T, const int32_t* __restrict__ tile_cls,
                                                 const uint32_t* __restrict__ tbase,
                                                 const int32_t* __restrict__ start,
                                                 const uint32_t* __restrict__ srcs, int32_t zcell,
                                                 const float* __restrict__ M, float* __restrict__ part) {
    constexpr int KS = KP / 2;
    constexpr int RB = KP / 32, CB = NT / 32;
    static_assert(RB % RW == 0 && CB % CW == 0 && RW * CW == 4, "wave grid");
    constexpr int NRB = RB / RW, NCB = CB / CW;
    constexpr int STR = KP + 4;
    constexpr int CH = 16;
    constexpr int NCH = KS / CH;
    constexpr int BV = NT * KP / 1024;
    static_assert(KS % CH == 0 && (NT * KP) % 1024 == 0, "tile shape");
    __shared__ __attribute__((aligned(16))) float Bs[NT * STR];

    const int tile = blockIdx.x;
    const int cls = tile_cls[tile];
    const int r0 = start[cls] + (tile - (int)tbase[cls]) * NT;
    const int nrow = min(NT, start[cls + 1] - r0);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l32 = lane & 31, h = lane >> 5;
    const int wr = w % RW, wc = w / RW;
    const float* A = T + (size_t)cls * KP * KP;

    {
        int sidx[BV];
#pragma unroll
        for (int v = 0; v < BV; v++) {
            const int col = (threadIdx.x + 256 * v) / (KP / 4);
            sidx[v] = col < nrow ? (int)srcs[r0 + col] : zcell;
        }
#pragma unroll
        for (int v = 0; v < BV; v++) {
            const int idx = threadIdx.x + 256 * v;
            const int col = idx / (KP / 4), k4 = idx - col * (KP / 4);
            *reinterpret_cast<f32x4*>(&Bs[col * STR + 4 * k4]) =
                reinterpret_cast<const f32x4*>(M + (size_t)sidx[v] * KP)[k4];
        }
    }
    floatx16 acc[NRB][NCB];
#pragma unroll
    for (int i = 0; i < NRB; i++)
#pragma unroll
        for (int b = 0; b < NCB; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[i][b][r] = 0.f;
    float a0[NRB][CH], a1[NRB][CH];
    auto load_A = [&](int c, float (&a)[NRB][CH]) {
#pragma unroll
        for (int i = 0; i < NRB; i++)
#pragma unroll
            for (int t = 0; t < CH; t++) a[i][t] = A[(size_t)(h * KS + c * CH + t) * KP + (wr + RW * i) * 32 + l32];
    };
    auto compute = [&](int c, const float (&a)[NRB][CH]) {
#pragma unroll
        for (int t = 0; t < CH; t += 4) {
            f32x4 b4[NCB];
#pragma unroll
            for (int b = 0; b < NCB; b++) {
                const int col = (wc + CW * b) * 32 + l32;
                b4[b] = *reinterpret_cast<const f32x4*>(&Bs[col * STR + h * KS + c * CH + t]);
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int b = 0; b < NCB; b++)
#pragma unroll
                    for (int i = 0; i < NRB; i++)
                        acc[i][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][t + u], b4[b][u], acc[i][b], 0, 0, 0);
        }
    };
    load_A(0, a0);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NCH; c++) {
        if ((c & 1) == 0) {
            if (c + 1 < NCH) load_A(c + 1, a1);
            compute(c, a0);
        } else {
            if (c + 1 < NCH) load_A(c + 1, a0);
            compute(c, a1);
        }
    }
#pragma unroll
    for (int b = 0; b < NCB; b++) {
        const int col = (wc + CW * b) * 32 + l32;
        if (col >= nrow) continue;
        float* dst = part + (size_t)(r0 + col) * KP;
#pragma unroll
        for (int i = 0; i < NRB; i++)
#pragma unroll
            for (int r = 0; r < 16; r++) dst[(wr + RW * i) * 32 + 8 * (r >> 2) + 4 * h + (r & 3)] = acc[i][b][r];
    }
}

// L[t][j] += sum over the target's batched pairs, in list order, of their partial rows
__global__ void k_cls_reduce(const int32_t* __restrict__ goff, const int32_t* __restrict__ pos, int32_t nbatched,
                             int32_t ncell, int KP, int K, const float* __restrict__ part, float* __restrict__ L) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)ncell * KP) return;
    const int t = (int)(i / KP), j = (int)(i - (int64_t)t * KP);
    const int a0 = goff[t], a1 = goff[t + 1];
    if (a0 == a1 || j >= K) return;
    float s = 0.f;
    bool any = false;
    for (int a = a0; a < a1; a++) {
        const int q = pos[a];
        if (q < nbatched) {
            s += part[(size_t)q * KP + j];
            any = true;
        }
    }
    if (any) L[(size_t)t * KP + j] += s;
}

__global__ void k_cls_end(const uint64_t* __restrict__ key, int64_t n, int32_t* __restrict__ start, int32_t ncls) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] != OVERSIZE) lo = mid + 1;
        else hi = mid;
    }
    start[ncls] = (int32_t)lo;
}

__global__ void k_cls_skip(const int32_t* __restrict__ pos, int64_t ng, int32_t nbatched, uint8_t* __restrict__ skip) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < ng) skip[a] = pos[a] < nbatched ? 1 : 0;
}

template <int KP, int NT, int RW, int CW>
void launch(const float* T, const ClsPlan& cp, const float* M, float* part, hipStream_t s) {
    k_m2l_cls<KP, NT, RW, CW><<<cp.ntiles, 256, 0, s>>>(T, cp.tile_cls, cp.tbase, cp.start, cp.srcs, cp.zcell, M,
                                                        part);
}

inline unsigned grid(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int cls_tile_cols(int KP) {
    switch (KP) {
        case 32: case 64: case 96: return 128;
        case 128: case 192: case 256: return 64;
        default: return 0;
    }
}

void cls_keys(const uint32_t* gt, const uint32_t* gs, int64_t ng, CellArrays cells, uint64_t* key, uint32_t* val,
              hipStream_t s) {
    if (ng <= 0) return;
    k_cls_keys<<<grid(ng), 256, 0, s>>>(gt, gs, ng, cells, key, val);
}

void cls_heads(const uint64_t* key, int64_t n, uint32_t* head, hipStream_t s) {
    if (n <= 0) return;
    k_cls_heads<<<grid(n), 256, 0, s>>>(key, n, head);
}

void cls_index(const uint32_t* head, const uint32_t* hoff, int64_t n, const uint32_t* val, const uint32_t* gs,
               int32_t* start, int32_t* pos, uint32_t* srcs, hipStream_t s) {
    if (n <= 0) return;
    k_cls_index<<<grid(n), 256, 0, s>>>(head, hoff, n, val, gs, start, pos, srcs);
}

void cls_end(const uint64_t* key, int64_t n, int32_t* start, int32_t ncls, hipStream_t s) {
    k_cls_end<<<1, 64, 0, s>>>(key, n, start, ncls);
}

void cls_ntiles(const int32_t* start, int32_t ncls, int NT, uint32_t* nt, hipStream_t s) {
    if (ncls <= 0) return;
    k_cls_ntiles<<<grid(ncls), 256, 0, s>>>(start, ncls, NT, nt);
}

void cls_tiles(const uint32_t* nt, const uint32_t* tbase, int32_t ncls, int32_t* tile_cls, hipStream_t s) {
    if (ncls <= 0) return;
    k_cls_tiles<<<grid(ncls), 256, 0, s>>>(nt, tbase, ncls, tile_cls);
}

void cls_ops(const uint64_t* key, const int32_t* start, int32_t ncls, int p, int KP, const float* W, float* T,
             hipStream_t s) {
    if (ncls <= 0) return;
    const size_t lds = (size_t)(2 * p + 1) * (2 * p + 2) / 2 * 2 * sizeof(double);
    k_cls_ops<<<ncls, 256, lds, s>>>(key, start, p, KP, W, T);
}

void cls_skip(const int32_t* pos, int64_t ng, int32_t nbatched, uint8_t* skip, hipStream_t s) {
    if (ng <= 0) return;
    k_cls_skip<<<grid(ng), 256, 0, s>>>(pos, ng, nbatched, skip);
}

void m2l_cls(const float* T, const ClsPlan& cp, int K, int KP, const float* M, float* part, const int32_t* goff,
             int32_t ncell, float* L, hipStream_t s) {
    if (cp.ntiles <= 0) return;
    switch (KP) {
        case 32: launch<32, 128, 1, 4>(T, cp, M, part, s); break;
        case 64: launch<64, 128, 2, 2>(T, cp, M, part, s); break;
        case 96: launch<96, 128, 1, 4>(T, cp, M, part, s); break;
        case 128: launch<128, 64, 4, 1>(T, cp, M, part, s); break;
        case 192: launch<192, 64, 2, 2>(T, cp, M, part, s); break;
        case 256: launch<256, 64, 4, 1>(T, cp, M, part, s); break;
        default: return;
    }
    k_cls_reduce<<<grid((int64_t)ncell * KP), 256, 0, s>>>(goff, cp.pos, cp.nbatched, ncell, KP, K, part, L);
}

}  // namespace fmm
