// k_m2l_bf16.hip -- same-level M2L GEMMs in split-BF16 on the matrix cores.
//
// The batching is that of k_m2l_gemm.hip (one octant class and a tile of
// targets per workgroup, K running over (slot, coefficient)).  Here every
// FP32 operand a is split into a_hi = bf16(a) and a_lo = bf16(a - a_hi)
// (round to nearest even), and each product is formed from three BF16
// products on v_mfma_f32_32x32x16_bf16 with FP32 accumulation:
//     a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// The dropped a_lo b_lo term and the residual of the two-term split bound
// the relative error of each product by about 2^-16.  The operators are split
// once on the host and stored k-blocked ([offset][KP/8][KP][8] bf16) so that
// a lane's 8 consecutive K values for its row are one 16-byte load; the
// gathered source vectors are split when staged into LDS.
#include "fmm_internal.h"

namespace fmm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ inline uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int KP, int NT, int RW, int CW, bool DBA>
__global__ __launch_bounds__(256) void k_m2l_bf16(const uint4* __restrict__ Thi, const uint4* __restrict__ Tlo,
                                                  const int32_t* __restrict__ offid,
                                                  const int32_t* __restrict__ gather,
                                                  const uint32_t* __restrict__ rowcell, GemmPlan plan, int K,
                                                  const float* __restrict__ M, float* __restrict__ L) {
    constexpr int KB = KP / 8;          // 8-wide K blocks
    constexpr int KS = KP / 16;         // MFMA K steps (16 values each)
    constexpr int RB = KP / 32, CB = NT / 32;
    static_assert(RB % RW == 0 && CB % CW == 0 && RW * CW == 4, "wave grid");
    constexpr int NRB = RB / RW, NCB = CB / CW;
    constexpr int STR = KB + 1;         // LDS row stride in 16-byte units
    constexpr int BV = NT * KP / 1024;  // float4 per thread per source tile
    static_assert((NT * KP) % 1024 == 0, "tile shape");
    __shared__ uint4 Bhi[2][NT * STR];
    __shared__ uint4 Blo[2][NT * STR];

    const int tile = blockIdx.x;
    int cls = 0;
    while (cls < 7 && tile >= plan.class_tile0[cls + 1]) cls++;
    const int r0 = plan.class_row0[cls] + (tile - plan.class_tile0[cls]) * NT;
    const int nrow = min(NT, plan.class_row0[cls + 1] - r0);
    const int J = plan.J;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l32 = lane & 31, h = lane >> 5;
    const int wr = w % RW, wc = w / RW;
    const int32_t* oid = offid + (size_t)cls * J;
    // the slots that some row of the tile uses (at least one for every tile)
    const int32_t* act = plan.act + (size_t)tile * J;
    const int na = plan.nact[tile];
    if (na <= 0) return;

    floatx16 acc[NRB][NCB];
#pragma unroll
    for (int i = 0; i < NRB; i++)
#pragma unroll
        for (int b = 0; b < NCB; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[i][b][r] = 0.f;

    float4 breg[BV];
    auto load_B = [&](int k) {
        const int j = act[k];
#pragma unroll
        for (int v = 0; v < BV; v++) {
            int idx = threadIdx.x + 256 * v;
            int col = idx / (KP / 4), k4 = idx - col * (KP / 4);
            int s = col < nrow ? gather[(size_t)(r0 + col) * J + j] : -1;
            breg[v] = s >= 0 ? reinterpret_cast<const float4*>(M + (size_t)s * KP)[k4]
                             : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    // each thread holds 4 consecutive K values of one column: half a 16-byte block
    auto store_B = [&](int buf) {
#pragma unroll
        for (int v = 0; v < BV; v++) {
            int idx = threadIdx.x + 256 * v;
            int col = idx / (KP / 4), k4 = idx - col * (KP / 4);
            float xs[4] = {breg[v].x, breg[v].y, breg[v].z, breg[v].w};
            uint16_t hi[4], lo[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                hi[e] = bf16_rne(xs[e]);
                lo[e] = bf16_rne(xs[e] - bf16_to_f(hi[e]));
            }
            uint2 ph = make_uint2((uint32_t)hi[0] | ((uint32_t)hi[1] << 16), (uint32_t)hi[2] | ((uint32_t)hi[3] << 16));
            uint2 pl = make_uint2((uint32_t)lo[0] | ((uint32_t)lo[1] << 16), (uint32_t)lo[2] | ((uint32_t)lo[3] << 16));
            uint2* dh = reinterpret_cast<uint2*>(&Bhi[buf][col * STR + (k4 >> 1)]) + (k4 & 1);
            uint2* dl = reinterpret_cast<uint2*>(&Blo[buf][col * STR + (k4 >> 1)]) + (k4 & 1);
            *dh = ph;
            *dl = pl;
        }
    };
    // operator fragments of one slot: step s, half h -> K block 2s + h
    constexpr int NA = DBA ? 2 : 1;
    uint4 ah[NA][NRB][KS], al[NA][NRB][KS];
    auto load_A = [&](int k, int buf) {
        const size_t base = (size_t)oid[act[k]] * KB * KP;
#pragma unroll
        for (int i = 0; i < NRB; i++)
#pragma unroll
            for (int s = 0; s < KS; s++) {
                const size_t ix = base + (size_t)(2 * s + h) * KP + (wr + RW * i) * 32 + l32;
                ah[buf][i][s] = Thi[ix];
                al[buf][i][s] = Tlo[ix];
            }
    };
    auto compute = [&](int bbuf, int abuf) {
#pragma unroll
        for (int s = 0; s < KS; s++) {
#pragma unroll
            for (int b = 0; b < NCB; b++) {
                const int col = (wc + CW * b) * 32 + l32;
                const uint4 bh = Bhi[bbuf][col * STR + 2 * s + h];
                const uint4 bl = Blo[bbuf][col * STR + 2 * s + h];
                const bf16x8 vbh = __builtin_bit_cast(bf16x8, bh);
                const bf16x8 vbl = __builtin_bit_cast(bf16x8, bl);
#pragma unroll
                for (int i = 0; i < NRB; i++) {
                    const bf16x8 vah = __builtin_bit_cast(bf16x8, ah[abuf][i][s]);
                    const bf16x8 val = __builtin_bit_cast(bf16x8, al[abuf][i][s]);
                    acc[i][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vah, vbh, acc[i][b], 0, 0, 0);
                    acc[i][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vah, vbl, acc[i][b], 0, 0, 0);
                    acc[i][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(val, vbh, acc[i][b], 0, 0, 0);
                }
            }
        }
    };

    load_B(0);
    store_B(0);
    load_A(0, 0);
    __syncthreads();
    if constexpr (DBA) {
        // operator fragments of the next slot load while this slot computes
        for (int k = 0; k < na; k += 2) {
            if (k + 1 < na) {
                load_B(k + 1);
                load_A(k + 1, 1);
            }
            compute(0, 0);
            if (k + 1 < na) store_B(1);
            __syncthreads();
            if (k + 1 >= na) break;
            if (k + 2 < na) {
                load_B(k + 2);
                load_A(k + 2, 0);
            }
            compute(1, 1);
            if (k + 2 < na) store_B(0);
            __syncthreads();
        }
    } else {
        for (int k = 0; k < na; k++) {
            if (k > 0) load_A(k, 0);
            if (k + 1 < na) load_B(k + 1);
            compute(k & 1, 0);
            if (k + 1 < na) store_B((k & 1) ^ 1);
            __syncthreads();
        }
    }
#pragma unroll
    for (int b = 0; b < NCB; b++) {
        int col = (wc + CW * b) * 32 + l32;
        if (col >= nrow) continue;
        size_t base = (size_t)rowcell[r0 + col] * KP;
#pragma unroll
        for (int i = 0; i < NRB; i++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                int row = (wr + RW * i) * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                if (row < K) L[base + row] = acc[i][b][r];
            }
    }
}

template <int KP, int NT, int RW, int CW, bool DBA>
void launch(const uint16_t* Thi, const uint16_t* Tlo, const int32_t* offid, const int32_t* gather,
            const uint32_t* rowcell, GemmPlan plan, int K, const float* M, float* L, int ntiles, hipStream_t s) {
    k_m2l_bf16<KP, NT, RW, CW, DBA><<<ntiles, 256, 0, s>>>((const uint4*)Thi, (const uint4*)Tlo, offid, gather, rowcell,
                                                     plan, K, M, L);
}

}  // namespace

void m2l_gemm_bf16(const uint16_t* Thi, const uint16_t* Tlo, const int32_t* offid, const int32_t* gather,
                   const uint32_t* rowcell, GemmPlan plan, int p, int KP, const float* M, float* L, int ntiles,
                   hipStream_t s) {
    if (ntiles <= 0) return;
    int K = ncoef(p);
    switch (KP) {
        case 32: launch<32, 128, 1, 4, true>(Thi, Tlo, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 64: launch<64, 128, 2, 2, true>(Thi, Tlo, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 96: launch<96, 128, 1, 4, false>(Thi, Tlo, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 128: launch<128, 64, 4, 1, true>(Thi, Tlo, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        default: break;
    }
}

bool m2l_bf16_supported(int p) {
    const int kp = kpad(p);
    return kp == 32 || kp == 64 || kp == 96 || kp == 128;
}

}  // namespace fmm
