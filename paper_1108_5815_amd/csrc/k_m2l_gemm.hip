// k_m2l_gemm.hip -- same-level M2L as dense GEMMs on the matrix cores.
//
// For cells of one level, the radius-scaled M2L operator depends only on the
// integer offset o between source and target (in cell sides), not on the
// level.  A target whose parent pair was split has its same-level sources at
// offsets o = 2*O + c_s - c_t, with O a non-accepted parent offset and c the
// octant of each cell in its parent, so each octant class of targets has one
// fixed ordered list of J accepted offsets (189 at theta = 0.5, 567 at
// theta = 0.4).  For a tile of targets of one class,
//     L[:, tile] = sum_j T(o_j) M[:, src(tile, j)]
// is a GEMM whose K dimension runs over (slot j, input coefficient); absent
// sources are zero columns.  Each workgroup owns its tile's outputs, so the
// sum over slots is done in registers, with no atomics, in slot order.
//
// Tiling (gfx950, wave64): a 256-lane workgroup computes KP x 64 outputs with
// v_mfma_f32_32x32x2f32; wave w owns the 32 x 32 blocks w, w+4, ...  Per slot
// the 64 gathered source vectors are staged in LDS (row stride KP+1, conflict
// free column reads) and the operator is read from global memory in k-major
// layout so that each half-wave load is one 128-byte line.
#include "fmm_internal.h"

namespace fmm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int KP>
__global__ __launch_bounds__(256) void k_m2l_gemm(const float* __restrict__ T, const int32_t* __restrict__ offid,
                                                  const int32_t* __restrict__ gather,
                                                  const uint32_t* __restrict__ rowcell, GemmPlan plan, int K,
                                                  const float* __restrict__ M, float* __restrict__ L) {
    constexpr int NT = kGemmTile;
    constexpr int STR = KP + 1;
    constexpr int RB = KP / 32;
    constexpr int NBLK = RB * (NT / 32);
    constexpr int PER = (NBLK + 3) / 4;
    __shared__ float Bs[NT * STR];
    __shared__ int32_t srcs[NT];

    const int tile = blockIdx.x;
    int cls = 0;
    while (cls < 7 && tile >= plan.class_tile0[cls + 1]) cls++;
    const int r0 = plan.class_row0[cls] + (tile - plan.class_tile0[cls]) * NT;
    const int r1 = min(r0 + NT, plan.class_row0[cls + 1]);
    const int nrow = r1 - r0;
    const int J = plan.J;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l32 = lane & 31, khalf = lane >> 5;

    int rbs[PER], cbs[PER];
    bool act[PER];
    floatx16 acc[PER];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        int b = w + 4 * i;
        act[i] = b < NBLK;
        rbs[i] = b % RB;
        cbs[i] = b / RB;
#pragma unroll
        for (int r = 0; r < 16; r++) acc[i][r] = 0.f;
    }
    const int Ke = (K + 1) & ~1;
    for (int j = 0; j < J; j++) {
        if (threadIdx.x < NT)
            srcs[threadIdx.x] = (int)threadIdx.x < nrow ? gather[(size_t)(r0 + threadIdx.x) * J + j] : -1;
        __syncthreads();
        for (int idx = threadIdx.x; idx < NT * (KP / 4); idx += 256) {
            int col = idx / (KP / 4), k4 = idx - col * (KP / 4);
            int s = srcs[col];
            float4 v = s >= 0 ? reinterpret_cast<const float4*>(M + (size_t)s * KP)[k4] : make_float4(0.f, 0.f, 0.f, 0.f);
            float* d = Bs + col * STR + 4 * k4;
            d[0] = v.x;
            d[1] = v.y;
            d[2] = v.z;
            d[3] = v.w;
        }
        __syncthreads();
        const float* A = T + (size_t)offid[cls * J + j] * KP * KP;
        for (int k0 = 0; k0 < Ke; k0 += 2) {
            const int kk = k0 + khalf;
#pragma unroll
            for (int i = 0; i < PER; i++) {
                if (!act[i]) continue;
                float a = A[(size_t)kk * KP + rbs[i] * 32 + l32];
                float bv = Bs[(cbs[i] * 32 + l32) * STR + kk];
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc[i], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < PER; i++) {
        if (!act[i]) continue;
        int col = cbs[i] * 32 + l32;
        if (col >= nrow) continue;
        size_t base = (size_t)rowcell[r0 + col] * KP;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            int row = rbs[i] * 32 + 8 * (r >> 2) + 4 * khalf + (r & 3);
            if (row < K) L[base + row] = acc[i][r];
        }
    }
}

template <int KP>
void launch(const float* T, const int32_t* offid, const int32_t* gather, const uint32_t* rowcell, GemmPlan plan,
            int K, const float* M, float* L, int ntiles, hipStream_t s) {
    k_m2l_gemm<KP><<<ntiles, 256, 0, s>>>(T, offid, gather, rowcell, plan, K, M, L);
}

}  // namespace

bool m2l_gemm_supported(int p) { return kpad(p) <= 224; }

void m2l_gemm(const float* T, const int32_t* offid, const int32_t* gather, const uint32_t* rowcell, GemmPlan plan,
              int p, int KP, const float* M, float* L, int ntiles, int precision, hipStream_t s) {
    (void)precision;
    if (ntiles <= 0) return;
    int K = ncoef(p);
    switch (KP) {
        case 32: launch<32>(T, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 64: launch<64>(T, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 96: launch<96>(T, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 128: launch<128>(T, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 160: launch<160>(T, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 192: launch<192>(T, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        case 224: launch<224>(T, offid, gather, rowcell, plan, K, M, L, ntiles, s); break;
        default: break;
    }
}

}  // namespace fmm
