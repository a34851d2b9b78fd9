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
// Slot groups (XCD-aware): the operators of one class take J x 64 KB at
// storage width 128 (36 MB at theta = 0.4), far more than one XCD's 4 MB L2,
// and tiles that run at the same time drift apart in slot, so streaming every
// slot through every tile makes each operator block an L2 miss.  Instead the
// slots are cut into G fixed ranges (G a multiple of 8) and work item (tile,
// group g) runs on XCD g mod 8 (workgroups are dealt to the 8 XCDs round
// robin by block index): each XCD then touches only its own slice of the
// operators, which stays in its L2.  Each item writes its partial locals to
// part[g][row]; m2l_reduce_groups sums the groups in order.  A row's result
// therefore depends only on its own sources, whatever rows share its tile.
//
// Tiling (gfx950, wave64, v_mfma_f32_32x32x2f32): a workgroup owns KP x NT
// outputs split over a RW x CW grid of waves; each wave keeps
// NRB x NCB 32x32 accumulator blocks.  The K index of step s, half h of the
// wave, is h*KS + s, so each lane reads its source vector contiguously
// (float4 LDS reads cover 4 steps).  Operator fragments stream from global
// memory (k-major, one 128-byte line per half-wave) through a register
// pipeline one chunk (CH steps) ahead; the next slot's 64 or 128 gathered source
// vectors are loaded into registers during the current slot and written to
// the other half of a double-buffered LDS tile.  At storage width 96 the
// 3 x 4 wave grid gives each wave one accumulator block: every operator row
// block is read by the 4 waves of its row (L1 hits after the first), and 12
// waves per CU hide the load latency that one wave per SIMD could not.
#include <algorithm>
#include <type_traits>

#include "fmm_internal.h"

namespace fmm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
// 16 bytes as a native vector (copies stay in registers; HIP's float4 struct
// copies can be lowered through private memory)
typedef float f32x4 __attribute__((ext_vector_type(4)));

// first index k in [0, n) with act[k] >= j (act ascending), or n
__device__ inline int lower_slot(const int32_t* act, int n, int j) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (act[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// work item of block b: b = (h * ntiles + tile) * 8 + x, group g = x + 8 h
__device__ inline void gemm_item(const GemmPlan& plan, int& tile, int& g) {
    const unsigned b = blockIdx.x;
    const unsigned rest = b >> 3;
    tile = (int)(rest % (unsigned)plan.ntiles);
    g = (int)(b & 7u) + 8 * (int)(rest / (unsigned)plan.ntiles);
}

template <int KP, int NT, int RW, int CW, int CH>
__global__ __launch_bounds__(64 * RW * CW) void k_m2l_gemm(const float* __restrict__ T, const int32_t* __restrict__ offid,
                                                  const int32_t* __restrict__ gather, GemmPlan plan,
                                                  const float* __restrict__ M, float* __restrict__ part) {
    constexpr int KS = KP / 2;
    constexpr int RB = KP / 32, CB = NT / 32;
    constexpr int NTH = 64 * RW * CW;   // lanes of the workgroup
    static_assert(RB % RW == 0 && CB % CW == 0, "wave grid");
    constexpr int NRB = RB / RW, NCB = CB / CW;
    constexpr int STR = KP + 4;
    constexpr int NCH = KS / CH;        // operator chunks (CH steps each) per slot
    constexpr int BV = NT * KP / (4 * NTH);  // float4 per thread per source tile
    static_assert(KS % CH == 0 && CH % 4 == 0 && (NT * KP) % (4 * NTH) == 0, "tile shape");
    __shared__ __attribute__((aligned(16))) float Bs[2][NT * STR];
    __shared__ int32_t s_slot[kGemmMaxGroupSlots], s_op[kGemmMaxGroupSlots];

    int tile, g;
    gemm_item(plan, tile, g);
    int cls = 0;
    while (cls < 7 && tile >= plan.class_tile0[cls + 1]) cls++;
    const int r0 = plan.class_row0[cls] + (tile - plan.class_tile0[cls]) * NT;
    const int nrow = min(NT, plan.class_row0[cls + 1] - r0);
    const int J = plan.J;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l32 = lane & 31, h = lane >> 5;
    const int wr = w % RW, wc = w / RW;
    // this group's slots [g J / G, (g + 1) J / G), restricted to those some row
    // of the tile uses: fixed slot ranges make each row's partial independent
    // of the other rows of its tile
    const int32_t* act = plan.act + (size_t)tile * J;
    const int na = plan.nact[tile];
    const int k0 = lower_slot(act, na, (int)(((int64_t)g * J) / plan.G));
    const int n = lower_slot(act, na, (int)(((int64_t)(g + 1) * J) / plan.G)) - k0;
    // the group's slots and their operators, staged once (n <= J / G + 1)
    for (int i = threadIdx.x; i < n; i += NTH) {
        const int j = act[k0 + i];
        s_slot[i] = j;
        s_op[i] = offid[(size_t)cls * J + j];
    }
    __syncthreads();

    floatx16 acc[NRB][NCB];
#pragma unroll
    for (int i = 0; i < NRB; i++)
#pragma unroll
        for (int b = 0; b < NCB; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[i][b][r] = 0.f;

    // Every load below is issued on every path, with the slot index clamped
    // to the group's last slot where the pipeline runs past it: loads
    // complete in issue order, and a load count that depends on the path
    // would force the wait for one operator chunk to drain every later load.
    f32x4 breg[BV];
    // gathered sources: the tile's source indices of a slot are contiguous
    // (gather[tile][slot][NT], padding columns -1) and are loaded one slot
    // before the data; the data loads read the zero row for absent sources
    int sidx[BV];
    auto load_idx = [&](int i) {
        const int32_t* gk = gather + ((size_t)tile * J + s_slot[min(i, n - 1)]) * NT;
#pragma unroll
        for (int v = 0; v < BV; v++) sidx[v] = gk[(threadIdx.x + NTH * v) / (KP / 4)];
    };
    auto load_data = [&]() {
#pragma unroll
        for (int v = 0; v < BV; v++) {
            const int idx = threadIdx.x + NTH * v;
            const int col = idx / (KP / 4), k4 = idx - col * (KP / 4);
            const int s = sidx[v] >= 0 ? sidx[v] : plan.zcell;
            breg[v] = reinterpret_cast<const f32x4*>(M + (size_t)s * KP)[k4];
        }
    };
    auto store_B = [&](int buf) {
#pragma unroll
        for (int v = 0; v < BV; v++) {
            int idx = threadIdx.x + NTH * v;
            int col = idx / (KP / 4), k4 = idx - col * (KP / 4);
            *reinterpret_cast<f32x4*>(&Bs[buf][col * STR + 4 * k4]) = breg[v];
        }
    };
    float ab[2][NRB][CH];
    auto load_A = [&](int op, int c, int buf) {
        const float* A = T + (size_t)op * KP * KP;
#pragma unroll
        for (int r = 0; r < NRB; r++)
#pragma unroll
            for (int t = 0; t < CH; t++)
                ab[buf][r][t] = A[(size_t)(h * KS + c * CH + t) * KP + (wr + RW * r) * 32 + l32];
    };
    auto compute = [&](int buf, int c, int abuf) {
#pragma unroll
        for (int t = 0; t < CH; t += 4) {
            f32x4 b4[NCB];
#pragma unroll
            for (int b = 0; b < NCB; b++) {
                int col = (wc + CW * b) * 32 + l32;
                b4[b] = *reinterpret_cast<const f32x4*>(&Bs[buf][col * STR + h * KS + c * CH + t]);
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int b = 0; b < NCB; b++) {
                    float bv = b4[b][u];
#pragma unroll
                    for (int i = 0; i < NRB; i++)
                        acc[i][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ab[abuf][i][t + u], bv, acc[i][b], 0,
                                                                         0, 0);
                }
        }
    };

    // slot i of the group; P0 = register buffer of its first chunk (buffers
    // alternate by chunk, so with an odd number of chunks the slots alternate
    // too).  The next slot's gathers (the slowest loads) are issued after
    // this slot's second operator chunk, so waiting for that chunk does not
    // wait for them; they are needed only at the slot's end.
    auto slot = [&](int i, auto P0) {
        constexpr int p0 = decltype(P0)::value;
        const int buf = i & 1;
        const int op = s_op[i], op_next = s_op[min(i + 1, n - 1)];
#pragma unroll
        for (int c = 0; c < NCH; c++) {
            if (c + 1 < NCH) load_A(op, c + 1, (p0 + c + 1) & 1);
            else load_A(op_next, 0, (p0 + c + 1) & 1);
            if (c == 0) {
                load_data();      // slot i + 1 (indices loaded during slot i - 1)
                load_idx(i + 2);
            }
            // keep the loads ahead of this chunk's products (the scheduler
            // would otherwise sink each load next to its first use)
            __builtin_amdgcn_sched_barrier(0);
            compute(buf, c, (p0 + c) & 1);
            __builtin_amdgcn_sched_barrier(0);
        }
        store_B(buf ^ 1);         // past the last slot: a copy nobody reads
        __syncthreads();
    };
    if (n > 0) {
        load_idx(0);
        load_data();
        store_B(0);
        load_idx(1);
        load_A(s_op[0], 0, 0);
        __syncthreads();
        if constexpr (NCH % 2 == 0) {
            for (int i = 0; i < n; i++) slot(i, std::integral_constant<int, 0>{});
        } else {
            for (int i = 0; i < n; i += 2) {
                slot(i, std::integral_constant<int, 0>{});
                if (i + 1 < n) slot(i + 1, std::integral_constant<int, 1>{});
            }
        }
    }
    // partial locals of this group (zero when it has no slots)
#pragma unroll
    for (int b = 0; b < NCB; b++) {
        int col = (wc + CW * b) * 32 + l32;
        if (col >= nrow) continue;
        float* dst = part + ((size_t)g * plan.nrows + r0 + col) * KP;
#pragma unroll
        for (int i = 0; i < NRB; i++)
#pragma unroll
            for (int r = 0; r < 16; r++) dst[(wr + RW * i) * 32 + 8 * (r >> 2) + 4 * h + (r & 3)] = acc[i][b][r];
    }
}

// L[rowcell[r]][k] = sum_g part[g][r][k] for k < K, groups in order
__global__ void k_reduce_groups(const float4* __restrict__ part, int G, int nrows, int KP4, int K,
                                const uint32_t* __restrict__ rowcell, float* __restrict__ L) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nrows * KP4) return;
    const int64_t r = i / KP4;
    const int k4 = (int)(i - r * KP4);
    float4 s = part[i];
    for (int g = 1; g < G; g++) {
        const float4 v = part[(int64_t)g * nrows * KP4 + i];
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
    }
    float* dst = L + (size_t)rowcell[r] * KP4 * 4 + 4 * k4;
    const float vals[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
    for (int e = 0; e < 4; e++)
        if (4 * k4 + e < K) dst[e] = vals[e];
}

template <int KP, int NT, int RW, int CW, int CH>
void launch(const float* T, const int32_t* offid, const int32_t* gather, GemmPlan plan, const float* M, float* part,
            hipStream_t s) {
    k_m2l_gemm<KP, NT, RW, CW, CH><<<plan.ntiles * plan.G, 64 * RW * CW, 0, s>>>(T, offid, gather, plan, M, part);
}

}  // namespace

bool m2l_gemm_supported(int p) { return gemm_tile_cols(p) > 0; }
bool m2l_gemm_supported_kp(int KP) { return gemm_tile_cols_kp(KP) > 0; }

// targets per tile for the storage width of order p (0 = no GEMM path)
int gemm_tile_cols(int p) { return gemm_tile_cols_kp(kpad(p)); }

int gemm_tile_cols_kp(int KP) {
    switch (KP) {
        case 32: case 64: case 96: return 128;
        case 128: case 192: case 256: return 64;
        default: return 0;
    }
}

bool gemm_tile_width_ok(int KP, int nt) {
    if (KP == 128) return nt == 64 || nt == 128;
    return nt > 0 && nt == gemm_tile_cols_kp(KP);
}

int gemm_slot_groups(int J) { return 8 * std::max(1, (J + 631) / 632); }

void m2l_reduce_groups(const float* part, GemmPlan plan, const uint32_t* rowcell, int KP, int K, float* L,
                       hipStream_t s) {
    const int64_t n = (int64_t)plan.nrows * (KP / 4);
    if (n <= 0) return;
    k_reduce_groups<<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const float4*)part, plan.G, plan.nrows, KP / 4, K,
                                                               rowcell, L);
}

void m2l_gemm(const float* T, const int32_t* offid, const int32_t* gather, const uint32_t* rowcell, GemmPlan plan,
              int K, int KP, const float* M, float* part, float* L, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (plan.ntiles <= 0) return;
    if (e0) (void)hipEventRecord(e0, s);
    switch (KP) {
        case 32: launch<32, 128, 1, 4, 16>(T, offid, gather, plan, M, part, s); break;
        case 64: launch<64, 128, 2, 2, 16>(T, offid, gather, plan, M, part, s); break;
        case 96: launch<96, 128, 3, 4, 8>(T, offid, gather, plan, M, part, s); break;
        case 128:
            if (plan.nt == 128) launch<128, 128, 4, 1, 8>(T, offid, gather, plan, M, part, s);
            else launch<128, 64, 4, 1, 8>(T, offid, gather, plan, M, part, s);
            break;
        case 192: launch<192, 64, 2, 2, 8>(T, offid, gather, plan, M, part, s); break;
        case 256: launch<256, 64, 4, 1, 8>(T, offid, gather, plan, M, part, s); break;
        default: return;
    }
    if (e1) (void)hipEventRecord(e1, s);
    m2l_reduce_groups(part, plan, rowcell, KP, K, L, s);
}

}  // namespace fmm
