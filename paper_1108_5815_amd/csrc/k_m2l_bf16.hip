// k_m2l_bf16.hip -- same-level M2L GEMMs in split-BF16 on the matrix cores.
//
// The batching is that of k_m2l_gemm.hip (one octant class and a tile of
// targets per workgroup, K running over (slot, coefficient); the slots of a
// tile cut into XCD-local groups whose partials are summed in group order).  Here every
// FP32 operand a is split into a_hi = bf16(a) and a_lo = bf16(a - a_hi)
// (round to nearest even), and each product is formed from three BF16
// products on v_mfma_f32_32x32x16_bf16 with FP32 accumulation:
//     a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// The dropped a_lo b_lo term and the residual of the two-term split bound
// the relative error of each product by about 2^-16.  The precision is
// graded by multipole degree: coefficients k >= 32 (degrees 5 and up) drop
// a_lo b_hi (two products, error 2^-9 of the product), and k >= 48 (degrees 6
// and up) keep a_hi b_hi alone (about 2^-8).  Summed over the local degrees, a
// degree-n multipole term is of order x^n / (1 - x)^(n + 1) of the pair's
// leading term, x the ratio of cell size to distance (about theta / 2 for the
// pairs of these tables), the same decay that makes the expansion converge,
// so the coarser products carry only a small share of the result.  The operators are split
// once on the host and stored k-blocked ([offset][KP/8][KP][8] bf16) so that
// a lane's 8 consecutive K values for its row are one 16-byte load.  The
// multipoles are split once per evaluation (k_split_cells: per cell the KP/8
// hi blocks of 8 bf16 and the lo blocks that products read), so staging a
// gathered source row into LDS is a plain copy.
#include <algorithm>
#include <type_traits>

#include "fmm_internal.h"

namespace fmm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// 16 bytes as a native vector (copies stay in registers; HIP's uint4 struct
// copies can be lowered through private memory)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ inline uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

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

// RS: 16-byte blocks per split multipole row (KP / 8 hi blocks, then the lo
// blocks of the first kBf16LoBlocks * 8 coefficients, the only low parts a
// product reads, then padding so that the workgroup's threads share a source
// row set evenly).
// Waves: RW row blocks x CW column blocks x KSP parts of K.  With KSP = 2 two
// waves share each (row block, column block), each summing the products of
// one half of K, and the halves are added once at the tile's end: a wave
// holds half the operator fragments and accumulators, so at storage width 128
// tiles of 64 targets run four waves per SIMD (two workgroups of eight per
// CU), and tiles of 128 load each operator fragment once per workgroup.  A
// row's sums, and their order, are the same at both widths.
template <int KP, int NT, int RW, int CW, int NQ, int KSP, int RS>
__global__ __launch_bounds__(64 * RW * CW * KSP) void k_m2l_bf16(const uint4* __restrict__ Thi, const uint4* __restrict__ Tlo,
                                                  const int32_t* __restrict__ offid,
                                                  const int32_t* __restrict__ gather, GemmPlan plan,
                                                  const uint4* __restrict__ Ms, float* __restrict__ part) {
    constexpr int KB = KP / 8;          // 8-wide K blocks
    constexpr int KS = KP / 16;         // MFMA K steps (16 values each)
    constexpr int KSW = KS / KSP;       // K steps of one wave
    constexpr int RB = KP / 32, CB = NT / 32;
    constexpr int NTH = 64 * RW * CW * KSP;  // lanes of the workgroup
    static_assert(RB % RW == 0 && CB % CW == 0 && KS % KSP == 0, "wave grid");
    constexpr int NRB = RB / RW, NCB = CB / CW;
    constexpr int LB = kBf16LoBlocks < KB ? kBf16LoBlocks : KB;  // lo blocks a product reads
    constexpr int STR = KB + 1;         // LDS row stride of the hi tile, 16-byte units
    constexpr int STRL = LB + 1;        // and of the lo tile
    constexpr int HL = NT * STR;        // the hi tile
    constexpr int HLL = NT * STRL;      // the lo tile
    constexpr int BV = NT * RS / NTH;   // 16-byte blocks per thread per source row set
    static_assert(RS >= KB + LB && (NT * RS) % NTH == 0, "tile shape");
    __shared__ u32x4 Bs[2][HL + HLL];   // [buffer][hi tile, lo tile]
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
    const int wr = w % RW, wc = (w / RW) % CW, wk = w / (RW * CW);
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
    // would force the wait for one operator part to drain every later load.
    u32x4 breg[BV];
    // gathered sources: the tile's source indices of a slot are contiguous
    // (gather[tile][slot][NT], padding columns -1) and are loaded one slot
    // before the data; the data loads read the zero row for absent sources
    int sidx[BV];
    auto load_idx = [&](int i) {
        const int32_t* gk = gather + ((size_t)tile * J + s_slot[min(i, n - 1)]) * NT;
#pragma unroll
        for (int v = 0; v < BV; v++) sidx[v] = gk[(threadIdx.x + NTH * v) / RS];
    };
    auto load_data = [&]() {
#pragma unroll
        for (int v = 0; v < BV; v++) {
            const int idx = threadIdx.x + NTH * v;
            const int col = idx / RS, rem = idx - col * RS;
            const int s = sidx[v] >= 0 ? sidx[v] : plan.zcell;
            breg[v] = reinterpret_cast<const u32x4*>(Ms)[(size_t)s * RS + rem];
        }
    };
    auto store_B = [&](int buf) {
#pragma unroll
        for (int v = 0; v < BV; v++) {
            const int idx = threadIdx.x + NTH * v;
            const int col = idx / RS, rem = idx - col * RS;
            if (rem < KB) Bs[buf][col * STR + rem] = breg[v];
            else if (rem < KB + LB) Bs[buf][HL + col * STRL + rem - KB] = breg[v];
        }
    };
    // operator fragments stream through two register buffers in NQ parts of a
    // slot (SC steps each): the next part (of this slot, or the first part of
    // the next slot) loads while the current part computes, so operator loads
    // run one part ahead.  Step s, half h of the wave -> K block 2s + h.
    constexpr int SC = KSW / NQ;
    static_assert(KSW % NQ == 0, "slot parts");
    u32x4 ah[2][NRB][SC], al[2][NRB][SC];

    // The wave's loop, compiled once per half of K so that every step's
    // product set is fixed at compile time (WK: the wave's half).
    auto run = [&](auto WKc) {
        constexpr int WK = decltype(WKc)::value;
        auto load_A = [&](int op, int half, int buf) {
            const size_t base = (size_t)op * KB * KP;
#pragma unroll
            for (int r = 0; r < NRB; r++)
#pragma unroll
                for (int s = 0; s < SC; s++) {
                    const int st = WK * KSW + half * SC + s;
                    const size_t ix = base + (size_t)(2 * st + h) * KP + (wr + RW * r) * 32 + l32;
                    ah[buf][r][s] = reinterpret_cast<const u32x4*>(Thi)[ix];
                    if (st < kBf16FullSteps) al[buf][r][s] = reinterpret_cast<const u32x4*>(Tlo)[ix];
                }
        };
        auto compute = [&](int bbuf, int half, int abuf) {
#pragma unroll
            for (int s = 0; s < SC; s++) {
                const int st = WK * KSW + half * SC + s;
#pragma unroll
                for (int b = 0; b < NCB; b++) {
                    const int col = (wc + CW * b) * 32 + l32;
                    const u32x4 bh = Bs[bbuf][col * STR + 2 * st + h];
                    const bf16x8 vbh = __builtin_bit_cast(bf16x8, bh);
                    bf16x8 vbl{};
                    if (st < kBf16TwoSteps) vbl = __builtin_bit_cast(bf16x8, Bs[bbuf][HL + col * STRL + 2 * st + h]);
#pragma unroll
                    for (int i = 0; i < NRB; i++) {
                        const bf16x8 vah = __builtin_bit_cast(bf16x8, ah[abuf][i][s]);
                        acc[i][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vah, vbh, acc[i][b], 0, 0, 0);
                        if (st < kBf16TwoSteps)
                            acc[i][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vah, vbl, acc[i][b], 0, 0, 0);
                        if (st < kBf16FullSteps) {
                            const bf16x8 val = __builtin_bit_cast(bf16x8, al[abuf][i][s]);
                            acc[i][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(val, vbh, acc[i][b], 0, 0, 0);
                        }
                    }
                }
            }
        };

        // slot i of the group; P0 = register buffer of its first part (buffers
        // alternate by part, so with an odd number of parts the slots alternate
        // too).  The next slot's gathers (the slowest loads) are issued after
        // this slot's second operator part, so waiting for that part does not
        // wait for them; they are needed only at the slot's end.
        auto slot = [&](int i, auto P0) {
            constexpr int p0 = decltype(P0)::value;
            const int bb = i & 1;
            const int op = s_op[i], op_next = s_op[min(i + 1, n - 1)];
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                if (q + 1 < NQ) load_A(op, q + 1, (p0 + q + 1) & 1);
                else load_A(op_next, 0, (p0 + q + 1) & 1);
                if (q == 0) {
                    load_data();      // slot i + 1 (indices loaded during slot i - 1)
                    load_idx(i + 2);
                }
                // keep the loads ahead of this part's products (the scheduler
                // would otherwise sink each load next to its first use); a wave
                // issuing products is favoured over waves issuing loads (about 1%
                // on the 4M-point Plummer lists)
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(1);
                compute(bb, q, (p0 + q) & 1);
                __builtin_amdgcn_s_setprio(0);
                __builtin_amdgcn_sched_barrier(0);
            }
            store_B(bb ^ 1);          // past the last slot: a copy nobody reads
            __syncthreads();
        };
        if (n > 0) {
            load_idx(0);
            load_data();
            store_B(0);
            load_idx(1);
            load_A(s_op[0], 0, 0);
            __syncthreads();
            if constexpr (NQ % 2 == 0) {
                for (int i = 0; i < n; i++) slot(i, std::integral_constant<int, 0>{});
            } else {
                for (int i = 0; i < n; i += 2) {
                    slot(i, std::integral_constant<int, 0>{});
                    if (i + 1 < n) slot(i + 1, std::integral_constant<int, 1>{});
                }
            }
        }
    };
    if constexpr (KSP == 2) {
        if (wk == 0) run(std::integral_constant<int, 0>{});
        else run(std::integral_constant<int, 1>{});
    } else {
        run(std::integral_constant<int, 0>{});
    }
    if constexpr (KSP == 2) {
        // the second half of K adds its sums to the first's through the LDS
        // tile (every wave is past the slot loop's last barrier)
        static_assert(RW * CW * NRB * NCB * 16 * 64 * 4 <= (int)sizeof(Bs), "K reduction fits the tile");
        float* red = reinterpret_cast<float*>(&Bs[0][0]);
        const int wi = wr + RW * wc;
        if (wk == 1) {
#pragma unroll
            for (int i = 0; i < NRB; i++)
#pragma unroll
                for (int b = 0; b < NCB; b++)
#pragma unroll
                    for (int r = 0; r < 16; r++) red[(((wi * NRB + i) * NCB + b) * 16 + r) * 64 + lane] = acc[i][b][r];
        }
        __syncthreads();
        if (wk == 1) return;
#pragma unroll
        for (int i = 0; i < NRB; i++)
#pragma unroll
            for (int b = 0; b < NCB; b++)
#pragma unroll
                for (int r = 0; r < 16; r++) acc[i][b][r] += red[(((wi * NRB + i) * NCB + b) * 16 + r) * 64 + lane];
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

template <int KP, int NT, int RW, int CW, int NQ, int KSP, int RS>
void launch(const uint16_t* Thi, const uint16_t* Tlo, const int32_t* offid, const int32_t* gather, GemmPlan plan,
            const uint4* Ms, float* part, hipStream_t s) {
    k_m2l_bf16<KP, NT, RW, CW, NQ, KSP, RS><<<plan.ntiles * plan.G, 64 * RW * CW * KSP, 0, s>>>(
        (const uint4*)Thi, (const uint4*)Tlo, offid, gather, plan, Ms, part);
}

// Multipoles of every cell split into bf16 hi and lo (round to nearest even):
// Ms[cell][kb] = hi of coefficients 8 kb .. 8 kb + 7 (kb < KB), then
// Ms[cell][KB + kb] = lo of the same for kb < LB, then zero blocks up to RS
// per row.
__global__ void k_split_cells(const float4* __restrict__ M, int64_t ncell, int KB, int LB, int RS,
                              uint4* __restrict__ Ms) {
    // ncell rows including the trailing zero row
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncell * KB) return;
    const int64_t c = i / KB;
    const int kb = (int)(i - c * KB);
    const float4 a = M[2 * i], b = M[2 * i + 1];
    const float x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint16_t hi[8], lo[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
        hi[e] = bf16_rne(x[e]);
        lo[e] = bf16_rne(x[e] - bf16_to_f(hi[e]));
    }
    auto pack = [](const uint16_t* v) {
        return make_uint4((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                          (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16));
    };
    uint4* row = Ms + c * RS;
    row[kb] = pack(hi);
    if (kb < LB) row[KB + kb] = pack(lo);
    if (kb < RS - KB - LB) row[KB + LB + kb] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

// 16-byte blocks per split multipole row, by storage width (the RS of the
// launches below): KP / 8 hi blocks and min(kBf16LoBlocks, KP / 8) lo blocks,
// padded so that every workgroup shape divides a tile's rows evenly
int split_row_blocks(int KP) {
    switch (KP) {
        case 32: return 8;
        case 64: return 14;
        case 96: return 18;
        case 128: return 24;
        case 192: return 36;
        default: return 0;
    }
}

void m2l_gemm_bf16(const uint16_t* Thi, const uint16_t* Tlo, const int32_t* offid, const int32_t* gather,
                   const uint32_t* rowcell, GemmPlan plan, int K, int KP, const float* M, int64_t ncell, uint4* Ms,
                   float* part, float* L, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (plan.ntiles <= 0) return;
    const int KB = KP / 8;
    const int LB = std::min(kBf16LoBlocks, KB);
    const int RS = split_row_blocks(KP);
    if (RS <= 0) return;
    const int64_t nb = (ncell + 1) * KB;  // with the zero row
    k_split_cells<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>((const float4*)M, ncell + 1, KB, LB, RS, Ms);
    if (e0) (void)hipEventRecord(e0, s);
    switch (KP) {
        case 32: launch<32, 128, 1, 4, 2, 1, 8>(Thi, Tlo, offid, gather, plan, Ms, part, s); break;
        case 64: launch<64, 128, 2, 2, 2, 1, 14>(Thi, Tlo, offid, gather, plan, Ms, part, s); break;
        case 96: launch<96, 128, 3, 2, 3, 2, 18>(Thi, Tlo, offid, gather, plan, Ms, part, s); break;
        case 128:
            if (plan.nt == 128) launch<128, 128, 4, 1, 2, 2, 24>(Thi, Tlo, offid, gather, plan, Ms, part, s);
            else launch<128, 64, 4, 1, 2, 2, 24>(Thi, Tlo, offid, gather, plan, Ms, part, s);
            break;
        case 192: launch<192, 64, 6, 1, 3, 2, 36>(Thi, Tlo, offid, gather, plan, Ms, part, s); break;
        default: return;
    }
    if (e1) (void)hipEventRecord(e1, s);
    m2l_reduce_groups(part, plan, rowcell, KP, K, L, s);
}

bool m2l_bf16_supported(int p) { return m2l_bf16_supported_kp(kpad(p)); }

bool m2l_bf16_supported_kp(int kp) { return kp == 32 || kp == 64 || kp == 96 || kp == 128 || kp == 192; }

}  // namespace fmm
