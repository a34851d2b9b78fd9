// host_ops.h -- FP64 host construction of the translation operators used by
// the kernels (radius-scaled, real layout; see fmm_internal.h).
#pragma once

#include <array>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace fmm {

// Row stride of the coefficient arrays for order p: (p+1)^2 rounded up to a
// multiple of 32, except that 160 and 224 become 192 and 256 so that every
// stride has a matrix-core tiling (see k_m2l_gemm.hip).
inline int kpad_n(int K) {
    int k = ((K + 31) / 32) * 32;
    if (k == 160) return 192;
    if (k == 224) return 256;
    return k;
}
inline int kpad(int p) { return kpad_n((p + 1) * (p + 1)); }
// the same for Cartesian expansions: (p+1)(p+2)(p+3)/6 coefficients
inline int kpad_cart(int p) { return kpad_n((p + 1) * (p + 2) * (p + 3) / 6); }

// Recurrence constants shared by the harmonic kernels (float table):
//   A(n,m) = (2n-1)/sqrt((n-m)(n+m)),  B(n,m) = sqrt((n-m-1)(n+m-1)/((n-m)(n+m)))
//   C1(m) = sqrt((2m-1)/(2m)),          C2(m) = sqrt(2m+1)
constexpr int kRcN = 2 * 16 + 2;                     // highest degree tabulated
constexpr int kRcTri = (kRcN + 1) * (kRcN + 2) / 2;  // entries per triangle
constexpr int kRcA = 0, kRcB = kRcTri, kRcC1 = 2 * kRcTri, kRcC2 = 2 * kRcTri + 40;
constexpr int kRcSize = 2 * kRcTri + 80;

struct HostTables {
    int p = -1, K = 0, KP = 0;
    std::vector<float> m2m;    // [8][K][K], element (oct, k, j) at (oct*K + k)*K + j
    std::vector<float> l2l;    // same layout
    std::vector<float> wm2l;   // [(p+1)(p+2)/2][K]
    std::vector<float> gl2p;   // [2][K]
    std::vector<float> hm2p;   // [2][K]
    std::vector<float> rcoef;  // kRcSize
    std::vector<float> wrot;   // [p+1][p+1][p+1]: axial M2L weights W(j, n, k) of the rotation-based M2L
};

struct M2LPlan {
    int p = -1;
    bool cartesian = false;
    double theta = 0;
    int R = 0;                               // offsets lie in [-R, R]^3
    int J = 0;                               // accepted offsets per octant class
    std::vector<int32_t> slot_of;            // [8][(2R+1)^3] -> slot or -1
    std::vector<int32_t> offid;              // [8][J] -> unique offset index
    std::vector<std::array<int, 3>> offsets; // unique offsets
    std::vector<float> T;                    // [noff][KP][KP], element (o, k, j) at (o*KP + k)*KP + j
};

// Split the same-level operators T ([noff][KP][KP] k-major FP32) into
// BF16 hi = bf16(T) and lo = bf16(T - hi) (round to nearest even), stored
// k-blocked: element (o, k, j) at ((o*KP/8 + k/8)*KP + j)*8 + k%8.
void split_bf16_kblocked(const std::vector<float>& T, size_t noff, int KP, std::vector<uint16_t>& hi,
                         std::vector<uint16_t>& lo);

void build_tables(int p, HostTables& t);
// Cartesian: m2m and l2l only (the other tables stay empty), K = (p+1)(p+2)(p+3)/6
void build_tables_cart(int p, HostTables& t);
// cartesian: operators of the Cartesian family (same offsets and slots)
void build_m2l_plan(int p, double theta, M2LPlan& plan, bool cartesian = false);
// J of build_m2l_plan for theta, counted without building operators
int m2l_plan_slots(double theta);
// the batched same-level GEMM is used up to this many slots per octant class
// (a pair's slot is stored in 16 bits; the gather table holds J entries per target)
constexpr int kGemmMaxSlots = 4096;

// Real-form operator of a general M2L: Ltilde = T Mtilde with source radius
// ratio rs/rt and offset (source centre - target centre) / rt.  Row-major K x K.
void m2l_operator(int p, const double q[3], double ratio, std::vector<double>& out);

}  // namespace fmm
