// cart.h -- Cartesian (Taylor) expansions on the device.
//
// The paper's hybrid method switches from spherical harmonics to Cartesian
// expansions when the required accuracy is low ("Hybrid treecode/FMM
// algorithm"); treecodes use Taylor series in Cartesian coordinates
// ("Introduction to treecodes & FMM").  With multi-indices k = (k1, k2, k3),
// |k| = k1 + k2 + k3 <= p, and x^k = x1^k1 x2^k2 x3^k3:
//   a_n(R) = (1/n!) d^n/dR^n (1/|R|), the Taylor coefficients of 1/|R|:
//            a_0 = 1/|R|,  |R|^2 a_n = -((2|n|-1)/|n|) sum_i R_i a_{n-e_i}
//                                      - ((|n|-1)/|n|) sum_i a_{n-2e_i}
//   multipole about s:  M_k = sum_j q_j (s - x_j)^k
//   local about t:      phi(t + u) = sum_m L_m u^m,
//                       L_m = sum_{|m|+|k|<=p} C(m,k) a_{m+k}(t - s) M_k,
//                       C(m,k) = prod_i (m_i + k_i)! / (m_i! k_i!)
//   M2P:                phi(x) = sum_k a_k(x - s) M_k
// Stored scaled by the cell half side r like the spherical coefficients:
// M~_k = M_k / r^|k|, L~_m = L_m r^(|m|+1); the translation operators are
// then level-independent.  Coefficients are in graded order: degree n =
// 0..p, within a degree k1 descending, then k2 descending.
#pragma once

#include <hip/hip_runtime.h>

namespace fmm {
namespace cart {

__host__ __device__ constexpr int count(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

__host__ __device__ constexpr int index(int a, int b, int c) {
    return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}

// a_n(R) for |n| <= P into a[index(n)] (T = float or double); the recurrence
// runs degree by degree, each degree's entries in stored order
template <int P, class T>
__device__ inline void taylor(T x, T y, T z, T* a) {
    const T r2 = x * x + y * y + z * z;
    const T ir2 = T(1) / r2;
    a[0] = sqrt(ir2);
#pragma unroll
    for (int n = 1; n <= P; n++) {
        const T c1 = T(2 * n - 1) / T(n), c2 = T(n - 1) / T(n);
#pragma unroll
        for (int i = n; i >= 0; i--)
#pragma unroll
            for (int j = n - i; j >= 0; j--) {
                const int k = n - i - j;
                T s1 = T(0), s2 = T(0);
                if (i >= 1) s1 += x * a[index(i - 1, j, k)];
                if (j >= 1) s1 += y * a[index(i, j - 1, k)];
                if (k >= 1) s1 += z * a[index(i, j, k - 1)];
                if (i >= 2) s2 += a[index(i - 2, j, k)];
                if (j >= 2) s2 += a[index(i, j - 2, k)];
                if (k >= 2) s2 += a[index(i, j, k - 2)];
                a[index(i, j, k)] = -(c1 * s1 + c2 * s2) * ir2;
            }
    }
}

// powers x^0 .. x^P
template <int P>
__device__ inline void powers(float x, float* px) {
    px[0] = 1.f;
#pragma unroll
    for (int e = 1; e <= P; e++) px[e] = px[e - 1] * x;
}

}  // namespace cart
}  // namespace fmm
