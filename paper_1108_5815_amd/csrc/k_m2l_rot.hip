// k_m2l_rot.hip -- rotation-based M2L of single cell pairs (spherical
// harmonics), O(p^3) per pair.
//
// The paper lets the traversal choose, per accepted pair, between kinds of
// translation (rotation-based or plane-wave, "Dual tree traversal"), and
// notes that fast translations cost p^4 or less instead of p^6
// ("Introduction to treecodes & FMM").  Here the multipole is rotated into
// the frame whose z axis points from the target centre to the source centre,
// translated along that axis, where the operator only couples equal orders
// m, and the local expansion is rotated back:
//   1. azimuth: c_m = e^{i m beta} M_n^m  (beta = azimuth of the offset q)
//   2. polar:   M'_n^{m'} = sum_m (eps_m / eps_m') d^n_{m'm}(-alpha) c_m
//      with eps_m = (-1)^m for m >= 0 and 1 for m < 0 (the harmonics here
//      lack the Condon-Shortley phase and are not normalised), and d^n the
//      Wigner small-d matrix, from Jacobi polynomials:
//      d^n_{m'm}(t) = sqrt((n+m)!(n-m)! / ((n+m')!(n-m')!))
//                     sin(t/2)^(m-m') cos(t/2)^(m+m') P_{n-m}^{(m-m', m+m')}(cos t)
//      for m >= |m'|, the other entries by d_{m'm} = (-1)^(m-m') d_{mm'}
//      = d_{-m,-m'};
//   3. axial:   L'_j^k = sum_n W(j,n,k) u^n v^(j+1) M'_n^k, u = rs/rho,
//      v = rt/rho (the scaled expansions), W from Greengard & Rokhlin's
//      theorem 3.4 at a polar angle of zero;
//   4. back:    L_j^m = e^{-i m beta} sum_m' (eps_m' / eps_m) d^j_{m'm}(-alpha) L'_j^m'.
// One workgroup per target cell, one pair per wave at a time; the Wigner
// matrices of a pair are built in the wave's LDS; each wave's partial
// locals are added in wave order (deterministic).
#include "fmm_internal.h"

namespace fmm {
namespace {

__device__ inline int idx_re(int n, int m) { return m == 0 ? n * n : n * n + 2 * m - 1; }
__device__ inline int dofs(int n) { return n * (4 * n * n - 1) / 3; }  // sum_{i<n} (2i+1)^2
__device__ inline float eps_of(int m) { return (m >= 0 && (m & 1)) ? -1.f : 1.f; }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS floats per wave for order p
__host__ __device__ inline int rot_wave_floats(int p, int KP) {
    const int nd = (p + 1) * (2 * p + 1) * (2 * p + 3) / 3;  // Wigner matrices of degrees 0..p
    const int njk = (p + 1) * (p + 2) / 2;
    return KP + nd + 2 * (p + 1) + 4 * njk;
}

__global__ __launch_bounds__(256) void k_m2l_rot(const int32_t* __restrict__ goff, const uint32_t* __restrict__ gsrc,
                                                 CellArrays c, int p, int KP, const float* __restrict__ Wax,
                                                 const float* __restrict__ M, float* __restrict__ L,
                                                 const uint8_t* __restrict__ skip, int nwaves) {
    extern __shared__ float sh[];
    const int t = blockIdx.x;
    const int32_t a0 = goff[t], a1 = goff[t + 1];
    if (a0 == a1) return;
    const int njk = (p + 1) * (p + 2) / 2;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int per = rot_wave_floats(p, KP);
    float* Ms = sh + w * per;               // source multipole (real layout)
    float* D = Ms + KP;                     // Wigner d^n, (2n+1)^2 each, [m'][m]
    float* em = D + (p + 1) * (2 * p + 1) * (2 * p + 3) / 3;  // e^{i m beta}, m = 0..p
    float* Mr = em + 2 * (p + 1);           // rotated multipole, complex, (n, m' >= 0)
    float* Lr = Mr + 2 * njk;               // axial local, complex, (j, k >= 0)
    float* red = sh + nwaves * per;         // per-wave partial locals
    float are[3] = {0.f, 0.f, 0.f}, aim[3] = {0.f, 0.f, 0.f};
    int oj[3], ok[3];
#pragma unroll
    for (int u = 0; u < 3; u++) {
        const int jk = lane + 64 * u;
        int j = 0;
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
    for (int32_t a = a0 + w; a < a1; a += nwaves) {
        if (skip && skip[a]) continue;  // handled by the class-batched products
        const int s = (int)gsrc[a];
        const int4 gs = c.geo[s];
        // offset source - target in half-grid units (exact integers)
        const float dx = (float)((int64_t)gs.x - gt.x), dy = (float)((int64_t)gs.y - gt.y),
                    dz = (float)((int64_t)gs.z - gt.z);
        const float rho = sqrtf(dx * dx + dy * dy + dz * dz);
        const float u = (float)gs.w / rho, v = (float)gt.w / rho;
        const float ca = dz / rho;                    // cos alpha
        const float rxy = sqrtf(dx * dx + dy * dy);
        const float cb = rxy > 0.f ? dx / rxy : 1.f, sb = rxy > 0.f ? dy / rxy : 0.f;
        // d(t) at t = -alpha: cos t = cos alpha, sin(t/2) = -sin(alpha/2)
        const float xh = ca;
        const float sh2 = -sqrtf(fmaxf(0.f, 0.5f * (1.f - ca))), ch2 = sqrtf(fmaxf(0.f, 0.5f * (1.f + ca)));
        for (int i = lane; i < KP; i += 64) Ms[i] = M[(size_t)s * KP + i];
        if (lane == 0) {
            float cr = 1.f, ci = 0.f;
            for (int m = 0; m <= p; m++) {
                em[2 * m] = cr;
                em[2 * m + 1] = ci;
                const float nr = cr * cb - ci * sb, ni = cr * sb + ci * cb;
                cr = nr;
                ci = ni;
            }
        }
        // Wigner d: the entries with m >= |m'| by Jacobi recurrences in the degree
        for (int e = lane; e < (p + 1) * (p + 1); e += 64) {
            const int m = (int)sqrtf((float)e + 0.5f);  // e in [m^2, (m+1)^2)
            const int mp = e - m * m - m;               // -m .. m
            const int A = m - mp, B = m + mp;
            float pw = 1.f;
            for (int i = 0; i < A; i++) pw *= sh2;
            for (int i = 0; i < B; i++) pw *= ch2;
            // prefactor at degree m: sqrt((2m)! / ((m+m')! (m-m')!)) = sqrt(binom(2m, m-m'))
            float bin = 1.f;
            for (int i = 1; i <= A; i++) bin = bin * (float)(B + i) / (float)i;
            float pref = sqrtf(bin);
            float P0 = 1.f, P1 = (float)(A + 1) + 0.5f * (float)(A + B + 2) * (xh - 1.f);
            for (int j = m; j <= p; j++) {
                const int k = j - m;
                float Pk;
                if (k == 0) {
                    Pk = P0;
                } else if (k == 1) {
                    Pk = P1;
                } else {
                    const float nn = (float)k, ab = (float)(A + B);
                    const float c1 = 2.f * nn * (nn + ab) * (2.f * nn + ab - 2.f);
                    const float c2 = (2.f * nn + ab - 1.f) * ((2.f * nn + ab) * (2.f * nn + ab - 2.f) * xh +
                                                             (float)(A * A - B * B));
                    const float c3 = 2.f * (nn + A - 1.f) * (nn + B - 1.f) * (2.f * nn + ab);
                    Pk = (c2 * P1 - c3 * P0) / c1;
                    P0 = P1;
                    P1 = Pk;
                }
                if (k > 0)  // sqrt((j+m)!(j-m)!/((j+m')!(j-m')!)) from its value at j - 1
                    pref *= sqrtf(((float)(j + m) * (float)(j - m)) / ((float)(j + mp) * (float)(j - mp)));
                D[dofs(j) + (mp + j) * (2 * j + 1) + (m + j)] = pref * pw * Pk;
            }
        }
        wave_sync();
        // the other entries by symmetry
        for (int n = 0; n <= p; n++)
            for (int e = lane; e < (2 * n + 1) * (2 * n + 1); e += 64) {
                const int mp = e / (2 * n + 1) - n, m = e % (2 * n + 1) - n;
                if (m >= (mp < 0 ? -mp : mp)) continue;
                float val;
                if (mp >= (m < 0 ? -m : m)) val = (((m - mp) & 1) ? -1.f : 1.f) * D[dofs(n) + (m + n) * (2 * n + 1) + (mp + n)];
                else if (-m >= (mp < 0 ? -mp : mp))
                    val = (((m - mp) & 1) ? -1.f : 1.f) * D[dofs(n) + (-mp + n) * (2 * n + 1) + (-m + n)];
                else val = D[dofs(n) + (-m + n) * (2 * n + 1) + (-mp + n)];
                D[dofs(n) + (mp + n) * (2 * n + 1) + (m + n)] = val;
            }
        wave_sync();
        // 1-2: azimuth then polar rotation of the multipole, outputs (n, m' >= 0)
        for (int e = lane; e < njk; e += 64) {
            int n = 0;
            while ((n + 1) * (n + 2) / 2 <= e) n++;
            const int mq = e - n * (n + 1) / 2;
            const float* Dr = D + dofs(n) + (mq + n) * (2 * n + 1) + n;  // row m', column m at Dr[m]
            const float inv = eps_of(mq);
            float re = Dr[0] * Ms[n * n], im = 0.f;
            for (int m = 1; m <= n; m++) {
                const float mr = Ms[n * n + 2 * m - 1], mi = Ms[n * n + 2 * m];
                const float ar = mr * em[2 * m] - mi * em[2 * m + 1], ai = mr * em[2 * m + 1] + mi * em[2 * m];
                const float dp = eps_of(m) * Dr[m], dm = Dr[-m];
                re += (dp + dm) * ar;
                im += (dp - dm) * ai;
            }
            Mr[2 * e] = re * inv;
            Mr[2 * e + 1] = im * inv;
        }
        wave_sync();
        // 3: translation along the axis
        for (int e = lane; e < njk; e += 64) {
            int j = 0;
            while ((j + 1) * (j + 2) / 2 <= e) j++;
            const int k = e - j * (j + 1) / 2;
            float vj = v;
            for (int i = 0; i < j; i++) vj *= v;
            float un = 1.f;
            for (int i = 0; i < k; i++) un *= u;
            float re = 0.f, im = 0.f;
            const float* wr = Wax + ((size_t)j * (p + 1)) * (p + 1);
            for (int n = k; n <= p; n++) {
                const float ww = wr[n * (p + 1) + k] * un;
                const int src = n * (n + 1) / 2 + k;
                re += ww * Mr[2 * src];
                im += ww * Mr[2 * src + 1];
                un *= u;
            }
            Lr[2 * e] = re * vj;
            Lr[2 * e + 1] = im * vj;
        }
        wave_sync();
        // 4: rotate back, outputs (j, m >= 0) of this lane
#pragma unroll
        for (int uu = 0; uu < 3; uu++) {
            if (oj[uu] < 0) continue;
            const int j = oj[uu], m = ok[uu];
            const float* Dc = D + dofs(j) + (m + j) + j * (2 * j + 1);  // column m, row m' at Dc[m' (2j+1)]
            const int st = 2 * j + 1;
            const int b0 = j * (j + 1) / 2;
            float re = Dc[0] * Lr[2 * b0], im = 0.f;
            for (int q = 1; q <= j; q++) {
                const float lr = Lr[2 * (b0 + q)], li = Lr[2 * (b0 + q) + 1];
                const float dp = eps_of(q) * Dc[q * st], dm = Dc[-q * st];
                re += (dp + dm) * lr;
                im += (dp - dm) * li;
            }
            const float inv = eps_of(m);
            re *= inv;
            im *= inv;
            // times e^{-i m beta}
            const float cr = em[2 * m], ci = em[2 * m + 1];
            are[uu] += re * cr + im * ci;
            aim[uu] += im * cr - re * ci;
        }
        wave_sync();
    }
#pragma unroll
    for (int uu = 0; uu < 3; uu++) {
        if (oj[uu] < 0) continue;
        const int jk = lane + 64 * uu;
        red[(w * njk + jk) * 2] = are[uu];
        red[(w * njk + jk) * 2 + 1] = aim[uu];
    }
    __syncthreads();
    for (int jk = threadIdx.x; jk < njk; jk += blockDim.x) {
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= jk) j++;
        const int k = jk - j * (j + 1) / 2;
        float sre = 0.f, sim = 0.f;
        for (int ww = 0; ww < nwaves; ww++) {
            sre += red[(ww * njk + jk) * 2];
            sim += red[(ww * njk + jk) * 2 + 1];
        }
        const int ix = idx_re(j, k);
        L[(size_t)t * KP + ix] += sre;
        if (k > 0) L[(size_t)t * KP + ix + 1] += sim;
    }
}

}  // namespace

void m2l_rotation(const int32_t* goff, const uint32_t* gsrc, CellArrays cells, int32_t ncell, int p, int KP,
                  const float* Wax, const float* M, float* L, const uint8_t* skip, hipStream_t s) {
    if (ncell <= 0) return;
    const int njk = (p + 1) * (p + 2) / 2;
    const size_t per = (size_t)rot_wave_floats(p, KP);
    // four waves while their LDS fits a 64 KB share, else two
    const int nw = (4 * per + 8 * (size_t)njk) * sizeof(float) <= 65536 ? 4 : 2;
    const size_t lds = (nw * per + 2 * (size_t)nw * njk) * sizeof(float);
    k_m2l_rot<<<ncell, 64 * nw, lds, s>>>(goff, gsrc, cells, p, KP, Wax, M, L, skip, nw);
}

}  // namespace fmm
