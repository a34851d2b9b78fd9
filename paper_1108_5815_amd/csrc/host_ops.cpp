// host_ops.cpp -- FP64 host construction of the expansion operators.
//
// Expansions follow Greengard & Rokhlin (Acta Numerica 1997, theorems
// 3.2-3.5), the spherical-harmonic form the paper's method uses for every
// far-field interaction ("Hybrid treecode/FMM algorithm"; "Results").  With
// N(n,m) = sqrt((n-m)!(n+m)!) the theorems' coefficients reduce to
//   M2M: M_j^k += O_{j-n}^{k-m} i^{|k|-|m|-|k-m|} N(j,k)/(N(n,m)N(j-n,k-m)) rho^n Y_n^{-m}
//   M2L: L_j^k += O_n^m i^{|k-m|-|k|-|m|} (-1)^n N(j+n,m-k)/(N(n,m)N(j,k)) Y_{j+n}^{m-k}/rho^{j+n+1}
//   L2L: L_j^k += O_n^m i^{|m|-|m-k|-|k|} (-1)^{n+j} N(n,m)/(N(n-j,m-k)N(j,k)) rho^{n-j} Y_{n-j}^{m-k}
// Solid harmonics come from Cartesian recurrences (no trigonometry):
//   S_n^m = rho^n Y_n^m:     S_m^m = C1(m)(x+iy) S_{m-1}^{m-1}, S_{m+1}^m = C2(m) z S_m^m,
//                            S_n^m = A(n,m) z S_{n-1}^m - B(n,m) r^2 S_{n-2}^m
//   J_n^m = Y_n^m/rho^{n+1}: the same with an extra 1/r^2 per step and J_0^0 = 1/r.
// Real layout: a complex linear map out(j,k) += w * c(n,m), where
// c(n,m<0) = conj(c_n^|m|), is accumulated column by column on the real and
// imaginary parts of c_n^|m|.
#include "host_ops.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <stdexcept>

namespace fmm {
namespace {

using cd = std::complex<double>;

double fact(int k) {
    static double F[200];
    static bool ready = false;
    if (!ready) {
        F[0] = 1;
        for (int i = 1; i < 200; i++) F[i] = F[i - 1] * i;
        ready = true;
    }
    return F[k];
}

double Nnm(int n, int m) {
    m = m < 0 ? -m : m;
    return std::sqrt(fact(n - m) * fact(n + m));
}

cd ipow(int e) {
    int r = ((e % 4) + 4) % 4;
    static const cd v[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    return v[r];
}

int ri(int n, int m, bool im) { return m == 0 ? n * n : n * n + 2 * m - (im ? 0 : 1); }

// triangular complex tables T[n][m], m = 0..n
struct Tri {
    int P;
    std::vector<cd> v;
    explicit Tri(int P_) : P(P_), v((P_ + 1) * (P_ + 2) / 2) {}
    cd& at(int n, int m) { return v[n * (n + 1) / 2 + m]; }
    cd full(int n, int m) {
        if (m >= 0) return at(n, m);
        return std::conj(at(n, -m));
    }
};

void regular(int P, double x, double y, double z, Tri& S) {
    double r2 = x * x + y * y + z * z;
    S.at(0, 0) = 1.0;
    for (int m = 1; m <= P; m++)
        S.at(m, m) = std::sqrt((2.0 * m - 1) / (2.0 * m)) * cd(x, y) * S.at(m - 1, m - 1);
    for (int m = 0; m < P; m++) S.at(m + 1, m) = std::sqrt(2.0 * m + 1) * z * S.at(m, m);
    for (int m = 0; m <= P; m++)
        for (int n = m + 2; n <= P; n++)
            S.at(n, m) = ((2.0 * n - 1) * z * S.at(n - 1, m) -
                          r2 * std::sqrt(double(n - m - 1) * (n + m - 1)) * S.at(n - 2, m)) /
                         std::sqrt(double(n - m) * (n + m));
}

void irregular(int P, double x, double y, double z, Tri& J) {
    double r2 = x * x + y * y + z * z;
    double ir2 = 1.0 / r2;
    J.at(0, 0) = 1.0 / std::sqrt(r2);
    for (int m = 1; m <= P; m++)
        J.at(m, m) = std::sqrt((2.0 * m - 1) / (2.0 * m)) * cd(x, y) * ir2 * J.at(m - 1, m - 1);
    for (int m = 0; m < P; m++) J.at(m + 1, m) = std::sqrt(2.0 * m + 1) * z * ir2 * J.at(m, m);
    for (int m = 0; m <= P; m++)
        for (int n = m + 2; n <= P; n++)
            J.at(n, m) = ((2.0 * n - 1) * z * J.at(n - 1, m) -
                          std::sqrt(double(n + m - 1) * (n - m - 1)) * J.at(n - 2, m)) *
                         ir2 / std::sqrt(double(n - m) * (n + m));
}

// out(j,k) += w * chat(n,m) into a row-major real matrix with `cols` columns
void add_term(std::vector<double>& Mt, int cols, int j, int k, int n, int m, cd w) {
    int am = m < 0 ? -m : m;
    int cre = ri(n, am, false);
    Mt[(size_t)ri(j, k, false) * cols + cre] += w.real();
    if (k > 0) Mt[(size_t)ri(j, k, true) * cols + cre] += w.imag();
    if (am > 0) {
        int cim = ri(n, am, true);
        cd wi = (m > 0) ? cd(0, 1) * w : cd(0, -1) * w;
        Mt[(size_t)ri(j, k, false) * cols + cim] += wi.real();
        if (k > 0) Mt[(size_t)ri(j, k, true) * cols + cim] += wi.imag();
    }
}

// M2M of a child whose centre is rc*sigma from its parent's centre; scaled
// child and parent multipoles (divided by r^n of their own cell).
void m2m_operator(int p, const double sig[3], std::vector<double>& Mt) {
    int K = (p + 1) * (p + 1);
    Mt.assign((size_t)K * K, 0.0);
    Tri S(p);
    regular(p, sig[0], sig[1], sig[2], S);
    for (int j = 0; j <= p; j++)
        for (int k = 0; k <= j; k++)
            for (int n = 0; n <= j; n++)
                for (int m = -n; m <= n; m++) {
                    int km = k - m;
                    if (km < -(j - n) || km > (j - n)) continue;
                    cd w = ipow(std::abs(k) - std::abs(m) - std::abs(km)) * Nnm(j, k) /
                           (Nnm(n, m) * Nnm(j - n, km));
                    add_term(Mt, K, j, k, j - n, km, w * S.full(n, -m) * std::ldexp(1.0, -j));
                }
}

// L2L parent -> child whose centre is rc*sigma from the parent's centre.
void l2l_operator(int p, const double sig[3], std::vector<double>& Mt) {
    int K = (p + 1) * (p + 1);
    Mt.assign((size_t)K * K, 0.0);
    Tri S(p);
    regular(p, -sig[0], -sig[1], -sig[2], S);
    for (int j = 0; j <= p; j++)
        for (int k = 0; k <= j; k++)
            for (int n = j; n <= p; n++)
                for (int m = -n; m <= n; m++) {
                    int mk = m - k;
                    if (mk < -(n - j) || mk > (n - j)) continue;
                    double sgn = ((n + j) & 1) ? -1.0 : 1.0;
                    cd w = ipow(std::abs(m) - std::abs(mk) - std::abs(k)) * sgn * Nnm(n, m) /
                           (Nnm(n - j, mk) * Nnm(j, k));
                    add_term(Mt, K, j, k, n, m, w * S.full(n - j, mk) * std::ldexp(1.0, -(n + 1)));
                }
}

}  // namespace

void m2l_operator(int p, const double q[3], double ratio, std::vector<double>& Mt) {
    int K = (p + 1) * (p + 1);
    Mt.assign((size_t)K * K, 0.0);
    Tri J(2 * p);
    irregular(2 * p, q[0], q[1], q[2], J);
    for (int j = 0; j <= p; j++)
        for (int k = 0; k <= j; k++) {
            double rn = 1.0;
            for (int n = 0; n <= p; n++) {
                for (int m = -n; m <= n; m++) {
                    double sgn = (n & 1) ? -1.0 : 1.0;
                    cd w = ipow(std::abs(k - m) - std::abs(k) - std::abs(m)) * sgn * Nnm(j + n, m - k) /
                           (Nnm(n, m) * Nnm(j, k));
                    add_term(Mt, K, j, k, n, m, w * rn * J.full(j + n, m - k));
                }
                rn *= ratio;
            }
        }
}

static uint16_t bf16_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static float bf16_value(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

void split_bf16_kblocked(const std::vector<float>& T, size_t noff, int KP, std::vector<uint16_t>& hi,
                         std::vector<uint16_t>& lo) {
    const size_t KB = KP / 8;
    hi.assign(noff * KP * KP, 0);
    lo.assign(noff * KP * KP, 0);
    for (size_t o = 0; o < noff; o++)
        for (int k = 0; k < KP; k++)
            for (int j = 0; j < KP; j++) {
                const float v = T[(o * KP + k) * KP + j];
                const uint16_t h = bf16_rne(v);
                const uint16_t l = bf16_rne(v - bf16_value(h));
                const size_t ix = ((o * KB + k / 8) * KP + j) * 8 + k % 8;
                hi[ix] = h;
                lo[ix] = l;
            }
}

void build_tables(int p, HostTables& t) {
    if (p < 0 || p > 16) throw std::invalid_argument("order out of range");
    int K = (p + 1) * (p + 1);
    t.p = p;
    t.K = K;
    t.KP = kpad(p);
    t.m2m.assign((size_t)8 * K * K, 0.f);
    t.l2l.assign((size_t)8 * K * K, 0.f);
    std::vector<double> Mt;
    for (int oct = 0; oct < 8; oct++) {
        double sig[3] = {(oct & 1) ? 1.0 : -1.0, (oct & 2) ? 1.0 : -1.0, (oct & 4) ? 1.0 : -1.0};
        m2m_operator(p, sig, Mt);
        for (int j = 0; j < K; j++)
            for (int k = 0; k < K; k++) t.m2m[((size_t)oct * K + k) * K + j] = (float)Mt[(size_t)j * K + k];
        l2l_operator(p, sig, Mt);
        for (int j = 0; j < K; j++)
            for (int k = 0; k < K; k++) t.l2l[((size_t)oct * K + k) * K + j] = (float)Mt[(size_t)j * K + k];
    }
    // general M2L weights W(j,k,n,m) (real: the power of i is +-1)
    int njk = (p + 1) * (p + 2) / 2;
    t.wm2l.assign((size_t)njk * K, 0.f);
    for (int j = 0; j <= p; j++)
        for (int k = 0; k <= j; k++)
            for (int n = 0; n <= p; n++)
                for (int m = -n; m <= n; m++) {
                    double sgn = (n & 1) ? -1.0 : 1.0;
                    cd w = ipow(std::abs(k - m) - std::abs(k) - std::abs(m)) * sgn * Nnm(j + n, m - k) /
                           (Nnm(n, m) * Nnm(j, k));
                    t.wm2l[(size_t)(j * (j + 1) / 2 + k) * K + n * n + n + m] = (float)w.real();
                }
    // gradient weights: L2P (local re-centred at the point, sign of -x folded in)
    t.gl2p.assign((size_t)2 * K, 0.f);
    t.hm2p.assign((size_t)2 * K, 0.f);
    for (int n = 0; n <= p; n++)
        for (int m = -n; m <= n; m++)
            for (int k = 0; k <= 1; k++) {
                if (n >= 1 && std::abs(m - k) <= n - 1) {
                    // w(1,k,n,m) (-1)^(n-1), w = i^{|m|-|m-k|-|k|} (-1)^(n+1) N(n,m)/(N(n-1,m-k)N(1,k))
                    cd w = ipow(std::abs(m) - std::abs(m - k) - std::abs(k)) * Nnm(n, m) /
                           (Nnm(n - 1, m - k) * Nnm(1, k));
                    t.gl2p[(size_t)k * K + n * n + n + m] = (float)w.real();
                }
                // W(1,k,n,m) (-1)^(n+1), W = i^{|k-m|-|k|-|m|} (-1)^n N(n+1,m-k)/(N(n,m)N(1,k))
                cd h = -ipow(std::abs(k - m) - std::abs(k) - std::abs(m)) * Nnm(n + 1, m - k) /
                       (Nnm(n, m) * Nnm(1, k));
                t.hm2p[(size_t)k * K + n * n + n + m] = (float)h.real();
            }
    // axial M2L (offset along +z): L_j^k = sum_n W(j,n,k) M_n^k / rho^(j+n+1),
    // theorem 3.4 at polar angle 0, W = (-1)^(k+n) (j+n)! / (N(n,k) N(j,k))
    t.wrot.assign((size_t)(p + 1) * (p + 1) * (p + 1), 0.f);
    for (int j = 0; j <= p; j++)
        for (int n = 0; n <= p; n++)
            for (int k = 0; k <= std::min(j, n); k++)
                t.wrot[((size_t)j * (p + 1) + n) * (p + 1) + k] =
                    (float)((((k + n) & 1) ? -1.0 : 1.0) * fact(j + n) / (Nnm(n, k) * Nnm(j, k)));
    t.rcoef.assign(kRcSize, 0.f);
    for (int n = 0; n <= kRcN; n++)
        for (int m = 0; m <= n; m++) {
            if (n >= m + 2) {
                t.rcoef[kRcA + n * (n + 1) / 2 + m] = (float)((2.0 * n - 1) / std::sqrt(double(n - m) * (n + m)));
                t.rcoef[kRcB + n * (n + 1) / 2 + m] =
                    (float)std::sqrt(double(n - m - 1) * (n + m - 1) / (double(n - m) * (n + m)));
            }
        }
    for (int m = 0; m < 40; m++) {
        t.rcoef[kRcC1 + m] = m == 0 ? 0.f : (float)std::sqrt((2.0 * m - 1) / (2.0 * m));
        t.rcoef[kRcC2 + m] = (float)std::sqrt(2.0 * m + 1);
    }
}

int m2l_plan_slots(double theta) {
    double theta2 = theta * theta;
    int omax = 0;
    while (theta2 * (double)((omax + 1) * (omax + 1)) < 1.0) omax++;
    // octant class 0 (target at the low corner of its parent): offsets
    // o = 2O + c_s over the parent offsets O that are not accepted
    int J = 0;
    for (int a = -omax; a <= omax; a++)
        for (int b = -omax; b <= omax; b++)
            for (int c = -omax; c <= omax; c++) {
                if (!(theta2 * (double)(a * a + b * b + c * c) < 1.0)) continue;
                for (int cs = 0; cs < 8; cs++) {
                    int o0 = 2 * a + (cs & 1), o1 = 2 * b + ((cs >> 1) & 1), o2 = 2 * c + ((cs >> 2) & 1);
                    if (1.0 <= theta2 * (double)(o0 * o0 + o1 * o1 + o2 * o2)) J++;
                }
            }
    return J;
}

namespace {

// Cartesian operators (multi-indices in graded order, see cart.h)
int cidx(int a, int b, int c) {
    int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}

double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; i++) r = r * (double)(n - k + i) / (double)i;
    return r;
}

template <class F>
void for_multi(int p, F f) {
    for (int n = 0; n <= p; n++)
        for (int a = n; a >= 0; a--)
            for (int b = n - a; b >= 0; b--) f(n, a, b, n - a - b);
}

// Taylor coefficients a_n(R) of 1/|R|, |n| <= P (the recurrence of cart.h in FP64)
void taylor(int P, const double R[3], std::vector<double>& a) {
    a.assign((size_t)(P + 1) * (P + 2) * (P + 3) / 6, 0.0);
    const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    a[0] = 1.0 / std::sqrt(r2);
    for_multi(P, [&](int n, int i, int j, int k) {
        if (n == 0) return;
        double s1 = 0.0, s2 = 0.0;
        if (i >= 1) s1 += R[0] * a[cidx(i - 1, j, k)];
        if (j >= 1) s1 += R[1] * a[cidx(i, j - 1, k)];
        if (k >= 1) s1 += R[2] * a[cidx(i, j, k - 1)];
        if (i >= 2) s2 += a[cidx(i - 2, j, k)];
        if (j >= 2) s2 += a[cidx(i, j - 2, k)];
        if (k >= 2) s2 += a[cidx(i, j, k - 2)];
        a[cidx(i, j, k)] = -((2.0 * n - 1.0) / n * s1 + (n - 1.0) / n * s2) / r2;
    });
}

double sgnpow(const double v[3], int a, int b, int c) {
    double r = 1.0;
    for (int e = 0; e < a; e++) r *= v[0];
    for (int e = 0; e < b; e++) r *= v[1];
    for (int e = 0; e < c; e++) r *= v[2];
    return r;
}

// scaled M2M of a child at rc*sig from its parent's centre: M~'_k =
// sum_{a<=k} binom(k,a) (-sig)^(k-a) 2^-|k| M~_a  (row-major out x in)
void m2m_operator_cart(int p, const double sig[3], std::vector<double>& Mt) {
    const int K = (p + 1) * (p + 2) * (p + 3) / 6;
    Mt.assign((size_t)K * K, 0.0);
    const double ms[3] = {-sig[0], -sig[1], -sig[2]};
    for_multi(p, [&](int n, int k1, int k2, int k3) {
        for (int a1 = 0; a1 <= k1; a1++)
            for (int a2 = 0; a2 <= k2; a2++)
                for (int a3 = 0; a3 <= k3; a3++)
                    Mt[(size_t)cidx(k1, k2, k3) * K + cidx(a1, a2, a3)] =
                        binom(k1, a1) * binom(k2, a2) * binom(k3, a3) * sgnpow(ms, k1 - a1, k2 - a2, k3 - a3) *
                        std::ldexp(1.0, -n);
    });
}

// scaled L2L to a child at rc*sig: L~'_m' = sum_{m>=m'} binom(m,m') sig^(m-m') 2^-(|m|+1) L~_m
void l2l_operator_cart(int p, const double sig[3], std::vector<double>& Mt) {
    const int K = (p + 1) * (p + 2) * (p + 3) / 6;
    Mt.assign((size_t)K * K, 0.0);
    for_multi(p, [&](int, int a1, int a2, int a3) {
        for_multi(p, [&](int nm, int m1, int m2, int m3) {
            if (m1 < a1 || m2 < a2 || m3 < a3) return;
            Mt[(size_t)cidx(a1, a2, a3) * K + cidx(m1, m2, m3)] =
                binom(m1, a1) * binom(m2, a2) * binom(m3, a3) * sgnpow(sig, m1 - a1, m2 - a2, m3 - a3) *
                std::ldexp(1.0, -(nm + 1));
        });
    });
}

// scaled same-level M2L with the source centre at q (target half sides) from
// the target's: L~_m = sum_{|m|+|k|<=p} C(m,k) a_{m+k}(-q) M~_k
void m2l_operator_cart(int p, const double q[3], std::vector<double>& Mt) {
    const int K = (p + 1) * (p + 2) * (p + 3) / 6;
    Mt.assign((size_t)K * K, 0.0);
    const double R[3] = {-q[0], -q[1], -q[2]};
    std::vector<double> a;
    taylor(p, R, a);
    for_multi(p, [&](int nm, int m1, int m2, int m3) {
        for_multi(p - nm, [&](int, int k1, int k2, int k3) {
            const double C = binom(m1 + k1, k1) * binom(m2 + k2, k2) * binom(m3 + k3, k3);
            Mt[(size_t)cidx(m1, m2, m3) * K + cidx(k1, k2, k3)] = C * a[cidx(m1 + k1, m2 + k2, m3 + k3)];
        });
    });
}

}  // namespace

void build_tables_cart(int p, HostTables& t) {
    if (p < 0 || p > 8) throw std::invalid_argument("order out of range");
    const int K = (p + 1) * (p + 2) * (p + 3) / 6;
    t = HostTables{};
    t.p = p;
    t.K = K;
    t.KP = kpad_cart(p);
    t.m2m.assign((size_t)8 * K * K, 0.f);
    t.l2l.assign((size_t)8 * K * K, 0.f);
    std::vector<double> Mt;
    for (int oct = 0; oct < 8; oct++) {
        double sig[3] = {(oct & 1) ? 1.0 : -1.0, (oct & 2) ? 1.0 : -1.0, (oct & 4) ? 1.0 : -1.0};
        m2m_operator_cart(p, sig, Mt);
        for (int j = 0; j < K; j++)
            for (int k = 0; k < K; k++) t.m2m[((size_t)oct * K + k) * K + j] = (float)Mt[(size_t)j * K + k];
        l2l_operator_cart(p, sig, Mt);
        for (int j = 0; j < K; j++)
            for (int k = 0; k < K; k++) t.l2l[((size_t)oct * K + k) * K + j] = (float)Mt[(size_t)j * K + k];
    }
}

void build_m2l_plan(int p, double theta, M2LPlan& plan, bool cartesian) {
    double theta2 = theta * theta;
    int omax = 0;
    while (theta2 * (double)((omax + 1) * (omax + 1)) < 1.0) omax++;
    // parent offsets O that are not accepted: theta2 |O|^2 < 1
    std::vector<std::array<int, 3>> near;
    for (int a = -omax; a <= omax; a++)
        for (int b = -omax; b <= omax; b++)
            for (int c = -omax; c <= omax; c++)
                if (theta2 * (double)(a * a + b * b + c * c) < 1.0) near.push_back({a, b, c});
    int R = 2 * omax + 1;
    int W = 2 * R + 1;
    plan.p = p;
    plan.theta = theta;
    plan.cartesian = cartesian;
    plan.R = R;
    plan.slot_of.assign((size_t)8 * W * W * W, -1);
    std::map<std::array<int, 3>, int> uid;
    std::vector<std::vector<std::array<int, 3>>> per(8);
    for (int ct = 0; ct < 8; ct++) {
        int t3[3] = {ct & 1, (ct >> 1) & 1, (ct >> 2) & 1};
        std::vector<std::array<int, 3>> L;
        for (auto& O : near)
            for (int cs = 0; cs < 8; cs++) {
                int s3[3] = {cs & 1, (cs >> 1) & 1, (cs >> 2) & 1};
                std::array<int, 3> o = {2 * O[0] + s3[0] - t3[0], 2 * O[1] + s3[1] - t3[1],
                                        2 * O[2] + s3[2] - t3[2]};
                int o2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
                if (1.0 <= theta2 * (double)o2) L.push_back(o);
            }
        // slots in generation order: the (up to) eight children of one parent
        // offset are consecutive, so the M2L pairs of one target and one
        // split source parent fill neighbouring entries of the gather table
        per[ct] = L;
        if (ct == 0) plan.J = (int)L.size();
        if ((int)L.size() != plan.J) throw std::runtime_error("asymmetric offset classes");
        for (auto& o : L)
            if (!uid.count(o)) {
                int id = (int)uid.size();
                uid[o] = id;
            }
    }
    plan.offsets.assign(uid.size(), {0, 0, 0});
    for (auto& kv : uid) plan.offsets[kv.second] = kv.first;
    plan.offid.assign((size_t)8 * plan.J, 0);
    for (int ct = 0; ct < 8; ct++)
        for (int s = 0; s < plan.J; s++) {
            auto& o = per[ct][s];
            plan.offid[(size_t)ct * plan.J + s] = uid[o];
            size_t ix = ((size_t)(o[0] + R) * W + (o[1] + R)) * W + (o[2] + R);
            plan.slot_of[(size_t)ct * W * W * W + ix] = s;
        }
    int K = cartesian ? (p + 1) * (p + 2) * (p + 3) / 6 : (p + 1) * (p + 1);
    int KP = cartesian ? kpad_cart(p) : kpad(p);
    size_t noff = plan.offsets.size();
    plan.T.assign(noff * KP * KP, 0.f);
    std::vector<double> Mt;
    for (size_t o = 0; o < noff; o++) {
        double q[3] = {2.0 * plan.offsets[o][0], 2.0 * plan.offsets[o][1], 2.0 * plan.offsets[o][2]};
        if (cartesian) m2l_operator_cart(p, q, Mt);
        else m2l_operator(p, q, 1.0, Mt);
        for (int j = 0; j < K; j++)
            for (int k = 0; k < K; k++) plan.T[(o * KP + k) * KP + j] = (float)Mt[(size_t)j * K + k];
    }
}

}  // namespace fmm
