// k_mlp.hip -- the learned cost model: a 6 -> 64 -> 64 -> 3 ReLU perceptron
// that predicts log2 of the time (ns) one accepted cell pair costs as M2L,
// M2P or P2P, trained on timings of the library's own kernels.  The paper
// ("Kernel pre-calculation") selects the interaction kind from pre-measured
// kernel times and notes that on GPUs small pre-tests mispredict because
// kernel time is not proportional to problem size ("Results"); the network
// replaces the fixed unit costs with a learned function of the pair.
//
// Parameter layout (FP32, kMlpParams = 4803):
//   W1[64][6], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]
// Features of a pair (t, s):
//   f0 = log2(r_t / r_s) / 2, f1 = log2(n_t) / 8, f2 = log2(n_s) / 8,
//   f3 = p / 10, f4 = ((r_t + r_s)/R) / theta, f5 = theta
//
// Kernels: per-record forward + backward (one wave per record, one lane per
// hidden unit), a fixed-order reduction of the per-record gradients, Adam,
// the artificial clustered particle sets used to generate the training
// timings, and the evaluation of the network over a quantised feature table
// that the traversal reads.
#include "fmm_internal.h"

#include <algorithm>

namespace fmm {
namespace {

constexpr int H = 64, F = 6, O = 3;
constexpr int OW1 = 0, OB1 = OW1 + H * F, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + O * H;
static_assert(OB3 + O == kMlpParams, "layout");

__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Forward + backward of a chunk of kMlpChunk records per 256-lane workgroup:
// lanes 0..63 hold the hidden units, every lane accumulates the gradient of
// the parameters j = lane + 256 i over the chunk's records in record order,
// and writes the chunk's partial gradient and loss.
constexpr int CH = kMlpChunk;
constexpr int PER_T = (kMlpParams + 255) / 256;

__global__ __launch_bounds__(256) void k_mlp_fwd_bwd(const float* __restrict__ w, const float* __restrict__ feat,
                                                     const int32_t* __restrict__ kind,
                                                     const float* __restrict__ tgt, int B,
                                                     float* __restrict__ grad_part, float* __restrict__ loss_part) {
    __shared__ float f[F], h1[H], h2[H], dz1[H], dz2[H], y[O], sdy[1];
    const int tid = threadIdx.x;
    float g[PER_T];
#pragma unroll
    for (int i = 0; i < PER_T; i++) g[i] = 0.f;
    float lsum = 0.f;
    const int r0 = blockIdx.x * CH, r1 = min(B, r0 + CH);
    for (int r = r0; r < r1; r++) {
        if (tid < F) f[tid] = feat[r * F + tid];
        __syncthreads();
        float z1 = 0.f, z2 = 0.f;
        if (tid < H) {
            z1 = w[OB1 + tid];
#pragma unroll
            for (int k = 0; k < F; k++) z1 = fmaf(w[OW1 + tid * F + k], f[k], z1);
            h1[tid] = fmaxf(z1, 0.f);
        }
        __syncthreads();
        if (tid < H) {
            z2 = w[OB2 + tid];
            for (int k = 0; k < H; k++) z2 = fmaf(w[OW2 + tid * H + k], h1[k], z2);
            h2[tid] = fmaxf(z2, 0.f);
        }
        __syncthreads();
        if (tid < O) {
            float o = w[OB3 + tid];
            for (int k = 0; k < H; k++) o = fmaf(w[OW3 + tid * H + k], h2[k], o);
            y[tid] = o;
        }
        __syncthreads();
        const int kk = kind[r];
        const float e = y[kk] - tgt[r];
        const float dy = 2.f * e / (float)B;
        lsum += e * e / (float)B;
        if (tid < H) dz2[tid] = z2 > 0.f ? dy * w[OW3 + kk * H + tid] : 0.f;
        __syncthreads();
        if (tid < H) {
            float dh1 = 0.f;
            for (int i = 0; i < H; i++) dh1 = fmaf(w[OW2 + i * H + tid], dz2[i], dh1);
            dz1[tid] = z1 > 0.f ? dh1 : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER_T; i++) {
            const int j = tid + 256 * i;
            float d = 0.f;
            if (j < OB1) d = dz1[j / F] * f[j % F];
            else if (j < OW2) d = dz1[j - OB1];
            else if (j < OB2) d = dz2[(j - OW2) / H] * h1[(j - OW2) % H];
            else if (j < OW3) d = dz2[j - OB2];
            else if (j < OB3) d = ((j - OW3) / H == kk) ? dy * h2[(j - OW3) % H] : 0.f;
            else if (j < kMlpParams) d = (j - OB3 == kk) ? dy : 0.f;
            g[i] += d;
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < PER_T; i++) {
        const int j = tid + 256 * i;
        if (j < kMlpParams) grad_part[(size_t)blockIdx.x * kMlpParams + j] = g[i];
    }
    if (tid == 0) loss_part[blockIdx.x] = lsum;
}

// grad[j] = sum over chunks in order of the partial gradients; loss likewise
__global__ void k_mlp_reduce(const float* __restrict__ grad_part, const float* __restrict__ loss_part, int nchunk,
                             float* __restrict__ grad, float* __restrict__ loss) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kMlpParams) {
        float s = 0.f;
        for (int c = 0; c < nchunk; c++) s += grad_part[(size_t)c * kMlpParams + j];
        grad[j] = s;
    }
    if (j == 0) {
        float s = 0.f;
        for (int c = 0; c < nchunk; c++) s += loss_part[c];
        *loss = s;
    }
}

// Adam (Kingma & Ba 2015) with bias correction; step counts from 1
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int step, float lr) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kMlpParams) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.f - b1) * gj;
    const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    const float mh = mj / (1.f - powf(b1, (float)step));
    const float vh = vj / (1.f - powf(b2, (float)step));
    w[j] -= lr * mh / (sqrtf(vh) + eps);
}

// Clustered artificial particles: the 8^L cells of level L, in Morton order,
// each hold `per` particles uniform inside the cell, except that cells in the
// lower x half hold `per_lo`.  With ncrit = per (and per_lo a multiple of 8
// of it, or equal) every leaf holds exactly `per` particles, so each kernel
// sees a homogeneous batch.  The lower-x cells are those whose top Morton
// digit is even, which gives the first particle of cell c in closed form.
__global__ void k_clustered(int L, int per, int per_lo, uint64_t seed, float* __restrict__ x,
                            float* __restrict__ y, float* __restrict__ z, float* __restrict__ q) {
    const int64_t c = (int64_t)blockIdx.x;
    const int64_t G = (int64_t)1 << (3 * (L - 1));
    const int64_t top = c / G, rem = c - top * G;
    const bool lo = (top & 1) == 0;
    const int cnt = lo ? per_lo : per;
    const int64_t first = (((top + 1) / 2) * per_lo + (top / 2) * per) * G + rem * cnt;
    uint32_t a[3] = {0, 0, 0};
    for (int b = 0; b < L; b++)
        for (int d = 0; d < 3; d++) a[d] |= (uint32_t)((c >> (3 * b + d)) & 1) << b;
    const float inv = 1.f / (float)(1u << L);
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
        const int64_t i = first + k;
        const uint64_t b = seed * 0x9E3779B97F4A7C15ull + (uint64_t)i * 4;
        x[i] = ((float)a[0] + 0.001f + 0.998f * (float)(mix64(b + 1) >> 40) * (1.0f / 16777216.0f)) * inv;
        y[i] = ((float)a[1] + 0.001f + 0.998f * (float)(mix64(b + 2) >> 40) * (1.0f / 16777216.0f)) * inv;
        z[i] = ((float)a[2] + 0.001f + 0.998f * (float)(mix64(b + 3) >> 40) * (1.0f / 16777216.0f)) * inv;
        q[i] = (mix64(b + 4) >> 63) ? 1.f : -1.f;
    }
}

// Evaluate the network over the quantised feature grid of the traversal:
// entry (dl, bt, bs, bq) -> kind of least predicted log time (ties: M2L, M2P).
// Where the two least predictions lie within kMlpFallbackMargin (log2 units)
// and unit costs are given (cost[3] > 0), the entry takes the timed
// pre-calculation's choice at the bucket's particle counts instead: c_m2l,
// c_m2p n_t, (c_p2p n_t) n_s in FP64 with n = 2^(bucket / 4), least wins,
// ties to M2L, then M2P.
__global__ void k_mlp_table(const float* __restrict__ w, int p, float theta, double c_m2l, double c_m2p,
                            double c_p2p, int use_costs, uint8_t* __restrict__ table) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kMlpTable) return;
    int rem = e;
    const int bq = rem % kMlpBq;
    rem /= kMlpBq;
    const int bs = rem % kMlpBn;
    rem /= kMlpBn;
    const int bt = rem % kMlpBn;
    const int dl = rem / kMlpBn - kMlpDl;
    float f[F];
    f[0] = (float)dl / 2.f;
    f[1] = ((float)bt / (float)kMlpNsub) / 8.f;
    f[2] = ((float)bs / (float)kMlpNsub) / 8.f;
    f[3] = (float)p / 10.f;
    f[4] = ((float)bq + 0.5f) / (float)kMlpBq;
    f[5] = theta;
    float h1[H];
    for (int i = 0; i < H; i++) {
        float a = w[OB1 + i];
        for (int k = 0; k < F; k++) a = fmaf(w[OW1 + i * F + k], f[k], a);
        h1[i] = fmaxf(a, 0.f);
    }
    float o[O] = {w[OB3], w[OB3 + 1], w[OB3 + 2]};
    for (int i = 0; i < H; i++) {
        float a = w[OB2 + i];
        for (int k = 0; k < H; k++) a = fmaf(w[OW2 + i * H + k], h1[k], a);
        a = fmaxf(a, 0.f);
        for (int j = 0; j < O; j++) o[j] = fmaf(w[OW3 + j * H + i], a, o[j]);
    }
    int k = 0;
    float best = o[0];
    if (o[1] < best) {
        best = o[1];
        k = 1;
    }
    if (o[2] < best) {
        best = o[2];
        k = 2;
    }
    float second = INFINITY;
    for (int j = 0; j < O; j++)
        if (j != k) second = fminf(second, o[j]);
    if (use_costs && second - best < kMlpFallbackMargin) {
        const double nt = exp2((double)bt / kMlpNsub), ns = exp2((double)bs / kMlpNsub);
        const double c0 = c_m2l, c1 = c_m2p * nt, c2 = (c_p2p * nt) * ns;
        k = 0;
        double b = c0;
        if (c1 < b) {
            b = c1;
            k = 1;
        }
        if (c2 < b) k = 2;
    }
    table[e] = (uint8_t)k;
}


}  // namespace

void mlp_grad(const float* w, const float* feat, const int32_t* kind, const float* tgt, int B, float* grad_part,
              float* loss_part, float* grad, float* loss, hipStream_t s) {
    if (B <= 0) return;
    const int nchunk = (B + kMlpChunk - 1) / kMlpChunk;
    k_mlp_fwd_bwd<<<nchunk, 256, 0, s>>>(w, feat, kind, tgt, B, grad_part, loss_part);
    k_mlp_reduce<<<(kMlpParams + 255) / 256, 256, 0, s>>>(grad_part, loss_part, nchunk, grad, loss);
}

void mlp_adam(float* w, float* m, float* v, const float* g, int step, float lr, hipStream_t s) {
    k_adam<<<(kMlpParams + 255) / 256, 256, 0, s>>>(w, m, v, g, step, lr);
}

int64_t clustered_points(int L, int per, int per_lo, uint64_t seed, float* x, float* y, float* z, float* q,
                         hipStream_t s) {
    const int64_t ncells = (int64_t)1 << (3 * L);
    if (x) k_clustered<<<(unsigned)ncells, 64, 0, s>>>(L, per, per_lo, seed, x, y, z, q);
    return (ncells / 2) * per_lo + (ncells / 2) * per;
}

void mlp_table(const float* w, int p, float theta, const double* costs, uint8_t* table, hipStream_t s) {
    k_mlp_table<<<(kMlpTable + 255) / 256, 256, 0, s>>>(w, p, theta, costs ? costs[0] : 0.0, costs ? costs[1] : 0.0,
                                                         costs ? costs[2] : 0.0, costs ? 1 : 0, table);
}

}  // namespace fmm
