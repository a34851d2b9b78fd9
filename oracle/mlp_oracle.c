/*
 * mlp_oracle.c -- CPU oracle of the learned cost model (test infrastructure
 * only; shares no code with the HIP library).
 *
 * The model is a perceptron with two hidden layers of 64 ReLU units mapping
 * 6 pair features to 3 predicted log2 times (M2L, M2P, P2P); it replaces the
 * fixed unit costs that the paper's kernel pre-calculation measures
 * ("Kernel pre-calculation").  Weights: W1[64][6], b1[64], W2[64][64], b2[64],
 * W3[3][64], b3[3].  Training loss: mean over records of the squared error of
 * the output of the record's kernel kind.
 *
 *  - ora_mlp_forward / ora_mlp_loss_grad: FP64, the plain definitions
 *    (backpropagation written out layer by layer).
 *  - ora_mlp_forward_f32 / ora_mlp_table: FP32 with the accumulation order
 *    a = b; a = fma(w_k, x_k, a) for k ascending, so that the kernel-kind
 *    decision is taken in the kernel's precision.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define H 64
#define F 6
#define O 3
#define OW1 0
#define OB1 (OW1 + H * F)
#define OW2 (OB1 + H)
#define OB2 (OW2 + H * H)
#define OW3 (OB2 + H)
#define OB3 (OW3 + O * H)
#define NPAR (OB3 + O)

int ora_mlp_params(void) { return NPAR; }

void ora_mlp_forward(const double *w, const double *f, double *y)
{
    double h1[H], h2[H];
    for (int i = 0; i < H; i++) {
        double a = w[OB1 + i];
        for (int k = 0; k < F; k++) a += w[OW1 + i * F + k] * f[k];
        h1[i] = a > 0 ? a : 0;
    }
    for (int i = 0; i < H; i++) {
        double a = w[OB2 + i];
        for (int k = 0; k < H; k++) a += w[OW2 + i * H + k] * h1[k];
        h2[i] = a > 0 ? a : 0;
    }
    for (int j = 0; j < O; j++) {
        double a = w[OB3 + j];
        for (int k = 0; k < H; k++) a += w[OW3 + j * H + k] * h2[k];
        y[j] = a;
    }
}

/* loss = (1/B) sum_r (y_r[kind_r] - t_r)^2 and its gradient with respect to w */
void ora_mlp_loss_grad(const double *w, int B, const double *feat, const int32_t *kind, const double *tgt,
                       double *loss, double *grad)
{
    memset(grad, 0, sizeof(double) * NPAR);
    double L = 0;
    for (int r = 0; r < B; r++) {
        const double *f = feat + (size_t)r * F;
        double z1[H], h1[H], z2[H], h2[H], y[O];
        for (int i = 0; i < H; i++) {
            double a = w[OB1 + i];
            for (int k = 0; k < F; k++) a += w[OW1 + i * F + k] * f[k];
            z1[i] = a;
            h1[i] = a > 0 ? a : 0;
        }
        for (int i = 0; i < H; i++) {
            double a = w[OB2 + i];
            for (int k = 0; k < H; k++) a += w[OW2 + i * H + k] * h1[k];
            z2[i] = a;
            h2[i] = a > 0 ? a : 0;
        }
        for (int j = 0; j < O; j++) {
            double a = w[OB3 + j];
            for (int k = 0; k < H; k++) a += w[OW3 + j * H + k] * h2[k];
            y[j] = a;
        }
        int kk = kind[r];
        double e = y[kk] - tgt[r];
        L += e * e / B;
        /* backward */
        double dy = 2.0 * e / B;
        for (int k = 0; k < H; k++) grad[OW3 + kk * H + k] += dy * h2[k];
        grad[OB3 + kk] += dy;
        double dz2[H];
        for (int i = 0; i < H; i++) dz2[i] = z2[i] > 0 ? dy * w[OW3 + kk * H + i] : 0;
        for (int i = 0; i < H; i++) {
            grad[OB2 + i] += dz2[i];
            for (int k = 0; k < H; k++) grad[OW2 + i * H + k] += dz2[i] * h1[k];
        }
        for (int k = 0; k < H; k++) {
            double dh1 = 0;
            for (int i = 0; i < H; i++) dh1 += w[OW2 + i * H + k] * dz2[i];
            double dz1 = z1[k] > 0 ? dh1 : 0;
            grad[OB1 + k] += dz1;
            for (int m = 0; m < F; m++) grad[OW1 + k * F + m] += dz1 * f[m];
        }
    }
    *loss = L;
}

void ora_mlp_forward_f32(const float *w, const float *f, float *y)
{
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
    for (int j = 0; j < O; j++) y[j] = o[j];
}

/* Decision grid: entry ((dl+4)*81 + bt)*81 + bs)*4 + bq with features
 * (dl/2, (bt/4)/8, (bs/4)/8, p/10, (bq+0.5)/4, theta); least predicted log
 * time wins, ties to the earlier kind.  `margin` receives the gap between
 * the two smallest outputs (may be NULL). */
void ora_mlp_table(const float *w, int p, float theta, uint8_t *table, float *margin)
{
    int e = 0;
    for (int dl = -4; dl <= 4; dl++)
        for (int bt = 0; bt < 81; bt++)
            for (int bs = 0; bs < 81; bs++)
                for (int bq = 0; bq < 4; bq++, e++) {
                    float f[F] = {(float)dl / 2.f, ((float)bt / 4.f) / 8.f, ((float)bs / 4.f) / 8.f,
                                  (float)p / 10.f, ((float)bq + 0.5f) / 4.f, theta};
                    float y[O];
                    ora_mlp_forward_f32(w, f, y);
                    int k = 0;
                    float best = y[0];
                    if (y[1] < best) { best = y[1]; k = 1; }
                    if (y[2] < best) { best = y[2]; k = 2; }
                    table[e] = (uint8_t)k;
                    if (margin) {
                        float second = INFINITY;
                        for (int j = 0; j < O; j++)
                            if (j != k && y[j] < second) second = y[j];
                        margin[e] = second - best;
                    }
                }
}
