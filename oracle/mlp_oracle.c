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
 *  - ora_mlp_table64: the choice (least predicted log time) over the
 *    quantised feature grid from the FP64 forward, with the gap between the
 *    two least outputs and a bound on how far an FP32 evaluation of the same
 *    network (any summation order, features rounded to FP32) can move each
 *    output.  A decision whose gap exceeds twice the bound is the same in any
 *    FP32 evaluation; closer ones are ties at FP32 resolution.
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

/* Standard forward error of an FP32 dot product plus bias (Higham, Accuracy
 * and Stability of Numerical Algorithms, 2nd ed., section 3.1): with unit
 * roundoff u = 2^-24 and gamma_n = n u / (1 - n u), evaluating
 * b + sum_k w_k x_k over K terms in any order errs by at most
 * gamma_{K+1} (|b| + sum_k |w_k| |x_k|); inputs already off by e_k add
 * sum_k |w_k| e_k.  ReLU does not increase an error. */
static double gamma_n(int n)
{
    const double u = ldexp(1.0, -24);
    return n * u / (1.0 - n * u);
}

/* FP64 forward with a bound e[j] on each output's FP32 evaluation error */
static void forward_bound(const double *w, const double *f, double *y, double *e)
{
    const double u = ldexp(1.0, -24);
    double h1[H], e1[H], h2[H], e2[H], ef[F];
    for (int k = 0; k < F; k++) ef[k] = u * fabs(f[k]);
    for (int i = 0; i < H; i++) {
        double a = w[OB1 + i], mag = fabs(w[OB1 + i]), prop = 0;
        for (int k = 0; k < F; k++) {
            double wk = w[OW1 + i * F + k];
            a += wk * f[k];
            mag += fabs(wk) * (fabs(f[k]) + ef[k]);
            prop += fabs(wk) * ef[k];
        }
        h1[i] = a > 0 ? a : 0;
        e1[i] = prop + gamma_n(F + 1) * mag;
    }
    for (int i = 0; i < H; i++) {
        double a = w[OB2 + i], mag = fabs(w[OB2 + i]), prop = 0;
        for (int k = 0; k < H; k++) {
            double wk = w[OW2 + i * H + k];
            a += wk * h1[k];
            mag += fabs(wk) * (h1[k] + e1[k]);
            prop += fabs(wk) * e1[k];
        }
        h2[i] = a > 0 ? a : 0;
        e2[i] = prop + gamma_n(H + 1) * mag;
    }
    for (int j = 0; j < O; j++) {
        double a = w[OB3 + j], mag = fabs(w[OB3 + j]), prop = 0;
        for (int k = 0; k < H; k++) {
            double wk = w[OW3 + j * H + k];
            a += wk * h2[k];
            mag += fabs(wk) * (h2[k] + e2[k]);
            prop += fabs(wk) * e2[k];
        }
        y[j] = a;
        e[j] = prop + gamma_n(H + 1) * mag;
    }
}

/* Decision grid: entry ((dl+4)*81 + bt)*81 + bs)*4 + bq holds the features
 * (dl/2, (bt/4)/8, (bs/4)/8, p/10, (bq+0.5)/4, theta), dl in [-4, 4],
 * bt, bs in [0, 80], bq in [0, 3]; the least predicted log time wins, ties
 * to the earlier kind.  margin = gap between the two least outputs;
 * bound = largest FP32 error bound of the three outputs. */
void ora_mlp_table64(const double *w, int p, double theta, uint8_t *table, double *margin, double *bound)
{
    int e = 0;
    for (int dl = -4; dl <= 4; dl++)
        for (int bt = 0; bt < 81; bt++)
            for (int bs = 0; bs < 81; bs++)
                for (int bq = 0; bq < 4; bq++, e++) {
                    double f[F] = {dl / 2.0, (bt / 4.0) / 8.0, (bs / 4.0) / 8.0, p / 10.0, (bq + 0.5) / 4.0, theta};
                    double y[O], eo[O];
                    forward_bound(w, f, y, eo);
                    int k = 0;
                    if (y[1] < y[k]) k = 1;
                    if (y[2] < y[k]) k = 2;
                    double second = INFINITY;
                    for (int j = 0; j < O; j++)
                        if (j != k && y[j] < second) second = y[j];
                    table[e] = (uint8_t)k;
                    margin[e] = second - y[k];
                    bound[e] = fmax(eo[0], fmax(eo[1], eo[2]));
                }
}
