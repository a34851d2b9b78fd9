/*
 * oracle_drive.c -- exercises every entry point of the CPU oracle on small
 * inputs (including the degenerate ones: one point, coincident points,
 * target and source sets that differ) so that a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer can report out-of-bounds accesses, leaks,
 * overflow and the like.  Test infrastructure; prints "ok" when done.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void ora_set_threads(int n);
void ora_direct(int64_t n, const double *x, const double *y, const double *z, const double *q, int64_t nt,
                const int64_t *tgt, double *phi, double *ex, double *ey, double *ez);
void *ora_build(int64_t n, const double *x, const double *y, const double *z, int32_t ncrit);
void *ora_build_ts(int64_t n, const double *x, const double *y, const double *z, int64_t nt, int32_t ncrit);
int64_t ora_ncells(void *h);
void ora_get_bbox(void *h, double *lo3, double *side);
void ora_get_keys(void *h, uint64_t *skey, int64_t *perm);
void ora_get_cells(void *h, int32_t *level, uint64_t *prefix, int32_t *begin, int32_t *end, int32_t *parent,
                   int32_t *first_child, int32_t *nchild, int64_t *centre_h, int64_t *radius_h, double *centre,
                   double *radius);
void ora_traverse(void *h, double theta, int policy, const double *costs);
void ora_traverse_table(void *h, double theta, const uint8_t *table);
int64_t ora_list_size(void *h, int kind);
void ora_get_list(void *h, int kind, int32_t *t, int32_t *s);
void ora_evaluate(void *h, int p, const double *q, double *phi, double *ex, double *ey, double *ez);
void ora_evaluate_cart(void *h, int p, const double *q, double *phi, double *ex, double *ey, double *ez);
void ora_get_expansions(void *h, cplx *M, cplx *L);
void ora_get_expansions_cart(void *h, double *M, double *L);
void ora_free(void *h);
int ora_mlp_params(void);
void ora_mlp_forward(const double *w, const double *f, double *y);
void ora_mlp_loss_grad(const double *w, int B, const double *feat, const int32_t *kind, const double *tgt,
                       double *loss, double *grad);
void ora_mlp_table64(const double *w, int p, double theta, uint8_t *table, double *margin, double *bound);

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static double urand(void)
{
    rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static void *xmalloc(size_t n) { void *p = calloc(n ? n : 1, 1); if (!p) abort(); return p; }

/* build, query, traverse under every policy, evaluate in both families */
static void run(int64_t n, int64_t nt, const double *x, const double *y, const double *z, const double *q,
                int ncrit, int p)
{
    void *h = nt < 0 ? ora_build(n, x, y, z, ncrit) : ora_build_ts(n, x, y, z, nt, ncrit);
    int64_t nc = ora_ncells(h);
    double lo[3], side;
    ora_get_bbox(h, lo, &side);
    uint64_t *key = xmalloc((size_t)n * 8);
    int64_t *perm = xmalloc((size_t)n * 8);
    ora_get_keys(h, key, perm);
    size_t c = (size_t)nc;
    int32_t *i32 = xmalloc(c * 4 * 6);
    uint64_t *pre = xmalloc(c * 8);
    int64_t *ch = xmalloc(c * 8 * 3), *rh = xmalloc(c * 8);
    double *cp = xmalloc(c * 8 * 3), *rp = xmalloc(c * 8);
    ora_get_cells(h, i32, pre, i32 + c, i32 + 2 * c, i32 + 3 * c, i32 + 4 * c, i32 + 5 * c, ch, rh, cp, rp);
    const double costs[3] = {1.0, 2.0, 0.01};
    uint8_t *table = xmalloc(9 * 81 * 81 * 4);
    for (int i = 0; i < 9 * 81 * 81 * 4; i++) table[i] = (uint8_t)(i % 3);
    for (int pol = 0; pol <= 3; pol++) {
        double theta = pol == 1 ? 0.7 : 0.4;
        if (pol == 3) ora_traverse_table(h, theta, table);
        else ora_traverse(h, theta, pol, costs);
        for (int k = 0; k < 3; k++) {
            int64_t m = ora_list_size(h, k);
            int32_t *t = xmalloc((size_t)m * 4), *s = xmalloc((size_t)m * 4);
            ora_get_list(h, k, t, s);
            free(t); free(s);
        }
        int64_t no = nt < 0 ? n : nt;
        double *out = xmalloc((size_t)(no ? no : 1) * 8 * 4);
        ora_evaluate(h, p, q, out, out + no, out + 2 * no, out + 3 * no);
        cplx *M = xmalloc(c * (size_t)(p + 1) * (p + 1) * sizeof(cplx) * 2);
        ora_get_expansions(h, M, M + c * (size_t)(p + 1) * (p + 1));
        free(M);
        int pc = p < 6 ? p : 6;
        ora_evaluate_cart(h, pc, q, out, out + no, out + 2 * no, out + 3 * no);
        size_t kc = (size_t)(pc + 1) * (pc + 2) * (pc + 3) / 6;
        double *Mc = xmalloc(c * kc * 8 * 2);
        ora_get_expansions_cart(h, Mc, Mc + c * kc);
        free(Mc);
        free(out);
    }
    free(table); free(key); free(perm); free(i32); free(pre); free(ch); free(rh); free(cp); free(rp);
    ora_free(h);
}

int main(void)
{
    ora_set_threads(2);
    enum { N = 2000 };
    double *x = xmalloc(N * 8), *y = xmalloc(N * 8), *z = xmalloc(N * 8), *q = xmalloc(N * 8);
    for (int i = 0; i < N; i++) {
        /* a clustered set: radius drawn from a steep law, plus a block of coincident points */
        double r = pow(urand(), 3.0), ct = 2 * urand() - 1, ph = 6.283185307179586 * urand();
        double st = sqrt(1 - ct * ct);
        x[i] = r * st * cos(ph); y[i] = r * st * sin(ph); z[i] = r * ct;
        q[i] = 2 * urand() - 1;
    }
    for (int i = 0; i < 40; i++) { x[i] = 0.25; y[i] = -0.125; z[i] = 0.5; }
    double *d = xmalloc(N * 8 * 4);
    int64_t tg[7] = {0, 1, 2, 39, 40, 1500, N - 1};
    ora_direct(N, x, y, z, q, 7, tg, d, d + 7, d + 14, d + 21);
    free(d);
    run(N, -1, x, y, z, q, 24, 5);          /* one set, adaptive */
    run(1, -1, x, y, z, q, 24, 4);          /* one point */
    run(40, -1, x, y, z, q, 8, 3);          /* all coincident: the level limit */
    run(N, 800, x, y, z, q + 800, 16, 4);  /* targets [0, 800), sources the rest */
    run(N, 1, x, y, z, q + 1, 16, 2);       /* one target */
    int np = ora_mlp_params();
    double *w = xmalloc((size_t)np * 8), *g = xmalloc((size_t)np * 8);
    for (int i = 0; i < np; i++) w[i] = 0.3 * (2 * urand() - 1);
    double f[6 * 5], t[5], yv[3], loss;
    int32_t kind[5];
    for (int i = 0; i < 30; i++) f[i] = urand();
    for (int r = 0; r < 5; r++) { t[r] = urand(); kind[r] = r % 3; }
    ora_mlp_forward(w, f, yv);
    ora_mlp_loss_grad(w, 5, f, kind, t, &loss, g);
    uint8_t *tab = xmalloc(9 * 81 * 81 * 4);
    double *mg = xmalloc(9 * 81 * 81 * 4 * 8), *bd = xmalloc(9 * 81 * 81 * 4 * 8);
    ora_mlp_table64(w, 10, 0.4, tab, mg, bd);
    free(tab); free(mg); free(bd); free(w); free(g);
    free(x); free(y); free(z); free(q);
    printf("ok\n");
    return 0;
}
