/*
 * fmm_oracle.c -- plain FP64 CPU oracle of the hierarchical N-body method of
 * Yokota & Barba, "Hierarchical N-body simulations with auto-tuning for
 * heterogeneous systems" (arXiv 1108.5815).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * constant generator with the HIP library; the two meet only in the seeded
 * inputs both are given.
 *
 * What it computes, in the paper's order:
 *  - the plain definition the method approximates: the Laplace potential and
 *    force of every target by direct all-pairs summation (paper: introduction
 *    and "Hierarchical N-body algorithms", the O(N^2) all-pairs sum);
 *  - the adaptive tree: cells split while they hold more than N_crit
 *    particles ("Results": N_crit is the maximum number of particles per cell);
 *  - the dual tree traversal with a last-in-first-out stack of (target,
 *    source) cell pairs, splitting the larger cell, and the acceptance
 *    criterion theta = (r_t + r_s) / R ("Dual tree traversal"; "Results");
 *  - the choice between cell-cell, cell-particle and particle-particle
 *    interaction per accepted pair ("Kernel pre-calculation"; "Results");
 *  - spherical-harmonic multipole and local expansions and their translations
 *    ("Hybrid treecode/FMM algorithm"; "Results": all methods use spherical
 *    harmonics).  The paper prints no formulas; the expansions follow
 *    Greengard & Rokhlin, Acta Numerica 6 (1997), theorems 3.2-3.5;
 *  - Cartesian (Taylor) expansions, the family the hybrid switches to at low
 *    accuracy ("Hybrid treecode/FMM algorithm"), on the same tree and lists;
 *  - targets that differ from the sources: a target tree and a source tree
 *    in one cube, traversed as a pair ("Dual tree traversal").
 *
 * Readings taken where the paper is silent are listed in the design notes
 * and repeated at each function.  Every floating-point value is IEEE FP64;
 * the file is compiled with -ffp-contract=off so that no product is fused.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* threads the OpenMP loops of the oracle use */
int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* set that count (n >= 1) */
void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

#define ORA_MAXLEVEL 21
#define ORA_PMAX 40

/* ------------------------------------------------------------------ */
/* Direct summation: the plain definition.                             */
/* phi_i = sum_{j != i, x_j != x_i} q_j / |x_i - x_j|                  */
/* E_i   = sum_{j != i, x_j != x_i} q_j (x_i - x_j) / |x_i - x_j|^3    */
/* (no 1/4pi, no softening; coincident points contribute nothing)      */
/* ------------------------------------------------------------------ */
void ora_direct(int64_t n, const double *x, const double *y, const double *z,
                const double *q, int64_t nt, const int64_t *tgt,
                double *phi, double *ex, double *ey, double *ez)
{
    int64_t a;
#pragma omp parallel for schedule(dynamic, 16)
    for (a = 0; a < nt; a++) {
        int64_t i = tgt[a];
        double p = 0, fx = 0, fy = 0, fz = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            p += q[j] / r;
            double f = q[j] / (r2 * r);
            fx += f * dx; fy += f * dy; fz += f * dz;
        }
        phi[a] = p; ex[a] = fx; ey[a] = fy; ez[a] = fz;
    }
}

/* Direct summation from an explicit source set to explicit target points. */
void ora_direct_st(int64_t ns, const double *sx, const double *sy, const double *sz,
                   const double *sq, int64_t nt, const double *tx, const double *ty,
                   const double *tz, double *phi, double *ex, double *ey, double *ez)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < nt; i++) {
        double p = 0, fx = 0, fy = 0, fz = 0;
        for (int64_t j = 0; j < ns; j++) {
            double dx = tx[i] - sx[j], dy = ty[i] - sy[j], dz = tz[i] - sz[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            p += sq[j] / r;
            double f = sq[j] / (r2 * r);
            fx += f * dx; fy += f * dy; fz += f * dz;
        }
        phi[i] = p; ex[i] = fx; ey[i] = fy; ez[i] = fz;
    }
}

/* ------------------------------------------------------------------ */
/* Morton keys.  Bounding cube anchored at the minimum corner with     */
/* side = the largest extent (1 if every point coincides); each        */
/* coordinate is quantised to 21 bits as                               */
/*   q_d = min(2^21 - 1, floor((x_d - lo_d) * (2^21 / side)))          */
/* with one FP64 subtraction then one FP64 multiplication, and the key */
/* interleaves x into bit 3b, y into 3b+1, z into 3b+2.                */
/* ------------------------------------------------------------------ */
void ora_bbox(int64_t n, const double *x, const double *y, const double *z,
              double *lo3, double *side)
{
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    const double *c[3] = {x, y, z};
    if (n > 0)
        for (int d = 0; d < 3; d++) { lo[d] = c[d][0]; hi[d] = c[d][0]; }
    for (int64_t i = 0; i < n; i++)
        for (int d = 0; d < 3; d++) {
            if (c[d][i] < lo[d]) lo[d] = c[d][i];
            if (c[d][i] > hi[d]) hi[d] = c[d][i];
        }
    double s = 0.0;
    for (int d = 0; d < 3; d++) {
        double e = hi[d] - lo[d];
        if (e > s) s = e;
    }
    if (s == 0.0) s = 1.0;
    for (int d = 0; d < 3; d++) lo3[d] = lo[d];
    *side = s;
}

static uint64_t quantise(double v, double lo, double scale)
{
    double t = (v - lo) * scale;
    double f = floor(t);
    uint64_t qv = (f <= 0.0) ? 0 : (uint64_t)f;
    if (qv > (1u << 21) - 1) qv = (1u << 21) - 1;
    return qv;
}

uint64_t ora_interleave(uint64_t qx, uint64_t qy, uint64_t qz)
{
    uint64_t k = 0;
    for (int b = 0; b < 21; b++) {
        k |= ((qx >> b) & 1ull) << (3 * b);
        k |= ((qy >> b) & 1ull) << (3 * b + 1);
        k |= ((qz >> b) & 1ull) << (3 * b + 2);
    }
    return k;
}

void ora_morton(int64_t n, const double *x, const double *y, const double *z,
                const double *lo3, double side, uint64_t *key)
{
    double scale = 2097152.0 / side; /* 2^21 / side */
    for (int64_t i = 0; i < n; i++)
        key[i] = ora_interleave(quantise(x[i], lo3[0], scale),
                                quantise(y[i], lo3[1], scale),
                                quantise(z[i], lo3[2], scale));
}

/* ------------------------------------------------------------------ */
/* Sort: ascending by (key, original index).                           */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t key; int64_t idx; int seg; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *u = (const kv_t *)a, *v = (const kv_t *)b;
    if (u->seg != v->seg) return u->seg < v->seg ? -1 : 1;
    if (u->key < v->key) return -1;
    if (u->key > v->key) return 1;
    return (u->idx < v->idx) ? -1 : (u->idx > v->idx);
}

/* ------------------------------------------------------------------ */
/* Tree and handle                                                     */
/* ------------------------------------------------------------------ */
typedef struct { int32_t t, s; } pair_t;
typedef struct { pair_t *v; int64_t n, cap; } plist_t;

static void pl_push(plist_t *l, int32_t t, int32_t s)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 1024;
        l->v = (pair_t *)realloc(l->v, (size_t)l->cap * sizeof(pair_t));
    }
    l->v[l->n].t = t; l->v[l->n].s = s; l->n++;
}

enum { K_M2L = 0, K_M2P = 1, K_P2P = 2 };
enum { POL_FMM = 0, POL_TREECODE = 1, POL_HYBRID = 2 };

typedef struct {
    int64_t n;
    int64_t nt;       /* targets != sources: particles [0, nt) of the input are the targets, the rest the
                         sources (two trees in one cube); -1 when targets and sources are the same set */
    double lo[3], side;
    uint64_t *skey;   /* sorted keys */
    int64_t *perm;    /* perm[k] = original index of the k-th sorted particle */
    double *px, *py, *pz; /* sorted positions */
    /* cells, breadth-first order (level, then key) */
    int64_t ncell, ccap;
    int32_t *level, *begin, *end, *parent, *first_child, *nchild;
    uint64_t *prefix;
    int64_t *ch;      /* half-grid centre, 3 per cell */
    int64_t *rh;      /* half-grid radius (half side) */
    double *cphys;    /* physical centre, 3 per cell */
    double *rphys;    /* physical radius (half side) */
    /* interaction lists */
    plist_t list[3];
    /* expansions after evaluate (full m = -n..n storage) */
    int p;
    cplx *M, *L;
    /* Cartesian expansions after ora_evaluate_cart */
    int pc;
    double *Mc, *Lc;
} ora_t;

static void grow_cells(ora_t *h)
{
    if (h->ncell < h->ccap) return;
    int64_t c = h->ccap ? 2 * h->ccap : 1024;
    h->level = (int32_t *)realloc(h->level, c * sizeof(int32_t));
    h->begin = (int32_t *)realloc(h->begin, c * sizeof(int32_t));
    h->end = (int32_t *)realloc(h->end, c * sizeof(int32_t));
    h->parent = (int32_t *)realloc(h->parent, c * sizeof(int32_t));
    h->first_child = (int32_t *)realloc(h->first_child, c * sizeof(int32_t));
    h->nchild = (int32_t *)realloc(h->nchild, c * sizeof(int32_t));
    h->prefix = (uint64_t *)realloc(h->prefix, c * sizeof(uint64_t));
    h->ccap = c;
}

/* digit of a key at level L (1..21): bits [3(21-L), 3(21-L)+3) */
static int key_digit(uint64_t key, int L) { return (int)((key >> (3 * (21 - L))) & 7u); }

/* de-interleave the 3L-bit prefix of a level-L cell into grid anchors */
static void prefix_anchor(uint64_t prefix, int L, int64_t a[3])
{
    a[0] = a[1] = a[2] = 0;
    for (int b = 0; b < L; b++) {
        a[0] |= (int64_t)((prefix >> (3 * b)) & 1u) << b;
        a[1] |= (int64_t)((prefix >> (3 * b + 1)) & 1u) << b;
        a[2] |= (int64_t)((prefix >> (3 * b + 2)) & 1u) << b;
    }
}

/*
 * Build: bounding cube, keys, sort, adaptive octree.
 * A cell at level l < 21 holding more than ncrit particles splits into its
 * non-empty octants (runs of equal 3(l+1)-bit key prefix), children in
 * octant order; a cell at level 21 never splits.  Cells are numbered in
 * breadth-first order, which is (level, key) order.
 */
static void *build_core(int64_t n, const double *x, const double *y, const double *z, int32_t ncrit, int64_t nt)
{
    ora_t *h = (ora_t *)calloc(1, sizeof(ora_t));
    h->n = n;
    h->nt = nt;
    ora_bbox(n, x, y, z, h->lo, &h->side);
    uint64_t *key = (uint64_t *)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    ora_morton(n, x, y, z, h->lo, h->side, key);
    kv_t *kv = (kv_t *)malloc((size_t)(n ? n : 1) * sizeof(kv_t));
    for (int64_t i = 0; i < n; i++) { kv[i].key = key[i]; kv[i].idx = i; kv[i].seg = (nt >= 0 && i >= nt); }
    qsort(kv, (size_t)n, sizeof(kv_t), kv_cmp);
    h->skey = key;
    h->perm = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    h->px = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    h->py = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    h->pz = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    for (int64_t k = 0; k < n; k++) {
        h->skey[k] = kv[k].key;
        h->perm[k] = kv[k].idx;
        h->px[k] = x[kv[k].idx]; h->py[k] = y[kv[k].idx]; h->pz[k] = z[kv[k].idx];
    }
    free(kv);

    h->ncell = 0;
    /* one root per non-empty set: the whole set, or the targets then the sources */
    int64_t seg[3] = {0, nt >= 0 ? nt : n, n};
    int nseg = nt >= 0 ? 2 : 1;
    for (int g = 0; g < nseg; g++) {
        if (seg[g + 1] == seg[g]) continue;
        grow_cells(h);
        int64_t r = h->ncell++;
        h->level[r] = 0; h->begin[r] = (int32_t)seg[g]; h->end[r] = (int32_t)seg[g + 1]; h->parent[r] = -1;
        h->prefix[r] = 0; h->first_child[r] = -1; h->nchild[r] = 0;
    }
    if (h->ncell > 0) {
        for (int64_t c = 0; c < h->ncell; c++) {
            int L = h->level[c];
            int32_t b = h->begin[c], e = h->end[c];
            if (e - b <= ncrit || L >= ORA_MAXLEVEL) continue;
            int32_t i = b;
            h->first_child[c] = (int32_t)h->ncell;
            while (i < e) {
                int d = key_digit(h->skey[i], L + 1);
                int32_t j = i;
                while (j < e && key_digit(h->skey[j], L + 1) == d) j++;
                grow_cells(h);
                int64_t k = h->ncell++;
                h->level[k] = L + 1; h->begin[k] = i; h->end[k] = j; h->parent[k] = (int32_t)c;
                h->prefix[k] = (h->prefix[c] << 3) | (uint64_t)d;
                h->first_child[k] = -1; h->nchild[k] = 0;
                h->nchild[c]++;
                i = j;
            }
        }
    }
    /* geometry: half-grid units (one unit = side / 2^22) */
    int64_t nc = h->ncell ? h->ncell : 1;
    h->ch = (int64_t *)malloc(3 * nc * sizeof(int64_t));
    h->rh = (int64_t *)malloc(nc * sizeof(int64_t));
    h->cphys = (double *)malloc(3 * nc * sizeof(double));
    h->rphys = (double *)malloc(nc * sizeof(double));
    for (int64_t c = 0; c < h->ncell; c++) {
        int L = h->level[c];
        int64_t a[3];
        prefix_anchor(h->prefix[c], L, a);
        int64_t r = (int64_t)1 << (21 - L);
        h->rh[c] = r;
        for (int d = 0; d < 3; d++) {
            h->ch[3 * c + d] = (2 * a[d] + 1) * r;
            h->cphys[3 * c + d] = h->lo[d] + (double)h->ch[3 * c + d] * (h->side / 4194304.0);
        }
        h->rphys[c] = (double)r * (h->side / 4194304.0);
    }
    return h;
}

void *ora_build(int64_t n, const double *x, const double *y, const double *z, int32_t ncrit)
{
    return build_core(n, x, y, z, ncrit, -1);
}

/*
 * Targets and sources that differ ("Dual tree traversal": the traversal pairs
 * a target tree with a source tree): particles [0, nt) of x, y, z are the
 * targets and [nt, n) the sources.  Both trees share one bounding cube (that
 * of all points), so their cells compare geometrically; each set is sorted
 * and split on its own (targets first), cell 0 is the target root and the
 * next root the source root.
 */
void *ora_build_ts(int64_t n, const double *x, const double *y, const double *z, int64_t nt, int32_t ncrit)
{
    return build_core(n, x, y, z, ncrit, nt);
}

int64_t ora_ncells(void *hv) { return ((ora_t *)hv)->ncell; }

void ora_get_bbox(void *hv, double *lo3, double *side)
{
    ora_t *h = (ora_t *)hv;
    for (int d = 0; d < 3; d++) lo3[d] = h->lo[d];
    *side = h->side;
}

void ora_get_keys(void *hv, uint64_t *skey, int64_t *perm)
{
    ora_t *h = (ora_t *)hv;
    memcpy(skey, h->skey, (size_t)h->n * sizeof(uint64_t));
    memcpy(perm, h->perm, (size_t)h->n * sizeof(int64_t));
}

void ora_get_cells(void *hv, int32_t *level, uint64_t *prefix, int32_t *begin, int32_t *end,
                   int32_t *parent, int32_t *first_child, int32_t *nchild,
                   int64_t *centre_h, int64_t *radius_h, double *centre, double *radius)
{
    ora_t *h = (ora_t *)hv;
    size_t c = (size_t)h->ncell;
    memcpy(level, h->level, c * 4); memcpy(prefix, h->prefix, c * 8);
    memcpy(begin, h->begin, c * 4); memcpy(end, h->end, c * 4);
    memcpy(parent, h->parent, c * 4); memcpy(first_child, h->first_child, c * 4);
    memcpy(nchild, h->nchild, c * 4);
    memcpy(centre_h, h->ch, 3 * c * 8); memcpy(radius_h, h->rh, c * 8);
    memcpy(centre, h->cphys, 3 * c * 8); memcpy(radius, h->rphys, c * 8);
}

/* ------------------------------------------------------------------ */
/* Dual tree traversal ("Dual tree traversal"; MAC from "Results").    */
/* ------------------------------------------------------------------ */
enum { C_ACCEPT = 0, C_P2P = 1, C_SPLIT = 2 };

static int is_leaf(const ora_t *h, int32_t c) { return h->nchild[c] == 0; }

/* accept iff (r_t + r_s)^2 <= theta^2 R^2, with integer half-grid radii and
 * squared centre distance; theta^2 is one FP64 product made once and the
 * right side is one FP64 product.  Equality accepts.  A pair that fails and
 * whose cells are both leaves is a particle-particle interaction. */
static int classify(const ora_t *h, int32_t t, int32_t s, double theta2)
{
    int64_t R2 = 0;
    for (int d = 0; d < 3; d++) {
        int64_t dd = h->ch[3 * t + d] - h->ch[3 * s + d];
        R2 += dd * dd;
    }
    int64_t rr = h->rh[t] + h->rh[s];
    if ((double)(rr * rr) <= theta2 * (double)R2) return C_ACCEPT;
    if (is_leaf(h, t) && is_leaf(h, s)) return C_P2P;
    return C_SPLIT;
}

/* choice among cell-cell (M2L), cell-particle (M2P) and particle-particle
 * (P2P) for an accepted pair.  The hybrid compares modelled times made of
 * unit costs: c_m2l, c_m2p * n_t, (c_p2p * n_t) * n_s; the smallest wins and
 * ties go to the earlier of M2L, M2P, P2P. */
/* Learned choice (policy 3): the kind the cost model picks for the pair's
 * quantised features, read from a choice table of 9 x 81 x 81 x 4 entries:
 * level difference l_s - l_t clamped to [-4, 4]; round(4 log2 n) clamped to
 * [0, 80] for n_t and n_s; floor(4 ((r_t + r_s)/R)/theta) clamped to [0, 3]. */
static const uint8_t *g_table = 0;
static double g_theta = 0;

static int table_choice(const ora_t *h, int32_t t, int32_t s)
{
    int dl = h->level[s] - h->level[t];
    dl = dl < -4 ? -4 : (dl > 4 ? 4 : dl);
    double nt = (double)(h->end[t] - h->begin[t]);
    double ns = (double)(h->end[s] - h->begin[s]);
    int bt = (int)rint(4.0 * log2(nt)), bs = (int)rint(4.0 * log2(ns));
    bt = bt < 0 ? 0 : (bt > 80 ? 80 : bt);
    bs = bs < 0 ? 0 : (bs > 80 ? 80 : bs);
    int64_t R2 = 0;
    for (int d = 0; d < 3; d++) {
        int64_t dd = h->ch[3 * t + d] - h->ch[3 * s + d];
        R2 += dd * dd;
    }
    int64_t rr = h->rh[t] + h->rh[s];
    double ratio = sqrt((double)(rr * rr) / (double)R2) / g_theta;
    int bq = (int)(ratio * 4);
    bq = bq < 0 ? 0 : (bq > 3 ? 3 : bq);
    return g_table[(((dl + 4) * 81 + bt) * 81 + bs) * 4 + bq];
}

static int choose(const ora_t *h, int32_t t, int32_t s, int policy, const double *costs)
{
    if (policy == POL_FMM) return K_M2L;
    if (policy == POL_TREECODE) return K_M2P;
    if (policy == 3) return table_choice(h, t, s);
    double nt = (double)(h->end[t] - h->begin[t]);
    double ns = (double)(h->end[s] - h->begin[s]);
    double c0 = costs[0];
    double c1 = costs[1] * nt;
    double c2 = (costs[2] * nt) * ns;
    int k = K_M2L;
    double best = c0;
    if (c1 < best) { best = c1; k = K_M2P; }
    if (c2 < best) { best = c2; k = K_P2P; }
    return k;
}

void ora_traverse(void *hv, double theta, int policy, const double *costs)
{
    ora_t *h = (ora_t *)hv;
    for (int k = 0; k < 3; k++) h->list[k].n = 0;
    if (h->ncell == 0) return;
    double theta2 = theta * theta;
    plist_t stack = {0, 0, 0};
    /* the root pair (target root, source root) is treated as a newly formed
     * pair; with separate sets it exists only when both are non-empty */
    int32_t rt = 0, rs = 0;
    if (h->nt >= 0) {
        if (h->nt == 0 || h->nt == h->n) return;
        rs = 1;
    }
    int c0 = classify(h, rt, rs, theta2);
    if (c0 == C_P2P) pl_push(&h->list[K_P2P], rt, rs);
    else if (c0 == C_SPLIT) pl_push(&stack, rt, rs);
    while (stack.n > 0) {
        pair_t pr = stack.v[--stack.n];
        int32_t T = pr.t, S = pr.s;
        /* split the larger cell; equal sizes split both */
        int splitT = !is_leaf(h, T) && (is_leaf(h, S) || h->level[T] <= h->level[S]);
        int splitS = !is_leaf(h, S) && (is_leaf(h, T) || h->level[S] <= h->level[T]);
        int32_t t0 = splitT ? h->first_child[T] : T;
        int32_t t1 = splitT ? h->first_child[T] + h->nchild[T] : T + 1;
        int32_t s0 = splitS ? h->first_child[S] : S;
        int32_t s1 = splitS ? h->first_child[S] + h->nchild[S] : S + 1;
        for (int32_t t = t0; t < t1; t++)
            for (int32_t s = s0; s < s1; s++) {
                int c = classify(h, t, s, theta2);
                if (c == C_ACCEPT) pl_push(&h->list[choose(h, t, s, policy, costs)], t, s);
                else if (c == C_P2P) pl_push(&h->list[K_P2P], t, s);
                else pl_push(&stack, t, s);
            }
    }
    free(stack.v);
}

int64_t ora_list_size(void *hv, int kind) { return ((ora_t *)hv)->list[kind].n; }

void ora_get_list(void *hv, int kind, int32_t *t, int32_t *s)
{
    ora_t *h = (ora_t *)hv;
    for (int64_t i = 0; i < h->list[kind].n; i++) {
        t[i] = h->list[kind].v[i].t;
        s[i] = h->list[kind].v[i].s;
    }
}

/* ------------------------------------------------------------------ */
/* Spherical harmonics and Greengard-Rokhlin expansions.               */
/*  Y_n^m(a, b) = sqrt((n-|m|)!/(n+|m|)!) P_n^|m|(cos a) e^{i m b}     */
/*  with P_n^m(x) = (1-x^2)^{m/2} d^m/dx^m P_n(x) (no Condon-Shortley   */
/*  phase).  A_n^m = (-1)^n / sqrt((n-m)!(n+m)!).                       */
/*  Coefficient arrays hold all m = -n..n at index n*n + n + m.         */
/* ------------------------------------------------------------------ */
static double FACT[171];
static double ATAB[2 * ORA_PMAX + 2][2 * ORA_PMAX + 2];
static int fact_ready = 0;

/* factorials and the table of A_n^m = (-1)^n / sqrt((n-m)!(n+m)!), 0 <= m <= n */
static void init_fact(void)
{
    if (fact_ready) return;
    FACT[0] = 1.0;
    for (int k = 1; k <= 170; k++) FACT[k] = FACT[k - 1] * (double)k;
    for (int n = 0; n <= 2 * ORA_PMAX + 1; n++)
        for (int m = 0; m <= n; m++)
            ATAB[n][m] = ((n & 1) ? -1.0 : 1.0) / sqrt(FACT[n - m] * FACT[n + m]);
    fact_ready = 1;
}

static inline int cidx(int n, int m) { return n * n + n + m; }

static inline double Anm(int n, int m) { return ATAB[n][m]; }

__attribute__((constructor)) static void ora_init(void) { init_fact(); }

static cplx ipow(int e)
{
    int r = ((e % 4) + 4) % 4;
    if (r == 0) return 1.0;
    if (r == 1) return I;
    if (r == 2) return -1.0;
    return -I;
}

/* spherical coordinates of a vector: rho, polar angle alpha, azimuth beta */
static void sph(double dx, double dy, double dz, double *rho, double *alpha, double *beta)
{
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    *rho = r;
    if (r == 0.0) { *alpha = 0.0; *beta = 0.0; return; }
    double c = dz / r;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    *alpha = acos(c);
    *beta = atan2(dy, dx);
}

/* Y_n^m(alpha, beta) for n = 0..P, all m; out has (P+1)^2 entries. */
void ora_ylm(int P, double alpha, double beta, cplx *Y)
{
    init_fact();
    double x = cos(alpha), s = sin(alpha);
    double Pnm[ORA_PMAX * 2 + 2][ORA_PMAX * 2 + 2];
    /* associated Legendre functions without the Condon-Shortley phase */
    Pnm[0][0] = 1.0;
    for (int m = 1; m <= P; m++) Pnm[m][m] = (double)(2 * m - 1) * s * Pnm[m - 1][m - 1];
    for (int m = 0; m < P; m++) Pnm[m + 1][m] = x * (double)(2 * m + 1) * Pnm[m][m];
    for (int m = 0; m <= P; m++)
        for (int n = m + 2; n <= P; n++)
            Pnm[n][m] = ((double)(2 * n - 1) * x * Pnm[n - 1][m] - (double)(n + m - 1) * Pnm[n - 2][m]) /
                        (double)(n - m);
    for (int n = 0; n <= P; n++)
        for (int m = -n; m <= n; m++) {
            int am = m < 0 ? -m : m;
            double nrm = sqrt(FACT[n - am] / FACT[n + am]);
            Y[cidx(n, m)] = nrm * Pnm[n][am] * cexp(I * (double)m * beta);
        }
}

/* Multipole expansion (Greengard-Rokhlin theorem 3.2):
 *   M_n^m = sum_i q_i rho_i^n Y_n^{-m}(alpha_i, beta_i)
 * about centre c, for n = 0..p. */
void ora_p2m(int p, const double *c, int64_t k, const double *x, const double *y,
             const double *z, const double *q, cplx *M)
{
    init_fact();
    int K = (p + 1) * (p + 1);
    cplx Y[(ORA_PMAX + 1) * (ORA_PMAX + 1)];
    for (int a = 0; a < K; a++) M[a] = 0;
    for (int64_t i = 0; i < k; i++) {
        double rho, al, be;
        sph(x[i] - c[0], y[i] - c[1], z[i] - c[2], &rho, &al, &be);
        ora_ylm(p, al, be, Y);
        double rn = 1.0;
        for (int n = 0; n <= p; n++) {
            for (int m = -n; m <= n; m++) M[cidx(n, m)] += q[i] * rn * Y[cidx(n, -m)];
            rn *= rho;
        }
    }
}

/* Translation of a multipole expansion (theorem 3.3).  Q = (old centre) -
 * (new centre).  Adds into Mout:
 *   M_j^k = sum_{n=0}^{j} sum_{m} O_{j-n}^{k-m} i^{|k|-|m|-|k-m|}
 *           A_n^m A_{j-n}^{k-m} rho^n Y_n^{-m}(alpha, beta) / A_j^k      */
void ora_m2m(int p, const cplx *O, const double *Q, cplx *Mout)
{
    init_fact();
    double rho, al, be;
    sph(Q[0], Q[1], Q[2], &rho, &al, &be);
    cplx Y[(ORA_PMAX + 1) * (ORA_PMAX + 1)];
    ora_ylm(p, al, be, Y);
    for (int j = 0; j <= p; j++)
        for (int k = -j; k <= j; k++) {
            cplx acc = 0;
            for (int n = 0; n <= j; n++) {
                double rn = pow(rho, n);
                for (int m = -n; m <= n; m++) {
                    int km = k - m;
                    if (km < -(j - n) || km > (j - n)) continue;
                    int e = abs(k) - abs(m) - abs(km);
                    acc += O[cidx(j - n, km)] * ipow(e) * Anm(n, abs(m)) * Anm(j - n, abs(km)) * rn *
                           Y[cidx(n, -m)] / Anm(j, abs(k));
                }
            }
            Mout[cidx(j, k)] += acc;
        }
}

/* Conversion of a multipole expansion into a local expansion (theorem 3.4).
 * Q = (source centre) - (target centre).  Adds into Lout for j = 0..pl:
 *   L_j^k = sum_{n=0}^{p} sum_m O_n^m i^{|k-m|-|k|-|m|} A_n^m A_j^k
 *           Y_{j+n}^{m-k}(alpha, beta) / ((-1)^n A_{j+n}^{m-k} rho^{j+n+1}) */
void ora_m2l(int p, int pl, const cplx *O, const double *Q, cplx *Lout)
{
    init_fact();
    double rho, al, be;
    sph(Q[0], Q[1], Q[2], &rho, &al, &be);
    int P2 = p + pl;
    cplx Y[(2 * ORA_PMAX + 1) * (2 * ORA_PMAX + 1)];
    ora_ylm(P2, al, be, Y);
    for (int j = 0; j <= pl; j++)
        for (int k = -j; k <= j; k++) {
            cplx acc = 0;
            for (int n = 0; n <= p; n++) {
                double sgn = (n & 1) ? -1.0 : 1.0;
                double rpow = pow(rho, j + n + 1);
                for (int m = -n; m <= n; m++) {
                    int mk = m - k;
                    int e = abs(k - m) - abs(k) - abs(m);
                    acc += O[cidx(n, m)] * ipow(e) * Anm(n, abs(m)) * Anm(j, abs(k)) *
                           Y[cidx(j + n, mk)] / (sgn * Anm(j + n, abs(mk)) * rpow);
                }
            }
            Lout[cidx(j, k)] += acc;
        }
}

/* Translation of a local expansion (theorem 3.5).  Q = (old centre) -
 * (new centre).  Adds into Lout for j = 0..pl:
 *   L_j^k = sum_{n=j}^{p} sum_m O_n^m i^{|m|-|m-k|-|k|} A_{n-j}^{m-k} A_j^k
 *           Y_{n-j}^{m-k}(alpha, beta) rho^{n-j} / ((-1)^{n+j} A_n^m)       */
void ora_l2l(int p, int pl, const cplx *O, const double *Q, cplx *Lout)
{
    init_fact();
    double rho, al, be;
    sph(Q[0], Q[1], Q[2], &rho, &al, &be);
    cplx Y[(ORA_PMAX + 1) * (ORA_PMAX + 1)];
    ora_ylm(p, al, be, Y);
    for (int j = 0; j <= pl; j++)
        for (int k = -j; k <= j; k++) {
            cplx acc = 0;
            for (int n = j; n <= p; n++) {
                double sgn = ((n + j) & 1) ? -1.0 : 1.0;
                double rn = pow(rho, n - j);
                for (int m = -n; m <= n; m++) {
                    int mk = m - k;
                    if (mk < -(n - j) || mk > (n - j)) continue;
                    int e = abs(m) - abs(mk) - abs(k);
                    acc += O[cidx(n, m)] * ipow(e) * Anm(n - j, abs(mk)) * Anm(j, abs(k)) *
                           Y[cidx(n - j, mk)] * rn / (sgn * Anm(n, abs(m)));
                }
            }
            Lout[cidx(j, k)] += acc;
        }
}

/* Value and gradient read off a local expansion of degree >= 1 about the
 * evaluation point: phi = L_0^0; with rho Y_1^0 = z and
 * rho Y_1^{+-1} = (x +- i y)/sqrt(2), grad phi = (Re(L_1^1 + L_1^-1)/sqrt2,
 * Re(i (L_1^1 - L_1^-1))/sqrt2, Re L_1^0).  Field E = -grad phi. */
static void read_point(const cplx *Lp, double *phi, double *e)
{
    double r2 = sqrt(0.5);
    *phi = creal(Lp[cidx(0, 0)]);
    e[0] = -creal(Lp[cidx(1, 1)] + Lp[cidx(1, -1)]) * r2;
    e[1] = -creal(I * (Lp[cidx(1, 1)] - Lp[cidx(1, -1)])) * r2;
    e[2] = -creal(Lp[cidx(1, 0)]);
}

/* Local expansion about c evaluated at point x: the expansion is re-centred
 * at x (theorem 3.5, exact for a polynomial) and value and gradient are read
 * off its degree-0 and degree-1 terms.  Avoids any division by sin(alpha). */
void ora_l2p(int p, const cplx *L, const double *c, const double *x, double *phi, double *e)
{
    cplx Lp[4] = {0, 0, 0, 0};
    double Q[3] = {c[0] - x[0], c[1] - x[1], c[2] - x[2]};
    ora_l2l(p, 1, L, Q, Lp);
    read_point(Lp, phi, e);
}

/* Multipole expansion about c evaluated at point x: converted into a local
 * expansion of degree 1 about x (theorem 3.4) and read off. */
void ora_m2p(int p, const cplx *M, const double *c, const double *x, double *phi, double *e)
{
    cplx Lp[4] = {0, 0, 0, 0};
    double Q[3] = {c[0] - x[0], c[1] - x[1], c[2] - x[2]};
    ora_m2l(p, 1, M, Q, Lp);
    read_point(Lp, phi, e);
}

/* The series definitions, value only, for cross-checks:
 *   multipole: sum M_n^m Y_n^m(theta, phi) / r^{n+1};  local: sum L_j^k Y_j^k r^j */
double ora_mp_series(int p, const cplx *M, const double *c, const double *x)
{
    double r, a, b;
    sph(x[0] - c[0], x[1] - c[1], x[2] - c[2], &r, &a, &b);
    cplx Y[(ORA_PMAX + 1) * (ORA_PMAX + 1)];
    ora_ylm(p, a, b, Y);
    cplx acc = 0;
    for (int n = 0; n <= p; n++)
        for (int m = -n; m <= n; m++) acc += M[cidx(n, m)] * Y[cidx(n, m)] / pow(r, n + 1);
    return creal(acc);
}

double ora_local_series(int p, const cplx *L, const double *c, const double *x)
{
    double r, a, b;
    sph(x[0] - c[0], x[1] - c[1], x[2] - c[2], &r, &a, &b);
    cplx Y[(ORA_PMAX + 1) * (ORA_PMAX + 1)];
    ora_ylm(p, a, b, Y);
    cplx acc = 0;
    for (int n = 0; n <= p; n++)
        for (int m = -n; m <= n; m++) acc += L[cidx(n, m)] * Y[cidx(n, m)] * pow(r, n);
    return creal(acc);
}

/* ------------------------------------------------------------------ */
/* Full evaluation over the lists: P2M at leaves, M2M upward, M2L,     */
/* L2L downward, then per target particle L2P + M2P + P2P.             */
/* Charges q and outputs are in the caller's original particle order. */
/* ------------------------------------------------------------------ */
typedef struct { int64_t *off; int32_t *src; } csr_t;

static void build_csr(const ora_t *h, const plist_t *l, csr_t *c)
{
    int64_t nc = h->ncell;
    c->off = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    c->src = (int32_t *)malloc((size_t)(l->n ? l->n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < l->n; i++) c->off[l->v[i].t + 1]++;
    for (int64_t i = 0; i < nc; i++) c->off[i + 1] += c->off[i];
    int64_t *fill = (int64_t *)malloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    memcpy(fill, c->off, (size_t)nc * sizeof(int64_t));
    for (int64_t i = 0; i < l->n; i++) c->src[fill[l->v[i].t]++] = l->v[i].s;
    free(fill);
}

void ora_evaluate(void *hv, int p, const double *q, double *phi, double *ex, double *ey, double *ez)
{
    ora_t *h = (ora_t *)hv;
    init_fact();
    int64_t n = h->n, nc = h->ncell;
    int K = (p + 1) * (p + 1);
    h->p = p;
    free(h->M); free(h->L);
    h->M = (cplx *)calloc((size_t)(nc ? nc : 1) * K, sizeof(cplx));
    h->L = (cplx *)calloc((size_t)(nc ? nc : 1) * K, sizeof(cplx));
    if (n == 0) return;
    /* with separate sets, q holds the sources' charges (targets carry none)
     * and the outputs are the targets' */
    const int64_t nt = h->nt;
    double *sq = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t k = 0; k < n; k++) {
        int64_t o = h->perm[k];
        sq[k] = nt < 0 ? q[o] : (o < nt ? 0.0 : q[o - nt]);
    }
    const int64_t nout = nt < 0 ? n : nt;  /* sorted positions [0, nout) are the targets */

    /* P2M at every leaf */
    int64_t c;
#pragma omp parallel for schedule(dynamic, 4)
    for (c = 0; c < nc; c++) {
        if (!is_leaf(h, (int32_t)c)) continue;
        int32_t b = h->begin[c], e = h->end[c];
        ora_p2m(p, &h->cphys[3 * c], e - b, h->px + b, h->py + b, h->pz + b, sq + b, h->M + c * K);
    }
    /* M2M bottom-up: a parent sums its children (cells with higher ids come later in BFS) */
    int maxl = 0;
    for (c = 0; c < nc; c++) if (h->level[c] > maxl) maxl = h->level[c];
    for (int L = maxl - 1; L >= 0; L--) {
#pragma omp parallel for schedule(dynamic, 4)
        for (c = 0; c < nc; c++) {
            if (h->level[c] != L || is_leaf(h, (int32_t)c)) continue;
            for (int32_t ch = h->first_child[c]; ch < h->first_child[c] + h->nchild[c]; ch++) {
                double Q[3] = {h->cphys[3 * ch] - h->cphys[3 * c], h->cphys[3 * ch + 1] - h->cphys[3 * c + 1],
                               h->cphys[3 * ch + 2] - h->cphys[3 * c + 2]};
                ora_m2m(p, h->M + (int64_t)ch * K, Q, h->M + c * K);
            }
        }
    }
    /* M2L into every target cell */
    csr_t cm2l, cm2p, cp2p;
    build_csr(h, &h->list[K_M2L], &cm2l);
    build_csr(h, &h->list[K_M2P], &cm2p);
    build_csr(h, &h->list[K_P2P], &cp2p);
#pragma omp parallel for schedule(dynamic, 4)
    for (c = 0; c < nc; c++) {
        for (int64_t a = cm2l.off[c]; a < cm2l.off[c + 1]; a++) {
            int32_t s = cm2l.src[a];
            double Q[3] = {h->cphys[3 * s] - h->cphys[3 * c], h->cphys[3 * s + 1] - h->cphys[3 * c + 1],
                           h->cphys[3 * s + 2] - h->cphys[3 * c + 2]};
            ora_m2l(p, p, h->M + (int64_t)s * K, Q, h->L + c * K);
        }
    }
    /* L2L top-down: each child adds its parent's complete local expansion */
    for (int L = 1; L <= maxl; L++) {
#pragma omp parallel for schedule(dynamic, 4)
        for (c = 0; c < nc; c++) {
            if (h->level[c] != L) continue;
            int32_t P = h->parent[c];
            double Q[3] = {h->cphys[3 * P] - h->cphys[3 * c], h->cphys[3 * P + 1] - h->cphys[3 * c + 1],
                           h->cphys[3 * P + 2] - h->cphys[3 * c + 2]};
            ora_l2l(p, p, h->L + (int64_t)P * K, Q, h->L + c * K);
        }
    }
    /* leaf of every sorted particle */
    int32_t *leaf = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (c = 0; c < nc; c++)
        if (is_leaf(h, (int32_t)c))
            for (int32_t i = h->begin[c]; i < h->end[c]; i++) leaf[i] = (int32_t)c;
    int64_t i;
#pragma omp parallel for schedule(dynamic, 64)
    for (i = 0; i < nout; i++) {
        double xi[3] = {h->px[i], h->py[i], h->pz[i]};
        int32_t t = leaf[i];
        double ph, e[3];
        ora_l2p(p, h->L + (int64_t)t * K, &h->cphys[3 * t], xi, &ph, e);
        double P = ph, F[3] = {e[0], e[1], e[2]};
        for (int32_t A = t; A >= 0; A = h->parent[A]) {
            for (int64_t a = cm2p.off[A]; a < cm2p.off[A + 1]; a++) {
                int32_t s = cm2p.src[a];
                ora_m2p(p, h->M + (int64_t)s * K, &h->cphys[3 * s], xi, &ph, e);
                P += ph; F[0] += e[0]; F[1] += e[1]; F[2] += e[2];
            }
            for (int64_t a = cp2p.off[A]; a < cp2p.off[A + 1]; a++) {
                int32_t s = cp2p.src[a];
                for (int32_t j = h->begin[s]; j < h->end[s]; j++) {
                    if (j == i) continue;
                    double dx = xi[0] - h->px[j], dy = xi[1] - h->py[j], dz = xi[2] - h->pz[j];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 == 0.0) continue;
                    double r = sqrt(r2);
                    P += sq[j] / r;
                    double f = sq[j] / (r2 * r);
                    F[0] += f * dx; F[1] += f * dy; F[2] += f * dz;
                }
            }
        }
        int64_t o = h->perm[i];
        phi[o] = P; ex[o] = F[0]; ey[o] = F[1]; ez[o] = F[2];
    }
    free(leaf); free(sq);
    free(cm2l.off); free(cm2l.src); free(cm2p.off); free(cm2p.src); free(cp2p.off); free(cp2p.src);
}

/* expansions of cell c after ora_evaluate, (p+1)^2 complex each */
void ora_get_expansions(void *hv, cplx *M, cplx *L)
{
    ora_t *h = (ora_t *)hv;
    size_t K = (size_t)(h->p + 1) * (h->p + 1);
    memcpy(M, h->M, (size_t)h->ncell * K * sizeof(cplx));
    memcpy(L, h->L, (size_t)h->ncell * K * sizeof(cplx));
}

/* ------------------------------------------------------------------ */
/* Cartesian (Taylor) expansions.  The paper's hybrid method can switch */
/* from spherical harmonics to Cartesian expansions when the required  */
/* accuracy is low ("Hybrid treecode/FMM algorithm"); treecodes use     */
/* Taylor series in Cartesian coordinates ("Introduction to treecodes   */
/* & FMM").  The paper gives no formulas; these are the plain Taylor    */
/* expansions of 1/|x - y|:                                            */
/*   a_n(R) = (1/n!) d^n/dR^n (1/|R|)   (multi-index n, n! = n1!n2!n3!) */
/*   f(R + w) = sum_n a_n(R) w^n                                        */
/* with, for |n| >= 1 (terms with a negative index dropped),            */
/*   |R|^2 a_n = -((2|n|-1)/|n|) sum_i R_i a_{n-e_i}                   */
/*              - ((|n|-1)/|n|) sum_i a_{n-2e_i},   a_0 = 1/|R|,       */
/* the Taylor-coefficient recurrence of 1/|R| (cf. Duan & Krasny, J.    */
/* Comput. Chem. 22 (2001); written here for derivatives in R).         */
/* Multipole about centre s: M_k = sum_j q_j (s - x_j)^k, |k| <= p.    */
/* Local about t: phi(t + u) = sum_m L_m u^m, |m| <= p, from           */
/*   L_m = sum_{|m|+|k|<=p} C(m,k) a_{m+k}(t - s) M_k,                 */
/*   C(m,k) = prod_i (m_i + k_i)! / (m_i! k_i!).                       */
/* Coefficients are stored in graded order: degree n = 0..p, within a  */
/* degree by k1 descending, then k2 descending.                        */
/* ------------------------------------------------------------------ */
int ora_cart_count(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int ora_cart_index(int a, int b, int c)
{
    int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

static double rpow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= x;
    return r;
}

static double binom_d(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; i++) r = r * (double)(n - k + i) / (double)i;
    return r;
}

/* a_n(R) for |n| <= P into a[ora_cart_index(n)] */
void ora_cart_taylor(int P, const double *R, double *a)
{
    double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    a[0] = 1.0 / sqrt(r2);
    for (int n = 1; n <= P; n++)
        for (int i = n; i >= 0; i--)
            for (int j = n - i; j >= 0; j--) {
                int k = n - i - j;
                int e[3] = {i, j, k};
                double s1 = 0.0, s2 = 0.0;
                for (int d = 0; d < 3; d++) {
                    if (e[d] >= 1) {
                        e[d] -= 1;
                        s1 += R[d] * a[ora_cart_index(e[0], e[1], e[2])];
                        e[d] += 1;
                    }
                    if (e[d] >= 2) {
                        e[d] -= 2;
                        s2 += a[ora_cart_index(e[0], e[1], e[2])];
                        e[d] += 2;
                    }
                }
                a[ora_cart_index(i, j, k)] = -((2.0 * n - 1.0) / n * s1 + (n - 1.0) / n * s2) / r2;
            }
}

/* P2M about c: M_k = sum_j q_j (c - x_j)^k */
void ora_cart_p2m(int p, const double *c, int64_t n, const double *x, const double *y, const double *z,
                  const double *q, double *M)
{
    int K = ora_cart_count(p);
    for (int i = 0; i < K; i++) M[i] = 0.0;
    for (int64_t j = 0; j < n; j++) {
        double v[3] = {c[0] - x[j], c[1] - y[j], c[2] - z[j]};
        for (int m = 0; m <= p; m++)
            for (int a = m; a >= 0; a--)
                for (int b = m - a; b >= 0; b--) {
                    int cc = m - a - b;
                    M[ora_cart_index(a, b, cc)] += q[j] * rpow(v[0], a) * rpow(v[1], b) * rpow(v[2], cc);
                }
    }
}

/* M2M: Mo (about s) re-centred at s' = s + d (d = new centre - old centre), added into Mn:
 * Mn_k += sum_{a <= k} binom(k, a) Mo_a d^(k - a) */
void ora_cart_m2m(int p, const double *Mo, const double *d, double *Mn)
{
    for (int n = 0; n <= p; n++)
        for (int k1 = n; k1 >= 0; k1--)
            for (int k2 = n - k1; k2 >= 0; k2--) {
                int k3 = n - k1 - k2;
                double s = 0.0;
                for (int a1 = 0; a1 <= k1; a1++)
                    for (int a2 = 0; a2 <= k2; a2++)
                        for (int a3 = 0; a3 <= k3; a3++)
                            s += binom_d(k1, a1) * binom_d(k2, a2) * binom_d(k3, a3) *
                                 Mo[ora_cart_index(a1, a2, a3)] * rpow(d[0], k1 - a1) * rpow(d[1], k2 - a2) *
                                 rpow(d[2], k3 - a3);
                Mn[ora_cart_index(k1, k2, k3)] += s;
            }
}

/* M2L: L_m += sum_{|m|+|k|<=p} C(m,k) a_{m+k}(R) M_k, R = t - s */
void ora_cart_m2l(int p, const double *M, const double *R, double *L)
{
    int K2 = ora_cart_count(p);
    double *a = (double *)malloc((size_t)K2 * sizeof(double));
    ora_cart_taylor(p, R, a);
    for (int nm = 0; nm <= p; nm++)
        for (int m1 = nm; m1 >= 0; m1--)
            for (int m2 = nm - m1; m2 >= 0; m2--) {
                int m3 = nm - m1 - m2;
                double s = 0.0;
                for (int nk = 0; nk + nm <= p; nk++)
                    for (int k1 = nk; k1 >= 0; k1--)
                        for (int k2 = nk - k1; k2 >= 0; k2--) {
                            int k3 = nk - k1 - k2;
                            double C = binom_d(m1 + k1, k1) * binom_d(m2 + k2, k2) * binom_d(m3 + k3, k3);
                            s += C * a[ora_cart_index(m1 + k1, m2 + k2, m3 + k3)] * M[ora_cart_index(k1, k2, k3)];
                        }
                L[ora_cart_index(m1, m2, m3)] += s;
            }
    free(a);
}

/* L2L: Lo (about t) re-centred at t' = t + d, added into Ln:
 * Ln_m' += sum_{m >= m'} binom(m, m') Lo_m d^(m - m') */
void ora_cart_l2l(int p, const double *Lo, const double *d, double *Ln)
{
    for (int n = 0; n <= p; n++)
        for (int a1 = n; a1 >= 0; a1--)
            for (int a2 = n - a1; a2 >= 0; a2--) {
                int a3 = n - a1 - a2;
                double s = 0.0;
                for (int nm = n; nm <= p; nm++)
                    for (int m1 = nm; m1 >= 0; m1--)
                        for (int m2 = nm - m1; m2 >= 0; m2--) {
                            int m3 = nm - m1 - m2;
                            if (m1 < a1 || m2 < a2 || m3 < a3) continue;
                            s += binom_d(m1, a1) * binom_d(m2, a2) * binom_d(m3, a3) * Lo[ora_cart_index(m1, m2, m3)] *
                                 rpow(d[0], m1 - a1) * rpow(d[1], m2 - a2) * rpow(d[2], m3 - a3);
                        }
                Ln[ora_cart_index(a1, a2, a3)] += s;
            }
}

/* L2P: phi = sum_m L_m (x - t)^m, E = -grad phi */
void ora_cart_l2p(int p, const double *L, const double *t, const double *x, double *phi, double *E)
{
    double u[3] = {x[0] - t[0], x[1] - t[1], x[2] - t[2]};
    double ph = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int n = 0; n <= p; n++)
        for (int m1 = n; m1 >= 0; m1--)
            for (int m2 = n - m1; m2 >= 0; m2--) {
                int m3 = n - m1 - m2;
                double Lm = L[ora_cart_index(m1, m2, m3)];
                ph += Lm * rpow(u[0], m1) * rpow(u[1], m2) * rpow(u[2], m3);
                if (m1 > 0) g[0] += m1 * Lm * rpow(u[0], m1 - 1) * rpow(u[1], m2) * rpow(u[2], m3);
                if (m2 > 0) g[1] += m2 * Lm * rpow(u[0], m1) * rpow(u[1], m2 - 1) * rpow(u[2], m3);
                if (m3 > 0) g[2] += m3 * Lm * rpow(u[0], m1) * rpow(u[1], m2) * rpow(u[2], m3 - 1);
            }
    *phi = ph;
    E[0] = -g[0]; E[1] = -g[1]; E[2] = -g[2];
}

/* M2P: phi = sum_k a_k(x - s) M_k, d phi/dx_i = sum_k (k_i + 1) a_{k + e_i}(x - s) M_k */
void ora_cart_m2p(int p, const double *M, const double *s, const double *x, double *phi, double *E)
{
    double R[3] = {x[0] - s[0], x[1] - s[1], x[2] - s[2]};
    double *a = (double *)malloc((size_t)ora_cart_count(p + 1) * sizeof(double));
    ora_cart_taylor(p + 1, R, a);
    double ph = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int n = 0; n <= p; n++)
        for (int k1 = n; k1 >= 0; k1--)
            for (int k2 = n - k1; k2 >= 0; k2--) {
                int k3 = n - k1 - k2;
                double Mk = M[ora_cart_index(k1, k2, k3)];
                ph += a[ora_cart_index(k1, k2, k3)] * Mk;
                g[0] += (k1 + 1) * a[ora_cart_index(k1 + 1, k2, k3)] * Mk;
                g[1] += (k2 + 1) * a[ora_cart_index(k1, k2 + 1, k3)] * Mk;
                g[2] += (k3 + 1) * a[ora_cart_index(k1, k2, k3 + 1)] * Mk;
            }
    free(a);
    *phi = ph;
    E[0] = -g[0]; E[1] = -g[1]; E[2] = -g[2];
}

/* The whole evaluation with Cartesian expansions of order p, on the same
 * tree and lists as ora_evaluate (P2M at leaves, M2M upward, M2L, L2L
 * downward, L2P + M2P + P2P per target, targets != sources as there). */
void ora_evaluate_cart(void *hv, int p, const double *q, double *phi, double *ex, double *ey, double *ez)
{
    ora_t *h = (ora_t *)hv;
    int64_t n = h->n, nc = h->ncell;
    int K = ora_cart_count(p);
    h->pc = p;
    free(h->Mc); free(h->Lc);
    h->Mc = (double *)calloc((size_t)(nc ? nc : 1) * K, sizeof(double));
    h->Lc = (double *)calloc((size_t)(nc ? nc : 1) * K, sizeof(double));
    if (n == 0) return;
    const int64_t nt = h->nt;
    double *sq = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t k = 0; k < n; k++) {
        int64_t o = h->perm[k];
        sq[k] = nt < 0 ? q[o] : (o < nt ? 0.0 : q[o - nt]);
    }
    const int64_t nout = nt < 0 ? n : nt;
    int64_t c;
#pragma omp parallel for schedule(dynamic, 4)
    for (c = 0; c < nc; c++) {
        if (!is_leaf(h, (int32_t)c)) continue;
        int32_t b = h->begin[c], e = h->end[c];
        ora_cart_p2m(p, &h->cphys[3 * c], e - b, h->px + b, h->py + b, h->pz + b, sq + b, h->Mc + c * K);
    }
    int maxl = 0;
    for (c = 0; c < nc; c++) if (h->level[c] > maxl) maxl = h->level[c];
    for (int L = maxl - 1; L >= 0; L--) {
#pragma omp parallel for schedule(dynamic, 4)
        for (c = 0; c < nc; c++) {
            if (h->level[c] != L || is_leaf(h, (int32_t)c)) continue;
            for (int32_t ch = h->first_child[c]; ch < h->first_child[c] + h->nchild[c]; ch++) {
                double d[3] = {h->cphys[3 * c] - h->cphys[3 * ch], h->cphys[3 * c + 1] - h->cphys[3 * ch + 1],
                               h->cphys[3 * c + 2] - h->cphys[3 * ch + 2]};
                ora_cart_m2m(p, h->Mc + (int64_t)ch * K, d, h->Mc + c * K);
            }
        }
    }
    csr_t cm2l, cm2p, cp2p;
    build_csr(h, &h->list[K_M2L], &cm2l);
    build_csr(h, &h->list[K_M2P], &cm2p);
    build_csr(h, &h->list[K_P2P], &cp2p);
#pragma omp parallel for schedule(dynamic, 4)
    for (c = 0; c < nc; c++) {
        for (int64_t a = cm2l.off[c]; a < cm2l.off[c + 1]; a++) {
            int32_t s = cm2l.src[a];
            double R[3] = {h->cphys[3 * c] - h->cphys[3 * s], h->cphys[3 * c + 1] - h->cphys[3 * s + 1],
                           h->cphys[3 * c + 2] - h->cphys[3 * s + 2]};
            ora_cart_m2l(p, h->Mc + (int64_t)s * K, R, h->Lc + c * K);
        }
    }
    for (int L = 1; L <= maxl; L++) {
#pragma omp parallel for schedule(dynamic, 4)
        for (c = 0; c < nc; c++) {
            if (h->level[c] != L) continue;
            int32_t P = h->parent[c];
            double d[3] = {h->cphys[3 * c] - h->cphys[3 * P], h->cphys[3 * c + 1] - h->cphys[3 * P + 1],
                           h->cphys[3 * c + 2] - h->cphys[3 * P + 2]};
            ora_cart_l2l(p, h->Lc + (int64_t)P * K, d, h->Lc + c * K);
        }
    }
    int32_t *leaf = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (c = 0; c < nc; c++)
        if (is_leaf(h, (int32_t)c))
            for (int32_t i = h->begin[c]; i < h->end[c]; i++) leaf[i] = (int32_t)c;
    int64_t i;
#pragma omp parallel for schedule(dynamic, 64)
    for (i = 0; i < nout; i++) {
        double xi[3] = {h->px[i], h->py[i], h->pz[i]};
        int32_t t = leaf[i];
        double ph, e[3];
        ora_cart_l2p(p, h->Lc + (int64_t)t * K, &h->cphys[3 * t], xi, &ph, e);
        double P = ph, F[3] = {e[0], e[1], e[2]};
        for (int32_t A = t; A >= 0; A = h->parent[A]) {
            for (int64_t a = cm2p.off[A]; a < cm2p.off[A + 1]; a++) {
                int32_t s = cm2p.src[a];
                ora_cart_m2p(p, h->Mc + (int64_t)s * K, &h->cphys[3 * s], xi, &ph, e);
                P += ph; F[0] += e[0]; F[1] += e[1]; F[2] += e[2];
            }
            for (int64_t a = cp2p.off[A]; a < cp2p.off[A + 1]; a++) {
                int32_t s = cp2p.src[a];
                for (int32_t j = h->begin[s]; j < h->end[s]; j++) {
                    if (j == i) continue;
                    double dx = xi[0] - h->px[j], dy = xi[1] - h->py[j], dz = xi[2] - h->pz[j];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 == 0.0) continue;
                    double r = sqrt(r2);
                    P += sq[j] / r;
                    double f = sq[j] / (r2 * r);
                    F[0] += f * dx; F[1] += f * dy; F[2] += f * dz;
                }
            }
        }
        int64_t o = h->perm[i];
        phi[o] = P; ex[o] = F[0]; ey[o] = F[1]; ez[o] = F[2];
    }
    free(leaf); free(sq);
    free(cm2l.off); free(cm2l.src); free(cm2p.off); free(cm2p.src); free(cp2p.off); free(cp2p.src);
}

/* Cartesian expansions of every cell after ora_evaluate_cart */
void ora_get_expansions_cart(void *hv, double *M, double *L)
{
    ora_t *h = (ora_t *)hv;
    size_t K = (size_t)ora_cart_count(h->pc);
    memcpy(M, h->Mc, (size_t)h->ncell * K * sizeof(double));
    memcpy(L, h->Lc, (size_t)h->ncell * K * sizeof(double));
}

void ora_free(void *hv)
{
    ora_t *h = (ora_t *)hv;
    if (!h) return;
    free(h->skey); free(h->perm); free(h->px); free(h->py); free(h->pz);
    free(h->level); free(h->begin); free(h->end); free(h->parent); free(h->first_child);
    free(h->nchild); free(h->prefix); free(h->ch); free(h->rh); free(h->cphys); free(h->rphys);
    for (int k = 0; k < 3; k++) free(h->list[k].v);
    free(h->M); free(h->L); free(h->Mc); free(h->Lc);
    free(h);
}

/* Traversal with the learned choice read from `table` (see table_choice). */
void ora_traverse_table(void *hv, double theta, const uint8_t *table)
{
    double none[3] = {0, 0, 0};
    g_table = table;
    g_theta = theta;
    ora_traverse(hv, theta, 3, none);
    g_table = 0;
}
