/*
 * CPU oracle for the Fast Kernel Transform matrix-vector product (FP64).
 *
 * TEST INFRASTRUCTURE ONLY: this file is compiled into the oracle's own
 * shared object, which only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load. It shares no code, header or table with the HIP
 * product path.
 *
 * What it computes, in the paper's terms:
 *   - dense direct sum z_i = sum_j K(|r_i - r_j|) x_j            (eq. nbody)
 *   - the binary space-partition tree                             (Sec. 3.1)
 *   - far sets by the distance criterion                          (eq. accparam)
 *     and near sets N_l (Sec. 3.2), by a per-target walk
 *   - Algorithm 1 ("Barnes-Hut with Multipoles"), node by node, with the
 *     compressed block m2t*s2m evaluated entry by entry through the
 *     Gegenbauer form of the truncated expansion of Theorem 3.1 /
 *     eq. (finaltrunc): the addition theorem (eq. additiontheorem) turns the
 *     sum over harmonics h back into C_k^alpha(cos g) / Z_k, and Z_k cancels
 *     against T = Z_k Tbar.
 *   - the same operator one output row at a time, for sampled checks at
 *     large N.
 *
 * Readings of points the paper leaves open (all shared with the product by
 * specification only, not by code):
 *   - root: the hypercube lo_a = min_i X_ia, side = max_a extent_a;
 *   - leaf iff count <= leaf_size or depth == max_depth;
 *   - a split halves one of the currently longest sides (aspect ratio <= 2);
 *     among those axes the one with min |2 n_left - n| wins, ties to the
 *     lowest axis; left = {X_a < mid}, right = {X_a >= mid}, stable order;
 *     empty children are dropped; nodes are numbered in preorder, left first;
 *   - node centre = box centre; rho^2 = max over the node's points of the
 *     squared distance to the centre;
 *   - far(t, b) iff rho_b^2 < theta^2 |t - c_b|^2, all in FP64, summed in
 *     axis order, multiply then add (built with -ffp-contract=off);
 *   - singular kernels (r^-q) take K(0) = 0, so coincident pairs add nothing.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 16
#define MAXP 32

enum { K_GAUSS = 0, K_EXP = 1, K_MATERN32 = 2, K_MATERN52 = 3,
       K_RQ = 4, K_CAUCHY = 5, K_POWER = 6 };

/* ----------------------------------------------------------------- kernels */

static int kern_singular(int kind) { return kind == K_POWER; }

/* Derivatives K^(m)(r), m = 0..p, closed forms (prm: lengthscale, shape, variance). */
static void kern_derivs(int kind, const double *prm, double r, int p, double *out)
{
    const double ell = prm[0], shape = prm[1], var = prm[2];
    int m;
    switch (kind) {
    case K_GAUSS: { /* exp(-r^2/(2 l^2)) = exp(-u^2), u = r s; d^m/du^m = (-1)^m H_m(u) e^{-u^2} */
        double s = 1.0 / (sqrt(2.0) * ell), u = r * s, e = exp(-u * u);
        double h0 = 1.0, h1 = 2.0 * u, sm = 1.0;
        for (m = 0; m <= p; ++m) {
            double hm = (m == 0) ? h0 : (m == 1 ? h1 : 0.0);
            if (m >= 2) { hm = 2.0 * u * h1 - 2.0 * (m - 1) * h0; h0 = h1; h1 = hm; }
            out[m] = var * sm * hm * e;
            sm *= -s;
        }
        break; }
    case K_EXP: { double a = 1.0 / ell, e = exp(-a * r), sm = 1.0;
        for (m = 0; m <= p; ++m) { out[m] = var * sm * e; sm *= -a; }
        break; }
    case K_MATERN32: { double a = sqrt(3.0) / ell, e = exp(-a * r), sm = 1.0;
        for (m = 0; m <= p; ++m) { out[m] = var * sm * (1.0 - m + a * r) * e; sm *= -a; }
        break; }
    case K_MATERN52: { /* Q e^{-ar}, Q = 1 + ar + a^2 r^2 / 3; Leibniz rule */
        double a = sqrt(5.0) / ell, e = exp(-a * r);
        double q0 = 1.0 + a * r + a * a * r * r / 3.0, q1 = a + 2.0 * a * a * r / 3.0, q2 = 2.0 * a * a / 3.0;
        for (m = 0; m <= p; ++m) {
            double t = pow(-a, m) * q0;
            if (m >= 1) t += m * pow(-a, m - 1) * q1;
            if (m >= 2) t += 0.5 * m * (m - 1) * pow(-a, m - 2) * q2;
            out[m] = var * t * e;
        }
        break; }
    case K_RQ:
    case K_CAUCHY: { /* w(r+h)^beta with w quadratic in h; power-series recurrence */
        double g[3], beta, f[MAXP + 1];
        if (kind == K_RQ) {
            double c = 1.0 / (2.0 * shape * ell * ell);
            g[0] = 1.0 + c * r * r; g[1] = 2.0 * c * r; g[2] = c; beta = -shape;
        } else {
            double c = 1.0 / (ell * ell);
            g[0] = 1.0 + c * r * r; g[1] = 2.0 * c * r; g[2] = c; beta = -1.0;
        }
        f[0] = pow(g[0], beta);
        for (m = 1; m <= p; ++m) {
            double acc = 0.0; int k;
            for (k = 1; k <= 2 && k <= m; ++k) acc += ((beta + 1.0) * k - m) * g[k] * f[m - k];
            f[m] = acc / (m * g[0]);
        }
        { double fact = 1.0; for (m = 0; m <= p; ++m) { if (m) fact *= m; out[m] = var * fact * f[m]; } }
        break; }
    case K_POWER: { /* r^-q: K^(m) = (-1)^m (q)_m r^(-q-m) */
        double q = shape, base = var * pow(r, -q), c = 1.0;
        for (m = 0; m <= p; ++m) { out[m] = c * base; base /= r; c *= -(q + m); }
        break; }
    default:
        for (m = 0; m <= p; ++m) out[m] = NAN;
    }
}

static double kern_value(int kind, const double *prm, double r)
{
    double v[1];
    if (r == 0.0 && kern_singular(kind)) return 0.0;
    kern_derivs(kind, prm, r, 0, v);
    return v[0];
}

void ref_kernel_derivs(int kind, const double *prm, double r, int p, double *out)
{
    kern_derivs(kind, prm, r, p, out);
}

double ref_kernel_value(int kind, const double *prm, double r) { return kern_value(kind, prm, r); }

/* -------------------------------------------------------------- dense (O1) */

static double dist(const double *a, const double *b, int d)
{
    double s = 0.0; int k;
    for (k = 0; k < d; ++k) { double t = a[k] - b[k]; s += t * t; }
    return sqrt(s);
}

/* out[t][c] = sum_j K(|X_targets[t] - X_j|) x[j][c]; targets given by index. */
void ref_dense(int64_t n, int d, const double *X, int kind, const double *prm,
               const double *x, int nrhs, int64_t nt, const int64_t *targets, double *out)
{
    int64_t t;
#pragma omp parallel for schedule(dynamic, 16)
    for (t = 0; t < nt; ++t) {
        const double *xt = X + targets[t] * d;
        double acc[64]; int c; int64_t j;
        for (c = 0; c < nrhs; ++c) acc[c] = 0.0;
        for (j = 0; j < n; ++j) {
            double k = kern_value(kind, prm, dist(xt, X + j * d, d));
            for (c = 0; c < nrhs; ++c) acc[c] += k * x[j * nrhs + c];
        }
        for (c = 0; c < nrhs; ++c) out[t * nrhs + c] = acc[c];
    }
}

/* -------------------------------------------------------------------- tree */

typedef struct {
    int d;
    int64_t n, nnodes, cap;
    int64_t *perm;          /* tree position -> original index */
    double *lo, *side, *ctr; /* [node][d] */
    double *rho2;
    int64_t *start, *end, *child0, *child1, *parent;
    int32_t *depth;
    const double *X;        /* caller's points, original order (borrowed) */
} ref_tree;

static int64_t tree_new_node(ref_tree *T)
{
    if (T->nnodes == T->cap) {
        int64_t c = T->cap ? 2 * T->cap : 64;
        T->lo = realloc(T->lo, sizeof(double) * c * T->d);
        T->side = realloc(T->side, sizeof(double) * c * T->d);
        T->ctr = realloc(T->ctr, sizeof(double) * c * T->d);
        T->rho2 = realloc(T->rho2, sizeof(double) * c);
        T->start = realloc(T->start, sizeof(int64_t) * c);
        T->end = realloc(T->end, sizeof(int64_t) * c);
        T->child0 = realloc(T->child0, sizeof(int64_t) * c);
        T->child1 = realloc(T->child1, sizeof(int64_t) * c);
        T->parent = realloc(T->parent, sizeof(int64_t) * c);
        T->depth = realloc(T->depth, sizeof(int32_t) * c);
        T->cap = c;
    }
    return T->nnodes++;
}

static void tree_split(ref_tree *T, int64_t b, int leaf_size, int max_depth, int64_t *scratch)
{
    const int d = T->d;
    int64_t s = T->start[b], e = T->end[b], cnt = e - s, i;
    double smax = 0.0, mid_best = 0.0;
    int a, best = -1; int64_t best_score = -1, nl_best = 0;
    T->child0[b] = T->child1[b] = -1;
    if (cnt <= leaf_size || T->depth[b] >= max_depth) return;
    for (a = 0; a < d; ++a) if (T->side[b * d + a] > smax) smax = T->side[b * d + a];
    for (a = 0; a < d; ++a) {
        double mid; int64_t nl = 0, score;
        if (T->side[b * d + a] != smax) continue;
        mid = T->lo[b * d + a] + 0.5 * T->side[b * d + a];
        for (i = s; i < e; ++i) if (T->X[T->perm[i] * d + a] < mid) ++nl;
        score = llabs(2 * nl - cnt);
        if (best < 0 || score < best_score) { best = a; best_score = score; nl_best = nl; mid_best = mid; }
    }
    /* stable partition of perm[s:e) on axis `best` */
    {
        int64_t li = s, ri = 0;
        for (i = s; i < e; ++i) {
            int64_t p = T->perm[i];
            if (T->X[p * d + best] < mid_best) T->perm[li++] = p; else scratch[ri++] = p;
        }
        memcpy(T->perm + li, scratch, sizeof(int64_t) * ri);
    }
    {
        int side_lr;
        for (side_lr = 0; side_lr < 2; ++side_lr) {
            int64_t cs = side_lr ? s + nl_best : s, ce = side_lr ? e : s + nl_best, c;
            if (ce == cs) continue;
            c = tree_new_node(T);
            for (a = 0; a < d; ++a) { T->lo[c * d + a] = T->lo[b * d + a]; T->side[c * d + a] = T->side[b * d + a]; }
            T->side[c * d + best] = 0.5 * T->side[b * d + best];
            if (side_lr) T->lo[c * d + best] = mid_best;
            T->start[c] = cs; T->end[c] = ce; T->parent[c] = b; T->depth[c] = T->depth[b] + 1;
            if (side_lr) T->child1[b] = c; else T->child0[b] = c;
            tree_split(T, c, leaf_size, max_depth, scratch);   /* preorder: recurse before the sibling */
        }
    }
}

void *ref_tree_new(int64_t n, int d, const double *X, int leaf_size, int max_depth)
{
    ref_tree *T = calloc(1, sizeof(ref_tree));
    int64_t i, b, *scratch; int a;
    double ext = 0.0;
    T->d = d; T->n = n; T->X = X;
    T->perm = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (i = 0; i < n; ++i) T->perm[i] = i;
    b = tree_new_node(T);
    for (a = 0; a < d; ++a) {
        double lo = X[a], hi = X[a];
        for (i = 1; i < n; ++i) { double v = X[i * d + a]; if (v < lo) lo = v; if (v > hi) hi = v; }
        T->lo[a] = lo;
        if (hi - lo > ext) ext = hi - lo;
    }
    for (a = 0; a < d; ++a) T->side[a] = ext;
    T->start[b] = 0; T->end[b] = n; T->parent[b] = -1; T->depth[b] = 0;
    scratch = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    tree_split(T, b, leaf_size, max_depth, scratch);
    free(scratch);
    /* centres and radii */
    for (b = 0; b < T->nnodes; ++b) {
        double r2max = 0.0;
        for (a = 0; a < d; ++a) T->ctr[b * d + a] = T->lo[b * d + a] + 0.5 * T->side[b * d + a];
        for (i = T->start[b]; i < T->end[b]; ++i) {
            double r2 = 0.0;
            for (a = 0; a < d; ++a) { double t = X[T->perm[i] * d + a] - T->ctr[b * d + a]; r2 = r2 + t * t; }
            if (r2 > r2max) r2max = r2;
        }
        T->rho2[b] = r2max;
    }
    return T;
}

int64_t ref_tree_nnodes(void *h) { return ((ref_tree *)h)->nnodes; }

void ref_tree_export(void *h, int64_t *perm, double *lo, double *side, double *ctr, double *rho2,
                     int64_t *start, int64_t *end, int64_t *child, int64_t *parent, int32_t *depth)
{
    ref_tree *T = h; int64_t b; int d = T->d;
    memcpy(perm, T->perm, sizeof(int64_t) * T->n);
    memcpy(lo, T->lo, sizeof(double) * T->nnodes * d);
    memcpy(side, T->side, sizeof(double) * T->nnodes * d);
    memcpy(ctr, T->ctr, sizeof(double) * T->nnodes * d);
    memcpy(rho2, T->rho2, sizeof(double) * T->nnodes);
    memcpy(start, T->start, sizeof(int64_t) * T->nnodes);
    memcpy(end, T->end, sizeof(int64_t) * T->nnodes);
    memcpy(parent, T->parent, sizeof(int64_t) * T->nnodes);
    memcpy(depth, T->depth, sizeof(int32_t) * T->nnodes);
    for (b = 0; b < T->nnodes; ++b) { child[2 * b] = T->child0[b]; child[2 * b + 1] = T->child1[b]; }
}

void ref_tree_free(void *h)
{
    ref_tree *T = h;
    if (!T) return;
    free(T->perm); free(T->lo); free(T->side); free(T->ctr); free(T->rho2);
    free(T->start); free(T->end); free(T->child0); free(T->child1); free(T->parent); free(T->depth);
    free(T);
}

/* ---------------------------------------------------------------- partition */

static int is_far(const ref_tree *T, int64_t b, const double *t, double theta2)
{
    double s = 0.0; int a; const int d = T->d;
    for (a = 0; a < d; ++a) { double u = t[a] - T->ctr[b * d + a]; s = s + u * u; }
    return T->rho2[b] < theta2 * s;
}

/* Per-target walk from the root: far -> stop; leaf -> near; else children.
 * Writes node ids (far) and leaf ids (near) in visit order; returns 0, or -1
 * when a capacity is exceeded. */
static int walk(const ref_tree *T, int64_t b, const double *t, double theta2,
                int64_t *fo, int64_t fcap, int64_t *nf, int64_t *no, int64_t ncap, int64_t *nn)
{
    if (is_far(T, b, t, theta2)) {
        if (*nf >= fcap) return -1;
        fo[(*nf)++] = b; return 0;
    }
    if (T->child0[b] < 0 && T->child1[b] < 0) {
        if (*nn >= ncap) return -1;
        no[(*nn)++] = b; return 0;
    }
    if (T->child0[b] >= 0 && walk(T, T->child0[b], t, theta2, fo, fcap, nf, no, ncap, nn)) return -1;
    if (T->child1[b] >= 0 && walk(T, T->child1[b], t, theta2, fo, fcap, nf, no, ncap, nn)) return -1;
    return 0;
}

int ref_walk(void *h, const double *t, double theta, int64_t *far_out, int64_t far_cap, int64_t *nfar,
             int64_t *near_out, int64_t near_cap, int64_t *nnear)
{
    ref_tree *T = h;
    *nfar = 0; *nnear = 0;
    if (T->nnodes == 0 || T->n == 0) return 0;
    return walk(T, 0, t, theta * theta, far_out, far_cap, nfar, near_out, near_cap, nnear);
}

/* ---------------------------------------------------------------- expansion */

/* Truncated expansion (eq. finaltrunc) for one source at offset rp = r' and one
 * target at offset r = r, both relative to the node centre:
 *   sum_{k<=p} C_k^alpha(cos g) sum_{j=k,k+2,..<=p} r'^j F_kj(r),
 *   F_kj(r) = [j=0] K(r) + sum_{m=1}^{j} K^(m)(r) r^(m-j) Tbar[k][j][m].
 * Tbar is the dense (p+1)^3 table of Tbar_{k,j,m}. */
static double expansion_pair(int d, int p, const double *Tb, int kind, const double *prm,
                             const double *rp, const double *r)
{
    double rr = 0.0, rrp = 0.0, dot = 0.0, cg, alpha = 0.5 * d - 1.0;
    double D[MAXP + 1], C[MAXP + 1], rpow[2 * MAXP + 2], total = 0.0;
    int a, k, j, m;
    for (a = 0; a < d; ++a) { rr += r[a] * r[a]; rrp += rp[a] * rp[a]; dot += r[a] * rp[a]; }
    rr = sqrt(rr); rrp = sqrt(rrp);
    kern_derivs(kind, prm, rr, p, D);
    if (rrp == 0.0) return D[0];             /* only the j = 0 term survives */
    cg = dot / (rr * rrp);
    if (cg > 1.0) cg = 1.0;
    if (cg < -1.0) cg = -1.0;
    C[0] = 1.0;                               /* Gegenbauer recurrence, Appendix A.1 */
    if (p >= 1) C[1] = 2.0 * alpha * cg;
    for (k = 2; k <= p; ++k) C[k] = (2.0 * cg * (k + alpha - 1.0) * C[k - 1] - (k + 2.0 * alpha - 2.0) * C[k - 2]) / k;
    /* rpow[q] = r^(q - p) for q = 0..2p */
    for (j = 0; j <= 2 * p; ++j) rpow[j] = pow(rr, (double)(j - p));
    for (k = 0; k <= p; ++k) {
        double sk = 0.0;
        for (j = k; j <= p; j += 2) {
            double F = (j == 0) ? D[0] : 0.0;
            for (m = 1; m <= j; ++m) F += D[m] * rpow[m - j + p] * Tb[(k * (p + 1) + j) * (p + 1) + m];
            sk += pow(rrp, (double)j) * F;
        }
        total += C[k] * sk;
    }
    return total;
}

double ref_expansion(int d, int p, const double *Tb, int kind, const double *prm,
                     const double *rp, const double *r)
{
    return expansion_pair(d, p, Tb, kind, prm, rp, r);
}

/* Row t of the FKT operator: far part through the expansion about each far
 * node's centre, near part as dense kernel entries with each near leaf. */
static void fkt_row(const ref_tree *T, const double *t, double theta2, int p, const double *Tb,
                    int kind, const double *prm, const double *x, int nrhs, double *out,
                    int64_t *fbuf, int64_t *nbuf)
{
    const int d = T->d;
    int64_t nf = 0, nn = 0, q, i; int c, a;
    for (c = 0; c < nrhs; ++c) out[c] = 0.0;
    walk(T, 0, t, theta2, fbuf, T->nnodes, &nf, nbuf, T->nnodes, &nn);
    for (q = 0; q < nf; ++q) {
        int64_t b = fbuf[q];
        double r[MAXD], rp[MAXD];
        for (a = 0; a < d; ++a) r[a] = t[a] - T->ctr[b * d + a];
        for (i = T->start[b]; i < T->end[b]; ++i) {
            int64_t s = T->perm[i]; double v;
            for (a = 0; a < d; ++a) rp[a] = T->X[s * d + a] - T->ctr[b * d + a];
            v = expansion_pair(d, p, Tb, kind, prm, rp, r);
            for (c = 0; c < nrhs; ++c) out[c] += v * x[s * nrhs + c];
        }
    }
    for (q = 0; q < nn; ++q) {
        int64_t l = nbuf[q];
        for (i = T->start[l]; i < T->end[l]; ++i) {
            int64_t s = T->perm[i];
            double v = kern_value(kind, prm, dist(t, T->X + s * d, d));
            for (c = 0; c < nrhs; ++c) out[c] += v * x[s * nrhs + c];
        }
    }
}

/* Selected rows (original indices) of the FKT operator applied to x. */
void ref_fkt_rows(void *h, double theta, int p, const double *Tb, int kind, const double *prm,
                  const double *x, int nrhs, int64_t nt, const int64_t *targets, double *out)
{
    ref_tree *T = h;
    int64_t q;
#pragma omp parallel
    {
        int64_t *fb = malloc(sizeof(int64_t) * T->nnodes), *nb = malloc(sizeof(int64_t) * T->nnodes);
#pragma omp for schedule(dynamic, 4)
        for (q = 0; q < nt; ++q)
            fkt_row(T, T->X + targets[q] * T->d, theta * theta, p, Tb, kind, prm, x, nrhs, out + q * nrhs, fb, nb);
        free(fb); free(nb);
    }
}

/* Algorithm 1, node by node: each node passes its points' weights through the
 * truncated expansion to every target in its far set, and each leaf adds the
 * exact kernel block times its weights to every target in its near set. The
 * far and near sets come from the per-target walk. */
void ref_fkt_alg1(void *h, double theta, int p, const double *Tb, int kind, const double *prm,
                  const double *x, int nrhs, double *out)
{
    ref_tree *T = h;
    const int d = T->d;
    const int64_t n = T->n, nn = T->nnodes;
    int64_t *fcnt = calloc(nn + 1, sizeof(int64_t)), *ncnt = calloc(nn + 1, sizeof(int64_t));
    int64_t *flist, *nlist, *fpos, *npos, t, b;
    int64_t *fb = malloc(sizeof(int64_t) * nn), *nb = malloc(sizeof(int64_t) * nn);
    int64_t ftot = 0, ntot = 0;
    memset(out, 0, sizeof(double) * n * nrhs);
    /* far and near sets as target lists per node */
    for (t = 0; t < n; ++t) {
        int64_t nf = 0, nq = 0, q;
        walk(T, 0, T->X + t * d, theta * theta, fb, nn, &nf, nb, nn, &nq);
        for (q = 0; q < nf; ++q) fcnt[fb[q] + 1]++;
        for (q = 0; q < nq; ++q) ncnt[nb[q] + 1]++;
    }
    for (b = 0; b < nn; ++b) { fcnt[b + 1] += fcnt[b]; ncnt[b + 1] += ncnt[b]; }
    ftot = fcnt[nn]; ntot = ncnt[nn];
    flist = malloc(sizeof(int64_t) * (ftot ? ftot : 1)); nlist = malloc(sizeof(int64_t) * (ntot ? ntot : 1));
    fpos = malloc(sizeof(int64_t) * nn); npos = malloc(sizeof(int64_t) * nn);
    memcpy(fpos, fcnt, sizeof(int64_t) * nn); memcpy(npos, ncnt, sizeof(int64_t) * nn);
    for (t = 0; t < n; ++t) {
        int64_t nf = 0, nq = 0, q;
        walk(T, 0, T->X + t * d, theta * theta, fb, nn, &nf, nb, nn, &nq);
        for (q = 0; q < nf; ++q) flist[fpos[fb[q]]++] = t;
        for (q = 0; q < nq; ++q) nlist[npos[nb[q]]++] = t;
    }
    for (b = 0; b < nn; ++b) {
        int64_t q;
        /* far set of node b: expansion about b's centre, pair by pair */
#pragma omp parallel for schedule(dynamic, 8)
        for (q = fcnt[b]; q < fcnt[b + 1]; ++q) {
            int64_t tt = flist[q], i; int a, c;
            double r[MAXD], rp[MAXD];
            for (a = 0; a < d; ++a) r[a] = T->X[tt * d + a] - T->ctr[b * d + a];
            for (i = T->start[b]; i < T->end[b]; ++i) {
                int64_t s = T->perm[i]; double v;
                for (a = 0; a < d; ++a) rp[a] = T->X[s * d + a] - T->ctr[b * d + a];
                v = expansion_pair(d, p, Tb, kind, prm, rp, r);
                for (c = 0; c < nrhs; ++c) out[tt * nrhs + c] += v * x[s * nrhs + c];
            }
        }
        /* near set of leaf b (empty for inner nodes): exact kernel entries */
#pragma omp parallel for schedule(dynamic, 8)
        for (q = ncnt[b]; q < ncnt[b + 1]; ++q) {
            int64_t tt = nlist[q], i; int c;
            for (i = T->start[b]; i < T->end[b]; ++i) {
                int64_t s = T->perm[i];
                double v = kern_value(kind, prm, dist(T->X + tt * d, T->X + s * d, d));
                for (c = 0; c < nrhs; ++c) out[tt * nrhs + c] += v * x[s * nrhs + c];
            }
        }
    }
    free(fcnt); free(ncnt); free(flist); free(nlist); free(fpos); free(npos); free(fb); free(nb);
}

/* Per-target interaction counts: number of far nodes, far (t, s) pairs,
 * near leaves and near (t, s) pairs, for every target (original order). */
void ref_counts(void *h, double theta, int64_t *nfar_nodes, int64_t *nfar_pts,
                int64_t *nnear_leaves, int64_t *nnear_pts)
{
    ref_tree *T = h;
    int64_t t;
#pragma omp parallel
    {
        int64_t *fb = malloc(sizeof(int64_t) * T->nnodes), *nb = malloc(sizeof(int64_t) * T->nnodes);
#pragma omp for schedule(dynamic, 64)
        for (t = 0; t < T->n; ++t) {
            int64_t nf = 0, nq = 0, q, fp = 0, np = 0;
            walk(T, 0, T->X + t * T->d, theta * theta, fb, T->nnodes, &nf, nb, T->nnodes, &nq);
            for (q = 0; q < nf; ++q) fp += T->end[fb[q]] - T->start[fb[q]];
            for (q = 0; q < nq; ++q) np += T->end[nb[q]] - T->start[nb[q]];
            nfar_nodes[t] = nf; nfar_pts[t] = fp; nnear_leaves[t] = nq; nnear_pts[t] = np;
        }
        free(fb); free(nb);
    }
}

/* ------------------------------------------- factorised CPU FKT (Cartesian) */
/*
 * The same operator as Algorithm 1 at the same tree, partition and
 * truncation, factorised through moments, but with a basis that shares
 * nothing with the harmonic one: by Theorem 3.1 the terms of radial power
 * j form the degree-j part of the Taylor expansion of y -> K(|r - y|) about
 * the node centre (r the target and y the source, both relative to it), so
 * the p-truncated expansion is that Taylor polynomial of total degree p:
 *     K~(y, r) = sum_{|beta| <= p} c_beta(r) y^beta,
 * with Cartesian monomials y^beta. Per node b the moments are
 *     M_b[beta] = sum_{s in b} x_s (X_s - c_b)^beta,
 * and each far target t gets sum_beta c_beta(t - c_b) M_b[beta].
 *
 * Taylor coefficients: with rho = |r - y|^2 and h(rho) = K(sqrt(rho)), set
 * g_n(y) = h^(n)(|r - y|^2). Differentiating, d g_n / d y_a =
 * -2 (r_a - y_a) g_{n+1}(y), and comparing the coefficients of y^(beta - e_a)
 * on both sides gives, for any axis a with beta_a >= 1,
 *     beta_a c^(n)_beta = 2 c^(n+1)_(beta - 2 e_a) - 2 r_a c^(n+1)_(beta - e_a)
 * (the first term only when beta_a >= 2), with c^(n)_0 = h^(n)(|r|^2); the
 * wanted coefficients are c^(0). The rho-derivatives h^(n) are closed forms
 * per kernel (rho_derivs below). */
typedef struct {
    int d, p, nm;
    int *expo;      /* [nm][d] exponents, ordered by total degree            */
    int *deg;       /* [nm] total degree                                       */
    int *axis;      /* [nm] first axis with a nonzero exponent (-1 for 0)      */
    int *m1, *m2;   /* [nm] index of beta - e_axis, beta - 2 e_axis (or -1)    */
} cart_basis;

static int cart_find(const cart_basis *B, const int *e, int upto)
{
    int i, a;
    for (i = 0; i < upto; ++i) {
        for (a = 0; a < B->d; ++a) if (B->expo[i * B->d + a] != e[a]) break;
        if (a == B->d) return i;
    }
    return -1;
}

static void cart_basis_init(cart_basis *B, int d, int p)
{
    int k, i, a, cnt = 0, e[MAXD];
    int64_t cap = 1;
    for (i = 1; i <= d; ++i) cap = cap * (p + i) / i;   /* C(p+d, d) */
    B->d = d; B->p = p; B->nm = (int)cap;
    B->expo = calloc((size_t)cap * d, sizeof(int));
    B->deg = malloc(sizeof(int) * cap); B->axis = malloc(sizeof(int) * cap);
    B->m1 = malloc(sizeof(int) * cap); B->m2 = malloc(sizeof(int) * cap);
    /* all exponent vectors of degree k, by counting in base k+1 (small d, p) */
    for (k = 0; k <= p; ++k) {
        for (a = 0; a < d; ++a) e[a] = 0;
        for (;;) {
            int s = 0;
            for (a = 0; a < d; ++a) s += e[a];
            if (s == k) { memcpy(B->expo + (size_t)cnt * d, e, sizeof(int) * d); B->deg[cnt++] = k; }
            for (a = 0; a < d; ++a) { if (++e[a] <= k) break; e[a] = 0; }
            if (a == d) break;
        }
    }
    for (i = 0; i < B->nm; ++i) {
        int *bi = B->expo + (size_t)i * d;
        B->axis[i] = -1; B->m1[i] = B->m2[i] = -1;
        for (a = 0; a < d; ++a) if (bi[a] > 0) break;
        if (a == d) continue;
        B->axis[i] = a;
        memcpy(e, bi, sizeof(int) * d);
        e[a] -= 1; B->m1[i] = cart_find(B, e, i);
        if (bi[a] >= 2) { e[a] -= 1; B->m2[i] = cart_find(B, e, i); }
    }
}

static void cart_basis_free(cart_basis *B)
{
    free(B->expo); free(B->deg); free(B->axis); free(B->m1); free(B->m2);
}

/* E_n = d^n/drho^n exp(-c sqrt(rho)) at sqrt(rho) = r: for n >= 1,
 * (-1)^n e^{-cr} sum_{k<n} (n-1+k)! / (k! (n-1-k)!) c^(n-k) / (2^(n+k) r^(n+k))
 * (the reverse Bessel polynomial; every term has the same sign). */
static double exp_sqrt_deriv(int n, double c, double r)
{
    double e = exp(-c * r), s = 0.0;
    int k;
    if (n == 0) return e;
    for (k = 0; k < n; ++k) {
        double w = 1.0; int i;
        for (i = n - k; i <= n - 1 + k; ++i) w *= i;       /* (n-1+k)! / (n-1-k)! */
        for (i = 2; i <= k; ++i) w /= i;                   /* / k! */
        s += w * pow(c, n - k) / (pow(2.0, n + k) * pow(r, n + k));
    }
    return ((n & 1) ? -1.0 : 1.0) * e * s;
}

/* h^(n)(rho) = d^n/drho^n K(sqrt(rho)) at rho = r^2, n = 0..p, in closed form
 * per kernel (prm: lengthscale, shape, variance):
 *   Gaussian exp(-c rho), c = 1/(2 l^2):   (-c)^n exp(-c rho)
 *   exponential exp(-c r), c = 1/l:        E_n
 *   Matern-3/2 (1 + cr) e^{-cr}:           K' = -c^2 r e^{-cr}, so h' = -(c^2/2) E_0
 *                                          and h^(n) = -(c^2/2) E_{n-1}
 *   Matern-5/2 (1 + cr + c^2 r^2/3) e^{-cr}: K' = -(c^2/3) r (1 + cr) e^{-cr}, so
 *                                          h^(n) = -(c^2/6) (Matern-3/2)^(n-1)
 *   rational quadratic (1 + c rho)^(-a):   (-a)(-a-1)..(-a-n+1) c^n (1 + c rho)^(-a-n)
 *   Cauchy: the same with a = 1, c = 1/l^2
 *   r^-q = rho^(-q/2):                      (-q/2)(-q/2-1)..(-q/2-n+1) rho^(-q/2-n) */
static void rho_derivs(int kind, const double *prm, double r, int p, double *h)
{
    const double ell = prm[0], shape = prm[1], var = prm[2], rho = r * r;
    int n;
    for (n = 0; n <= p; ++n) {
        double v = NAN;
        switch (kind) {
        case K_GAUSS: { double c = 1.0 / (2.0 * ell * ell); v = pow(-c, n) * exp(-c * rho); break; }
        case K_EXP: v = exp_sqrt_deriv(n, 1.0 / ell, r); break;
        case K_MATERN32: { double c = sqrt(3.0) / ell;
            v = (n == 0) ? (1.0 + c * r) * exp(-c * r) : -0.5 * c * c * exp_sqrt_deriv(n - 1, c, r); break; }
        case K_MATERN52: { double c = sqrt(5.0) / ell;
            if (n == 0) v = (1.0 + c * r + c * c * r * r / 3.0) * exp(-c * r);
            else if (n == 1) v = -(c * c / 6.0) * (1.0 + c * r) * exp(-c * r);
            else v = (c * c / 6.0) * (0.5 * c * c) * exp_sqrt_deriv(n - 2, c, r);
            break; }
        case K_RQ:
        case K_CAUCHY: { double a = (kind == K_RQ) ? shape : 1.0;
            double c = (kind == K_RQ) ? 1.0 / (2.0 * shape * ell * ell) : 1.0 / (ell * ell), f = 1.0; int i;
            for (i = 0; i < n; ++i) f *= -a - i;
            v = f * pow(c, n) * pow(1.0 + c * rho, -a - n); break; }
        case K_POWER: { double f = 1.0; int i;
            for (i = 0; i < n; ++i) f *= -0.5 * shape - i;
            v = f * pow(rho, -0.5 * shape - n); break; }
        }
        h[n] = var * v;
    }
}

/* Taylor coefficients c^(0)_beta of y -> K(|r - y|) at y = 0 (work: 2 nm doubles) */
static void cart_coeffs(const cart_basis *B, int kind, const double *prm, const double *r, double *c, double *work)
{
    const int p = B->p, d = B->d;
    double h[MAXP + 1], rr = 0.0, *cur = work, *nxt = work + B->nm;
    int n, i, a;
    for (a = 0; a < d; ++a) rr += r[a] * r[a];
    rho_derivs(kind, prm, sqrt(rr), p, h);
    /* level n holds degrees 0..p-n; start at n = p, go down to n = 0 */
    nxt[0] = h[p];
    for (n = p - 1; n >= 0; --n) {
        double *lev = (n == 0) ? c : cur;
        lev[0] = h[n];
        for (i = 1; i < B->nm && B->deg[i] <= p - n; ++i) {
            int ax = B->axis[i], ba = B->expo[i * d + ax];
            double v = -r[ax] * nxt[B->m1[i]];
            if (B->m2[i] >= 0) v += nxt[B->m2[i]];
            lev[i] = 2.0 * v / ba;
        }
        if (n > 0) { double *t = cur; cur = nxt; nxt = t; }
    }
    if (p == 0) c[0] = h[0];
}

/* The Cartesian truncated expansion for one (source offset rp, target offset
 * r) pair: sum_beta c_beta(r) rp^beta (compared with ref_expansion by tests). */
double ref_cart_pair(int d, int p, int kind, const double *prm, const double *rp, const double *r)
{
    cart_basis B;
    double *c, *w, *mono, s = 0.0;
    int i;
    cart_basis_init(&B, d, p);
    c = malloc(sizeof(double) * B.nm); w = malloc(sizeof(double) * 2 * B.nm); mono = malloc(sizeof(double) * B.nm);
    cart_coeffs(&B, kind, prm, r, c, w);
    mono[0] = 1.0;
    for (i = 1; i < B.nm; ++i) mono[i] = mono[B.m1[i]] * rp[B.axis[i]];
    for (i = 0; i < B.nm; ++i) s += c[i] * mono[i];
    free(c); free(w); free(mono); cart_basis_free(&B);
    return s;
}

/* h^(n)(|r|^2) for n = 0..p (exported for tests). */
void ref_rho_derivs(int p, int kind, const double *prm, double rr, double *h)
{
    rho_derivs(kind, prm, rr, p, h);
}

/*
 * Factorised FKT, selected rows: moments of every node from its own points,
 * then, for each target, the Taylor coefficients about each far node's
 * centre against that node's moments, plus the exact kernel entries of its
 * near leaves. targets (original indices) may be NULL for all rows in
 * original order; nthreads <= 0 uses the OpenMP default.
 */
void ref_fkt_cart(void *h, double theta, int p, int kind, const double *prm, const double *x, int nrhs,
                  int64_t nt, const int64_t *targets, double *out)
{
    ref_tree *T = h;
    const int d = T->d;
    const int64_t nn = T->nnodes;
    cart_basis B;
    double *mom;
    int64_t b, q;
    cart_basis_init(&B, d, p);
    mom = calloc((size_t)nn * B.nm * nrhs, sizeof(double));
#pragma omp parallel
    {
        double *mono = malloc(sizeof(double) * B.nm);
#pragma omp for schedule(dynamic, 1)
        for (b = 0; b < nn; ++b) {
            double *M = mom + (size_t)b * B.nm * nrhs;
            int64_t i;
            for (i = T->start[b]; i < T->end[b]; ++i) {
                int64_t s = T->perm[i];
                double y[MAXD];
                int a, k, c;
                for (a = 0; a < d; ++a) y[a] = T->X[s * d + a] - T->ctr[b * d + a];
                mono[0] = 1.0;
                for (k = 1; k < B.nm; ++k) mono[k] = mono[B.m1[k]] * y[B.axis[k]];
                for (k = 0; k < B.nm; ++k)
                    for (c = 0; c < nrhs; ++c) M[(size_t)k * nrhs + c] += mono[k] * x[s * nrhs + c];
            }
        }
        free(mono);
    }
#pragma omp parallel
    {
        int64_t *fb = malloc(sizeof(int64_t) * nn), *nb = malloc(sizeof(int64_t) * nn);
        double *cf = malloc(sizeof(double) * B.nm), *w = malloc(sizeof(double) * 2 * B.nm);
#pragma omp for schedule(dynamic, 16)
        for (q = 0; q < nt; ++q) {
            const int64_t t = targets ? targets[q] : q;
            const double *xt = T->X + t * d;
            double *o = out + q * nrhs;
            int64_t nf = 0, nq = 0, f, i;
            int a, c, k;
            for (c = 0; c < nrhs; ++c) o[c] = 0.0;
            walk(T, 0, xt, theta * theta, fb, nn, &nf, nb, nn, &nq);
            for (f = 0; f < nf; ++f) {
                const double *M = mom + (size_t)fb[f] * B.nm * nrhs;
                double r[MAXD];
                for (a = 0; a < d; ++a) r[a] = xt[a] - T->ctr[fb[f] * d + a];
                cart_coeffs(&B, kind, prm, r, cf, w);
                for (k = 0; k < B.nm; ++k)
                    for (c = 0; c < nrhs; ++c) o[c] += cf[k] * M[(size_t)k * nrhs + c];
            }
            for (f = 0; f < nq; ++f) {
                const int64_t l = nb[f];
                for (i = T->start[l]; i < T->end[l]; ++i) {
                    const int64_t s = T->perm[i];
                    const double v = kern_value(kind, prm, dist(xt, T->X + s * d, d));
                    for (c = 0; c < nrhs; ++c) o[c] += v * x[s * nrhs + c];
                }
            }
        }
        free(fb); free(nb); free(cf); free(w);
    }
    free(mom);
    cart_basis_free(&B);
}
