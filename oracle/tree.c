/*
 * Oracle B -- FP64 reference tree solver.  TEST INFRASTRUCTURE ONLY.
 *
 * Written from the description of the modified tree algorithm (Sec. 3.2):
 * an equal-area quad-tree whose boxes are leaves below a particle count,
 * multipole moments of each box about its centre of mass, the opening
 * radius r_cut = r_cm / theta_force (Eq. r_cut), the per-box "big particle"
 * lists, and the walk that accepts a box when |x - x_cm| > r_cut, opens it
 * otherwise and sums leaves directly.  Plain recursion, FP64 throughout.
 *
 * Readings fixed here (the paper leaves them open):
 *  - root square: centre of the particles' bounding box, side =
 *    max extent * (1 + 2^-40) (1 if the extent is 0); equal-area children are
 *    decided on 32-bit quantised coordinates, so a particle on a dividing line
 *    goes to the upper/right child;
 *  - a box is a leaf when it holds <= leaf_size particles or sits at depth 32;
 *  - moments are the complex multipoles Q_k = sum_j m_j (z_j - z_cm)^k,
 *    k = 0..p ("monopole and quadrupole" is p = 2);
 *  - r_cm is the distance from the centre of mass to the farthest box corner;
 *  - a particle's "size" is its support radius (q s for a Gaussian, the
 *    truncation radius for an NFW halo); it is listed in the highest box where
 *    size > side / 2, if that box is not below its leaf;
 *  - listed particles are points inside moments and leaf sums; every visited
 *    box (accepted or opened) adds "exact kernel - point" for each of its
 *    listed particles that the ray falls inside.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef struct {
    int level;
    uint32_t ix, iy;     /* box index at its level */
    int64_t beg, end;    /* members: perm[beg, end) */
    int leaf;
    int nchild;
    int64_t child[4];
    int64_t next;        /* preorder index one past the subtree */
    int64_t lbeg, lend;  /* list members: lst[lbeg, lend) */
    double M, cx, cy, rcut2;
} ocell;

typedef struct {
    uint8_t* buf;
    int64_t len, cap, pos;
    int mode; /* 0 free, 1 record, 2 replay */
} tape_t;

struct ora_tree {
    int64_t n;
    int kind;   /* 0: Gaussian particles and point masses; 1: truncated NFW halos */
    double q, theta; /* q: Gaussian cutoff, or the NFW concentration */
    int L, p;
    double *x, *y, *m, *s;
    double x0, y0, S, scale;
    uint32_t *qx, *qy;
    int64_t* perm;
    int64_t* listed_at; /* cell index or -1 */
    ocell* cells;
    int64_t nc, cap;
    int64_t* lst;
    double complex* Q; /* nc * (p + 1) */
    tape_t* tapes;
    int64_t ntapes;
};

/* The particle type of the tree: support radius ("size"), inside test and
 * per-unit-mass terms. */
static double support(const ora_tree* t, int64_t i) { return t->kind ? t->s[i] : t->q * t->s[i]; }

static int inside_of(const ora_tree* t, int64_t i, double d1, double d2)
{
    return t->kind ? ora_nfw_inside(d1, d2, t->s[i]) : ora_inside(d1, d2, t->s[i], t->q);
}

static double psi_of(const ora_tree* t, int64_t i, double d1, double d2, int in)
{
    return t->kind ? ora_nfw_psi(d1, d2, t->s[i], t->q, in) : ora_unit_psi(d1, d2, t->s[i], t->q, in);
}

static void terms_of(const ora_tree* t, int64_t i, double d1, double d2, int in, double out[7])
{
    if (t->kind) ora_nfw_terms(d1, d2, t->s[i], t->q, in, out);
    else ora_unit_terms(d1, d2, t->s[i], t->q, in, out);
}

/* ---------------------------------------------------------------- build */

static uint32_t quantise(double v, double v0, double scale)
{
    const double t = (v - v0) * scale;
    if (!(t >= 0.0)) return 0u;
    if (t >= 4294967295.0) return 4294967295u;
    return (uint32_t)floor(t);
}

static int64_t push_cell(ora_tree* t)
{
    if (t->nc == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 1024;
        t->cells = (ocell*)realloc(t->cells, (size_t)t->cap * sizeof(ocell));
    }
    memset(&t->cells[t->nc], 0, sizeof(ocell));
    return t->nc++;
}

static int64_t build_rec(ora_tree* t, int level, uint32_t ix, uint32_t iy, int64_t beg, int64_t end,
                         int64_t* tmp)
{
    const int64_t c = push_cell(t);
    t->cells[c].level = level;
    t->cells[c].ix = ix;
    t->cells[c].iy = iy;
    t->cells[c].beg = beg;
    t->cells[c].end = end;
    if (end - beg <= t->L || level == 32) {
        t->cells[c].leaf = 1;
        t->cells[c].next = t->nc;
        return c;
    }
    /* split into the four equal-area children; child index = 2*ybit + xbit */
    const int shift = 31 - level;
    int64_t cnt[4] = {0, 0, 0, 0}, off[4];
    for (int64_t k = beg; k < end; ++k) {
        const int64_t i = t->perm[k];
        cnt[(((t->qy[i] >> shift) & 1u) << 1) | ((t->qx[i] >> shift) & 1u)]++;
    }
    off[0] = beg;
    for (int k = 1; k < 4; ++k) off[k] = off[k - 1] + cnt[k - 1];
    int64_t pos[4] = {off[0], off[1], off[2], off[3]};
    for (int64_t k = beg; k < end; ++k) {
        const int64_t i = t->perm[k];
        tmp[pos[(((t->qy[i] >> shift) & 1u) << 1) | ((t->qx[i] >> shift) & 1u)]++] = i;
    }
    memcpy(t->perm + beg, tmp + beg, (size_t)(end - beg) * sizeof(int64_t));
    for (int k = 0; k < 4; ++k) {
        if (cnt[k] == 0) continue;
        const int64_t ch = build_rec(t, level + 1, 2u * ix + (uint32_t)(k & 1), 2u * iy + (uint32_t)(k >> 1),
                                     off[k], off[k] + cnt[k], tmp);
        t->cells[c].child[t->cells[c].nchild++] = ch;
    }
    t->cells[c].next = t->nc;
    return c;
}

/* centre of mass, multipoles about it, and the opening radius (Sec. 3.2) */
static void cell_moments(ora_tree* t, int64_t c)
{
    ocell* cl = &t->cells[c];
    double complex* Q = t->Q + c * (t->p + 1);
    const double side = ldexp(t->S, -cl->level);
    const double bx0 = t->x0 + (double)cl->ix * side, bx1 = t->x0 + ((double)cl->ix + 1.0) * side;
    const double by0 = t->y0 + (double)cl->iy * side, by1 = t->y0 + ((double)cl->iy + 1.0) * side;
    double M = 0, sx = 0, sy = 0;
    for (int64_t k = cl->beg; k < cl->end; ++k) {
        const int64_t i = t->perm[k];
        M += t->m[i];
        sx += t->m[i] * t->x[i];
        sy += t->m[i] * t->y[i];
    }
    cl->M = M;
    if (M > 0) {
        cl->cx = sx / M;
        cl->cy = sy / M;
    } else {
        cl->cx = 0.5 * (bx0 + bx1);
        cl->cy = 0.5 * (by0 + by1);
    }
    for (int k = 0; k <= t->p; ++k) Q[k] = 0;
    for (int64_t k = cl->beg; k < cl->end; ++k) {
        const int64_t i = t->perm[k];
        const double complex d = (t->x[i] - cl->cx) + I * (t->y[i] - cl->cy);
        double complex dk = 1.0;
        for (int j = 0; j <= t->p; ++j) {
            Q[j] += t->m[i] * dk;
            dk *= d;
        }
    }
    const double X[4] = {bx0, bx1, bx0, bx1}, Y[4] = {by0, by0, by1, by1};
    double dmax2 = 0;
    for (int k = 0; k < 4; ++k) {
        const double e1 = X[k] - cl->cx, e2 = Y[k] - cl->cy;
        const double d2 = e1 * e1 + e2 * e2;
        if (d2 > dmax2) dmax2 = d2;
    }
    cl->rcut2 = t->theta > 0 ? dmax2 / (t->theta * t->theta) : INFINITY;
}

static void assign_lists(ora_tree* t)
{
    const int64_t n = t->n;
    int64_t* leaf_of = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    for (int64_t c = 0; c < t->nc; ++c)
        if (t->cells[c].leaf)
            for (int64_t k = t->cells[c].beg; k < t->cells[c].end; ++k) leaf_of[t->perm[k]] = c;
    for (int64_t i = 0; i < n; ++i) {
        t->listed_at[i] = -1;
        if (!(t->s[i] > 0)) continue;
        const double qs = support(t, i);
        int l = 0;
        while (l <= 32 && !(qs > ldexp(t->S, -(l + 1)))) ++l;
        if (l > 32 || l > t->cells[leaf_of[i]].level) continue;
        int64_t c = 0;
        while (t->cells[c].level < l) {
            const int cl = t->cells[c].level + 1;
            const uint32_t bx = (uint32_t)((uint64_t)t->qx[i] >> (32 - cl));
            const uint32_t by = (uint32_t)((uint64_t)t->qy[i] >> (32 - cl));
            int64_t next = -1;
            for (int k = 0; k < t->cells[c].nchild; ++k) {
                const ocell* ch = &t->cells[t->cells[c].child[k]];
                if (ch->ix == bx && ch->iy == by) next = t->cells[c].child[k];
            }
            c = next;
        }
        t->listed_at[i] = c;
    }
    int64_t* cnt = (int64_t*)calloc((size_t)t->nc + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        if (t->listed_at[i] >= 0) cnt[t->listed_at[i] + 1]++;
    for (int64_t c = 0; c < t->nc; ++c) cnt[c + 1] += cnt[c];
    t->lst = (int64_t*)malloc((size_t)(cnt[t->nc] + 1) * sizeof(int64_t));
    for (int64_t c = 0; c < t->nc; ++c) {
        t->cells[c].lbeg = cnt[c];
        t->cells[c].lend = cnt[c];
    }
    for (int64_t i = 0; i < n; ++i)
        if (t->listed_at[i] >= 0) {
            ocell* cl = &t->cells[t->listed_at[i]];
            t->lst[cl->lend++] = i;
        }
    free(cnt);
    free(leaf_of);
}

static ora_tree* build_kind(const double* x, const double* y, const double* m, const double* s, int64_t n,
                            double q, double theta, int leaf_size, int order, int kind)
{
    if (n <= 0 || leaf_size < 1 || order < 0) return NULL;
    ora_tree* t = (ora_tree*)calloc(1, sizeof(ora_tree));
    t->n = n;
    t->kind = kind;
    t->q = q;
    t->theta = theta;
    t->L = leaf_size;
    t->p = order;
    t->x = (double*)malloc((size_t)n * sizeof(double));
    t->y = (double*)malloc((size_t)n * sizeof(double));
    t->m = (double*)malloc((size_t)n * sizeof(double));
    t->s = (double*)calloc((size_t)n, sizeof(double));
    memcpy(t->x, x, (size_t)n * sizeof(double));
    memcpy(t->y, y, (size_t)n * sizeof(double));
    memcpy(t->m, m, (size_t)n * sizeof(double));
    if (s) memcpy(t->s, s, (size_t)n * sizeof(double));

    double xmin = x[0], xmax = x[0], ymin = y[0], ymax = y[0];
    for (int64_t i = 1; i < n; ++i) {
        if (x[i] < xmin) xmin = x[i];
        if (x[i] > xmax) xmax = x[i];
        if (y[i] < ymin) ymin = y[i];
        if (y[i] > ymax) ymax = y[i];
    }
    const double ext = (xmax - xmin) > (ymax - ymin) ? (xmax - xmin) : (ymax - ymin);
    double S = ext * (1.0 + 0x1p-40);
    if (!(S > 0)) S = 1.0;
    t->S = S;
    t->x0 = 0.5 * (xmin + xmax) - 0.5 * S;
    t->y0 = 0.5 * (ymin + ymax) - 0.5 * S;
    t->scale = 4294967296.0 / S;

    t->qx = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    t->qy = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    t->perm = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    t->listed_at = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        t->qx[i] = quantise(x[i], t->x0, t->scale);
        t->qy[i] = quantise(y[i], t->y0, t->scale);
        t->perm[i] = i;
    }
    int64_t* tmp = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    build_rec(t, 0, 0u, 0u, 0, n, tmp);
    free(tmp);
    t->Q = (double complex*)calloc((size_t)t->nc * (size_t)(t->p + 1), sizeof(double complex));
    for (int64_t c = 0; c < t->nc; ++c) cell_moments(t, c);
    assign_lists(t);
    return t;
}

ora_tree* ora_tree_build(const double* x, const double* y, const double* m, const double* s,
                         int64_t n, double q, double theta, int leaf_size, int order)
{
    return build_kind(x, y, m, s, n, q, theta, leaf_size, order, 0);
}

ora_tree* ora_tree_build_nfw(const double* x, const double* y, const double* m, const double* R, int64_t n,
                             double c, double theta, int leaf_size, int order)
{
    return build_kind(x, y, m, R, n, c, theta, leaf_size, order, 1);
}

void ora_tree_free(ora_tree* t)
{
    if (!t) return;
    for (int64_t r = 0; r < t->ntapes; ++r) free(t->tapes[r].buf);
    free(t->tapes);
    free(t->x);
    free(t->y);
    free(t->m);
    free(t->s);
    free(t->qx);
    free(t->qy);
    free(t->perm);
    free(t->listed_at);
    free(t->cells);
    free(t->lst);
    free(t->Q);
    free(t);
}

int64_t ora_tree_ncells(const ora_tree* t) { return t->nc; }

void ora_tree_root(const ora_tree* t, double out[3])
{
    out[0] = t->x0;
    out[1] = t->y0;
    out[2] = t->S;
}

void ora_tree_export(const ora_tree* t, int32_t* level, uint32_t* ix, uint32_t* iy, int32_t* np,
                     int32_t* leaf, int32_t* nl, int64_t* next, double* M, double* cx, double* cy,
                     double* rcut2, double* Q)
{
    const int P = t->p + 1;
    for (int64_t c = 0; c < t->nc; ++c) {
        const ocell* cl = &t->cells[c];
        level[c] = cl->level;
        ix[c] = cl->ix;
        iy[c] = cl->iy;
        np[c] = (int32_t)(cl->end - cl->beg);
        leaf[c] = cl->leaf;
        nl[c] = (int32_t)(cl->lend - cl->lbeg);
        next[c] = cl->next;
        M[c] = cl->M;
        cx[c] = cl->cx;
        cy[c] = cl->cy;
        rcut2[c] = cl->rcut2;
        for (int k = 0; k < P; ++k) {
            Q[(c * P + k) * 2 + 0] = creal(t->Q[c * P + k]);
            Q[(c * P + k) * 2 + 1] = cimag(t->Q[c * P + k]);
        }
    }
}

static int cmp_i32(const void* a, const void* b)
{
    const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

int64_t ora_tree_members(const ora_tree* t, int64_t cell, int32_t* out)
{
    const ocell* cl = &t->cells[cell];
    for (int64_t k = cl->beg; k < cl->end; ++k) out[k - cl->beg] = (int32_t)t->perm[k];
    qsort(out, (size_t)(cl->end - cl->beg), sizeof(int32_t), cmp_i32);
    return cl->end - cl->beg;
}

int64_t ora_tree_list(const ora_tree* t, int64_t cell, int32_t* out)
{
    const ocell* cl = &t->cells[cell];
    for (int64_t k = cl->lbeg; k < cl->lend; ++k) out[k - cl->lbeg] = (int32_t)t->lst[k];
    qsort(out, (size_t)(cl->lend - cl->lbeg), sizeof(int32_t), cmp_i32);
    return cl->lend - cl->lbeg;
}

/* ----------------------------------------------------------------- walk */

static int decide(tape_t* tp, int cond)
{
    if (!tp || tp->mode == 0) return cond;
    if (tp->mode == 1) {
        if (tp->len == tp->cap) {
            tp->cap = tp->cap ? 2 * tp->cap : 256;
            tp->buf = (uint8_t*)realloc(tp->buf, (size_t)tp->cap);
        }
        tp->buf[tp->len++] = (uint8_t)(cond != 0);
        return cond;
    }
    return tp->buf[tp->pos++];
}

/* multipole expansion of a box about its centre of mass, w = z - z_cm:
 *   alpha1 - i alpha2 = sum_k Q_k w^-(k+1),
 *   gamma1 - i gamma2 = -sum_k (k+1) Q_k w^-(k+2),  kappa = 0. */
static void multipole(const double complex* Q, int p, double w1, double w2, double acc[5])
{
    const double complex w = w1 + I * w2;
    const double complex iw = 1.0 / w;
    double complex pw = iw, F = 0, Gm = 0;
    for (int k = 0; k <= p; ++k) {
        F += Q[k] * pw;
        Gm -= (double)(k + 1) * Q[k] * pw * iw;
        pw *= iw;
    }
    acc[0] += creal(F);
    acc[1] -= cimag(F);
    acc[3] += creal(Gm);
    acc[4] -= cimag(Gm);
}

/* potential of a box (Sec. 3.2, alpha = grad psi): for point masses,
 * psi = Re sum_i m_i ln(w - d_i) = Re [Q_0 ln w - sum_{k>=1} Q_k / (k w^k)]. */
static double multipole_psi(const double complex* Q, int p, double w1, double w2)
{
    const double complex w = w1 + I * w2;
    const double complex iw = 1.0 / w;
    double complex pw = iw, S = Q[0] * clog(w);
    for (int k = 1; k <= p; ++k) {
        S -= Q[k] * pw / (double)k;
        pw *= iw;
    }
    return creal(S);
}

typedef struct {
    const double* ga; /* cotangents of the ray: alpha (2), kappa, gamma (2) */
    double *dm, *dx, *dy, *ds;
    double complex *Abar, *Bbar;
} adj_t;

/* particle i enters with weight m_i: forward accumulation, or the adjoint of
 * sign * (its per-unit-mass terms t; dt their kappa and gamma derivatives) */
static void particle_term(const ora_tree* t, int64_t i, const double tt[7], const double dt[9], double sign,
                          double acc[5], adj_t* adj)
{
    const double mi = t->m[i];
    if (!adj) {
        for (int k = 0; k < 5; ++k) acc[k] += sign * mi * tt[k];
        return;
    }
    const double g1 = adj->ga[0], g2 = adj->ga[1], gk = adj->ga[2], h1 = adj->ga[3], h2 = adj->ga[4];
    adj->dm[i] += sign * (g1 * tt[0] + g2 * tt[1] + gk * tt[2] + h1 * tt[3] + h2 * tt[4]);
    adj->dx[i] -= sign * mi * (g1 * (tt[2] + tt[3]) + g2 * tt[4] + gk * dt[0] + h1 * dt[2] + h2 * dt[4]);
    adj->dy[i] -= sign * mi * (g1 * tt[4] + g2 * (tt[2] - tt[3]) + gk * dt[1] + h1 * dt[3] + h2 * dt[5]);
    adj->ds[i] += sign * mi * (g1 * tt[5] + g2 * tt[6] + gk * dt[6] + h1 * dt[7] + h2 * dt[8]);
}

/* kappa and gamma derivatives of particle i (zero unless the adjoint needs them) */
static void dterms_of(const ora_tree* t, int64_t i, double d1, double d2, int in, const adj_t* adj, double out[9])
{
    if (!adj) memset(out, 0, 9 * sizeof(double));
    else if (t->kind) ora_nfw_dterms(d1, d2, t->s[i], t->q, in, out);
    else ora_unit_dterms(d1, d2, t->s[i], t->q, in, out);
}

static void visit(const ora_tree* t, int64_t c, double X, double Y, double acc[5], int64_t cnt[5],
                  tape_t* tp, adj_t* adj, double* psi)
{
    const ocell* cl = &t->cells[c];
    cnt[0]++;
    for (int64_t k = cl->lbeg; k < cl->lend; ++k) {
        const int64_t i = t->lst[k];
        const double d1 = X - t->x[i], d2 = Y - t->y[i];
        cnt[3]++;
        if (decide(tp, inside_of(t, i, d1, d2))) {
            double te[7], tpnt[7], de[9], dpnt[9];
            cnt[4]++;
            terms_of(t, i, d1, d2, 1, te);
            terms_of(t, i, d1, d2, 0, tpnt);
            dterms_of(t, i, d1, d2, 1, adj, de);
            dterms_of(t, i, d1, d2, 0, adj, dpnt);
            particle_term(t, i, te, de, 1.0, acc, adj);
            particle_term(t, i, tpnt, dpnt, -1.0, acc, adj);
            if (psi)
                *psi += t->m[i] * (psi_of(t, i, d1, d2, 1) - psi_of(t, i, d1, d2, 0));
        }
    }
    const double w1 = X - cl->cx, w2 = Y - cl->cy;
    if (decide(tp, w1 * w1 + w2 * w2 > cl->rcut2)) {
        cnt[1]++;
        const double complex* Q = t->Q + c * (t->p + 1);
        if (!adj) {
            multipole(Q, t->p, w1, w2, acc);
            if (psi) *psi += multipole_psi(Q, t->p, w1, w2);
        } else {
            /* L = Re[gh F + gg F'] with F = sum_k Q_k w^-(k+1) = alpha1 - i alpha2,
             * F' = gamma1 - i gamma2, gh = ga1 + i ga2, gg = gg1 + i gg2; w = z - z_cm, so
             * dL/dQ_k = gh w^-(k+1) - gg (k+1) w^-(k+2), dL/dz_cm = -(gh F' + gg F'') */
            const double complex w = w1 + I * w2, iw = 1.0 / w;
            const double complex gh = adj->ga[0] + I * adj->ga[1];
            const double complex gg = adj->ga[3] + I * adj->ga[4];
            double complex pw = iw;
            for (int k = 0; k <= t->p; ++k) {
                adj->Abar[c * (t->p + 1) + k] += gh * pw - gg * (double)(k + 1) * pw * iw;
                adj->Bbar[c] += gh * (double)(k + 1) * Q[k] * pw * iw;
                adj->Bbar[c] -= gg * (double)((k + 1) * (k + 2)) * Q[k] * pw * iw * iw;
                pw *= iw;
            }
        }
    } else if (cl->leaf) {
        for (int64_t k = cl->beg; k < cl->end; ++k) {
            const int64_t j = t->perm[k];
            const double d1 = X - t->x[j], d2 = Y - t->y[j];
            const int in = t->listed_at[j] >= 0 ? 0 : decide(tp, inside_of(t, j, d1, d2));
            double tt[7], dt[9];
            cnt[2]++;
            terms_of(t, j, d1, d2, in, tt);
            dterms_of(t, j, d1, d2, in, adj, dt);
            particle_term(t, j, tt, dt, 1.0, acc, adj);
            if (psi) *psi += t->m[j] * psi_of(t, j, d1, d2, in);
        }
    } else {
        for (int k = 0; k < cl->nchild; ++k) visit(t, cl->child[k], X, Y, acc, cnt, tp, adj, psi);
    }
}

int ora_tree_shoot(const ora_tree* t, const double* rx, const double* ry, int64_t nr, double* a1,
                   double* a2, double* kap, double* g1, double* g2, int64_t* counts, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t r = 0; r < nr; ++r) {
        double acc[5] = {0, 0, 0, 0, 0};
        int64_t cnt[5] = {0, 0, 0, 0, 0};
        visit(t, 0, rx[r], ry[r], acc, cnt, NULL, NULL, NULL);
        a1[r] = acc[0];
        a2[r] = acc[1];
        kap[r] = acc[2];
        g1[r] = acc[3];
        g2[r] = acc[4];
        if (counts)
            for (int k = 0; k < 5; ++k) counts[r * 5 + k] = cnt[k];
    }
    return 0;
}

int ora_tree_shoot_psi(const ora_tree* t, const double* rx, const double* ry, int64_t nr, double* psi, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t r = 0; r < nr; ++r) {
        double acc[5] = {0, 0, 0, 0, 0}, ps = 0.0;
        int64_t cnt[5] = {0, 0, 0, 0, 0};
        visit(t, 0, rx[r], ry[r], acc, cnt, NULL, NULL, &ps);
        psi[r] = ps;
    }
    return 0;
}

int ora_tree_record(ora_tree* t, const double* rx, const double* ry, int64_t nr)
{
    for (int64_t r = 0; r < t->ntapes; ++r) free(t->tapes[r].buf);
    free(t->tapes);
    t->tapes = (tape_t*)calloc((size_t)nr, sizeof(tape_t));
    t->ntapes = nr;
    for (int64_t r = 0; r < nr; ++r) {
        double acc[5] = {0, 0, 0, 0, 0};
        int64_t cnt[5] = {0, 0, 0, 0, 0};
        t->tapes[r].mode = 1;
        visit(t, 0, rx[r], ry[r], acc, cnt, &t->tapes[r], NULL, NULL);
        t->tapes[r].mode = 2;
    }
    return 0;
}

int ora_tree_set_particles(ora_tree* t, const double* x, const double* y, const double* m,
                           const double* s)
{
    memcpy(t->x, x, (size_t)t->n * sizeof(double));
    memcpy(t->y, y, (size_t)t->n * sizeof(double));
    memcpy(t->m, m, (size_t)t->n * sizeof(double));
    if (s) memcpy(t->s, s, (size_t)t->n * sizeof(double));
    for (int64_t c = 0; c < t->nc; ++c) cell_moments(t, c);
    return 0;
}

int ora_tree_shoot_frozen(const ora_tree* t, const double* rx, const double* ry, int64_t nr,
                          double* a1, double* a2, double* kap, double* g1, double* g2)
{
    if (nr != t->ntapes) return -1;
    for (int64_t r = 0; r < nr; ++r) {
        double acc[5] = {0, 0, 0, 0, 0};
        int64_t cnt[5] = {0, 0, 0, 0, 0};
        tape_t tp = t->tapes[r];
        tp.pos = 0;
        visit(t, 0, rx[r], ry[r], acc, cnt, &tp, NULL, NULL);
        a1[r] = acc[0];
        a2[r] = acc[1];
        kap[r] = acc[2];
        g1[r] = acc[3];
        g2[r] = acc[4];
    }
    return 0;
}

/* --------------------------------------------------------------- adjoint */

/*
 * With g_hat = ga1 + i ga2 and F = alpha1 - i alpha2, dL = Re(g_hat dF).
 * An accepted box contributes F = sum_k Q_k w^-(k+1) with w = z - z_cm, so
 *   dL = Re( sum_k Abar_k dQ_k + Bbar dz_cm ),
 *   Abar_k = sum_r g_hat w^-(k+1),  Bbar = sum_r g_hat sum_k (k+1) Q_k w^-(k+2).
 * For a member i with d_i = z_i - z_cm and box mass M:
 *   dQ_k/dm_i = d_i^k - k Q_{k-1} d_i / M,   dz_cm/dm_i = d_i / M,
 *   dQ_k/dz_i = k m_i d_i^(k-1) - k Q_{k-1} m_i / M,   dz_cm/dz_i = m_i / M,
 * all holomorphic in z_i, so dL/dx_i = Re G, dL/dy_i = -Im G.
 */
int ora_tree_grad(const ora_tree* t, const double* rx, const double* ry, int64_t nr,
                  const double* ga1, const double* ga2, double* dm, double* dx, double* dy,
                  double* ds)
{
    return ora_tree_grad_kg(t, rx, ry, nr, ga1, ga2, NULL, NULL, NULL, dm, dx, dy, ds);
}

int ora_tree_grad_kg(const ora_tree* t, const double* rx, const double* ry, int64_t nr,
                     const double* ga1, const double* ga2, const double* gk, const double* gg1,
                     const double* gg2, double* dm, double* dx, double* dy, double* ds)
{
    const int P = t->p + 1;
    adj_t adj;
    double* ds_local = ds ? ds : (double*)malloc((size_t)t->n * sizeof(double));
    memset(dm, 0, (size_t)t->n * sizeof(double));
    memset(dx, 0, (size_t)t->n * sizeof(double));
    memset(dy, 0, (size_t)t->n * sizeof(double));
    memset(ds_local, 0, (size_t)t->n * sizeof(double));
    adj.dm = dm;
    adj.dx = dx;
    adj.dy = dy;
    adj.ds = ds_local;
    adj.Abar = (double complex*)calloc((size_t)t->nc * (size_t)P, sizeof(double complex));
    adj.Bbar = (double complex*)calloc((size_t)t->nc, sizeof(double complex));
    for (int64_t r = 0; r < nr; ++r) {
        double acc[5] = {0, 0, 0, 0, 0};
        int64_t cnt[5] = {0, 0, 0, 0, 0};
        double g[5] = {ga1[r], ga2[r], gk ? gk[r] : 0.0, gg1 ? gg1[r] : 0.0, gg2 ? gg2[r] : 0.0};
        adj.ga = g;
        visit(t, 0, rx[r], ry[r], acc, cnt, NULL, &adj, NULL);
    }
    for (int64_t c = 0; c < t->nc; ++c) {
        const ocell* cl = &t->cells[c];
        const double complex* Ab = adj.Abar + c * P;
        const double complex Bb = adj.Bbar[c];
        const double complex* Q = t->Q + c * P;
        int any = Bb != 0;
        for (int k = 0; k < P; ++k) any |= Ab[k] != 0;
        if (!any) continue;
        for (int64_t kk = cl->beg; kk < cl->end; ++kk) {
            const int64_t i = t->perm[kk];
            const double mi = t->m[i];
            const double complex d = (t->x[i] - cl->cx) + I * (t->y[i] - cl->cy);
            double complex sm = 0, sz = 0, dk = 1.0, dkm1 = 0.0;
            for (int k = 0; k < P; ++k) {
                const double complex Qm1 = k > 0 ? Q[k - 1] : 0.0;
                double complex dQdm = dk, dQdz = (double)k * mi * dkm1;
                if (cl->M > 0) {
                    dQdm -= (double)k * Qm1 * d / cl->M;
                    dQdz -= (double)k * Qm1 * mi / cl->M;
                }
                sm += Ab[k] * dQdm;
                sz += Ab[k] * dQdz;
                dkm1 = dk;
                dk *= d;
            }
            if (cl->M > 0) {
                sm += Bb * d / cl->M;
                sz += Bb * mi / cl->M;
            }
            dm[i] += creal(sm);
            dx[i] += creal(sz);
            dy[i] -= cimag(sz);
        }
    }
    free(adj.Abar);
    free(adj.Bbar);
    if (!ds) free(ds_local);
    return 0;
}
