/*
 * CPU oracle for the lensing hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 reference implementations used by the tests, the smoke
 * check and the benchmark's CPU-baseline leg.  Nothing in the product path
 * links, loads or calls this code, and it shares no source with the GPU
 * library.
 *
 *   oracle A  (direct.c) : brute-force superposition of every particle
 *                          (Sec. 3.2, "superposition"; Sec. 5.1, theta = 0).
 *   oracle B  (tree.c)   : the modified quad-tree solver of Sec. 3.2 written
 *                          out as a pointer-free recursive tree in FP64.
 *
 * Code units: masses are m / (pi Sigma_crit), so a point mass deflects
 * alpha = m d / |d|^2 and its Einstein radius is sqrt(m) (Sec. 3.5).
 */
#ifndef GLAMER_ORACLE_H
#define GLAMER_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Contribution of one particle at offset d = ray - particle.
 * Per unit mass; `inside` selects the truncated Gaussian kernel, otherwise the
 * point-mass form.  out: a1 a2 kappa g1 g2 da1/ds da2/ds. */
void ora_unit_terms(double d1, double d2, double s, double q, int inside, double out[7]);
/* Per unit mass: derivatives of kappa, gamma1, gamma2 with respect to the
 * offset (d1, d2) and to s: dk/dd1, dk/dd2, dg1/dd1, dg1/dd2, dg2/dd1,
 * dg2/dd2, dk/ds, dg1/ds, dg2/ds. */
void ora_unit_dterms(double d1, double d2, double s, double q, int inside, double out[9]);

/* Lensing potential of one particle per unit mass (point mass: ln r; the
 * truncated Gaussian inside its support: ln(q s) - (Ein(q^2/2) - Ein(u)) / (2C)). */
double ora_unit_psi(double d1, double d2, double s, double q, int inside);

/* Ein(z) = integral_0^z (1 - exp(-t)) / t dt. */
double ora_ein(double z);

/* inside the truncated support: s > 0 and r^2 < (q s)^2 (Sec. 3.1) */
int ora_inside(double d1, double d2, double s, double q);

/* 1 - exp(-q^2/2), the kernel normalisation of the truncated Gaussian. */
double ora_kernel_norm(double q);

/* Oracle A: FP64 brute force.  Outputs are overwritten. */
int ora_direct(const double* x, const double* y, const double* m, const double* s, int64_t n,
               double q, const double* rx, const double* ry, int64_t nr,
               double* a1, double* a2, double* kap, double* g1, double* g2, int nthreads);

/* Oracle A for the potential psi (alpha = grad psi, Sec. 3.2). */
int ora_direct_psi(const double* x, const double* y, const double* m, const double* s, int64_t n, double q,
                   const double* rx, const double* ry, int64_t nr, double* psi, int nthreads);

/* Oracle A adjoint: gradient of L = sum_r ga_r . alpha_r with respect to the
 * particle masses, positions and smoothing lengths (FP64 brute force). */
int ora_direct_grad(const double* x, const double* y, const double* m, const double* s, int64_t n,
                    double q, const double* rx, const double* ry, int64_t nr,
                    const double* ga1, const double* ga2,
                    double* dm, double* dx, double* dy, double* ds, int nthreads);
/* The same for L = sum_r ga_r . alpha_r + gk_r kappa_r + gg_r . gamma_r
 * (gk, gg1, gg2 nullable: zero). */
int ora_direct_grad_kg(const double* x, const double* y, const double* m, const double* s, int64_t n,
                       double q, const double* rx, const double* ry, int64_t nr,
                       const double* ga1, const double* ga2, const double* gk, const double* gg1,
                       const double* gg2, double* dm, double* dx, double* dy, double* ds, int nthreads);

/* Smoothing lengths (Sec. 3.1): for each particle the 2D distance to its
 * k-th nearest other particle, by brute force.  Returns -1 unless
 * 1 <= k <= n - 1. */
int ora_knn(const double* x, const double* y, int64_t n, int k, double* s_out, int nthreads);
/* The same for the particles queries[0..nq-1] only (out[t] for queries[t]). */
int ora_knn_at(const double* x, const double* y, int64_t n, int k, const int64_t* queries, int64_t nq,
               double* s_out, int nthreads);
/* General form: 3D distances when z is not NULL, and only particles of the
 * same species when species is not NULL (queries may be NULL: all n).
 * Returns -1 unless 1 <= k <= n - 1 and every queried particle has at least k
 * others of its species (those get NaN). */
int ora_knn_ex(const double* x, const double* y, const double* z, const int32_t* species, int64_t n, int k,
               const int64_t* queries, int64_t nq, double* s_out, int nthreads);

/* Truncated NFW halos (nfw.c): shape functions of the projected profile,
 * per-unit-mass terms (a1 a2 kappa g1 g2, 0 0) of a halo of size R and
 * concentration c, inside test r < R, and the brute force. */
double ora_nfw_F(double x);
double ora_nfw_f(double x);
double ora_nfw_g(double x);
int ora_nfw_inside(double d1, double d2, double R);
void ora_nfw_terms(double d1, double d2, double R, double c, int inside, double out[7]);
/* NFW derivatives: f'(x), and per unit mass d(kappa, gamma) by offset and size
 * (as ora_unit_dterms; ora_nfw_terms gives d alpha / dR in out[5..6]). */
double ora_nfw_df(double x);
void ora_nfw_dterms(double d1, double d2, double R, double c, int inside, double out[9]);
/* NFW potential: H(x) with H' = g(x)/x, psi per unit mass, and the direct sum. */
double ora_nfw_H(double x);
double ora_nfw_psi(double d1, double d2, double R, double c, int inside);
int ora_direct_nfw_psi(const double* x, const double* y, const double* m, const double* R, int64_t n, double c,
                       const double* rx, const double* ry, int64_t nr, double* psi, int nthreads);
int ora_direct_nfw(const double* x, const double* y, const double* m, const double* R, int64_t n, double c,
                   const double* rx, const double* ry, int64_t nr, double* a1, double* a2, double* kap,
                   double* g1, double* g2, int nthreads);

/* Oracle B: reference tree. */
typedef struct ora_tree ora_tree;

ora_tree* ora_tree_build(const double* x, const double* y, const double* m, const double* s,
                         int64_t n, double q, double theta, int leaf_size, int order);
/* The same tree of truncated NFW halos: sizes R (support), concentration c. */
ora_tree* ora_tree_build_nfw(const double* x, const double* y, const double* m, const double* R, int64_t n,
                             double c, double theta, int leaf_size, int order);
void ora_tree_free(ora_tree* t);
int64_t ora_tree_ncells(const ora_tree* t);
/* root square: x0, y0, side */
void ora_tree_root(const ora_tree* t, double out[3]);
/* Per cell, in depth-first preorder with children in Morton order. */
void ora_tree_export(const ora_tree* t, int32_t* level, uint32_t* ix, uint32_t* iy,
                     int32_t* np, int32_t* leaf, int32_t* nl, int64_t* next,
                     double* M, double* cx, double* cy, double* rcut2, double* Q /* 2(p+1) */);
/* Member / list particle indices of one cell, ascending. Returns count. */
int64_t ora_tree_members(const ora_tree* t, int64_t cell, int32_t* out);
int64_t ora_tree_list(const ora_tree* t, int64_t cell, int32_t* out);

/* Forward walk.  counts (nullable) receives per ray:
 *   [0] cells visited (MAC tests)  [1] cells accepted  [2] leaf particles summed
 *   [3] list entries examined      [4] list particles the ray falls inside */
int ora_tree_shoot(const ora_tree* t, const double* rx, const double* ry, int64_t nr,
                   double* a1, double* a2, double* kap, double* g1, double* g2,
                   int64_t* counts, int nthreads);

/* The potential psi along the same walk (boxes: Re[Q_0 ln w - sum Q_k / (k w^k)];
 * leaves and list corrections from ora_unit_psi). */
int ora_tree_shoot_psi(const ora_tree* t, const double* rx, const double* ry, int64_t nr, double* psi,
                       int nthreads);

/* Decision tape: record every branch of the walk for these rays, then replay
 * it after ora_tree_set_particles has changed masses/positions/smoothing
 * (membership, lists and accept/open/inside decisions stay frozen). */
int ora_tree_record(ora_tree* t, const double* rx, const double* ry, int64_t nr);
int ora_tree_set_particles(ora_tree* t, const double* x, const double* y, const double* m,
                           const double* s);
int ora_tree_shoot_frozen(const ora_tree* t, const double* rx, const double* ry, int64_t nr,
                          double* a1, double* a2, double* kap, double* g1, double* g2);

/* Adjoint of the tree walk for L = sum_r ga_r . alpha_r (decisions of the
 * unperturbed walk), FP64. */
int ora_tree_grad(const ora_tree* t, const double* rx, const double* ry, int64_t nr,
                  const double* ga1, const double* ga2,
                  double* dm, double* dx, double* dy, double* ds);
/* The same for L = sum_r ga_r . alpha_r + gk_r kappa_r + gg_r . gamma_r
 * (gk, gg1, gg2 nullable); ds is the derivative by s, or by the size R for a
 * tree of NFW halos (fixed concentration). */
int ora_tree_grad_kg(const ora_tree* t, const double* rx, const double* ry, int64_t nr,
                     const double* ga1, const double* ga2, const double* gk, const double* gg1,
                     const double* gg2, double* dm, double* dx, double* dy, double* ds);

#ifdef __cplusplus
}
#endif
#endif
