/*
 * Oracle A -- FP64 brute-force superposition.  TEST INFRASTRUCTURE ONLY.
 *
 * Every ray sums the contribution of every particle (Sec. 3.2: the lensing
 * quantities obey superposition; Sec. 5.1: theta_force = 0 is this direct
 * sum).  Nothing here is blocked, reordered or approximated.
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

/* Normalisation of the truncated Gaussian surface density (Sec. 3.1): the
 * kernel is divided by 1 - exp(-q^2/2) so that its total mass is m. */
double ora_kernel_norm(double q) { return -expm1(-0.5 * q * q); }

/*
 * One particle, per unit mass, at offset d = ray - particle.
 *
 * Deflection (Sec. 3.2, smoothed particle; Sec. 3.5, star):
 *   alpha = G(r) d / r^2, G = (1 - exp(-u)) / C inside the support, 1 outside,
 *   u = r^2 / (2 s^2), C = 1 - exp(-q^2/2).  The printed exponent lacks the
 *   square on the smoothing length; the square is what makes alpha the
 *   enclosed mass of the Gaussian of Sec. 3.1 (checked by the kappa = div/2
 *   tests).
 * Convergence kappa = (1/2) div alpha (Sec. 3.2) = exp(-u) / (2 s^2 C) inside,
 *   0 outside.
 * Shear gamma1 = (d1 a1 - d2 a2)/2, gamma2 = d1 a2 (Sec. 3.2).  For
 *   alpha = f(r) d one finds gamma = (kappa - G/r^2) (d1^2 - d2^2, 2 d1 d2)/r^2.
 * Smoothing derivative d alpha / d s = -d exp(-u) / (s^3 C) inside, 0 outside.
 */
void ora_unit_terms(double d1, double d2, double s, double q, int inside, double out[7])
{
    memset(out, 0, 7 * sizeof(double));
    const double r2 = d1 * d1 + d2 * d2;
    const double C = ora_kernel_norm(q);
    if (r2 == 0.0) {
        /* a ray exactly on a particle: alpha and gamma vanish by symmetry */
        if (inside) out[2] = 1.0 / (2.0 * s * s * C);
        return;
    }
    double G = 1.0, K = 0.0, dG = 0.0;
    if (inside) {
        const double u = r2 / (2.0 * s * s);
        const double e = exp(-u);
        G = -expm1(-u) / C;
        K = e / (2.0 * s * s * C);
        dG = -e / (s * s * s * C); /* (d alpha / d s) = dG * d */
    }
    const double h = G / r2;
    out[0] = h * d1;
    out[1] = h * d2;
    out[2] = K;
    const double Gam = h - K;
    out[3] = -Gam * (d1 * d1 - d2 * d2) / r2;
    out[4] = -Gam * 2.0 * d1 * d2 / r2;
    out[5] = dG * d1;
    out[6] = dG * d2;
}

/*
 * Derivatives of kappa and gamma of one particle, per unit mass, with respect
 * to the offset d = ray - particle and to the smoothing length s (for the
 * adjoint of L = sum_r gk_r kappa_r + gg_r . gamma_r).  Every circular profile
 * has kappa(r) and gamma = -Gam(r) (c, sn) with c = (d1^2 - d2^2)/r^2,
 * sn = 2 d1 d2 / r^2, Gam = A - kappa, A = G(r)/r^2 (G = enclosed-mass
 * fraction, G' = 2 r kappa):
 *   d kappa / d d_j = kappa'(r) d_j / r,
 *   d gamma1 / d d_j = -Gam'(r) (d_j / r) c - Gam dc/dd_j   (likewise gamma2 with sn),
 *   A' = 2 kappa / r - 2 A / r,  Gam' = A' - kappa'.
 * Gaussian inside: kappa' = -(r / s^2) kappa; d kappa / d s = e^-u (u - 1)/(s^3 C),
 * d A / d s = -e^-u / (s^3 C).  Point mass: kappa = 0, A = 1/r^2.  A ray exactly
 * on the particle gets 0.
 * out = dk/dd1, dk/dd2, dg1/dd1, dg1/dd2, dg2/dd1, dg2/dd2, dk/ds, dg1/ds, dg2/ds.
 */
void ora_unit_dterms(double d1, double d2, double s, double q, int inside, double out[9])
{
    memset(out, 0, 9 * sizeof(double));
    const double r2 = d1 * d1 + d2 * d2;
    if (r2 == 0.0) return;
    const double C = ora_kernel_norm(q);
    const double r = sqrt(r2), r4 = r2 * r2;
    double A = 1.0 / r2, K = 0.0, dKr = 0.0, dKs = 0.0, dAs = 0.0;
    if (inside) {
        const double u = r2 / (2.0 * s * s), e = exp(-u);
        A = (-expm1(-u) / C) / r2;
        K = e / (2.0 * s * s * C);
        dKr = -(r / (s * s)) * K;
        dKs = e * (u - 1.0) / (s * s * s * C);
        dAs = -e / (s * s * s * C);
    }
    const double dAr = 2.0 * K / r - 2.0 * A / r;
    const double Gam = A - K, dGr = dAr - dKr, dGs = dAs - dKs;
    const double c = (d1 * d1 - d2 * d2) / r2, sn = 2.0 * d1 * d2 / r2;
    const double dc1 = 4.0 * d1 * d2 * d2 / r4, dc2 = -4.0 * d2 * d1 * d1 / r4;
    const double dsn1 = 2.0 * d2 * (d2 * d2 - d1 * d1) / r4, dsn2 = 2.0 * d1 * (d1 * d1 - d2 * d2) / r4;
    out[0] = dKr * d1 / r;
    out[1] = dKr * d2 / r;
    out[2] = -dGr * (d1 / r) * c - Gam * dc1;
    out[3] = -dGr * (d2 / r) * c - Gam * dc2;
    out[4] = -dGr * (d1 / r) * sn - Gam * dsn1;
    out[5] = -dGr * (d2 / r) * sn - Gam * dsn2;
    out[6] = dKs;
    out[7] = -dGs * c;
    out[8] = -dGs * sn;
}

/* Ein(z) = int_0^z (1 - e^-t) / t dt = sum_{k>=1} (-1)^(k+1) z^k / (k k!), an
 * entire function; the series is summed until its terms stop changing the
 * sum (z <= q^2 / 2 here, a few dozen terms). */
double ora_ein(double z)
{
    double term = z, sum = 0.0; /* term = (-1)^(k+1) z^k / k! */
    for (int k = 1; k < 400; ++k) {
        const double add = term / (double)k;
        const double next = sum + add;
        if (next == sum && k > 1) break;
        sum = next;
        term *= -z / (double)(k + 1);
    }
    return sum;
}

/*
 * Lensing potential of one particle, per unit mass, at offset d (Sec. 3.2:
 * alpha = grad psi).  A point mass has psi = ln r.  The truncated Gaussian
 * equals the point mass outside its support R = q s (its alpha does, and psi
 * is fixed to agree there); inside, integrating d psi / d r = G(r) / r from R,
 *   psi = ln R - (Ein(q^2/2) - Ein(u)) / (2 C),  u = r^2 / (2 s^2).
 * A point mass exactly at the ray contributes 0, like its deflection.
 */
double ora_unit_psi(double d1, double d2, double s, double q, int inside)
{
    const double r2 = d1 * d1 + d2 * d2;
    if (!inside) return r2 > 0.0 ? 0.5 * log(r2) : 0.0;
    const double C = ora_kernel_norm(q);
    return log(q * s) - (ora_ein(0.5 * q * q) - ora_ein(r2 / (2.0 * s * s))) / (2.0 * C);
}

/* inside iff s > 0 and r^2 < (q s)^2 (strict, Sec. 3.1). */
int ora_inside(double d1, double d2, double s, double q)
{
    if (!(s > 0.0)) return 0;
    const double qs = q * s;
    return d1 * d1 + d2 * d2 < qs * qs;
}

int ora_direct(const double* x, const double* y, const double* m, const double* s, int64_t n,
               double q, const double* rx, const double* ry, int64_t nr,
               double* a1, double* a2, double* kap, double* g1, double* g2, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t r = 0; r < nr; ++r) {
        double acc[5] = {0, 0, 0, 0, 0};
        for (int64_t i = 0; i < n; ++i) {
            const double d1 = rx[r] - x[i], d2 = ry[r] - y[i];
            const double si = s ? s[i] : 0.0;
            double t[7];
            ora_unit_terms(d1, d2, si, q, ora_inside(d1, d2, si, q), t);
            for (int k = 0; k < 5; ++k) acc[k] += m[i] * t[k];
        }
        a1[r] = acc[0];
        a2[r] = acc[1];
        kap[r] = acc[2];
        g1[r] = acc[3];
        g2[r] = acc[4];
    }
    return 0;
}

int ora_direct_psi(const double* x, const double* y, const double* m, const double* s, int64_t n, double q,
                   const double* rx, const double* ry, int64_t nr, double* psi, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t r = 0; r < nr; ++r) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double d1 = rx[r] - x[i], d2 = ry[r] - y[i];
            const double si = s ? s[i] : 0.0;
            acc += m[i] * ora_unit_psi(d1, d2, si, q, ora_inside(d1, d2, si, q));
        }
        psi[r] = acc;
    }
    return 0;
}

/*
 * Gradient of L = sum_r (ga1_r alpha1_r + ga2_r alpha2_r).
 *   dL/dm_i = sum_r ga_r . alpha_ri / m_i   (alpha is linear in m_i)
 *   dL/dx_i = -sum_r (J_ri ga_r)_1, dL/dy_i = -sum_r (J_ri ga_r)_2, with the
 *     symmetric magnification-matrix part J = [[k+g1, g2], [g2, k-g1]] of the
 *     single particle (alpha depends on ray - particle only).
 *   dL/ds_i = sum_r ga_r . d alpha_ri / d s_i.
 */
int ora_direct_grad(const double* x, const double* y, const double* m, const double* s, int64_t n,
                    double q, const double* rx, const double* ry, int64_t nr,
                    const double* ga1, const double* ga2,
                    double* dm, double* dx, double* dy, double* ds, int nthreads)
{
    return ora_direct_grad_kg(x, y, m, s, n, q, rx, ry, nr, ga1, ga2, NULL, NULL, NULL, dm, dx, dy, ds, nthreads);
}

int ora_direct_grad_kg(const double* x, const double* y, const double* m, const double* s, int64_t n,
                       double q, const double* rx, const double* ry, int64_t nr,
                       const double* ga1, const double* ga2, const double* gk, const double* gg1,
                       const double* gg2, double* dm, double* dx, double* dy, double* ds, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) {
        double gm = 0, gx = 0, gy = 0, gs = 0;
        const double si = s ? s[i] : 0.0;
        for (int64_t r = 0; r < nr; ++r) {
            const double d1 = rx[r] - x[i], d2 = ry[r] - y[i];
            const int in = ora_inside(d1, d2, si, q);
            double t[7];
            ora_unit_terms(d1, d2, si, q, in, t);
            gm += ga1[r] * t[0] + ga2[r] * t[1];
            gx -= ga1[r] * (t[2] + t[3]) + ga2[r] * t[4];
            gy -= ga1[r] * t[4] + ga2[r] * (t[2] - t[3]);
            gs += ga1[r] * t[5] + ga2[r] * t[6];
            if (gk || gg1 || gg2) {
                const double a = gk ? gk[r] : 0.0, b1 = gg1 ? gg1[r] : 0.0, b2 = gg2 ? gg2[r] : 0.0;
                double dt[9];
                ora_unit_dterms(d1, d2, si, q, in, dt);
                gm += a * t[2] + b1 * t[3] + b2 * t[4];
                gx -= a * dt[0] + b1 * dt[2] + b2 * dt[4];
                gy -= a * dt[1] + b1 * dt[3] + b2 * dt[5];
                gs += a * dt[6] + b1 * dt[7] + b2 * dt[8];
            }
        }
        dm[i] = gm;
        dx[i] = m[i] * gx;
        dy[i] = m[i] * gy;
        if (ds) ds[i] = m[i] * gs;
    }
    return 0;
}
