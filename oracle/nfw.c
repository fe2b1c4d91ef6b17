/*
 * Oracle for truncated NFW halos as "particles" (Sec. 3.2: every particle
 * type has its own expressions for the lensing quantities; outside its outer
 * radius a spherically symmetric profile lenses like a point mass) --
 * TEST INFRASTRUCTURE ONLY.
 *
 * A halo of mass m, size (truncation radius) R and concentration c has the
 * projected NFW surface density, cut at projected radius R and normalised so
 * that its mass inside R is m.  With r_s = R / c and x = r / r_s:
 *   F(x) = arccosh(1/x) / sqrt(1 - x^2) (x < 1), arccos(1/x) / sqrt(x^2 - 1) (x > 1), 1 at x = 1;
 *   f(x) = (1 - F(x)) / (x^2 - 1)   (surface-density shape, f(1) = 1/3);
 *   g(x) = ln(x / 2) + F(x)         (enclosed-mass shape, g' = x f, g(0) = 0).
 * Inside R: alpha = m G d / r^2 with G = g(x) / g(c); kappa = m f(x) / (2 r_s^2 g(c));
 * gamma = -(m G / r^2 - kappa)(cos 2phi, sin 2phi).  Outside: a point mass.
 * Near x = 1 the formulas are 0/0: there (|e| < 1e-2) the series
 * F = sum_k (-e)^k / (2k + 1), e = x^2 - 1, is used, converged to rounding by
 * 12 terms.  For x < 1 the two large logarithms of g cancel; g is
 * regrouped so that they do not (see ora_nfw_g).
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

double ora_nfw_F(double x)
{
    const double e = (x - 1.0) * (x + 1.0); /* x^2 - 1 without cancellation near x = 1 */
    if (fabs(e) < 1e-2) {
        double s = 0.0, p = 1.0;
        for (int k = 0; k < 12; ++k) {
            s += p / (double)(2 * k + 1);
            p *= -e;
        }
        return s;
    }
    /* arccosh(1/x) = ln((1 + y) / x) = log1p((y + (1 - x)) / x) and
     * arccos(1/x) = atan(y): the same values as the textbook forms, without
     * arguments near 1 where those lose digits */
    if (x < 1.0) {
        const double y = sqrt(-e);
        return log1p((y + (1.0 - x)) / x) / y;
    }
    const double y = sqrt(e);
    return atan(y) / y;
}

double ora_nfw_f(double x)
{
    const double e = (x - 1.0) * (x + 1.0); /* x^2 - 1 without cancellation near x = 1 */
    if (fabs(e) < 1e-2) { /* (1 - F) / e = sum_{k>=1} (-1)^(k+1) e^(k-1) / (2k + 1) */
        double s = 0.0, p = 1.0;
        for (int k = 1; k < 13; ++k) {
            s += p / (double)(2 * k + 1);
            p *= -e;
        }
        return s;
    }
    return (1.0 - ora_nfw_F(x)) / e;
}

double ora_nfw_g(double x)
{
    if (x <= 0.0) return 0.0;
    const double e = (x - 1.0) * (x + 1.0); /* x^2 - 1 without cancellation near x = 1 */
    if (x < 1.0 && fabs(e) >= 1e-2) {
        /* ln(x/2) + arccosh(1/x)/y with y = sqrt(1 - x^2), arccosh(1/x) = L + ln((1+y)/2),
         * L = ln(2/x): both large terms cancel; regrouped without cancellation as
         * [L x^2 / (1 + y) + log1p(-x^2 / (2 (1 + y)))] / y */
        const double y = sqrt(-e), L = log(2.0 / x), x2 = x * x;
        return (L * x2 / (1.0 + y) + log1p(-x2 / (2.0 * (1.0 + y)))) / y;
    }
    return log(0.5 * x) + ora_nfw_F(x);
}

int ora_nfw_inside(double d1, double d2, double R)
{
    return R > 0.0 && d1 * d1 + d2 * d2 < R * R;
}

/* f'(x): (3 x F - 2 x - 1/x) / (x^2 - 1)^2, or near x = 1 from the series of f
 * in e = x^2 - 1 (f = sum (-e)^k / (2k + 3), so df/dx = 2x sum_{k>=1} k (-1)^k e^(k-1) / (2k + 3)). */
double ora_nfw_df(double x)
{
    const double e = (x - 1.0) * (x + 1.0);
    if (fabs(e) < 1e-2) {
        double s = 0.0, p = 1.0; /* p = e^(k-1) */
        for (int k = 1; k < 14; ++k) {
            s += ((k & 1) ? -1.0 : 1.0) * (double)k * p / (double)(2 * k + 3);
            p *= e;
        }
        return 2.0 * x * s;
    }
    return (3.0 * x * ora_nfw_F(x) - 2.0 * x - 1.0 / x) / (e * e);
}

/* per unit mass: out = a1 a2 kappa g1 g2, and d(a1, a2)/dR at fixed c; a ray
 * exactly at the centre gets nothing (alpha and gamma vanish by symmetry;
 * kappa diverges there).  With G = g(x)/g(c), x = r c / R:
 * dG/dR = -x g'(x) / (R g(c)) = -x^2 f(x) / (R g(c)). */
void ora_nfw_terms(double d1, double d2, double R, double c, int inside, double out[7])
{
    memset(out, 0, 7 * sizeof(double));
    const double r2 = d1 * d1 + d2 * d2;
    if (r2 == 0.0) return;
    double G = 1.0, K = 0.0, dGR = 0.0;
    if (inside) {
        const double rs = R / c, x = sqrt(r2) / rs, gc = ora_nfw_g(c);
        G = ora_nfw_g(x) / gc;
        K = ora_nfw_f(x) / (2.0 * rs * rs * gc);
        dGR = -x * x * ora_nfw_f(x) / (R * gc);
    }
    out[5] = dGR * d1 / r2;
    out[6] = dGR * d2 / r2;
    const double h = G / r2;
    out[0] = h * d1;
    out[1] = h * d2;
    out[2] = K;
    const double Gam = h - K;
    out[3] = -Gam * (d1 * d1 - d2 * d2) / r2;
    out[4] = -Gam * 2.0 * d1 * d2 / r2;
}

/* Per unit mass, as ora_unit_dterms for the halo: d(kappa, gamma1, gamma2)
 * with respect to the offset and to the size R (fixed c).  kappa(r) =
 * f(x) / (2 r_s^2 g(c)), A = G / r^2, Gam = A - kappa:
 *   dkappa/dr = f'(x) (c / R) / (2 r_s^2 g(c)),
 *   dA/dr = x f(x) (c / R) / (g(c) r^2) - 2 A / r,
 *   dkappa/dR = -(x f'(x) + 2 f(x)) / (2 r_s^2 R g(c)),  dA/dR = (dG/dR) / r^2. */
void ora_nfw_dterms(double d1, double d2, double R, double c, int inside, double out[9])
{
    memset(out, 0, 9 * sizeof(double));
    const double r2 = d1 * d1 + d2 * d2;
    if (r2 == 0.0) return;
    const double r = sqrt(r2), r4 = r2 * r2;
    double A = 1.0 / r2, K = 0.0, dKr = 0.0, dAr = -2.0 / (r2 * r), dKR = 0.0, dAR = 0.0;
    if (inside) {
        const double rs = R / c, x = r / rs, gc = ora_nfw_g(c), f = ora_nfw_f(x), df = ora_nfw_df(x);
        A = ora_nfw_g(x) / gc / r2;
        K = f / (2.0 * rs * rs * gc);
        dKr = df * (c / R) / (2.0 * rs * rs * gc);
        dAr = x * f * (c / R) / (gc * r2) - 2.0 * A / r;
        dKR = -(x * df + 2.0 * f) / (2.0 * rs * rs * R * gc);
        dAR = -x * x * f / (R * gc) / r2;
    }
    const double Gam = A - K, dGr = dAr - dKr, dGR = dAR - dKR;
    const double cc = (d1 * d1 - d2 * d2) / r2, sn = 2.0 * d1 * d2 / r2;
    const double dc1 = 4.0 * d1 * d2 * d2 / r4, dc2 = -4.0 * d2 * d1 * d1 / r4;
    const double dsn1 = 2.0 * d2 * (d2 * d2 - d1 * d1) / r4, dsn2 = 2.0 * d1 * (d1 * d1 - d2 * d2) / r4;
    out[0] = dKr * d1 / r;
    out[1] = dKr * d2 / r;
    out[2] = -dGr * (d1 / r) * cc - Gam * dc1;
    out[3] = -dGr * (d2 / r) * cc - Gam * dc2;
    out[4] = -dGr * (d1 / r) * sn - Gam * dsn1;
    out[5] = -dGr * (d2 / r) * sn - Gam * dsn2;
    out[6] = dKR;
    out[7] = -dGR * cc;
    out[8] = -dGR * sn;
}

int ora_direct_nfw(const double* x, const double* y, const double* m, const double* R, int64_t n, double c,
                   const double* rx, const double* ry, int64_t nr, double* a1, double* a2, double* kap,
                   double* g1, double* g2, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t r = 0; r < nr; ++r) {
        double acc[5] = {0, 0, 0, 0, 0};
        for (int64_t i = 0; i < n; ++i) {
            const double d1 = rx[r] - x[i], d2 = ry[r] - y[i];
            double t[7];
            ora_nfw_terms(d1, d2, R[i], c, ora_nfw_inside(d1, d2, R[i]), t);
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

/* Potential (alpha = grad psi, Sec. 3.2).  H(x) = ln^2(x/2)/2 - arccosh^2(1/x)/2 for
 * x < 1 and ln^2(x/2)/2 + arccos^2(1/x)/2 for x > 1 has H' = g(x)/x, so inside R
 *   psi = m [H(x) - H(c)] / g(c) + m ln R,
 * which joins the point mass's m ln r at r = R; outside, psi = m ln r.  The two
 * inverse functions are taken as log1p((y + 1 - x)/x) and atan(y) with
 * y = sqrt|x^2 - 1| (the same values, without arguments near 1). */
double ora_nfw_H(double x)
{
    const double e = (x - 1.0) * (x + 1.0), L = log(0.5 * x);
    if (x < 1.0) {
        const double y = sqrt(-e), a = log1p((y + (1.0 - x)) / x);
        return 0.5 * L * L - 0.5 * a * a;
    }
    const double y = sqrt(e), a = atan(y);
    return 0.5 * L * L + 0.5 * a * a;
}

/* per unit mass; a ray exactly at the centre gets the value of the limit x -> 0
 * would be -inf there, so 0 is returned for r = 0 as for alpha */
double ora_nfw_psi(double d1, double d2, double R, double c, int inside)
{
    const double r2 = d1 * d1 + d2 * d2;
    if (r2 == 0.0) return 0.0;
    if (!inside) return 0.5 * log(r2);
    const double x = sqrt(r2) * c / R;
    return (ora_nfw_H(x) - ora_nfw_H(c)) / ora_nfw_g(c) + log(R);
}

int ora_direct_nfw_psi(const double* x, const double* y, const double* m, const double* R, int64_t n, double c,
                       const double* rx, const double* ry, int64_t nr, double* psi, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t r = 0; r < nr; ++r) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double d1 = rx[r] - x[i], d2 = ry[r] - y[i];
            acc += m[i] * ora_nfw_psi(d1, d2, R[i], c, ora_nfw_inside(d1, d2, R[i]));
        }
        psi[r] = acc;
    }
    return 0;
}
