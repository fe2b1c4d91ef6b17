// Per-lane evaluation of one particle or one accepted box, shared by the
// tree walk, its adjoint and the direct sum.
#pragma once

#include <math.h>

#include "common.hpp"

namespace glm {

// Per-lane accumulators.  Deflection and shear are sums of large terms of
// both signs that nearly cancel near a mass concentration: their FP32 terms
// are added into FP64 accumulators (an FP64 add costs what an FP32 add costs
// on this chip, and is cheaper than compensated FP32 summation).  The
// point-mass terms of big-list particles that a ray lies inside (added once
// with each sign, see leaf_particle) thus cancel there without leaving FP32
// rounding of size m / r behind.  kappa, a sum of positive terms, stays FP32.
// The debug mode without FP64 alpha sums the alpha terms in plain FP32 (p1,
// p2) and keeps only the balanced point terms in a1, a2.
struct Acc {
    double a1, a2;
    float p1, p2, k;
    double g1, g2;
    double ps; // lensing potential (FP64 sum of FP32 terms), when asked for
};

// Ein(u) = integral_0^u (1 - e^-t) / t dt = sum_k c_k u^k with
// c_k = (-1)^(k+1) / (k k!), by Horner in FP64 over the first `terms`
// coefficients (chosen per tree so the series is converged for u <= q^2/2).
constexpr int kEinTerms = 100;
struct EinTable {
    double c[kEinTerms];
};
constexpr EinTable make_ein_table()
{
    EinTable t{};
    double f = 1.0;
    for (int k = 1; k <= kEinTerms; ++k) {
        f *= (double)k;
        t.c[k - 1] = ((k & 1) ? 1.0 : -1.0) / ((double)k * f);
    }
    return t;
}
__constant__ inline EinTable c_ein = make_ein_table();

__device__ inline double ein(double u, int terms)
{
    double s = c_ein.c[terms - 1];
    for (int k = terms - 2; k >= 0; --k) s = fma(s, u, c_ein.c[k]);
    return s * u;
}

// The same series in FP32 where a tree needs at most 34 FP64 terms (u below
// about 4.75, q up to 3): 24 terms leave a tail below 2e-9, the coefficients
// are instruction constants, and the rounding of the alternating sum (about
// 1e-6 absolute at the top of the range) is far below what an FP32 potential
// term resolves.
constexpr int kEin32Terms = 24;
__device__ inline float ein32(float u)
{
    constexpr EinTable t = make_ein_table();
    float s = (float)t.c[kEin32Terms - 1];
#pragma unroll
    for (int k = kEin32Terms - 2; k >= 0; --k) s = fmaf(s, u, (float)t.c[k]);
    return s * u;
}

// Potential of a truncated Gaussian inside its support, per unit mass
// (alpha = grad psi, Sec. 3.2; equal to the point mass's ln r at the edge):
//   ln(q s) - (Ein(q^2/2) - Ein(u)) / (2C),  u = r^2 / (2 s^2).
// Ein(q^2/2) (psiK) is the host's FP64 value; Ein(u) is FP32 up to q = 3
// (terms <= 34 marks that range), FP64 beyond.
__device__ inline float gauss_psi(const PRec& pr, double r2, double psiK, int terms, float invC)
{
    const double u = r2 * (double)pr.h;
    const double e = terms <= 34 ? (double)ein32((float)u) : ein(u, terms);
    return 0.5f * __logf((float)pr.qs2) - (float)((psiK - e) * (0.5 * (double)invC));
}

// alpha += (v1, v2): in FP64, or in plain FP32 when F64A is false (debug)
template <bool F64A>
__device__ inline void add_alpha(Acc& A, float v1, float v2)
{
    if constexpr (F64A) {
        A.a1 += (double)v1;
        A.a2 += (double)v2;
    } else {
        A.p1 += v1;
        A.p2 += v2;
    }
}

// The alpha of one ray from its accumulators
__device__ inline double alpha1(const Acc& A) { return A.a1 + (double)A.p1; }
__device__ inline double alpha2(const Acc& A) { return A.a2 + (double)A.p2; }

// FP64 offset and its squared length, rounded exactly as written (the inside
// and opening decisions must not depend on FMA contraction).
__device__ inline double sqdist(double X, double Y, double px, double py, double* d1, double* d2)
{
#pragma clang fp contract(off)
    *d1 = X - px;
    *d2 = Y - py;
    return (*d1) * (*d1) + (*d2) * (*d2);
}

// Truncated Gaussian (Sec. 3.1) at u = r^2 / (2 s^2), with mC = m / C and
// mh = mC / (2 s^2): the deflection coefficient A (alpha = A d) and
// Gamma = A - kappa (gamma = -Gamma (cos 2phi, sin 2phi)):
//   A = mC (1 - e^-u) / r^2 = mh (1 - e^-u)/u,  Gamma = mh ((1 - e^-u)/u - e^-u).
// Below u = 1/2, where 1 - e^-u cancels, both use their Taylor series.  Each
// branch is evaluated only if some lane of the wavefront needs it.
__device__ inline void gauss_terms(float u, float e, float ir2, float mC, float mh, float* A, float* G)
{
    const bool small = u < 0.5f;
    float As = 0.0f, Gs = 0.0f, Al = 0.0f, Gl = 0.0f;
    if (__any(small)) {
        const float sg = 1.0f +
                         u * (-1.0f / 2 +
                              u * (1.0f / 6 +
                                   u * (-1.0f / 24 +
                                        u * (1.0f / 120 +
                                             u * (-1.0f / 720 + u * (1.0f / 5040 + u * (-1.0f / 40320 + u * (1.0f / 362880))))))));
        const float sd = u * (1.0f / 2 +
                              u * (-1.0f / 3 +
                                   u * (1.0f / 8 +
                                        u * (-1.0f / 30 +
                                             u * (1.0f / 144 + u * (-1.0f / 840 + u * (1.0f / 5760 + u * (-1.0f / 45360 + u * (1.0f / 403200)))))))));
        As = mh * sg;
        Gs = mh * sd;
    }
    if (__any(!small)) {
        Al = mC * (1.0f - e) * ir2;
        Gl = Al - mh * e;
    }
    *A = small ? As : Al;
    *G = small ? Gs : Gl;
}

// ---------------------------------------------------------------------------
// Truncated NFW halo (Sec. 3.2: analytic halos are particles with their own
// closed forms; outside its size a halo lenses as a point mass).  A halo of
// mass m inside its size R and concentration c has scale radius r_s = R / c;
// at x = r / r_s, with e = x^2 - 1,
//   F(x) = atan(y) / y  (x > 1, y = sqrt(e)),   atanh(y) / y  (x < 1, y = sqrt(-e)),
//   f(x) = (1 - F) / e        projected density shape (f(1) = 1/3),
//   g(x) = ln(x / 2) + F      enclosed-mass shape (g' = x f, g(c) normalises m),
// and with mC = m / g(c), h = 1 / r_s:
//   alpha = mC h^2 (g / x^2) d,   kappa = mC h^2 f / 2,   gamma from both.
// nfw_shape returns g / x^2 and f from x^2 and e, both of which the caller
// forms in FP64 from r^2, so that e has no cancellation near x = 1:
//  - |e| < eps: F = sum_k (-e)^k / (2k + 1), f = sum_k (-e)^k / (2k + 3),
//    g = ln x - ln 2 + F with ln x = log1p(e) / 2;
//  - x > 1 beyond: F = atan(y) / y, f = (1 - F) / e, g as above;
//  - x < 1 beyond: atanh(y) = log1p(2 y (1 + y) / x^2) / 2 (as 1 - y = x^2 / (1 + y)),
//    f = (F - 1) / y^2, and g / x^2 = [ln(2 / x) / (1 + y) + log1p(-a) / x^2] / y
//    with a = x^2 / (2 (1 + y)), which keeps ln(x / 2) and F from cancelling.
// NSER series terms suit eps: 17 at 0.1 for FP64 (the FP32 walk uses nfw_shape32).
// ---------------------------------------------------------------------------
__host__ __device__ inline float nfw_log1p(float v) { return log1pf(v); }
__host__ __device__ inline double nfw_log1p(double v) { return log1p(v); }
__device__ inline float nfw_log(float v) { return __logf(v); } // v <= 0.75: no cancellation near 1
__host__ __device__ inline double nfw_log(double v) { return log(v); }
__host__ __device__ inline float nfw_atan(float v) { return atanf(v); }
__host__ __device__ inline double nfw_atan(double v) { return atan(v); }
// FP32 (the walk's shapes): hardware square root and reciprocal (about 1 ulp
// each), well inside the 1e-6 the FP32 shapes are held to; FP64 stays exact.
__device__ inline float nfw_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__host__ __device__ inline double nfw_sqrt(double v) { return sqrt(v); }
__device__ inline float nfw_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__host__ __device__ inline double nfw_div(double a, double b) { return a / b; }

// sum_{k < N} z^k / (2k + OFF) by Horner
template <class T, int N, int OFF>
__host__ __device__ inline T odd_series(T z)
{
    T s = (T)(1.0 / (double)(2 * (N - 1) + OFF));
#pragma unroll
    for (int k = N - 2; k >= 0; --k) s = s * z + (T)(1.0 / (double)(2 * k + OFF));
    return s;
}

// sum_{k < N} (k + 1) z^k / (2k + 5) by Horner (the series of -df/de)
template <class T, int N>
__host__ __device__ inline T dseries(T z)
{
    T s = (T)((double)N / (double)(2 * (N - 1) + 5));
#pragma unroll
    for (int k = N - 2; k >= 0; --k) s = s * z + (T)((double)(k + 1) / (double)(2 * k + 5));
    return s;
}

// With dfde: also df/de = f'(x) / (2x) = (3F - 2 - 1/x^2) / (2 e^2), or -sum (k+1)(-e)^k/(2k+5)
// in the series range (for the adjoint).
template <class T, int NSER>
__host__ __device__ inline void nfw_shape(T x2, T e, T eps, T* gx2, T* f, T* dfde = nullptr)
{
    const T ln2 = (T)0.693147180559945309417;
    if (e > -eps && e < eps) {
        const T F = odd_series<T, NSER, 1>(-e);
        *f = odd_series<T, NSER + 1, 3>(-e);
        *gx2 = nfw_div((T)0.5 * nfw_log1p(e) - ln2 + F, x2);
        if (dfde) *dfde = -dseries<T, NSER + 1>(-e);
    } else if (e > (T)0) {
        const T y = nfw_sqrt(e);
        const T F = nfw_div(nfw_atan(y), y);
        *f = nfw_div((T)1 - F, e);
        *gx2 = nfw_div((T)0.5 * nfw_log1p(e) - ln2 + F, x2);
        if (dfde) *dfde = nfw_div((T)3 * F - (T)2 - nfw_div((T)1, x2), (T)2 * e * e);
    } else {
        // x^2 is kept above a tiny floor, so that a ray at the centre gives finite values
        const T tiny = sizeof(T) == 4 ? (T)1e-30 : (T)1e-300;
        const T xx = x2 > tiny ? x2 : tiny;
        const T y = nfw_sqrt(-e), opy = (T)1 + y;
        const T F = nfw_div((T)0.5 * nfw_log1p(nfw_div((T)2 * y * opy, xx)), y);
        *f = nfw_div(F - (T)1, -e);
        const T L = ln2 - (T)0.5 * nfw_log(xx);
        *gx2 = nfw_div(nfw_div(L, opy) + nfw_div(nfw_log1p(nfw_div(-xx, (T)2 * opy)), xx), y);
        if (dfde) *dfde = nfw_div((T)3 * F - (T)2 - nfw_div((T)1, xx), (T)2 * e * e);
    }
}

// g(x) / x^2 as a power series in z = -e = 1 - x^2: sum_j T_j z^j with
// T_j = sum_{k > j} 1 / (2k (2k + 1)) = (1 - ln 2) - sum_{k <= j} 1 / (2k (2k + 1)).
// It follows from g = ln(x / 2) + F with ln x = log1p(e) / 2 and
// F = sum_k z^k / (2k + 1), divided by x^2 = 1 - z; T_0 = g(1).  No logarithm
// and no cancellation: for x < 1 every term is positive.
__host__ __device__ constexpr double nfw_gx2_coef(int j)
{
    double t = 1.0 - 0.693147180559945309417;
    for (int k = 1; k <= j; ++k) t -= 1.0 / ((2.0 * k) * (2.0 * k + 1.0));
    return t;
}

template <class T, int N>
__host__ __device__ inline T gx2_series(T z)
{
    T s = (T)nfw_gx2_coef(N - 1);
#pragma unroll
    for (int j = N - 2; j >= 0; --j) s = s * z + (T)nfw_gx2_coef(j);
    return s;
}

// The walk's FP32 shapes.  Within |e| < 0.6 (0.63 < x < 1.26) g / x^2, f and
// df/de come from their power series in e (30, 32 and 36 terms: the first term
// left out is below 1e-8 of the sum); beyond, the closed forms of nfw_shape.
// Near x = 1 the closed forms lose digits to cancellation (1 - F, F - 1 and
// 3F - 2 - 1/x^2 are small differences of O(1) terms): the series keep the
// shapes within about 5e-7 of their FP64 values where the closed forms alone
// left 2e-6 next to |e| = 0.25.
__device__ inline void nfw_shape32(float x2, float e, float* gx2, float* f, float* dfde = nullptr)
{
    if (e > -0.6f && e < 0.6f) {
        *gx2 = gx2_series<float, 30>(-e);
        *f = odd_series<float, 32, 3>(-e);
        if (dfde) *dfde = -dseries<float, 36>(-e);
    } else {
        nfw_shape<float, 1>(x2, e, 0.0f, gx2, f, dfde); // no series range left
    }
}

// g(c) on the host (FP64), for the mass normalisation of a halo of concentration c
inline double nfw_g_at(double c)
{
    double gx2, f;
    nfw_shape<double, 17>(c * c, (c - 1.0) * (c + 1.0), 0.1, &gx2, &f);
    return gx2 * (c * c);
}

// Potential shape of the NFW halo: H with H' = g(x)/x, from x^2 and e = x^2 - 1
// (FP64).  For x < 1, H = (L^2 - a^2)/2 with L = ln(x/2), a = arccosh(1/x),
// taken as (L - a)(L + a)/2 with L + a = ln((1 + y)/2) = log1p(-x^2/(2 + 2y)) and
// L - a = ln x^2 - ln(2 + 2y), y = sqrt(1 - x^2), so that the two large
// logarithms do not cancel; for x >= 1, H = (L^2 + atan(y)^2)/2, y = sqrt(x^2 - 1).
__host__ __device__ inline double nfw_H(double x2, double e)
{
    if (e < 0.0) {
        const double y = sqrt(-e), t = 2.0 + 2.0 * y;
        return 0.5 * (log(x2) - log(t)) * log1p(-x2 / t);
    }
    const double L = 0.5 * log1p(e) - 0.693147180559945309417, a = atan(sqrt(e));
    return 0.5 * (L * L + a * a);
}

// Mass-weighted potential of one smoothed particle for a lane inside its
// support (equal to the point mass's m ln r at its edge): the Gaussian's
// m psi of gauss_psi, or the halo's mC (H(x) - H(c)) + m ln R (0 at the centre).
template <int KIND>
__device__ inline float profile_psi(const PRec& pr, double r2, double psiK, int terms, float invC)
{
    if constexpr (KIND == kKindNfw) {
        if (r2 == 0.0) return 0.0f;
        const double x2 = r2 * ((double)pr.h * (double)pr.h);
        return (float)((double)pr.mC * (nfw_H(x2, x2 - 1.0) - psiK)) + pr.m * (0.5f * __logf((float)pr.qs2));
    } else {
        return pr.m * gauss_psi(pr, r2, psiK, terms, invC);
    }
}

// Profile terms of one smoothed particle for a lane inside its support (r^2
// in FP64 and FP32, ir2 = 1 / r^2): alpha = A d, kappa = K and
// gamma = -G (cos 2phi, sin 2phi) with G = A - K.
template <int KIND>
__device__ inline void profile_terms(const PRec& pr, double r2, float r2f, float ir2, float* A, float* G, float* K)
{
    if constexpr (KIND == kKindNfw) {
        const double x2 = r2 * ((double)pr.h * (double)pr.h);
        float gx2, f;
        nfw_shape32((float)x2, (float)(x2 - 1.0), &gx2, &f);
        const float mh2 = (pr.mC * pr.h) * pr.h;
        *A = mh2 * gx2;
        *K = r2 > 0.0 ? 0.5f * mh2 * f : 0.0f; // a ray at the centre gets nothing
        *G = *A - *K;
    } else {
        const float u = r2f * pr.h;
        const float e = __expf(-u);
        const float mh = pr.mC * pr.h;
        gauss_terms(u, e, ir2, pr.mC, mh, A, G);
        *K = mh * e;
    }
}

// Point-mass terms of one particle (Sec. 3.5): alpha = m d / r^2 and
// gamma = -(m / r^2) (cos 2phi, sin 2phi).  Kept free of FMA contraction so
// that the two call sites of a balanced pair produce identical values.
__device__ inline void point_terms(float m, float f1, float f2, float ir2, float* P)
{
#pragma clang fp contract(off)
    const float pm = m * ir2;
    const float c2 = (f1 * f1 - f2 * f2) * ir2, s2 = (2.0f * f1 * f2) * ir2;
    P[0] = pm * f1;
    P[1] = pm * f2;
    P[2] = -(pm * c2);
    P[3] = -(pm * s2);
}

// Accumulate alpha += coef * (f1, f2) and gamma -= Gam * (cos 2phi, sin 2phi)
// (with ir2 = 1 / r^2: cos 2phi = (f1^2 - f2^2) ir2, sin 2phi = 2 f1 f2 ir2).
template <bool AONLY, bool F64A>
__device__ inline void add_radial(float coef, float Gam, float f1, float f2, float ir2, Acc& A)
{
    add_alpha<F64A>(A, coef * f1, coef * f2);
    if (!AONLY) {
        const float c2 = (f1 * f1 - f2 * f2) * ir2, s2 = 2.0f * f1 * f2 * ir2;
        A.g1 -= (double)(Gam * c2);
        A.g2 -= (double)(Gam * s2);
    }
}

// One particle of a leaf for this lane (a direct-sum term).
//  - listed particle: a point mass (its box's moments and leaf treat it as
//    one).  A lane inside its support also gets Gaussian - point from the
//    list of the box that holds it; the two point parts meet in the FP64
//    alpha and shear sums, where they cancel exactly.
//  - unlisted particle: the truncated Gaussian of Sec. 3.1 inside the
//    support, a point mass outside.
// All cases share one select-based path (no divergent branches).  The point
// terms' shear is formed without FMA contraction, exactly as in point_terms,
// so a balanced pair cancels bit for bit there; alpha is coef * d with the
// FP64 offset d, and a balanced pair meets the list's (A - pm) d in the FP64
// sums (cancelling to FP64 rounding of the point term).
template <bool AONLY, bool F64A, bool PSI = false, int KIND = kKindGauss>
__device__ inline void leaf_particle(const PRec& pr, double X, double Y, Acc& A, double psiK = 0.0,
                                     int terms = 1, float invC = 0.0f)
{
#pragma clang fp contract(off)
    double d1, d2;
    const double r2 = sqdist(X, Y, pr.x, pr.y, &d1, &d2);
    const bool inside = r2 < pr.qs2;
    const bool listed = (pr.meta >> 31) != 0;
    const bool gauss = inside && !listed;  // the Gaussian kernel applies here
    const bool balance = inside && listed; // the box list adds Gaussian - point
    const float f1 = (float)d1, f2 = (float)d2, r2f = (float)r2;
    const float ir2 = r2f > 0.0f ? __builtin_amdgcn_rcpf(r2f) : 0.0f;
    const float pm = pr.m * ir2;
    float coef = pm, Gam = pm;
    if (__any(gauss)) {
        float Ag, Gg, Kg;
        profile_terms<KIND>(pr, r2, r2f, ir2, &Ag, &Gg, &Kg);
        coef = gauss ? Ag : pm;
        Gam = gauss ? Gg : pm;
        if (!AONLY) A.k += gauss ? Kg : 0.0f;
    }
    if constexpr (F64A) {
        // alpha = coef d with the FP64 offset; a balanced point term (coef = pm)
        // meets the list's (A - pm) d in the same FP64 sums
        const double cd = (double)coef;
        A.a1 = fma(cd, d1, A.a1);
        A.a2 = fma(cd, d2, A.a2);
    } else {
        const float v1 = coef * f1, v2 = coef * f2;
        add_alpha<false>(A, balance ? 0.0f : v1, balance ? 0.0f : v2);
        A.a1 += (double)(balance ? v1 : 0.0f);
        A.a2 += (double)(balance ? v2 : 0.0f);
    }
    if (!AONLY) {
        const float c2 = (f1 * f1 - f2 * f2) * ir2, s2 = (2.0f * f1 * f2) * ir2;
        A.g1 -= (double)(Gam * c2);
        A.g2 -= (double)(Gam * s2);
    }
    if constexpr (PSI) {
        // point mass m ln r (0 at r = 0), or the Gaussian inside its support
        const float lnr = r2f > 0.0f ? 0.5f * __logf(r2f) : 0.0f;
        A.ps += (double)(gauss ? profile_psi<KIND>(pr, r2, psiK, terms, invC) : pr.m * lnr);
    }
}

// One entry of the big-particle list of a visited box (Sec. 3.2): a lane
// inside the particle's support adds Gaussian - point (the tree part counted
// the particle as a point mass); the point part is taken off in FP64.
template <bool AONLY, bool F64A, bool PSI = false, int KIND = kKindGauss>
__device__ inline void list_particle(const PRec& pr, double X, double Y, Acc& A, int& hits, double psiK = 0.0,
                                     int terms = 1, float invC = 0.0f)
{
    double d1, d2;
    const double r2 = sqdist(X, Y, pr.x, pr.y, &d1, &d2);
    if (!(r2 < pr.qs2)) return;
    const float f1 = (float)d1, f2 = (float)d2, r2f = (float)r2;
    const float ir2 = r2f > 0.0f ? __builtin_amdgcn_rcpf(r2f) : 0.0f;
    float P[4];
    point_terms(pr.m, f1, f2, ir2, P);
    float Ag, Gg, Kg;
    profile_terms<KIND>(pr, r2, r2f, ir2, &Ag, &Gg, &Kg);
    if constexpr (F64A) {
        // (A - pm) d in FP64: the leaf sums this lane's point term as pm d
        const double diff = (double)Ag - (double)(pr.m * ir2);
        A.a1 = fma(diff, d1, A.a1);
        A.a2 = fma(diff, d2, A.a2);
        if (!AONLY) {
            const float c2 = (f1 * f1 - f2 * f2) * ir2, s2 = 2.0f * f1 * f2 * ir2;
            A.g1 -= (double)(Gg * c2);
            A.g2 -= (double)(Gg * s2);
        }
    } else {
        add_radial<AONLY, F64A>(Ag, Gg, f1, f2, ir2, A);
        A.a1 -= (double)P[0];
        A.a2 -= (double)P[1];
    }
    hits++;
    if (!AONLY) {
        A.k += Kg;
        A.g1 -= (double)P[2];
        A.g2 -= (double)P[3];
    }
    if constexpr (PSI) {
        const float lnr = r2f > 0.0f ? 0.5f * __logf(r2f) : 0.0f;
        A.ps += (double)profile_psi<KIND>(pr, r2, psiK, terms, invC) - (double)(pr.m * lnr);
    }
}

// Multipole expansion of an accepted box about its centre of mass (Sec. 3.2):
//   alpha1 - i alpha2 = v B(t),  gamma1 - i gamma2 = -v^2 (B(t) + t B'(t)),
// v = 1/w, t = r_cm v, B(t) = M P(t) = M + sum_{k>=2} (M Qn_k) t^k with
// Qn_k = Q_k / (M r_cm^k); the record holds M, r_cm and M Qn_k = Q_k / r_cm^k.
template <int P, bool AONLY, bool F64A, bool PSI = false>
__device__ inline void eval_box(const float* __restrict__ mo, double w1, double w2, Acc& A)
{
    const float M = mo[0], rcm = mo[1];
    const float f1 = (float)w1, f2 = (float)w2;
    const float inv = __builtin_amdgcn_rcpf(fmaf(f1, f1, f2 * f2));
    const float v1 = f1 * inv, v2 = -f2 * inv;
    const float t1 = rcm * v1, t2 = rcm * v2;
    // Horner in t for b = B(t) and c = B'(t): c <- c t + b, b <- b t + M Qn_k,
    // each complex multiply-add as two FMAs per component
    float b1 = M, b2 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    if constexpr (P >= 2) {
        b1 = mo[2 + 2 * (P - 2)];
        b2 = mo[3 + 2 * (P - 2)];
        c1 = b1; // first step: c = 0 * t + b
        c2 = b2;
#pragma unroll
        for (int k = P - 1; k >= 0; --k) {
            const float q1 = k >= 2 ? mo[2 + 2 * (k - 2)] : (k == 0 ? M : 0.0f);
            const float q2 = k >= 2 ? mo[3 + 2 * (k - 2)] : 0.0f;
            const float n1 = fmaf(b1, t1, fmaf(-b2, t2, q1));
            const float n2 = fmaf(b1, t2, fmaf(b2, t1, q2));
            b1 = n1;
            b2 = n2;
            if constexpr (!AONLY) {
                if (k > 0) {
                    const float m1 = fmaf(c1, t1, fmaf(-c2, t2, b1));
                    const float m2 = fmaf(c1, t2, fmaf(c2, t1, b2));
                    c1 = m1;
                    c2 = m2;
                }
            }
        }
    }
    // alpha1 - i alpha2 = v b
    const float F1 = fmaf(v1, b1, -v2 * b2), F2 = fmaf(v1, b2, v2 * b1);
    add_alpha<F64A>(A, F1, -F2);
    if constexpr (!AONLY) {
        // gamma1 - i gamma2 = -v^2 (b + t c)
        const float S1 = fmaf(t1, c1, fmaf(-t2, c2, b1)), S2 = fmaf(t1, c2, fmaf(t2, c1, b2));
        const float w21 = fmaf(v1, v1, -v2 * v2), w22 = 2.0f * v1 * v2;
        const float G1 = fmaf(w21, S1, -w22 * S2), G2 = fmaf(w21, S2, w22 * S1);
        A.g1 -= (double)G1;
        A.g2 += (double)G2;
    }
    if constexpr (PSI) {
        // psi = Re[Q_0 ln w - sum_k Q_k / (k w^k)] = M ln|w| - Re sum_{k>=2} (M Qn_k / k) t^k
        float re = 0.0f;
        if constexpr (P >= 2) {
            float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
            for (int k = P; k >= 2; --k) {
                const float q1 = mo[2 + 2 * (k - 2)] * (1.0f / (float)k);
                const float q2 = mo[3 + 2 * (k - 2)] * (1.0f / (float)k);
                const float n1 = fmaf(s1, t1, fmaf(-s2, t2, q1)), n2 = fmaf(s1, t2, fmaf(s2, t1, q2));
                s1 = n1;
                s2 = n2;
            }
            const float u1 = fmaf(t1, t1, -t2 * t2), u2 = 2.0f * t1 * t2; // t^2
            re = fmaf(s1, u1, -s2 * u2);
        }
        A.ps += (double)(fmaf(0.5f * M, __logf(fmaf(f1, f1, f2 * f2)), -re));
    }
}

// Whether some ray of the group (bounding box [gx0, gx1] x [gy0, gy1]) can
// lie inside a particle of box c's big-particle list (see the list reach).
__device__ inline bool list_reaches(const TreeDev& T, int c, double gx0, double gx1, double gy0, double gy1)
{
    // the four bounds load together and the tests combine without branches
    const int64_t i = 4 * (int64_t)c;
    const double r0 = uniform_ld(T.lreach, i), r1 = uniform_ld(T.lreach, i + 1);
    const double r2 = uniform_ld(T.lreach, i + 2), r3 = uniform_ld(T.lreach, i + 3);
    return (gx1 >= r0) & (gx0 <= r1) & (gy1 >= r2) & (gy0 <= r3);
}

// The walk of a preorder range [c0, c1) of boxes: every ancestor of a box in
// the range is either in the range or an ancestor of c0.  A lane that accepts
// an ancestor of c0 skips that ancestor's whole subtree; returns the preorder
// index at which the lane becomes active (its current skip if none).  c0 must
// be a box (c0 < ncells): an empty range at the end of the array has no
// ancestors to replay, and its walk is not made.
__device__ inline int ancestor_skip(const TreeDev& T, double X, double Y, int c0, int skip)
{
    const int nc = T.ncells;
    int a = 0;
    while (a < c0 && a < nc) {
        a = __builtin_amdgcn_readfirstlane(a);
        const CellHdr ha = T.hdr[a];
        double w1, w2;
        const double d2 = sqdist(X, Y, ha.cx, ha.cy, &w1, &w2);
        if (skip == 0 && d2 > ha.rcut2) skip = ha.next;
        int ch = a + 1; // the child of a whose subtree holds c0
        for (int guard = 0; guard < 4 && ch < nc; ++guard) {
            const int nx = T.hdr[ch].next;
            if (c0 < nx) break;
            ch = nx;
        }
        a = ch > a ? ch : a + 1;
    }
    return skip;
}

// Box range [c0, c1) of split k of K: everything before box B, K-2 equal
// slices of B's subtree [B, NB), everything after it (B = the deepest box
// holding all rays of the launch, so that the slices share the work).
__device__ inline void split_range(int k, int K, int B, int NB, int nc, int* c0, int* c1)
{
    if (K == 1) {
        *c0 = 0;
        *c1 = nc;
        return;
    }
    if (k == 0) {
        *c0 = 0;
        *c1 = B;
        return;
    }
    if (k == K - 1) {
        *c0 = NB;
        *c1 = nc;
        return;
    }
    const int64_t w = NB - B;
    *c0 = B + (int)((int64_t)(k - 1) * w / (K - 2));
    *c1 = B + (int)((int64_t)k * w / (K - 2));
}

// Work of one wavefront in a walk launch over `groups` ray groups, each walked
// by K wavefronts (one per box range).  Workgroups are dispatched round-robin
// over the 8 XCDs; inside an XCD the waves run range-major, so that the first
// range of every group is dispatched first.
constexpr int kXcds = 8;

// Groups go to the XCDs in chunks of C consecutive groups (C = groups / 512,
// 1 to 128), round robin, so that every XCD gets a share of each part of the
// image, whose cost per ray varies a lot across it (one contiguous eighth per
// XCD left the XCDs holding the dense centre running 12% longer), while
// neighbouring groups stay together on one XCD for its L2.
__host__ __device__ inline int64_t walk_chunk(int64_t groups)
{
    const int64_t c = groups / (64 * kXcds);
    return c < 1 ? 1 : (c > 128 ? 128 : c);
}
__host__ __device__ inline int64_t walk_slots(int64_t groups) // group slots per XCD
{
    const int64_t c = walk_chunk(groups);
    const int64_t chunks = (groups + c - 1) / c;
    return (chunks + kXcds - 1) / kXcds * c;
}

__host__ __device__ inline int64_t walk_grid_blocks(int64_t groups, int K)
{
    const int64_t gx = walk_slots(groups);
    return kXcds * ((K * gx + kBlock / kWave - 1) / (kBlock / kWave));
}

// b: workgroup index, w: wave in the workgroup (both wave-uniform).  Returns
// false for the waves of the padded grid that have no work.
__device__ inline bool walk_task(int b, int w, int64_t groups, int K, int* k, int64_t* group)
{
    const int64_t gx = walk_slots(groups), c = walk_chunk(groups);
    const int64_t wj = (int64_t)(b / kXcds) * (kBlock / kWave) + w;
    *k = (int)(wj / gx);
    const int64_t slot = wj % gx;
    *group = ((slot / c) * kXcds + b % kXcds) * c + slot % c;
    return *k < K && *group < groups;
}

__device__ inline double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

} // namespace glm
