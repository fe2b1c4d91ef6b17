// Per-lane evaluation of one particle or one accepted box, shared by the
// tree walk, its adjoint and the direct sum.
#pragma once

#include <math.h>

#include "common.hpp"

namespace glm {

// Per-lane accumulators.  alpha is summed in FP32 with Kahan compensation;
// the point-mass terms of big-list particles that a ray lies inside (added
// once with each sign, see eval_particle) go to an FP64 balance where they
// cancel without leaving FP32 rounding of size m / r behind.
struct Acc {
    float a1, c1, a2, c2, k, g1, g2;
    double b1, b2, bg1, bg2;
};

__device__ inline void kadd(float& s, float& c, float v, bool kahan)
{
    const float y = v - c;
    const float t = s + y;
    c = kahan ? (t - s) - y : 0.0f;
    s = t;
}

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
// Below u = 1/2, where 1 - e^-u cancels, both use their Taylor series.
__device__ inline void gauss_terms(float u, float e, float ir2, float mC, float mh, float* A, float* G)
{
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
    const float Al = mC * (1.0f - e) * ir2;
    const bool small = u < 0.5f;
    *A = small ? mh * sg : Al;
    *G = small ? mh * sd : Al - mh * e;
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

// One particle for this lane.
//  mode 0 (leaf sum): an unlisted particle enters with the Gaussian kernel if
//    the ray is inside its support, as a point mass otherwise; a listed
//    particle enters as a point mass (its moments and leaf treat it as one).
//  mode 1 (big-particle list of a visited box): if the ray is inside the
//    support, add Gaussian - point (Sec. 3.2: listed particles are added
//    individually and removed from the tree part).
// The point part of every "inside" pair (mode 1, and mode 0 for a listed
// particle) goes to the FP64 balance so the pair cancels exactly.
template <bool AONLY>
__device__ inline void eval_particle(const PRec& pr, double X, double Y, int mode, Acc& A, bool kahan, int& hits)
{
    double d1, d2;
    const double r2 = sqdist(X, Y, pr.x, pr.y, &d1, &d2);
    const bool inside = r2 < pr.qs2;
    const bool listed = (pr.meta >> 31) != 0;
    if (mode == 1 && !inside) return;
    const float f1 = (float)d1, f2 = (float)d2, r2f = (float)r2;
    const float ir2 = r2f > 0.0f ? __builtin_amdgcn_rcpf(r2f) : 0.0f;
    float P[4];
    point_terms(pr.m, f1, f2, ir2, P);
    if (!inside || (mode == 0 && listed)) {
        if (inside) { // listed and inside: the list box already added Gaussian - point
            A.b1 += (double)P[0];
            A.b2 += (double)P[1];
            if (!AONLY) {
                A.bg1 += (double)P[2];
                A.bg2 += (double)P[3];
            }
        } else {
            kadd(A.a1, A.c1, P[0], kahan);
            kadd(A.a2, A.c2, P[1], kahan);
            if (!AONLY) {
                A.g1 += P[2];
                A.g2 += P[3];
            }
        }
        return;
    }
    // Gaussian kernel (Sec. 3.1)
    const float u = r2f * pr.h;
    const float e = __expf(-u);
    const float mh = pr.mC * pr.h;
    float Acoef, Gam;
    gauss_terms(u, e, ir2, pr.mC, mh, &Acoef, &Gam);
    kadd(A.a1, A.c1, Acoef * f1, kahan);
    kadd(A.a2, A.c2, Acoef * f2, kahan);
    if (!AONLY) {
        A.k += mh * e;
        const float c2 = (f1 * f1 - f2 * f2) * ir2, s2 = 2.0f * f1 * f2 * ir2;
        A.g1 -= Gam * c2;
        A.g2 -= Gam * s2;
    }
    if (mode == 1) {
        hits++;
        A.b1 -= (double)P[0];
        A.b2 -= (double)P[1];
        if (!AONLY) {
            A.bg1 -= (double)P[2];
            A.bg2 -= (double)P[3];
        }
    }
}

// Multipole expansion of an accepted box about its centre of mass (Sec. 3.2):
//   alpha1 - i alpha2 = M v P(t),  gamma1 - i gamma2 = -M v^2 (P(t) + t P'(t)),
// v = 1/w, t = r_cm v, P(t) = 1 + sum_{k>=2} Qn_k t^k, Qn_k = Q_k / (M r_cm^k).
template <int P, bool AONLY>
__device__ inline void eval_box(const float* __restrict__ mo, double w1, double w2, Acc& A, bool kahan)
{
    const float M = mo[0], rcm = mo[1];
    const float f1 = (float)w1, f2 = (float)w2;
    const float inv = __builtin_amdgcn_rcpf(f1 * f1 + f2 * f2);
    const float v1 = f1 * inv, v2 = -f2 * inv;
    const float t1 = rcm * v1, t2 = rcm * v2;
    float b1 = 1.0f, b2 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    if constexpr (P >= 2) {
        b1 = mo[2 + 2 * (P - 2)];
        b2 = mo[3 + 2 * (P - 2)];
#pragma unroll
        for (int k = P - 1; k >= 0; --k) {
            if constexpr (!AONLY) {
                const float n1 = c1 * t1 - c2 * t2 + b1;
                const float n2 = c1 * t2 + c2 * t1 + b2;
                c1 = n1;
                c2 = n2;
            }
            const float q1 = k >= 2 ? mo[2 + 2 * (k - 2)] : (k == 0 ? 1.0f : 0.0f);
            const float q2 = k >= 2 ? mo[3 + 2 * (k - 2)] : 0.0f;
            const float n1 = b1 * t1 - b2 * t2 + q1;
            const float n2 = b1 * t2 + b2 * t1 + q2;
            b1 = n1;
            b2 = n2;
        }
    }
    const float F1 = M * (v1 * b1 - v2 * b2), F2 = M * (v1 * b2 + v2 * b1);
    kadd(A.a1, A.c1, F1, kahan);
    kadd(A.a2, A.c2, -F2, kahan);
    if constexpr (!AONLY) {
        const float S1 = b1 + t1 * c1 - t2 * c2, S2 = b2 + t1 * c2 + t2 * c1;
        const float w21 = v1 * v1 - v2 * v2, w22 = 2.0f * v1 * v2;
        const float G1 = -M * (w21 * S1 - w22 * S2), G2 = -M * (w21 * S2 + w22 * S1);
        A.g1 += G1;
        A.g2 -= G2;
    }
}

__device__ inline int xcd_remap(int b, int nb)
{
    // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of ray groups so that its L2 sees neighbouring rays
    constexpr int nx = 8;
    const int per = nb / nx, rem = nb % nx;
    const int x = b % nx, k = b / nx;
    return x * per + (x < rem ? x : rem) + k;
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
