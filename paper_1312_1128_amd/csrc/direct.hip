// Plain direct summation over every particle (the theta = 0 limit of the
// tree, Sec. 5.1), FP32 terms summed in FP64 for alpha and shear, or FP64 throughout, for truncated
// Gaussians or truncated NFW halos (and point masses with either).  One thread per ray;
// particles stream through LDS in tiles of 256 and every lane reads the same
// record (LDS broadcast).
#include <math.h>

#include "eval.hpp"
#include "walk.hpp"

namespace glm {

namespace {

// q: Gaussian cutoff or halo concentration; norm: 1 / C or 1 / g(c)
template <int KIND>
__device__ inline void make_rec(PRec& r, double x, double y, double m, double s, double q, double norm, uint32_t idx)
{
#pragma clang fp contract(off)
    const double qs = KIND == kKindNfw ? s : q * s;
    r.x = x;
    r.y = y;
    r.qs2 = s > 0.0 ? qs * qs : 0.0;
    r.m = (float)m;
    r.mC = (float)(m * norm);
    r.h = s > 0.0 ? (float)(KIND == kKindNfw ? q / s : 1.0 / (2.0 * s * s)) : 0.0f;
    r.meta = idx; // not listed: the profile inside the support, a point outside
}

template <bool AONLY, int KIND>
__global__ __launch_bounds__(kBlock) void k_direct32(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ m, const double* __restrict__ s, int n,
                                                    double q, double norm, const double* __restrict__ rx,
                                                    const double* __restrict__ ry, int64_t nr, float* __restrict__ a1,
                                                    float* __restrict__ a2, float* __restrict__ ka,
                                                    float* __restrict__ g1, float* __restrict__ g2)
{
    __shared__ PRec tile[kBlock];
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = r < nr;
    const double X = valid ? rx[r] : 0.0, Y = valid ? ry[r] : 0.0;
    Acc A = {};
    for (int base = 0; base < n; base += kBlock) {
        const int j = base + threadIdx.x;
        PRec t;
        if (j < n) make_rec<KIND>(t, x[j], y[j], m[j], s ? s[j] : 0.0, q, norm, (uint32_t)j);
        else make_rec<KIND>(t, 0.0, 0.0, 0.0, 0.0, q, norm, 0u);
        tile[threadIdx.x] = t;
        __syncthreads();
        const int cnt = min(kBlock, n - base);
        for (int k = 0; k < cnt; ++k) leaf_particle<AONLY, true, false, KIND>(tile[k], X, Y, A);
        __syncthreads();
    }
    if (!valid) return;
    a1[r] = (float)alpha1(A);
    a2[r] = (float)alpha2(A);
    if (!AONLY) {
        ka[r] = A.k;
        g1[r] = (float)A.g1;
        g2[r] = (float)A.g2;
    }
}

// FP64: the brute-force sum term by term (Sec. 3.1 kernel or the NFW halo of
// Sec. 3.2 inside the support, Sec. 3.5 point mass outside).  C: the Gaussian
// normalisation 1 - exp(-q^2/2), or g(c) for halos.
template <bool AONLY, int KIND>
__global__ __launch_bounds__(kBlock) void k_direct64(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ m, const double* __restrict__ s, int n,
                                                    double q, double C, const double* __restrict__ rx,
                                                    const double* __restrict__ ry, int64_t nr, double* __restrict__ a1,
                                                    double* __restrict__ a2, double* __restrict__ ka,
                                                    double* __restrict__ g1, double* __restrict__ g2)
{
    __shared__ double tx[kBlock], ty[kBlock], tm[kBlock], ts[kBlock];
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = r < nr;
    const double X = valid ? rx[r] : 0.0, Y = valid ? ry[r] : 0.0;
    double sa1 = 0, sa2 = 0, sk = 0, sg1 = 0, sg2 = 0;
    for (int base = 0; base < n; base += kBlock) {
        const int j = base + threadIdx.x;
        tx[threadIdx.x] = j < n ? x[j] : 0.0;
        ty[threadIdx.x] = j < n ? y[j] : 0.0;
        tm[threadIdx.x] = j < n ? m[j] : 0.0;
        ts[threadIdx.x] = (j < n && s) ? s[j] : 0.0;
        __syncthreads();
        const int cnt = min(kBlock, n - base);
        for (int k = 0; k < cnt; ++k) {
            double d1, d2;
            const double r2 = sqdist(X, Y, tx[k], ty[k], &d1, &d2);
            const double sj = ts[k], mj = tm[k];
            double qs2;
            {
#pragma clang fp contract(off)
                const double qs = KIND == kKindNfw ? sj : q * sj;
                qs2 = qs * qs;
            }
            const bool inside = sj > 0.0 && r2 < qs2;
            if (r2 == 0.0) { // a Gaussian's centre has finite kappa; a halo's gives nothing
                if (KIND == kKindGauss && inside) sk += mj / (2.0 * sj * sj * C);
                continue;
            }
            double hh = mj / r2, K = 0.0; // alpha = hh d
            if (inside) {
                if constexpr (KIND == kKindNfw) {
                    const double hs = q / sj, x2 = r2 * (hs * hs);
                    double gx2, f;
                    nfw_shape<double, 17>(x2, x2 - 1.0, 0.1, &gx2, &f);
                    const double mh2 = mj / C * (hs * hs);
                    hh = mh2 * gx2;
                    K = 0.5 * mh2 * f;
                } else {
                    const double u = r2 / (2.0 * sj * sj);
                    hh = mj * (-expm1(-u) / C) / r2;
                    K = mj * exp(-u) / (2.0 * sj * sj * C);
                }
            }
            sa1 += hh * d1;
            sa2 += hh * d2;
            if (!AONLY) {
                const double Gam = hh - K;
                sk += K;
                sg1 -= Gam * (d1 * d1 - d2 * d2) / r2;
                sg2 -= Gam * 2.0 * d1 * d2 / r2;
            }
        }
        __syncthreads();
    }
    if (!valid) return;
    a1[r] = sa1;
    a2[r] = sa2;
    if (!AONLY) {
        ka[r] = sk;
        g1[r] = sg1;
        g2[r] = sg2;
    }
}

} // namespace

glm_status direct_device(const double* x, const double* y, const double* m, const double* s, int64_t n, double q,
                         int kind, const double* rx, const double* ry, int64_t nrays, int fp64, void* const out5[5],
                         hipStream_t st)
{
    if (nrays == 0) return GLM_OK;
    const double C = kind == kKindNfw ? nfw_g_at(q) : -expm1(-0.5 * q * q);
    const bool aonly = !out5[2] || !out5[3] || !out5[4];
    const dim3 g(ceil_div(nrays, kBlock)), b(kBlock);
    if (fp64) {
        double* o[5];
        for (int k = 0; k < 5; ++k) o[k] = static_cast<double*>(out5[k]);
#define GLM_D64(AO, KD) \
    hipLaunchKernelGGL((k_direct64<AO, KD>), g, b, 0, st, x, y, m, s, (int)n, q, C, rx, ry, nrays, o[0], o[1], o[2], o[3], o[4])
        if (kind == kKindNfw) {
            if (aonly) GLM_D64(true, kKindNfw);
            else GLM_D64(false, kKindNfw);
        } else {
            if (aonly) GLM_D64(true, kKindGauss);
            else GLM_D64(false, kKindGauss);
        }
#undef GLM_D64
    } else {
        float* o[5];
        for (int k = 0; k < 5; ++k) o[k] = static_cast<float*>(out5[k]);
#define GLM_D32(AO, KD)                                                                                                 \
    hipLaunchKernelGGL((k_direct32<AO, KD>), g, b, 0, st, x, y, m, s, (int)n, q, 1.0 / C, rx, ry, nrays, o[0], o[1], o[2], \
                       o[3], o[4])
        if (kind == kKindNfw) {
            if (aonly) GLM_D32(true, kKindNfw);
            else GLM_D32(false, kKindNfw);
        } else {
            if (aonly) GLM_D32(true, kKindGauss);
            else GLM_D32(false, kKindGauss);
        }
#undef GLM_D32
    }
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

} // namespace glm
