// Plain direct summation over every particle (the theta = 0 limit of the
// tree, Sec. 5.1), FP32 with compensated alpha or FP64.  One thread per ray;
// particles stream through LDS in tiles of 256 and every lane reads the same
// record (LDS broadcast).
#include <math.h>

#include "eval.hpp"
#include "walk.hpp"

namespace glm {

namespace {

__device__ inline void make_rec(PRec& r, double x, double y, double m, double s, double q, double invC, uint32_t idx)
{
#pragma clang fp contract(off)
    const double qs = q * s;
    r.x = x;
    r.y = y;
    r.qs2 = s > 0.0 ? qs * qs : 0.0;
    r.m = (float)m;
    r.mC = (float)(m * invC);
    r.h = s > 0.0 ? (float)(1.0 / (2.0 * s * s)) : 0.0f;
    r.meta = idx; // not listed: Gaussian inside the support, point outside
}

template <bool AONLY>
__global__ __launch_bounds__(kBlock) void k_direct32(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ m, const double* __restrict__ s, int n,
                                                    double q, double invC, const double* __restrict__ rx,
                                                    const double* __restrict__ ry, int64_t nr, float* __restrict__ a1,
                                                    float* __restrict__ a2, float* __restrict__ ka,
                                                    float* __restrict__ g1, float* __restrict__ g2)
{
    __shared__ PRec tile[kBlock];
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = r < nr;
    const double X = valid ? rx[r] : 0.0, Y = valid ? ry[r] : 0.0;
    Acc A = {0, 0, 0, 0, 0, 0.0, 0.0, 0.0, 0.0};
    for (int base = 0; base < n; base += kBlock) {
        const int j = base + threadIdx.x;
        PRec t;
        if (j < n) make_rec(t, x[j], y[j], m[j], s ? s[j] : 0.0, q, invC, (uint32_t)j);
        else make_rec(t, 0.0, 0.0, 0.0, 0.0, q, invC, 0u);
        tile[threadIdx.x] = t;
        __syncthreads();
        const int cnt = min(kBlock, n - base);
        for (int k = 0; k < cnt; ++k) leaf_particle<AONLY, true>(tile[k], X, Y, A);
        __syncthreads();
    }
    if (!valid) return;
    a1[r] = A.a1;
    a2[r] = A.a2;
    if (!AONLY) {
        ka[r] = A.k;
        g1[r] = (float)A.g1;
        g2[r] = (float)A.g2;
    }
    (void)A.b1;
}

// FP64: the brute-force sum term by term (Sec. 3.1 kernel, Sec. 3.5 point mass)
template <bool AONLY>
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
                const double qs = q * sj;
                qs2 = qs * qs;
            }
            const bool inside = sj > 0.0 && r2 < qs2;
            if (r2 == 0.0) {
                if (inside) sk += mj / (2.0 * sj * sj * C);
                continue;
            }
            double G = 1.0, K = 0.0;
            if (inside) {
                const double u = r2 / (2.0 * sj * sj);
                G = -expm1(-u) / C;
                K = mj * exp(-u) / (2.0 * sj * sj * C);
            }
            const double hh = mj * G / r2;
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
                         const double* rx, const double* ry, int64_t nrays, int fp64, void* const out5[5],
                         hipStream_t st)
{
    if (nrays == 0) return GLM_OK;
    const double C = -expm1(-0.5 * q * q);
    const bool aonly = !out5[2] || !out5[3] || !out5[4];
    const dim3 g(ceil_div(nrays, kBlock)), b(kBlock);
    if (fp64) {
        double* o[5];
        for (int k = 0; k < 5; ++k) o[k] = static_cast<double*>(out5[k]);
        if (aonly)
            hipLaunchKernelGGL(k_direct64<true>, g, b, 0, st, x, y, m, s, (int)n, q, C, rx, ry, nrays, o[0], o[1], o[2],
                               o[3], o[4]);
        else
            hipLaunchKernelGGL(k_direct64<false>, g, b, 0, st, x, y, m, s, (int)n, q, C, rx, ry, nrays, o[0], o[1],
                               o[2], o[3], o[4]);
    } else {
        float* o[5];
        for (int k = 0; k < 5; ++k) o[k] = static_cast<float*>(out5[k]);
        if (aonly)
            hipLaunchKernelGGL(k_direct32<true>, g, b, 0, st, x, y, m, s, (int)n, q, 1.0 / C, rx, ry, nrays, o[0], o[1],
                               o[2], o[3], o[4]);
        else
            hipLaunchKernelGGL(k_direct32<false>, g, b, 0, st, x, y, m, s, (int)n, q, 1.0 / C, rx, ry, nrays, o[0],
                               o[1], o[2], o[3], o[4]);
    }
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

} // namespace glm
