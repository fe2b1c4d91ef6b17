// One round of adaptive grid refinement on the device: rank the current
// square cells by side^2 (kappa^2 + |gamma|^2) (the squared Frobenius norm of
// the deflection gradient times the cell area, from the shot outputs), split
// the top `nrefine` cells 3x3 (Sec. 4: cells are refined by adding rays around
// an already shot ray), and append the 8 new cells whose centres are the new
// rays.  Sizes are fixed by the caller, so a sequence of rounds and walks can
// be captured in a HIP graph.
#include <math.h>

#include "walk.hpp"

namespace glm {

namespace {

__global__ __launch_bounds__(kBlock) void k_refine_keys(const double* __restrict__ side, const float* __restrict__ ka,
                                                       const float* __restrict__ g1, const float* __restrict__ g2,
                                                       int64_t n, uint32_t* __restrict__ key, uint32_t* __restrict__ val)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float h = (float)side[i];
    const float k = ka[i], a = g1[i], b = g2[i];
    float sc = (h * h) * ((k * k + a * a) + b * b);
    if (!(sc >= 0.0f) || isinf(sc)) sc = isinf(sc) ? INFINITY : 0.0f;
    key[i] = 0xFFFFFFFFu - __float_as_uint(sc); // descending score, ties keep index order
    val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_refine_spawn(const uint32_t* __restrict__ order, int64_t nrefine,
                                                        int64_t ncells, double* __restrict__ cx, double* __restrict__ cy,
                                                        double* __restrict__ side, int32_t* __restrict__ refined)
{
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nrefine) return;
    const uint32_t c = order[t];
    const double h3 = side[c] / 3.0;
    const double x = cx[c], y = cy[c];
    int j = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int64_t o = ncells + 8 * t + j++;
            cx[o] = x + (double)dx * h3;
            cy[o] = y + (double)dy * h3;
            side[o] = h3;
        }
    side[c] = h3;
    if (refined) refined[t] = (int32_t)c;
}

struct RefineLayout {
    size_t k0, k1, v0, v1, hist, bytes;
};

RefineLayout refine_layout(int64_t n)
{
    RefineLayout R;
    Arena a;
    R.k0 = a.take(4ull * n);
    R.k1 = a.take(4ull * n);
    R.v0 = a.take(4ull * n);
    R.v1 = a.take(4ull * n);
    R.hist = a.take(4ull * radix_hist_words(n));
    R.bytes = a.size;
    return R;
}

} // namespace

size_t refine_workspace_bytes(int64_t ncells) { return refine_layout(ncells).bytes; }

glm_status refine_rank_device(const double* side, const float* ka, const float* g1, const float* g2,
                              int64_t ncells, void* ws, const uint32_t** order, hipStream_t st)
{
    const RefineLayout R = refine_layout(ncells);
    char* W = static_cast<char*>(ws);
    uint32_t* k0 = reinterpret_cast<uint32_t*>(W + R.k0);
    uint32_t* k1 = reinterpret_cast<uint32_t*>(W + R.k1);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(W + R.v0);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(W + R.v1);
    uint32_t* hist = reinterpret_cast<uint32_t*>(W + R.hist);
    hipLaunchKernelGGL(k_refine_keys, dim3(ceil_div(ncells, kBlock)), dim3(kBlock), 0, st, side, ka, g1, g2, ncells,
                       k0, v0);
    const int w = radix_sort_u32(k0, v0, k1, v1, ncells, 4, hist, st);
    *order = w ? v1 : v0;
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

glm_status refine_spawn_device(const uint32_t* order, int64_t nrefine, int64_t ncells, double* cx, double* cy,
                               double* side, int32_t* refined, hipStream_t st)
{
    hipLaunchKernelGGL(k_refine_spawn, dim3(ceil_div(nrefine, kBlock)), dim3(kBlock), 0, st, order, nrefine, ncells,
                       cx, cy, side, refined);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

glm_status refine_round_device(double* cx, double* cy, double* side, const float* ka, const float* g1,
                               const float* g2, int64_t ncells, int64_t nrefine, int32_t* refined, void* ws,
                               hipStream_t st)
{
    if (nrefine == 0) return GLM_OK;
    const uint32_t* order = nullptr;
    glm_status rc = refine_rank_device(side, ka, g1, g2, ncells, ws, &order, st);
    if (rc != GLM_OK) return rc;
    return refine_spawn_device(order, nrefine, ncells, cx, cy, side, refined, st);
}

} // namespace glm
