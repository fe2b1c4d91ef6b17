// Smoothing lengths on gfx950 (Sec. 3.1): for every particle of a built tree
// the 2D distance to its k-th nearest other particle (the particle itself
// excluded, coincident particles counted at distance 0).
//
// One wavefront serves 64 particles that are neighbours in Morton order (one
// per lane).  Each lane keeps the k smallest squared distances found so far
// in an ascending register list of fixed capacity KC >= k whose first KC - k
// slots hold -inf, so the k-th smallest always sits in the last slot.  The
// list starts from the group's own 64 particles (a tight first bound), then
// the wave walks the preorder box array: it enters a box if some lane's
// distance to the box square is below that lane's current k-th distance, and
// scans the particles of the leaves it reaches.  Every distance is FP64 and
// formed exactly as in the definition, so the result is the k-th smallest
// FP64 distance.
#include <math.h>

#include "build.hpp"

namespace glm {

namespace {

// Insert v into the ascending list h (the largest entry drops out):
// h[i] <- max(h[i-1], min(v, h[i])), no branches.
template <int KC>
__device__ inline void knn_insert(double (&h)[KC], double v)
{
#pragma unroll
    for (int i = KC - 1; i > 0; --i) h[i] = fmax(h[i - 1], fmin(v, h[i]));
    h[0] = fmin(v, h[0]);
}

__device__ inline double knn_d2(double X, double Y, double px, double py)
{
#pragma clang fp contract(off)
    const double dx = X - px, dy = Y - py;
    return dx * dx + dy * dy;
}

template <int KC>
__global__ __launch_bounds__(kBlock) void k_knn(TreeDev T, BoxArrays b, double x0, double y0, double S,
                                               double margin, int k, double* __restrict__ s_out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int n = T.n;
    const int g0 = (blockIdx.x * (kBlock / kWave) + w) * kWave; // first particle of the group
    if (g0 >= n) return;
    const int g1 = min(n, g0 + kWave);
    const int j = g0 + lane;
    const bool valid = j < n;
    const PRec me = T.prt[valid ? j : g0];
    const double X = me.x, Y = me.y;
    double h[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) h[i] = i < KC - k ? -INFINITY : INFINITY;

    // the group's own particles first
    for (int c = g0; c < g1; ++c) {
        const PRec pr = T.prt[c];
        knn_insert<KC>(h, c == j ? INFINITY : knn_d2(X, Y, pr.x, pr.y));
    }

    // then every box that some lane still needs, in preorder
    const int nc = T.ncells;
    int cur = 0;
    while (cur < nc) {
        cur = __builtin_amdgcn_readfirstlane(cur);
        const int lev = b.level[cur], nx = b.next[cur];
        const double side = ldexp(S, -lev);
        const double bx0 = x0 + (double)b.ix[cur] * side - margin;
        const double bx1 = x0 + ((double)b.ix[cur] + 1.0) * side + margin;
        const double by0 = y0 + (double)b.iy[cur] * side - margin;
        const double by1 = y0 + ((double)b.iy[cur] + 1.0) * side + margin;
        const double dx = fmax(fmax(bx0 - X, X - bx1), 0.0), dy = fmax(fmax(by0 - Y, Y - by1), 0.0);
        const bool need = valid && dx * dx + dy * dy < h[KC - 1];
        if (!__any(need)) {
            cur = nx > cur ? nx : cur + 1; // skip the subtree
            continue;
        }
        if (b.leaf[cur]) {
            const int pe = b.end[cur];
            for (int c = b.beg[cur]; c < pe; ++c) {
                if (c >= g0 && c < g1) continue; // already in the lists
                const PRec pr = T.prt[c];
                const double d2 = knn_d2(X, Y, pr.x, pr.y);
                if (__any(d2 < h[KC - 1])) knn_insert<KC>(h, d2);
            }
        }
        cur = cur + 1;
    }
    if (valid) s_out[T.perm[j]] = sqrt(h[KC - 1]);
}

} // namespace

glm_status knn_device(const TreeStorage& ts, int k, double* s_out, hipStream_t st)
{
    const int64_t groups = ((int64_t)ts.n + kWave - 1) / kWave;
    const dim3 g(ceil_div(groups, kBlock / kWave)), blk(kBlock);
    // box squares widened by far more than the rounding of the quantisation,
    // so that pruning never drops a particle of the box
    const double margin = 1e-12 * ts.side;
    if (k <= 16)
        hipLaunchKernelGGL((k_knn<16>), g, blk, 0, st, ts.dev, ts.b, ts.x0, ts.y0, ts.side, margin, k, s_out);
    else if (k <= 32)
        hipLaunchKernelGGL((k_knn<32>), g, blk, 0, st, ts.dev, ts.b, ts.x0, ts.y0, ts.side, margin, k, s_out);
    else
        hipLaunchKernelGGL((k_knn<64>), g, blk, 0, st, ts.dev, ts.b, ts.x0, ts.y0, ts.side, margin, k, s_out);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

} // namespace glm
