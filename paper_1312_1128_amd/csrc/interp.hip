// The interpolation shortcut of adaptive refinement (Sec. 3.4) on the device.
//
// Cells are squares of a nested grid: base cells of side h0 at level 0, and
// every refinement splits a cell 3 x 3 (Sec. 4), so a cell at level l is
// named by integer coordinates (i, j) with centre x0 + (i + 1/2) h0 / 3^l.
// An open-addressing hash maps (l, i, j) to the cell.  Before a refined cell
// is split, its neighbours are located (the same-level cell on each of the 8
// sides, else the coarser cell that covers that spot) and their kappa and
// gamma are compared with the cell's; if every one agrees within the
// tolerance, the magnification matrix is taken as uniform over the cell and
// the 8 new cells get their values from the linear lens equation
//   alpha(x) = alpha_c + (I - A_c)(x - x_c),  I - A_c = [[k + g1, g2], [g2, k - g1]],
// with kappa and gamma those of the centre.  The other new cells are listed
// for the tree walk.  Without kappa and gamma (deflection-only walks), the
// magnification matrix comes from deflections at three points (App. A): every
// pair of neighbours not collinear with the centre gives an estimate of A,
// the cell is uniform if each element agrees over the pairs within the
// tolerance, and its new cells use the mean estimate.
#include <math.h>

#include "walk.hpp"

namespace glm {

namespace {

constexpr uint64_t kEmpty = ~0ull;

__host__ __device__ inline uint64_t cell_key(int level, int64_t i, int64_t j)
{
    return ((uint64_t)level << 56) | ((uint64_t)(uint32_t)i << 28) | (uint64_t)(uint32_t)j;
}

__device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ inline void table_insert(uint64_t* keys, int32_t* vals, int64_t cap, uint64_t key, int32_t val)
{
    uint64_t s = mix64(key) & (uint64_t)(cap - 1);
    for (int64_t probe = 0; probe < cap; ++probe) {
        const unsigned long long prev = atomicCAS((unsigned long long*)(keys + s), (unsigned long long)kEmpty,
                                                  (unsigned long long)key);
        if (prev == kEmpty || prev == key) {
            vals[s] = val;
            return;
        }
        s = (s + 1) & (uint64_t)(cap - 1);
    }
}

__device__ inline int32_t table_find(const uint64_t* keys, const int32_t* vals, int64_t cap, uint64_t key)
{
    uint64_t s = mix64(key) & (uint64_t)(cap - 1);
    for (int64_t probe = 0; probe < cap; ++probe) {
        const uint64_t k = keys[s];
        if (k == key) return vals[s];
        if (k == kEmpty) return -1;
        s = (s + 1) & (uint64_t)(cap - 1);
    }
    return -1;
}

// The cell holding the spot of (level, i, j): that cell, else the nearest
// coarser one; -1 outside the grid.
__device__ inline int32_t locate(const uint64_t* keys, const int32_t* vals, int64_t cap, int level, int64_t i,
                                 int64_t j, int64_t nb)
{
    for (int l = level < 30 ? level : 29; l >= 0; --l) {
        int64_t span = 1;
        for (int t = 0; t < l; ++t) span *= 3;
        if (i < 0 || j < 0 || i >= nb * span || j >= nb * span) return -1;
        const int32_t c = table_find(keys, vals, cap, cell_key(l, i, j));
        if (c >= 0) return c;
        i /= 3; // coordinates are non-negative here
        j /= 3;
    }
    return -1;
}

// The located neighbours of cell c (the same-level cell on each of the 8
// sides, else the coarser cell covering that spot), in row order; returns how many.
__device__ inline int neighbours(int32_t c, const int32_t* __restrict__ lev, const int32_t* __restrict__ ci,
                                 const int32_t* __restrict__ cj, const uint64_t* keys, const int32_t* vals,
                                 int64_t cap, int64_t nb, int32_t out[8])
{
    int found = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int32_t n = locate(keys, vals, cap, lev[c], (int64_t)ci[c] + dx, (int64_t)cj[c] + dy, nb);
            if (n < 0 || n == c) continue;
            out[found++] = n;
        }
    return found;
}

// Magnification matrix A = dy/dx from deflections at three points (App. A):
// for two neighbours P, Q of cell c, with u = x_P - x_c, v = x_Q - x_c and
// s, t the matching source-plane offsets (y = x - alpha), y_1 = a11 x_1 + a21 x_2
// and y_2 = a12 x_1 + a22 x_2 solve to
//   a11 = (v2 s1 - u2 t1)/det, a21 = (u1 t1 - v1 s1)/det,
//   a12 = (v2 s2 - u2 t2)/det, a22 = (u1 t2 - v1 s2)/det,  det = u1 v2 - u2 v1.
// Every pair of neighbours not collinear with the centre (|det| above 1e-6
// |u| |v|) gives one estimate; FP64, no contraction.  Returns the number of
// pairs and the element-wise minimum, maximum and sum over them.
struct ThreePoint {
    int npairs;
    double mn[4], mx[4], sum[4]; // a11, a21, a12, a22
};

__device__ inline ThreePoint three_point(int32_t c, const int32_t* nbr, int nn, const double* __restrict__ cx,
                                         const double* __restrict__ cy, const float* __restrict__ a1,
                                         const float* __restrict__ a2)
{
#pragma clang fp contract(off)
    ThreePoint r;
    r.npairs = 0;
    for (int k = 0; k < 4; ++k) {
        r.mn[k] = INFINITY;
        r.mx[k] = -INFINITY;
        r.sum[k] = 0.0;
    }
    const double xc = cx[c], yc = cy[c], ac1 = (double)a1[c], ac2 = (double)a2[c];
    for (int p = 0; p < nn; ++p)
        for (int q = p + 1; q < nn; ++q) {
            const int32_t P = nbr[p], Q = nbr[q];
            const double u1 = cx[P] - xc, u2 = cy[P] - yc, v1 = cx[Q] - xc, v2 = cy[Q] - yc;
            const double s1 = u1 - ((double)a1[P] - ac1), s2 = u2 - ((double)a2[P] - ac2);
            const double t1 = v1 - ((double)a1[Q] - ac1), t2 = v2 - ((double)a2[Q] - ac2);
            const double det = u1 * v2 - u2 * v1;
            if (!(fabs(det) > 1e-6 * sqrt((u1 * u1 + u2 * u2) * (v1 * v1 + v2 * v2)))) continue;
            const double e[4] = {(v2 * s1 - u2 * t1) / det, (u1 * t1 - v1 * s1) / det, (v2 * s2 - u2 * t2) / det,
                                 (u1 * t2 - v1 * s2) / det};
            for (int k = 0; k < 4; ++k) {
                r.mn[k] = fmin(r.mn[k], e[k]);
                r.mx[k] = fmax(r.mx[k], e[k]);
                r.sum[k] += e[k];
            }
            ++r.npairs;
        }
    return r;
}

// Uniformity from deflections alone (App. A): each element of the three-point
// estimates of A agrees over all non-collinear pairs of neighbours within tol.
__global__ __launch_bounds__(kBlock) void k_interp_test3(const uint32_t* __restrict__ order, int64_t nrefine,
                                                        const int32_t* __restrict__ lev, const int32_t* __restrict__ ci,
                                                        const int32_t* __restrict__ cj, const uint64_t* keys,
                                                        const int32_t* vals, int64_t cap, int64_t nb,
                                                        const double* __restrict__ cx, const double* __restrict__ cy,
                                                        const float* __restrict__ a1, const float* __restrict__ a2,
                                                        float tol, int32_t* __restrict__ shots,
                                                        double* __restrict__ amean)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nrefine) return;
    const int32_t c = (int32_t)order[t];
    int32_t nbr[8];
    const int nn = neighbours(c, lev, ci, cj, keys, vals, cap, nb, nbr);
    const ThreePoint r = three_point(c, nbr, nn, cx, cy, a1, a2);
    bool uniform = r.npairs > 0;
    for (int k = 0; k < 4; ++k) {
        uniform = uniform && r.mx[k] - r.mn[k] <= (double)tol;
        amean[4 * t + k] = r.npairs > 0 ? r.sum[k] / (double)r.npairs : 0.0;
    }
    shots[t] = uniform ? 0 : 8;
}

// kappa and gamma of the listed cells from their three-point magnification
// matrix (the mean over neighbour pairs; 0 without a non-collinear pair):
// kappa = 1 - (a11 + a22)/2, gamma1 = (a22 - a11)/2, gamma2 = -(a12 + a21)/2.
__global__ __launch_bounds__(kBlock) void k_interp_estimate(const int32_t* __restrict__ idx,
                                                           const int32_t* __restrict__ count, int64_t max_count,
                                                           const int32_t* __restrict__ lev,
                                                           const int32_t* __restrict__ ci,
                                                           const int32_t* __restrict__ cj, const uint64_t* keys,
                                                           const int32_t* vals, int64_t cap, int64_t nb,
                                                           const double* __restrict__ cx, const double* __restrict__ cy,
                                                           const float* __restrict__ a1, const float* __restrict__ a2,
                                                           float* __restrict__ ka, float* __restrict__ g1,
                                                           float* __restrict__ g2)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t n = count ? (int64_t)*count : max_count;
    if (t >= n || t >= max_count) return;
    const int32_t c = idx ? idx[t] : (int32_t)t;
    int32_t nbr[8];
    const int nn = neighbours(c, lev, ci, cj, keys, vals, cap, nb, nbr);
    const ThreePoint r = three_point(c, nbr, nn, cx, cy, a1, a2);
    double A[4] = {0.0, 0.0, 0.0, 0.0};
    if (r.npairs > 0)
        for (int k = 0; k < 4; ++k) A[k] = r.sum[k] / (double)r.npairs;
    ka[c] = r.npairs > 0 ? (float)(1.0 - 0.5 * (A[0] + A[3])) : 0.0f;
    g1[c] = r.npairs > 0 ? (float)(0.5 * (A[3] - A[0])) : 0.0f;
    g2[c] = r.npairs > 0 ? (float)(-0.5 * (A[2] + A[1])) : 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(uint64_t* p, int64_t n, uint64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// Base cells: level 0, coordinates from the centres.
__global__ __launch_bounds__(kBlock) void k_interp_base(const double* __restrict__ cx, const double* __restrict__ cy,
                                                       int64_t n, double x0, double y0, double h0,
                                                       int32_t* __restrict__ lev, int32_t* __restrict__ ci,
                                                       int32_t* __restrict__ cj, uint64_t* keys, int32_t* vals,
                                                       int64_t cap)
{
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const int32_t i = (int32_t)floor((cx[c] - x0) / h0), j = (int32_t)floor((cy[c] - y0) / h0);
    lev[c] = 0;
    ci[c] = i;
    cj[c] = j;
    table_insert(keys, vals, cap, cell_key(0, i, j), (int32_t)c);
}

// Uniformity of each cell about to be refined (the state before the split).
__global__ __launch_bounds__(kBlock) void k_interp_test(const uint32_t* __restrict__ order, int64_t nrefine,
                                                       const int32_t* __restrict__ lev, const int32_t* __restrict__ ci,
                                                       const int32_t* __restrict__ cj, const uint64_t* keys,
                                                       const int32_t* vals, int64_t cap, int64_t nb,
                                                       const float* __restrict__ ka, const float* __restrict__ g1,
                                                       const float* __restrict__ g2, float tol,
                                                       int32_t* __restrict__ shots)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nrefine) return;
    const int32_t c = (int32_t)order[t];
    const float k0 = ka[c], a0 = g1[c], b0 = g2[c];
    bool uniform = true;
    int found = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int32_t nb_cell = locate(keys, vals, cap, lev[c], (int64_t)ci[c] + dx, (int64_t)cj[c] + dy, nb);
            if (nb_cell < 0 || nb_cell == c) continue;
            ++found;
            uniform = uniform && fabsf(ka[nb_cell] - k0) <= tol && fabsf(g1[nb_cell] - a0) <= tol &&
                      fabsf(g2[nb_cell] - b0) <= tol;
        }
    shots[t] = (uniform && found > 0) ? 0 : 8;
}

// New cells' level and coordinates, the refined cell's new ones, their hash
// entries; values of the new cells of uniform cells; the list of new cells
// to shoot (offsets from the exclusive scan of shots).
__global__ __launch_bounds__(kBlock) void k_interp_spawn(const uint32_t* __restrict__ order, int64_t nrefine,
                                                        int64_t ncells, const double* __restrict__ cx,
                                                        const double* __restrict__ cy, int32_t* __restrict__ lev,
                                                        int32_t* __restrict__ ci, int32_t* __restrict__ cj,
                                                        uint64_t* keys, int32_t* vals, int64_t cap,
                                                        const int32_t* __restrict__ shots,
                                                        const int32_t* __restrict__ offs, float* __restrict__ a1,
                                                        float* __restrict__ a2, float* __restrict__ ka,
                                                        float* __restrict__ g1, float* __restrict__ g2,
                                                        int32_t* __restrict__ shoot_idx,
                                                        const double* __restrict__ amean)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nrefine) return;
    const int32_t c = (int32_t)order[t];
    const int32_t l = lev[c] + 1;
    const int64_t i = 3 * (int64_t)ci[c] + 1, j = 3 * (int64_t)cj[c] + 1;
    const bool fill = shots[t] == 0;
    // beyond the key range a cell is not indexed (its neighbours then fall
    // back to coarser cells)
    const bool keyed = l < 30 && i + 1 < (1ll << 28) && j + 1 < (1ll << 28);
    const double xc = cx[c], yc = cy[c];
    const double A1 = a1[c], A2 = a2[c];
    // I - A: from the cell's kappa and gamma, or (deflection mode) the mean three-point A
    double K = ka[c], G1 = g1[c], G2 = g2[c];
    double m11 = K + G1, m12 = G2, m21 = G2, m22 = K - G1; // alpha_new = alpha_c + [[m11, m12], [m21, m22]] u
    if (amean && fill) {
        const double* am = amean + 4 * t; // a11, a21, a12, a22
        m11 = 1.0 - am[0];
        m12 = -am[1];
        m21 = -am[2];
        m22 = 1.0 - am[3];
        K = 1.0 - 0.5 * (am[0] + am[3]);
        G1 = 0.5 * (am[3] - am[0]);
        G2 = -0.5 * (am[2] + am[1]);
    }
    int q = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int64_t o = ncells + 8 * t + q;
            lev[o] = l;
            ci[o] = (int32_t)(i + dx);
            cj[o] = (int32_t)(j + dy);
            if (keyed) table_insert(keys, vals, cap, cell_key(l, i + dx, j + dy), (int32_t)o);
            if (fill) {
                const double ux = cx[o] - xc, uy = cy[o] - yc;
                a1[o] = (float)(A1 + m11 * ux + m12 * uy);
                a2[o] = (float)(A2 + m21 * ux + m22 * uy);
                ka[o] = (float)K;
                g1[o] = (float)G1;
                g2[o] = (float)G2;
            } else {
                shoot_idx[offs[t] + q] = (int32_t)o;
            }
            ++q;
        }
    lev[c] = l;
    ci[c] = (int32_t)i;
    cj[c] = (int32_t)j;
    if (keyed) table_insert(keys, vals, cap, cell_key(l, i, j), c);
}

__global__ void k_copy_count(const int32_t* __restrict__ offs, int64_t n, int32_t* __restrict__ count)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *count = offs[n];
}

__global__ __launch_bounds__(kBlock) void k_gather_xy(const double* __restrict__ cx, const double* __restrict__ cy,
                                                     const int32_t* __restrict__ idx, int64_t n,
                                                     double* __restrict__ gx, double* __restrict__ gy)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    gx[t] = cx[idx[t]];
    gy[t] = cy[idx[t]];
}

__global__ __launch_bounds__(kBlock) void k_scatter_out(const float* __restrict__ src, const int32_t* __restrict__ idx,
                                                       int64_t n, int nq, float* o0, float* o1, float* o2, float* o3,
                                                       float* o4)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const int64_t d = idx[t];
    float* dst[5] = {o0, o1, o2, o3, o4};
    for (int q = 0; q < nq; ++q)
        if (dst[q]) dst[q][d] = src[(int64_t)q * n + t];
}

} // namespace

// Layout of the interpolation state (cell level and coordinates, hash table).
InterpLayout interp_layout(int64_t capacity)
{
    InterpLayout L;
    Arena a;
    int64_t cap = 1;
    while (cap < 4 * capacity) cap <<= 1;
    L.table_cap = cap;
    L.lev = a.take(4ull * capacity);
    L.ci = a.take(4ull * capacity);
    L.cj = a.take(4ull * capacity);
    L.keys = a.take(8ull * cap);
    L.vals = a.take(4ull * cap);
    L.bytes = a.size;
    return L;
}

// Round scratch on top of the ranking scratch of refine_round.
size_t interp_round_workspace_bytes(int64_t ncells, int64_t nrefine)
{
    Arena a;
    a.take(refine_workspace_bytes(ncells));
    a.take(4ull * (nrefine + 1));               // shots
    a.take(4ull * (nrefine + 1));               // offsets
    a.take(4ull * scan_scratch_words(nrefine)); // scan scratch
    a.take(32ull * (nrefine + 1));              // mean three-point A per refined cell
    return a.size;
}

glm_status interp_init_device(const double* cx, const double* cy, int64_t ncells, double x0, double y0, double h0,
                              int64_t capacity, void* state, hipStream_t st)
{
    const InterpLayout L = interp_layout(capacity);
    char* S = static_cast<char*>(state);
    uint64_t* keys = reinterpret_cast<uint64_t*>(S + L.keys);
    hipLaunchKernelGGL(k_fill_u64, dim3(ceil_div(L.table_cap, kBlock)), dim3(kBlock), 0, st, keys, L.table_cap, kEmpty);
    if (ncells > 0)
        hipLaunchKernelGGL(k_interp_base, dim3(ceil_div(ncells, kBlock)), dim3(kBlock), 0, st, cx, cy, ncells, x0, y0,
                           h0, reinterpret_cast<int32_t*>(S + L.lev), reinterpret_cast<int32_t*>(S + L.ci),
                           reinterpret_cast<int32_t*>(S + L.cj), keys, reinterpret_cast<int32_t*>(S + L.vals),
                           L.table_cap);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

glm_status interp_round_device(double* cx, double* cy, double* side, float* a1, float* a2, float* ka, float* g1,
                               float* g2, int64_t ncells, int64_t nrefine, int64_t nbase, float tol, bool deflections,
                               int32_t* refined, int32_t* shoot_idx, int32_t* shoot_count, int64_t capacity,
                               void* state, void* ws, hipStream_t st)
{
    const InterpLayout L = interp_layout(capacity);
    char* S = static_cast<char*>(state);
    int32_t* lev = reinterpret_cast<int32_t*>(S + L.lev);
    int32_t* ci = reinterpret_cast<int32_t*>(S + L.ci);
    int32_t* cj = reinterpret_cast<int32_t*>(S + L.cj);
    uint64_t* keys = reinterpret_cast<uint64_t*>(S + L.keys);
    int32_t* vals = reinterpret_cast<int32_t*>(S + L.vals);
    Arena a;
    const size_t o_rank = a.take(refine_workspace_bytes(ncells));
    const size_t o_shots = a.take(4ull * (nrefine + 1));
    const size_t o_offs = a.take(4ull * (nrefine + 1));
    const size_t o_scan = a.take(4ull * scan_scratch_words(nrefine));
    const size_t o_amean = a.take(32ull * (nrefine + 1));
    char* W = static_cast<char*>(ws);
    double* amean = reinterpret_cast<double*>(W + o_amean);
    int32_t* shots = reinterpret_cast<int32_t*>(W + o_shots);
    int32_t* offs = reinterpret_cast<int32_t*>(W + o_offs);
    const uint32_t* order = nullptr;
    glm_status rc = refine_rank_device(side, ka, g1, g2, ncells, W + o_rank, &order, st);
    if (rc != GLM_OK) return rc;
    const dim3 g(ceil_div(nrefine, kBlock)), b(kBlock);
    if (deflections)
        hipLaunchKernelGGL(k_interp_test3, g, b, 0, st, order, nrefine, lev, ci, cj, keys, vals, L.table_cap, nbase,
                           cx, cy, a1, a2, tol, shots, amean);
    else
        hipLaunchKernelGGL(k_interp_test, g, b, 0, st, order, nrefine, lev, ci, cj, keys, vals, L.table_cap, nbase, ka,
                           g1, g2, tol, shots);
    exclusive_scan_i32(shots, offs, nrefine, reinterpret_cast<int32_t*>(W + o_scan), st);
    // positions and sides of the new cells (the plain refinement split)
    rc = refine_spawn_device(order, nrefine, ncells, cx, cy, side, refined, st);
    if (rc != GLM_OK) return rc;
    hipLaunchKernelGGL(k_interp_spawn, g, b, 0, st, order, nrefine, ncells, cx, cy, lev, ci, cj, keys, vals,
                       L.table_cap, shots, offs, a1, a2, ka, g1, g2, shoot_idx, deflections ? amean : nullptr);
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, st, offs, nrefine, shoot_count);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

glm_status interp_estimate_device(const double* cx, const double* cy, const float* a1, const float* a2, float* ka,
                                  float* g1, float* g2, const int32_t* idx, const int32_t* count, int64_t max_count,
                                  int64_t nbase, int64_t capacity, const void* state, hipStream_t st)
{
    if (max_count == 0) return GLM_OK;
    const InterpLayout L = interp_layout(capacity);
    const char* S = static_cast<const char*>(state);
    hipLaunchKernelGGL(k_interp_estimate, dim3(ceil_div(max_count, kBlock)), dim3(kBlock), 0, st, idx, count,
                       max_count, reinterpret_cast<const int32_t*>(S + L.lev), reinterpret_cast<const int32_t*>(S + L.ci),
                       reinterpret_cast<const int32_t*>(S + L.cj), reinterpret_cast<const uint64_t*>(S + L.keys),
                       reinterpret_cast<const int32_t*>(S + L.vals), L.table_cap, nbase, cx, cy, a1, a2, ka, g1, g2);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

size_t shoot_indexed_workspace_bytes(int64_t count)
{
    Arena a;
    a.take(16ull * count); // gathered x, y
    a.take(20ull * count); // staged outputs
    a.take(ray_layout(count).bytes);
    return a.size;
}

glm_status shoot_indexed_device(const TreeStorage& ts, const double* cx, const double* cy, const int32_t* idx,
                                int64_t count, float* a1, float* a2, float* ka, float* g1, float* g2, uint32_t flags,
                                void* ws, hipStream_t st)
{
    if (count == 0) return GLM_OK;
    Arena a;
    const size_t o_xy = a.take(16ull * count);
    const size_t o_out = a.take(20ull * count);
    const size_t o_ws = a.take(ray_layout(count).bytes);
    char* W = static_cast<char*>(ws);
    double* gx = reinterpret_cast<double*>(W + o_xy);
    double* gy = gx + count;
    float* so = reinterpret_cast<float*>(W + o_out);
    const dim3 g(ceil_div(count, kBlock)), b(kBlock);
    hipLaunchKernelGGL(k_gather_xy, g, b, 0, st, cx, cy, idx, count, gx, gy);
    const bool aonly = (flags & GLM_ALPHA_ONLY) != 0;
    glm_status rc = shoot_device(ts, gx, gy, count, so, so + count, aonly ? nullptr : so + 2 * count,
                                 aonly ? nullptr : so + 3 * count, aonly ? nullptr : so + 4 * count, nullptr,
                                 flags & ~GLM_RAYS_ORDERED, W + o_ws, st);
    if (rc != GLM_OK) return rc;
    hipLaunchKernelGGL(k_scatter_out, g, b, 0, st, so, idx, count, aonly ? 2 : 5, a1, a2, aonly ? nullptr : ka,
                       aonly ? nullptr : g1, aonly ? nullptr : g2);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

} // namespace glm
