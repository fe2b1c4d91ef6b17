// Smoothing lengths from raw positions on gfx950 (Sec. 3.1): for every
// particle the distance to its k-th nearest other particle, counted in
// projection (2D) or in space (3D, which the paper prefers), and with several
// species only among particles of the particle's own species.
//
// Particles are sorted by Morton key (3 x 21 bits, or 2 x 31 bits), then
// stably by species, so that every species is one contiguous, spatially
// ordered segment.  Over each segment an implicit bounding-box hierarchy is
// built bottom-up: buckets of kBucket consecutive particles with their exact
// FP64 bounding boxes (widened by a margin far above rounding), then parents
// of kFan consecutive children, up to one root.  No topology pass is needed:
// node (level, j) covers particles [j B F^level, (j + 1) B F^level).
//
// One wavefront serves 64 consecutive particles of a segment (one per lane):
// each lane keeps the k smallest squared distances in an ascending register
// list of capacity KC >= k padded with -inf, seeded with the group's own
// particles; the wave then walks the hierarchy depth first (stackless, the
// next node follows from (level, j) arithmetically), entering a node if some
// lane's distance to its box is below that lane's current k-th distance.
// Squared distances are FP64, (dx^2 + dy^2) + dz^2 without contraction, so
// the result is the k-th smallest FP64 squared distance of the definition.
#include <math.h>

#include <string>
#include <vector>

#include "build.hpp"

namespace glm {

namespace {

constexpr int kBucket = 32;   // particles per leaf bucket
constexpr int kFan = 8;       // children per node
constexpr int kMaxLevels = 16;
constexpr int kMaxSpecies = 1 << 16;

struct KnnSync {
    double lo[3], hi[3]; // bounding box
    double x0[3];        // cube origin
    double scale;        // quantisation scale
    int32_t bad;         // non-finite position
    int32_t bad_species; // species id outside [0, 2^16)
    int32_t nseg;        // number of species segments
    int32_t pad;
};

// Bounding boxes of the hierarchy, SoA per bound, levels packed one after the other.
struct Bvh {
    double* lo[3];
    double* hi[3];
    int32_t off[kMaxLevels];
    int32_t cnt[kMaxLevels];
    int32_t top;
};

__device__ inline uint64_t spread3(uint32_t v) // 21 bits -> every third bit
{
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline uint64_t spread2(uint32_t v) // 32 bits -> every second bit
{
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__global__ __launch_bounds__(kBlock) void k_knn_bbox(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, int64_t n,
                                                    double* __restrict__ part)
{
    __shared__ double red[7][kBlock];
    double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double p[3] = {x[i], y[i], z ? z[i] : 0.0};
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(p[a])) v[6] = 1.0;
            v[a] = fmin(v[a], p[a]);
            v[3 + a] = fmax(v[3 + a], p[a]);
        }
    }
    for (int a = 0; a < 7; ++a) red[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = fmin(red[a][threadIdx.x], red[a][threadIdx.x + o]);
            for (int a = 3; a < 7; ++a) red[a][threadIdx.x] = fmax(red[a][threadIdx.x], red[a][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) part[blockIdx.x * 7 + threadIdx.x] = red[threadIdx.x][0];
}

// Cube over the bounding box; quantisation to `bits` bits per axis.
__global__ __launch_bounds__(kBlock) void k_knn_root(const double* __restrict__ part, int nb, int bits,
                                                    KnnSync* __restrict__ sync)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0) return;
    double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
    for (int b = 0; b < nb; ++b) {
        for (int a = 0; a < 3; ++a) v[a] = fmin(v[a], part[b * 7 + a]);
        for (int a = 3; a < 7; ++a) v[a] = fmax(v[a], part[b * 7 + a]);
    }
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = fmax(ext, v[3 + a] - v[a]);
    double S = ext * (1.0 + 0x1p-40);
    if (!(S > 0.0)) S = 1.0;
    for (int a = 0; a < 3; ++a) {
        sync->lo[a] = v[a];
        sync->hi[a] = v[3 + a];
        sync->x0[a] = 0.5 * (v[a] + v[3 + a]) - 0.5 * S;
    }
    sync->scale = ldexp(1.0, bits) / S;
    sync->bad = v[6] != 0.0;
    sync->bad_species = 0;
    sync->nseg = 1;
}

__device__ inline uint32_t knn_quant(double v, double v0, double scale, uint32_t qmax)
{
#pragma clang fp contract(off)
    const double t = (v - v0) * scale;
    if (!(t >= 0.0)) return 0u;
    if (t >= (double)qmax) return qmax;
    return (uint32_t)floor(t);
}

__global__ __launch_bounds__(kBlock) void k_knn_keys(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, int64_t n,
                                                    const KnnSync* __restrict__ sync, uint64_t* __restrict__ key,
                                                    uint32_t* __restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (z) {
        const uint32_t qm = (1u << 21) - 1u;
        key[i] = spread3(knn_quant(x[i], sync->x0[0], sync->scale, qm)) |
                 (spread3(knn_quant(y[i], sync->x0[1], sync->scale, qm)) << 1) |
                 (spread3(knn_quant(z[i], sync->x0[2], sync->scale, qm)) << 2);
    } else {
        const uint32_t qm = 0x7FFFFFFFu;
        key[i] = spread2(knn_quant(x[i], sync->x0[0], sync->scale, qm)) |
                 (spread2(knn_quant(y[i], sync->x0[1], sync->scale, qm)) << 1);
    }
    val[i] = (uint32_t)i;
}

// species of the Morton-sorted particles, as keys for the stable species sort
__global__ __launch_bounds__(kBlock) void k_knn_species_keys(const int32_t* __restrict__ species,
                                                            const uint32_t* __restrict__ perm, int64_t n,
                                                            uint32_t* __restrict__ skey, uint32_t* __restrict__ sval,
                                                            KnnSync* __restrict__ sync)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint32_t i = perm[j];
    const int32_t s = species[i];
    if (s < 0 || s >= kMaxSpecies) atomicOr(&sync->bad_species, 1);
    skey[j] = (uint32_t)(s < 0 ? 0 : (s >= kMaxSpecies ? kMaxSpecies - 1 : s));
    sval[j] = i;
}

// 1 where a new species starts in the sorted order
__global__ __launch_bounds__(kBlock) void k_knn_seg_flags(const uint32_t* __restrict__ skey, int64_t n,
                                                         int32_t* __restrict__ flag)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    flag[j] = (j == 0 || skey[j] != skey[j - 1]) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_knn_seg_starts(const uint32_t* __restrict__ skey, int64_t n,
                                                          const int32_t* __restrict__ pos,
                                                          int32_t* __restrict__ starts, KnnSync* __restrict__ sync)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    if (j == 0 || skey[j] != skey[j - 1]) starts[pos[j]] = (int32_t)j;
    if (j == n - 1) sync->nseg = pos[n]; // the scan's total: number of species
}

__global__ __launch_bounds__(kBlock) void k_knn_gather(const uint32_t* __restrict__ perm, const double* __restrict__ x,
                                                      const double* __restrict__ y, const double* __restrict__ z,
                                                      int64_t n, double* __restrict__ xs, double* __restrict__ ys,
                                                      double* __restrict__ zs)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint32_t i = perm[j];
    xs[j] = x[i];
    ys[j] = y[i];
    if (z) zs[j] = z[i];
}

// bounding boxes of the buckets of one segment (particles [0, ns) of xs/ys/zs)
template <bool D3>
__global__ __launch_bounds__(kBlock) void k_bvh_leaves(const double* __restrict__ xs, const double* __restrict__ ys,
                                                      const double* __restrict__ zs, int ns, double margin, Bvh B)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= B.cnt[0]) return;
    const int c0 = j * kBucket, c1 = min(ns, c0 + kBucket);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int c = c0; c < c1; ++c) {
        lo[0] = fmin(lo[0], xs[c]);
        hi[0] = fmax(hi[0], xs[c]);
        lo[1] = fmin(lo[1], ys[c]);
        hi[1] = fmax(hi[1], ys[c]);
        if (D3) {
            lo[2] = fmin(lo[2], zs[c]);
            hi[2] = fmax(hi[2], zs[c]);
        }
    }
    for (int a = 0; a < (D3 ? 3 : 2); ++a) {
        B.lo[a][j] = lo[a] - margin;
        B.hi[a][j] = hi[a] + margin;
    }
}

// parents at level l from their children at level l - 1
template <bool D3>
__global__ __launch_bounds__(kBlock) void k_bvh_level(Bvh B, int l)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= B.cnt[l]) return;
    const int c0 = B.off[l - 1] + j * kFan, c1 = B.off[l - 1] + min(B.cnt[l - 1], (j + 1) * kFan);
    const int o = B.off[l] + j;
    for (int a = 0; a < (D3 ? 3 : 2); ++a) {
        double lo = INFINITY, hi = -INFINITY;
        for (int c = c0; c < c1; ++c) {
            lo = fmin(lo, B.lo[a][c]);
            hi = fmax(hi, B.hi[a][c]);
        }
        B.lo[a][o] = lo;
        B.hi[a][o] = hi;
    }
}

// Insert v into the ascending list h (the largest entry drops out).
template <int KC>
__device__ inline void knn3_insert(double (&h)[KC], double v)
{
#pragma unroll
    for (int i = KC - 1; i > 0; --i) h[i] = fmax(h[i - 1], fmin(v, h[i]));
    h[0] = fmin(v, h[0]);
}

template <bool D3>
__device__ inline double knn3_d2(double X, double Y, double Z, double px, double py, double pz)
{
#pragma clang fp contract(off)
    const double dx = X - px, dy = Y - py;
    double r2 = dx * dx + dy * dy;
    if (D3) {
        const double dz = Z - pz;
        r2 = r2 + dz * dz;
    }
    return r2;
}

// One segment: particles [0, ns) of the sorted arrays (already offset to the
// segment); perm maps them to their original index.
template <int KC, bool D3>
__global__ __launch_bounds__(kBlock) void k_knn_bvh(const double* __restrict__ xs, const double* __restrict__ ys,
                                                   const double* __restrict__ zs, int ns, Bvh B, int k,
                                                   const uint32_t* __restrict__ perm, double* __restrict__ s_out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int g0 = (blockIdx.x * (kBlock / kWave) + w) * kWave;
    if (g0 >= ns) return;
    const int g1 = min(ns, g0 + kWave);
    const int j = g0 + lane;
    const bool valid = j < ns;
    const int jj = valid ? j : g0;
    const double X = xs[jj], Y = ys[jj], Z = D3 ? zs[jj] : 0.0;
    double h[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) h[i] = i < KC - k ? -INFINITY : INFINITY;

    for (int c = g0; c < g1; ++c) {
        const double d2 = knn3_d2<D3>(X, Y, Z, xs[c], ys[c], D3 ? zs[c] : 0.0);
        knn3_insert<KC>(h, c == j ? INFINITY : d2);
    }

    const int top = B.top;
    int l = top, nj = 0;
    for (;;) {
        l = __builtin_amdgcn_readfirstlane(l);
        nj = __builtin_amdgcn_readfirstlane(nj);
        const int o = B.off[l] + nj;
        double dx = fmax(fmax(B.lo[0][o] - X, X - B.hi[0][o]), 0.0);
        double dy = fmax(fmax(B.lo[1][o] - Y, Y - B.hi[1][o]), 0.0);
        double bd = dx * dx + dy * dy;
        if (D3) {
            const double dz = fmax(fmax(B.lo[2][o] - Z, Z - B.hi[2][o]), 0.0);
            bd += dz * dz;
        }
        const bool need = valid && bd < h[KC - 1];
        if (__any(need)) {
            if (l > 0) { // first child
                --l;
                nj *= kFan;
                continue;
            }
            const int c0 = nj * kBucket, c1 = min(ns, c0 + kBucket);
            for (int c = c0; c < c1; ++c) {
                if (c >= g0 && c < g1) continue; // already in the lists
                const double d2 = knn3_d2<D3>(X, Y, Z, xs[c], ys[c], D3 ? zs[c] : 0.0);
                if (__any(d2 < h[KC - 1])) knn3_insert<KC>(h, d2);
            }
        }
        // next node in depth-first order: the next sibling, else up
        bool done = false;
        for (;;) {
            if (l == top) {
                done = true;
                break;
            }
            if ((nj % kFan) != kFan - 1 && nj + 1 < B.cnt[l]) {
                ++nj;
                break;
            }
            nj /= kFan;
            ++l;
        }
        if (done) break;
    }
    if (valid) s_out[perm[j]] = sqrt(h[KC - 1]);
}

struct KnnLayout {
    size_t sync, part, k0, k1, v0, v1, hist, sk0, sk1, flag, pos, scan, starts, xs, ys, zs, nodes, bytes;
    int64_t node_cap;
};

constexpr int kBboxBlocks = 256;

// nodes of the hierarchy over ns particles, per level
inline int bvh_levels(int64_t ns, int32_t* cnt)
{
    int64_t c = (ns + kBucket - 1) / kBucket;
    int L = 0;
    cnt[L++] = (int32_t)c;
    while (c > 1 && L < kMaxLevels) {
        c = (c + kFan - 1) / kFan;
        cnt[L++] = (int32_t)c;
    }
    return L;
}

KnnLayout knn_layout(int64_t n, bool species)
{
    KnnLayout L{};
    Arena a;
    L.sync = a.take(sizeof(KnnSync));
    L.part = a.take(sizeof(double) * 7 * kBboxBlocks);
    L.k0 = a.take(8ull * n);
    L.k1 = a.take(8ull * n);
    L.v0 = a.take(4ull * n);
    L.v1 = a.take(4ull * n);
    L.hist = a.take(4ull * radix_hist_words(n));
    if (species) {
        L.sk0 = a.take(4ull * n);
        L.sk1 = a.take(4ull * n);
        L.flag = a.take(4ull * (n + 1));
        L.pos = a.take(4ull * (n + 1));
        L.scan = a.take(4ull * scan_scratch_words(n + 1));
        L.starts = a.take(4ull * (n + 1));
    }
    L.xs = a.take(8ull * n);
    L.ys = a.take(8ull * n);
    L.zs = a.take(8ull * n);
    int32_t cnt[kMaxLevels];
    const int nl = bvh_levels(n, cnt);
    int64_t nodes = 0;
    for (int l = 0; l < nl; ++l) nodes += cnt[l];
    L.node_cap = nodes;
    L.nodes = a.take(8ull * 6 * nodes);
    L.bytes = a.size;
    return L;
}

} // namespace

size_t knn_workspace_bytes(int64_t n, bool species) { return knn_layout(n, species).bytes; }

glm_status knn_positions_device(const double* x, const double* y, const double* z, const int32_t* species,
                                int64_t n, int k, double* s_out, void* ws, hipStream_t st)
{
    const KnnLayout L = knn_layout(n, species != nullptr);
    char* W = static_cast<char*>(ws);
    KnnSync* sync = reinterpret_cast<KnnSync*>(W + L.sync);
    double* part = reinterpret_cast<double*>(W + L.part);
    uint64_t* k0 = reinterpret_cast<uint64_t*>(W + L.k0);
    uint64_t* k1 = reinterpret_cast<uint64_t*>(W + L.k1);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(W + L.v0);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(W + L.v1);
    uint32_t* hist = reinterpret_cast<uint32_t*>(W + L.hist);
    double* xs = reinterpret_cast<double*>(W + L.xs);
    double* ys = reinterpret_cast<double*>(W + L.ys);
    double* zs = reinterpret_cast<double*>(W + L.zs);
    double* nodes = reinterpret_cast<double*>(W + L.nodes);
    const bool d3 = z != nullptr;
    const int g = ceil_div(n, kBlock);

    hipLaunchKernelGGL(k_knn_bbox, dim3(kBboxBlocks), dim3(kBlock), 0, st, x, y, z, n, part);
    hipLaunchKernelGGL(k_knn_root, dim3(1), dim3(64), 0, st, part, kBboxBlocks, d3 ? 21 : 31, sync);
    hipLaunchKernelGGL(k_knn_keys, dim3(g), dim3(kBlock), 0, st, x, y, z, n, sync, k0, v0);
    const int w = radix_sort_u64(k0, v0, k1, v1, n, 8, hist, st);
    const uint32_t* perm = w ? v1 : v0;
    std::vector<int32_t> seg_start{0};
    KnnSync hs{};
    if (species) {
        uint32_t* sk0 = reinterpret_cast<uint32_t*>(W + L.sk0);
        uint32_t* sk1 = reinterpret_cast<uint32_t*>(W + L.sk1);
        int32_t* flag = reinterpret_cast<int32_t*>(W + L.flag);
        int32_t* pos = reinterpret_cast<int32_t*>(W + L.pos);
        int32_t* scan = reinterpret_cast<int32_t*>(W + L.scan);
        int32_t* starts = reinterpret_cast<int32_t*>(W + L.starts);
        // species values into (sk0, the free value buffer); the sort ping-pongs with (sk1, perm's buffer)
        uint32_t* sv0 = w ? v0 : v1;
        uint32_t* sv1 = const_cast<uint32_t*>(perm);
        hipLaunchKernelGGL(k_knn_species_keys, dim3(g), dim3(kBlock), 0, st, species, perm, n, sk0, sv0, sync);
        const int ws2 = radix_sort_u32(sk0, sv0, sk1, sv1, n, 2, hist, st);
        const uint32_t* skey = ws2 ? sk1 : sk0;
        perm = ws2 ? sv1 : sv0;
        hipLaunchKernelGGL(k_knn_seg_flags, dim3(g), dim3(kBlock), 0, st, skey, n, flag);
        exclusive_scan_i32(flag, pos, n, scan, st);
        hipLaunchKernelGGL(k_knn_seg_starts, dim3(g), dim3(kBlock), 0, st, skey, n, pos, starts, sync);
        GLM_HIP(hipMemcpyAsync(&hs, sync, sizeof(KnnSync), hipMemcpyDeviceToHost, st));
        GLM_HIP(hipStreamSynchronize(st));
        if (hs.bad) return fail(GLM_EDATA, "knn: NaN/Inf position");
        if (hs.bad_species) return fail(GLM_EDATA, "knn: species id outside [0, 65535]");
        if (hs.nseg < 1 || hs.nseg > n) return fail(GLM_EHIP, "knn: species segments inconsistent");
        seg_start.resize(hs.nseg);
        GLM_HIP(hipMemcpyAsync(seg_start.data(), starts, 4ull * hs.nseg, hipMemcpyDeviceToHost, st));
        GLM_HIP(hipStreamSynchronize(st));
    } else {
        GLM_HIP(hipMemcpyAsync(&hs, sync, sizeof(KnnSync), hipMemcpyDeviceToHost, st));
        GLM_HIP(hipStreamSynchronize(st));
        if (hs.bad) return fail(GLM_EDATA, "knn: NaN/Inf position");
    }
    seg_start.push_back((int32_t)n);
    for (size_t sgi = 0; sgi + 1 < seg_start.size(); ++sgi) {
        const int64_t ns = (int64_t)seg_start[sgi + 1] - seg_start[sgi];
        if (ns <= k)
            return fail(GLM_EDATA, "knn: a species has " + std::to_string(ns) + " particles, fewer than k + 1 = " +
                                       std::to_string(k + 1));
    }
    hipLaunchKernelGGL(k_knn_gather, dim3(g), dim3(kBlock), 0, st, perm, x, y, z, n, xs, ys, zs);
    // box margin far above the rounding of the box distance, so that pruning never drops a neighbour
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = fmax(ext, fabs(hs.hi[a]) + fabs(hs.lo[a]));
    const double margin = 1e-12 * (ext > 0.0 ? ext : 1.0);
    for (size_t sgi = 0; sgi + 1 < seg_start.size(); ++sgi) {
        const int64_t off = seg_start[sgi], ns = (int64_t)seg_start[sgi + 1] - off;
        Bvh B{};
        const int nl = bvh_levels(ns, B.cnt);
        int64_t tot = 0;
        for (int l = 0; l < nl; ++l) {
            B.off[l] = (int32_t)tot;
            tot += B.cnt[l];
        }
        if (tot > L.node_cap || B.cnt[nl - 1] != 1) return fail(GLM_EHIP, "knn: hierarchy larger than its workspace");
        B.top = nl - 1;
        for (int a = 0; a < 3; ++a) {
            B.lo[a] = nodes + (size_t)(2 * a) * L.node_cap;
            B.hi[a] = nodes + (size_t)(2 * a + 1) * L.node_cap;
        }
        const double* sx = xs + off;
        const double* sy = ys + off;
        const double* sz = zs + off;
        const uint32_t* sp = perm + off;
        if (d3) hipLaunchKernelGGL(k_bvh_leaves<true>, dim3(ceil_div(B.cnt[0], kBlock)), dim3(kBlock), 0, st, sx, sy,
                                   sz, (int)ns, margin, B);
        else hipLaunchKernelGGL(k_bvh_leaves<false>, dim3(ceil_div(B.cnt[0], kBlock)), dim3(kBlock), 0, st, sx, sy,
                                sz, (int)ns, margin, B);
        for (int l = 1; l < nl; ++l) {
            if (d3) hipLaunchKernelGGL(k_bvh_level<true>, dim3(ceil_div(B.cnt[l], kBlock)), dim3(kBlock), 0, st, B, l);
            else hipLaunchKernelGGL(k_bvh_level<false>, dim3(ceil_div(B.cnt[l], kBlock)), dim3(kBlock), 0, st, B, l);
        }
        const dim3 gb(ceil_div(ceil_div(ns, kWave), kBlock / kWave)), blk(kBlock);
#define GLM_KNN(KC)                                                                                             \
    do {                                                                                                        \
        if (d3) hipLaunchKernelGGL((k_knn_bvh<KC, true>), gb, blk, 0, st, sx, sy, sz, (int)ns, B, k, sp, s_out); \
        else hipLaunchKernelGGL((k_knn_bvh<KC, false>), gb, blk, 0, st, sx, sy, sz, (int)ns, B, k, sp, s_out);  \
    } while (0)
        if (k <= 16) GLM_KNN(16);
        else if (k <= 32) GLM_KNN(32);
        else GLM_KNN(64);
#undef GLM_KNN
    }
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

} // namespace glm
