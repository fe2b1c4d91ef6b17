// Forward tree walk on gfx950 (Sec. 3.2) with ray staging.
//
// One wavefront walks the tree for a group of 64 rays that are neighbours in
// Morton order.  The group shares one depth-first traversal of the preorder
// box array without a stack: every lane keeps the preorder index at which it
// becomes active again (after it accepted a box, it sleeps until the end of
// that box's subtree), the wave descends into a box if any awake lane opens
// it and jumps over the subtree otherwise.  Every decision is per ray, as in
// the paper's walk: per lane FP64 opening test |x - x_cm|^2 > r_cut^2, per
// lane FP64 inside test for each particle.  Box headers, moments and particle
// records are wave-uniform and come through scalar loads; only the
// big-particle lists are first filtered lane-parallel against the group's
// bounding box.  Evaluation is FP32: the multipole series is a Horner scheme
// in t = r_cm / w on moments normalised by M r_cm^k, alpha is accumulated with
// FP64 accumulation of the FP32 terms.
#include <math.h>

#include <algorithm>
#include <vector>

#include "eval.hpp"
#include "walk.hpp"

namespace glm {

namespace {

// The traversal of one 64-ray group (see the file comment).  Every lane of
// the wave must call it; `valid` lanes carry a ray.
// MODE: 0 = alpha summed in FP64 (the product walk), 1 = the same plus
// per-ray interaction counts, 2 = plain FP32 sum of the alpha terms (debug).
template <int MODE>
struct WalkMode {
    static constexpr bool f64a = MODE != 2;
    static constexpr bool stats = MODE == 1;
};

template <int P, bool AONLY, int MODE, bool PSI = false, int KIND = kKindGauss>
__device__ inline void walk_group(const TreeDev& T, double X, double Y, bool valid, int lane, Acc& A, int cnt[kCounts],
                                  int c0, int c1)
{
    constexpr bool F64A = WalkMode<MODE>::f64a;
    constexpr bool STATS = WalkMode<MODE>::stats;
    const double gx0 = wave_min(valid ? X : INFINITY), gx1 = wave_max(valid ? X : -INFINITY);
    const double gy0 = wave_min(valid ? Y : INFINITY), gy1 = wave_max(valid ? Y : -INFINITY);
    int n_vis = 0, n_acc = 0, n_dir = 0, n_hit = 0, n_scan = 0, w_acc = 0, w_dir = 0, w_cand = 0;
    int skip = valid ? 0 : 0x7fffffff;
    if (c0 > 0 && c0 < c1) skip = ancestor_skip(T, X, Y, c0, skip); // (an empty range walks nothing)
    int cur = c0;
    while (cur < c1) {
        cur = __builtin_amdgcn_readfirstlane(cur);
        const CellHdr h = T.hdr[cur];
        const bool act = cur >= skip;
        if constexpr (STATS) n_vis += act;
        if ((h.info & kInfoList) && list_reaches(T, cur, gx0, gx1, gy0, gy1)) {
            const CellExt e = T.ext[cur];
            for (int base = e.lbeg; base < e.lend; base += kWave) {
                if constexpr (STATS) n_scan += (base + kWave < e.lend ? kWave : e.lend - base);
                const int j = base + lane;
                bool cand = false;
                if (j < e.lend) {
                    const PRec pr = T.lst[j];
                    const double dx = fmax(fmax(gx0 - pr.x, pr.x - gx1), 0.0);
                    const double dy = fmax(fmax(gy0 - pr.y, pr.y - gy1), 0.0);
                    cand = dx * dx + dy * dy < pr.qs2 * (1.0 + 1e-9);
                }
                uint64_t cm = __ballot(cand);
                if constexpr (STATS) w_cand += __popcll(cm);
                while (cm) {
                    const int k = __ffsll((unsigned long long)cm) - 1;
                    cm &= cm - 1;
                    const PRec pr = T.lst[__builtin_amdgcn_readfirstlane(base + k)];
                    if (act) list_particle<AONLY, F64A, PSI, KIND>(pr, X, Y, A, n_hit, T.psiK, T.einTerms, T.invC);
                }
            }
        }
        double w1, w2;
        const double d2 = sqdist(X, Y, h.cx, h.cy, &w1, &w2);
        const bool acc = act && d2 > h.rcut2;
        const bool opn = act && !acc;
        if constexpr (STATS) n_acc += acc;
        if (__any(acc)) {
            if constexpr (STATS) ++w_acc;
            if (acc) eval_box<P, AONLY, F64A, PSI>(T.mom + (size_t)cur * mom_stride(P), w1, w2, A);
        }
        if (h.info & kInfoLeaf) {
            if (__any(opn)) {
                const CellExt e = T.ext[cur];
                if constexpr (STATS) {
                    if (opn) n_dir += e.pend - e.pbeg;
                    w_dir += e.pend - e.pbeg;
                }
                for (int j = e.pbeg; j < e.pend; ++j) {
                    const PRec pr = T.prt[j];
                    if (opn) leaf_particle<AONLY, F64A, PSI, KIND>(pr, X, Y, A, T.psiK, T.einTerms, T.invC);
                }
            }
            cur = cur + 1;
        } else if (__any(opn)) {
            if (acc) skip = h.next;
            cur = cur + 1;
        } else {
            cur = h.next > cur ? h.next : cur + 1; // preorder: the subtree ends after cur
        }
    }
    cnt[0] = n_vis;
    cnt[1] = n_acc;
    cnt[2] = n_dir;
    cnt[3] = n_hit;
    cnt[4] = n_scan;
    cnt[5] = w_acc;
    cnt[6] = w_dir;
    cnt[7] = w_cand;
}

template <bool AONLY, bool STATS, bool PSI = false>
__device__ inline void write_out(const Acc& A, const int cnt[kCounts], int64_t o, const WalkOut& out)
{
    const double a1 = alpha1(A), a2 = alpha2(A);
    out.a1[o] = (float)a1;
    out.a2[o] = (float)a2;
    if constexpr (PSI) {
        out.psi[o] = (float)A.ps;
        if (out.td) out.td[o] = (float)(0.5 * (a1 * a1 + a2 * a2) - A.ps); // Sec. 3.2: |alpha|^2 / 2 - psi
    }
    if (!AONLY) {
        if (out.k) out.k[o] = A.k;
        if (out.g1) out.g1[o] = (float)A.g1;
        if (out.g2) out.g2[o] = (float)A.g2;
    }
    if (STATS && out.counts)
        for (int i = 0; i < kCounts; ++i) out.counts[kCounts * o + i] = cnt[i];
}

template <int P, bool AONLY, int MODE, bool PSI = false, int KIND = kKindGauss>
__global__ __launch_bounds__(kBlock) void k_walk(TreeDev T, const double* __restrict__ rxs,
                                                const double* __restrict__ rys, const uint32_t* __restrict__ rperm,
                                                int64_t nrays, WalkOut out, int K, Partial* __restrict__ parts,
                                                const int* __restrict__ split_box)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t groups = (nrays + kWave - 1) / kWave;
    // wave-uniform work item (kept in SGPRs): box range k, ray group grp
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    int k;
    int64_t grp;
    if (!walk_task(blockIdx.x, w, groups, K, &k, &grp)) return;
    const int64_t r = grp * kWave + lane;
    const bool valid = r < nrays;
    const double X = valid ? rxs[r] : 0.0, Y = valid ? rys[r] : 0.0;
    const int nc = T.ncells;
    int c0, c1;
    if (K > 1) {
        const int B = __builtin_amdgcn_readfirstlane(*split_box);
        if (B >= 0) {
            split_range(k, K, B, T.hdr[B].next, nc, &c0, &c1);
        } else { // no split: the first range takes every box
            c0 = 0;
            c1 = k == 0 ? nc : 0;
        }
    } else {
        c0 = 0;
        c1 = nc;
    }
    Acc A = {};
    int cnt[kCounts];
    walk_group<P, AONLY, MODE, PSI, KIND>(T, X, Y, valid, lane, A, cnt, c0, c1);
    if (!valid) return;
    if (K == 1) {
        write_out<AONLY, WalkMode<MODE>::stats, PSI>(A, cnt, rperm ? (int64_t)rperm[r] : r, out);
        return;
    }
    Partial q;
    q.a1 = alpha1(A);
    q.a2 = alpha2(A);
    q.k = A.k;
    q.g1 = A.g1;
    q.g2 = A.g2;
    for (int i = 0; i < kCounts; ++i) q.cnt[i] = WalkMode<MODE>::stats ? cnt[i] : 0;
    parts[(int64_t)k * nrays + r] = q;
}

// Per ray, the partial sums of the K box ranges in range order.
template <bool AONLY>
__global__ __launch_bounds__(kBlock) void k_walk_merge(const Partial* __restrict__ parts, int K, int64_t nrays,
                                                      const uint32_t* __restrict__ rperm, WalkOut out)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= nrays) return;
    double a1 = 0.0, a2 = 0.0, g1 = 0.0, g2 = 0.0;
    float ka = 0.0f;
    int c[kCounts] = {};
    for (int k = 0; k < K; ++k) {
        const Partial& q = parts[(int64_t)k * nrays + r];
        a1 += q.a1;
        a2 += q.a2;
        ka += q.k;
        g1 += q.g1;
        g2 += q.g2;
        for (int i = 0; i < kCounts; ++i) c[i] += q.cnt[i];
    }
    const int64_t o = rperm ? (int64_t)rperm[r] : r;
    out.a1[o] = (float)a1;
    out.a2[o] = (float)a2;
    if (!AONLY) {
        if (out.k) out.k[o] = ka;
        if (out.g1) out.g1[o] = (float)g1;
        if (out.g2) out.g2[o] = (float)g2;
    }
    if (out.counts)
        for (int i = 0; i < kCounts; ++i) out.counts[kCounts * o + i] = c[i];
}

// Persistent walk over many lenses: every wavefront takes (lens, 64-ray group)
// items from a device counter until the queue is empty.  Lenses are ranked by
// estimated cost, so the largest ray groups start first.
template <int P, bool AONLY, int MODE, int KIND>
__global__ __launch_bounds__(kBlock) void k_walk_batched(const BatchLens* __restrict__ lenses, int nlens,
                                                        const int64_t* __restrict__ gprefix, int* __restrict__ counter,
                                                        const double* __restrict__ xs, const double* __restrict__ ys,
                                                        const uint32_t* __restrict__ perm)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t total = gprefix[nlens];
    for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(counter, 1);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, kWave));
        if (it >= total) break;
        int lo = 0, hi = nlens; // largest l with gprefix[l] <= it
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (gprefix[mid] <= it) lo = mid;
            else hi = mid;
        }
        const BatchLens& L = lenses[lo];
        const int64_t rl = (int64_t)(it - gprefix[lo]) * kWave + lane;
        const bool valid = rl < L.nrays;
        const int64_t gi = L.ray_off + (valid ? rl : 0);
        const double X = valid ? xs[gi] : 0.0, Y = valid ? ys[gi] : 0.0;
        Acc A = {};
        int cnt[kCounts];
        walk_group<P, AONLY, MODE, false, KIND>(L.tree, X, Y, valid, lane, A, cnt, 0, L.tree.ncells);
        if (valid) write_out<AONLY, false>(A, cnt, (int64_t)perm[gi] - L.ray_off, L.out);
    }
}

// ------------------------------------------------------------ ray staging

// blocks of the first pass of the ray bounding box (enough waves in flight to
// stream the coordinates at full bandwidth)
constexpr int kRayBboxBlocks = 1024;

__global__ __launch_bounds__(kBlock) void k_ray_bbox(const double* __restrict__ x, const double* __restrict__ y,
                                                    int64_t n, double* __restrict__ part)
{
    __shared__ double red[4][kBlock];
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        x0 = fmin(x0, x[i]);
        x1 = fmax(x1, x[i]);
        y0 = fmin(y0, y[i]);
        y1 = fmax(y1, y[i]);
    }
    red[0][threadIdx.x] = x0;
    red[1][threadIdx.x] = x1;
    red[2][threadIdx.x] = y0;
    red[3][threadIdx.x] = y1;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + o]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + o]);
            red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + o]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) part[blockIdx.x * 4 + k] = red[k][0];
}

__device__ inline uint32_t spread16(uint32_t v)
{
    uint32_t x = v & 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// bounding box of the rays from the per-block partials
__global__ __launch_bounds__(kBlock) void k_ray_root(const double* __restrict__ part, int nb, double* __restrict__ bb)
{
    __shared__ double red[4][kBlock];
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        v[0] = fmin(v[0], part[b * 4 + 0]);
        v[1] = fmax(v[1], part[b * 4 + 1]);
        v[2] = fmin(v[2], part[b * 4 + 2]);
        v[3] = fmax(v[3], part[b * 4 + 3]);
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + o]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + o]);
            red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + o]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) bb[threadIdx.x] = red[threadIdx.x][0];
}

// Morton keys of the rays in their bounding square, `bits` (<= 16) per axis
__global__ __launch_bounds__(kBlock) void k_ray_keys(const double* __restrict__ x, const double* __restrict__ y,
                                                    int64_t n, const double* __restrict__ bb, int bits,
                                                    uint32_t* __restrict__ key, uint32_t* __restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double bx0 = bb[0], by0 = bb[2];
    double ext = fmax(bb[1] - bx0, bb[3] - by0);
    if (!(ext > 0.0)) ext = 1.0;
    const double top = (double)((1u << bits) - 1u);
    const double sc = top / ext;
    const uint32_t qx = (uint32_t)fmin(fmax((x[i] - bx0) * sc, 0.0), top);
    const uint32_t qy = (uint32_t)fmin(fmax((y[i] - by0) * sc, 0.0), top);
    key[i] = spread16(qx) | (spread16(qy) << 1);
    val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_ray_gather(const uint32_t* __restrict__ perm, const double* __restrict__ x,
                                                      const double* __restrict__ y, int64_t n, double* __restrict__ xs,
                                                      double* __restrict__ ys)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    xs[k] = x[perm[k]];
    ys[k] = y[perm[k]];
}

// The deepest box whose square holds the rays' bounding box (one thread);
// -1 when the rays cover under 5% of the root square: their work then sits in
// a small part of the tree and splitting by box ranges would not spread it.
__global__ void k_split_box(BoxArrays b, const int32_t* __restrict__ next, double x0, double y0, double S,
                            const double* __restrict__ bb, int ncells, int* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if ((bb[1] - bb[0]) * (bb[3] - bb[2]) < 0.05 * S * S) {
        *out = -1;
        return;
    }
    int c = 0;
    for (int guard = 0; guard <= kMaxLevel; ++guard) {
        if (b.leaf[c]) break;
        int found = -1;
        for (int ch = c + 1, n = 0; ch < next[c] && n < 4; ch = next[ch] > ch ? next[ch] : ch + 1, ++n) {
            const double side = ldexp(S, -b.level[ch]);
            const double bx0 = x0 + (double)b.ix[ch] * side, by0 = y0 + (double)b.iy[ch] * side;
            if (bb[0] >= bx0 && bb[1] < bx0 + side && bb[2] >= by0 && bb[3] < by0 + side) {
                found = ch;
                break;
            }
        }
        if (found < 0) break;
        c = found;
    }
    *out = c < ncells ? c : 0;
}

template <int P, bool AONLY>
void launch_walk(const TreeDev& T, const double* rxs, const double* rys, const uint32_t* rperm, int64_t nrays,
                 const WalkOut& out, int mode, int K, Partial* parts, const int* split_box, hipStream_t st)
{
    const dim3 g((unsigned)walk_grid_blocks((nrays + kWave - 1) / kWave, K)), b(kBlock);
#define GLM_WALK(MD, KD) \
    hipLaunchKernelGGL((k_walk<P, AONLY, MD, false, KD>), g, b, 0, st, T, rxs, rys, rperm, nrays, out, K, parts, split_box)
    if (T.kind == kKindNfw) {
        if (mode == 1) GLM_WALK(1, kKindNfw);
        else if (mode == 2) GLM_WALK(2, kKindNfw);
        else GLM_WALK(0, kKindNfw);
    } else {
        if (mode == 1) GLM_WALK(1, kKindGauss);
        else if (mode == 2) GLM_WALK(2, kKindGauss);
        else GLM_WALK(0, kKindGauss);
    }
#undef GLM_WALK
    if (K > 1)
        hipLaunchKernelGGL((k_walk_merge<AONLY>), dim3(ceil_div(nrays, kBlock)), b, 0, st, parts, K, nrays, rperm, out);
}

// alpha and psi in one walk, no split (K = 1)
template <int P>
void launch_potential(const TreeDev& T, const double* rxs, const double* rys, const uint32_t* rperm, int64_t nrays,
                      const WalkOut& out, hipStream_t st)
{
    const dim3 g((unsigned)walk_grid_blocks((nrays + kWave - 1) / kWave, 1)), b(kBlock);
    if (T.kind == kKindNfw)
        hipLaunchKernelGGL((k_walk<P, true, 0, true, kKindNfw>), g, b, 0, st, T, rxs, rys, rperm, nrays, out, 1, nullptr,
                           nullptr);
    else
        hipLaunchKernelGGL((k_walk<P, true, 0, true, kKindGauss>), g, b, 0, st, T, rxs, rys, rperm, nrays, out, 1,
                           nullptr, nullptr);
}

template <bool AONLY>
void dispatch_walk(int p, const TreeDev& T, const double* rxs, const double* rys, const uint32_t* rperm,
                   int64_t nrays, const WalkOut& out, int mode, int K, Partial* parts, const int* split_box,
                   hipStream_t st)
{
#define GLM_CASE(PP) \
    case PP: launch_walk<PP, AONLY>(T, rxs, rys, rperm, nrays, out, mode, K, parts, split_box, st); break;
    switch (p) {
        GLM_CASE(0) GLM_CASE(1) GLM_CASE(2) GLM_CASE(3) GLM_CASE(4) GLM_CASE(5) GLM_CASE(6)
        GLM_CASE(7) GLM_CASE(8) GLM_CASE(9) GLM_CASE(10) GLM_CASE(11) GLM_CASE(12)
        default: break;
    }
#undef GLM_CASE
}

void dispatch_potential(int p, const TreeDev& T, const double* rxs, const double* rys, const uint32_t* rperm,
                        int64_t nrays, const WalkOut& out, hipStream_t st)
{
#define GLM_CASE(PP) \
    case PP: launch_potential<PP>(T, rxs, rys, rperm, nrays, out, st); break;
    switch (p) {
        GLM_CASE(0) GLM_CASE(1) GLM_CASE(2) GLM_CASE(3) GLM_CASE(4) GLM_CASE(5) GLM_CASE(6)
        GLM_CASE(7) GLM_CASE(8) GLM_CASE(9) GLM_CASE(10) GLM_CASE(11) GLM_CASE(12)
        default: break;
    }
#undef GLM_CASE
}

} // namespace

RayLayout ray_layout(int64_t nrays)
{
    RayLayout L;
    Arena a;
    L.k0 = a.take(4ull * nrays);
    L.k1 = a.take(4ull * nrays);
    L.v0 = a.take(4ull * nrays);
    L.v1 = a.take(4ull * nrays);
    L.xs = a.take(8ull * nrays);
    L.ys = a.take(8ull * nrays);
    L.hist = a.take(4ull * radix_hist_words(nrays));
    L.part = a.take(sizeof(double) * 4 * (kRayBboxBlocks + 1));
    L.sbox = a.take(64);
    L.split = walk_split(nrays);
    L.parts = a.take(sizeof(Partial) * (size_t)split_slots(nrays));
    L.bytes = a.size;
    return L;
}

// Bits per axis of the ray sort key.  The key only forms the 64-ray groups
// (per-ray results do not depend on them): about four cells per ray suffice,
// 8 to 16 bits per axis.
static int ray_key_bits(int64_t nrays)
{
    int bits = 8;
    while (bits < 16 && (1ll << (2 * bits)) < 4 * nrays) ++bits;
    return bits;
}

glm_status stage_rays(const double* rx, const double* ry, int64_t nrays, void* ws, const RayLayout& L,
                      StagedRays* out, hipStream_t st)
{
    char* W = static_cast<char*>(ws);
    uint32_t* k0 = reinterpret_cast<uint32_t*>(W + L.k0);
    uint32_t* k1 = reinterpret_cast<uint32_t*>(W + L.k1);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(W + L.v0);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(W + L.v1);
    double* xs = reinterpret_cast<double*>(W + L.xs);
    double* ys = reinterpret_cast<double*>(W + L.ys);
    uint32_t* hist = reinterpret_cast<uint32_t*>(W + L.hist);
    double* part = reinterpret_cast<double*>(W + L.part);
    const int nbb = kRayBboxBlocks;
    const int g = ceil_div(nrays, kBlock);
    hipLaunchKernelGGL(k_ray_bbox, dim3(nbb), dim3(kBlock), 0, st, rx, ry, nrays, part);
    hipLaunchKernelGGL(k_ray_root, dim3(1), dim3(kBlock), 0, st, part, nbb, part + 4 * nbb);
    const int bits = ray_key_bits(nrays);
    hipLaunchKernelGGL(k_ray_keys, dim3(g), dim3(kBlock), 0, st, rx, ry, nrays, part + 4 * nbb, bits, k0, v0);
    const int w = radix_sort_u32(k0, v0, k1, v1, nrays, (2 * bits + 7) / 8, hist, st);
    const uint32_t* perm = w ? v1 : v0;
    hipLaunchKernelGGL(k_ray_gather, dim3(g), dim3(kBlock), 0, st, perm, rx, ry, nrays, xs, ys);
    GLM_HIP(hipGetLastError());
    *out = staged_rays_view(nrays, ws, L);
    return GLM_OK;
}

StagedRays staged_rays_view(int64_t nrays, void* ws, const RayLayout& L)
{
    char* W = static_cast<char*>(ws);
    // the sort ends in (k1, v1) after an odd number of passes (radix_sort_u32)
    const int passes = (2 * ray_key_bits(nrays) + 7) / 8;
    const uint32_t* perm = reinterpret_cast<const uint32_t*>(W + ((passes & 1) ? L.v1 : L.v0));
    return StagedRays{reinterpret_cast<const double*>(W + L.xs), reinterpret_cast<const double*>(W + L.ys), perm};
}

// ------------------------------------------------------------ batched walk

namespace {

constexpr int kBboxSplit = 32; // blocks per lens for the ray bounding boxes

__global__ __launch_bounds__(kBlock) void k_batch_bbox(const BatchLens* __restrict__ lenses, double* __restrict__ part)
{
    __shared__ double red[4][kBlock];
    const BatchLens& L = lenses[blockIdx.x];
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.y * kBlock + threadIdx.x; i < L.nrays; i += (int64_t)kBlock * kBboxSplit) {
        const double x = L.rx[i], y = L.ry[i];
        v[0] = fmin(v[0], x);
        v[1] = fmax(v[1], x);
        v[2] = fmin(v[2], y);
        v[3] = fmax(v[3], y);
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + o]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + o]);
            red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + o]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[((size_t)blockIdx.x * kBboxSplit + blockIdx.y) * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_batch_bbox_final(const double* __restrict__ part, int nlens, double* __restrict__ bb)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * nlens) return;
    const int l = t / 4, k = t % 4;
    double v = (k & 1) ? -INFINITY : INFINITY;
    for (int b = 0; b < kBboxSplit; ++b) {
        const double p = part[((size_t)l * kBboxSplit + b) * 4 + k];
        v = (k & 1) ? fmax(v, p) : fmin(v, p);
    }
    bb[t] = v;
}

__device__ inline int find_lens(const int64_t* __restrict__ roff, int nlens, int64_t gi)
{
    int lo = 0, hi = nlens;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (roff[mid] <= gi) lo = mid;
        else hi = mid;
    }
    return lo;
}

// key = lens rank << 32 | 16-bit-per-axis Morton code in the lens's ray box
__global__ __launch_bounds__(kBlock) void k_batch_keys(const BatchLens* __restrict__ lenses, int nlens,
                                                      const int64_t* __restrict__ roff, const double* __restrict__ bb,
                                                      int64_t total, int bits, uint64_t* __restrict__ key,
                                                      uint32_t* __restrict__ val)
{
    const int64_t gi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gi >= total) return;
    const int l = find_lens(roff, nlens, gi);
    const int64_t i = gi - roff[l];
    const double bx0 = bb[4 * l], by0 = bb[4 * l + 2];
    double ext = fmax(bb[4 * l + 1] - bx0, bb[4 * l + 3] - by0);
    if (!(ext > 0.0)) ext = 1.0;
    const double top = (double)((1u << bits) - 1u);
    const double sc = top / ext;
    const uint32_t qx = (uint32_t)fmin(fmax((lenses[l].rx[i] - bx0) * sc, 0.0), top);
    const uint32_t qy = (uint32_t)fmin(fmax((lenses[l].ry[i] - by0) * sc, 0.0), top);
    key[gi] = ((uint64_t)l << (2 * bits)) | (uint64_t)(spread16(qx) | (spread16(qy) << 1));
    val[gi] = (uint32_t)gi;
}

__global__ __launch_bounds__(kBlock) void k_batch_gather(const BatchLens* __restrict__ lenses,
                                                        const int64_t* __restrict__ roff,
                                                        const uint64_t* __restrict__ key,
                                                        const uint32_t* __restrict__ val, int64_t total, int bits,
                                                        double* __restrict__ xs, double* __restrict__ ys)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= total) return;
    const int l = (int)(key[k] >> (2 * bits));
    const int64_t i = (int64_t)val[k] - roff[l];
    xs[k] = lenses[l].rx[i];
    ys[k] = lenses[l].ry[i];
}

__global__ void k_zero_int(int* p) { *p = 0; }

struct BatchLayout {
    size_t table, roff, gpre, bb, bbpart, counter, k0, k1, v0, v1, xs, ys, hist, bytes;
};

BatchLayout batch_layout(int nlens, int64_t total)
{
    BatchLayout B;
    Arena a;
    B.table = a.take(sizeof(BatchLens) * (size_t)nlens);
    B.roff = a.take(8ull * (nlens + 1));
    B.gpre = a.take(8ull * (nlens + 1));
    B.bb = a.take(32ull * nlens);
    B.bbpart = a.take(32ull * nlens * kBboxSplit);
    B.counter = a.take(64);
    B.k0 = a.take(8ull * total);
    B.k1 = a.take(8ull * total);
    B.v0 = a.take(4ull * total);
    B.v1 = a.take(4ull * total);
    B.xs = a.take(8ull * total);
    B.ys = a.take(8ull * total);
    B.hist = a.take(4ull * radix_hist_words(total));
    B.bytes = a.size;
    return B;
}

template <int P, bool AONLY>
void launch_batched(const BatchLens* table, int nlens, const int64_t* gpre, int* counter, const double* xs,
                    const double* ys, const uint32_t* perm, int64_t items, int f64a, int kind, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>((items + 3) / 4, 256 * 8);
#define GLM_WALK(MD, KD)                                                                                    \
    hipLaunchKernelGGL((k_walk_batched<P, AONLY, MD, KD>), dim3(blocks), dim3(kBlock), 0, st, table, nlens, gpre, \
                       counter, xs, ys, perm)
    if (kind == kKindNfw) {
        if (f64a) GLM_WALK(0, kKindNfw);
        else GLM_WALK(2, kKindNfw);
    } else {
        if (f64a) GLM_WALK(0, kKindGauss);
        else GLM_WALK(2, kKindGauss);
    }
#undef GLM_WALK
}

} // namespace

size_t batch_workspace_bytes(int nlens, int64_t total) { return batch_layout(nlens, total).bytes; }

glm_status shoot_batched_device(const BatchLens* host_table, int nlens, int order, uint32_t flags, void* ws,
                                hipStream_t st)
{
    int64_t total = 0, items = 0;
    std::vector<int64_t> roff(nlens + 1), gpre(nlens + 1);
    for (int l = 0; l < nlens; ++l) {
        roff[l] = total;
        gpre[l] = items;
        total += host_table[l].nrays;
        items += (host_table[l].nrays + kWave - 1) / kWave;
    }
    roff[nlens] = total;
    gpre[nlens] = items;
    if (total == 0) return GLM_OK;
    std::vector<BatchLens> tab(host_table, host_table + nlens);
    for (int l = 0; l < nlens; ++l) tab[l].ray_off = roff[l];
    const BatchLayout B = batch_layout(nlens, total);
    char* W = static_cast<char*>(ws);
    BatchLens* dtab = reinterpret_cast<BatchLens*>(W + B.table);
    int64_t* droff = reinterpret_cast<int64_t*>(W + B.roff);
    int64_t* dgpre = reinterpret_cast<int64_t*>(W + B.gpre);
    double* bb = reinterpret_cast<double*>(W + B.bb);
    int* counter = reinterpret_cast<int*>(W + B.counter);
    uint64_t* k0 = reinterpret_cast<uint64_t*>(W + B.k0);
    uint64_t* k1 = reinterpret_cast<uint64_t*>(W + B.k1);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(W + B.v0);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(W + B.v1);
    double* xs = reinterpret_cast<double*>(W + B.xs);
    double* ys = reinterpret_cast<double*>(W + B.ys);
    uint32_t* hist = reinterpret_cast<uint32_t*>(W + B.hist);
    GLM_HIP(hipMemcpyAsync(dtab, tab.data(), sizeof(BatchLens) * nlens, hipMemcpyHostToDevice, st));
    GLM_HIP(hipMemcpyAsync(droff, roff.data(), 8ull * (nlens + 1), hipMemcpyHostToDevice, st));
    GLM_HIP(hipMemcpyAsync(dgpre, gpre.data(), 8ull * (nlens + 1), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, counter);
    double* bbpart = reinterpret_cast<double*>(W + B.bbpart);
    hipLaunchKernelGGL(k_batch_bbox, dim3(nlens, kBboxSplit), dim3(kBlock), 0, st, dtab, bbpart);
    hipLaunchKernelGGL(k_batch_bbox_final, dim3(ceil_div(4 * nlens, 64)), dim3(64), 0, st, bbpart, nlens, bb);
    const int g = ceil_div(total, kBlock);
    // per lens, about four Morton cells per ray (the largest lens sets the width)
    int64_t most = 0;
    for (int l = 0; l < nlens; ++l) most = std::max(most, host_table[l].nrays);
    int bits = 8;
    while (bits < 16 && (1ll << (2 * bits)) < 4 * most) ++bits;
    hipLaunchKernelGGL(k_batch_keys, dim3(g), dim3(kBlock), 0, st, dtab, nlens, droff, bb, total, bits, k0, v0);
    int lens_bits = 0;
    while ((1 << lens_bits) < nlens) ++lens_bits;
    const int passes = (2 * bits + lens_bits + 7) / 8;
    const int w = radix_sort_u64(k0, v0, k1, v1, total, passes, hist, st);
    const uint64_t* ks = w ? k1 : k0;
    const uint32_t* perm = w ? v1 : v0;
    hipLaunchKernelGGL(k_batch_gather, dim3(g), dim3(kBlock), 0, st, dtab, droff, ks, perm, total, bits, xs, ys);
    const int f64a = (flags & GLM_FP32_ALPHA) ? 0 : 1;
    const int kind = host_table[0].tree.kind; // every lens of a batch has the same particle kind
#define GLM_CASE(PP)                                                                                     \
    case PP:                                                                                             \
        if (flags & GLM_ALPHA_ONLY)                                                                      \
            launch_batched<PP, true>(dtab, nlens, dgpre, counter, xs, ys, perm, items, f64a, kind, st); \
        else                                                                                             \
            launch_batched<PP, false>(dtab, nlens, dgpre, counter, xs, ys, perm, items, f64a, kind, st);\
        break;
    switch (order) {
        GLM_CASE(0) GLM_CASE(1) GLM_CASE(2) GLM_CASE(3) GLM_CASE(4) GLM_CASE(5) GLM_CASE(6)
        GLM_CASE(7) GLM_CASE(8) GLM_CASE(9) GLM_CASE(10) GLM_CASE(11) GLM_CASE(12)
        default: return fail(GLM_EINVAL, "unsupported order");
    }
#undef GLM_CASE
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

glm_status split_box_device(const TreeStorage& ts, const double* rx, const double* ry, int64_t nrays, void* ws,
                            const RayLayout& L, bool have_bbox, int** out, hipStream_t st)
{
    char* W = static_cast<char*>(ws);
    double* part = reinterpret_cast<double*>(W + L.part);
    const int nbb = kRayBboxBlocks;
    if (!have_bbox) {
        hipLaunchKernelGGL(k_ray_bbox, dim3(nbb), dim3(kBlock), 0, st, rx, ry, nrays, part);
        hipLaunchKernelGGL(k_ray_root, dim3(1), dim3(kBlock), 0, st, part, nbb, part + 4 * nbb);
    }
    int* sb = reinterpret_cast<int*>(W + L.sbox);
    hipLaunchKernelGGL(k_split_box, dim3(1), dim3(1), 0, st, ts.b, ts.b.next, ts.x0, ts.y0, ts.side, part + 4 * nbb,
                       ts.ncells, sb);
    GLM_HIP(hipGetLastError());
    *out = sb;
    return GLM_OK;
}

glm_status shoot_device(const TreeStorage& ts, const double* rx, const double* ry, int64_t nrays, float* a1,
                        float* a2, float* k, float* g1, float* g2, int32_t* counts, uint32_t flags, void* ws,
                        hipStream_t st)
{
    if (nrays == 0) return GLM_OK;
    StagedRays sr{rx, ry, nullptr};
    const RayLayout L = ray_layout(nrays);
    if (flags & GLM_RAYS_STAGED) {
        sr = staged_rays_view(nrays, ws, L); // glm_stage_rays left them in the workspace
    } else if (!(flags & GLM_RAYS_ORDERED)) {
        glm_status rc = stage_rays(rx, ry, nrays, ws, L, &sr, st);
        if (rc != GLM_OK) return rc;
    }
    // box ranges per group: never more than one range per 64 boxes
    int K = L.split;
    while (K > 1 && (int64_t)K * 64 > ts.ncells) --K;
    if (K < 4) K = 1;
    Partial* parts = K > 1 ? reinterpret_cast<Partial*>(static_cast<char*>(ws) + L.parts) : nullptr;
    int* split_box = nullptr;
    if (K > 1) {
        glm_status rc = split_box_device(ts, rx, ry, nrays, ws, L, !(flags & GLM_RAYS_ORDERED), &split_box, st);
        if (rc != GLM_OK) return rc;
    }
    // counts requested: the product walk with counters; else the product or the plain-FP32 walk
    const int mode = counts ? 1 : ((flags & GLM_FP32_ALPHA) ? 2 : 0);
    if (flags & GLM_ALPHA_ONLY)
        dispatch_walk<true>(ts.params.order, ts.dev, sr.xs, sr.ys, sr.perm, nrays,
                            WalkOut{a1, a2, nullptr, nullptr, nullptr, counts}, mode, K, parts, split_box, st);
    else
        dispatch_walk<false>(ts.params.order, ts.dev, sr.xs, sr.ys, sr.perm, nrays, WalkOut{a1, a2, k, g1, g2, counts},
                             mode, K, parts, split_box, st);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

glm_status potential_device(const TreeStorage& ts, const double* rx, const double* ry, int64_t nrays, float* a1,
                            float* a2, float* psi, float* td, uint32_t flags, void* ws, hipStream_t st)
{
    if (nrays == 0) return GLM_OK;
    StagedRays sr{rx, ry, nullptr};
    const RayLayout L = ray_layout(nrays);
    if (!(flags & GLM_RAYS_ORDERED)) {
        glm_status rc = stage_rays(rx, ry, nrays, ws, L, &sr, st);
        if (rc != GLM_OK) return rc;
    }
    WalkOut out{a1, a2, nullptr, nullptr, nullptr, nullptr};
    out.psi = psi;
    out.td = td;
    dispatch_potential(ts.params.order, ts.dev, sr.xs, sr.ys, sr.perm, nrays, out, st);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

} // namespace glm
