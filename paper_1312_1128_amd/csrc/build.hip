// Tree construction on gfx950 (Sec. 3.2): root square, Morton order, the
// equal-area quad-tree as Morton-prefix ranges in depth-first preorder,
// big-particle lists, and FP64 multipole moments built bottom-up.
//
// Layout: a box is identified by (first particle in Morton order, level).
// Sorting boxes by that pair is exactly depth-first preorder with children in
// Morton order, so a box's preorder index is (number of boxes starting before
// its first particle) + (its level - the shallowest level that starts there),
// and the box after its subtree starts at its end position.  Every step is a
// flat per-particle or per-box kernel; the only host round trip reads the box
// count to size the box arrays.
#include <math.h>
#include <stddef.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "build.hpp"
#include "eval.hpp"

namespace glm {

namespace {

constexpr uint32_t kUnlisted32 = 0xFFFFFFFFu;

__device__ inline uint64_t spread_bits(uint32_t v)
{
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ inline uint32_t compact_bits(uint64_t x)
{
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}

__device__ inline uint64_t prefix_at(uint64_t k, int level) { return level == 0 ? 0ull : (k >> (64 - 2 * level)); }

// shallowest level at which a box starts at Morton position i (33: none)
__device__ inline int level_start(const uint64_t* K, int i)
{
    if (i == 0) return 0;
    const uint64_t d = K[i] ^ K[i - 1];
    if (d == 0) return 33;
    const int b = 63 - __clzll((long long)d);
    return (65 - b) >> 1;
}

// first j in [lo, hi) whose level-`level` prefix exceeds P
__device__ inline int upper_prefix(const uint64_t* K, int lo, int hi, uint64_t P, int level)
{
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (prefix_at(K[mid], level) > P) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// first j in [lo, hi) whose prefix is >= P
__device__ inline int lower_prefix(const uint64_t* K, int lo, int hi, uint64_t P, int level)
{
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (prefix_at(K[mid], level) >= P) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// ----------------------------------------------------------------- inputs

__global__ __launch_bounds__(kBlock) void k_bbox_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                        const double* __restrict__ m, const double* __restrict__ s,
                                                        int64_t n, double* __restrict__ part)
{
    __shared__ double red[4][kBlock];
    __shared__ uint32_t bad_s;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double xi = x[i], yi = y[i], mi = m[i], si = s ? s[i] : 0.0;
        if (!isfinite(xi) || !isfinite(yi) || !isfinite(mi) || !isfinite(si) || mi < 0.0 || si < 0.0) bad = 1;
        x0 = fmin(x0, xi);
        x1 = fmax(x1, xi);
        y0 = fmin(y0, yi);
        y1 = fmax(y1, yi);
    }
    if (bad) atomicOr(&bad_s, 1u);
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
    if (threadIdx.x == 0) {
        part[blockIdx.x * 5 + 0] = red[0][0];
        part[blockIdx.x * 5 + 1] = red[1][0];
        part[blockIdx.x * 5 + 2] = red[2][0];
        part[blockIdx.x * 5 + 3] = red[3][0];
        part[blockIdx.x * 5 + 4] = bad_s ? 1.0 : 0.0;
    }
}

// Root square: centre of the bounding box, side = max extent * (1 + 2^-40)
// (1 if the extent is 0), 32-bit quantisation scale 2^32 / side.
__global__ __launch_bounds__(kBlock) void k_root(const double* __restrict__ part, int nb, BuildSync* __restrict__ sync)
{
#pragma clang fp contract(off)
    __shared__ double red[5][kBlock];
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY, bad = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        x0 = fmin(x0, part[b * 5 + 0]);
        x1 = fmax(x1, part[b * 5 + 1]);
        y0 = fmin(y0, part[b * 5 + 2]);
        y1 = fmax(y1, part[b * 5 + 3]);
        bad = fmax(bad, part[b * 5 + 4]);
    }
    red[0][threadIdx.x] = x0;
    red[1][threadIdx.x] = x1;
    red[2][threadIdx.x] = y0;
    red[3][threadIdx.x] = y1;
    red[4][threadIdx.x] = bad;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + o]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + o]);
            red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + o]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + o]);
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    x0 = red[0][0];
    x1 = red[1][0];
    y0 = red[2][0];
    y1 = red[3][0];
    const double ex = x1 - x0, ey = y1 - y0;
    const double ext = ex > ey ? ex : ey;
    double S = ext * (1.0 + 0x1p-40);
    if (!(S > 0.0)) S = 1.0;
    sync->x0 = 0.5 * (x0 + x1) - 0.5 * S;
    sync->y0 = 0.5 * (y0 + y1) - 0.5 * S;
    sync->side = S;
    sync->scale = 4294967296.0 / S;
    sync->bad = red[4][0] != 0.0;
}

__device__ inline uint32_t quantise(double v, double v0, double scale)
{
#pragma clang fp contract(off)
    const double t = (v - v0) * scale;
    if (!(t >= 0.0)) return 0u;
    if (t >= 4294967295.0) return 4294967295u;
    return (uint32_t)floor(t);
}

// One particle's inputs side by side, so that the gather after the sort
// reads one 32-byte record per particle instead of four scattered words.
struct alignas(32) Particle4 {
    double x, y, m, s;
};

__global__ __launch_bounds__(kBlock) void k_morton(const double* __restrict__ x, const double* __restrict__ y,
                                                  const double* __restrict__ m, const double* __restrict__ s,
                                                  int64_t n, const BuildSync* __restrict__ sync,
                                                  uint64_t* __restrict__ key, uint32_t* __restrict__ val,
                                                  Particle4* __restrict__ packed)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i];
    const uint32_t qx = quantise(xi, sync->x0, sync->scale);
    const uint32_t qy = quantise(yi, sync->y0, sync->scale);
    key[i] = spread_bits(qx) | (spread_bits(qy) << 1);
    val[i] = (uint32_t)i;
    packed[i] = Particle4{xi, yi, m[i], s ? s[i] : 0.0};
}

__global__ __launch_bounds__(kBlock) void k_gather(const uint32_t* __restrict__ perm,
                                                  const Particle4* __restrict__ packed, int64_t n,
                                                  double* __restrict__ xs, double* __restrict__ ys,
                                                  double* __restrict__ ms, double* __restrict__ ss)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const Particle4 p = packed[perm[k]];
    xs[k] = p.x;
    ys[k] = p.y;
    ms[k] = p.m;
    ss[k] = p.s;
}

// --------------------------------------------------------------- topology

// Per Morton position i: number of boxes whose range starts at i.  A box at
// level l >= 1 exists iff its parent holds more than L particles (every
// ancestor then does too); the boxes starting at i form a chain from the
// shallowest new level down to the first leaf.  With ls(j) = level_start(j)
// (the shallowest level at which the box of particle j differs from that of
// particle j - 1; positions 0 and n count as level 0), the box (i, l) ends
// at the first j > i with ls(j) <= l, so:
//  - (i, l) is a leaf iff some j in (i, i + L] has ls(j) <= l (or l is the
//    deepest level);
//  - the parent of (i, ls(i)) holds at most L particles only if it starts in
//    [i - L, i) and ends in (i, i + L].
// A window of L positions on either side of i decides both; the block keeps
// ls over its window in LDS.
// After the sort on the keys' top digits: the runs of keys equal in those
// digits ordered by the whole key, from (Ki, Vi) into (Ko, Vo), with the
// values also into perm.  Thread i finds its run (a scan of at most kTieRun
// keys each way) and its rank in it by (key, position), so equal keys keep
// their order.  Runs longer than kTieRun keep their order: they hold more than
// L particles, which the topology count flags.
__global__ __launch_bounds__(kBlock) void k_order_ties(const uint64_t* __restrict__ Ki, const uint32_t* __restrict__ Vi,
                                                       uint64_t* __restrict__ Ko, uint32_t* __restrict__ Vo,
                                                       uint32_t* __restrict__ perm, int n)
{
    constexpr int sh = 64 - 2 * kTopLevel;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = Ki[i];
    const uint64_t top = key >> sh;
    int b = i, e = i + 1;
    while (b > 0 && i - b < kTieRun && (Ki[b - 1] >> sh) == top) --b;
    while (e < n && e - i <= kTieRun && (Ki[e] >> sh) == top) ++e;
    int pos = i;
    // every thread of a run of at most kTieRun keys sees all of it; a longer
    // run is seen as longer by each of its threads, so all of them keep their place
    const bool long_run = e - b > kTieRun || (b > 0 && (Ki[b - 1] >> sh) == top) || (e < n && (Ki[e] >> sh) == top);
    if (e - b > 1 && !long_run) {
        pos = b;
        for (int j = b; j < e; ++j) {
            const uint64_t kj = Ki[j];
            pos += (kj < key || (kj == key && j < i)) ? 1 : 0;
        }
    }
    const uint32_t v = Vi[i];
    Ko[pos] = key;
    Vo[pos] = v;
    perm[pos] = v;
}

__global__ __launch_bounds__(kBlock) void k_topo_count(const uint64_t* __restrict__ K, int n, int L,
                                                      int32_t* __restrict__ cnt, int8_t* __restrict__ lstart,
                                                      BuildSync* __restrict__ sync, int check)
{
    __shared__ int32_t hist[kMaxLevel + 1];
    __shared__ int8_t lsw[kBlock + 2 * kMaxLeafSize + 1]; // ls(j) for j in [base - L, base + kBlock + L]
    if (threadIdx.x <= kMaxLevel) hist[threadIdx.x] = 0;
    const int base = blockIdx.x * kBlock, w0 = base - L, wn = kBlock + 2 * L + 1;
    for (int t = threadIdx.x; t < wn; t += kBlock) {
        const int j = w0 + t;
        lsw[t] = (int8_t)((j <= 0 || j >= n) ? 0 : level_start(K, j));
    }
    __syncthreads();
    const int i = base + threadIdx.x;
    if (i < n) {
        const int ls = lsw[i - w0];
        lstart[i] = (int8_t)ls;
        int c = 0;
        if (ls <= kMaxLevel) {
            bool exists = true;
            if (ls > 0) {
                int lo = -1, hi = -1; // the parent's range, if it lies within the window
                for (int j = i - 1; j >= i - L && j >= 0; --j)
                    if (lsw[j - w0] <= ls - 1) {
                        lo = j;
                        break;
                    }
                for (int j = i + 1; j <= i + L && j <= n; ++j)
                    if (lsw[j - w0] <= ls - 1) {
                        hi = j;
                        break;
                    }
                exists = lo < 0 || hi < 0 || hi - lo > L;
            }
            if (exists) {
                int mL = kMaxLevel + 1;
                for (int j = i + 1; j <= i + L && j <= n; ++j) mL = min(mL, (int)lsw[j - w0]);
                const int last = min(max(ls, mL), kMaxLevel); // level of the chain's leaf
                c = last - ls + 1;
                for (int l = ls; l <= last; ++l) atomicAdd(&hist[l], 1);
            }
        }
        cnt[i] = c;
    }
    // check: is there a box below level kTopLevel, i.e. L + 1 consecutive
    // keys sharing their top 2 kTopLevel bits?  (After the sort on the top
    // digits only, the counts above hold unless there is.)
    const bool full = check && i + L < n &&
                      (K[i] >> (64 - 2 * kTopLevel)) == (K[i + L] >> (64 - 2 * kTopLevel));
    if (__syncthreads_or(full) && threadIdx.x == 0) atomicOr(&sync->deep, 1);
    if (threadIdx.x <= kMaxLevel && hist[threadIdx.x])
        atomicAdd(&sync->levrep[blockIdx.x % kLevReps][threadIdx.x], hist[threadIdx.x]);
}

// The box total, and the boxes per level summed over their copies (thread l:
// level l).
__global__ void k_sync_counts(const int32_t* __restrict__ cs, int n, BuildSync* __restrict__ sync)
{
    const int l = threadIdx.x;
    if (l == 0) sync->ncells = cs[n];
    if (l <= kMaxLevel) {
        int sum = 0;
#pragma unroll
        for (int r = 0; r < kLevReps; ++r) sum += sync->levrep[r][l];
        sync->levcnt[l] = sum;
    }
}

// One thread per box: the particle whose chain holds box idx is the i with
// cs[i] <= idx < cs[i + 1] (cs = exclusive scan of the per-particle counts);
// the box's level is ls(i) + (idx - cs[i]) and its end a binary search over
// the sorted keys.
__global__ __launch_bounds__(kBlock) void k_topo_emit(const uint64_t* __restrict__ K, int n, int ncells,
                                                     const int32_t* __restrict__ cs, const int8_t* __restrict__ lstart,
                                                     BoxArrays b, BuildSync* __restrict__ sync, LevelTable lt,
                                                     int32_t* __restrict__ levidx)
{
    __shared__ int32_t lcnt[kMaxLevel + 1], lbase[kMaxLevel + 1];
    __shared__ int32_t s_leaves, s_maxl;
    if (threadIdx.x <= kMaxLevel) lcnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        s_leaves = 0;
        s_maxl = 0;
    }
    __syncthreads();
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    int i = 0, l = 0;
    bool leaf = false;
    if (idx < ncells) {
        int lo = 0, hi = n; // largest i in [0, n) with cs[i] <= idx
        while (hi - lo > 1) {
            const int mid = lo + ((hi - lo) >> 1);
            if (cs[mid] <= idx) lo = mid;
            else hi = mid;
        }
        i = lo;
        const int k = idx - cs[i];
        l = lstart[i] + k;
        leaf = idx == cs[i + 1] - 1;
        atomicAdd(&lcnt[l], 1);
    }
    __syncthreads();
    if (threadIdx.x <= kMaxLevel) {
        lbase[threadIdx.x] = lcnt[threadIdx.x] ? atomicAdd(&sync->levfill[threadIdx.x], lcnt[threadIdx.x]) : 0;
        lcnt[threadIdx.x] = 0;
    }
    __syncthreads();
    if (idx < ncells) {
        const uint64_t Ki = K[i];
        const int end = l == 0 ? n : upper_prefix(K, i, n, prefix_at(Ki, l), l);
        const uint32_t qx = compact_bits(Ki), qy = compact_bits(Ki >> 1);
        b.beg[idx] = i;
        b.end[idx] = end;
        b.level[idx] = l;
        b.next[idx] = cs[end];
        b.leaf[idx] = leaf ? 1 : 0;
        b.ix[idx] = l == 0 ? 0u : (uint32_t)((uint64_t)qx >> (32 - l));
        b.iy[idx] = l == 0 ? 0u : (uint32_t)((uint64_t)qy >> (32 - l));
        b.lbeg[idx] = 0;
        b.lend[idx] = 0;
        const int slot = lbase[l] + atomicAdd(&lcnt[l], 1);
        if (slot < lt.cnt[l]) levidx[lt.off[l] + slot] = idx;
        else atomicOr(&sync->internal, 4);
        if (leaf) {
            atomicAdd(&s_leaves, 1);
            atomicMax(&s_maxl, l);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_leaves) atomicAdd(&sync->nleaves, s_leaves);
        atomicMax(&sync->max_level, s_maxl);
    }
}

// Each particle's leaf, and each internal box's children (preorder: c + 1,
// then each child's next, up to the box's own next; -1 past the last child).
__global__ __launch_bounds__(kBlock) void k_leaf_of(BoxArrays b, int ncells, int32_t* __restrict__ leaf_of,
                                                    int32_t* __restrict__ kids)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncells) return;
    if (b.leaf[c]) {
        for (int j = b.beg[c]; j < b.end[c]; ++j) leaf_of[j] = c;
        return;
    }
    const int cend = b.next[c];
    int ch = c + 1;
    for (int u = 0; u < 4; ++u) {
        const bool has = ch < cend;
        kids[4 * (size_t)c + u] = has ? ch : -1;
        if (has) {
            const int nx = b.next[ch];
            ch = nx > ch ? nx : ch + 1;
        }
    }
}

// Big-particle lists (Sec. 3.2): a smoothed particle of support radius
// supp * s (q s for a Gaussian, the size s for an NFW halo) is listed in the
// highest box where the support exceeds side / 2, provided that box is not
// below the particle's leaf.  Key = box index (kUnlisted otherwise).
__global__ __launch_bounds__(kBlock) void k_list_assign(const uint64_t* __restrict__ K, int n, const double* __restrict__ ss,
                                                       double supp, BuildSync* __restrict__ sync, int ncells,
                                                       const int32_t* __restrict__ leaf_of, BoxArrays b,
                                                       const int32_t* __restrict__ cs, const int8_t* __restrict__ lstart,
                                                       uint32_t unlisted, uint32_t* __restrict__ lkey,
                                                       uint32_t* __restrict__ lval)
{
#pragma clang fp contract(off)
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    uint32_t key = unlisted;
    const double sj = ss[j];
    if (sj > 0.0) {
        const double qs = supp * sj;
        int l = 0;
        while (l <= kMaxLevel && !(qs > ldexp(sync->side, -(l + 1)))) ++l;
        const int lf = leaf_of[j];
        if (lf < 0 || lf >= ncells) {
            atomicOr(&sync->internal, 1);
        } else if (l <= kMaxLevel && l <= b.level[lf]) {
            const int bb = l == 0 ? 0 : lower_prefix(K, 0, j, prefix_at(K[j], l), l);
            const int cell = cs[bb] + (l - lstart[bb]);
            if (cell >= 0 && cell < ncells) key = (uint32_t)cell;
            else atomicOr(&sync->internal, 2);
        }
    }
    lkey[j] = key;
    lval[j] = (uint32_t)j;
}

// Walk record of one particle of the tree's kind.  q: the Gaussian cutoff or
// the halo concentration; norm: 1 / C for Gaussians, 1 / g(c) for halos.
__device__ inline void fill_rec(PRec& r, double x, double y, double m, double s, int kind, double q, double norm,
                                bool listed, uint32_t pos)
{
#pragma clang fp contract(off)
    const double qs = kind == kKindNfw ? s : q * s;
    r.x = x;
    r.y = y;
    r.qs2 = s > 0.0 ? qs * qs : 0.0;
    r.m = (float)m;
    r.mC = (float)(m * norm);
    r.h = s > 0.0 ? (float)(kind == kKindNfw ? q / s : 1.0 / (2.0 * s * s)) : 0.0f;
    r.meta = pos | (listed ? 0x80000000u : 0u);
}

__global__ __launch_bounds__(kBlock) void k_particle_records(int n, const double* __restrict__ xs,
                                                            const double* __restrict__ ys, const double* __restrict__ ms,
                                                            const double* __restrict__ ss,
                                                            const uint32_t* __restrict__ lkey, uint32_t unlisted,
                                                            int kind, double q, double norm, PRec* __restrict__ prt)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    PRec r;
    fill_rec(r, xs[j], ys[j], ms[j], ss[j], kind, q, norm, lkey[j] != unlisted, (uint32_t)j);
    prt[j] = r;
}

__global__ __launch_bounds__(kBlock) void k_list_ranges(int n, const uint32_t* __restrict__ lkey,
                                                       const uint32_t* __restrict__ lval, uint32_t unlisted,
                                                       const double* __restrict__ xs, const double* __restrict__ ys,
                                                       const double* __restrict__ ms, const double* __restrict__ ss,
                                                       int kind, double q, double norm,
                                                       BoxArrays b, PRec* __restrict__ lst,
                                                       BuildSync* __restrict__ sync)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const uint32_t key = lkey[k];
    if (key == unlisted) return;
    if (k == 0 || lkey[k - 1] != key) b.lbeg[key] = k;
    const bool last = (k == n - 1) || lkey[k + 1] != key;
    if (last) b.lend[key] = k + 1;
    if (k == n - 1 || lkey[k + 1] == unlisted) sync->nlisted = k + 1;
    const uint32_t j = lval[k];
    PRec r;
    fill_rec(r, xs[j], ys[j], ms[j], ss[j], kind, q, norm, true, j);
    lst[k] = r;
}

// Reach of each box's big-particle list: the bounding box of its particles'
// supports, widened by far more than the rounding of any distance test, so
// that a ray group whose bounding box misses it cannot be inside any of them.
// One wavefront per box: the lanes stride over the list (coalesced records)
// and a min/max reduction across the wavefront ends it.
__global__ __launch_bounds__(kBlock) void k_list_reach(BoxArrays b, int ncells, const PRec* __restrict__ lst,
                                                      double* __restrict__ lreach)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int c = blockIdx.x * (kBlock / kWave) + (int)(threadIdx.x / kWave);
    if (c >= ncells) return; // uniform across the wavefront
    const int lb = b.lbeg[c], le = b.lend[c];
    if (lb >= le) return; // no list: the walk never reads this box's reach
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int k = lb + lane; k < le; k += kWave) {
        const PRec pr = lst[k];
        const double r = sqrt(pr.qs2) * (1.0 + 4e-9);
        const double mx = r + 4.5e-16 * fabs(pr.x), my = r + 4.5e-16 * fabs(pr.y);
        x0 = fmin(x0, pr.x - mx);
        x1 = fmax(x1, pr.x + mx);
        y0 = fmin(y0, pr.y - my);
        y1 = fmax(y1, pr.y + my);
    }
    x0 = wave_min(x0);
    x1 = wave_max(x1);
    y0 = wave_min(y0);
    y1 = wave_max(y1);
    if (lane < 4) lreach[4 * (size_t)c + lane] = lane == 0 ? x0 : lane == 1 ? x1 : lane == 2 ? y0 : y1;
}

// ---------------------------------------------------------------- moments

// Binomial coefficient C(n, k) (exact in FP64 for n <= 12); folds to a
// constant inside the unrolled moment loops.
__host__ __device__ constexpr double binomial(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

__device__ inline void box_bounds(const BoxArrays& b, int c, const BuildSync* sync, double* bx0, double* bx1,
                                  double* by0, double* by1)
{
#pragma clang fp contract(off)
    const double side = ldexp(sync->side, -b.level[c]);
    *bx0 = sync->x0 + (double)b.ix[c] * side;
    *bx1 = sync->x0 + ((double)b.ix[c] + 1.0) * side;
    *by0 = sync->y0 + (double)b.iy[c] * side;
    *by1 = sync->y0 + ((double)b.iy[c] + 1.0) * side;
}

// Sum of v over an aligned group of G lanes (G a power of two, at most the
// wavefront) by butterfly exchanges; a + b == b + a in IEEE arithmetic, so
// every lane of the group ends with the same bits.
template <int G>
__device__ inline double group_sum(double v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// Store the moments Q_0 .. Q_P of box c (identical in every lane of a group of
// G lanes): lane u writes the words u, u + G, ... of the box's record.
template <int P, int G>
__device__ inline void store_moments(int c, int u, const double* Qr, const double* Qi, double* __restrict__ cQ)
{
    double* q = cQ + (size_t)c * (P + 1) * 2;
#pragma unroll
    for (int k = 0; k <= P; ++k) {
        if ((2 * k) % G == u) q[2 * k] = Qr[k];
        if ((2 * k + 1) % G == u) q[2 * k + 1] = Qi[k];
    }
}

// Leaf moments (Sec. 3.2) about the leaf's centre of mass, Q_k = sum m (z - z_cm)^k,
// for every leaf at once (they depend on no other box): kLeafLanes lanes per
// box, lane u summing the leaf's particles u, u + kLeafLanes, ...; the lanes'
// partial sums meet by butterfly exchanges.
constexpr int kLeafLanes = 4;

template <int P>
__global__ __launch_bounds__(kBlock) void k_moments_leaves(int ncells, BoxArrays b, const double* __restrict__ xs,
                                                          const double* __restrict__ ys, const double* __restrict__ ms,
                                                          const BuildSync* __restrict__ sync, double* __restrict__ cM,
                                                          double* __restrict__ ccx, double* __restrict__ ccy,
                                                          double* __restrict__ cQ)
{
    constexpr int P1 = P + 1;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int c = (int)(gid / kLeafLanes), u = (int)(gid % kLeafLanes);
    // a group's lanes share c, so whole groups leave together
    if (c >= ncells || !b.leaf[c]) return;
    const int j0 = b.beg[c], j1 = b.end[c];
    double M = 0.0, sx = 0.0, sy = 0.0;
    for (int j = j0 + u; j < j1; j += kLeafLanes) {
        const double mm = ms[j];
        M += mm;
        sx += mm * xs[j];
        sy += mm * ys[j];
    }
    M = group_sum<kLeafLanes>(M);
    sx = group_sum<kLeafLanes>(sx);
    sy = group_sum<kLeafLanes>(sy);
    double cx, cy;
    if (M > 0.0) {
        cx = sx / M;
        cy = sy / M;
    } else {
        double bx0, bx1, by0, by1;
        box_bounds(b, c, sync, &bx0, &bx1, &by0, &by1);
        cx = 0.5 * (bx0 + bx1);
        cy = 0.5 * (by0 + by1);
    }
    double Qr[P1], Qi[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) Qr[k] = Qi[k] = 0.0;
    for (int j = j0 + u; j < j1; j += kLeafLanes) {
        const double dr = xs[j] - cx, di = ys[j] - cy;
        double pr = ms[j], pi = 0.0;
#pragma unroll
        for (int k = 0; k < P1; ++k) {
            Qr[k] += pr;
            Qi[k] += pi;
            const double t = pr * dr - pi * di;
            pi = pr * di + pi * dr;
            pr = t;
        }
    }
#pragma unroll
    for (int k = 0; k < P1; ++k) {
        Qr[k] = group_sum<kLeafLanes>(Qr[k]);
        Qi[k] = group_sum<kLeafLanes>(Qi[k]);
    }
    if (u == 0) {
        cM[c] = M;
        ccx[c] = cx;
        ccy[c] = cy;
    }
    store_moments<P, kLeafLanes>(c, u, Qr, Qi, cQ);
}

// An internal box c from its (at most four) children, lane u of an aligned
// group of four holding child u: the centre of mass of the children, then each
// child's moments translated, Q_k = sum_children sum_j C(k, j) Q_j(child) t^(k-j)
// with t = z_child - z_cm (the exact re-expansion of sum m (z - z_cm)^k).  All
// four lanes load their child's records together.
template <int P>
__device__ inline void moments_internal(int c, int u, const BoxArrays& b, const int32_t* __restrict__ kids,
                                        const BuildSync* __restrict__ sync, double* __restrict__ cM,
                                        double* __restrict__ ccx, double* __restrict__ ccy, double* __restrict__ cQ)
{
    constexpr int P1 = P + 1;
    const int ch = kids[4 * (size_t)c + u];
    const bool has = ch >= 0;
    const int cc = has ? ch : c; // an in-bounds index for the loads of an absent child
    double qr[P1], qi[P1];
    const double* q = cQ + (size_t)cc * P1 * 2;
#pragma unroll
    for (int k = 0; k < P1; ++k) {
        qr[k] = q[2 * k];
        qi[k] = q[2 * k + 1];
    }
    const double m = has ? cM[cc] : 0.0, x = ccx[cc], y = ccy[cc];
    const double M = group_sum<4>(m), sx = group_sum<4>(has ? m * x : 0.0), sy = group_sum<4>(has ? m * y : 0.0);
    double cx, cy;
    if (M > 0.0) {
        cx = sx / M;
        cy = sy / M;
    } else {
        double bx0, bx1, by0, by1;
        box_bounds(b, c, sync, &bx0, &bx1, &by0, &by1);
        cx = 0.5 * (bx0 + bx1);
        cy = 0.5 * (by0 + by1);
    }
    const double tr = x - cx, ti = y - cy;
    double tpr[P1], tpi[P1];
    tpr[0] = 1.0;
    tpi[0] = 0.0;
#pragma unroll
    for (int k = 1; k < P1; ++k) {
        tpr[k] = tpr[k - 1] * tr - tpi[k - 1] * ti;
        tpi[k] = tpr[k - 1] * ti + tpi[k - 1] * tr;
    }
    double Qr[P1], Qi[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int j = 0; j <= k; ++j) {
            const double br = binomial(k, j) * qr[j], bi = binomial(k, j) * qi[j];
            sr += br * tpr[k - j] - bi * tpi[k - j];
            si += br * tpi[k - j] + bi * tpr[k - j];
        }
        Qr[k] = group_sum<4>(has ? sr : 0.0);
        Qi[k] = group_sum<4>(has ? si : 0.0);
    }
    if (u == 0) {
        cM[c] = M;
        ccx[c] = cx;
        ccy[c] = cy;
    }
    store_moments<P, 4>(c, u, Qr, Qi, cQ);
}

// The internal boxes of one level, four lanes per box (its leaves are done).
template <int P>
__global__ __launch_bounds__(kBlock) void k_moments_level(const int32_t* __restrict__ levidx, int count, BoxArrays b,
                                                         const int32_t* __restrict__ kids,
                                                         const BuildSync* __restrict__ sync, double* __restrict__ cM,
                                                         double* __restrict__ ccx, double* __restrict__ ccy,
                                                         double* __restrict__ cQ)
{
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int t = (int)(gid >> 2), u = (int)(gid & 3);
    if (t >= count) return;
    const int c = levidx[t];
    if (b.leaf[c]) return;
    moments_internal<P>(c, u, b, kids, sync, cM, ccx, ccy, cQ);
}

// Levels ltop .. 0 (each with at most kBlock boxes) in one block of
// kTopThreads = 4 kBlock lanes, deepest first; the barrier between levels
// makes a level's results visible to its parents' lanes.
constexpr int kTopThreads = 4 * kBlock;

template <int P>
__global__ __launch_bounds__(kTopThreads) void k_moments_top(const int32_t* __restrict__ levidx, LevelTable lt, int ltop,
                                                            BoxArrays b, const int32_t* __restrict__ kids,
                                                            const BuildSync* __restrict__ sync, double* __restrict__ cM,
                                                            double* __restrict__ ccx, double* __restrict__ ccy,
                                                            double* __restrict__ cQ)
{
    const int t = (int)threadIdx.x >> 2, u = (int)threadIdx.x & 3;
    for (int l = ltop; l >= 0; --l) {
        if (t < lt.cnt[l]) {
            const int c = levidx[lt.off[l] + t];
            if (!b.leaf[c]) moments_internal<P>(c, u, b, kids, sync, cM, ccx, ccy, cQ);
        }
        __syncthreads();
    }
}

// Opening radius and the FP32 walk records.
__global__ __launch_bounds__(kBlock) void k_finalize(int ncells, int p, double theta, BoxArrays b,
                                                    const BuildSync* __restrict__ sync, const double* __restrict__ cM,
                                                    const double* __restrict__ ccx, const double* __restrict__ ccy,
                                                    const double* __restrict__ cQ, CellHdr* __restrict__ hdr,
                                                    CellExt* __restrict__ ext, float* __restrict__ mom)
{
#pragma clang fp contract(off)
    __shared__ double s_irc[kBlock]; // 1 / r_cm of the block's boxes
    const int c0 = blockIdx.x * kBlock, c = c0 + threadIdx.x;
    const int st = mom_stride(p);
    if (c < ncells) {
        double bx0, bx1, by0, by1;
        box_bounds(b, c, sync, &bx0, &bx1, &by0, &by1);
        const double cx = ccx[c], cy = ccy[c];
        const double X[4] = {bx0, bx1, bx0, bx1}, Y[4] = {by0, by0, by1, by1};
        double dmax2 = 0.0;
        for (int k = 0; k < 4; ++k) {
            const double e1 = X[k] - cx, e2 = Y[k] - cy;
            const double d2 = e1 * e1 + e2 * e2;
            if (d2 > dmax2) dmax2 = d2;
        }
        CellHdr h;
        h.cx = cx;
        h.cy = cy;
        h.rcut2 = theta > 0.0 ? dmax2 / (theta * theta) : INFINITY;
        h.next = b.next[c];
        h.info = (b.leaf[c] ? kInfoLeaf : 0u) | (b.lend[c] > b.lbeg[c] ? kInfoList : 0u);
        hdr[c] = h;
        CellExt e;
        e.pbeg = b.beg[c];
        e.pend = b.end[c];
        e.lbeg = b.lbeg[c];
        e.lend = b.lend[c];
        ext[c] = e;
        float* mo = mom + (size_t)c * st;
        const double rcm = sqrt(dmax2);
        mo[0] = (float)cM[c];
        mo[1] = (float)rcm;
        for (int k = 2 + 2 * (p > 1 ? p - 1 : 0); k < st; ++k) mo[k] = 0.0f;
        s_irc[threadIdx.x] = 1.0 / rcm;
    }
    __syncthreads();
    // M Qn_k = Q_k / r_cm^k for k = 2..p (Qn_k = Q_k / (M r_cm^k)): the walk's
    // series then carries the box mass in its coefficients.  One (box, k) item
    // per thread, so that the block reads its boxes' FP64 moments and writes
    // their FP32 records in consecutive words.
    const int per = p - 1, nb = ncells - c0 < kBlock ? ncells - c0 : kBlock;
    for (int i = threadIdx.x; i < nb * per; i += kBlock) {
        const int bi = i / per, k = 2 + i % per;
        const double irc = s_irc[bi];
        double scale = irc; // irc^k by the same k - 1 products for every k
        for (int j = 2; j <= k; ++j) scale *= irc;
        const double* q = cQ + (size_t)(c0 + bi) * (p + 1) * 2;
        float* mo = mom + (size_t)(c0 + bi) * st;
        mo[2 + 2 * (k - 2)] = (float)(q[2 * k] * scale);
        mo[3 + 2 * (k - 2)] = (float)(q[2 * k + 1] * scale);
    }
}

} // namespace

// ------------------------------------------------------------------- host

// Ein(z) = integral_0^z (1 - e^-t) / t dt by its power series (host).
static double ein_host(double z)
{
    double term = z, sum = 0.0;
    for (int k = 1; k < 400; ++k) {
        const double next = sum + term / (double)k;
        if (next == sum && k > 1) break;
        sum = next;
        term *= -z / (double)(k + 1);
    }
    return sum;
}

// Terms of the Ein series that reach FP64 accuracy on [0, U] (at most 100,
// which covers q up to about 7).
static int32_t ein_terms(double U)
{
    double term = U; // U^k / k!
    for (int k = 1; k < 100; ++k) {
        if (term / (double)k < 1e-17 && k > 2) return k;
        term *= U / (double)(k + 1);
    }
    return 100;
}

// Offsets of the per-particle part of a tree's workspace.
struct ParticleLayout {
    size_t sync, part, k0, k1, v0, v1, perm, hist, xs, ys, ms, ss, cnt, scr, ls, leafof, prt, lst, size;
};

constexpr int kBboxBlocks = 256;

static ParticleLayout particle_layout(int64_t n)
{
    ParticleLayout o;
    Arena pa;
    o.sync = pa.take(sizeof(BuildSync));
    o.part = pa.take(sizeof(double) * 5 * kBboxBlocks);
    o.k0 = pa.take(8ull * n);
    o.k1 = pa.take(8ull * n);
    o.v0 = pa.take(4ull * n);
    o.v1 = pa.take(4ull * n);
    o.perm = pa.take(4ull * n);
    o.hist = pa.take(4ull * radix_hist_words(n));
    o.xs = pa.take(8ull * n);
    o.ys = pa.take(8ull * n);
    o.ms = pa.take(8ull * n);
    o.ss = pa.take(8ull * n);
    o.cnt = pa.take(4ull * (n + 1));
    o.scr = pa.take(4ull * scan_scratch_words(n + 1));
    o.ls = pa.take((size_t)n);
    o.leafof = pa.take(4ull * n);
    o.prt = pa.take(sizeof(PRec) * (size_t)n);
    o.lst = pa.take(sizeof(PRec) * (size_t)n);
    o.size = pa.size;
    return o;
}

// Offsets of the per-box part (after the per-particle part).
struct BoxLayout {
    size_t beg, end, lev, next, leaf, ix, iy, lbeg, lend, M, cx, cy, Q, hdr, ext, mom, levidx, kids, lreach, size;
};

static BoxLayout box_layout(int64_t nc, int p)
{
    BoxLayout o;
    Arena ca;
    o.beg = ca.take(4ull * nc);
    o.end = ca.take(4ull * nc);
    o.lev = ca.take(4ull * nc);
    o.next = ca.take(4ull * nc);
    o.leaf = ca.take(4ull * nc);
    o.ix = ca.take(4ull * nc);
    o.iy = ca.take(4ull * nc);
    o.lbeg = ca.take(4ull * nc);
    o.lend = ca.take(4ull * nc);
    o.M = ca.take(8ull * nc);
    o.cx = ca.take(8ull * nc);
    o.cy = ca.take(8ull * nc);
    o.Q = ca.take(16ull * (p + 1) * nc);
    o.hdr = ca.take(sizeof(CellHdr) * (size_t)nc);
    o.ext = ca.take(sizeof(CellExt) * (size_t)nc);
    o.mom = ca.take(4ull * mom_stride(p) * nc);
    o.levidx = ca.take(4ull * nc);
    o.kids = ca.take(16ull * nc);
    o.lreach = ca.take(32ull * nc);
    o.size = ca.size;
    return o;
}

int64_t max_boxes(int64_t n, int L)
{
    const int64_t per_level = n / (L + 1);
    int64_t internal = 0, pow4 = 1;
    for (int l = 0; l < kMaxLevel; ++l) {
        internal += pow4 < per_level ? pow4 : per_level;
        if (pow4 < per_level) pow4 *= 4;
    }
    const int64_t a = n + internal, b = 4 * internal + 1;
    return a < b ? a : b;
}

size_t tree_particle_bytes(int64_t n) { return particle_layout(n).size; }
size_t tree_box_bytes(int64_t ncells, int order) { return box_layout(ncells, order).size; }

// Page-locked host blocks for the build's one read of its counts.  A copy into
// pageable memory passes through the runtime's staging buffer, which cost
// about 30 us per build at 1e6 particles.  A block serves one build at a time
// and returns to the pool afterwards; the pool holds as many blocks as builds
// ever ran at once and keeps them until the process ends, so a handle owns
// none and releasing it frees nothing.  Without a block (the page-locked
// allocation failed) the build reads into pageable memory instead.
namespace {
std::mutex g_pin_mu;
std::vector<BuildSync*> g_pin_free;

struct PinnedSync {
    BuildSync* p = nullptr;
    PinnedSync()
    {
        {
            std::lock_guard<std::mutex> lk(g_pin_mu);
            if (!g_pin_free.empty()) {
                p = g_pin_free.back();
                g_pin_free.pop_back();
                return;
            }
        }
        void* q = nullptr;
        if (hipHostMalloc(&q, sizeof(BuildSync), hipHostMallocDefault) == hipSuccess)
            p = static_cast<BuildSync*>(q);
        else
            (void)hipGetLastError();
    }
    ~PinnedSync()
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(g_pin_mu);
        try {
            g_pin_free.push_back(p);
        } catch (...) { // no room to keep it: the block stays allocated, unused
        }
    }
    PinnedSync(const PinnedSync&) = delete;
    PinnedSync& operator=(const PinnedSync&) = delete;
};
} // namespace

glm_status build_tree_device(TreeStorage& ts, const double* x, const double* y, const double* m, const double* s,
                             int64_t n64, const glm_params& prm, hipStream_t st)
{
    const int n = (int)n64;
    const int p = prm.order, L = prm.leaf_size;
    const double q = prm.q;
    const double invC = 1.0 / (-expm1(-0.5 * q * q));
    // particle kind: truncated Gaussians (support q s), or NFW halos of size s
    // and concentration q (support s, mass normalised by g(q))
    const int kind = (prm.flags & GLM_NFW_HALOS) ? kKindNfw : kKindGauss;
    const double supp = kind == kKindNfw ? 1.0 : q;
    const double norm = kind == kKindNfw ? 1.0 / nfw_g_at(q) : invC;

    // ---- per-particle part of the workspace
    const ParticleLayout pl = particle_layout(n);
    const int nbb = kBboxBlocks;
    ts.need = pl.size;
    if (pl.size > ts.ws_bytes)
        return fail(GLM_ENOMEM, "build_tree: workspace of " + std::to_string(ts.ws_bytes) +
                                    " bytes is smaller than the particle part (" + std::to_string(pl.size) + ")");
    char* P0 = ts.ws;
    BuildSync* sync = reinterpret_cast<BuildSync*>(P0 + pl.sync);
    double* part = reinterpret_cast<double*>(P0 + pl.part);
    uint64_t* k0 = reinterpret_cast<uint64_t*>(P0 + pl.k0);
    uint64_t* k1 = reinterpret_cast<uint64_t*>(P0 + pl.k1);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(P0 + pl.v0);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(P0 + pl.v1);
    uint32_t* perm = reinterpret_cast<uint32_t*>(P0 + pl.perm);
    uint32_t* hist = reinterpret_cast<uint32_t*>(P0 + pl.hist);
    double* xs = reinterpret_cast<double*>(P0 + pl.xs);
    double* ys = reinterpret_cast<double*>(P0 + pl.ys);
    double* ms = reinterpret_cast<double*>(P0 + pl.ms);
    double* ss = reinterpret_cast<double*>(P0 + pl.ss);
    int32_t* cnt = reinterpret_cast<int32_t*>(P0 + pl.cnt);
    int32_t* scr = reinterpret_cast<int32_t*>(P0 + pl.scr);
    int8_t* lstart = reinterpret_cast<int8_t*>(P0 + pl.ls);
    int32_t* leaf_of = reinterpret_cast<int32_t*>(P0 + pl.leafof);
    PRec* prt = reinterpret_cast<PRec*>(P0 + pl.prt);
    PRec* lst = reinterpret_cast<PRec*>(P0 + pl.lst);

    GLM_HIP(hipMemsetAsync(sync, 0, sizeof(BuildSync), st));
    const int gb = ceil_div(n, kBlock);
    hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(kBlock), 0, st, x, y, m, s, (int64_t)n, part);
    hipLaunchKernelGGL(k_root, dim3(1), dim3(kBlock), 0, st, part, nbb, sync);
    // the particle records' space holds the packed inputs until the records are made
    static_assert(sizeof(PRec) >= sizeof(Particle4), "packed inputs must fit the record array");
    Particle4* packed = reinterpret_cast<Particle4*>(prt);
    hipLaunchKernelGGL(k_morton, dim3(gb), dim3(kBlock), 0, st, x, y, m, s, (int64_t)n, sync, k0, v0, packed);
    // the keys' top digits, then the runs equal in them (see kTopDigits); all
    // 64 bits where a box below level kTopLevel exists.  Either way the
    // particles end in the full-key order.
    const bool full_first = ts.deep;
    int where = full_first ? radix_sort_u64(k0, v0, k1, v1, n, 8, hist, st)
                           : radix_sort_u64_digits(k0, v0, k1, v1, n, 8 - kTopDigits, kTopDigits, hist, st);
    uint64_t* K = where ? k1 : k0;
    uint32_t* pv = where ? v1 : v0;
    if (!full_first) { // the runs equal in the top digits, into the spare buffers (and perm)
        hipLaunchKernelGGL(k_order_ties, dim3(gb), dim3(kBlock), 0, st, K, pv, where ? k0 : k1, where ? v0 : v1,
                           perm, n);
        where = !where;
        K = where ? k1 : k0;
        pv = where ? v1 : v0;
    }
    BuildSync hs;
    PinnedSync pin;
    auto count_boxes = [&](bool copy_perm) -> glm_status {
        if (copy_perm) GLM_HIP(hipMemcpyAsync(perm, pv, 4ull * n, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_gather, dim3(gb), dim3(kBlock), 0, st, perm, packed, (int64_t)n, xs, ys, ms, ss);
        hipLaunchKernelGGL(k_topo_count, dim3(gb), dim3(kBlock), 0, st, K, n, L, cnt, lstart, sync, 1);
        exclusive_scan_i32(cnt, cnt, n, scr, st);
        hipLaunchKernelGGL(k_sync_counts, dim3(1), dim3(kWave), 0, st, cnt, n, sync);
        GLM_HIP(hipGetLastError());
        BuildSync* dst = pin.p ? pin.p : &hs;
        // the host needs the record up to the per-copy level counters
        hipError_t e = hipMemcpyAsync(dst, sync, offsetof(BuildSync, levrep), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            pin.p = nullptr; // a copy into it may still be pending: it leaves the pool
            return fail(GLM_EHIP, std::string("reading the box count failed: ") + hipGetErrorString(e));
        }
        if (pin.p) memcpy(&hs, pin.p, offsetof(BuildSync, levrep));
        return GLM_OK;
    };
    glm_status cst = count_boxes(full_first);
    if (cst != GLM_OK) return cst;
    if (hs.bad) return fail(GLM_EDATA, "build_tree: NaN/Inf value or negative mass/smoothing length");
    ts.deep = hs.deep != 0;
    if (hs.deep && !full_first) {
        // a box at level kTopLevel holds more than L particles: order on every
        // digit (a stable sort of the top-digit order gives the full-key order)
        // and count the boxes again
        const int w2 = radix_sort_u64(K, pv, where ? k0 : k1, where ? v0 : v1, n, 8, hist, st);
        if (w2) {
            K = where ? k0 : k1;
            pv = where ? v0 : v1;
            where = !where;
        }
        GLM_HIP(hipMemsetAsync(sync->levrep, 0, sizeof(sync->levrep), st));
        cst = count_boxes(true);
        if (cst != GLM_OK) return cst;
    }
    const int nc = hs.ncells;

    // ---- per-box part of the workspace, after the per-particle part
    const BoxLayout bl = box_layout(nc, p);
    ts.need = pl.size + bl.size;
    if (ts.need > ts.ws_bytes)
        return fail(GLM_ENOMEM, "build_tree: " + std::to_string(nc) + " boxes need a workspace of " +
                                    std::to_string(ts.need) + " bytes, got " + std::to_string(ts.ws_bytes));
    char* C0 = ts.ws + pl.size;
    BoxArrays b;
    b.beg = reinterpret_cast<int32_t*>(C0 + bl.beg);
    b.end = reinterpret_cast<int32_t*>(C0 + bl.end);
    b.level = reinterpret_cast<int32_t*>(C0 + bl.lev);
    b.next = reinterpret_cast<int32_t*>(C0 + bl.next);
    b.leaf = reinterpret_cast<int32_t*>(C0 + bl.leaf);
    b.ix = reinterpret_cast<uint32_t*>(C0 + bl.ix);
    b.iy = reinterpret_cast<uint32_t*>(C0 + bl.iy);
    b.lbeg = reinterpret_cast<int32_t*>(C0 + bl.lbeg);
    b.lend = reinterpret_cast<int32_t*>(C0 + bl.lend);
    double* cM = reinterpret_cast<double*>(C0 + bl.M);
    double* ccx = reinterpret_cast<double*>(C0 + bl.cx);
    double* ccy = reinterpret_cast<double*>(C0 + bl.cy);
    double* cQ = reinterpret_cast<double*>(C0 + bl.Q);
    CellHdr* hdr = reinterpret_cast<CellHdr*>(C0 + bl.hdr);
    CellExt* ext = reinterpret_cast<CellExt*>(C0 + bl.ext);
    float* mom = reinterpret_cast<float*>(C0 + bl.mom);
    int32_t* levidx = reinterpret_cast<int32_t*>(C0 + bl.levidx);
    int32_t* kids = reinterpret_cast<int32_t*>(C0 + bl.kids);
    double* lreach = reinterpret_cast<double*>(C0 + bl.lreach);
    LevelTable lt;
    {
        int off = 0;
        for (int l = 0; l <= kMaxLevel + 1; ++l) {
            lt.off[l] = off;
            lt.cnt[l] = l <= kMaxLevel ? hs.levcnt[l] : 0;
            off += lt.cnt[l];
        }
        if (off != nc) return fail(GLM_EHIP, "build_tree: per-level box counts disagree with the box total");
    }

    const int gc = ceil_div(nc, kBlock);
    hipLaunchKernelGGL(k_topo_emit, dim3(gc), dim3(kBlock), 0, st, K, n, nc, cnt, lstart, b, sync, lt, levidx);
    GLM_HIP(hipMemsetAsync(leaf_of, 0xff, 4ull * n, st)); // -1: no leaf (an internal error if it stays)
    hipLaunchKernelGGL(k_leaf_of, dim3(gc), dim3(kBlock), 0, st, b, nc, leaf_of, kids);
    // list keys: box index, or all-ones on the sorted bits for unlisted particles
    int passes = 1;
    while (passes < 4 && ((uint64_t)nc >= (1ull << (8 * passes)) - 1)) ++passes;
    const uint32_t unlisted = passes >= 4 ? kUnlisted32 : (uint32_t)((1ull << (8 * passes)) - 1);
    uint32_t* lk0 = reinterpret_cast<uint32_t*>(k1);        // reuse the spare key buffers
    uint32_t* lk1 = reinterpret_cast<uint32_t*>(k1) + n;
    uint32_t* lv0 = where ? v0 : v1;
    uint32_t* lv1 = reinterpret_cast<uint32_t*>(leaf_of);   // leaf_of is dead after assignment
    if (where) { // K lives in k1: use k0 as the spare
        lk0 = reinterpret_cast<uint32_t*>(k0);
        lk1 = reinterpret_cast<uint32_t*>(k0) + n;
    }
    hipLaunchKernelGGL(k_list_assign, dim3(gb), dim3(kBlock), 0, st, K, n, ss, supp, sync, nc, leaf_of, b, cnt,
                       lstart, unlisted, lk0, lv0);
    hipLaunchKernelGGL(k_particle_records, dim3(gb), dim3(kBlock), 0, st, n, xs, ys, ms, ss, lk0, unlisted, kind, q,
                       norm, prt);
    const int lw = radix_sort_u32(lk0, lv0, lk1, lv1, n, passes, hist, st);
    hipLaunchKernelGGL(k_list_ranges, dim3(gb), dim3(kBlock), 0, st, n, lw ? lk1 : lk0, lw ? lv1 : lv0, unlisted, xs,
                       ys, ms, ss, kind, q, norm, b, lst, sync);
    hipLaunchKernelGGL(k_list_reach, dim3(ceil_div(nc, kBlock / kWave)), dim3(kBlock), 0, st, b, nc, lst, lreach);
    // every leaf at once; then the internal boxes: the top levels, as long as
    // each holds at most kBlock boxes, in one block, the deeper ones in a
    // launch per level, deepest first
    {
        const dim3 g((unsigned)ceil_div((int64_t)nc * kLeafLanes, (int64_t)kBlock)), blk(kBlock);
#define GLM_CASE(PP)                                                                                                \
    case PP:                                                                                                        \
        hipLaunchKernelGGL((k_moments_leaves<PP>), g, blk, 0, st, nc, b, xs, ys, ms, sync, cM, ccx, ccy, cQ); \
        break;
        switch (p) {
            GLM_CASE(0) GLM_CASE(1) GLM_CASE(2) GLM_CASE(3) GLM_CASE(4) GLM_CASE(5) GLM_CASE(6)
            GLM_CASE(7) GLM_CASE(8) GLM_CASE(9) GLM_CASE(10) GLM_CASE(11) GLM_CASE(12)
            default: break;
        }
#undef GLM_CASE
    }
    int ltop = -1;
    while (ltop < kMaxLevel && lt.cnt[ltop + 1] <= kBlock) ++ltop;
    for (int l = kMaxLevel; l > ltop; --l)
        if (lt.cnt[l] > 0) {
            const dim3 g((unsigned)ceil_div(4 * (int64_t)lt.cnt[l], (int64_t)kBlock)), blk(kBlock);
#define GLM_CASE(PP)                                                                                          \
    case PP:                                                                                                  \
        hipLaunchKernelGGL((k_moments_level<PP>), g, blk, 0, st, levidx + lt.off[l], lt.cnt[l], b, kids, sync, \
                           cM, ccx, ccy, cQ);                                                                 \
        break;
            switch (p) {
                GLM_CASE(0) GLM_CASE(1) GLM_CASE(2) GLM_CASE(3) GLM_CASE(4) GLM_CASE(5) GLM_CASE(6)
                GLM_CASE(7) GLM_CASE(8) GLM_CASE(9) GLM_CASE(10) GLM_CASE(11) GLM_CASE(12)
                default: break;
            }
#undef GLM_CASE
        }
    if (ltop >= 0) {
#define GLM_CASE(PP)                                                                                            \
    case PP:                                                                                                    \
        hipLaunchKernelGGL((k_moments_top<PP>), dim3(1), dim3(kTopThreads), 0, st, levidx, lt, ltop, b, kids, sync, \
                           cM, ccx, ccy, cQ);                                                                   \
        break;
        switch (p) {
            GLM_CASE(0) GLM_CASE(1) GLM_CASE(2) GLM_CASE(3) GLM_CASE(4) GLM_CASE(5) GLM_CASE(6)
            GLM_CASE(7) GLM_CASE(8) GLM_CASE(9) GLM_CASE(10) GLM_CASE(11) GLM_CASE(12)
            default: break;
        }
#undef GLM_CASE
    }
    hipLaunchKernelGGL(k_finalize, dim3(gc), dim3(kBlock), 0, st, nc, p, prm.theta, b, sync, cM, ccx, ccy, cQ, hdr, ext,
                       mom);
    GLM_HIP(hipGetLastError());

    ts.n = n;
    ts.ncells = nc;
    ts.params = prm;
    ts.x0 = hs.x0;
    ts.y0 = hs.y0;
    ts.side = hs.side;
    ts.sync = sync;
    ts.b = b;
    ts.perm = reinterpret_cast<int32_t*>(perm);
    ts.key = K;
    ts.dev.hdr = hdr;
    ts.dev.ext = ext;
    ts.dev.mom = mom;
    ts.dev.prt = prt;
    ts.dev.lst = lst;
    ts.dev.cq = cQ;
    ts.dev.cM = cM;
    ts.dev.cbeg = b.beg;
    ts.dev.cend = b.end;
    ts.dev.perm = reinterpret_cast<int32_t*>(perm);
    ts.dev.kids = kids;
    ts.dev.lreach = lreach;
    ts.dev.ncells = nc;
    ts.dev.n = n;
    ts.dev.nlisted = -1; // read on demand (sync->nlisted)
    ts.dev.order = p;
    ts.dev.kind = kind;
    ts.dev.invC = (float)norm; // per-unit-mass normalisation: 1/C, or 1/g(c) for halos
    ts.dev.q = q;
    ts.dev.psiK = kind == kKindNfw ? nfw_H(q * q, (q - 1.0) * (q + 1.0)) : ein_host(0.5 * q * q);
    ts.dev.einTerms = ein_terms(0.5 * q * q);
    ts.ccx = ccx;
    ts.ms = ms;
    ts.ccy = ccy;
    ts.built = true;
    return GLM_OK;
}

} // namespace glm
