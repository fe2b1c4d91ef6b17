// Stable LSD radix sort (8-bit digits) and exclusive scan for gfx950.
//
// Sort pass = histogram per 2048-key tile -> per digit, an exclusive scan of
// its counts over the tiles (and the digit's total) -> scatter, where each
// tile takes its digit bases from the digit totals, ranks its keys stably
// with wave ballots (8 ballots give the lanes holding the same digit) and
// per-wave digit counts in LDS, reorders them by digit in LDS and writes each
// digit's run with consecutive lanes.  Loads and stores are coalesced.
#include "common.hpp"

namespace glm {

namespace {

constexpr int kItems = 8;                  // keys per thread per tile
constexpr int kTile = kBlock * kItems;     // 2048
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems; // 4096

__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan over the 256 threads of a block; returns the block total in *tot
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* lds_w, uint32_t* tot)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (lane == kWave - 1) lds_w[w] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) {
        const uint32_t x = lds_w[k];
        off += (k < w) ? x : 0u;
        all += x;
    }
    __syncthreads();
    *tot = all;
    return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t* in, int64_t n, uint32_t* part)
{
    __shared__ uint32_t lw[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if (i < n) s += (uint32_t)in[i];
    }
    uint32_t tot;
    block_excl_scan(s, lw, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single block: exclusive scan of nb partials, total into out[n]
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* part, int nb, int32_t* out, int64_t n)
{
    __shared__ uint32_t lw[1024 / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const int per = (nb + 1023) / 1024;
    const int b0 = t * per;
    uint32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) s += part[b0 + k];
    const uint32_t inc = wave_incl_scan(s, lane);
    if (lane == kWave - 1) lw[w] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
    for (int k = 0; k < 1024 / kWave; ++k) {
        off += (k < w) ? lw[k] : 0u;
        all += lw[k];
    }
    uint32_t run = off + inc - s;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) {
            const uint32_t x = part[b0 + k];
            part[b0 + k] = run;
            run += x;
        }
    if (t == 0) out[n] = (int32_t)all;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int32_t* in, int32_t* out, int64_t n,
                                                      const uint32_t* part)
{
    __shared__ uint32_t lw[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        v[j] = i < n ? (uint32_t)in[i] : 0u;
        s += v[j];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, lw, &tot) + part[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        if (i < n) out[i] = (int32_t)run;
        run += v[j];
    }
}

// Digit counts of one tile into hist[d * nb + tile].
template <class K>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const K* keys, int64_t n, int shift, uint32_t* hist,
                                                      int nb)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    // all of the thread's keys in flight together, then the counts
    K k[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        k[j] = i < n ? keys[i] : (K)0;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j)
        if (base + (int64_t)j * kBlock + threadIdx.x < n) atomicAdd(&h[(uint32_t)(k[j] >> shift) & 255u], 1u);
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// One block per digit d: exclusive scan of hist[d * nb .. d * nb + nb) over
// the tiles into pre[], and the digit's total into dtot[d].
__global__ __launch_bounds__(kBlock) void k_radix_rowscan(const uint32_t* __restrict__ hist, int nb,
                                                         uint32_t* __restrict__ pre, uint32_t* __restrict__ dtot)
{
    __shared__ uint32_t lw[kBlock / kWave];
    const int d = blockIdx.x, t = threadIdx.x;
    const int per = (nb + kBlock - 1) / kBlock;
    const int64_t row = (int64_t)d * nb;
    const int b0 = t * per;
    uint32_t sum = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) sum += hist[row + b0 + k];
    uint32_t tot;
    uint32_t run = block_excl_scan(sum, lw, &tot);
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) {
            const uint32_t c = hist[row + b0 + k];
            pre[row + b0 + k] = run;
            run += c;
        }
    if (t == 0) dtot[d] = tot;
}

// Scatter of one tile: the keys are ranked stably per digit (wave ballots and
// per-wave digit counts in LDS, chunk by chunk), placed in LDS in digit order,
// then written out slot by slot, so that consecutive lanes write consecutive
// addresses of the same digit's run.  The tile's run of digit d starts at
// (keys of digits below d) + pre[d * nb + tile] and holds hist[d * nb + tile] keys.
template <class K>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const K* kin, const uint32_t* vin, K* kout,
                                                         uint32_t* vout, int64_t n, int shift,
                                                         const uint32_t* __restrict__ hist,
                                                         const uint32_t* __restrict__ pre,
                                                         const uint32_t* __restrict__ dtot, int nb)
{
    __shared__ K sk[kTile];
    __shared__ uint32_t sv[kTile];
    __shared__ uint32_t lrun[256];  // next free tile slot of digit d
    __shared__ uint32_t gbase[256]; // global position of slot 0 for digit d's run
    __shared__ uint32_t wcnt[kBlock / kWave][256];
    __shared__ uint32_t lw[kBlock / kWave];
    const int t = threadIdx.x, w = t / kWave;
    // the thread's keys and values of the whole tile are loaded up front, so
    // their latency overlaps the digit bases' loads and is paid once per tile
    const int64_t base = (int64_t)blockIdx.x * kTile;
    K keys[kItems];
    uint32_t vals[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t i = base + (int64_t)j * kBlock + t;
        keys[j] = i < n ? kin[i] : (K)0;
        vals[j] = i < n ? vin[i] : 0u;
    }
    {
        const int64_t hi = (int64_t)t * nb + blockIdx.x;
        uint32_t tot;
        const uint32_t dbase = block_excl_scan(dtot[t], lw, &tot); // keys of the digits below t
        const uint32_t g0 = dbase + pre[hi];
        const uint32_t cnt = hist[hi];
        const uint32_t l0 = block_excl_scan(cnt, lw, &tot);
        lrun[t] = l0;
        gbase[t] = g0 - l0;
    }
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) wcnt[k][t] = 0;
    __syncthreads();
    const uint64_t lt = __lanemask_lt();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t i = base + (int64_t)j * kBlock + t;
        const bool valid = i < n;
        const K key = keys[j];
        const uint32_t val = vals[j];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            same &= bit ? bb : ~bb;
        }
        const uint32_t lrank = (uint32_t)__popcll(same & lt);
        if (valid && lrank == 0) wcnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = lrun[d] + lrank;
            for (int k = 0; k < w; ++k) pos += wcnt[k][d];
            sk[pos] = key;
            sv[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < kBlock / kWave; ++k) {
            add += wcnt[k][t];
            wcnt[k][t] = 0;
        }
        lrun[t] += add;
        __syncthreads();
    }
    const int m = (int)(n - base < (int64_t)kTile ? n - base : (int64_t)kTile);
    for (int q = t; q < m; q += kBlock) {
        const K key = sk[q];
        const uint32_t pos = gbase[(uint32_t)(key >> shift) & 255u] + (uint32_t)q;
        kout[pos] = key;
        vout[pos] = sv[q];
    }
}

template <class K>
int radix_sort_impl(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n, int first, int passes, uint32_t* hist,
                    hipStream_t s)
{
    if (n <= 1 || passes <= 0) return 0;
    const int nb = ceil_div(n, kTile);
    const int64_t hn = (int64_t)256 * nb;
    uint32_t* pre = hist + hn;
    uint32_t* dtot = pre + hn; // 256 digit totals
    K* ki = k0;
    uint32_t* vi = v0;
    K* ko = k1;
    uint32_t* vo = v1;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * (first + p);
        hipLaunchKernelGGL(k_radix_hist<K>, dim3(nb), dim3(kBlock), 0, s, ki, n, shift, hist, nb);
        hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kBlock), 0, s, hist, nb, pre, dtot);
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nb), dim3(kBlock), 0, s, ki, vi, ko, vo, n, shift, hist,
                           pre, dtot, nb);
        K* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    return (passes & 1) ? 1 : 0;
}

} // namespace

size_t scan_scratch_words(int64_t n) { return (size_t)ceil_div(n > 0 ? n : 1, kScanTile) + 1; }

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t s)
{
    const int nb = ceil_div(n > 0 ? n : 1, kScanTile);
    uint32_t* part = reinterpret_cast<uint32_t*>(scratch);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, part, nb, out, n);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0, s, in, out, n, part);
}

size_t radix_hist_words(int64_t n)
{
    const int64_t hn = (int64_t)256 * ceil_div(n > 0 ? n : 1, kTile);
    return 2 * (size_t)hn + 256; // counts, their per-digit prefixes, digit totals
}

int radix_sort_u64(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t n, int passes,
                   uint32_t* hist, hipStream_t s)
{
    return radix_sort_impl<uint64_t>(k0, v0, k1, v1, n, 0, passes, hist, s);
}

int radix_sort_u64_digits(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t n, int first, int passes,
                          uint32_t* hist, hipStream_t s)
{
    return radix_sort_impl<uint64_t>(k0, v0, k1, v1, n, first, passes, hist, s);
}

int radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int passes,
                   uint32_t* hist, hipStream_t s)
{
    return radix_sort_impl<uint32_t>(k0, v0, k1, v1, n, 0, passes, hist, s);
}

} // namespace glm
