// Internal declarations of the gfx950 tree ray-shooting library: device data
// layout of a built tree, launch helpers and error plumbing.  Not installed;
// the public interface is include/glamer.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "glamer.h"

namespace glm {

constexpr int kWave = 64;     // CDNA wavefront
constexpr int kBlock = 256;   // 4 waves per workgroup
constexpr int kMaxOrder = 12;
constexpr int kMaxLevel = 32; // 32-bit quantised coordinates per axis
constexpr int kMaxLeafSize = 64; // largest accepted leaf size L

// ---------------------------------------------------------------------------
// Walk-side records.  Box and particle records are read with wave-uniform
// (scalar) loads by every lane of a ray group, so they are AoS and aligned.
// ---------------------------------------------------------------------------

// 32 B: what the opening test needs.
struct alignas(32) CellHdr {
    double cx, cy;   // centre of mass (FP64)
    double rcut2;    // (r_cm / theta)^2, +inf when theta = 0
    int32_t next;    // preorder index one past the subtree
    uint32_t info;   // bit0 leaf, bit1 non-empty big-particle list
};

// 16 B: ranges into the leaf-particle and list arrays.
struct alignas(16) CellExt {
    int32_t pbeg, pend; // particles (Morton order) -- leaves only
    int32_t lbeg, lend; // big-particle list entries
};

// Particle kinds of a tree (one per tree): truncated Gaussians of Sec. 3.1,
// or truncated NFW halos (Sec. 3.2: a halo type with its own closed forms).
// Point masses (s = 0) go with either.
constexpr int kKindGauss = 0;
constexpr int kKindNfw = 1;

// 40 B: one particle as the walk evaluates it.
//   Gaussian: qs2 = (q s)^2, mC = m / (1 - exp(-q^2/2)), h = 1 / (2 s^2);
//   NFW halo of size R = s and concentration c: qs2 = R^2, mC = m / g(c),
//     h = c / R (the inverse scale radius);
//   point mass: qs2 = 0, h = 0.
struct alignas(8) PRec {
    double x, y;   // position (FP64)
    double qs2;    // squared support radius in FP64 (outside it the particle is a point mass)
    float m;       // mass
    float mC;      // mass scaled by the profile's normalisation
    float h;       // profile scale
    uint32_t meta; // Morton position of the particle | (listed in a big-particle list) << 31
};

constexpr uint32_t kInfoLeaf = 1u;
constexpr uint32_t kInfoList = 2u;

// Moment stride (floats) per box for order p: M, r_cm, then (Re, Im) of the
// normalised moments Q_k / (M r_cm^k) for k = 2..p, padded to 4 floats.
__host__ __device__ constexpr int mom_stride(int p) { return ((2 + 2 * (p > 1 ? p - 1 : 0)) + 3) & ~3; }

// Device view of a built tree (passed by value to kernels).
struct TreeDev {
    const CellHdr* hdr;
    const CellExt* ext;
    const float* mom;       // ncells * mom_stride(p)
    const PRec* prt;        // n, Morton order
    const PRec* lst;        // nlisted, grouped by box, Morton order inside a box
    const double* cq;       // FP64 moments about the centre of mass: ncells * (p+1) * 2
    const double* cM;       // FP64 box masses
    const int32_t* cbeg;    // box particle range (Morton order)
    const int32_t* cend;
    const int32_t* perm;    // Morton position -> original index
    const int32_t* kids;    // internal box c: its children at 4c .. 4c + 3 in preorder, -1 past the last
    const double* lreach;   // per box with a list: x0, x1, y0, y1 of the union of its list particles' supports
    int32_t ncells;
    int32_t n;
    int32_t nlisted;
    int32_t order;
    int32_t kind;           // kKindGauss or kKindNfw
    float invC;             // mass normalisation: 1 / (1 - exp(-q^2/2)), or 1 / g(c) for NFW halos
    int32_t einTerms;       // series terms of Ein on [0, q^2/2]
    double q;
    double psiK;            // potential constant: Ein(q^2/2) (Gaussians) or H(c) (NFW halos)
};

// Element i of tree data that no kernel writes while the reading kernel runs,
// at a wavefront-uniform index: read through the constant address space, so
// that it becomes a scalar load whatever else the kernel stores (LDS stores
// at computed addresses otherwise make the compiler fall back to vector loads).
// (Read as 32-bit words: a class type has no copy from that address space.)
template <class E>
__device__ __forceinline__ E uniform_ld(const E* p, int64_t i)
{
    static_assert(sizeof(E) % 4 == 0, "whole 32-bit words");
    using ConstW = const __attribute__((address_space(4))) uint32_t;
    ConstW* q = (ConstW*)(p + i); // an address-space conversion, which only a C-style cast spells
    struct Words {
        uint32_t w[sizeof(E) / 4];
    } v;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(E) / 4); ++k) v.w[k] = q[k];
    return __builtin_bit_cast(E, v);
}

// ---------------------------------------------------------------------------
// host-side error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
glm_status fail(glm_status st, const std::string& msg);

#define GLM_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::glm::fail(GLM_EHIP, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// radix sort and scans (sort.hip)
// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs on bits [0, 8*passes) with 8-bit
// digits.  Ping-pongs between (k0, v0) and (k1, v1); returns 0 if the result
// ends in (k0, v0), 1 if in (k1, v1).  hist needs radix_hist_words(n) words.
size_t radix_hist_words(int64_t n);
int radix_sort_u64(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t n, int passes,
                   uint32_t* hist, hipStream_t s);
int radix_sort_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int passes,
                   uint32_t* hist, hipStream_t s);
// Exclusive scan of n int32 values into out[0..n] (out[n] = total).  in and
// out may alias.  scratch needs scan_scratch_words(n) words.
size_t scan_scratch_words(int64_t n);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t s);

} // namespace glm
