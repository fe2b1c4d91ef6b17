// Adjoint of the forward tree walk: dL/d(m, x, y, s) of the particles for
// cotangents ga = dL/dalpha of the rays, and optionally gk = dL/dkappa and
// gg = dL/dgamma, on the frozen topology and decisions of the forward walk
// (the same traversal runs again and takes the same FP64 decisions).
//
// Direct terms (leaf particles, big-particle corrections) give particle
// gradients directly:
//   dL/dm_i = ga . alpha_i / m_i,  dL/dz_i = -J_i ga  (alpha depends on x - x_i,
//   J_i = [[k + g1, g2], [g2, k - g1]] of the single particle),
//   dL/ds_i = ga . d alpha_i / d s_i = -m (ga . d) e^-u / (s^3 C) inside.
// An accepted box contributes F = alpha1 - i alpha2 = sum_k Q_k w^-(k+1), so
// with g_hat = ga1 + i ga2 the walk accumulates per box
//   Abar_k r_cm^k = sum_r g_hat v t^k   (v = 1/w, t = r_cm v), k = 0 .. P + 1,
// and the centre-of-mass adjoint sum_r g_hat dF/dz_cm = sum_{k <= P} (k + 1) Q_k Abar_{k+1}
// follows from them in the push-down.  With kappa and gamma cotangents the
// walk keeps Abar_0 .. Abar_P and accumulates that adjoint directly:
//   Bbar          = sum_r g_hat M v^2 (P(t) + t P'(t))     (= g_hat dF/dz_cm)
// A gamma cotangent adds, with gg_hat = gg1 + i gg2 (gamma1 - i gamma2 = F'(w)),
//   Abar_k r_cm^k -= (k + 1) gg_hat v^2 t^k,   Bbar -= gg_hat F''(w) = gg_hat M v^3 T(t),
//   T(t) = sum (k+1)(k+2) Qn_k t^k;  kappa gets nothing from a box.
// Direct terms of a circular profile, with u = r^2, A = alpha / d, kappa(u):
//   gamma1 - i gamma2 = a conj(w)^2,  a = (kappa - A)/u,  b = u A'' = dkappa/du - 2a,
//   d kappa / d d_j = 2 (dkappa/du) d_j,
//   d gamma1/d d1 = 2 d1 (b c + a), d gamma1/d d2 = 2 d2 (b c - a),
//   d gamma2/d d1 = 2 d2 (b (1 + c) + a), d gamma2/d d2 = 2 d1 (b (1 - c) + a),  c = cos 2phi;
// for the Gaussian a = -m h^2 (Gam-series / x) (no cancellation at small x = h u),
// dkappa/du = -h kappa, d kappa/ds - dA/ds = m e^-x x / (C s^3).
// A push-down pass gives every particle its share through
//   dQ_k/dm_i = d^k - k Q_{k-1} d / M,  dQ_k/dz_i = k m_i d^(k-1) - k Q_{k-1} m_i / M,
//   dz_cm/dm_i = d / M,  dz_cm/dz_i = m_i / M  (d = z_i - z_cm; all holomorphic).
// Per-lane terms are reduced across the wavefront before one FP64 atomic per
// quantity; the point-mass parts of big-particle pairs are reduced in FP64 so
// that they cancel like the forward's balance.
#include <math.h>

#include "eval.hpp"
#include "walk.hpp"

namespace glm {

namespace {

// The wavefronts add their box adjoints into kAdjCopies copies (wavefront w
// into copy w % kAdjCopies), summed into copy 0 before the push-down: the boxes
// near the root are accepted by nearly every ray group, and with one copy their
// FP64 atomics all queued on the same few lines.
constexpr int kAdjCopies = 8;
// Likewise the per-particle direct-term sums, in kPgCopies copies that the
// push-down adds up.
constexpr int kPgCopies = 4;


// Cotangents of one ray: alpha (g1, g2), kappa (k), gamma (h1, h2).
struct Cot {
    float g1, g2, k, h1, h2;
};

// kappa and gamma part of a term's gradient, per unit mass (m, then d/d d1,
// d/d d2 of L, the s part separately): kap = kappa, Am = A = alpha / d,
// dk = dkappa/du, a = (kappa - A) / u.
__device__ inline void kg_grad(const Cot& cg, float f1, float f2, float ir2, float kap, float a, float dk, float* em,
                               float* e1, float* e2)
{
    const float c = (f1 * f1 - f2 * f2) * ir2, sn = 2.0f * f1 * f2 * ir2;
    const float b = dk - 2.0f * a;
    const float u = (f1 * f1 + f2 * f2);
    // gamma1 = a (d1^2 - d2^2) = a u c, gamma2 = a u sn
    *em = cg.k * kap + (cg.h1 * c + cg.h2 * sn) * (a * u);
    *e1 = 2.0f * (cg.k * dk * f1 + cg.h1 * f1 * fmaf(b, c, a) + cg.h2 * f2 * fmaf(b, 1.0f + c, a));
    *e2 = 2.0f * (cg.k * dk * f2 + cg.h1 * f2 * fmaf(b, c, -a) + cg.h2 * f1 * fmaf(b, 1.0f - c, a));
}

// Gradient terms of one particle for this lane, per the same cases as the
// forward's leaf_particle and list_particle.  Returns FP64 (m, x, y, s) contributions in G.
// mode 0: leaf sum; mode 1: big-particle correction (Gaussian - point).
template <bool KG, int KIND>
__device__ inline bool particle_grad(const PRec& pr, double X, double Y, int mode, bool act, const Cot& cg,
                                     float invC, double G[4])
{
    G[0] = G[1] = G[2] = G[3] = 0.0;
    if (!act) return false;
    const float g1 = cg.g1, g2 = cg.g2;
    double d1, d2;
    const double r2 = sqdist(X, Y, pr.x, pr.y, &d1, &d2);
    const bool inside = r2 < pr.qs2;
    const bool listed = (pr.meta >> 31) != 0;
    if (mode == 1 && !inside) return false;
    const float f1 = (float)d1, f2 = (float)d2, r2f = (float)r2;
    const float ir2 = r2f > 0.0f ? __builtin_amdgcn_rcpf(r2f) : 0.0f;
    const float gd = g1 * f1 + g2 * f2;
    // point mass, per unit mass: alpha = d / r^2, gamma = -(cos 2phi, sin 2phi) / r^2, kappa = 0
    float P[4];
    point_terms(1.0f, f1, f2, ir2, P);
    float pm_m = g1 * P[0] + g2 * P[1];
    float pm_x = -(g1 * P[2] + g2 * P[3]) * pr.m;
    float pm_y = -(g1 * P[3] - g2 * P[2]) * pr.m;
    if constexpr (KG) {
        // point mass: kappa = 0, A = 1/u, a = -1/u^2, dkappa/du = 0
        float km, k1, k2;
        kg_grad(cg, f1, f2, ir2, 0.0f, -(ir2 * ir2), 0.0f, &km, &k1, &k2);
        pm_m += km;
        pm_x -= k1 * pr.m;
        pm_y -= k2 * pr.m;
    }
    const bool gauss = inside && !(mode == 0 && listed);
    if (!gauss) { // point mass (a listed+inside point pairs with the list box's -point)
        G[0] = (double)pm_m;
        G[1] = (double)pm_x;
        G[2] = (double)pm_y;
        return true;
    }
    const float c2 = (f1 * f1 - f2 * f2) * ir2, s2 = 2.0f * f1 * f2 * ir2;
    if constexpr (KIND == kKindNfw) {
        // truncated NFW halo per unit mass (invC = 1/g(c), h = c/R): A = h^2 g/x^2 / g(c),
        // kappa = h^2 f / (2 g(c)); size derivatives of a scale family: d alpha/dR = -(2 kappa/R) d,
        // d kappa/dR = -2 (kappa + u dkappa/du)/R, d(kappa - A)/dR = -2 u dkappa/du / R
        const double x2 = r2 * ((double)pr.h * (double)pr.h);
        float gx2, f, dfde;
        nfw_shape32((float)x2, (float)(x2 - 1.0), &gx2, &f, &dfde);
        const float hh2 = (invC * pr.h) * pr.h;
        const float Au = hh2 * gx2;
        const float Ku = r2 > 0.0 ? 0.5f * hh2 * f : 0.0f;
        const float Gu = Au - Ku;
        const float iR = __builtin_amdgcn_rsqf((float)pr.qs2);
        const float ga1 = -Gu * c2, ga2 = -Gu * s2;
        float em = Au * gd;
        float ex = -(g1 * (Ku + ga1) + g2 * ga2) * pr.m;
        float ey = -(g1 * ga2 + g2 * (Ku - ga1)) * pr.m;
        float es = -pr.m * 2.0f * Ku * iR * gd;
        if constexpr (KG) {
            const float a = (Ku - Au) * ir2;
            const float dk = r2 > 0.0 ? 0.5f * hh2 * (pr.h * pr.h) * dfde : 0.0f;
            float km, k1, k2;
            kg_grad(cg, f1, f2, ir2, Ku, a, dk, &km, &k1, &k2);
            em += km;
            ex -= k1 * pr.m;
            ey -= k2 * pr.m;
            const float ks = -2.0f * (Ku + r2f * dk) * iR, gs = -2.0f * r2f * dk * iR;
            es += pr.m * (cg.k * ks + (cg.h1 * c2 + cg.h2 * s2) * gs);
        }
        if (mode == 1) {
            G[0] = (double)em - (double)pm_m;
            G[1] = (double)ex - (double)pm_x;
            G[2] = (double)ey - (double)pm_y;
        } else {
            G[0] = (double)em;
            G[1] = (double)ex;
            G[2] = (double)ey;
        }
        G[3] = (double)es;
        return true;
    }
    const float u = r2f * pr.h;
    const float e = __expf(-u);
    const float hu = invC * pr.h; // per unit mass m/C/(2 s^2)
    float Au, Gu;
    gauss_terms(u, e, ir2, invC, hu, &Au, &Gu);
    const float Ku = hu * e;
    const float ga1 = -Gu * c2, ga2 = -Gu * s2; // gamma per unit mass
    float em = Au * gd;
    float ex = -(g1 * (Ku + ga1) + g2 * ga2) * pr.m;
    float ey = -(g1 * ga2 + g2 * (Ku - ga1)) * pr.m;
    // d alpha / d s = -m d e^-u / (s^3 C), 1/s^3 = 2h sqrt(2h)
    float es = -pr.m * hu * e * 2.0f * __builtin_sqrtf(2.0f * pr.h) * gd;
    if constexpr (KG) {
        // a = -Gam / u with Gam = hu * sd(x), x = u_gauss: a = -hu * h * sd(x) / x
        float sdx;
        if (u < 0.5f) {
            sdx = 1.0f / 2 + u * (-1.0f / 3 + u * (1.0f / 8 + u * (-1.0f / 30 + u * (1.0f / 144 + u * (-1.0f / 840 + u * (1.0f / 5760 + u * (-1.0f / 45360 + u * (1.0f / 403200))))))));
        } else {
            const float iu = __builtin_amdgcn_rcpf(u);
            sdx = ((1.0f - e) * iu - e) * iu;
        }
        const float a = -hu * pr.h * sdx;
        const float dk = -pr.h * Ku;
        float km, k1, k2;
        kg_grad(cg, f1, f2, ir2, Ku, a, dk, &km, &k1, &k2);
        em += km;
        ex -= k1 * pr.m;
        ey -= k2 * pr.m;
        // d/ds: kappa_s and (kappa_s - A_s) = invC e x / s^3 (per unit mass)
        const float is3 = 2.0f * pr.h * __builtin_sqrtf(2.0f * pr.h);
        const float ks = invC * e * (u - 1.0f) * is3;
        const float gs = invC * e * u * is3;
        es += pr.m * (cg.k * ks + (cg.h1 * c2 + cg.h2 * s2) * gs);
    }
    if (mode == 1) {
        G[0] = (double)em - (double)pm_m;
        G[1] = (double)ex - (double)pm_x;
        G[2] = (double)ey - (double)pm_y;
    } else {
        G[0] = (double)em;
        G[1] = (double)ex;
        G[2] = (double)ey;
    }
    G[3] = (double)es;
    return true;
}

// Position of the c-th set bit (from 0) of m, for c < popcount(m).
__device__ inline int nth_set_bit(uint64_t m, int c)
{
    int pos = 0;
#pragma unroll
    for (int w = 32; w > 0; w >>= 1) {
        const int low = __popcll(m & ((1ull << w) - 1));
        if (c >= low) {
            c -= low;
            m >>= w;
            pos += w;
        }
    }
    return pos;
}

// Orders this wavefront's LDS accesses around a hand-over between its lanes
// (LDS operations of one wavefront complete in program order).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The rays of a wavefront that take part in a particle pass, packed in the
// wavefront's LDS slice: ray slot s (s < popcount(rays)) is the s-th set bit.
struct RayTable {
    double* x;
    double* y;
    float2* g;   // alpha cotangent
    float* k;    // kappa cotangent
    float2* h;   // gamma cotangent
};

__device__ inline RayTable ray_table(float* lds)
{
    RayTable t;
    t.x = reinterpret_cast<double*>(lds);
    t.y = t.x + kWave;
    t.g = reinterpret_cast<float2*>(t.y + kWave);
    t.k = reinterpret_cast<float*>(t.g + kWave);
    t.h = reinterpret_cast<float2*>(t.k + kWave);
    return t;
}
constexpr int kRayTableFloats = 2 * 2 * kWave + 2 * kWave + kWave + 2 * kWave; // 2304 bytes

// Gradient terms of the particles selected by `sel` (bit k: record rec[k])
// for the rays of the wavefront whose bit is set in `rays`, summed over those
// rays into the particles' four FP64 accumulators (m, x, y, s) at
// pg + 4 * (Morton position).  Lanes hold (particle, ray slot) pairs rather
// than rays: the taking-part rays are first packed into the wavefront's LDS
// slice (their positions and cotangents), then a pass takes up to 32
// particles, splits the lanes into G = 64 / count groups, and each lane sums
// its particle's terms over the ray slots g, g + G, ... of the packed table
// (so no pass is spent on rays that do not take part); the G partial sums
// then meet in the lanes of group 0, which add them with one atomic
// instruction per accumulator.
template <bool KG, int KIND>
__device__ inline void particles_grad(const PRec* __restrict__ rec, uint64_t sel, int mode, uint64_t rays, double X,
                                      double Y, const Cot& cg, float invC, double* __restrict__ pg, int lane,
                                      float* lds)
{
    const RayTable tab = ray_table(lds);
    const int nr = __popcll(rays);
    if ((rays >> lane) & 1ull) {
        const int slot = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(rays >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)rays, 0u));
        tab.x[slot] = X;
        tab.y[slot] = Y;
        tab.g[slot] = make_float2(cg.g1, cg.g2);
        if constexpr (KG) {
            tab.k[slot] = cg.k;
            tab.h[slot] = make_float2(cg.h1, cg.h2);
        }
    }
    wave_lds_sync();
    while (sel) {
        const int total = __popcll(sel);
        const int C = total < 32 ? total : 32; // particles in this pass
        const int G = kWave / C;               // ray groups (>= 2)
        const int its = (nr + G - 1) / G;      // ray slots per group
        const int c = lane % C, g = lane / C;
        const PRec pr = rec[nth_set_bit(sel, c)];
        double A[4] = {0.0, 0.0, 0.0, 0.0};
        for (int t = 0; t < its; ++t) {
            const int s = g + G * t;
            const bool act = g < G && s < nr;
            const int ss = act ? s : 0;
            Cot cr;
            const float2 gg = tab.g[ss];
            cr.g1 = gg.x;
            cr.g2 = gg.y;
            if constexpr (KG) {
                cr.k = tab.k[ss];
                const float2 hh = tab.h[ss];
                cr.h1 = hh.x;
                cr.h2 = hh.y;
            } else {
                cr.k = cr.h1 = cr.h2 = 0.0f;
            }
            double Gt[4];
            particle_grad<KG, KIND>(pr, tab.x[ss], tab.y[ss], mode, act, cr, invC, Gt);
            A[0] += Gt[0];
            A[1] += Gt[1];
            A[2] += Gt[2];
            A[3] += Gt[3];
        }
        // the G ray groups' sums meet in group 0 pairwise, in ceil(log2 G) rounds
        for (int st = 1; st < G; st <<= 1) {
            const bool take = (g & (2 * st - 1)) == 0 && g + st < G;
            const int src = take ? lane + st * C : lane;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const double v = __shfl(A[w], src, kWave);
                if (take) A[w] += v;
            }
        }
        if (g == 0) {
            double* dst = pg + 4 * (size_t)(pr.meta & 0x7fffffffu);
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (A[w] != 0.0) unsafeAtomicAdd(dst + w, A[w]);
        }
        for (int q = 0; q < C; ++q) sel &= sel - 1; // drop this pass's particles
    }
    wave_lds_sync(); // the slice is written again by the next user
}

// The words of one lane handed to the lane that DPP control CTRL names, within
// its 16-lane row.
template <int CTRL>
__device__ inline float row_peer(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// One halving step inside the rows: the M words of each lane become ceil(M / 2).
// Partner lanes (as DPP control CTRL pairs them) keep opposite words of each
// pair (hi: the second) and add the partner's copy; an odd last word is summed
// over both partners, who then hold the same total.
template <int M, int CTRL>
__device__ inline void row_halve(float* v, bool hi)
{
    constexpr int NP = M / 2;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const float keep = hi ? v[2 * p + 1] : v[2 * p];
        const float send = hi ? v[2 * p] : v[2 * p + 1];
        v[p] = keep + row_peer<CTRL>(send);
    }
    if constexpr ((M & 1) != 0) v[NP] = v[M - 1] + row_peer<CTRL>(v[M - 1]);
}

// The halving steps inside a row pair lane j with j ^ 8 (row_ror:8), with
// 7 - j inside its 8-lane half (row_half_mirror), then with j ^ 2 and j ^ 1
// (quad_perm); lane bit 3, 2, 1, 0 in turn picks the word kept.
constexpr int kRowStep[4] = {0x128, 0x141, 0x04E, 0x0B1};

// Totals over the wavefront of NA per-lane words (NA even), by recursive
// halving across the lanes, in registers.  The 32-lane halves swap the half of
// the words that the other one keeps (v_permlane32_swap: lane i < 32 exchanges
// its second operand with the first operand of lane i + 32) and add, so that
// half h holds words h H .. h H + H - 1 (H = NA / 2), each summed over two
// lanes; the two 16-lane rows of each half do the same with v_permlane16_swap,
// so that row R = 2 h + r holds words h H + r Q .. h H + r Q + Q - 1
// (Q = ceil(H / 2), a zero word filling an odd H) summed over four lanes; four
// halving steps inside the rows complete the sums over each row's 16 lanes.
// A lane's total is that of the word word_slot names.  Every lane of the
// wavefront takes part.
template <int NA>
__device__ inline float word_totals(const float* a)
{
    static_assert(NA % 2 == 0 && NA <= 64, "an even number of words");
    constexpr int H = NA / 2;
    constexpr int Q = (H + 1) / 2;
    constexpr int M2 = (Q + 1) / 2, M3 = (M2 + 1) / 2, M4 = (M3 + 1) / 2;
    static_assert((M4 + 1) / 2 == 1, "one word per lane after four steps");
    float b[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a[k]), __float_as_uint(a[H + k]), false,
                                                        false);
        b[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float c[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const float hi = k + Q < H ? b[k + Q] : 0.0f;
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[k]), __float_as_uint(hi), false, false);
        c[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const int j = (int)__lane_id() & 15;
    row_halve<Q, kRowStep[0]>(c, (j >> 3) & 1);
    row_halve<M2, kRowStep[1]>(c, (j >> 2) & 1);
    row_halve<M3, kRowStep[2]>(c, (j >> 1) & 1);
    row_halve<M4, kRowStep[3]>(c, j & 1);
    return c[0];
}

// The word whose total word_totals leaves in this lane: the same halving
// steps applied to word indices.  -1 where the lane holds no word, or a copy of
// a total that another lane holds too (only one lane adds it).
template <int NA>
__device__ inline int word_slot(int lane)
{
    constexpr int H = NA / 2;
    constexpr int Q = (H + 1) / 2;
    const int j = lane & 15, R = lane >> 4;
    int wd[Q];
    bool own[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        wd[k] = k;
        own[k] = true;
    }
    int m = Q;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const bool hi = ((j >> (3 - st)) & 1) != 0;
        const int np = m / 2;
#pragma unroll
        for (int p = 0; p < Q / 2; ++p) {
            if (p < np) {
                wd[p] = hi ? wd[2 * p + 1] : wd[2 * p];
                own[p] = hi ? own[2 * p + 1] : own[2 * p];
            }
        }
        if (m & 1) {
            wd[np] = wd[m - 1];
            own[np] = own[m - 1] && !hi;
        }
        m = np + (m & 1);
    }
    const int i = (R & 1) * Q + wd[0];
    return own[0] && i < H ? (R >> 1) * H + i : -1;
}

// Cotangent arrays of the rays (input order); any may be NULL (zero).
struct CotIn {
    const float *ga1, *ga2, *gk, *gg1, *gg2;
};

template <int P, bool KG, int KIND>
__global__ __launch_bounds__(kBlock) void k_adjoint_walk(TreeDev T, const double* __restrict__ rxs,
                                                        const double* __restrict__ rys,
                                                        const uint32_t* __restrict__ rperm, int64_t nrays,
                                                        CotIn ci, double* __restrict__ pg, double* __restrict__ abar,
                                                        int K, const int* __restrict__ split_box)
{
    // (Re, Im) of Abar_0 .. Abar_{P+1}, or with KG of Abar_0 .. Abar_P and Bbar
    constexpr int NA = 2 * (P + 1) + 2;
    // per wavefront: the packed ray table of a particle pass
    __shared__ __align__(16) float red_all[(kBlock / kWave) * kRayTableFloats];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t groups = (nrays + kWave - 1) / kWave;
    // wave-uniform work item (kept in SGPRs): box range kr, ray group grp
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    float* red = red_all + (size_t)w * kRayTableFloats;
    int kr;
    int64_t grp;
    if (!walk_task(blockIdx.x, w, groups, K, &kr, &grp)) return;
    // this wavefront's copies of the box adjoints and of the particle sums (see kAdjCopies)
    const int wid = (int)(blockIdx.x * (kBlock / kWave) + w);
    double* abox = abar + (size_t)(wid % kAdjCopies) * T.ncells * NA;
    pg += (size_t)(wid % kPgCopies) * 4 * T.n;
    const int64_t r = grp * kWave + lane;
    const bool valid = r < nrays;
    const double X = valid ? rxs[r] : 0.0, Y = valid ? rys[r] : 0.0;
    const int64_t o = valid ? (rperm ? (int64_t)rperm[r] : r) : 0;
    Cot cg{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (valid) {
        cg.g1 = ci.ga1 ? ci.ga1[o] : 0.0f;
        cg.g2 = ci.ga2 ? ci.ga2[o] : 0.0f;
        if constexpr (KG) {
            cg.k = ci.gk ? ci.gk[o] : 0.0f;
            cg.h1 = ci.gg1 ? ci.gg1[o] : 0.0f;
            cg.h2 = ci.gg2 ? ci.gg2[o] : 0.0f;
        }
    }
    const float g1 = cg.g1, g2 = cg.g2;
    const double gx0 = wave_min(valid ? X : INFINITY), gx1 = wave_max(valid ? X : -INFINITY);
    const double gy0 = wave_min(valid ? Y : INFINITY), gy1 = wave_max(valid ? Y : -INFINITY);
    const float invC = T.invC;
    const int wslot = word_slot<NA>(lane); // the box word this lane adds (see word_totals)

    // this wavefront's range of the preorder box array (see ancestor_skip)
    const int nc = T.ncells;
    int c0 = 0, c1 = nc;
    if (K > 1) {
        const int B = __builtin_amdgcn_readfirstlane(*split_box);
        if (B >= 0) {
            split_range(kr, K, B, uniform_ld(T.hdr, B).next, nc, &c0, &c1);
        } else { // no split: the first range takes every box
            c1 = kr == 0 ? nc : 0;
        }
    }
    int skip = valid ? 0 : 0x7fffffff;
    if (c0 > 0 && c0 < c1) skip = ancestor_skip(T, X, Y, c0, skip); // (an empty range walks nothing)
    int cur = c0;
    while (cur < c1) {
        cur = __builtin_amdgcn_readfirstlane(cur);
        const CellHdr h = uniform_ld(T.hdr, cur);
        const bool act = cur >= skip;
        if ((h.info & kInfoList) && list_reaches(T, cur, gx0, gx1, gy0, gy1)) {
            const CellExt e = uniform_ld(T.ext, cur);
            for (int base = e.lbeg; base < e.lend; base += kWave) {
                const int j = base + lane;
                bool cand = false;
                if (j < e.lend) {
                    const PRec pr = T.lst[j];
                    const double dxb = fmax(fmax(gx0 - pr.x, pr.x - gx1), 0.0);
                    const double dyb = fmax(fmax(gy0 - pr.y, pr.y - gy1), 0.0);
                    cand = dxb * dxb + dyb * dyb < pr.qs2 * (1.0 + 1e-9);
                }
                const uint64_t cm = __ballot(cand);
                if (cm) particles_grad<KG, KIND>(T.lst + base, cm, 1, __ballot(act), X, Y, cg, invC, pg, lane, red);
            }
        }
        double w1, w2;
        const double d2 = sqdist(X, Y, h.cx, h.cy, &w1, &w2);
        const bool acc = act && d2 > h.rcut2;
        const bool opn = act && !acc;
        if (__any(acc)) {
            // per-lane box adjoint terms; every lane evaluates them, the lanes that
            // did not accept with zero cotangents and w = (1, 0), so that their
            // words are exactly 0 (no branch, no clearing of the words)
            float a[NA];
            const float f1 = acc ? (float)w1 : 1.0f, f2 = acc ? (float)w2 : 0.0f;
            const float e1 = acc ? g1 : 0.0f, e2 = acc ? g2 : 0.0f;
            if constexpr (!KG) {
                // alpha cotangents only: the words are g_hat v t^k for k = 0 .. P + 1; the
                // centre-of-mass adjoint sum_k (k + 1) Q_k Abar_{k+1} is formed from them
                // in the push-down
                const float rcm = uniform_ld(T.mom, (int64_t)cur * mom_stride(P) + 1);
                const float inv = __builtin_amdgcn_rcpf(f1 * f1 + f2 * f2);
                const float v1 = f1 * inv, v2 = -f2 * inv;
                const float t1 = rcm * v1, t2 = rcm * v2;
                float p1 = fmaf(e1, v1, -e2 * v2), p2 = fmaf(e1, v2, e2 * v1);
#pragma unroll
                for (int k = 0; k <= P + 1; ++k) {
                    a[2 * k] = p1;
                    a[2 * k + 1] = p2;
                    const float n1 = fmaf(p1, t1, -p2 * t2), n2 = fmaf(p1, t2, p2 * t1);
                    p1 = n1;
                    p2 = n2;
                }
            } else {
                const float* mo = T.mom + (size_t)cur * mom_stride(P);
                const float M = mo[0], rcm = mo[1];
                const float inv = __builtin_amdgcn_rcpf(f1 * f1 + f2 * f2);
                const float v1 = f1 * inv, v2 = -f2 * inv;
                const float t1 = rcm * v1, t2 = rcm * v2;
                // g_hat v t^k
                float p1 = fmaf(e1, v1, -e2 * v2), p2 = fmaf(e1, v2, e2 * v1);
#pragma unroll
                for (int k = 0; k <= P; ++k) {
                    a[2 * k] = p1;
                    a[2 * k + 1] = p2;
                    const float n1 = fmaf(p1, t1, -p2 * t2), n2 = fmaf(p1, t2, p2 * t1);
                    p1 = n1;
                    p2 = n2;
                }
                // M S = M (P(t) + t P'(t)) = sum (k+1) M Qn_k t^k  (Qn_0 = 1, Qn_1 = 0;
                // the record holds M Qn_k)
                float b1 = M, b2 = 0.0f, c1 = 0.0f, c2 = 0.0f;
                if constexpr (P >= 2) {
                    b1 = mo[2 + 2 * (P - 2)];
                    b2 = mo[3 + 2 * (P - 2)];
                    c1 = b1;
                    c2 = b2;
#pragma unroll
                    for (int k = P - 1; k >= 0; --k) {
                        const float q1 = k >= 2 ? mo[2 + 2 * (k - 2)] : (k == 0 ? M : 0.0f);
                        const float q2 = k >= 2 ? mo[3 + 2 * (k - 2)] : 0.0f;
                        const float m1 = fmaf(b1, t1, fmaf(-b2, t2, q1)), m2 = fmaf(b1, t2, fmaf(b2, t1, q2));
                        b1 = m1;
                        b2 = m2;
                        if (k > 0) {
                            const float n1 = fmaf(c1, t1, fmaf(-c2, t2, b1)), n2 = fmaf(c1, t2, fmaf(c2, t1, b2));
                            c1 = n1;
                            c2 = n2;
                        }
                    }
                }
                const float S1 = fmaf(t1, c1, fmaf(-t2, c2, b1)), S2 = fmaf(t1, c2, fmaf(t2, c1, b2));
                const float w21 = fmaf(v1, v1, -v2 * v2), w22 = 2.0f * v1 * v2;
                const float V1 = fmaf(w21, S1, -w22 * S2), V2 = fmaf(w21, S2, w22 * S1);
                a[NA - 2] = e1 * V1 - e2 * V2;
                a[NA - 1] = e1 * V2 + e2 * V1;
                {
                    // gamma: Abar_k r_cm^k -= (k+1) gg v^2 t^k, Bbar -= gg M v^3 T(t)
                    const float h1 = acc ? cg.h1 : 0.0f, h2 = acc ? cg.h2 : 0.0f;
                    float q1 = fmaf(h1, w21, -h2 * w22), q2 = fmaf(h1, w22, h2 * w21); // gg v^2
#pragma unroll
                    for (int k = 0; k <= P; ++k) {
                        a[2 * k] -= (float)(k + 1) * q1;
                        a[2 * k + 1] -= (float)(k + 1) * q2;
                        const float n1 = fmaf(q1, t1, -q2 * t2), n2 = fmaf(q1, t2, q2 * t1);
                        q1 = n1;
                        q2 = n2;
                    }
                    // M T(t) = sum_k (k+1)(k+2) M Qn_k t^k by Horner (Qn_0 = 1, Qn_1 = 0)
                    float T1 = 0.0f, T2 = 0.0f;
#pragma unroll
                    for (int k = P; k >= 0; --k) {
                        const float cf = (float)((k + 1) * (k + 2));
                        const float q1k = k >= 2 ? cf * mo[2 + 2 * (k - 2)] : (k == 0 ? cf * M : 0.0f);
                        const float q2k = k >= 2 ? cf * mo[3 + 2 * (k - 2)] : 0.0f;
                        const float n1 = fmaf(T1, t1, fmaf(-T2, t2, q1k)), n2 = fmaf(T1, t2, fmaf(T2, t1, q2k));
                        T1 = n1;
                        T2 = n2;
                    }
                    const float w31 = fmaf(w21, v1, -w22 * v2), w32 = fmaf(w21, v2, w22 * v1); // v^3
                    const float U1 = fmaf(w31, T1, -w32 * T2), U2 = fmaf(w31, T2, w32 * T1);
                    a[NA - 2] -= h1 * U1 - h2 * U2;
                    a[NA - 1] -= h1 * U2 + h2 * U1;
                }
            }
            // one atomic instruction over the NA adjacent words
            const float mine = word_totals<NA>(a);
            if (wslot >= 0) unsafeAtomicAdd(abox + (size_t)cur * NA + wslot, (double)mine);
        }
        if (h.info & kInfoLeaf) {
            if (__any(opn)) {
                const CellExt e = uniform_ld(T.ext, cur);
                const uint64_t rays = __ballot(opn);
                for (int j = e.pbeg; j < e.pend; j += kWave) { // a leaf at the depth cap may exceed 64
                    const int np = e.pend - j < kWave ? e.pend - j : kWave;
                    const uint64_t sel = np == kWave ? ~0ull : ((1ull << np) - 1);
                    particles_grad<KG, KIND>(T.prt + j, sel, 0, rays, X, Y, cg, invC, pg, lane, red);
                }
            }
            cur = cur + 1;
        } else if (__any(opn)) {
            if (acc) skip = h.next;
            cur = cur + 1;
        } else {
            cur = h.next > cur ? h.next : cur + 1;
        }
    }
}

// Box adjoints -> particles.  One thread per particle walks its ancestors,
// then adds the direct-term gradients the walk gathered.  Without kappa and
// gamma cotangents (KG false) a box holds Abar_0 .. Abar_{P+1} (scaled by
// r_cm^k) and its centre-of-mass adjoint is Bbar = sum_{k <= P} (k + 1) Q_k Abar_{k+1}
// (dF/dz_cm = sum (k + 1) Q_k w^-(k+2)), formed here in FP64; with them the
// walk accumulated Bbar itself in the last two words.
template <int P, bool KG>
__global__ __launch_bounds__(kBlock) void k_pushdown(TreeDev T, const double* __restrict__ ms,
                                                    const double* __restrict__ abar, const double* __restrict__ pg,
                                                    double* __restrict__ dm, double* __restrict__ dx,
                                                    double* __restrict__ dy, double* __restrict__ ds)
{
    constexpr int NA = 2 * (P + 1) + 2;
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= T.n) return;
    const PRec pr = T.prt[k];
    const int32_t i = T.perm[k]; // original index
    const double mi = ms[k];
    double gm = 0.0, gzr = 0.0, gzi = 0.0;
    int c = 0;
    for (int guard = 0; guard <= kMaxLevel && c < T.ncells; ++guard) {
        const double* ab = abar + (size_t)c * NA;
        bool any = false;
#pragma unroll
        for (int q = 0; q < NA; ++q) any |= ab[q] != 0.0;
        const CellHdr h = T.hdr[c];
        if (any) {
            const double M = T.cM[c];
            const double rcm = (double)T.mom[(size_t)c * mom_stride(P) + 1];
            const double* Q = T.cq + (size_t)c * (P + 1) * 2;
            const double dr = pr.x - h.cx, di = pr.y - h.cy;
            double Br, Bi;
            if constexpr (KG) {
                Br = ab[NA - 2];
                Bi = ab[NA - 1];
            } else {
                Br = Bi = 0.0;
                double irk = 1.0 / rcm; // r_cm^-(k+1)
                const double irc = irk;
                for (int kk = 0; kk <= P; ++kk) {
                    const double Ar = ab[2 * (kk + 1)] * irk, Ai = ab[2 * (kk + 1) + 1] * irk;
                    const double qr = Q[2 * kk], qi = Q[2 * kk + 1];
                    Br += (kk + 1) * (qr * Ar - qi * Ai);
                    Bi += (kk + 1) * (qr * Ai + qi * Ar);
                    irk *= irc;
                }
            }
            // sm = sum_k Abar_k dQ_k/dm + Bbar d/M ; sz = sum_k Abar_k dQ_k/dz + Bbar m/M
            // (one reciprocal of M per box: an FP64 division is a long instruction sequence)
            const double iM = M > 0.0 ? 1.0 / M : 0.0, miM = mi * iM;
            double smr = 0.0, smi = 0.0, szr = 0.0, szi = 0.0;
            double dkr = 1.0, dki = 0.0, dkm1r = 0.0, dkm1i = 0.0; // d^k, d^(k-1)
            double irk = 1.0;                                      // r_cm^-k
            const double irc = 1.0 / rcm;
            for (int kk = 0; kk <= P; ++kk) {
                const double Ar = ab[2 * kk] * irk, Ai = ab[2 * kk + 1] * irk;
                double tmr = dkr, tmi = dki;                     // d^k
                double tzr = kk * mi * dkm1r, tzi = kk * mi * dkm1i; // k m d^(k-1)
                if (M > 0.0 && kk > 0) {
                    const double qr = Q[2 * (kk - 1)], qi = Q[2 * (kk - 1) + 1];
                    // k Q_{k-1} d / M and k Q_{k-1} m / M
                    tmr -= kk * (qr * dr - qi * di) * iM;
                    tmi -= kk * (qr * di + qi * dr) * iM;
                    tzr -= kk * qr * miM;
                    tzi -= kk * qi * miM;
                }
                smr += Ar * tmr - Ai * tmi;
                smi += Ar * tmi + Ai * tmr;
                szr += Ar * tzr - Ai * tzi;
                szi += Ar * tzi + Ai * tzr;
                dkm1r = dkr;
                dkm1i = dki;
                const double nr = dkr * dr - dki * di, ni = dkr * di + dki * dr;
                dkr = nr;
                dki = ni;
                irk *= irc;
            }
            if (M > 0.0) {
                smr += (Br * dr - Bi * di) * iM;
                smi += (Br * di + Bi * dr) * iM;
                szr += Br * miM;
                szi += Bi * miM;
            }
            gm += smr;
            gzr += szr;
            gzi += szi;
        }
        if (h.info & kInfoLeaf) break;
        // descend into the child whose Morton range holds position k (the four
        // children's ranges load together)
        const int4 kc = *reinterpret_cast<const int4*>(T.kids + 4 * (size_t)c);
        const int cu[4] = {kc.x, kc.y, kc.z, kc.w};
        int ch = -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (cu[u] >= 0 && k >= T.cbeg[cu[u]] && k < T.cend[cu[u]]) ch = cu[u];
        if (ch < 0) break;
        c = ch;
    }
    // plus the direct terms the walk gathered for this particle
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < kPgCopies; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) q[j] += pg[(size_t)r * 4 * T.n + 4 * (size_t)k + j];
    if (dm) dm[i] += gm + q[0];
    if (dx) dx[i] += gzr + q[1];
    if (dy) dy[i] += q[2] - gzi;
    if (ds) ds[i] += q[3];
}

__global__ void k_fill_zero(double* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// copy 0 of the box adjoints += copies 1 .. kAdjCopies - 1 (n words each)
__global__ void k_sum_copies(double* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = p[i];
#pragma unroll
    for (int r = 1; r < kAdjCopies; ++r) s += p[(size_t)r * n + i];
    p[i] = s;
}

// FP64 scratch words: kAdjCopies copies of the box adjoints (NA per box),
// then 4 direct-term gradients per particle.
size_t adjoint_scratch_words(const TreeStorage& ts)
{
    const int NA = 2 * (ts.params.order + 1) + 2;
    return (size_t)kAdjCopies * ts.ncells * NA + 4 * (size_t)kPgCopies * ts.n;
}

template <int P>
glm_status launch_adjoint(const TreeStorage& ts, const StagedRays& sr, int64_t nrays, const CotIn& ci, double* dm,
                          double* dx, double* dy, double* ds, int K, const int* split_box, double* abar,
                          hipStream_t st)
{
    constexpr int NA = 2 * (P + 1) + 2;
    const size_t words = adjoint_scratch_words(ts);
    const int64_t nbox = (int64_t)ts.ncells * NA;
    double* pg = abar + (size_t)kAdjCopies * nbox;
    hipLaunchKernelGGL(k_fill_zero, dim3(ceil_div((int64_t)words, kBlock)), dim3(kBlock), 0, st, abar, (int64_t)words);
    const int64_t blocks = walk_grid_blocks((nrays + kWave - 1) / kWave, K);
    const bool kg = ci.gk || ci.gg1 || ci.gg2;
#define GLM_ADJ(KGV, KD)                                                                                          \
    hipLaunchKernelGGL((k_adjoint_walk<P, KGV, KD>), dim3((unsigned)blocks), dim3(kBlock), 0, st, ts.dev, sr.xs, \
                       sr.ys, sr.perm, nrays, ci, pg, abar, K, split_box)
    if (ts.dev.kind == kKindNfw) {
        if (kg) GLM_ADJ(true, kKindNfw);
        else GLM_ADJ(false, kKindNfw);
    } else {
        if (kg) GLM_ADJ(true, kKindGauss);
        else GLM_ADJ(false, kKindGauss);
    }
#undef GLM_ADJ
    hipLaunchKernelGGL(k_sum_copies, dim3(ceil_div(nbox, (int64_t)kBlock)), dim3(kBlock), 0, st, abar, nbox);
    if (kg)
        hipLaunchKernelGGL((k_pushdown<P, true>), dim3(ceil_div(ts.n, kBlock)), dim3(kBlock), 0, st, ts.dev, ts.ms, abar,
                           pg, dm, dx, dy, ds);
    else
        hipLaunchKernelGGL((k_pushdown<P, false>), dim3(ceil_div(ts.n, kBlock)), dim3(kBlock), 0, st, ts.dev, ts.ms,
                           abar, pg, dm, dx, dy, ds);
    GLM_HIP(hipGetLastError());
    return GLM_OK;
}

} // namespace

size_t adjoint_workspace_bytes(const TreeStorage& ts, int64_t nrays)
{
    return ray_layout(nrays).bytes + sizeof(double) * adjoint_scratch_words(ts);
}

glm_status adjoint_device(const TreeStorage& ts, const double* rx, const double* ry, int64_t nrays, const float* ga1,
                          const float* ga2, const float* gk, const float* gg1, const float* gg2, double* dm,
                          double* dx, double* dy, double* ds, uint32_t flags, void* ws, hipStream_t st)
{
    if (nrays == 0) return GLM_OK;
    StagedRays sr{rx, ry, nullptr};
    const RayLayout L = ray_layout(nrays);
    if (flags & GLM_RAYS_STAGED) {
        sr = staged_rays_view(nrays, ws, L); // glm_stage_rays left them at the workspace's start
    } else if (!(flags & GLM_RAYS_ORDERED)) {
        glm_status rc = stage_rays(rx, ry, nrays, ws, L, &sr, st);
        if (rc != GLM_OK) return rc;
    }
    int K = L.split;
    while (K > 1 && (int64_t)K * 64 > ts.ncells) --K;
    if (K < 4) K = 1;
    int* split_box = nullptr;
    if (K > 1) {
        glm_status rc = split_box_device(ts, rx, ry, nrays, ws, L, !(flags & GLM_RAYS_ORDERED), &split_box, st);
        if (rc != GLM_OK) return rc;
    }
    double* abar = reinterpret_cast<double*>(static_cast<char*>(ws) + L.bytes);
#define GLM_CASE(PP)                                                                                              \
    case PP:                                                                                                      \
        return launch_adjoint<PP>(ts, sr, nrays, CotIn{ga1, ga2, gk, gg1, gg2}, dm, dx, dy, ds, K, split_box, abar, \
                                  st);
    switch (ts.params.order) {
        GLM_CASE(0) GLM_CASE(1) GLM_CASE(2) GLM_CASE(3) GLM_CASE(4) GLM_CASE(5) GLM_CASE(6)
        GLM_CASE(7) GLM_CASE(8) GLM_CASE(9) GLM_CASE(10) GLM_CASE(11) GLM_CASE(12)
        default: return fail(GLM_ESTATE, "unsupported order");
    }
#undef GLM_CASE
}

} // namespace glm
