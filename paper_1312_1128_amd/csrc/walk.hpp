// Ray staging and the forward / adjoint walks.
#pragma once

#include "build.hpp"

namespace glm {

// Outputs of a walk (input order of the rays).
struct WalkOut {
    float *a1, *a2, *k, *g1, *g2;
    int32_t* counts;
    float* psi = nullptr; // potential walk only
    float* td = nullptr;  // time delay |alpha|^2 / 2 - psi (nullable)
};

// One lens of a batched walk (device table entry).
struct BatchLens {
    TreeDev tree;
    int64_t nrays;
    int64_t ray_off;   // offset of its rays in the concatenated staged arrays
    const double* rx;  // the caller's rays (input order)
    const double* ry;
    WalkOut out;
};

// Persistent walk over several lenses; host_table is in queue order (largest
// expected work first), every tree built with the same order.
size_t batch_workspace_bytes(int nlens, int64_t total_rays);
glm_status shoot_batched_device(const BatchLens* host_table, int nlens, int order, uint32_t flags, void* ws,
                                hipStream_t st);

size_t refine_workspace_bytes(int64_t ncells);
glm_status refine_round_device(double* cx, double* cy, double* side, const float* ka, const float* g1,
                               const float* g2, int64_t ncells, int64_t nrefine, int32_t* refined, void* ws,
                               hipStream_t st);
// The two halves of a round: rank the cells (order = cell indices by
// descending score, in ws), then split the first nrefine of them.
glm_status refine_rank_device(const double* side, const float* ka, const float* g1, const float* g2,
                              int64_t ncells, void* ws, const uint32_t** order, hipStream_t st);
glm_status refine_spawn_device(const uint32_t* order, int64_t nrefine, int64_t ncells, double* cx, double* cy,
                               double* side, int32_t* refined, hipStream_t st);

// Interpolation shortcut of refinement (interp.hip): per-cell level and
// integer coordinates plus a (level, i, j) -> cell hash, in a caller buffer.
struct InterpLayout {
    size_t lev, ci, cj, keys, vals, bytes;
    int64_t table_cap;
};
InterpLayout interp_layout(int64_t capacity);
size_t interp_round_workspace_bytes(int64_t ncells, int64_t nrefine);
glm_status interp_init_device(const double* cx, const double* cy, int64_t ncells, double x0, double y0, double h0,
                              int64_t capacity, void* state, hipStream_t st);
glm_status interp_round_device(double* cx, double* cy, double* side, float* a1, float* a2, float* ka, float* g1,
                               float* g2, int64_t ncells, int64_t nrefine, int64_t nbase, float tol, bool deflections,
                               int32_t* refined, int32_t* shoot_idx, int32_t* shoot_count, int64_t capacity,
                               void* state, void* ws, hipStream_t st);
// kappa, gamma of cells idx[0 .. min(*count, max_count)) (idx NULL: cells 0 ..
// max_count; count NULL: max_count) from their three-point magnification matrix.
glm_status interp_estimate_device(const double* cx, const double* cy, const float* a1, const float* a2, float* ka,
                                  float* g1, float* g2, const int32_t* idx, const int32_t* count, int64_t max_count,
                                  int64_t nbase, int64_t capacity, const void* state, hipStream_t st);
size_t shoot_indexed_workspace_bytes(int64_t count);

// Wavefronts per 64-ray group.  A small launch (few groups) splits the
// preorder box array into K ranges walked by separate wavefronts, so that
// about kSplitWaves wavefronts keep the chip busy; their partial sums are
// merged per ray in range order.  A split has a range before, K - 2 slices
// of, and a range after one box: below kMinSplit ranges it rarely spreads the
// work, so there is none.
constexpr int64_t kSplitWaves = 16384;
constexpr int64_t kMinSplit = 4;
constexpr int64_t kMaxSplit = 32;

inline int walk_split(int64_t nrays)
{
    const int64_t groups = (nrays + 63) / 64;
    if (groups <= 0) return 1;
    int64_t k = (kSplitWaves + groups - 1) / groups;
    if (k > kMaxSplit) k = kMaxSplit;
    if (k < kMinSplit) k = 1;
    return (int)k;
}

// Partial-sum slots (K x rays) to reserve for up to nrays rays: a bound that
// grows with nrays, so that a workspace sized for a launch also fits every
// smaller one (K * groups < kSplitWaves + kSplitWaves / kMinSplit).
inline int64_t split_slots(int64_t nrays)
{
    const int64_t groups = (nrays + 63) / 64;
    const int64_t cap = kSplitWaves + kSplitWaves / kMinSplit;
    return 64 * (kMaxSplit * groups < cap ? kMaxSplit * groups : cap);
}

// Per-ray counts of a walk: boxes visited (opening tests), boxes accepted,
// leaf particles summed, list particles the ray falls inside; then counts of
// its wavefront (the same for the 64 rays of a group): list entries tested
// against the ray group (the search overhead), boxes some lane accepted, leaf
// particles evaluated, list candidates evaluated.  The per-lane counts over the
// wavefront's give the lane use of each phase.
constexpr int kCounts = 8;

// Partial sums of one ray over one range of boxes (merged by k_walk_merge);
// 72 bytes, so that the largest partial-sum region (20480 groups x 64 rays)
// stays at 94 MB.
struct alignas(8) Partial {
    double a1, a2, g1, g2;
    float k;
    int32_t cnt[kCounts];
};
static_assert(sizeof(Partial) == 72, "partial-sum record size");

// Byte offsets of the ray workspace pieces.
struct RayLayout {
    size_t k0, k1, v0, v1, xs, ys, hist, part, sbox, parts, bytes;
    int split;
};
RayLayout ray_layout(int64_t nrays);

struct StagedRays {
    const double* xs;
    const double* ys;
    const uint32_t* perm; // sorted -> input position, or null when unsorted
};

// Morton-sort the rays (8 to 16 bits per axis in their bounding square) so that
// each 64-ray group is spatially compact.
glm_status stage_rays(const double* rx, const double* ry, int64_t nrays, void* ws, const RayLayout& L,
                      StagedRays* out, hipStream_t st);
// The staged rays that stage_rays left in the workspace (no launch).
StagedRays staged_rays_view(int64_t nrays, void* ws, const RayLayout& L);

// Index of the deepest box holding the rays' bounding box, written to the
// workspace (computes the box unless stage_rays did).
glm_status split_box_device(const TreeStorage& ts, const double* rx, const double* ry, int64_t nrays, void* ws,
                            const RayLayout& L, bool have_bbox, int** out, hipStream_t st);

glm_status shoot_device(const TreeStorage& ts, const double* rx, const double* ry, int64_t nrays, float* a1,
                        float* a2, float* k, float* g1, float* g2, int32_t* counts, uint32_t flags, void* ws,
                        hipStream_t st);

glm_status shoot_indexed_device(const TreeStorage& ts, const double* cx, const double* cy, const int32_t* idx,
                                int64_t count, float* a1, float* a2, float* ka, float* g1, float* g2, uint32_t flags,
                                void* ws, hipStream_t st);

// alpha and the potential psi (and the time delay when td is not NULL) of
// the rays; one wavefront per 64-ray group (no split).
glm_status potential_device(const TreeStorage& ts, const double* rx, const double* ry, int64_t nrays, float* a1,
                            float* a2, float* psi, float* td, uint32_t flags, void* ws, hipStream_t st);

// kind: kKindGauss (q = cutoff) or kKindNfw (s = sizes, q = concentration)
glm_status direct_device(const double* x, const double* y, const double* m, const double* s, int64_t n, double q,
                         int kind, const double* rx, const double* ry, int64_t nrays, int fp64, void* const out5[5],
                         hipStream_t st);

// Cotangents: ga1, ga2 = dL/dalpha, gk = dL/dkappa, gg1, gg2 = dL/dgamma (each nullable: zero).
// The workspace holds the ray staging, then the box adjoints and the
// per-particle direct-term sums.
size_t adjoint_workspace_bytes(const TreeStorage& ts, int64_t nrays);
glm_status adjoint_device(const TreeStorage& ts, const double* rx, const double* ry, int64_t nrays, const float* ga1,
                          const float* ga2, const float* gk, const float* gg1, const float* gg2, double* dm,
                          double* dx, double* dy, double* ds, uint32_t flags, void* ws, hipStream_t st);

} // namespace glm
