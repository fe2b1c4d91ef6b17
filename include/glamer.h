/*
 * glamer.h -- C ABI of the MI355X (gfx950) tree ray-shooting library.
 *
 * For a batch of image-plane points ("rays") on one lens plane the library
 * computes the deflection alpha, the convergence kappa and the shear
 * (gamma1, gamma2) (Sec. 3.2, definitions of the lensing quantities), summed
 * over point masses (Sec. 3.5) and smoothed particles with the truncated
 * Gaussian profile of Sec. 3.1, by the modified quad-tree of Sec. 3.2:
 * equal-area boxes, multipole moments about each box's centre of mass, the
 * opening test |x - x_cm| > r_cut = r_cm / theta (Eq. r_cut), per-box lists of
 * "big" particles, and direct sums in the leaves.
 *
 * Units: masses are m / (pi Sigma_crit) (units of length^2), so a point mass
 * deflects alpha = m d / |d|^2 and has Einstein radius sqrt(m) (Sec. 3.5).
 *
 * Conventions for every entry point
 *  - Array arguments are DEVICE pointers (HIP global memory) unless stated;
 *    they stay owned by the caller and are never freed or retained past the
 *    call except where a tree handle says so.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Work
 *    is enqueued on it; calls return without waiting unless stated.
 *  - Arguments are validated on the host before anything is launched; a
 *    rejected call launches nothing and returns GLM_EINVAL.  glm_last_error()
 *    returns a message for the last failing call on the calling thread.
 *  - A failing HIP runtime call returns GLM_EHIP; asynchronous kernel faults
 *    surface at the next synchronising call.
 *  - No C++ exception crosses this interface.
 */
#ifndef GLAMER_H
#define GLAMER_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define GLM_API __attribute__((visibility("default")))
#else
#define GLM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GLM_OK = 0,
    GLM_EINVAL = -1, /* bad argument (null pointer, size, parameter range) */
    GLM_ENOMEM = -2, /* device or host allocation failed / workspace too small */
    GLM_EHIP = -3,   /* HIP runtime error */
    GLM_ESTATE = -4, /* handle not built, or built with other parameters */
    GLM_EDATA = -5   /* input values rejected (NaN/Inf, negative mass or smoothing) */
} glm_status;

/* int32 counts per ray written by glm_shoot and glm_shoot_noalloc */
#define GLM_COUNTS 8

/* flags */
#define GLM_ALPHA_ONLY 1u   /* skip kappa and gamma (Sec. 3.2: the solver's option) */
#define GLM_FP32_ALPHA 2u   /* alpha terms summed in plain FP32, not FP64 (debug) */
#define GLM_RAYS_ORDERED 4u /* rays already in a spatially coherent order: skip the ray sort */
#define GLM_RAYS_STAGED 16u /* the workspace holds these rays as glm_stage_rays left them: skip the ray sort */
/* build: the particles are truncated NFW halos (Sec. 3.2: analytic halos as
 * particles), not Gaussians.  A halo of mass m, size s = R (its truncation
 * radius, the support) and concentration c = q has the projected NFW surface
 * density with scale radius r_s = R / c, cut at projected radius R and
 * normalised to mass m inside R; beyond R it is a point mass.  With x = r / r_s,
 * F = arccosh(1/x)/sqrt(1-x^2) (x < 1), arccos(1/x)/sqrt(x^2-1) (x > 1),
 * f = (1 - F)/(x^2 - 1), g = ln(x/2) + F:  alpha = m g(x)/g(c) d/r^2,
 * kappa = m f(x) / (2 r_s^2 g(c)).  A ray exactly at a halo's centre gets
 * nothing from it.  s = 0 is a point mass.  Same big-particle lists (a halo is
 * listed where R > side / 2) and the same walk.  Its potential (glm_shoot_potential)
 * is psi = m [H(x) - H(c)] / g(c) + m ln R inside R, with H(x) = ln^2(x/2)/2 -
 * arccosh^2(1/x)/2 (x < 1) or + arccos^2(1/x)/2 (x > 1), and m ln r outside.
 * The adjoint walk gives dL/dR (size, at fixed c) in place of dL/ds. */
#define GLM_NFW_HALOS 8u

/* Solver parameters (Sec. 3.2 and 3.1). */
typedef struct {
    double theta;      /* opening parameter theta_force, 0 <= theta < 1 (0 = direct sum) */
    double q;          /* Gaussian cutoff in smoothing lengths, q > 0 (Sec. 3.1); the halo
                          concentration c with GLM_NFW_HALOS */
    int32_t leaf_size; /* a box is a leaf when it holds <= leaf_size particles, 1..64 */
    int32_t order;     /* multipole order p: moments Q_0..Q_p, 0..12 ("monopole and quadrupole" = 2) */
    uint32_t flags;    /* GLM_* flags */
} glm_params;

/* Opaque tree handle: a host struct that points into the caller's tree
 * workspace (see glm_build_tree), which holds every device array of the
 * built tree.  The library never allocates or frees device memory for it. */
typedef struct glm_tree glm_tree;

typedef struct {
    int64_t n;           /* particles */
    int64_t ncells;      /* boxes (depth-first preorder) */
    int64_t nleaves;
    int64_t nlisted;     /* particles held in some box's big-particle list */
    int32_t max_level;   /* deepest box level (root = 0, cap 32) */
    int32_t order;
    int32_t check_flags; /* 0 when the build's internal consistency checks passed */
    int32_t reserved;
    double root_x0, root_y0, root_side; /* root square */
    size_t device_bytes; /* bytes of the caller's tree workspace the built tree occupies */
} glm_tree_info;

/* Create an empty handle.  *out receives it.  Host allocation only. */
GLM_API glm_status glm_tree_create(glm_tree** out);

/* Release the host handle.  The tree workspace stays the caller's; nothing
 * is synchronised or freed on the device.  NULL is ignored. */
GLM_API void glm_tree_destroy(glm_tree* t);

/*
 * Upper bound of the device workspace glm_build_tree needs for n particles
 * with these parameters (host arithmetic only, no device call).  The bound
 * counts the particle arrays (Morton sort, sorted copies, walk records, list
 * entries: about 150 bytes per particle) and the box arrays for the largest
 * box count such a tree can have: every leaf holds at least one particle and
 * every internal box more than leaf_size, so a level holds at most
 * min(4^l, n / (leaf_size + 1)) internal boxes, and a tree of I internal
 * boxes at most 4 I + 1 boxes (Sec. 3.2: boxes split into four until they
 * hold at most the leaf size).  Real trees need far less (the 1e6-particle
 * NFW halo at leaf size 16 holds 181k boxes of the 2.4M the bound allows):
 * glm_tree_required_bytes gives the exact figure after a build.
 */
GLM_API glm_status glm_tree_workspace_bytes(int64_t n, const glm_params* params, size_t* bytes);

/*
 * Build the tree of n particles (Sec. 3.2): the root square covers the
 * particles' bounding box (side = max extent * (1 + 2^-40)); particles are
 * ordered by 64-bit Morton keys of 32-bit quantised coordinates, compared on
 * their top 32 bits when the tree has no box below level 16 and on all 64
 * otherwise (equal keys in input order; both orders give the same boxes);
 * boxes are the Morton-prefix ranges, a box with <= leaf_size particles (or at
 * depth 32) is a leaf; the moments Q_k = sum m (z - z_cm)^k, k <= order, are built in FP64;
 * r_cut^2 = (farthest-corner distance from the centre of mass / theta)^2; a
 * smoothed particle is listed in the highest box where q s > side / 2, if that
 * box is not below its leaf.
 *
 *   x, y, m : device FP64 arrays of length n (positions, masses >= 0)
 *   s       : device FP64 smoothing lengths >= 0 (0 = point mass), or NULL for
 *             all point masses
 *   n       : 1 .. 2^31 - 1
 *
 *   workspace, workspace_bytes: caller-owned device memory that receives
 *             every array of the tree; it must stay allocated and unmodified
 *             while the handle is used (walks, adjoints, exports) and may be
 *             reused by the next build on this or another handle.
 *             glm_tree_workspace_bytes(n, params) always suffices.  A smaller
 *             one is accepted: the build fails with GLM_ENOMEM if it cannot
 *             hold the particle arrays (before anything is launched) or,
 *             after the box count is known, the box arrays; then
 *             glm_tree_required_bytes gives the exact size this input needs.
 *
 * Synchronises `stream` once (to size the box arrays); the inputs may be
 * reused or freed after return.  The box count is read through a small
 * page-locked host block (the build's count record, under 5 KB)
 * taken from a process-wide pool: a block is allocated when more builds run
 * at once than ever before and is kept until the process ends; the handle
 * owns none.  If that allocation fails, the read uses pageable memory.
 * GLM_EDATA if any value is NaN/Inf or a mass or smoothing length is
 * negative.
 */
GLM_API glm_status glm_build_tree(glm_tree* t, const double* x, const double* y, const double* m,
                          const double* s, int64_t n, const glm_params* params, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Exact workspace bytes the last glm_build_tree on this handle needed (also
 * when it failed with GLM_ENOMEM for lack of space).  GLM_ESTATE before any
 * build got that far. */
GLM_API glm_status glm_tree_required_bytes(const glm_tree* t, size_t* bytes);

/* Host copy of the tree summary. */
GLM_API glm_status glm_tree_get_info(const glm_tree* t, glm_tree_info* out);

/*
 * Copy the tree out to HOST arrays (each may be NULL to skip), for checking:
 *   per box, preorder (ncells): level, ix, iy (box index at its level), beg,
 *     end (range in Morton order), next (preorder index past the subtree),
 *     leaf (0/1), lbeg, lend (range in the list arrays);
 *     M, cx, cy, rcut2 (FP64); Q: 2*(order+1) doubles per box, (Re, Im) of
 *     Q_0..Q_order about the centre of mass (Q_1 as computed, ~0);
 *   per particle (n, the build's order): perm (original index of the k-th
 *     particle), key (its 64-bit Morton key, x bits even, y bits odd);
 *   per list entry (nlisted): list_idx (original particle index).
 * Synchronises the device.
 */
GLM_API glm_status glm_tree_export(const glm_tree* t, int32_t* level, uint32_t* ix, uint32_t* iy,
                           int32_t* beg, int32_t* end, int32_t* next, int32_t* leaf,
                           int32_t* lbeg, int32_t* lend, double* M, double* cx, double* cy,
                           double* rcut2, double* Q, int32_t* perm, uint64_t* key,
                           int32_t* list_idx);

/*
 * Smoothing lengths (Sec. 3.1: the smoothing scale of a particle is the
 * radius holding its N_sph nearest neighbours) of the tree's n particles, in
 * 2D: for each particle the distance to its k-th nearest other particle
 * (itself excluded; coincident particles count, at distance 0), from the FP64
 * positions given to glm_build_tree, by a pruned walk of the tree's boxes.
 *   s_out: device FP64, n values, original particle order (overwritten)
 *   k    : 1 .. 64 and at most n - 1, else GLM_EINVAL
 * Masses, moments and lists are not used: a tree built with unit masses and
 * s = NULL serves.  Enqueued on `stream`; no workspace.
 */
GLM_API glm_status glm_tree_knn(const glm_tree* t, int32_t k, double* s_out, void* stream);

/*
 * Smoothing lengths from raw positions (Sec. 3.1): for each particle the
 * distance to its k-th nearest other particle (itself excluded, coincident
 * particles at distance 0), counted in projection when z is NULL and in space
 * (the paper's preferred 3D smoothing) otherwise; with species != NULL only
 * particles of the same species count (each species is smoothed on its own).
 * The squared distance is (dx^2 + dy^2) + dz^2 in FP64, so the result is the
 * square root of the k-th smallest FP64 squared distance.
 *   x, y, z : device FP64 positions, length n (z nullable); n in 2 .. 2^31 - 1
 *   species : device int32 ids in [0, 65535], nullable
 *   k       : 1 .. 64, and every species must hold at least k + 1 particles
 *   s_out   : device FP64, length n, original order (written)
 *   workspace: at least glm_knn_workspace_bytes(n, species != NULL) bytes
 * Synchronises `stream` once (twice with species). GLM_EDATA for a non-finite
 * position, a species id out of range or a species with <= k particles.
 */
GLM_API glm_status glm_knn_workspace_bytes(int64_t n, int32_t with_species, size_t* bytes);
GLM_API glm_status glm_knn(const double* x, const double* y, const double* z, const int32_t* species, int64_t n,
                   int32_t k, double* s_out, void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of device workspace glm_shoot / glm_shoot_adjoint need for nrays rays. */
GLM_API glm_status glm_shoot_workspace_bytes(int64_t nrays, size_t* bytes);

/*
 * Forward tree walk (Sec. 3.2) for nrays rays at (rx[i], ry[i]) (device FP64).
 * Outputs (device FP32, length nrays, input order): a1, a2, kappa, g1, g2.
 * kappa, g1, g2 may be NULL when the tree was built with GLM_ALPHA_ONLY or
 * `flags` carries it.  counts (device int32, GLM_COUNTS = 8 per ray, nullable)
 * receives per ray: boxes visited (opening tests), boxes accepted, leaf
 * particles summed, list particles the ray falls inside; then four counts of
 * the wavefront that walked the ray's 64-ray group (summed over the box
 * ranges of a split walk): big-particle list entries tested against the
 * group's bounding box (the list search), boxes some ray of the group
 * accepted, leaf particles evaluated, list candidates evaluated.  The per-ray
 * counts over the wavefront counts give each phase's lane use.  A box's list
 * is tested 64 entries at a time, and not at all when the bounding box of its
 * particles' supports misses the group.  The walk evaluates its terms in FP32
 * and sums alpha and gamma in FP64; ray-particle and ray-box offsets and every
 * accept/inside decision are taken in FP64.
 *   workspace: device buffer of at least glm_shoot_workspace_bytes(nrays)
 *   (ray sort, and for small ray counts the partial sums of several
 *   wavefronts per ray group, each walking one range of the box array).
 *   flags: GLM_ALPHA_ONLY, GLM_FP32_ALPHA, GLM_RAYS_ORDERED or GLM_RAYS_STAGED
 *   (not both; see glm_stage_rays), or-ed with the tree's.
 * nrays may be 0 (nothing is launched).
 */
GLM_API glm_status glm_shoot(const glm_tree* t, const double* rx, const double* ry, int64_t nrays,
                     float* a1, float* a2, float* kappa, float* g1, float* g2, int32_t* counts,
                     uint32_t flags, void* workspace, size_t workspace_bytes, void* stream);

/*
 * The ray staging of glm_shoot (Sec. 3.3: rays are independent; here they are
 * sorted along a Morton curve of their bounding square into spatially compact
 * 64-ray groups, and copied in that order) on its own, so that it can run on
 * another stream than the tree build, which it does not depend on.  It writes
 * the staged rays into `workspace` (at least glm_shoot_workspace_bytes(nrays)
 * bytes, device); a following glm_shoot of the same rx, ry, nrays with flag
 * GLM_RAYS_STAGED and the same workspace skips its own staging and gives the
 * same results, bit for bit.  The caller orders that glm_shoot after this call
 * (an event between the streams), and keeps rx, ry and the workspace unchanged
 * in between.  rx, ry: device FP64, length nrays; nrays may be 0.
 */
GLM_API glm_status glm_stage_rays(const double* rx, const double* ry, int64_t nrays, void* workspace,
                          size_t workspace_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): glm_shoot
 * with no workspace argument.  The same walk and the same results as
 * glm_shoot; its ray workspace is a static device array of 128 MiB that the
 * library holds on every GPU it runs on until the process ends, so the call
 * allocates nothing.  All calls on one GPU share that array (each call's
 * contents are left behind and overwritten by the next): calls that overlap
 * on one GPU -- on different streams or from different threads -- race, and
 * must be ordered by the caller.
 *   nrays: 0 .. GLM_NOALLOC_MAX_RAYS, else GLM_EINVAL with nothing launched;
 *   stream: must belong to the current device (GLM_EINVAL otherwise);
 *   flags: as glm_shoot except GLM_RAYS_STAGED (GLM_EINVAL: the static array
 *   holds no rays the caller staged);
 *   other arguments as glm_shoot.
 */
#define GLM_NOALLOC_MAX_RAYS 1048576
GLM_API glm_status glm_shoot_noalloc(const glm_tree* t, const double* rx, const double* ry, int64_t nrays,
                                     float* a1, float* a2, float* kappa, float* g1, float* g2, int32_t* counts,
                                     uint32_t flags, void* stream);

/*
 * Deflection and lensing potential (Sec. 3.2: alpha = grad psi; the time
 * delay of a single plane is |alpha|^2 / 2 - psi), in one tree walk with the
 * decisions of glm_shoot.  A point mass contributes m ln r (0 for a ray
 * exactly on it), a truncated Gaussian the point-mass value outside its
 * support and, inside, m [ln(q s) - (Ein(q^2/2) - Ein(u)) / (2C)] with
 * Ein(z) = integral_0^z (1 - e^-t) / t dt; a box contributes
 * Re[Q_0 ln w - sum_k Q_k / (k w^k)].  FP32 terms, FP64 sums.
 *   a1, a2, psi: device FP32 outputs (nrays, input order);
 *   tdelay: device FP32 |alpha|^2 / 2 - psi, or NULL;
 *   flags: GLM_RAYS_ORDERED or 0; workspace as for glm_shoot.
 * One wavefront per 64-ray group (small launches are not split).
 */
GLM_API glm_status glm_shoot_potential(const glm_tree* t, const double* rx, const double* ry, int64_t nrays,
                                       float* a1, float* a2, float* psi, float* tdelay, uint32_t flags,
                                       void* workspace, size_t workspace_bytes, void* stream);

/*
 * Plain direct sum over all n particles (theta = 0 equivalent; Sec. 5.1), for
 * rays (device FP64).  fp64 != 0: outputs are device double arrays; else
 * float arrays with FP32 evaluation and FP64 sums of alpha and gamma.
 * out5: device pointers a1, a2, kappa, g1, g2 (kappa/g1/g2 nullable).
 * s may be NULL (point masses).
 */
GLM_API glm_status glm_shoot_direct(const double* x, const double* y, const double* m, const double* s,
                            int64_t n, double q, const double* rx, const double* ry,
                            int64_t nrays, int fp64, void* const out5[5], void* stream);

/*
 * Plain direct sum over n truncated NFW halos (the profile of GLM_NFW_HALOS;
 * Sec. 3.2 and the halo tests of Sec. 5.1): R = sizes (device FP64, >= 0,
 * 0 = point mass), c = concentration > 0, other arguments as glm_shoot_direct.
 * fp64 != 0 evaluates the profile in FP64; else FP32 terms summed in FP64,
 * as the tree walk does.
 */
GLM_API glm_status glm_shoot_direct_nfw(const double* x, const double* y, const double* m, const double* R,
                                int64_t n, double c, const double* rx, const double* ry,
                                int64_t nrays, int fp64, void* const out5[5], void* stream);

/*
 * Adjoint of glm_shoot for L with cotangents ga1 = dL/dalpha1, ga2 = dL/dalpha2,
 * gk = dL/dkappa, gg1 = dL/dgamma1, gg2 = dL/dgamma2 (device FP32, length
 * nrays, input order; each may be NULL, meaning zero, but not all five).
 * Replays the forward walk's decisions on the same tree and rays, and
 * ACCUMULATES (+=) into the device FP64 arrays (original particle order,
 * length n): dm, dx, dy, ds (each nullable; ds is zero for point masses).
 * Moment contributions are pushed down from boxes to particles through
 * dQ_k/dm_i, dQ_k/dz_i and dz_cm (kappa has no box term; gamma1 - i gamma2 of
 * a box is the derivative of its alpha1 - i alpha2 series).  Uses FP64
 * atomics: results are reproducible to rounding, not bitwise.  For a tree of
 * GLM_NFW_HALOS, ds receives dL/dR (the halo size, concentration fixed).
 *   workspace: at least glm_adjoint_workspace_bytes(t, nrays) bytes: the ray
 *   staging of glm_shoot, then FP64 scratch for the box adjoints (2 (order +
 *   1) + 2 words per box, in several copies that the wavefronts add into in
 *   turn and that are summed before the push-down, so that the atomics on the
 *   boxes near the root spread over more memory lines) and the per-particle
 *   direct-term sums (4 words per particle, likewise in copies).  The tree
 *   itself is only read, so adjoints on one tree may run concurrently on
 *   separate streams with separate workspaces.
 *   flags: GLM_RAYS_ORDERED, or GLM_RAYS_STAGED when glm_stage_rays staged
 *   these rays into the start of this workspace (a glm_shoot with the same
 *   workspace and flag may use them too), or 0.
 */
GLM_API glm_status glm_adjoint_workspace_bytes(const glm_tree* t, int64_t nrays, size_t* bytes);
GLM_API glm_status glm_shoot_adjoint(const glm_tree* t, const double* rx, const double* ry,
                             int64_t nrays, const float* ga1, const float* ga2, const float* gk,
                             const float* gg1, const float* gg2, double* dm, double* dx, double* dy,
                             double* ds, uint32_t flags, void* workspace, size_t workspace_bytes,
                             void* stream);

/* One lens of a batched walk. */
typedef struct {
    const glm_tree* tree; /* built tree; every tree of a batch has the same order and particle kind */
    const double* rx;     /* device FP64 ray positions, nrays each */
    const double* ry;
    int64_t nrays;        /* >= 0 */
    float* a1;            /* device FP32 outputs, input order; kappa/g1/g2 NULL with GLM_ALPHA_ONLY */
    float* a2;
    float* kappa;
    float* g1;
    float* g2;
} glm_lens_rays;

/* Bytes of device workspace for a batch with these ray counts (host array). */
GLM_API glm_status glm_shoot_batched_workspace_bytes(const int64_t* nrays, int nlens, size_t* bytes);

/*
 * Walk many independent lenses in ONE persistent launch (Sec. 3.3: the solver
 * parallelises over points, and bigger batches are more efficient): the rays
 * of every lens are Morton-sorted within their lens, cut into 64-ray groups,
 * and the wavefronts of one launch take (lens, group) items from a device
 * counter, lenses with the most expected work (rays x log2 particles) first.
 * Results equal glm_shoot per lens.  `lenses` is a HOST array of nlens
 * entries.  Copies the small lens table host->device (not graph-capturable).
 */
GLM_API glm_status glm_shoot_batched(const glm_lens_rays* lenses, int nlens, uint32_t flags,
                                     void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of device workspace for glm_refine_round on ncells cells. */
GLM_API glm_status glm_refine_workspace_bytes(int64_t ncells, size_t* bytes);

/*
 * One adaptive refinement round of a grid of square cells (Sec. 4: a cell is
 * refined by adding rays around its already shot centre ray, 3 x 3).
 *   cx, cy, side: device FP64 cell centres and sides, capacity >= ncells + 8 nrefine;
 *   kappa, g1, g2: device FP32 shot outputs of the ncells cells;
 * The nrefine cells with the largest side^2 (kappa^2 + g1^2 + g2^2) (ties: lower
 * index first) are split: their side becomes side/3 and 8 cells of side/3 are
 * appended at [ncells, ncells + 8 nrefine), 8 per refined cell in row order
 * (dy = -1, 0, 1; dx = -1, 0, 1; centre skipped).  The appended centres are
 * the new rays to shoot.  refined (device int32, nrefine, nullable) receives
 * the refined cells in rank order.  No host synchronisation, no memset:
 * capturable in a HIP graph.
 */
GLM_API glm_status glm_refine_round(double* cx, double* cy, double* side, const float* kappa,
                                    const float* g1, const float* g2, int64_t ncells, int64_t nrefine,
                                    int32_t* refined, void* workspace, size_t workspace_bytes,
                                    void* stream);

/*
 * Interpolation shortcut of refinement (Sec. 3.4).  The cells of a refined
 * grid form a nested grid: an nbase x nbase base grid of side h0 with
 * lower-left corner (x0, y0) at level 0, every split 3 x 3 one level deeper,
 * a cell named by its level l and integer coordinates (i, j) with centre
 * (x0 + (i + 1/2) h0 / 3^l, y0 + (j + 1/2) h0 / 3^l).  The caller-owned state
 * holds per cell its level and coordinates and a hash (l, i, j) -> cell.
 * Levels are supported while nbase * 3^l <= 2^28.
 */

/* Bytes of the interpolation state for grids of up to capacity cells. */
GLM_API glm_status glm_interp_state_bytes(int64_t capacity, size_t* bytes);

/* Bytes of device workspace for one glm_refine_interp_round. */
GLM_API glm_status glm_interp_round_workspace_bytes(int64_t ncells, int64_t nrefine, size_t* bytes);

/*
 * Index the base grid: the ncells cells centred at (cx, cy) (device FP64) are
 * cells of the base grid described above.  state: device buffer of at least
 * glm_interp_state_bytes(capacity); capacity >= the largest cell count the
 * rounds will reach.  No host synchronisation.
 */
GLM_API glm_status glm_interp_init(const double* cx, const double* cy, int64_t ncells, double x0, double y0,
                                   double h0, int64_t capacity, void* state, size_t state_bytes, void* stream);

/*
 * One refinement round with the interpolation shortcut.  Ranks and splits the
 * cells exactly as glm_refine_round (same cx, cy, side and `refined`).  Before
 * a cell is split, its neighbours (on each of the 8 sides the cell of the same
 * level, else the coarser cell covering that spot; none outside the grid) are
 * compared with it: if there is at least one and every neighbour's kappa, g1
 * and g2 differ from the cell's by at most tol (FP32 differences), the
 * magnification matrix is taken as uniform over the cell, and its 8 new
 * cells get, at their centres x (FP64 arithmetic, stored FP32),
 *   alpha = alpha_c + [[k + g1, g2], [g2, k - g1]] (x - x_c),
 *   kappa, g1, g2 = those of the cell,
 * in a1, a2, kappa, g1, g2 (device FP32, capacity).  The new cells of the
 * other refined cells are listed in shoot_idx (device int32, >= 8 nrefine), 8
 * per cell in rank order and row order, and their number is written to
 * *shoot_count (device int32): shoot them with glm_shoot_indexed.
 * 1 <= nrefine <= ncells, ncells + 8 nrefine <= capacity.  No host
 * synchronisation.
 */
GLM_API glm_status glm_refine_interp_round(double* cx, double* cy, double* side, float* a1, float* a2,
                                           float* kappa, float* g1, float* g2, int64_t ncells, int64_t nrefine,
                                           int64_t nbase, float tol, uint32_t flags, int32_t* refined,
                                           int32_t* shoot_idx, int32_t* shoot_count, int64_t capacity,
                                           void* state, size_t state_bytes, void* workspace,
                                           size_t workspace_bytes, void* stream);

/*
 * Deflection-only magnification matrix (App. A), for walks without kappa and
 * gamma.  For two neighbours P, Q of a cell c not collinear with its centre
 * (|det| > 1e-6 |u| |v|), with u = x_P - x_c, v = x_Q - x_c and s, t the
 * matching source-plane offsets (y = x - alpha), the magnification matrix
 * A = [[a11, a21], [a12, a22]] (y_1 = a11 x_1 + a21 x_2, y_2 = a12 x_1 + a22 x_2) is
 *   a11 = (v2 s1 - u2 t1)/det, a21 = (u1 t1 - v1 s1)/det,
 *   a12 = (v2 s2 - u2 t2)/det, a22 = (u1 t2 - v1 s2)/det,  det = u1 v2 - u2 v1
 * (FP64).  Neighbours as for glm_refine_interp_round.
 *
 * GLM_INTERP_DEFLECTIONS (flags of glm_refine_interp_round): a cell is
 * uniform if it has at least one such pair and every element of A agrees over
 * all pairs within tol; its new cells then get alpha = alpha_c + (I - A)(x - x_c)
 * with A the mean over the pairs, and kappa = 1 - (a11 + a22)/2,
 * g1 = (a22 - a11)/2, g2 = -(a12 + a21)/2.  kappa, g1, g2 of the cells are
 * still what ranks them.
 *
 * glm_interp_estimate writes those kappa, g1, g2 (from the mean A; 0 without a
 * pair) for the cells idx[0 .. min(*count, max_count)) -- the cells just walked
 * without kappa and gamma -- or, with idx NULL, for cells 0 .. max_count - 1
 * (count NULL reads as max_count).  No host synchronisation.
 */
#define GLM_INTERP_DEFLECTIONS 1u
GLM_API glm_status glm_interp_estimate(const double* cx, const double* cy, const float* a1, const float* a2,
                                       float* kappa, float* g1, float* g2, const int32_t* idx,
                                       const int32_t* count, int64_t max_count, int64_t nbase, int64_t capacity,
                                       const void* state, size_t state_bytes, void* stream);

/* Bytes of device workspace for glm_shoot_indexed of count rays. */
GLM_API glm_status glm_shoot_indexed_workspace_bytes(int64_t count, size_t* bytes);

/*
 * glm_shoot of the rays at (cx[idx[t]], cy[idx[t]]), t < count, with the
 * outputs written at index idx[t] of a1, a2, kappa, g1, g2 (device arrays
 * indexed like cx; kappa, g1, g2 unused with GLM_ALPHA_ONLY).  idx: device
 * int32, distinct indices.  workspace >= glm_shoot_indexed_workspace_bytes.
 */
GLM_API glm_status glm_shoot_indexed(const glm_tree* t, const double* cx, const double* cy, const int32_t* idx,
                                     int64_t count, float* a1, float* a2, float* kappa, float* g1, float* g2,
                                     uint32_t flags, void* workspace, size_t workspace_bytes, void* stream);

/* Message for the last non-OK status on this thread ("" if none). */
GLM_API const char* glm_last_error(void);

/* Library version string. */
GLM_API const char* glm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GLAMER_H */
