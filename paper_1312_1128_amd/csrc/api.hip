// C ABI of the gfx950 tree ray-shooting library (include/glamer.h): argument
// validation, handle and buffer ownership, error messages.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "walk.hpp"

namespace glm {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

glm_status fail(glm_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

static glm_status check_params(const glm_params* p)
{
    if (!p) return fail(GLM_EINVAL, "params is NULL");
    if (!(p->theta >= 0.0 && p->theta < 1.0)) return fail(GLM_EINVAL, "theta must be in [0, 1)");
    if (!(p->q > 0.0) || !isfinite(p->q)) return fail(GLM_EINVAL, "q must be finite and > 0");
    if (p->leaf_size < 1 || p->leaf_size > kMaxLeafSize) return fail(GLM_EINVAL, "leaf_size must be in 1..64");
    if (p->order < 0 || p->order > kMaxOrder) return fail(GLM_EINVAL, "order must be in 0..12");
    if (p->flags & ~(GLM_ALPHA_ONLY | GLM_FP32_ALPHA | GLM_RAYS_ORDERED | GLM_NFW_HALOS))
        return fail(GLM_EINVAL, "unknown flag bits");
    return GLM_OK;
}

} // namespace glm

struct glm_tree {
    glm::TreeStorage ts;
};

using namespace glm;

extern "C" {

const char* glm_last_error(void) { return g_err.c_str(); }

const char* glm_version(void) { return "glamer-gfx950 0.1"; }

glm_status glm_tree_create(glm_tree** out)
{
    if (!out) return fail(GLM_EINVAL, "out is NULL");
    *out = new (std::nothrow) glm_tree();
    if (!*out) return fail(GLM_ENOMEM, "host allocation failed");
    return GLM_OK;
}

void glm_tree_destroy(glm_tree* t) { delete t; }

glm_status glm_tree_workspace_bytes(int64_t n, const glm_params* params, size_t* bytes)
{
    if (!bytes) return fail(GLM_EINVAL, "bytes is NULL");
    glm_status rc = check_params(params);
    if (rc != GLM_OK) return rc;
    if (n < 1 || n > 0x7ffffff0) return fail(GLM_EINVAL, "n must be in 1 .. 2^31 - 16");
    *bytes = tree_particle_bytes(n) + tree_box_bytes(max_boxes(n, params->leaf_size), params->order);
    return GLM_OK;
}

glm_status glm_build_tree(glm_tree* t, const double* x, const double* y, const double* m, const double* s, int64_t n,
                          const glm_params* params, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!t) return fail(GLM_EINVAL, "tree handle is NULL");
    glm_status rc = check_params(params);
    if (rc != GLM_OK) return rc;
    if (!x || !y || !m) return fail(GLM_EINVAL, "x, y and m must be device pointers");
    if (n < 1 || n > 0x7ffffff0) return fail(GLM_EINVAL, "n must be in 1 .. 2^31 - 16");
    if (!workspace) return fail(GLM_EINVAL, "workspace must be a device pointer");
    t->ts.built = false;
    t->ts.ws = static_cast<char*>(workspace);
    t->ts.ws_bytes = workspace_bytes;
    return build_tree_device(t->ts, x, y, m, s, n, *params, static_cast<hipStream_t>(stream));
}

glm_status glm_tree_required_bytes(const glm_tree* t, size_t* bytes)
{
    if (!t || !bytes) return fail(GLM_EINVAL, "NULL argument");
    if (t->ts.need == 0) return fail(GLM_ESTATE, "no build has been attempted on this handle");
    *bytes = t->ts.need;
    return GLM_OK;
}

glm_status glm_tree_get_info(const glm_tree* t, glm_tree_info* out)
{
    if (!t || !out) return fail(GLM_EINVAL, "NULL argument");
    if (!t->ts.built) return fail(GLM_ESTATE, "tree not built");
    BuildSync hs;
    GLM_HIP(hipDeviceSynchronize());
    GLM_HIP(hipMemcpy(&hs, t->ts.sync, sizeof(hs), hipMemcpyDeviceToHost));
    out->n = t->ts.n;
    out->ncells = t->ts.ncells;
    out->nleaves = hs.nleaves;
    out->nlisted = hs.nlisted;
    out->max_level = hs.max_level;
    out->order = t->ts.params.order;
    out->check_flags = hs.internal;
    out->reserved = 0;
    out->root_x0 = t->ts.x0;
    out->root_y0 = t->ts.y0;
    out->root_side = t->ts.side;
    out->device_bytes = t->ts.need;
    return GLM_OK;
}

glm_status glm_tree_export(const glm_tree* t, int32_t* level, uint32_t* ix, uint32_t* iy, int32_t* beg, int32_t* end,
                           int32_t* next, int32_t* leaf, int32_t* lbeg, int32_t* lend, double* M, double* cx,
                           double* cy, double* rcut2, double* Q, int32_t* perm, uint64_t* key, int32_t* list_idx)
{
    if (!t) return fail(GLM_EINVAL, "tree handle is NULL");
    if (!t->ts.built) return fail(GLM_ESTATE, "tree not built");
    const TreeStorage& ts = t->ts;
    const size_t nc = (size_t)ts.ncells, n = (size_t)ts.n;
    GLM_HIP(hipDeviceSynchronize());
    auto cp = [](void* dst, const void* src, size_t bytes) -> hipError_t {
        return dst ? hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) : hipSuccess;
    };
    GLM_HIP(cp(level, ts.b.level, 4 * nc));
    GLM_HIP(cp(ix, ts.b.ix, 4 * nc));
    GLM_HIP(cp(iy, ts.b.iy, 4 * nc));
    GLM_HIP(cp(beg, ts.b.beg, 4 * nc));
    GLM_HIP(cp(end, ts.b.end, 4 * nc));
    GLM_HIP(cp(next, ts.b.next, 4 * nc));
    GLM_HIP(cp(leaf, ts.b.leaf, 4 * nc));
    GLM_HIP(cp(lbeg, ts.b.lbeg, 4 * nc));
    GLM_HIP(cp(lend, ts.b.lend, 4 * nc));
    GLM_HIP(cp(M, ts.dev.cM, 8 * nc));
    GLM_HIP(cp(cx, ts.ccx, 8 * nc));
    GLM_HIP(cp(cy, ts.ccy, 8 * nc));
    GLM_HIP(cp(Q, ts.dev.cq, 16 * nc * (size_t)(ts.params.order + 1)));
    GLM_HIP(cp(perm, ts.perm, 4 * n));
    GLM_HIP(cp(key, ts.key, 8 * n));
    if (rcut2) {
        std::vector<CellHdr> h(nc);
        GLM_HIP(hipMemcpy(h.data(), ts.dev.hdr, sizeof(CellHdr) * nc, hipMemcpyDeviceToHost));
        for (size_t c = 0; c < nc; ++c) rcut2[c] = h[c].rcut2;
    }
    if (list_idx) {
        BuildSync hs;
        GLM_HIP(hipMemcpy(&hs, ts.sync, sizeof(hs), hipMemcpyDeviceToHost));
        std::vector<PRec> l((size_t)hs.nlisted);
        if (hs.nlisted > 0)
            GLM_HIP(hipMemcpy(l.data(), ts.dev.lst, sizeof(PRec) * l.size(), hipMemcpyDeviceToHost));
        std::vector<int32_t> pm((size_t)n);
        GLM_HIP(hipMemcpy(pm.data(), ts.perm, 4 * n, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < l.size(); ++k) list_idx[k] = pm[l[k].meta & 0x7fffffffu];
    }
    return GLM_OK;
}

glm_status glm_tree_knn(const glm_tree* t, int32_t k, double* s_out, void* stream)
{
    if (!t || !s_out) return fail(GLM_EINVAL, "NULL argument");
    if (!t->ts.built) return fail(GLM_ESTATE, "tree not built");
    if (k < 1 || k > 64) return fail(GLM_EINVAL, "k must be in 1..64");
    if ((int64_t)k > (int64_t)t->ts.n - 1) return fail(GLM_EINVAL, "k must be at most n - 1");
    return knn_device(t->ts, k, s_out, static_cast<hipStream_t>(stream));
}

glm_status glm_shoot_workspace_bytes(int64_t nrays, size_t* bytes)
{
    if (!bytes || nrays < 0) return fail(GLM_EINVAL, "bad argument");
    *bytes = ray_layout(nrays).bytes;
    return GLM_OK;
}

glm_status glm_shoot(const glm_tree* t, const double* rx, const double* ry, int64_t nrays, float* a1, float* a2,
                     float* kappa, float* g1, float* g2, int32_t* counts, uint32_t flags, void* workspace,
                     size_t workspace_bytes, void* stream)
{
    if (!t) return fail(GLM_EINVAL, "tree handle is NULL");
    if (!t->ts.built) return fail(GLM_ESTATE, "tree not built");
    if (nrays < 0 || nrays > 0x7fffff00) return fail(GLM_EINVAL, "nrays must be in 0 .. 2^31 - 256");
    if (nrays == 0) return GLM_OK;
    if (!rx || !ry || !a1 || !a2) return fail(GLM_EINVAL, "rx, ry, a1, a2 must be device pointers");
    if (flags & ~(GLM_ALPHA_ONLY | GLM_FP32_ALPHA | GLM_RAYS_ORDERED | GLM_RAYS_STAGED))
        return fail(GLM_EINVAL, "unknown flag bits");
    if ((flags & GLM_RAYS_ORDERED) && (flags & GLM_RAYS_STAGED))
        return fail(GLM_EINVAL, "GLM_RAYS_ORDERED and GLM_RAYS_STAGED exclude each other");
    flags |= t->ts.params.flags;
    if (!(flags & GLM_ALPHA_ONLY) && (!kappa || !g1 || !g2))
        return fail(GLM_EINVAL, "kappa, g1, g2 are required unless GLM_ALPHA_ONLY");
    {
        const size_t need = ray_layout(nrays).bytes;
        if (!workspace || workspace_bytes < need)
            return fail(GLM_ENOMEM, "workspace smaller than glm_shoot_workspace_bytes(nrays) = " + std::to_string(need));
    }
    return shoot_device(t->ts, rx, ry, nrays, a1, a2, kappa, g1, g2, counts, flags, workspace,
                        static_cast<hipStream_t>(stream));
}

glm_status glm_stage_rays(const double* rx, const double* ry, int64_t nrays, void* workspace, size_t workspace_bytes,
                          void* stream)
{
    if (nrays < 0 || nrays > 0x7fffff00) return fail(GLM_EINVAL, "nrays must be in 0 .. 2^31 - 256");
    if (nrays == 0) return GLM_OK;
    if (!rx || !ry) return fail(GLM_EINVAL, "rx, ry must be device pointers");
    const RayLayout L = ray_layout(nrays);
    if (!workspace || workspace_bytes < L.bytes)
        return fail(GLM_ENOMEM, "workspace smaller than glm_shoot_workspace_bytes(nrays) = " + std::to_string(L.bytes));
    StagedRays sr{};
    return stage_rays(rx, ry, nrays, workspace, L, &sr, static_cast<hipStream_t>(stream));
}

glm_status glm_shoot_potential(const glm_tree* t, const double* rx, const double* ry, int64_t nrays, float* a1,
                               float* a2, float* psi, float* tdelay, uint32_t flags, void* workspace,
                               size_t workspace_bytes, void* stream)
{
    if (!t) return fail(GLM_EINVAL, "tree handle is NULL");
    if (!t->ts.built) return fail(GLM_ESTATE, "tree not built");
    if (nrays < 0 || nrays > 0x7fffff00) return fail(GLM_EINVAL, "nrays must be in 0 .. 2^31 - 256");
    if (nrays == 0) return GLM_OK;
    if (!rx || !ry || !a1 || !a2 || !psi) return fail(GLM_EINVAL, "rx, ry, a1, a2, psi must be device pointers");
    if (flags & ~GLM_RAYS_ORDERED) return fail(GLM_EINVAL, "unknown flag bits");
    const size_t need = ray_layout(nrays).bytes;
    if (!workspace || workspace_bytes < need)
        return fail(GLM_ENOMEM, "workspace smaller than glm_shoot_workspace_bytes(nrays) = " + std::to_string(need));
    return potential_device(t->ts, rx, ry, nrays, a1, a2, psi, tdelay, flags, workspace,
                            static_cast<hipStream_t>(stream));
}

glm_status glm_knn_workspace_bytes(int64_t n, int32_t with_species, size_t* bytes)
{
    if (!bytes || n < 0 || n > 0x7fffffff) return fail(GLM_EINVAL, "bad argument");
    *bytes = knn_workspace_bytes(n, with_species != 0);
    return GLM_OK;
}

glm_status glm_knn(const double* x, const double* y, const double* z, const int32_t* species, int64_t n, int32_t k,
                   double* s_out, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!x || !y || !s_out) return fail(GLM_EINVAL, "x, y, s_out must be device pointers");
    if (n < 2 || n > 0x7fffffff) return fail(GLM_EINVAL, "n must be in 2 .. 2^31 - 1");
    if (k < 1 || k > 64 || k > n - 1) return fail(GLM_EINVAL, "k must be in 1 .. min(64, n - 1)");
    const size_t need = knn_workspace_bytes(n, species != nullptr);
    if (!workspace || workspace_bytes < need)
        return fail(GLM_ENOMEM, "workspace smaller than glm_knn_workspace_bytes = " + std::to_string(need));
    return knn_positions_device(x, y, z, species, n, k, s_out, workspace, static_cast<hipStream_t>(stream));
}

glm_status glm_shoot_direct(const double* x, const double* y, const double* m, const double* s, int64_t n, double q,
                            const double* rx, const double* ry, int64_t nrays, int fp64, void* const out5[5],
                            void* stream)
{
    if (!x || !y || !m || !rx || !ry || !out5 || !out5[0] || !out5[1])
        return fail(GLM_EINVAL, "NULL device pointer");
    if (n < 1 || n > 0x7ffffff0) return fail(GLM_EINVAL, "n must be in 1 .. 2^31 - 16");
    if (nrays < 0 || nrays > 0x7fffff00) return fail(GLM_EINVAL, "nrays out of range");
    if (!(q > 0.0) || !isfinite(q)) return fail(GLM_EINVAL, "q must be finite and > 0");
    return direct_device(x, y, m, s, n, q, kKindGauss, rx, ry, nrays, fp64, out5, static_cast<hipStream_t>(stream));
}

glm_status glm_shoot_direct_nfw(const double* x, const double* y, const double* m, const double* R, int64_t n,
                                double c, const double* rx, const double* ry, int64_t nrays, int fp64,
                                void* const out5[5], void* stream)
{
    if (!x || !y || !m || !R || !rx || !ry || !out5 || !out5[0] || !out5[1])
        return fail(GLM_EINVAL, "NULL device pointer");
    if (n < 1 || n > 0x7ffffff0) return fail(GLM_EINVAL, "n must be in 1 .. 2^31 - 16");
    if (nrays < 0 || nrays > 0x7fffff00) return fail(GLM_EINVAL, "nrays out of range");
    if (!(c > 0.0) || !isfinite(c)) return fail(GLM_EINVAL, "c must be finite and > 0");
    return direct_device(x, y, m, R, n, c, kKindNfw, rx, ry, nrays, fp64, out5, static_cast<hipStream_t>(stream));
}

glm_status glm_adjoint_workspace_bytes(const glm_tree* t, int64_t nrays, size_t* bytes)
{
    if (!t || !bytes) return fail(GLM_EINVAL, "NULL argument");
    if (!t->ts.built) return fail(GLM_ESTATE, "tree not built");
    if (nrays < 0 || nrays > 0x7fffff00) return fail(GLM_EINVAL, "nrays out of range");
    *bytes = adjoint_workspace_bytes(t->ts, nrays);
    return GLM_OK;
}

glm_status glm_shoot_adjoint(const glm_tree* t, const double* rx, const double* ry, int64_t nrays, const float* ga1,
                             const float* ga2, const float* gk, const float* gg1, const float* gg2, double* dm,
                             double* dx, double* dy, double* ds, uint32_t flags, void* workspace,
                             size_t workspace_bytes, void* stream)
{
    if (!t) return fail(GLM_EINVAL, "tree handle is NULL");
    if (!t->ts.built) return fail(GLM_ESTATE, "tree not built");
    if (nrays < 0 || nrays > 0x7fffff00) return fail(GLM_EINVAL, "nrays out of range");
    if (nrays == 0) return GLM_OK;
    if (!rx || !ry) return fail(GLM_EINVAL, "rx, ry must be device pointers");
    if (!ga1 && !ga2 && !gk && !gg1 && !gg2) return fail(GLM_EINVAL, "every cotangent is NULL");
    if (flags & ~(GLM_FP32_ALPHA | GLM_RAYS_ORDERED | GLM_ALPHA_ONLY | GLM_RAYS_STAGED))
        return fail(GLM_EINVAL, "unknown flag bits");
    if ((flags & GLM_RAYS_ORDERED) && (flags & GLM_RAYS_STAGED))
        return fail(GLM_EINVAL, "GLM_RAYS_ORDERED and GLM_RAYS_STAGED exclude each other");
    {
        const size_t need = adjoint_workspace_bytes(t->ts, nrays);
        if (!workspace || workspace_bytes < need)
            return fail(GLM_ENOMEM, "workspace smaller than glm_adjoint_workspace_bytes(tree, nrays) = " +
                                        std::to_string(need));
    }
    return adjoint_device(t->ts, rx, ry, nrays, ga1, ga2, gk, gg1, gg2, dm, dx, dy, ds, flags, workspace,
                          static_cast<hipStream_t>(stream));
}

glm_status glm_shoot_batched_workspace_bytes(const int64_t* nrays, int nlens, size_t* bytes)
{
    if (!nrays || !bytes || nlens < 1 || nlens > 4096) return fail(GLM_EINVAL, "bad argument");
    int64_t total = 0;
    for (int l = 0; l < nlens; ++l) {
        if (nrays[l] < 0) return fail(GLM_EINVAL, "negative ray count");
        total += nrays[l];
    }
    if (total > 0x7fffff00) return fail(GLM_EINVAL, "too many rays in one batch");
    *bytes = batch_workspace_bytes(nlens, total);
    return GLM_OK;
}

glm_status glm_shoot_batched(const glm_lens_rays* lenses, int nlens, uint32_t flags, void* workspace,
                             size_t workspace_bytes, void* stream)
{
    if (!lenses || nlens < 1 || nlens > 4096) return fail(GLM_EINVAL, "lenses must hold 1..4096 entries");
    if (flags & ~(GLM_ALPHA_ONLY | GLM_FP32_ALPHA)) return fail(GLM_EINVAL, "unknown flag bits");
    std::vector<int64_t> counts(nlens);
    std::vector<std::pair<double, int>> rank(nlens);
    int order = -1;
    int64_t total = 0;
    for (int l = 0; l < nlens; ++l) {
        const glm_lens_rays& e = lenses[l];
        if (!e.tree || !e.tree->ts.built) return fail(GLM_ESTATE, "lens " + std::to_string(l) + ": tree not built");
        if (e.nrays < 0) return fail(GLM_EINVAL, "lens " + std::to_string(l) + ": negative ray count");
        if (e.nrays > 0 && (!e.rx || !e.ry || !e.a1 || !e.a2))
            return fail(GLM_EINVAL, "lens " + std::to_string(l) + ": NULL ray or output pointer");
        if (e.nrays > 0 && !(flags & GLM_ALPHA_ONLY) && (!e.kappa || !e.g1 || !e.g2))
            return fail(GLM_EINVAL, "lens " + std::to_string(l) + ": kappa, g1, g2 required unless GLM_ALPHA_ONLY");
        const int p = e.tree->ts.params.order;
        if (order >= 0 && p != order) return fail(GLM_EINVAL, "all trees of a batch must have the same order");
        if (l > 0 && e.tree->ts.dev.kind != lenses[0].tree->ts.dev.kind)
            return fail(GLM_EINVAL, "all trees of a batch must hold the same particle kind");
        order = p;
        counts[l] = e.nrays;
        total += e.nrays;
        rank[l] = {-(double)e.nrays * log2((double)e.tree->ts.n + 1.0), l};
    }
    if (total > 0x7fffff00) return fail(GLM_EINVAL, "too many rays in one batch");
    const size_t need = batch_workspace_bytes(nlens, total);
    if (!workspace || workspace_bytes < need)
        return fail(GLM_ENOMEM, "workspace smaller than glm_shoot_batched_workspace_bytes = " + std::to_string(need));
    std::stable_sort(rank.begin(), rank.end());
    std::vector<BatchLens> tab(nlens);
    for (int r = 0; r < nlens; ++r) {
        const glm_lens_rays& e = lenses[rank[r].second];
        BatchLens& b = tab[r];
        b.tree = e.tree->ts.dev;
        b.nrays = e.nrays;
        b.ray_off = 0;
        b.rx = e.rx;
        b.ry = e.ry;
        b.out = WalkOut{e.a1, e.a2, (flags & GLM_ALPHA_ONLY) ? nullptr : e.kappa,
                        (flags & GLM_ALPHA_ONLY) ? nullptr : e.g1, (flags & GLM_ALPHA_ONLY) ? nullptr : e.g2, nullptr};
    }
    return shoot_batched_device(tab.data(), nlens, order, flags, workspace, static_cast<hipStream_t>(stream));
}

glm_status glm_refine_workspace_bytes(int64_t ncells, size_t* bytes)
{
    if (!bytes || ncells < 0 || ncells > 0x7fffff00) return fail(GLM_EINVAL, "bad argument");
    *bytes = refine_workspace_bytes(ncells);
    return GLM_OK;
}

glm_status glm_refine_round(double* cx, double* cy, double* side, const float* kappa, const float* g1, const float* g2,
                            int64_t ncells, int64_t nrefine, int32_t* refined, void* workspace, size_t workspace_bytes,
                            void* stream)
{
    if (!cx || !cy || !side || !kappa || !g1 || !g2) return fail(GLM_EINVAL, "NULL device pointer");
    if (ncells < 1 || ncells > 0x7fffff00) return fail(GLM_EINVAL, "ncells out of range");
    if (nrefine < 0 || nrefine > ncells) return fail(GLM_EINVAL, "nrefine must be in 0..ncells");
    if (ncells + 8 * nrefine > 0x7fffff00) return fail(GLM_EINVAL, "too many cells");
    const size_t need = refine_workspace_bytes(ncells);
    if (!workspace || workspace_bytes < need)
        return fail(GLM_ENOMEM, "workspace smaller than glm_refine_workspace_bytes = " + std::to_string(need));
    return refine_round_device(cx, cy, side, kappa, g1, g2, ncells, nrefine, refined, workspace,
                               static_cast<hipStream_t>(stream));
}

glm_status glm_interp_state_bytes(int64_t capacity, size_t* bytes)
{
    if (!bytes || capacity < 1 || capacity > 0x7fffff00) return fail(GLM_EINVAL, "bad argument");
    *bytes = interp_layout(capacity).bytes;
    return GLM_OK;
}

glm_status glm_interp_round_workspace_bytes(int64_t ncells, int64_t nrefine, size_t* bytes)
{
    if (!bytes || ncells < 1 || nrefine < 0 || nrefine > ncells || ncells > 0x7fffff00)
        return fail(GLM_EINVAL, "bad argument");
    *bytes = interp_round_workspace_bytes(ncells, nrefine);
    return GLM_OK;
}

glm_status glm_interp_init(const double* cx, const double* cy, int64_t ncells, double x0, double y0, double h0,
                           int64_t capacity, void* state, size_t state_bytes, void* stream)
{
    if (!cx || !cy || !state) return fail(GLM_EINVAL, "NULL device pointer");
    if (ncells < 1 || capacity < ncells || capacity > 0x7fffff00) return fail(GLM_EINVAL, "need 1 <= ncells <= capacity");
    if (!(h0 > 0.0) || !isfinite(h0) || !isfinite(x0) || !isfinite(y0)) return fail(GLM_EINVAL, "bad base grid");
    const size_t need = interp_layout(capacity).bytes;
    if (state_bytes < need) return fail(GLM_ENOMEM, "state smaller than glm_interp_state_bytes = " + std::to_string(need));
    return interp_init_device(cx, cy, ncells, x0, y0, h0, capacity, state, static_cast<hipStream_t>(stream));
}

glm_status glm_refine_interp_round(double* cx, double* cy, double* side, float* a1, float* a2, float* kappa,
                                   float* g1, float* g2, int64_t ncells, int64_t nrefine, int64_t nbase, float tol,
                                   uint32_t flags, int32_t* refined, int32_t* shoot_idx, int32_t* shoot_count,
                                   int64_t capacity, void* state, size_t state_bytes, void* workspace,
                                   size_t workspace_bytes, void* stream)
{
    if (flags & ~GLM_INTERP_DEFLECTIONS) return fail(GLM_EINVAL, "unknown flag bits");
    if (!cx || !cy || !side || !a1 || !a2 || !kappa || !g1 || !g2 || !shoot_idx || !shoot_count || !state)
        return fail(GLM_EINVAL, "NULL device pointer");
    if (ncells < 1 || nrefine < 0 || nrefine > ncells) return fail(GLM_EINVAL, "need 0 <= nrefine <= ncells");
    if (ncells + 8 * nrefine > capacity || capacity > 0x7fffff00) return fail(GLM_EINVAL, "capacity too small");
    if (nbase < 1 || nbase > (1 << 28)) return fail(GLM_EINVAL, "nbase out of range");
    if (!(tol >= 0.0f) || !isfinite(tol)) return fail(GLM_EINVAL, "tol must be finite and >= 0");
    const size_t sneed = interp_layout(capacity).bytes;
    if (state_bytes < sneed) return fail(GLM_ENOMEM, "state smaller than glm_interp_state_bytes = " + std::to_string(sneed));
    const size_t need = interp_round_workspace_bytes(ncells, nrefine);
    if (!workspace || workspace_bytes < need)
        return fail(GLM_ENOMEM, "workspace smaller than glm_interp_round_workspace_bytes = " + std::to_string(need));
    if (nrefine == 0) return fail(GLM_EINVAL, "nrefine must be >= 1");
    return interp_round_device(cx, cy, side, a1, a2, kappa, g1, g2, ncells, nrefine, nbase, tol,
                               (flags & GLM_INTERP_DEFLECTIONS) != 0, refined, shoot_idx, shoot_count, capacity, state,
                               workspace, static_cast<hipStream_t>(stream));
}

glm_status glm_interp_estimate(const double* cx, const double* cy, const float* a1, const float* a2, float* kappa,
                               float* g1, float* g2, const int32_t* idx, const int32_t* count, int64_t max_count,
                               int64_t nbase, int64_t capacity, const void* state, size_t state_bytes, void* stream)
{
    if (!cx || !cy || !a1 || !a2 || !kappa || !g1 || !g2 || !state) return fail(GLM_EINVAL, "NULL device pointer");
    if (max_count < 0 || max_count > capacity || capacity > 0x7fffff00) return fail(GLM_EINVAL, "max_count out of range");
    if (nbase < 1 || nbase > (1 << 28)) return fail(GLM_EINVAL, "nbase out of range");
    const size_t sneed = interp_layout(capacity).bytes;
    if (state_bytes < sneed) return fail(GLM_ENOMEM, "state smaller than glm_interp_state_bytes = " + std::to_string(sneed));
    return interp_estimate_device(cx, cy, a1, a2, kappa, g1, g2, idx, count, max_count, nbase, capacity, state,
                                  static_cast<hipStream_t>(stream));
}

glm_status glm_shoot_indexed_workspace_bytes(int64_t count, size_t* bytes)
{
    if (!bytes || count < 0 || count > 0x7fffff00) return fail(GLM_EINVAL, "bad argument");
    *bytes = shoot_indexed_workspace_bytes(count);
    return GLM_OK;
}

glm_status glm_shoot_indexed(const glm_tree* t, const double* cx, const double* cy, const int32_t* idx, int64_t count,
                             float* a1, float* a2, float* kappa, float* g1, float* g2, uint32_t flags, void* workspace,
                             size_t workspace_bytes, void* stream)
{
    if (!t) return fail(GLM_EINVAL, "tree handle is NULL");
    if (!t->ts.built) return fail(GLM_ESTATE, "tree not built");
    if (count < 0 || count > 0x7fffff00) return fail(GLM_EINVAL, "count out of range");
    if (count == 0) return GLM_OK;
    if (!cx || !cy || !idx || !a1 || !a2) return fail(GLM_EINVAL, "NULL device pointer");
    if (flags & ~(GLM_ALPHA_ONLY | GLM_FP32_ALPHA)) return fail(GLM_EINVAL, "unknown flag bits");
    flags |= t->ts.params.flags;
    if (!(flags & GLM_ALPHA_ONLY) && (!kappa || !g1 || !g2))
        return fail(GLM_EINVAL, "kappa, g1, g2 are required unless GLM_ALPHA_ONLY");
    const size_t need = shoot_indexed_workspace_bytes(count);
    if (!workspace || workspace_bytes < need)
        return fail(GLM_ENOMEM, "workspace smaller than glm_shoot_indexed_workspace_bytes = " + std::to_string(need));
    return shoot_indexed_device(t->ts, cx, cy, idx, count, a1, a2, kappa, g1, g2, flags, workspace,
                                static_cast<hipStream_t>(stream));
}

} // extern "C"
