// glm_shoot for callers that cannot allocate device memory: the ray workspace
// (ray sort keys and values, sorted ray copies, partial sums of split walks)
// is a file-scope device array instead of a caller buffer.  Each GPU the
// library runs on holds one copy of the array until the process ends; every
// call on that GPU shares it, so calls that overlap on one GPU (on different
// streams, or from different threads) race on it.
#include <mutex>
#include <string>

#include "walk.hpp"

namespace glm {

namespace {

constexpr size_t kScratchBytes = 128ull << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device, looked up once
// per device (the array's name is only a host-side stand-in in host code).
glm_status scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(GLM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GLM_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GLM_OK;
}

} // namespace

} // namespace glm

using namespace glm;

extern "C" glm_status glm_shoot_noalloc(const glm_tree* t, const double* rx, const double* ry, int64_t nrays,
                                        float* a1, float* a2, float* kappa, float* g1, float* g2, int32_t* counts,
                                        uint32_t flags, void* stream)
{
    if (nrays < 0 || nrays > GLM_NOALLOC_MAX_RAYS)
        return fail(GLM_EINVAL, "glm_shoot_noalloc takes at most GLM_NOALLOC_MAX_RAYS = " +
                                    std::to_string((long long)GLM_NOALLOC_MAX_RAYS) + " rays, got " +
                                    std::to_string((long long)nrays));
    if (flags & GLM_RAYS_STAGED) return fail(GLM_EINVAL, "GLM_RAYS_STAGED needs a caller workspace (glm_stage_rays)");
    const size_t need = ray_layout(nrays).bytes;
    if (need > kScratchBytes) return fail(GLM_EINVAL, "ray workspace exceeds the static scratch array");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    GLM_HIP(hipGetDevice(&dev));
    if (st) {
        int sdev = 0;
        GLM_HIP(hipStreamGetDevice(st, &sdev));
        if (sdev != dev) return fail(GLM_EINVAL, "stream belongs to another device than the current one");
    }
    void* ws = nullptr;
    glm_status rc = scratch_address(dev, &ws);
    if (rc != GLM_OK) return rc;
    return glm_shoot(t, rx, ry, nrays, a1, a2, kappa, g1, g2, counts, flags, ws, kScratchBytes, stream);
}
