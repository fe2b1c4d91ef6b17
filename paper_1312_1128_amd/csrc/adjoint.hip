// Adjoint tree walk (placeholder until the backward walk lands).
#include "walk.hpp"

namespace glm {

glm_status adjoint_device(TreeStorage&, const double*, const double*, int64_t, const float*, const float*, double*,
                          double*, double*, double*, uint32_t, void*, hipStream_t)
{
    return fail(GLM_ESTATE, "shoot_adjoint is not available in this build");
}

} // namespace glm
