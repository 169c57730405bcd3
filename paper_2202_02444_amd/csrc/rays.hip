// Ray casting (Procedure 2): filled in by the persistent ray-march kernel.
#include "spk_impl.h"

namespace spk {

spk_status launch_rays(const spk_net*, const spk_ray_params&, int64_t, const float*, const float*, float*, int32_t*,
                       hipStream_t, int) {
  return SPK_E_UNSUPPORTED;
}

}  // namespace spk
