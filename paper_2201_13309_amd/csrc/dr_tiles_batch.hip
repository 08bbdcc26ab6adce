// Persistent batch kernel instantiations for single and first passes.
#include "dr_device.h"

namespace dr {

hipError_t launch_batch_f32_single(const TileCfg& t, const BatchArgs& a, dim3 grid, hipStream_t s)
{
    DR_DISPATCH(t, batch_f32_kernel, false, grid, a, s);
    return hipGetLastError();
}

}  // namespace dr
