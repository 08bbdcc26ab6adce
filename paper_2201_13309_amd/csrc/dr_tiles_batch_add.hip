// Persistent batch kernel instantiations for second passes.
#include "dr_device.h"

namespace dr {

hipError_t launch_batch_f32_add(const TileCfg& t, const BatchArgs& a, dim3 grid, hipStream_t s)
{
    DR_DISPATCH(t, batch_f32_kernel, true, grid, a, s);
    return hipGetLastError();
}

}  // namespace dr
