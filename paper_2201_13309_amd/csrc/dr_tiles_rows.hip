// Row-tile kernel instantiations for a single pass or the first pass of two.
#include "dr_device.h"

namespace dr {

hipError_t launch_rows_f32_single(const TileCfg& t, const ScanArgs& a, dim3 grid, hipStream_t s)
{
    DR_DISPATCH(t, rows_f32_kernel, false, grid, a, s);
    return hipGetLastError();
}

}  // namespace dr
