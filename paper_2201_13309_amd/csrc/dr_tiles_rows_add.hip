// Row-tile kernel instantiations for the second pass of two, which adds onto
// the first pass's output.
#include "dr_device.h"

namespace dr {

hipError_t launch_rows_f32_add(const TileCfg& t, const ScanArgs& a, dim3 grid, hipStream_t s)
{
    DR_DISPATCH(t, rows_f32_kernel, true, grid, a, s);
    return hipGetLastError();
}

}  // namespace dr
