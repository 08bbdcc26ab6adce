// Reconstruction without allocation: the scratch of a device-image
// reconstruction (per-wave partial totals and the totals workspace) taken
// from one fixed device array instead of the geometry's lazily grown buffers,
// for callers that cannot call hipMalloc (graph capture, tight serving loops).
//
// The array is a file-scope __device__ object: every GPU that loads this
// library holds its own copy, at its own address, until the process ends.  In
// host code its name is only a host-side stand-in, so its device address is
// looked up once per device (with that device current) when a context is
// created, and only that address is passed to kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "dr_runtime.h"

namespace dr {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex scratch_mu;
static void* scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the calling thread's current
// device must be `device`); looked up once per device.
dr_status noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return set_error(DR_E_UNSUPPORTED, "noalloc scratch: device index beyond the table");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_ptr[device]) return DR_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(DR_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    scratch_ptr[device] = p;
    return DR_OK;
}

static void* scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    return scratch_ptr[device];
}

size_t noalloc_scratch_need(const dr_geom g, const TileCfg& t, bool totals)
{
    return totals ? partials_bytes(g, t) + totals_work_bytes(g) : 0;
}

}  // namespace dr

using namespace dr;

extern "C" dr_status dr_reconstruct_noalloc(dr_geom g, const uint16_t* images_dev, float* out,
                                            float* totals, void* stream)
{
    if (!g || !images_dev || !out)
        return set_error(DR_E_INVAL, "dr_reconstruct_noalloc: NULL argument");
    auto misaligned = [](const void* p, uintptr_t a) {
        return (reinterpret_cast<uintptr_t>(p) % a) != 0;
    };
    if (misaligned(out, 4) || (totals && misaligned(totals, 4)) || misaligned(images_dev, 2))
        return set_error(DR_E_INVAL, "dr_reconstruct_noalloc: misaligned buffer");
    DR_HIP(hipSetDevice(g->ctx->device));
    const TileCfg t = choose_tile(g, images_dev, out);
    const size_t need = noalloc_scratch_need(g, t, totals != nullptr);
    if (need > kNoAllocScratchBytes)
        return set_error(DR_E_INVAL,
                         "dr_reconstruct_noalloc: this scan's totals need " +
                             std::to_string(need) + " bytes of scratch, more than the fixed " +
                             std::to_string(kNoAllocScratchBytes) +
                             " (pass totals = NULL, or use dr_reconstruct)");
    unsigned char* base = static_cast<unsigned char*>(scratch_of(g->ctx->device));
    if (!base)
        return set_error(DR_E_DEVICE, "dr_reconstruct_noalloc: scratch address not looked up");
    float* part = totals ? reinterpret_cast<float*>(base) : nullptr;
    double* work = totals ? reinterpret_cast<double*>(base + partials_bytes(g, t)) : nullptr;
    const dr_status st = reconstruct_device_into(g, t, images_dev, out, totals, part, work,
                                                 (hipStream_t)stream);
    if (st != DR_OK) return st;
    set_error(DR_OK, "");
    return DR_OK;
}
