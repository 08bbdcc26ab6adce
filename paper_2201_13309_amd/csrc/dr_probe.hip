// dr_probe.hip - streaming reference kernels for the benchmark (libdr_probe.so).
// Not part of the reconstruction: they move the same bytes as one
// reconstruction pass with nothing else to do (per element a uint16 read and a
// float written, non-temporal), so the benchmark can report the HBM rate plain
// kernels with the same 1:2 read:write mix reach on the box it runs on: in
// address order (16-byte accesses, grid-stride) and in the reconstruction's
// order (tiles of pixels walking the step and bin planes); and the read and
// the write half of the latter on their own.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void stream_kernel(const u32x4* __restrict__ in,
                                                     f32x4* __restrict__ out, int64_t n8)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n8; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(in + i);
        const f32x4 lo = {(float)(v.x & 0xffffu), (float)(v.x >> 16), (float)(v.y & 0xffffu),
                          (float)(v.y >> 16)};
        const f32x4 hi = {(float)(v.z & 0xffffu), (float)(v.z >> 16), (float)(v.w & 0xffffu),
                          (float)(v.w >> 16)};
        __builtin_nontemporal_store(lo, out + 2 * i);
        __builtin_nontemporal_store(hi, out + 2 * i + 1);
    }
}

// Same bytes in the reconstruction's order: one workgroup per tile of 512
// consecutive pixels, 2 per lane, walking all planes (steps in, bins out),
// with kRing loads in flight per lane (a ring consumed in place, as the
// reconstruction keeps its prefetch): a plain loop has one load in flight and
// measures the latency, not the memory system.
constexpr int kRing = 16;

__global__ __launch_bounds__(256) void planes_kernel(const unsigned int* __restrict__ in,
                                                     f32x2* __restrict__ out, int64_t plane2,
                                                     int planes)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;  // pixel pair
    if (j >= plane2) return;
    auto load = [&](int k) {
        return __builtin_nontemporal_load(in + (int64_t)min(k, planes - 1) * plane2 + j);
    };
    auto store = [&](int k, unsigned int v) {
        const f32x2 o = {(float)(v & 0xffffu), (float)(v >> 16)};
        __builtin_nontemporal_store(o, out + (int64_t)k * plane2 + j);
    };
    unsigned int r[kRing];
#pragma unroll
    for (int d = 0; d < kRing; ++d) r[d] = load(d);
    int k = 0;
    for (; k + kRing <= planes; k += kRing) {
#pragma unroll
        for (int d = 0; d < kRing; ++d) {
            store(k + d, r[d]);
            r[d] = load(k + d + kRing);
        }
    }
#pragma unroll
    for (int d = 0; d < kRing; ++d)
        if (k + d < planes) store(k + d, r[d]);
}

// The two halves of that traffic on their own, same order and access width:
// every plane of the input read (one sum per lane pair written at the end), and
// every plane of the output written.
__global__ __launch_bounds__(256) void planes_read_kernel(const unsigned int* __restrict__ in,
                                                          f32x2* __restrict__ out, int64_t plane2,
                                                          int planes)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= plane2) return;
    auto load = [&](int k) {
        return __builtin_nontemporal_load(in + (int64_t)min(k, planes - 1) * plane2 + j);
    };
    unsigned int r[kRing];
#pragma unroll
    for (int d = 0; d < kRing; ++d) r[d] = load(d);
    unsigned int a = 0u, b = 0u;
    int k = 0;
    for (; k + kRing <= planes; k += kRing) {
#pragma unroll
        for (int d = 0; d < kRing; ++d) {
            a += r[d] & 0xffffu;
            b += r[d] >> 16;
            r[d] = load(k + d + kRing);
        }
    }
#pragma unroll
    for (int d = 0; d < kRing; ++d)
        if (k + d < planes) {
            a += r[d] & 0xffffu;
            b += r[d] >> 16;
        }
    const f32x2 o = {(float)a, (float)b};
    __builtin_nontemporal_store(o, out + j);
}

__global__ __launch_bounds__(256) void planes_write_kernel(f32x2* __restrict__ out, int64_t plane2,
                                                           int planes)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= plane2) return;
    for (int k = 0; k < planes; ++k) {
        const f32x2 o = {(float)k, (float)j};
        __builtin_nontemporal_store(o, out + (int64_t)k * plane2 + j);
    }
}

}  // namespace

// out[i] = (float)in[i] for i < n.  in: device uint16 [n], out: device float
// [n], both 16-byte aligned, n a multiple of 8; groups: workgroups of 256
// lanes (<= 0: 8192).  Enqueued on `stream` (a hipStream_t, NULL = default).
// Returns 0, or -1 for bad arguments, or the HIP error code of the launch.
extern "C" int dr_probe_stream(const void* in, void* out, int64_t n, int groups, void* stream)
{
    if (!in || !out || n <= 0 || n % 8 != 0 || ((uintptr_t)in & 15) || ((uintptr_t)out & 15))
        return -1;
    const int64_t n8 = n / 8;
    int64_t g = groups > 0 ? groups : 8192;
    if (g > (n8 + 255) / 256) g = (n8 + 255) / 256;
    hipLaunchKernelGGL(stream_kernel, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4*)in, (f32x4*)out, n8);
    return (int)hipGetLastError();
}

// Same bytes, reconstruction order: out[k][p] = (float)in[k][p] for planes
// k < planes of `plane` elements (even), walked plane by plane within tiles of
// 512 pixels.  Alignment 8 bytes.  Returns as dr_probe_stream.
extern "C" int dr_probe_planes(const void* in, void* out, int64_t plane, int planes, void* stream)
{
    if (!in || !out || plane <= 0 || plane % 2 != 0 || planes <= 0 || ((uintptr_t)in & 7) ||
        ((uintptr_t)out & 7))
        return -1;
    const int64_t plane2 = plane / 2;
    hipLaunchKernelGGL(planes_kernel, dim3((unsigned)((plane2 + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, (const unsigned int*)in, (f32x2*)out, plane2, planes);
    return (int)hipGetLastError();
}

// The read half of dr_probe_planes: in[k][p] read for planes k < planes of
// `plane` elements, out[p] = per-pixel sum (float, plane elements written).
// The write half: out[k][p] written for every plane.  Same arguments,
// alignment and return values as dr_probe_planes (write: in unused).
extern "C" int dr_probe_planes_read(const void* in, void* out, int64_t plane, int planes,
                                    void* stream)
{
    if (!in || !out || plane <= 0 || plane % 2 != 0 || planes <= 0 || ((uintptr_t)in & 7) ||
        ((uintptr_t)out & 7))
        return -1;
    const int64_t plane2 = plane / 2;
    hipLaunchKernelGGL(planes_read_kernel, dim3((unsigned)((plane2 + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, (const unsigned int*)in, (f32x2*)out, plane2, planes);
    return (int)hipGetLastError();
}

extern "C" int dr_probe_planes_write(const void* in, void* out, int64_t plane, int planes,
                                     void* stream)
{
    (void)in;
    if (!out || plane <= 0 || plane % 2 != 0 || planes <= 0 || ((uintptr_t)out & 7)) return -1;
    const int64_t plane2 = plane / 2;
    hipLaunchKernelGGL(planes_write_kernel, dim3((unsigned)((plane2 + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, (f32x2*)out, plane2, planes);
    return (int)hipGetLastError();
}
