// Pixel activity and top-k pixel selection (gfx950), for reconstructing a
// chosen fraction of the detector (the paper's second experiment, Sec. IV,
// processes a percentage of the pixels without stating which).
//
// Rule: the activity of a pixel is A = sum_k |I_k - I_{k+1}| over its samples
// (exact, 64-bit integers); the top-k selection keeps the k pixels of largest
// A, ties going to the lower pixel index, listed in increasing pixel index.
//
//   activity_kernel    one pass over the stack, 4 pixels per lane (8-byte
//                      loads) when aligned, 16 loads in flight per lane;
//                      HBM-bound.
//   select_hist/pick   radix select of the k-th largest activity, 8 bits per
//                      pass from the top, with the state kept on the device;
//                      digits above the top bit of the OR of all keys
//                      (select_or) are 0 in every key and are skipped.
//   select_reduce /    two-level scan of the packed counts (greater, equal)
//   scan / scatter     and a scatter of the selected indices in index order.
#include "dr_device.h"

namespace dr {

template <int PPL>
__global__ __launch_bounds__(256) void activity_kernel(const uint16_t* img, int64_t npix,
                                                       int n_steps, uint64_t* act)
{
    using V = typename U16V<PPL>::T;
    const int64_t p0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * PPL;
    if (p0 >= npix) return;
    uint64_t acc[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) acc[q] = 0;
    auto at = [&](int k) { return stream_load((const V*)(img + (int64_t)k * npix + p0)); };
    auto add = [&](const V& prev, const V& cur) {
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int d = pix<PPL>(prev, q) - pix<PPL>(cur, q);
            acc[q] += (uint64_t)(uint32_t)(d < 0 ? -d : d);
        }
    };
    // a ring of U samples in registers, U loads in flight: slot i holds step
    // k + i at the start of each block of U steps (only steps below n_steps
    // are loaded; the condition is the same for every lane)
    constexpr int U = 16;
    V ring[U];
    V prev = at(0);
#pragma unroll
    for (int i = 0; i < U; ++i)
        if (1 + i < n_steps) ring[i] = at(1 + i);
    int k = 1;
    for (; k + U <= n_steps; k += U) {
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const V cur = ring[i];
            if (k + i + U < n_steps) ring[i] = at(k + i + U);
            add(prev, cur);
            prev = cur;
        }
    }
#pragma unroll
    for (int i = 0; i < U; ++i)
        if (k + i < n_steps) {
            add(prev, ring[i]);
            prev = ring[i];
        }
#pragma unroll
    for (int q = 0; q < PPL; ++q) act[p0 + q] = acc[q];
}

__global__ void select_init_kernel(SelectState* st, int64_t k)
{
    const int t = threadIdx.x;
    st->hist[t] = 0;
    if (t == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->need = k;
        st->above = 0;
        st->bits = 0;
    }
}

// OR of all keys into st->bits
__global__ __launch_bounds__(256) void select_or_kernel(const uint64_t* act, int64_t npix,
                                                        SelectState* st)
{
    __shared__ unsigned long long red;
    if (threadIdx.x == 0) red = 0;
    __syncthreads();
    unsigned long long v = 0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * 256)
        v |= act[p];
    if (v) atomicOr(&red, v);
    __syncthreads();
    if (threadIdx.x == 0 && red) atomicOr(&st->bits, red);
}

// Digit `shift` is 0 in every key when no key has a bit at or above it: its
// pass would find every remaining key in bucket 0 and leave the state as it
// is (the prefix keeps a 0 there, the count above and the need do not move),
// so it is skipped.
__device__ __forceinline__ bool digit_empty(const SelectState* st, int shift)
{
    return (st->bits >> shift) == 0;
}

// histogram of digit `shift` over the keys that match the selected prefix
__global__ __launch_bounds__(256) void select_hist_kernel(const uint64_t* act, int64_t npix,
                                                          int shift, SelectState* st)
{
    __shared__ unsigned int h[256];
    if (digit_empty(st, shift)) return;  // the same for every thread
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * 256) {
        const uint64_t a = act[p];
        if ((a & mask) == prefix) atomicAdd(&h[(a >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// The digit bucket, from the top, that holds the need-th largest key: thread
// t holds bucket 255 - t, and an inclusive scan over t counts the keys in the
// buckets from the top down to it; the one thread whose bucket takes the
// count from below need to need or more (exactly one: the keys that match the
// prefix number need or more) records the bucket and the keys above it.
__global__ __launch_bounds__(256) void select_pick_kernel(int shift, SelectState* st)
{
    __shared__ unsigned long long h[256];
    if (digit_empty(st, shift)) return;  // the same for every thread
    const int t = threadIdx.x, b = 255 - t;
    const unsigned long long c = st->hist[b];
    const unsigned long long need = (unsigned long long)st->need;
    h[t] = c;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {  // inclusive Hillis-Steele scan
        const unsigned long long x = t >= w ? h[t - w] : 0;
        __syncthreads();
        h[t] += x;
        __syncthreads();
    }
    const unsigned long long incl = h[t], excl = incl - c;
    st->hist[b] = 0;
    if (excl < need && incl >= need) {
        st->prefix |= (uint64_t)b << shift;
        st->mask |= (uint64_t)255 << shift;
        st->above += (int64_t)excl;
        st->need -= (int64_t)excl;
    }
}

// counts packed as (greater << 32) | equal; block b covers 4096 keys
__device__ __forceinline__ uint64_t sel_flag(uint64_t a, uint64_t thr)
{
    return (a > thr ? (uint64_t)1 << 32 : 0) | (a == thr ? 1u : 0u);
}

// The block's kSelectBlock keys, read in address order (coalesced) into LDS,
// key j at keys[j + j/16] so that thread t's sixteen keys (16t .. 16t+15)
// sit 17 apart between threads (few bank conflicts); keys past the end read
// as 0.
constexpr int kKeysLds = (int)(kSelectBlock + kSelectBlock / 16);
__device__ __forceinline__ int key_slot(int j) { return j + (j >> 4); }

__device__ __forceinline__ void stage_keys(const uint64_t* act, int64_t npix, uint64_t* keys)
{
    const int64_t b0 = (int64_t)blockIdx.x * kSelectBlock;
#pragma unroll
    for (int i = 0; i < (int)(kSelectBlock / 256); ++i) {
        const int j = i * 256 + (int)threadIdx.x;
        keys[key_slot(j)] = b0 + j < npix ? act[b0 + j] : 0;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void select_reduce_kernel(const uint64_t* act, int64_t npix,
                                                            const SelectState* st, uint64_t* bsum)
{
    __shared__ uint64_t keys[kKeysLds];
    __shared__ uint64_t s[256];
    const uint64_t thr = st->prefix;
    stage_keys(act, npix, keys);
    const int64_t base = (int64_t)blockIdx.x * kSelectBlock + threadIdx.x * 16;
    uint64_t c = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < npix) c += sel_flag(keys[key_slot((int)threadIdx.x * 16 + i)], thr);
    s[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

// exclusive scan of the block sums in place (one workgroup, chunks of 256)
__global__ __launch_bounds__(256) void select_scan_kernel(uint64_t* bsum, int64_t nblocks)
{
    __shared__ uint64_t s[256];
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < nblocks; c0 += 256) {
        const int64_t i = c0 + threadIdx.x;
        const uint64_t v = i < nblocks ? bsum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int w = 1; w < 256; w <<= 1) {  // inclusive Hillis-Steele scan
            const uint64_t x = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
            __syncthreads();
            s[threadIdx.x] += x;
            __syncthreads();
        }
        if (i < nblocks) bsum[i] = carry + s[threadIdx.x] - v;
        carry += s[255];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void select_scatter_kernel(const uint64_t* act, int64_t npix,
                                                             const SelectState* st,
                                                             const uint64_t* bsum, int64_t* list)
{
    __shared__ uint64_t keys[kKeysLds];
    __shared__ uint64_t s[256];
    const uint64_t thr = st->prefix;
    const int64_t need = st->need;
    stage_keys(act, npix, keys);
    const int64_t base = (int64_t)blockIdx.x * kSelectBlock + threadIdx.x * 16;
    uint64_t c = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < npix) c += sel_flag(keys[key_slot((int)threadIdx.x * 16 + i)], thr);
    s[threadIdx.x] = c;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {
        const uint64_t x = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    uint64_t run = bsum[blockIdx.x] + s[threadIdx.x] - c;  // exclusive prefix at `base`
    for (int i = 0; i < 16; ++i) {
        const int64_t p = base + i;
        if (p >= npix) break;
        const uint64_t f = sel_flag(keys[key_slot((int)threadIdx.x * 16 + i)], thr);
        const int64_t gt = (int64_t)(run >> 32), eq = (int64_t)(run & 0xffffffffu);
        if ((f >> 32) || ((f & 1) && eq < need)) list[gt + (eq < need ? eq : need)] = p;
        run += f;
    }
}

// caller's list: every entry in [0, npix), strictly increasing (bit 1, bit 2)
__global__ __launch_bounds__(256) void list_check_kernel(const int64_t* list, int64_t n,
                                                         int64_t npix, int* status)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t p = list[i];
    int bad = 0;
    if (p < 0 || p >= npix) bad |= 1;
    if (i > 0 && !(list[i - 1] < p)) bad |= 2;
    if (bad) atomicOr(status, bad);
}

// first entry of every row: starts[j] = #entries below j*nx, j = 0..ny
__global__ __launch_bounds__(256) void list_rows_kernel(const int64_t* list, int64_t n, int nx,
                                                        int ny, int64_t* starts)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j > ny) return;
    const int64_t key = (int64_t)j * nx;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (list[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    starts[j] = lo;
}

hipError_t launch_activity(const uint16_t* img, int64_t npix, int n_steps, uint64_t* act,
                           bool vec4, hipStream_t s)
{
    if (npix <= 0) return hipSuccess;
    if (vec4) {  // 4 pixels per lane: 5.6% faster than 8 (16-byte loads), same sums
        const int64_t lanes = npix / 4;
        hipLaunchKernelGGL(activity_kernel<4>, dim3((unsigned)((lanes + 255) / 256)), dim3(256),
                           0, s, img, npix, n_steps, act);
    } else {
        hipLaunchKernelGGL(activity_kernel<1>, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0,
                           s, img, npix, n_steps, act);
    }
    return hipGetLastError();
}

hipError_t launch_select_top(const uint64_t* act, int64_t npix, int64_t k, SelectState* st,
                             uint64_t* bsum, int64_t* list, hipStream_t s)
{
    hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, st, k);
    const unsigned hist_groups = (unsigned)std::min<int64_t>(1024, (npix + 255) / 256);
    hipLaunchKernelGGL(select_or_kernel, dim3(hist_groups), dim3(256), 0, s, act, npix, st);
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(select_hist_kernel, dim3(hist_groups), dim3(256), 0, s, act, npix,
                           shift, st);
        hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(256), 0, s, shift, st);
    }
    const int64_t nb = (npix + kSelectBlock - 1) / kSelectBlock;
    hipLaunchKernelGGL(select_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, s, act, npix,
                       (const SelectState*)st, bsum);
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(256), 0, s, bsum, nb);
    hipLaunchKernelGGL(select_scatter_kernel, dim3((unsigned)nb), dim3(256), 0, s, act, npix,
                       (const SelectState*)st, (const uint64_t*)bsum, list);
    return hipGetLastError();
}

hipError_t launch_list_check(const int64_t* list, int64_t n, int64_t npix, int* status,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(list_check_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, list,
                       n, npix, status);
    return hipGetLastError();
}

hipError_t launch_list_rows(const int64_t* list, int64_t n, int nx, int ny, int64_t* starts,
                            hipStream_t s)
{
    hipLaunchKernelGGL(list_rows_kernel, dim3((unsigned)((ny + 1 + 255) / 256)), dim3(256), 0, s,
                       list, n, nx, ny, starts);
    return hipGetLastError();
}

}  // namespace dr
