// HIP kernels (gfx950) of the wire-scan depth reconstruction: geometry
// tables, totals, debug and general-geometry kernels, and the launch wrappers
// (the row-tile and batch instantiations are in dr_tiles_*.hip).
#include "dr_device.h"
#include "dr_fastpos.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace dr {

__global__ __launch_bounds__(256) void build_plans_kernel(GeomArgs g, PlanTables t, int side,
                                                          double scale, int* status)
{
    const int row = blockIdx.x;
    const int N = g.n_steps, B = g.n_bins, nint = N - 1;
    const Frame f = axis_frame(g);
    double py, pz;
    pixel_key(g, f, (int64_t)row * g.nx, py, pz);
    const int s = side ? -leading_sign(g, py, pz) : leading_sign(g, py, pz);
    const double sr = (double)s * g.radius;
    const double e0 = g.first_center - g.width / 2.0;
    const double invw = 1.0 / g.width;
    int inc = 1, dec = 1, bad = 0;
    for (int k = threadIdx.x; k < nint; k += blockDim.x) {
        const double ua = edge_position(g, py, pz, k, sr, f.c, e0, invw);
        const double ub = edge_position(g, py, pz, k + 1, sr, f.c, e0, invw);
        if (!__builtin_isfinite(ua) || !__builtin_isfinite(ub)) bad |= 1;
        for (int kk = k; kk <= k + 1; ++kk) {
            const double cy = g.wire_yz[2 * kk];
            if (!(cy > 0.0 && cy < py)) bad |= 2;
        }
        inc &= (ub >= ua);
        dec &= (ub <= ua);
        const PlanD e = make_plan(ua, ub, B);
        const int64_t o = (int64_t)row * nint + k;
        // scale is +-1 or +-1/2: exact, so the FP64 fractions stay the
        // oracle's ov/len up to sign and a power of two
        const double f0 = e.f0 * scale, fm = e.fm * scale, f1 = e.f1 * scale;
        t.bl[o] = e.bl;
        t.nb[o] = e.nb;
        t.f0[o] = (float)f0;
        t.fm[o] = (float)fm;
        t.f1[o] = (float)f1;
        if (t.d0) {
            t.d0[o] = f0;
            t.dm[o] = fm;
            t.d1[o] = f1;
        }
    }
    inc = __syncthreads_and(inc);
    dec = __syncthreads_and(dec);
    const int bad1 = __syncthreads_or(bad & 1) ? 1 : 0;
    const int bad2 = __syncthreads_or(bad & 2) ? 2 : 0;
    bad = bad1 | bad2;
    // Range of bins the row touches, and a check that a monotone row visits
    // them contiguously (each interval starts in, or right after, the last bin
    // of the previous touched interval), which the streaming tile relies on.
    __shared__ int s_lo, s_hi;
    if (threadIdx.x == 0) {
        s_lo = B;
        s_hi = -1;
    }
    __syncthreads();  // also makes this row's plan entries visible block-wide
    int lo = B, hi = -1, gap = 0, wide = 0;
    const int64_t base = (int64_t)row * nint;
    for (int k = threadIdx.x; k < nint; k += blockDim.x) {
        const int nb = t.nb[base + k];
        if (nb == 0) continue;
        const int bl = t.bl[base + k], bh = bl + nb - 1;
        wide |= nb > 2;
        lo = min(lo, bl);
        hi = max(hi, bh);
        // nearest touched interval after k
        for (int k2 = k + 1; k2 < nint; ++k2) {
            const int nb2 = t.nb[base + k2];
            if (nb2 == 0) continue;
            const int bl2 = t.bl[base + k2], bh2 = bl2 + nb2 - 1;
            if (inc && !(bl2 == bh || bl2 == bh + 1)) gap = 1;
            if (dec && !(bh2 == bl || bh2 == bl - 1)) gap = 1;
            break;
        }
    }
    atomicMin(&s_lo, lo);
    atomicMax(&s_hi, hi);
    gap = __syncthreads_or(gap);
    wide = __syncthreads_or(wide);
    if (threadIdx.x == 0) {
        int cls = inc ? kRowIncreasing : (dec ? kRowDecreasing : kRowGeneric);
        if (gap) cls = kRowGeneric;
        if (cls != kRowGeneric && !wide) cls |= kRowNarrow;
        t.row_class[row] = (int8_t)cls;
        t.row_sign[row] = (int8_t)s;
        t.row_lo[row] = s_lo;
        t.row_hi[row] = s_hi;
        if (bad) atomicOr(status, bad);
    }
}

__global__ void unify_classes_kernel(int8_t* a, int8_t* b, int ny)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ny) return;
    if (a[j] == kRowGeneric || b[j] == kRowGeneric) a[j] = b[j] = kRowGeneric;
}


__global__ void reset_counter_kernel(unsigned long long* c) { *c = 0ull; }

// ------------------------------------------------------------------ totals

// Rows sl, sl + step, ... (below slots) of column b, added in that order;
// eight loads are issued before their adds, so a thread does not wait for
// each row in turn (the sum is the same, in the same order).
template <typename T>
__device__ __forceinline__ double column_sum(const T* part, int64_t sl, int64_t slots,
                                             int64_t step, int B, int b)
{
    double s = 0.0;
    for (; sl + 7 * step < slots; sl += 8 * step) {
        T v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = part[(sl + i * step) * B + b];
#pragma unroll
        for (int i = 0; i < 8; ++i) s += (double)v[i];
    }
    for (; sl < slots; sl += step) s += (double)part[sl * B + b];
    return s;
}

// Sum of column b of work[rows][B], rows added in order 0, 1, ...; sixteen
// rows' loads are issued before their adds (a loop of one load and one add
// waits out a full memory latency per row: these kernels run on a handful of
// workgroups).
__device__ __forceinline__ double rows_in_order(const double* work, int rows, int B, int b)
{
    double s = 0.0;
    int r = 0;
    for (; r + 16 <= rows; r += 16) {
        double v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = work[(int64_t)(r + i) * B + b];
#pragma unroll
        for (int i = 0; i < 16; ++i) s += v[i];
    }
    for (; r < rows; ++r) s += work[(int64_t)r * B + b];
    return s;
}

template <typename T>
__global__ __launch_bounds__(256) void totals_stage1(const T* part, int64_t slots, int B,
                                                     double* work)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.x * 64 + lane;
    const double s =
        b < B ? column_sum(part, (int64_t)blockIdx.y * 4 + w, slots, (int64_t)gridDim.y * 4, B, b)
              : 0.0;
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B)
        work[(int64_t)blockIdx.y * B + b] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Totals of many scans at once: each block finds its job (jobs are few and
// ordered by first block) and runs the single-scan stage on it.
__device__ __forceinline__ int find_job(const TotalsJob* jobs, int n, int block, bool second)
{
    int j = 0;
    while (j + 1 < n && (second ? jobs[j + 1].first2 : jobs[j + 1].first1) <= block) ++j;
    return j;
}

__global__ __launch_bounds__(256) void totals_multi_stage1(const TotalsJob* jobs, int n)
{
    __shared__ double red[4][64];
    const TotalsJob& jb = jobs[find_job(jobs, n, (int)blockIdx.x, false)];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = ((int)blockIdx.x - jb.first1) * 64 + lane;
    const int B = jb.n_bins;
    const double s = b < B ? column_sum(jb.parts, (int64_t)blockIdx.y * 4 + w, jb.slots,
                                        (int64_t)gridDim.y * 4, B, b)
                           : 0.0;
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B)
        jb.work[(int64_t)blockIdx.y * B + b] =
            ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ __launch_bounds__(256) void totals_multi_stage2(const TotalsJob* jobs, int n, int rows)
{
    const TotalsJob& jb = jobs[find_job(jobs, n, (int)blockIdx.x, true)];
    const int b = ((int)blockIdx.x - jb.first2) * 256 + threadIdx.x;
    if (b >= jb.n_bins) return;
    jb.totals[b] = (float)rows_in_order(jb.work, rows, jb.n_bins, b);
}

// Column sums of an FP64 output [B][P] in a fixed order: block (b, chunk)
// sums its chunk of plane b (256 strided partial sums, then a tree) into
// work[chunk][b]; totals_stage2 adds the chunks in order.
__global__ __launch_bounds__(256) void plane_sums_f64(const double* out, int64_t P, int B,
                                                     double* work)
{
    __shared__ double red[256];
    const int b = (int)blockIdx.x, ch = (int)blockIdx.y, nch = (int)gridDim.y;
    const int64_t p0 = P * ch / nch, p1 = P * (ch + 1) / nch;
    const double* plane = out + (int64_t)b * P;
    double s = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) s += plane[p];
    red[threadIdx.x] = s;
    for (int h = 128; h > 0; h >>= 1) {
        __syncthreads();
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    }
    if (threadIdx.x == 0) work[(int64_t)ch * B + b] = red[0];
}

template <typename T>
__global__ __launch_bounds__(256) void totals_stage2(const double* work, int rows, int B, T* tot)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    tot[b] = (T)rows_in_order(work, rows, B, b);
}

// ------------------------------------------------------------------- debug

__global__ __launch_bounds__(64) void debug_plan_kernel(GeomArgs g, const int64_t* pix, int n,
                                                        int side, int32_t* bins, double* upos)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const Frame f = axis_frame(g);
    double py, pz;
    pixel_key(g, f, pix[idx], py, pz);
    const int s = side ? -leading_sign(g, py, pz) : leading_sign(g, py, pz);
    const double sr = (double)s * g.radius;
    const double e0 = g.first_center - g.width / 2.0;
    const double invw = 1.0 / g.width;
    for (int k = 0; k < g.n_steps; ++k) {
        const double u = edge_position(g, py, pz, k, sr, f.c, e0, invw);
        if (bins) bins[(int64_t)idx * g.n_steps + k] = floor_to_i32(u);
        if (upos) upos[(int64_t)idx * g.n_steps + k] = u;
    }
}

// -------------------------------------------------------- general geometry

__global__ __launch_bounds__(256) void project_wire_kernel(GeomArgs g, double* wyz, int* status)
{
    const Frame f = axis_frame(g);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (!f.ok) {
        if (k == 0) atomicOr(status, 4);
        return;
    }
    if (k >= g.n_steps) return;
    double eta, xi;
    project(f, g.wire_raw + 3 * k, eta, xi);
    wyz[2 * k] = eta;
    wyz[2 * k + 1] = xi;
}

// flags[j] stays 1 when every pixel of row j shares the row's first key bits
__global__ __launch_bounds__(256) void row_uniform_kernel(GeomArgs g, int* flags)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)g.nx * g.ny) return;
    const Frame f = axis_frame(g);
    const int64_t j = p / g.nx;
    double y, z, y0, z0;
    pixel_key(g, f, p, y, z);
    pixel_key(g, f, j * g.nx, y0, z0);
    if (__double_as_longlong(y) != __double_as_longlong(y0) ||
        __double_as_longlong(z) != __double_as_longlong(z0))
        flags[j] = 0;
}

// every (pixel, step) of a per-pixel geometry: finite positions on the edge
// sides in `sides` (bit 0 leading, bit 1 trailing), wire between beam and
// pixel (status bits 1 and 2 as in build_plans_kernel), |u| < 2^30 (bit 8),
// and, as the bits of non-negative doubles (unsigned order is then numeric
// order): bounds[0] the largest bound on the distance between the per-pixel
// kernel's fast positions and the exact ones, bounds[1] the shortest step
// between two positions that differ (the smallest |u_{k+1} - u_k| > 0), and
// bounds[2] the largest distance actually found between the two forms
__global__ __launch_bounds__(256) void validate_pixels_kernel(GeomArgs g, int sides, int* status,
                                                              unsigned long long* bounds)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // lanes past the last pixel repeat it, so that every lane of the wave
    // takes part in the wave's maximum below
    const int64_t n = (int64_t)g.nx * g.ny;
    const Frame f = axis_frame(g);
    double py, pz;
    pixel_key(g, f, p < n ? p : n - 1, py, pz);
    const double e0 = g.first_center - g.width / 2.0;
    const double invw = 1.0 / g.width;
    const double r = g.radius;
    // the fast form as the kernel evaluates it, walking upwards (a walk the
    // other way negates every value, exactly)
    const bool tilt = g.axis[2] != 0.0;
    FastPos fp;
    fp.py = py;
    fp.pz = pz;
    fp.mrr = -(r * r);
    fp.scale = tilt ? invw / f.c : invw;
    fp.offs = -e0 * invw;
    int bad = 0;
    for (int side = 0; side < 2; ++side) {
        if (!(sides & (1 << side))) continue;
        const int s = side ? -leading_sign(g, py, pz) : leading_sign(g, py, pz);
        const double sr = (double)s * r;
        double bound = 0.0, min_step = 0x1p1000, u_prev = 0.0, err = 0.0;
        fp.sr = sr;
        fp.srrr = sr * (r * r);
        for (int k = 0; k < g.n_steps; ++k) {
            // the operations of tangent_depth and edge_position, in their
            // order, keeping the parts the bound below needs
            const double cy = g.wire_yz[2 * k], cz = g.wire_yz[2 * k + 1];
            const double ay = cy - py, az = cz - pz;
            const double L2 = az * az + ay * ay;
            const double q = L2 - r * r;
            double kk;
            if (q >= 0x1p-767 && q < __builtin_inf())
                kk = sqrt_newton(q);
            else
                kk = q > 0.0 ? __builtin_sqrt(q) : __builtin_nan("");
            const double tz = az * kk - ay * sr;
            const double ty = ay * kk + az * sr;
            const double Q = (cy * tz + sr * L2) / ty;
            const double t = cz - Q;
            const double d = f.c == 1.0 ? t : t / f.c;
            const double u = (d - e0) * invw;
            if (!__builtin_isfinite(u)) bad |= 1;
            else if (!(__builtin_fabs(u) < 0x1p30)) bad |= 8;
            if (k > 0) {
                const double len = __builtin_fabs(u - u_prev);
                if (len > 0.0 && len < min_step) min_step = len;
            }
            u_prev = u;
            const double e = __builtin_fabs(position_fast(cy, cz, fp) - u);
            if (e > err) err = e;  // NaN (a bad pixel, flagged above) is skipped
            // How far the per-pixel kernel's fast position (one Newton step
            // after the hardware reciprocal square root and reciprocal,
            // relative errors below 2^-47, and 1/c for a tilted axis) can lie
            // from this exact one: its square root moves t_xi, t_eta and so
            // the quotient Q = num / t_eta by (|C_eta a_xi| + |Q a_eta|) kk /
            // |t_eta| times its relative error, the division Q by |Q| times
            // its error, and the roundings of every term are of the order of
            // the terms; 2^-38, 2^9 above the errors, times the sum of the
            // magnitudes, in bins.
            const double terms =
                (__builtin_fabs(cy) * (__builtin_fabs(az) * kk + __builtin_fabs(ay) * r) + r * L2 +
                 __builtin_fabs(Q) * (__builtin_fabs(ay) * kk + __builtin_fabs(az) * r)) /
                __builtin_fabs(ty);
            const double b = 0x1p-38 *
                             (__builtin_fabs(cz) + __builtin_fabs(Q) + __builtin_fabs(e0) + terms) /
                             __builtin_fabs(f.c) * invw;
            bound = __builtin_isfinite(b) ? __builtin_fmax(bound, b) : 1.0;
        }
        // the wave's largest bound and error and shortest step, then one
        // atomic each
        unsigned long long bits = (unsigned long long)__double_as_longlong(bound);
        unsigned long long sbits = (unsigned long long)__double_as_longlong(min_step);
        unsigned long long ebits = (unsigned long long)__double_as_longlong(err);
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(bits, off, 64);
            bits = o > bits ? o : bits;
            const unsigned long long so = __shfl_xor(sbits, off, 64);
            sbits = so < sbits ? so : sbits;
            const unsigned long long eo = __shfl_xor(ebits, off, 64);
            ebits = eo > ebits ? eo : ebits;
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMax(bounds, bits);
            atomicMin(bounds + 1, sbits);
            atomicMax(bounds + 2, ebits);
        }
    }
    for (int k = 0; k < g.n_steps; ++k) {
        const double cy = g.wire_yz[2 * k];
        if (!(cy > 0.0 && cy < py)) bad |= 2;
        // the per-pixel kernels take the square root's Newton form unguarded
        const double ay = cy - py, az = g.wire_yz[2 * k + 1] - pz;
        if (!((az * az + ay * ay) - r * r >= 0x1p-767)) bad |= 1;
    }
    if (bad) atomicOr(status, bad);
}

// ---------------------------------------------------------- launch wrappers

static const TileCfg kVariants[] = {
    {1, 2, 4}, {1, 2, 8}, {1, 2, 16}, {1, 4, 4}, {1, 4, 8}, {1, 4, 16},
    {2, 2, 4}, {2, 2, 8}, {2, 2, 16}, {2, 4, 4}, {2, 4, 8}, {2, 4, 16},
    {4, 2, 4}, {4, 2, 8}, {4, 2, 16}, {4, 4, 4}, {4, 4, 8}, {4, 4, 16},
    {8, 2, 4}, {8, 2, 8}, {8, 2, 16}, {8, 4, 4}, {8, 4, 8}, {8, 4, 16},
};

int num_tile_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
TileCfg tile_variant(int i) { return kVariants[i]; }

bool tile_supported(const TileCfg& t)
{
    for (const TileCfg& v : kVariants)
        if (v.ppl == t.ppl && v.waves == t.waves && v.prefetch == t.prefetch) return true;
    return false;
}

int tile_width(const TileCfg& t) { return 64 * t.waves * t.ppl; }



hipError_t launch_build_plans(const GeomArgs& g, const PlanTables& t, int side, double scale,
                              int* d_status, hipStream_t s)
{
    hipLaunchKernelGGL(build_plans_kernel, dim3(g.ny), dim3(256), 0, s, g, t, side, scale,
                       d_status);
    return hipGetLastError();
}

hipError_t launch_unify_classes(int8_t* a, int8_t* b, int ny, hipStream_t s)
{
    hipLaunchKernelGGL(unify_classes_kernel, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, s,
                       a, b, ny);
    return hipGetLastError();
}

hipError_t launch_rows_f32(const TileCfg& t, const ScanArgs& a, hipStream_t s)
{
    const int64_t rows = a.row_end - a.row_begin;
    if (rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)(rows * a.tiles_per_row));
    return a.pass == 2 ? launch_rows_f32_add(t, a, grid, s) : launch_rows_f32_single(t, a, grid, s);
}

hipError_t launch_rows_f64(const ScanArgs& a, hipStream_t s)
{
    const int64_t rows = a.row_end - a.row_begin;
    if (rows <= 0) return hipSuccess;
    if (a.pass == 2) return hipErrorInvalidValue;  // FP64 passes are each launched on their own
    const dim3 grid((unsigned)(rows * a.tiles_per_row));
    if (a.wk)
        hipLaunchKernelGGL((rows_f64_kernel<true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((rows_f64_kernel<false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void add_into_kernel(double* out, const double* other, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = out[i] + other[i];
}

hipError_t launch_add_f64(double* out, const double* other, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t groups = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(add_into_kernel, dim3((unsigned)groups), dim3(256), 0, s, out, other, n);
    return hipGetLastError();
}

hipError_t launch_batch_f32(const TileCfg& t, const BatchArgs& b, bool add, int groups,
                            hipStream_t s)
{
    const dim3 grid((unsigned)groups);
    return add ? launch_batch_f32_add(t, b, grid, s) : launch_batch_f32_single(t, b, grid, s);
}

hipError_t launch_reset_counter(unsigned long long* counter, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_totals(const T* partials, int64_t slots, int n_bins, double* work,
                                int work_rows, T* totals, hipStream_t s)
{
    const dim3 g1((unsigned)((n_bins + 63) / 64), (unsigned)work_rows);
    hipLaunchKernelGGL(totals_stage1<T>, g1, dim3(256), 0, s, partials, slots, n_bins, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(totals_stage2<T>, dim3((unsigned)((n_bins + 255) / 256)), dim3(256), 0, s,
                       (const double*)work, work_rows, n_bins, totals);
    return hipGetLastError();
}

hipError_t launch_totals_f32(const float* partials, int64_t slots, int n_bins, double* work,
                             int work_rows, float* totals, hipStream_t s)
{
    return launch_totals<float>(partials, slots, n_bins, work, work_rows, totals, s);
}

hipError_t launch_totals_f64(const double* partials, int64_t slots, int n_bins, double* work,
                             int work_rows, double* totals, hipStream_t s)
{
    return launch_totals<double>(partials, slots, n_bins, work, work_rows, totals, s);
}

hipError_t launch_totals_multi_f32(const TotalsJob* jobs, int n, int blocks1, int blocks2,
                                   hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(totals_multi_stage1, dim3((unsigned)blocks1, (unsigned)kTotalsWorkRows),
                       dim3(256), 0, s, jobs, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(totals_multi_stage2, dim3((unsigned)blocks2), dim3(256), 0, s, jobs, n,
                       kTotalsWorkRows);
    return hipGetLastError();
}

hipError_t launch_plane_totals_f64(const double* out, int64_t P, int n_bins, double* work,
                                  int work_rows, double* totals, hipStream_t s)
{
    if (P <= 0 || n_bins <= 0) return hipSuccess;
    const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(work_rows, P / 65536));
    hipLaunchKernelGGL(plane_sums_f64, dim3((unsigned)n_bins, (unsigned)chunks), dim3(256), 0, s,
                       out, P, n_bins, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(totals_stage2<double>, dim3((unsigned)((n_bins + 255) / 256)), dim3(256),
                       0, s, (const double*)work, chunks, n_bins, totals);
    return hipGetLastError();
}

hipError_t launch_project_wire(const GeomArgs& g, double* wire_yz, int* d_status, hipStream_t s)
{
    hipLaunchKernelGGL(project_wire_kernel, dim3((unsigned)((g.n_steps + 255) / 256)), dim3(256),
                       0, s, g, wire_yz, d_status);
    return hipGetLastError();
}

hipError_t launch_row_uniform(const GeomArgs& g, int* flags, hipStream_t s)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL(row_uniform_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                       flags);
    return hipGetLastError();
}

hipError_t launch_validate_pixels(const GeomArgs& g, int sides, int* d_status,
                                  unsigned long long* bounds, hipStream_t s)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL(validate_pixels_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       g, sides, d_status, bounds);
    return hipGetLastError();
}

hipError_t launch_list_f32(const ScanArgs& a, const ListArgs& lt, int64_t n_tiles, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    ListArgs l = lt;
    l.tile_end = l.tile_first + n_tiles;
    const dim3 grid((unsigned)((n_tiles + 3) / 4));  // four wave tiles per workgroup
    const int v = (a.pass == 2 ? 1 : 0) + (a.wk ? 2 : 0);
    switch (v) {
    case 0: hipLaunchKernelGGL((list_f32_kernel<16, false, false>), grid, dim3(256), 0, s, a, l); break;
    case 1: hipLaunchKernelGGL((list_f32_kernel<16, true, false>), grid, dim3(256), 0, s, a, l); break;
    case 2: hipLaunchKernelGGL((list_f32_kernel<16, false, true>), grid, dim3(256), 0, s, a, l); break;
    default: hipLaunchKernelGGL((list_f32_kernel<16, true, true>), grid, dim3(256), 0, s, a, l); break;
    }
    return hipGetLastError();
}

hipError_t launch_list_f64(const ScanArgs& a, const ListArgs& lt, int64_t n_tiles, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (a.pass == 2) return hipErrorInvalidValue;  // FP64 passes are each launched on their own
    ListArgs l = lt;
    l.tile_end = l.tile_first + n_tiles;
    const dim3 grid((unsigned)((n_tiles + 3) / 4));  // four wave tiles per workgroup
    if (a.wk)
        hipLaunchKernelGGL((list_f64_kernel<true>), grid, dim3(256), 0, s, a, l);
    else
        hipLaunchKernelGGL((list_f64_kernel<false>), grid, dim3(256), 0, s, a, l);
    return hipGetLastError();
}

hipError_t launch_rows_norm_f32(const ScanArgs& a, hipStream_t s)
{
    const int64_t rows = a.row_end - a.row_begin;
    if (rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)(rows * a.tiles_per_row));
    if (a.pass == 2)
        hipLaunchKernelGGL(rows_norm_f32_kernel<true>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(rows_norm_f32_kernel<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_debug_plan(const GeomArgs& g, const int64_t* pixels, int n, int side,
                             int32_t* bins, double* upos, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(debug_plan_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, g,
                       pixels, n, side, bins, upos);
    return hipGetLastError();
}

}  // namespace dr
