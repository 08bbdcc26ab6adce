// Device code shared by the kernel translation units of the wire-scan depth
// reconstruction (gfx950): FP64 geometry helpers, the row-tile bodies and the
// row, FP64 and persistent batch kernel templates.  The heavy template
// instantiations live in separate translation units that compile in parallel.
//
// Work split (paper Sec. III-C maps one GPU thread to one image element and
// adds into shared depth arrays with an emulated double atomicAdd; here a lane
// owns PPL adjacent pixels of one detector row for the whole scan, so every
// output element has exactly one writer and the bins need no atomics):
//
//   build_plans_kernel   once per geometry: FP64 edge positions u_k of each
//                        detector row (all pixels of a row share their
//                        projected (eta, xi) bit for bit), and the bins and
//                        overlap fractions of every interval [u_k, u_{k+1}].
//   rows kernels         per (row, tile of PPL*64*WAVES pixels): stage the
//                        row's plan in LDS, stream uint16 images step by step
//                        with PF steps in flight, FP32 differences, accumulate
//                        the open bin in registers, store each finished bin
//                        once (non-temporal), per-wave partial totals.
//   batch kernel         the same tile body in a persistent grid pulling
//                        (scan, tile) items from a queue counter.
//   pixels kernel        geometries whose rows do not share one position: one
//                        lane per pixel computes its own FP64 positions.
//   totals kernels       FP64 sum of the partial totals.
//
// FP64 geometry follows a fixed operation order without contraction so that
// bin indices are exact; build with -ffp-contract=off.
#pragma once

#include "dr_internal.h"

#pragma clang fp contract(off)

// Cache policy of the streaming accesses (each image element is read once and
// each bin written once): 1 = non-temporal, 0 = default.
#ifndef DR_NT_LOADS
#define DR_NT_LOADS 1
#endif
#ifndef DR_NT_STORES
#define DR_NT_STORES 1
#endif

namespace dr {

template <typename T>
__device__ __forceinline__ void stream_store(T v, T* p)
{
#if DR_NT_STORES
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

template <typename T>
__device__ __forceinline__ T stream_load(const T* p)
{
#if DR_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// ------------------------------------------------------------- FP64 geometry

// Square root of a finite q >= 2^-767, correctly rounded: the Newton
// sequence the compiler itself expands sqrt into (reciprocal square root
// estimate, then two refinements of the root and of half its reciprocal),
// without the rescaling of smaller inputs and the special-value select that
// it adds around it: the same bits, a third fewer instructions.
__device__ __forceinline__ double sqrt_newton(double q)
{
    const double y = __builtin_amdgcn_rsq(q);
    double g = q * y, h = y * 0.5;
    const double e = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, e, g);
    h = __builtin_fma(h, e, h);
    double d = __builtin_fma(-g, g, q);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, q);
    return __builtin_fma(d, h, g);
}

// Depth at which the ray from pixel (py, pz), tangent to the wire disc centred
// at (cy, cz) on side sr/r (sr = s*r, s = +1 is the +z side), meets the beam:
// d = Cz - (Cy*tz + s*r*L2)/ty with a = C - P, L2 = |a|^2, kk = sqrt(L2 - r^2),
// t = a*kk + s*r*a_perp.  Every term is O(wire height), free of cancellation.
__device__ __forceinline__ double tangent_depth(double py, double pz, double cy, double cz,
                                                double r, double sr)
{
    const double ay = cy - py;
    const double az = cz - pz;
    const double L2 = az * az + ay * ay;
    const double q = L2 - r * r;
    // q <= 0 (the pixel inside the wire) gives NaN, which the depth inherits
    double kk;
    if (__builtin_expect(q >= 0x1p-767 && q < __builtin_inf(), 1))
        kk = sqrt_newton(q);
    else
        kk = q > 0.0 ? __builtin_sqrt(q) : __builtin_nan("");  // tiny or infinite: the library's
    const double tz = az * kk - ay * sr;
    const double ty = ay * kk + az * sr;
    return cz - (cy * tz + sr * L2) / ty;
}

// Frame of the plane normal to the wire axis a: e1 = (z - (z.a)a)/|...| (the
// projected beam direction), e2 = e1 x a, c = e1.z (depth = xi / c).  For the
// x axis: e1 = z, e2 = y, c = 1 exactly.
struct Frame {
    double e1[3], e2[3], c;
    bool ok;
};

__device__ __forceinline__ Frame axis_frame(const GeomArgs& g)
{
    Frame f;
    const double n = __builtin_sqrt((g.axis[0] * g.axis[0] + g.axis[1] * g.axis[1]) +
                                    g.axis[2] * g.axis[2]);
    const double a0 = g.axis[0] / n, a1 = g.axis[1] / n, a2 = g.axis[2] / n;
    const double z0 = 0.0 - a2 * a0, z1 = 0.0 - a2 * a1, z2 = 1.0 - a2 * a2;
    const double m = __builtin_sqrt((z0 * z0 + z1 * z1) + z2 * z2);
    f.ok = (n > 0.0) && (m > 1e-6);
    f.e1[0] = z0 / m;
    f.e1[1] = z1 / m;
    f.e1[2] = z2 / m;
    f.e2[0] = f.e1[1] * a2 - f.e1[2] * a1;
    f.e2[1] = f.e1[2] * a0 - f.e1[0] * a2;
    f.e2[2] = f.e1[0] * a1 - f.e1[1] * a0;
    f.c = f.e1[2];
    return f;
}

__device__ __forceinline__ void project(const Frame& f, const double* X, double& eta, double& xi)
{
    xi = (X[0] * f.e1[0] + X[1] * f.e1[1]) + X[2] * f.e1[2];
    eta = (X[0] * f.e2[0] + X[1] * f.e2[1]) + X[2] * f.e2[2];
}

// Projected (eta, xi) of pixel p: centre (origin + i*u) + j*v or the table.
__device__ __forceinline__ void pixel_key(const GeomArgs& g, const Frame& f, int64_t p,
                                          double& py, double& pz)
{
    double X[3];
    if (g.pix_xyz) {
        X[0] = g.pix_xyz[3 * p];
        X[1] = g.pix_xyz[3 * p + 1];
        X[2] = g.pix_xyz[3 * p + 2];
    } else {
        const double i = (double)(p % g.nx);
        const double j = (double)(p / g.nx);
#pragma unroll
        for (int q = 0; q < 3; ++q) X[q] = (g.origin[q] + i * g.u[q]) + j * g.v[q];
    }
    project(f, X, py, pz);
}

// Leading-edge side: +1 when the +xi tangent point of the last step lies
// beyond that of the first.
__device__ __forceinline__ int leading_sign(const GeomArgs& g, double py, double pz)
{
    const int l = g.n_steps - 1;
    const double d0 = tangent_depth(py, pz, g.wire_yz[0], g.wire_yz[1], g.radius, g.radius);
    const double d1 = tangent_depth(py, pz, g.wire_yz[2 * l], g.wire_yz[2 * l + 1], g.radius,
                                    g.radius);
    return d1 > d0 ? 1 : -1;
}

__device__ __forceinline__ double edge_position(const GeomArgs& g, double py, double pz, int k,
                                                double sr, double c, double e0, double invw)
{
    const double t = tangent_depth(py, pz, g.wire_yz[2 * k], g.wire_yz[2 * k + 1], g.radius, sr);
    const double d = c == 1.0 ? t : t / c;  // t / 1 == t: the division only for tilted axes
    return (d - e0) * invw;
}

__device__ __forceinline__ int32_t floor_to_i32(double x)
{
    const double f = __builtin_floor(x);
    if (f < -2147483648.0) return INT32_MIN;
    if (f > 2147483647.0) return INT32_MAX;
    return (int32_t)f;
}

struct PlanD {
    int bl, nb;
    double f0, fm, f1;
};

// Bins of the interval between positions ua and ub (bin units) that overlap it
// by a positive length, and their fractions overlap/length.  A zero-length
// interval is a point mass in bin floor(ua).  Parts outside [0, B) drop out.
// EXACT divides each overlap by the length (the FP64 order); otherwise the
// overlaps are multiplied by one reciprocal (for fractions rounded to FP32).
template <bool EXACT = true>
__device__ __forceinline__ PlanD make_plan(double ua, double ub, int B)
{
    PlanD e{0, 0, 0.0, 0.0, 0.0};
    const double lo = ua < ub ? ua : ub;
    const double hi = ua < ub ? ub : ua;
    const double len = hi - lo;
    if (len > 0.0) {
        double first = __builtin_floor(lo), last = __builtin_floor(hi);
        if (first < 0.0) first = 0.0;
        if (last > (double)(B - 1)) last = (double)(B - 1);
        double ovf = 0.0, ovl = 0.0;
        while (first <= last) {
            const double top = hi < first + 1.0 ? hi : first + 1.0;
            const double bot = lo > first ? lo : first;
            ovf = top - bot;
            if (ovf > 0.0) break;
            first += 1.0;
        }
        while (last >= first) {
            const double top = hi < last + 1.0 ? hi : last + 1.0;
            const double bot = lo > last ? lo : last;
            ovl = top - bot;
            if (ovl > 0.0) break;
            last -= 1.0;
        }
        if (first <= last) {
            e.bl = (int)first;
            e.nb = (int)(last - first) + 1;
            if constexpr (EXACT) {
                e.f0 = ovf / len;
                e.f1 = ovl / len;
                e.fm = 1.0 / len;  // interior bins overlap by exactly one bin
            } else {
                const double rl = 1.0 / len;
                e.f0 = ovf * rl;
                e.f1 = ovl * rl;
                e.fm = rl;
            }
        }
    } else {
        const double bd = __builtin_floor(lo);
        if (bd >= 0.0 && bd < (double)B) {
            e.bl = (int)bd;
            e.nb = 1;
            e.f0 = e.fm = e.f1 = 1.0;
        }
    }
    return e;
}

// One workgroup per detector row: plan tables, row class, checks.
// status bit 0: a non-finite position (pixel inside the wire or degenerate);
// bit 1: a wire position not strictly between beam and detector in y.
// ------------------------------------------------------------ tile kernels

template <int PPL> struct U16V;
template <> struct U16V<1> { typedef unsigned short T; };
template <> struct U16V<2> { typedef unsigned int T; };
template <> struct U16V<4> { typedef unsigned int T __attribute__((ext_vector_type(2))); };
template <> struct U16V<8> { typedef unsigned int T __attribute__((ext_vector_type(4))); };

template <int PPL>
__device__ __forceinline__ int pix(const typename U16V<PPL>::T& v, int p)
{
    if constexpr (PPL == 1) return (int)v;
    else if constexpr (PPL == 2) return (int)((v >> (16 * p)) & 0xffffu);
    else return (int)((v[p >> 1] >> (16 * (p & 1))) & 0xffffu);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename Acc, int PPL>
__device__ __forceinline__ void store_bins(Acc* p, const Acc (&a)[PPL])
{
    if constexpr (sizeof(Acc) == 8 || PPL == 1) {
#pragma unroll
        for (int q = 0; q < PPL; ++q) stream_store(a[q], p + q);
    } else if constexpr (PPL == 2) {
        f32x2 v = {a[0], a[1]};
        stream_store(v, (f32x2*)p);
    } else {
#pragma unroll
        for (int q = 0; q < PPL; q += 4) {
            f32x4 v = {a[q], a[q + 1], a[q + 2], a[q + 3]};
            stream_store(v, (f32x4*)(p + q));
        }
    }
}

// Sum over the 64 lanes of a wave, returned to every lane (deterministic order).
// FP32: inclusive scan inside each 16-lane row with DPP row shifts, then the
// row totals carried by row broadcasts; lane 63 ends with the total.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_shift(float v)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

__device__ __forceinline__ float wave_total(float v)
{
    v += dpp_shift<0x111, 0xf>(v);  // row_shr:1
    v += dpp_shift<0x112, 0xf>(v);  // row_shr:2
    v += dpp_shift<0x114, 0xf>(v);  // row_shr:4
    v += dpp_shift<0x118, 0xf>(v);  // row_shr:8
    v += dpp_shift<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_shift<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_total(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// `old` with lane `lane` replaced by the uniform value v.
template <typename T>
__device__ __forceinline__ T write_lane(T old, T v, int lane)
{
    return ((int)(threadIdx.x & 63) == lane) ? v : old;
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uni(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename Acc, int CH = kPlanChunk> struct PlanLds {
    int bl[CH];
    int nb[CH];
    Acc f0[CH];
    Acc fm[CH];
    Acc f1[CH];
};

// WT (wave tiles): each wave owns its tile and its plan buffer; the waves of
// a workgroup never wait for each other, and a wave orders its own LDS
// writes before its reads.
template <bool WT>
__device__ __forceinline__ void tile_sync()
{
    if constexpr (WT) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <typename Acc, int CH = kPlanChunk, bool WT = false>
__device__ __forceinline__ void stage_plan(const ScanArgs& a, int row, int kc, int nk,
                                           PlanLds<Acc, CH>& L)
{
    const int64_t base = (int64_t)row * (a.n_steps - 1) + kc;
    auto copy = [&](int e) {
        L.bl[e] = a.bl[base + e];
        L.nb[e] = a.nb[base + e];
        if constexpr (sizeof(Acc) == 4) {
            L.f0[e] = a.f0[base + e];
            L.fm[e] = a.fm[base + e];
            L.f1[e] = a.f1[base + e];
        } else {
            L.f0[e] = a.d0[base + e];
            L.fm[e] = a.dm[base + e];
            L.f1[e] = a.d1[base + e];
        }
    };
    if constexpr (WT) {
        for (int e = (int)(threadIdx.x & 63); e < nk; e += 64) copy(e);
    } else {
        for (int e = threadIdx.x; e < nk; e += blockDim.x) copy(e);
    }
}

// acc + f*dI: one rounding (fma) in FP32; in FP64 the product and the sum are
// rounded separately, the oracle's order.
__device__ __forceinline__ float madd(float f, float dI, float acc) { return __builtin_fmaf(f, dI, acc); }
__device__ __forceinline__ double madd(double f, double dI, double acc) { return acc + dI * f; }

// Per-wave partial totals: lane l of `pw` holds the total of bin pbase + l of
// the current 64-bin window; a window is written to the wave's partial row
// when the tile moves past it.  Bins are visited monotonically, so each
// window is written once; windows never visited are written as zeros.
template <typename Acc>
struct PartialWindow {
    Acc* row = nullptr;  // this wave's partial row [B], or null (no totals)
    int B = 0;
    int pbase = -1, wfirst = -1;
    Acc pw = (Acc)0;
    __device__ __forceinline__ void flush(int lane)
    {
        if (pbase >= 0 && pbase + lane < B) row[pbase + lane] = pw;
    }
    __device__ __forceinline__ void add(int b, Acc s, int lane)
    {
        const int wb = b & ~63;
        if (wb != pbase) {
            flush(lane);
            if (wfirst < 0) wfirst = wb;
            pbase = wb;
            pw = (Acc)0;
        }
        pw = write_lane(pw, s, b - wb);
    }
    __device__ __forceinline__ void finish(int lane)
    {
        flush(lane);
        const int a0 = wfirst < 0 ? B : min(wfirst, pbase), a1 = wfirst < 0 ? -1 : max(wfirst, pbase);
        for (int wb = 0; wb < B; wb += 64)
            if ((wb < a0 || wb > a1) && wb + lane < B) row[wb + lane] = (Acc)0;
    }
};

// Where the lanes of one tile read and write: uniform bases plus 32-bit lane
// offsets.  A lane's PPL pixels hold step k at ibase[k*istep + ioff + q] and
// bin b at obase[b*plane + ooff + q]; `part` is the wave's partial-total row.
template <typename Acc>
struct TileAddr {
    const uint16_t* ibase;
    int64_t istep;
    uint32_t ioff;
    Acc* obase;
    int64_t plane;
    uint32_t ooff;
    bool act;   // the lane holds pixels (lanes past the end read valid data, never store)
    Acc* part;  // null: no totals
};

// Tile `tile` of detector row `row`: PPL adjacent pixels per lane.
template <typename Acc, int PPL, int WAVES>
__device__ __forceinline__ TileAddr<Acc> row_tile_addr(const ScanArgs& a, int row, int tile)
{
    constexpr int TW = 64 * WAVES * PPL;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int col0 = tile * TW + tid * PPL;
    TileAddr<Acc> t;
    t.act = col0 < a.nx;
    t.ibase = a.img + (int64_t)(row - a.row_base) * a.img_row;
    t.istep = a.img_step;
    t.ioff = t.act ? (uint32_t)col0 : 0u;
    t.obase = (Acc*)a.out + (int64_t)row * a.nx;
    t.plane = a.out_plane;
    t.ooff = (uint32_t)col0;
    t.part = a.partials ? (Acc*)a.partials +
                              ((int64_t)(row * a.tiles_per_row + tile) * WAVES + wave) * a.n_bins
                        : nullptr;
    return t;
}

// Wave tile t of a pixel list: entries [tile_start, tile_start + tile_count)
// of one detector row, at most 64 from the start rounded down to kListAlign;
// lane i holds entry (start rounded down) + i, so the wave reads and writes
// whole aligned lines; the output is [n_bins][n] in list order.  Images are
// compact [N][entries] in list order (the buffer holding entries from
// entry_base on) or gathered from full frames.  One partial-total row per
// wave tile.
template <typename Acc>
__device__ __forceinline__ TileAddr<Acc> list_wave_addr(const ScanArgs& a, const ListArgs& l,
                                                        int64_t t, int row)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t e0 = l.tile_start[t];
    const int64_t base = e0 & ~(int64_t)(kListAlign - 1);  // lane 0's entry
    TileAddr<Acc> ta;
    ta.act = base + lane >= e0 && base + lane < e0 + l.tile_count[t];
    const int64_t e = ta.act ? base + lane : e0;
    if (l.compact) {
        ta.ibase = a.img;
        ta.ioff = (uint32_t)(e - l.entry_base);
    } else {
        ta.ibase = a.img + (int64_t)(row - a.row_base) * a.img_row;
        ta.ioff = (uint32_t)(l.pixels[e] - (int64_t)row * a.nx);
    }
    ta.istep = a.img_step;
    ta.obase = (Acc*)a.out;
    ta.plane = a.out_plane;
    ta.ooff = (uint32_t)(base + lane);
    ta.part = a.partials ? (Acc*)a.partials + t * a.n_bins : nullptr;
    return ta;
}

// Difference of two consecutive samples: exact in integers, or with per-step
// weights (NORM) both weighted samples formed in FP64 (one rounding each, the
// oracle's order) and their difference rounded once to Acc.
template <typename Acc, bool NORM>
__device__ __forceinline__ Acc sample_diff(int i0, int i1, const double* wk, int k)
{
    if constexpr (NORM)
        return (Acc)((double)i0 * wk[k] - (double)i1 * wk[k + 1]);
    else
        return (Acc)(i0 - i1);
}

// Non-monotone rows: zero the tile's bins, then read-modify-write every
// contribution in step order (each lane touches only its own pixels).
template <typename Acc, int PPL, int WAVES, bool NORM, int CH, bool WT>
__device__ __forceinline__ void process_tile_generic(const ScanArgs& a, int row,
                                                     const TileAddr<Acc>& ta, PlanLds<Acc, CH>& L)
{
    const int tid = threadIdx.x, lane = tid & 63;
    (void)tid;
    const bool act = ta.act;
    const int N = a.n_steps, B = a.n_bins, nint = N - 1;
    const uint16_t* ip = ta.ibase + ta.ioff;
    Acc* op = ta.obase + ta.ooff;
    const int64_t plane = ta.plane;
    if (act && a.pass != 2)  // the second pass adds onto the first pass's output
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int q = 0; q < PPL; ++q) op[(int64_t)b * plane + q] = (Acc)0;
    for (int kc = 0; kc < nint; kc += CH) {
        const int nk = min(CH, nint - kc);
        tile_sync<WT>();
        stage_plan<Acc, CH, WT>(a, row, kc, nk, L);
        tile_sync<WT>();
        for (int kk = 0; kk < nk; ++kk) {
            int bl = uni(L.bl[kk]), nb = uni(L.nb[kk]);
            if constexpr (WT) {  // keep every address inside the output, whatever was read
                bl = min(max(bl, 0), B - 1);
                nb = min(max(nb, 0), B - bl);
            }
            if (nb == 0 || !act) continue;
            const Acc f0 = uni(L.f0[kk]), fm = uni(L.fm[kk]), f1 = uni(L.f1[kk]);
            const int k = kc + kk;
            const int bh = bl + nb - 1;
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                const Acc dI = sample_diff<Acc, NORM>((int)ip[(int64_t)k * ta.istep + q],
                                                      (int)ip[(int64_t)(k + 1) * ta.istep + q],
                                                      a.wk, k);
                for (int b = bl; b <= bh; ++b) {
                    const Acc f = (b == bl) ? f0 : ((b == bh) ? f1 : fm);
                    Acc* o = op + (int64_t)b * plane + q;
                    *o = madd(f, dI, *o);
                }
            }
        }
    }
    if (ta.part) {
        // partial totals of the final values; a first pass of two leaves them
        // to the second (a row is generic in both passes or in neither)
        PartialWindow<Acc> pwin;
        pwin.row = ta.part;
        pwin.B = B;
        if (a.pass != 1) {
            for (int b = 0; b < B; ++b) {
                Acc s = (Acc)0;
                if (act)
#pragma unroll
                    for (int q = 0; q < PPL; ++q) s += op[(int64_t)b * plane + q];
                pwin.add(b, wave_total(s), lane);
            }
        }
        pwin.finish(lane);
    }
}

// One tile: PPL adjacent pixels per lane, 64*WAVES lanes, one detector row.
// Monotone rows stream the steps once: PF image loads in flight per lane (all
// unconditional, so the prefetch ring stays in registers), the open bin in
// registers, each touched bin stored once as soon as the edge has passed it,
// untouched bins zeroed after the last load.
template <typename Acc, int PPL, int WAVES, int PF, bool NB2, bool ADD, bool NORM, int CH,
          bool WT>
__device__ __forceinline__ void process_tile_mono(const ScanArgs& a, int row,
                                                  const TileAddr<Acc>& ta, PlanLds<Acc, CH>& L,
                                                  int cls)
{
    using V = typename U16V<PPL>::T;
    const int dir = ((cls & 3) == kRowIncreasing) ? 1 : -1;
    const int tid = threadIdx.x, lane = tid & 63;
    (void)tid;
    const bool act = ta.act;
    const int N = a.n_steps, B = a.n_bins, nint = N - 1;
    // uniform 64-bit bases plus 32-bit lane offsets; lanes past the end read
    // valid pixels and never store
    const uint16_t* irow = ta.ibase;
    const uint32_t ioff = ta.ioff;
    Acc* orow = ta.obase;
    const uint32_t ooff = ta.ooff;
    const int64_t plane = ta.plane;
    const int64_t istep = ta.istep;
    PartialWindow<Acc> pwin;
    pwin.row = ta.part;
    pwin.B = B;

    auto load = [&](int k) -> V {
        return stream_load((const V*)(irow + (int64_t)k * istep + ioff));
    };
    auto outp = [&](int b) -> Acc* { return orow + (int64_t)b * plane + ooff; };
    Acc acc[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) acc[q] = (Acc)0;
    int cb = -1;  // open bin (uniform), -1 = none

    // ADD (second pass of two edges): the open bin accumulates this pass's own
    // contributions from zero, in step order, and is stored as the first
    // pass's value plus that sum, so that the output is the first pass's
    // reconstruction plus the second's, each formed on its own; base holds the
    // first pass's value of the open bin
    Acc base[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) base[q] = (Acc)0;
    auto put = [&]() {
        if (act) {
            if constexpr (ADD) {
                Acc v[PPL];
#pragma unroll
                for (int q = 0; q < PPL; ++q) v[q] = base[q] + acc[q];
                store_bins<Acc, PPL>(outp(cb), v);
            } else {
                store_bins<Acc, PPL>(outp(cb), acc);
            }
        }
        if (pwin.row) {
            Acc s = (Acc)0;
#pragma unroll
            for (int q = 0; q < PPL; ++q) s += acc[q];
            pwin.add(cb, wave_total(act ? s : (Acc)0), lane);
        }
    };
    auto interval = [&](int kk, int k, const V& prev, const V& cur) {
        int nb = uni(L.nb[kk]);
        if (nb == 0) return;
        int bl = uni(L.bl[kk]);
        if constexpr (WT) {  // keep every address inside the output, whatever was read
            bl = min(max(bl, 0), B - 1);
            nb = min(max(nb, 0), B - bl);
        }
        const Acc f0 = uni(L.f0[kk]), fm = uni(L.fm[kk]), f1 = uni(L.f1[kk]);
        Acc dI[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            dI[q] = sample_diff<Acc, NORM>(pix<PPL>(prev, q), pix<PPL>(cur, q), a.wk, k);
        const int bh = bl + nb - 1;
        auto visit = [&](int b, Acc f) {
            if (b != cb) {
                if (cb >= 0) put();
                cb = b;
                if constexpr (ADD) {
                    const Acc* o = outp(b);
#pragma unroll
                    for (int q = 0; q < PPL; ++q) base[q] = act ? o[q] : (Acc)0;
                }
#pragma unroll
                for (int q = 0; q < PPL; ++q) acc[q] = madd(f, dI[q], (Acc)0);
            } else {
#pragma unroll
                for (int q = 0; q < PPL; ++q) acc[q] = madd(f, dI[q], acc[q]);
            }
        };
        if constexpr (NB2) {
            // at most two bins: straight-line code keeps the load pipeline
            // analysable (no loop with stores between a load and its use)
            if (dir > 0) {
                visit(bl, f0);
                if (nb == 2) visit(bh, f1);
            } else {
                visit(bh, f1);
                if (nb == 2) visit(bl, f0);
            }
        } else {
            int b = dir > 0 ? bl : bh;
            for (int e = 0; e < nb; ++e, b += dir) visit(b, (b == bl) ? f0 : ((b == bh) ? f1 : fm));
        }
    };

    // Ring of U = PF+1 image slots consumed in place: interval k reads slots
    // k % U (step k) and (k+1) % U (step k+1), then slot k % U is refilled
    // with step k + U.  Steps past the end re-read the last image (unused).
    constexpr int U = PF + 1;
    constexpr int KCU = (CH / U) * U;  // plan chunk, a whole number of rings
    // Bins outside the row's touched range are zero.  Those on the side where
    // the walk starts are stored before it, the others after it, so that the
    // tile's stores run through the bin planes in one direction (0.6% faster
    // than all after the walk on the 2048^2 x 1001 x 1001 scan).
    const int blo = a.row_lo[row], bhi = a.row_hi[row];
    Acc zero[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) zero[q] = (Acc)0;
    if (act && !ADD && blo <= bhi) {
        if (dir > 0)
            for (int b = 0; b < blo; ++b) store_bins<Acc, PPL>(outp(b), zero);
        else
            for (int b = B - 1; b > bhi; --b) store_bins<Acc, PPL>(outp(b), zero);
    }
    V ring[U];
#pragma unroll
    for (int d = 0; d < U; ++d) ring[d] = load(min(d, N - 1));

    for (int kc = 0; kc < nint; kc += KCU) {
        const int nk = min(KCU, nint - kc);
        tile_sync<WT>();
        stage_plan<Acc, CH, WT>(a, row, kc, nk, L);
        tile_sync<WT>();
        int kk = 0;
        for (; kk + U <= nk; kk += U) {
#pragma unroll
            for (int d = 0; d < U; ++d) {
                interval(kk + d, kc + kk + d, ring[d], ring[(d + 1) % U]);
                ring[d] = load(min(kc + kk + d + U, N - 1));
            }
        }
#pragma unroll
        for (int d = 0; d < U; ++d) {
            if (kk + d < nk) {
                interval(kk + d, kc + kk + d, ring[d], ring[(d + 1) % U]);
                ring[d] = load(min(kc + kk + d + U, N - 1));
            }
        }
    }
    if (cb >= 0) put();
    // the other side's zero bins (every bin when the walk touches none)
    if (act && !ADD) {
        if (blo > bhi)
            for (int b = 0; b < B; ++b) store_bins<Acc, PPL>(outp(b), zero);
        else if (dir > 0)
            for (int b = bhi + 1; b < B; ++b) store_bins<Acc, PPL>(outp(b), zero);
        else
            for (int b = blo - 1; b >= 0; --b) store_bins<Acc, PPL>(outp(b), zero);
    }
    if (pwin.row) pwin.finish(lane);
}

// ADD: the scan's pass is 2 (compile-time, so that a single pass carries no
// code for adding onto an earlier output).  NORM: per-step sample weights
// (a.wk) apply.
template <typename Acc, int PPL, int WAVES, int PF, bool ADD, bool NORM = false,
          int CH = kPlanChunk, bool WT = false>
__device__ __forceinline__ void process_tile(const ScanArgs& a, int row, const TileAddr<Acc>& ta,
                                             PlanLds<Acc, CH>& L)
{
    const int cls = a.row_class[row];
    if (cls == kRowGeneric)
        process_tile_generic<Acc, PPL, WAVES, NORM, CH, WT>(a, row, ta, L);
    else if (cls & kRowNarrow)
        process_tile_mono<Acc, PPL, WAVES, PF, true, ADD, NORM, CH, WT>(a, row, ta, L, cls);
    else  // intervals wider than two bins: rare, a short prefetch suffices
        process_tile_mono<Acc, PPL, WAVES, (PF < 4 ? PF : 4), false, ADD, NORM, CH, WT>(a, row, ta,
                                                                                        L, cls);
}

template <int PPL, int WAVES, int PF, bool ADD>
__global__ __launch_bounds__(64 * WAVES) void rows_f32_kernel(ScanArgs a)
{
    __shared__ PlanLds<float> L;
    const int row = a.row_begin + (int)(blockIdx.x / (unsigned)a.tiles_per_row);
    const int tile = (int)(blockIdx.x % (unsigned)a.tiles_per_row);
    process_tile<float, PPL, WAVES, PF, ADD>(a, row, row_tile_addr<float, PPL, WAVES>(a, row, tile),
                                             L);
}

// FP64 instance: every pass is launched as a pass of its own (a two-edge
// reconstruction forms its second pass in a buffer of its own and adds the two
// afterwards), so there is no adding variant.
template <bool NORM>
__global__ __launch_bounds__(256) void rows_f64_kernel(ScanArgs a)
{
    __shared__ PlanLds<double> L;
    const int row = a.row_begin + (int)(blockIdx.x / (unsigned)a.tiles_per_row);
    const int tile = (int)(blockIdx.x % (unsigned)a.tiles_per_row);
    process_tile<double, 1, 4, 4, false, NORM>(a, row, row_tile_addr<double, 1, 4>(a, row, tile),
                                               L);
}

// Scans with per-step sample weights: one launch shape (a pixel per lane,
// four waves, 16 steps in flight).
template <bool ADD>
__global__ __launch_bounds__(256) void rows_norm_f32_kernel(ScanArgs a)
{
    __shared__ PlanLds<float> L;
    const int row = a.row_begin + (int)(blockIdx.x / (unsigned)a.tiles_per_row);
    const int tile = (int)(blockIdx.x % (unsigned)a.tiles_per_row);
    process_tile<float, 1, 4, 16, ADD, true>(a, row, row_tile_addr<float, 1, 4>(a, row, tile), L);
}

// Pixel lists (per-row plans): four independent wave tiles per workgroup,
// tiles [tile_first, tile_end) of the list's table; each wave stages its own
// row's plan, kWaveChunk intervals at a time.
constexpr int kWaveChunk = 256;

template <typename Acc, int PF, bool ADD, bool NORM>
__device__ __forceinline__ void list_wave_tile(const ScanArgs& a, const ListArgs& l,
                                               PlanLds<Acc, kWaveChunk>* L)
{
    const int wave = (int)(threadIdx.x >> 6);
    const int64_t t = l.tile_first + (int64_t)blockIdx.x * 4 + wave;
    if (t >= l.tile_end) return;  // no workgroup barrier follows
    const int row = l.tile_row[t];
    process_tile<Acc, 1, 1, PF, ADD, NORM, kWaveChunk, true>(
        a, row, list_wave_addr<Acc>(a, l, t, row), L[wave]);
}

template <int PF, bool ADD, bool NORM>
__global__ __launch_bounds__(256) void list_f32_kernel(ScanArgs a, ListArgs l)
{
    __shared__ PlanLds<float, kWaveChunk> L[4];
    list_wave_tile<float, PF, ADD, NORM>(a, l, L);
}

template <bool NORM>
__global__ __launch_bounds__(256) void list_f64_kernel(ScanArgs a, ListArgs l)
{
    __shared__ PlanLds<double, kWaveChunk> L[4];
    list_wave_tile<double, 4, false, NORM>(a, l, L);
}

// Persistent grid: workgroups pull (scan, tile) items until the queue is dry.
// Every scan of one launch has the same ADD.
template <int PPL, int WAVES, int PF, bool ADD>
__global__ __launch_bounds__(64 * WAVES) void batch_f32_kernel(BatchArgs b)
{
    __shared__ PlanLds<float> L;
    __shared__ unsigned long long s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(b.counter, 1ull);
        __syncthreads();
        const long long item = (long long)s_item;
        if (item >= b.total_tiles) break;
        int si = 0;
        while (si + 1 < b.n_scans && b.tile_start[si + 1] <= item) ++si;
        const ScanArgs a = b.scans[si];
        const long long t = item - b.tile_start[si];
        const int row = a.row_begin + (int)(t / a.tiles_per_row);
        const int tile = (int)(t % a.tiles_per_row);
        process_tile<float, PPL, WAVES, PF, ADD>(a, row,
                                                 row_tile_addr<float, PPL, WAVES>(a, row, tile), L);
    }
}

#define DR_CASE(KERNEL, P, W, F, ADD, GRID, ARGS, STREAM)                                \
    case P * 1000 + W * 100 + F:                                                         \
        hipLaunchKernelGGL((KERNEL<P, W, F, ADD>), GRID, dim3(64 * W), 0, STREAM, ARGS); \
        break;
#define DR_CASES_P(KERNEL, P, ADD, GRID, ARGS, STREAM)   \
    DR_CASE(KERNEL, P, 2, 4, ADD, GRID, ARGS, STREAM)    \
    DR_CASE(KERNEL, P, 2, 8, ADD, GRID, ARGS, STREAM)    \
    DR_CASE(KERNEL, P, 2, 16, ADD, GRID, ARGS, STREAM)   \
    DR_CASE(KERNEL, P, 4, 4, ADD, GRID, ARGS, STREAM)    \
    DR_CASE(KERNEL, P, 4, 8, ADD, GRID, ARGS, STREAM)    \
    DR_CASE(KERNEL, P, 4, 16, ADD, GRID, ARGS, STREAM)
#define DR_DISPATCH(T, KERNEL, ADD, GRID, ARGS, STREAM)              \
    do {                                                             \
        switch ((T).ppl * 1000 + (T).waves * 100 + (T).prefetch) {   \
            DR_CASES_P(KERNEL, 1, ADD, GRID, ARGS, STREAM)           \
            DR_CASES_P(KERNEL, 2, ADD, GRID, ARGS, STREAM)           \
            DR_CASES_P(KERNEL, 4, ADD, GRID, ARGS, STREAM)           \
            DR_CASES_P(KERNEL, 8, ADD, GRID, ARGS, STREAM)           \
        default: return hipErrorInvalidValue;                        \
        }                                                            \
    } while (0)

}  // namespace dr
