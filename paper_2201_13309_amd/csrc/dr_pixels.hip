// Per-pixel path (gfx950): geometries whose detector rows do not share one
// projected position (a tilted detector, a wire axis not along x, an explicit
// pixel table), so every pixel computes its own FP64 edge positions, one per
// wire step, in the fixed operation order of the tangent construction (the
// paper leaves the geometry to the wire-scan method it cites; the construction
// here is the reading stated in the library header) without contraction, and
// spreads each intensity difference over the bins its interval overlaps
// (Sec. III-C: each pixel's differences are added into depth arrays).
//
//   pixels_f32_kernel  FP32 accumulation.  ALU-bound: per (pixel, step) one
//                      FP64 square root and one FP64 division, in a shorter
//                      form (dr_fastpos.h) whose floors are certified at
//                      init, exact where they are not; a step inside one bin
//                      costs an integer add, a step across a bin boundary one
//                      FP64 reciprocal and one FP64 fma; wire positions come
//                      through scalar loads; totals are summed in a fixed
//                      order through per-wave LDS rings.
//   pixels_kernel      FP64 instance (validation): each overlap divided by the
//                      length in FP64, the oracle's order of accumulation.
#include <type_traits>

#include "dr_device.h"
#include "dr_fastpos.h"

#pragma clang fp contract(off)

namespace dr {

// tangent_depth for the per-pixel kernels: the square root always in its
// Newton form.  dr_geometry_init checks for these geometries that
// L2 - r^2 >= 2^-767 at every pixel and wire step, where the Newton form and
// the guarded one in tangent_depth give the same bits.  rr is the product
// r * r.
__device__ __forceinline__ double tangent_depth_checked(double py, double pz, double cy,
                                                       double cz, double rr, double sr)
{
    const double ay = cy - py;
    const double az = cz - pz;
    const double L2 = az * az + ay * ay;
    const double kk = sqrt_newton(L2 - rr);
    const double tz = az * kk - ay * sr;
    const double ty = ay * kk + az * sr;
    return cz - (cy * tz + sr * L2) / ty;
}

// Edge position in bin units times `sinvw` = (+-1) / width: the position u,
// or -u for a walk that runs the other way (exact: a sign); TILT: the wire
// axis has a z component, so the tangent point's xi is divided by c = e1.z;
// otherwise c is exactly 1 and the division (t / 1 == t) is left out.  rr is
// the product r * r.
template <bool TILT>
__device__ __forceinline__ double position_at(double cy, double cz, double py, double pz,
                                              double rr, double sr, double c, double e0,
                                              double sinvw)
{
    const double t = tangent_depth_checked(py, pz, cy, cz, rr, sr);
    const double d = TILT ? t / c : t;
    return (d - e0) * sinvw;
}

struct PlanF {
    int bl, nb;      // first bin (natural order) and number of bins
    float f0, fm, f1;
};

// The bins of the interval between positions u0 and u1 (bin units) that it
// overlaps by a positive length, as make_plan finds them, without its loops:
// floor(lo) can only fail to overlap when it was clamped up to 0 past hi, and
// floor(hi) only when hi is exactly that integer (then the bin below it is the
// last one), so after one correction of the last bin the interval is empty
// exactly when first > last.  fl0 and fl1 are floor(u0) and floor(u1) (the
// floor of the smaller end is the smaller floor).  Fractions overlap/length in
// FP32, from one reciprocal of the length.
__device__ __forceinline__ PlanF plan_f32(double u0, double u1, double fl0, double fl1, int B)
{
    PlanF e;
    // positions are finite (checked when the geometry is built), so min and
    // max need no NaN rules
    const double lo = __builtin_fmin(u0, u1), hi = __builtin_fmax(u0, u1);
    const double flo = __builtin_fmin(fl0, fl1), fhi = __builtin_fmax(fl0, fl1);
    const double len = hi - lo;
    const double top = uni((double)(B - 1));
    if (len > 0.0) {
        const double f = __builtin_fmax(flo, 0.0);
        double l = __builtin_fmin(fhi, top);
        if (hi == l) l -= 1.0;
        const bool any = f <= l;
        const double ovf = __builtin_fmin(hi, f + 1.0) - __builtin_fmax(lo, f);
        const double ovl = __builtin_fmin(hi, l + 1.0) - __builtin_fmax(lo, l);
        const float rl = __builtin_amdgcn_rcpf((float)len);
        e.bl = (int)(any ? f : 0.0);
        e.nb = any ? (int)(l - f) + 1 : 0;
        // an interval inside one bin puts all of it there (ov/len is exactly 1)
        e.f0 = ovf == len ? 1.0f : (float)ovf * rl;
        e.f1 = ovl == len ? 1.0f : (float)ovl * rl;
        e.fm = rl;
    } else {  // a point: all of it in bin floor(lo), if that bin exists
        const bool in = flo >= 0.0 && flo <= top;
        e.bl = (int)(in ? flo : 0.0);
        e.nb = in ? 1 : 0;
        e.f0 = e.fm = e.f1 = 1.0f;
    }
    return e;
}

constexpr int kPixelWaves = kPixelTile / 64;
static_assert(kPixelPartialRows == kPixelWaves + 1, "a partial row per wave, one for atomics");

// Totals of the FP32 kernel, summed in a fixed order.  Each wave owns a ring
// of kRingBins bins x 64 lanes in LDS: the lane that closes bin p (counted in
// its walk direction) writes its value into slot (p mod kRingBins, lane)
// while p lies in the ring's window [F, F + kRingBins).  At the start of each
// block of steps the bins below the wave's lowest open bin are complete; each
// is summed over the 64 lanes in a fixed tree and stored into the wave's own
// partial row in device memory (every bin of that row is written once: a sum,
// or zero for a bin the window never held), and the window moves up.  A
// close outside the window (a walk that turns back, lanes of one wave far
// apart, lanes walking opposite ways) adds into the workgroup's fifth row
// with a device atomic instead; only those closes are order-dependent.  The
// rows live in device memory rather than LDS so that the LDS of a workgroup
// is its four rings alone, and six waves fit on a SIMD.
constexpr int kRingBins = 16;
constexpr size_t kRingBytes = (size_t)kPixelWaves * kRingBins * 64 * sizeof(float);

// Prefetch depth PF of the FP32 per-pixel kernel; a block of steps between
// two flushes of the ring is PF + 1 steps, within which a lane's fast steps
// move it by at most PF + 1 bins.  Twelve-step blocks where the registers
// allow it (the instances without step weights and axis tilt: 1.6% faster
// than nine); nine where the weights or the tilted axis's division need the
// registers (twelve spill there and are slower).
constexpr int pixel_pf(bool norm, bool tilt) { return (norm || tilt) ? 8 : 11; }
static_assert(pixel_pf(false, false) + 1 < kRingBins && pixel_pf(true, true) + 1 < kRingBins,
              "a block of steps fits the ring's window");

// v from the DPP source lane; lanes without one (or in rows outside ROW_MASK)
// keep their own v
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_keep(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, ROW_MASK, 0xf, false);
}

// minimum over the 64 lanes of a wave, as a uniform value
__device__ __forceinline__ int wave_min(int v)
{
    v = min(v, dpp_keep<0x111, 0xf>(v));  // row_shr:1
    v = min(v, dpp_keep<0x112, 0xf>(v));  // row_shr:2
    v = min(v, dpp_keep<0x114, 0xf>(v));  // row_shr:4
    v = min(v, dpp_keep<0x118, 0xf>(v));  // row_shr:8
    v = min(v, dpp_keep<0x142, 0xa>(v));  // row_bcast:15 into rows 1 and 3
    v = min(v, dpp_keep<0x143, 0xc>(v));  // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(v, 63);
}

// FP32 per-pixel kernel: one lane per pixel of a row tile (or of a list tile,
// as in the FP64 instance below).  The lane's FP64 positions u_k (bin units;
// position_fast, or position_at where the fast form lies within the
// geometry's margin of an integer, so that every floor is the exact
// position's) are turned into its walk direction by v = sgn*u, with sgn = +1
// when its positions rise over the scan and -1 otherwise (negation is
// exact); bin p = floor(v) + off (off = 0, or B for sgn = -1) counts bins in
// the order the walk meets them (p = b, or B - 1 - b).  Bins below the open
// bin `nxt` are stored; bin nxt accumulates.
//
// Fast form: the step starts in the open bin and ends in it or in the next
// one.  Let C(x) be the mass of the intervals so far below x; a bin holds
// C(upper boundary) - C(lower boundary).  In a walk of this kind every
// earlier interval lies below the open bin's upper boundary bd, so C(bd) is
// the mass before the step (the sum of the differences so far, kept exactly:
// an integer, or FP64 with step weights) plus the step's part below bd,
// dI_k (bd - v_k) / (v_{k+1} - v_k).  A step that stays inside the open bin
// costs one integer add; one that crosses bd costs one FP64 fma and stores
// the closed bin.  The values differ from the per-step sums only by rounding:
// the fraction carries the hardware FP64 reciprocal of the length (relative
// error about 2^-24), each C one FP64 rounding, the stored difference one
// FP32 rounding.
//
// General form, for any other step (entering or leaving the grid, more than
// one boundary in a step, a walk that turns back): the interval's bins and
// fractions (plan_f32) are visited one by one, the open bin's value `acc` in
// FP32.  acc is taken from C as the mass so far minus the mass below the open
// bin (`clast`), and given back the same way; nothing lies above the open
// bin, so the two agree.  A bin behind nxt that is visited again is read,
// added to and rewritten.
//
// Untouched bins are stored as zeros, except in the second pass of a
// two-edge reconstruction (ADD), whose values are added onto the first
// pass's.  Values are scaled (by +-1 or +-1/2, exactly) as they are stored.
template <int PF, bool NORM, bool TILT, bool ADD>
// Six waves per SIMD (at most 80 VGPRs, all of them used by the main
// instance, with the wave-uniform values in scalar registers): 7% faster than
// five; seven (72) spill inside the step loop and are slower.
__global__ __launch_bounds__(kPixelTile, 6) void pixels_f32_kernel(ScanArgs a, GeomArgs g, int side,
                                                                float scale, ListArgs l)
{
    using Cum = typename std::conditional<NORM, double, int>::type;
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int N = a.n_steps, B = a.n_bins, nint = N - 1;
    const bool tot = a.partials != nullptr;
    // wire positions: the same for every lane, read with scalar loads
    typedef const __attribute__((address_space(4))) double cdouble;
    const cdouble* const wire = (const cdouble*)g.wire_yz;
    bool act;
    int64_t pixel, slot;
    const uint16_t* ip;
    float* op;
    if (l.pixels) {
        const int64_t t = l.tile_first + blockIdx.x;
        const int64_t e0 = l.tile_start[t];
        const int64_t base = e0 & ~(int64_t)(kListAlign - 1);
        act = base + tid >= e0 && base + tid < e0 + l.tile_count[t];
        const int64_t e = act ? base + tid : e0;
        pixel = l.pixels[e];
        ip = l.compact ? a.img + (e - l.entry_base) : a.img + pixel;
        op = (float*)a.out + base + tid;
        slot = t;
    } else {
        const int row = a.row_begin + (int)(blockIdx.x / (unsigned)a.tiles_per_row);
        const int tile = (int)(blockIdx.x % (unsigned)a.tiles_per_row);
        const int col = tile * kPixelTile + tid;
        act = col < a.nx;
        const int ccol = act ? col : a.nx - 1;  // lanes past the row's end follow its last pixel
        pixel = (int64_t)row * a.nx + ccol;
        ip = a.img + (int64_t)(row - a.row_base) * a.img_row + ccol;
        op = (float*)a.out + (int64_t)row * a.nx + col;
        slot = (int64_t)row * a.tiles_per_row + tile;
    }
    // totals: the wave's ring in LDS, its partial row and the workgroup's
    // atomics row in the partials buffer (kPixelPartialRows per workgroup)
    float* const gbase = tot ? (float*)a.partials + slot * kPixelPartialRows * B : nullptr;
    const int uwave = __builtin_amdgcn_readfirstlane(wave);  // uniform: a scalar row base
    float* const gw = tot ? gbase + (int64_t)uwave * B : nullptr;
    float* const gp = tot ? gbase + (int64_t)kPixelWaves * B : nullptr;
    float* const ring = reinterpret_cast<float*>(dyn_lds) + wave * (kRingBins * 64);
    float* const ring_lane = ring + lane;  // this lane's slot of ring bin 0
    if (tot) {
        for (int i = lane; i < kRingBins * 64; i += 64) ring[i] = 0.0f;
        for (int b = tid; b < B; b += kPixelTile) gp[b] = 0.0f;
        __syncthreads();  // cleared before any wave adds
    }

    const Frame f = axis_frame(g);
    double py, pz;
    pixel_key(g, f, pixel, py, pz);
    const int s = side ? -leading_sign(g, py, pz) : leading_sign(g, py, pz);
    // wave-uniform values through readfirstlane, so that they are held in
    // scalar registers (the vector registers bound the kernel's occupancy)
    const double r = uni(g.radius), sr = (double)s * g.radius, rr = uni(r * r);
    const double e0 = uni(g.first_center - g.width / 2.0);
    const double invw = 1.0 / g.width;
    const double c = uni(f.c);
    const double u_first =
        position_at<TILT>(g.wire_yz[0], g.wire_yz[1], py, pz, rr, sr, c, e0, invw);
    const double u_last = position_at<TILT>(g.wire_yz[2 * (N - 1)], g.wire_yz[2 * (N - 1) + 1],
                                            py, pz, rr, sr, c, e0, invw);
    const int dir = (u_last >= u_first) ? 1 : -1;
    const double sgn = (double)dir, sinvw = sgn * invw;
    const double margin = g.pos_margin, half_in = uni(0.5 - margin);
    FastPos fp;
    fp.py = py;
    fp.pz = pz;
    fp.sr = sr;
    fp.mrr = uni(-rr);
    fp.srrr = sr * rr;
    fp.scale = TILT ? sinvw / c : sinvw;
    fp.offs = -e0 * sinvw;
    const int off = dir > 0 ? 0 : B;
    // |u| < 2^30 and B <= 2^30 (checked when the geometry is built): exact in int
    auto pbin = [&](double v) { return (int)__builtin_floor(v) + off; };
    const bool up_w = __all(dir > 0), down_w = __all(dir < 0);  // wave-uniform
    const bool uni = up_w || down_w;
    const bool ring_on = tot && uni;
    const int64_t plane = a.out_plane;
    const int64_t ostep = dir > 0 ? plane : -plane;
    auto nat = [&](int p) { return dir > 0 ? p : B - 1 - p; };

    int F = 0;  // the ring's window [F, F + kRingBins) (wave-uniform)
    auto atomic_total = [&](int b, float v) {  // b: natural bin
        __hip_atomic_fetch_add(&gp[b], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto put_total = [&](int p, float v) {  // this lane closed bin p with value v
        if (!tot || !act) return;
        if (ring_on && (unsigned)(p - F) < (unsigned)kRingBins)
            ring_lane[(p & (kRingBins - 1)) * 64] = v;
        else
            atomic_total(nat(p), v);
    };
    // bins [F, upto) are complete for every lane of the wave: sum their ring
    // slots over the lanes (16 lanes per quarter in order, then the quarters
    // pairwise) into the wave's row, clear them, and move the window; bins of
    // [F, upto) beyond the window were never held: zero in the row
    auto flush = [&](int upto) {
        const int n = min(upto, F + kRingBins) - F;
        if (n > 0) {
            const int si = lane & (kRingBins - 1), q = lane >> 4;
            float v = 0.0f;
            if (si < n) {
                f32x4* rs = reinterpret_cast<f32x4*>(
                    ring + ((F + si) & (kRingBins - 1)) * 64 + 16 * q);
                const f32x4 r0 = rs[0], r1 = rs[1], r2 = rs[2], r3 = rs[3];
                v = (((r0.x + r0.y) + (r0.z + r0.w)) + ((r1.x + r1.y) + (r1.z + r1.w))) +
                    (((r2.x + r2.y) + (r2.z + r2.w)) + ((r3.x + r3.y) + (r3.z + r3.w)));
                const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                rs[0] = z;
                rs[1] = z;
                rs[2] = z;
                rs[3] = z;
            }
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (q == 0 && si < n) {
                const int p = F + si;
                gw[up_w ? p : B - 1 - p] = v;
            }
        }
        for (int p = F + kRingBins + lane; p < upto; p += 64) gw[up_w ? p : B - 1 - p] = 0.0f;
        F = max(F, upto);
    };
    if (ring_on) {  // start the window just below the lowest first bin of the wave
        const int p0 = min(max(pbin(sgn * u_first), 0), B);
        F = max(0, wave_min(act ? p0 : B) - 1);
    }
    const int F0 = F;  // bins below it (walk order) are never held: zero in the row

    int nxt = 0;  // first bin (walk order) not stored
    // the lane's element of bin nxt; after the last bin it is moved once more
    // and never used again (an integer address instead measured 6% slower)
    float* on = op + (dir > 0 ? 0 : (int64_t)(B - 1) * plane);
    bool open = false;
    double clast = 0.0;  // when open: mass below the open bin (unscaled)
    Cum cum = 0;         // mass of the steps so far (unscaled)
    float prev = 0.0f;   // ADD: the first pass's value of the open bin
    // store the open bin with this pass's value v (unscaled); move to the next
    auto emit = [&](float v) {
        v *= scale;
        if (act) stream_store(ADD ? prev + v : v, on);
        put_total(nxt, v);
        on += ostep;
        ++nxt;
    };
    // general form of one step from walk position vp to vn; returns the open
    // bin's value
    auto general = [&](double vp, double vn, float dI) {
        // The natural positions and their floors are formed here only: the
        // empty statement keeps the compiler from computing them ahead of the
        // branch on every step, where the fast form has no use for them.
        asm volatile("" : "+v"(vp), "+v"(vn));
        const double u_prev = sgn * vp, u_next = sgn * vn;
        float acc = open ? (float)((double)cum - clast) : 0.0f;
        auto bin = [&](int p, float fr) {
            if (open && p == nxt) {
                acc = madd(fr, dI, acc);
            } else if (p > nxt || (p == nxt && !open)) {
                if (open) {
                    emit(acc);
                    open = false;
                }
                for (; nxt < p; ++nxt, on += ostep)
                    if (!ADD && act) stream_store(0.0f, on);
                if (ADD && act) prev = *on;
                acc = fr * dI;
                open = true;
            } else if (act) {  // stored already: read, add, rewrite
                const int b = nat(p);
                float* o = op + (int64_t)b * plane;
                const float v = (fr * dI) * scale;
                *o = *o + v;
                if (tot) atomic_total(b, v);
            }
        };
        const PlanF e =
            plan_f32(u_prev, u_next, __builtin_floor(u_prev), __builtin_floor(u_next), B);
        if (e.nb > 0) {
            const int bh = e.bl + e.nb - 1;
            const int p0 = dir > 0 ? e.bl : B - 1 - bh;
            bin(p0, dir > 0 ? e.f0 : e.f1);
            if (e.nb > 1) {
                for (int q = 1; q + 1 < e.nb; ++q) bin(p0 + q, e.fm);
                bin(p0 + e.nb - 1, dir > 0 ? e.f1 : e.f0);
            }
        }
        return acc;
    };

    double v_prev = sgn * u_first;
    // open, and the last position lies in the open bin: true after every
    // step of the fast form (it keeps the bin open and moves nxt with it)
    bool ok = false;
    // the wire position of the coming step, loaded one step ahead (the table
    // repeats its last position twice: no clamp)
    double wy = wire[2], wz = wire[3];
    auto step = [&](int k, int s0, int s1) {
        const double cy = wy, cz = wz;
        wy = wire[2 * (unsigned)(k + 2)];
        wz = wire[2 * (unsigned)(k + 2) + 1];
        double v_next = position_fast(cy, cz, fp);
        double fl = __builtin_floor(v_next);
        const double fr = v_next - fl;  // exact: |v| < 2^30
        // fr within the margin of 0 or 1: the exact position
        bool zero_int = false;
        if (!(__builtin_fabs(fr - 0.5) < half_in)) {
            v_next = position_at<TILT>(cy, cz, py, pz, rr, sr, c, e0, sinvw);
            fl = __builtin_floor(v_next);
            // a zero-length step of a falling walk is a point mass in bin
            // floor(u), which is floor(v)'s bin unless u is an integer (then
            // the general form): such a position is always evaluated here
            zero_int = dir < 0 && v_next == v_prev;
        }
        const int p_next = (int)fl + off;
        Cum dI;  // this step's intensity difference (unscaled)
        if constexpr (NORM)
            dI = (double)s0 * a.wk[k] - (double)s1 * a.wk[k + 1];
        else
            dI = s0 - s1;
        const int d = p_next - nxt;
        // chosen per lane from its own walk alone, so that a pixel's values do
        // not depend on the pixels it shares a wave with
        const bool fast = ok && (unsigned)d <= 1u && p_next <= B - 1 && !zero_int;
        if (fast) {
            if (d != 0) {  // the step crosses the open bin's upper boundary bd = fl
                const double rl = __builtin_amdgcn_rcp(v_next - v_prev);  // ~2^-24 relative
                const double bd = fl;
                const double cb = __builtin_fma((bd - v_prev) * rl, (double)dI, (double)cum);
                emit((float)(cb - clast));
                if (ADD && act) prev = *on;
                clast = cb;
            }
        } else {
            const float acc = general(v_prev, v_next, (float)dI);
            if (open) clast = ((double)cum + (double)dI) - (double)acc;
            ok = open && p_next == nxt;
        }
        cum += dI;
        v_prev = v_next;
    };

    // ring of U samples: slot k % U holds step k; blocks of U steps
    constexpr int U = PF + 1;
    unsigned short smp[U];
    // sample k at ip + k * img_step: an unsigned 32 x 32 -> 64-bit product
    // (k < 2^31, img_step <= ny * nx < 2^32)
    const uint32_t istep = (uint32_t)a.img_step;
    auto sample_at = [&](int k) {
        return stream_load(ip + (uint64_t)(uint32_t)min(k, N - 1) * istep);
    };
#pragma unroll
    for (int dd = 0; dd < U; ++dd) smp[dd] = sample_at(dd);
    int k0 = 0;
    for (; k0 + U <= nint; k0 += U) {
        if (ring_on) flush(wave_min(act ? nxt : B));
#pragma unroll
        for (int dd = 0; dd < U; ++dd) {
            step(k0 + dd, (int)smp[dd], (int)smp[(dd + 1) % U]);
            smp[dd] = sample_at(k0 + dd + U);
        }
    }
    if (ring_on) flush(wave_min(act ? nxt : B));
#pragma unroll
    for (int dd = 0; dd < U; ++dd)
        if (k0 + dd < nint) step(k0 + dd, (int)smp[dd], (int)smp[(dd + 1) % U]);
    if (open) {
        emit((float)((double)cum - clast));
        open = false;
    }
    if (!ADD)
        for (; nxt < B; ++nxt, on += ostep)
            if (act) stream_store(0.0f, on);
    if (tot) {  // complete the wave's row: every bin written once
        if (ring_on) {
            flush(B);
            for (int p = lane; p < F0; p += 64) gw[up_w ? p : B - 1 - p] = 0.0f;
        } else {
            for (int b = lane; b < B; b += 64) gw[b] = 0.0f;
        }
    }
}

// FP64 instance of the per-pixel path: one lane per pixel of a row tile of
// kPixelTile pixels; every pass is launched as a pass of its own (the second
// pass of two edges writes into a buffer of its own).  Each
// lane computes its own FP64 positions step by step, plans the interval, and
// streams its bins in the direction its edge moves (bins are visited in order
// then; a bin already stored and visited again is read, added to and
// rewritten, so any sequence of positions is handled).  Partial totals are
// accumulated per workgroup in LDS and written as one row per workgroup.
// With a pixel list (l.pixels set) workgroup w takes list tile
// l.tile_first + w: lane i holds entry tile_start + i, its output goes to
// column `entry` of [n_bins][n], and its images are gathered from full frames
// (pixel index) or read from a compact [N][entries] buffer.
template <typename Acc, int PF, bool NORM>
__global__ __launch_bounds__(kPixelTile) void pixels_kernel(ScanArgs a, GeomArgs g, int side,
                                                            double scale, ListArgs l)
{
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    const int tid = threadIdx.x;
    const int N = a.n_steps, B = a.n_bins;
    const bool tot = a.partials != nullptr;
    bool act;
    int64_t pixel, slot;              // pixel index; partial-total row of the workgroup
    const uint16_t* ip;               // the lane's step-0 sample
    Acc* op;                          // the lane's bin 0
    if (l.pixels) {
        const int64_t t = l.tile_first + blockIdx.x;
        const int64_t e0 = l.tile_start[t];
        const int64_t base = e0 & ~(int64_t)(kListAlign - 1);
        act = base + tid >= e0 && base + tid < e0 + l.tile_count[t];
        const int64_t e = act ? base + tid : e0;
        pixel = l.pixels[e];
        ip = l.compact ? a.img + (e - l.entry_base) : a.img + pixel;
        op = (Acc*)a.out + base + tid;
        slot = t;
    } else {
        const int row = a.row_begin + (int)(blockIdx.x / (unsigned)a.tiles_per_row);
        const int tile = (int)(blockIdx.x % (unsigned)a.tiles_per_row);
        const int col = tile * kPixelTile + tid;
        act = col < a.nx;
        pixel = (int64_t)row * a.nx + (act ? col : 0);
        ip = a.img + (int64_t)(row - a.row_base) * a.img_row + (act ? col : 0);
        op = (Acc*)a.out + (int64_t)row * a.nx + col;
        slot = (int64_t)row * a.tiles_per_row + tile;
    }
    // the workgroup's partial-total row: summed in LDS when it fits, else in
    // place in its own row of the partials buffer
    Acc* const gp = tot ? (Acc*)a.partials + slot * B : nullptr;
    const bool in_lds = (size_t)B * sizeof(Acc) <= kPixelLdsBytes;
    Acc* const ltot = in_lds ? reinterpret_cast<Acc*>(dyn_lds) : gp;
    if (tot)
        for (int b = tid; b < B; b += kPixelTile) ltot[b] = (Acc)0;
    __syncthreads();

    const Frame f = axis_frame(g);
    double py, pz;
    pixel_key(g, f, pixel, py, pz);
    const int s = side ? -leading_sign(g, py, pz) : leading_sign(g, py, pz);
    const double sr = (double)s * g.radius;
    const double e0 = g.first_center - g.width / 2.0;
    const double invw = 1.0 / g.width;
    const double u_first = edge_position(g, py, pz, 0, sr, f.c, e0, invw);
    const double u_last = edge_position(g, py, pz, N - 1, sr, f.c, e0, invw);
    const int dir = (u_last >= u_first) ? 1 : -1;

    const int64_t plane = a.out_plane;
    auto binp = [&](int bp) { return dir > 0 ? bp : B - 1 - bp; };

    Acc acc = (Acc)0;
    Acc tacc = (Acc)0;  // this pass's contributions to the open bin, for the totals
    int cbp = -1;  // open bin in the direction frame (-1: none); when open, cbp == nxt
    int nxt = 0;   // first bin (direction frame) not yet stored
    auto store = [&](int bp, Acc v) {
        if (act) stream_store(v, op + (int64_t)binp(bp) * plane);
    };
    auto close_open = [&]() {
        if (cbp >= 0) {
            store(cbp, acc);
            if (tot && act) atomicAdd(&ltot[binp(cbp)], tacc);
            nxt = cbp + 1;
            cbp = -1;
        }
    };
    auto visit = [&](int b, Acc fr, Acc dI) {
        const int bp = dir > 0 ? b : B - 1 - b;
        if (bp == cbp) {
            acc = madd(fr, dI, acc);
            tacc = madd(fr, dI, tacc);
        } else if (bp >= nxt) {
            close_open();
            for (int z = nxt; z < bp; ++z) store(z, (Acc)0);
            cbp = bp;
            nxt = bp;
            acc = madd(fr, dI, (Acc)0);
            tacc = acc;
        } else if (act) {  // stored already: read, add, rewrite
            Acc* o = op + (int64_t)b * plane;
            *o = madd(fr, dI, *o);
            if (tot) atomicAdd(&ltot[b], fr * dI);
        }
    };

    constexpr int U = PF + 1;
    unsigned short ring[U];
#pragma unroll
    for (int d = 0; d < U; ++d) ring[d] = stream_load(ip + (int64_t)min(d, N - 1) * a.img_step);
    double u_prev = u_first;
    int k = 0;
    for (; k + U <= N - 1; k += U) {
#pragma unroll
        for (int d = 0; d < U; ++d) {
            const double u_next = edge_position(g, py, pz, k + d + 1, sr, f.c, e0, invw);
            const PlanD e = make_plan<(sizeof(Acc) == 8)>(u_prev, u_next, B);
            const Acc dI =
                sample_diff<Acc, NORM>((int)ring[d], (int)ring[(d + 1) % U], a.wk, k + d);
            const Acc f0 = (Acc)(e.f0 * scale), fm = (Acc)(e.fm * scale), f1 = (Acc)(e.f1 * scale);
            const int bh = e.bl + e.nb - 1;
            int b = dir > 0 ? e.bl : bh;
            for (int q = 0; q < e.nb; ++q, b += dir)
                visit(b, (b == e.bl) ? f0 : ((b == bh) ? f1 : fm), dI);
            u_prev = u_next;
            ring[d] = stream_load(ip + (int64_t)min(k + d + U, N - 1) * a.img_step);
        }
    }
#pragma unroll
    for (int d = 0; d < U; ++d) {
        if (k + d < N - 1) {
            const double u_next = edge_position(g, py, pz, k + d + 1, sr, f.c, e0, invw);
            const PlanD e = make_plan<(sizeof(Acc) == 8)>(u_prev, u_next, B);
            const Acc dI =
                sample_diff<Acc, NORM>((int)ring[d], (int)ring[(d + 1) % U], a.wk, k + d);
            const Acc f0 = (Acc)(e.f0 * scale), fm = (Acc)(e.fm * scale), f1 = (Acc)(e.f1 * scale);
            const int bh = e.bl + e.nb - 1;
            int b = dir > 0 ? e.bl : bh;
            for (int q = 0; q < e.nb; ++q, b += dir)
                visit(b, (b == e.bl) ? f0 : ((b == bh) ? f1 : fm), dI);
            u_prev = u_next;
        }
    }
    close_open();
    for (int z = nxt; z < B; ++z) store(z, (Acc)0);
    if (tot && in_lds) {
        __syncthreads();
        for (int b = tid; b < B; b += kPixelTile) gp[b] = ltot[b];
    }
}

// ---------------------------------------------------------- launch wrappers

template <typename Acc>
static hipError_t launch_pixels(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                                const ListArgs* l, int64_t n_tiles, hipStream_t s)
{
    const int64_t groups = l ? n_tiles : (int64_t)(a.row_end - a.row_begin) * a.tiles_per_row;
    if (groups <= 0) return hipSuccess;
    size_t lds = 0;
    if (a.partials) {
        if (sizeof(Acc) == 4)
            lds = kRingBytes;
        else
            lds = (size_t)a.n_bins * sizeof(Acc) <= kPixelLdsBytes ? (size_t)a.n_bins * sizeof(Acc)
                                                                    : 0;
    }
    const ListArgs none{};
    const ListArgs& la = l ? *l : none;
    const dim3 grid((unsigned)groups), block(kPixelTile);
    if constexpr (sizeof(Acc) == 4) {
        // an axis without a z component has c == 1 exactly
        const bool tilt = g.axis[2] != 0.0;
        const float sc = (float)scale;  // +-1 or +-1/2
        const int v = (a.wk ? 1 : 0) + (tilt ? 2 : 0) + (a.pass == 2 ? 4 : 0);
        switch (v) {
#define DR_PIX(V, NORM, TILT, ADD)                                                              \
    case V:                                                                                     \
        hipLaunchKernelGGL((pixels_f32_kernel<pixel_pf(NORM, TILT), NORM, TILT, ADD>), grid,    \
                           block, lds, s, a, g, side, sc, la);                                  \
        break;
            DR_PIX(0, false, false, false)
            DR_PIX(1, true, false, false)
            DR_PIX(2, false, true, false)
            DR_PIX(3, true, true, false)
            DR_PIX(4, false, false, true)
            DR_PIX(5, true, false, true)
            DR_PIX(6, false, true, true)
            DR_PIX(7, true, true, true)
#undef DR_PIX
        default: break;
        }
    } else {
        if (a.wk)
            hipLaunchKernelGGL((pixels_kernel<Acc, 8, true>), grid, block, lds, s, a, g, side,
                               scale, la);
        else
            hipLaunchKernelGGL((pixels_kernel<Acc, 8, false>), grid, block, lds, s, a, g, side,
                               scale, la);
    }
    return hipGetLastError();
}

hipError_t launch_pixels_f32(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                             hipStream_t s)
{
    return launch_pixels<float>(a, g, side, scale, nullptr, 0, s);
}

hipError_t launch_pixels_f64(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                             hipStream_t s)
{
    return launch_pixels<double>(a, g, side, scale, nullptr, 0, s);
}

hipError_t launch_list_pixels_f32(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                                  const ListArgs& l, int64_t n_tiles, hipStream_t s)
{
    return launch_pixels<float>(a, g, side, scale, &l, n_tiles, s);
}

hipError_t launch_list_pixels_f64(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                                  const ListArgs& l, int64_t n_tiles, hipStream_t s)
{
    return launch_pixels<double>(a, g, side, scale, &l, n_tiles, s);
}

}  // namespace dr
