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
//                      FP64 square root and one FP64 division; the interval's
//                      plan is straight-line code and its fractions come from
//                      one FP32 reciprocal; wire positions are staged in LDS.
//   pixels_kernel      FP64 instance (validation): each overlap divided by the
//                      length in FP64, the oracle's order of accumulation.
#include "dr_device.h"

#pragma clang fp contract(off)

namespace dr {

// Edge position in bin units; TILT: the wire axis has a z component, so the
// tangent point's xi is divided by c = e1.z; otherwise c is exactly 1 and the
// division (t / 1 == t) is left out.
template <bool TILT>
__device__ __forceinline__ double position_at(double cy, double cz, double py, double pz,
                                              double r, double sr, double c, double e0,
                                              double invw)
{
    const double t = tangent_depth(py, pz, cy, cz, r, sr);
    const double d = TILT ? t / c : t;
    return (d - e0) * invw;
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
    const double top = (double)(B - 1);
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

constexpr int kWireChunk = 512;  // wire positions staged in LDS at a time
constexpr int kPixelTotalCopies = 4;  // copies of the LDS partial totals (FP32 kernel)

// FP32 per-pixel kernel: one lane per pixel of a row tile (or of a list tile,
// as in the FP64 instance below).  Each lane walks its bins in the direction
// its edge moves (direction frame p: p = b when the positions increase, else
// p = B-1-b): bins below `nxt` are stored; when `open`, bin `nxt` is
// accumulating in `acc` (and this pass's part of it in `tacc`, for the
// totals).  A bin behind `nxt` that is visited again (a position sequence that
// turns back) is read, added to and rewritten.  Untouched bins are stored as
// zeros, except in the second pass of a two-edge reconstruction, which only
// adds.  Partial totals are summed per workgroup in LDS when they fit, else in
// the workgroup's own row of the partials buffer.
template <int PF, bool NORM, bool TILT, bool ADD>
__global__ __launch_bounds__(kPixelTile) void pixels_f32_kernel(ScanArgs a, GeomArgs g, int side,
                                                                float scale, ListArgs l)
{
    __shared__ double wyz[2 * kWireChunk];
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    const int tid = threadIdx.x;
    const int N = a.n_steps, B = a.n_bins, nint = N - 1;
    constexpr bool add_on = ADD;  // the second pass of two (compile-time: no output reads otherwise)
    const bool tot = a.partials != nullptr;
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
        pixel = (int64_t)row * a.nx + (act ? col : 0);
        ip = a.img + (int64_t)(row - a.row_base) * a.img_row + (act ? col : 0);
        op = (float*)a.out + (int64_t)row * a.nx + col;
        slot = (int64_t)row * a.tiles_per_row + tile;
    }
    // the workgroup's partial totals: in LDS, four copies (one per 16-lane
    // row of a wave, so that the lanes of a wave adding to one bin meet at
    // most 16 to an address), summed at the end; in place in the workgroup's
    // row of the partials buffer when they do not fit
    float* const gp = tot ? (float*)a.partials + slot * B : nullptr;
    const bool in_lds = (size_t)B * kPixelTotalCopies * sizeof(float) <= kPixelLdsBytes;
    float* const ltot = reinterpret_cast<float*>(dyn_lds);
    const int lane = (int)(threadIdx.x & 63);
    if (tot) {
        if (in_lds)
            for (int b = tid; b < kPixelTotalCopies * B; b += kPixelTile) ltot[b] = 0.0f;
        else
            for (int b = tid; b < B; b += kPixelTile) gp[b] = 0.0f;
    }

    const Frame f = axis_frame(g);
    double py, pz;
    pixel_key(g, f, pixel, py, pz);
    const int s = side ? -leading_sign(g, py, pz) : leading_sign(g, py, pz);
    const double r = g.radius, sr = (double)s * g.radius;
    const double e0 = g.first_center - g.width / 2.0;
    const double invw = 1.0 / g.width;
    const double c = f.c;
    const double u_first =
        position_at<TILT>(g.wire_yz[0], g.wire_yz[1], py, pz, r, sr, c, e0, invw);
    const double u_last = position_at<TILT>(g.wire_yz[2 * (N - 1)], g.wire_yz[2 * (N - 1) + 1],
                                            py, pz, r, sr, c, e0, invw);
    const int dir = (u_last >= u_first) ? 1 : -1;

    const int64_t plane = a.out_plane;
    const int64_t ostep = dir > 0 ? plane : -plane;
    auto nat = [&](int p) { return dir > 0 ? p : B - 1 - p; };
    auto add_total = [&](int b, float v) {  // an LDS atomic when the row fits there
        if (in_lds)
            __hip_atomic_fetch_add(&ltot[(lane >> 4) * B + b], v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_fetch_add(&gp[b], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // v summed over the wave (every lane active) into bin b: in LDS, per
    // 16-lane row by DPP, each row's last lane adding into its own copy
    auto wave_sum_into = [&](int b, float v) {
        if (in_lds) {
            v += dpp_shift<0x111, 0xf>(v);  // row_shr:1
            v += dpp_shift<0x112, 0xf>(v);  // row_shr:2
            v += dpp_shift<0x114, 0xf>(v);  // row_shr:4
            v += dpp_shift<0x118, 0xf>(v);  // row_shr:8
            if ((lane & 15) == 15)
                __hip_atomic_fetch_add(&ltot[(lane >> 4) * B + b], v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            const float sum = wave_total(v);
            if (lane == 0)
                __hip_atomic_fetch_add(&gp[b], sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    int nxt = 0;                                        // first bin not stored
    int64_t woff = dir > 0 ? 0 : (int64_t)(B - 1) * plane;  // element offset of bin nxt
    bool open = false;
    float acc = 0.0f, tacc = 0.0f;
    auto close = [&]() {
        if (open) {
            if (act) {
                stream_store(acc, op + woff);
                if (tot) add_total(nat(nxt), tacc);
            }
            woff += ostep;
            ++nxt;
            open = false;
        }
    };
    auto bin = [&](int p, float fr, float dI) {
        if (open && p == nxt) {
            acc = madd(fr, dI, acc);
            tacc = madd(fr, dI, tacc);
        } else if (p > nxt || (p == nxt && !open)) {
            close();
            for (; nxt < p; ++nxt, woff += ostep)
                if (!add_on && act) stream_store(0.0f, op + woff);
            acc = madd(fr, dI, (add_on && act) ? op[woff] : 0.0f);
            tacc = madd(fr, dI, 0.0f);
            open = true;
        } else if (act) {  // stored already: read, add, rewrite
            const int b = nat(p);
            float* o = op + (int64_t)b * plane;
            *o = madd(fr, dI, *o);
            if (tot) add_total(b, fr * dI);
        }
    };

    // Lanes with `on` add v to the total of bin b.  Called with every lane of
    // the wave active: when all those lanes close the same bin (neighbouring
    // pixels of a row usually do), their sum is formed with DPP and added by
    // one lane, instead of one LDS atomic per lane on a single address.
    auto wave_add_total = [&](bool on, int b, float v) {
        const unsigned long long m = __ballot(on);
        if (m == 0) return;
        const int b0 = __builtin_amdgcn_readlane(b, __builtin_ctzll(m));
        if (__ballot(on && b != b0) == 0)
            wave_sum_into(b0, on ? v : 0.0f);
        else if (on)
            add_total(b, v);
    };
    // Lanes with `on` close the open bin nxt and open nxt + 1 (the common
    // step of the walk); the bin closed and the partial total it carries are
    // returned in cb and cv for wave_add_totals.
    auto advance = [&](bool on, int& cb, float& cv) {
        cb = nat(nxt);
        cv = tacc;
        if (on && act) stream_store(acc, op + woff);
        if (on) {
            woff += ostep;
            ++nxt;
            acc = 0.0f;
            tacc = 0.0f;
            if (add_on && act) acc = op[woff];
        }
    };
    // The partial totals of the (at most two) bins each lane closed in one
    // step: one wave sum when every closed bin is the same bin (a lane that
    // closes two bins never is), else one wave_add_total per kind of close.
    auto wave_add_totals = [&](bool ca, int ba, float va, bool cb, int bb, float vb) {
        const unsigned long long m = __ballot(ca || cb);
        if (m == 0) return;
        const int b0 = __builtin_amdgcn_readlane(ca ? ba : bb, __builtin_ctzll(m));
        if (__ballot((ca && ba != b0) || (cb && bb != b0)) == 0) {
            wave_sum_into(b0, (ca ? va : 0.0f) + (cb ? vb : 0.0f));
        } else {
            wave_add_total(ca, ba, va);
            wave_add_total(cb, bb, vb);
        }
    };

    // a floor as an int, clamped to [-2, B + 1] (both ends lie outside the grid)
    auto ifloor = [&](double fl) {
        return (int)__builtin_fmin(__builtin_fmax(fl, -2.0), (double)(B + 1));
    };
    double u_prev = u_first, fl_prev = __builtin_floor(u_first);
    int ifl_prev = ifloor(fl_prev);
    auto step = [&](int kk, int k, int s0, int s1) {
        const double u_next =
            position_at<TILT>(wyz[2 * kk], wyz[2 * kk + 1], py, pz, r, sr, c, e0, invw);
        const double fl_next = __builtin_floor(u_next);
        const int ifl_next = ifloor(fl_next);
        const float dI = sample_diff<float, NORM>(s0, s1, a.wk, k) * scale;
        // Fast form, taken when every lane of the wave qualifies: the interval
        // lies inside the grid, covers one or two bins, and starts in the open
        // bin or the one after it.  Same bins, fractions and order of
        // accumulation as the general form below.
        const double lo = __builtin_fmin(u_prev, u_next), hi = __builtin_fmax(u_prev, u_next);
        const double len = hi - lo;
        const double fh = __builtin_fmax(fl_prev, fl_next);
        const int f = min(ifl_prev, ifl_next);
        // last bin: floor(hi), or the one below when hi is exactly that integer
        const int l = max(ifl_prev, ifl_next) - ((hi == fh && len > 0.0) ? 1 : 0);
        const bool two = l > f;
        const int p1 = dir > 0 ? f : B - 1 - l;  // first bin visited (direction frame)
        const bool fast =
            open && f >= 0 && l <= B - 1 && l <= f + 1 && (unsigned)(p1 - nxt) <= 1u;
        if (__all(fast)) {
            float fr1 = 1.0f, fr2 = 0.0f;
            if (two) {  // bins f and f + 1, split at bd
                const double bd = (double)(f + 1);
                const float rl = __builtin_amdgcn_rcpf((float)len);
                const float lower = (float)(bd - lo) * rl, upper = (float)(hi - bd) * rl;
                fr1 = dir > 0 ? lower : upper;
                fr2 = dir > 0 ? upper : lower;
            }
            const bool one = p1 != nxt;
            int ba, bb;
            float va, vb;
            advance(one, ba, va);
            acc = madd(fr1, dI, acc);
            tacc = madd(fr1, dI, tacc);
            advance(two, bb, vb);
            if (two) {
                acc = madd(fr2, dI, acc);
                tacc = madd(fr2, dI, tacc);
            }
            if (tot) wave_add_totals(one && act, ba, va, two && act, bb, vb);
        } else {
            const PlanF e = plan_f32(u_prev, u_next, fl_prev, fl_next, B);
            if (e.nb > 0) {
                const int bh = e.bl + e.nb - 1;
                const int p0 = dir > 0 ? e.bl : B - 1 - bh;
                bin(p0, dir > 0 ? e.f0 : e.f1, dI);
                if (e.nb > 1) {
                    for (int q = 1; q + 1 < e.nb; ++q) bin(p0 + q, e.fm, dI);
                    bin(p0 + e.nb - 1, dir > 0 ? e.f1 : e.f0, dI);
                }
            }
        }
        u_prev = u_next;
        fl_prev = fl_next;
        ifl_prev = ifl_next;
    };

    // ring of U samples: slot k % U holds step k; wire chunks are whole rings
    constexpr int U = PF + 1;
    constexpr int KCU = (kWireChunk / U) * U;
    unsigned short ring[U];
#pragma unroll
    for (int d = 0; d < U; ++d) ring[d] = stream_load(ip + (int64_t)min(d, N - 1) * a.img_step);
    for (int kc = 0; kc < nint; kc += KCU) {
        const int nk = min(KCU, nint - kc);
        __syncthreads();
        for (int e = tid; e < 2 * nk; e += kPixelTile) wyz[e] = g.wire_yz[2 * (kc + 1) + e];
        __syncthreads();
        int kk = 0;
        for (; kk + U <= nk; kk += U) {
#pragma unroll
            for (int d = 0; d < U; ++d) {
                step(kk + d, kc + kk + d, (int)ring[d], (int)ring[(d + 1) % U]);
                ring[d] = stream_load(ip + (int64_t)min(kc + kk + d + U, N - 1) * a.img_step);
            }
        }
#pragma unroll
        for (int d = 0; d < U; ++d)
            if (kk + d < nk) step(kk + d, kc + kk + d, (int)ring[d], (int)ring[(d + 1) % U]);
    }
    close();
    if (!add_on)
        for (; nxt < B; ++nxt, woff += ostep)
            if (act) stream_store(0.0f, op + woff);
    if (tot && in_lds) {
        __syncthreads();
        for (int b = tid; b < B; b += kPixelTile)
            gp[b] = (ltot[b] + ltot[B + b]) + (ltot[2 * B + b] + ltot[3 * B + b]);
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
    const size_t need = (size_t)a.n_bins * sizeof(Acc) * (sizeof(Acc) == 4 ? kPixelTotalCopies : 1);
    const size_t lds = (a.partials && need <= kPixelLdsBytes) ? need : 0;
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
        hipLaunchKernelGGL((pixels_f32_kernel<8, NORM, TILT, ADD>), grid, block, lds, s, a, g,  \
                           side, sc, la);                                                       \
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
