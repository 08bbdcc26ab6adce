// Shorter FP64 form of an edge position for the per-pixel kernel, shared
// with the geometry check that bounds its distance from the exact form.
#pragma once

#include <hip/hip_runtime.h>

namespace dr {

// The same position in fewer instructions: the square root and the division
// each one Newton step after the hardware reciprocal square root and
// reciprocal (relative errors below 2^-47 instead of correctly rounded), the
// products and sums fused where one operand is a product (sr*L2 as
// sr*q + sr*r^2, so that L2 itself is not formed), and the division by c of a
// tilted axis, the offset and the bin width folded into one fused step.  Every
// rounding stays of the order of the terms it rounds.  dr_geometry_init bounds
// its distance from position_at at every pixel and step (GeomArgs::pos_margin)
// and also evaluates it there, finding its largest actual distance e; the
// kernel takes its floor only where the margin keeps it away from an integer,
// and the geometry takes the fast form only when e is below half the margin,
// so bin indices are those of the exact positions, and when its shortest
// non-zero step is at least 2^28 e, so that fractions move by less than 2^-26.
struct FastPos {
    double py, pz;  // the pixel's projected position
    double sr;      // signed wire radius of the edge
    double mrr;     // -r^2
    double srrr;    // sr * r^2
    double scale;   // sgn / (c * width): bin units, walk direction
    double offs;    // -e0 * sgn / width
};

__device__ __forceinline__ double position_fast(double cy, double cz, const FastPos& P)
{
    const double ay = cy - P.py;
    const double az = cz - P.pz;
    const double q = __builtin_fma(az, az, __builtin_fma(ay, ay, P.mrr));  // L2 - r^2
    const double y = __builtin_amdgcn_rsq(q);
    const double g = q * y, h = y * 0.5;
    const double kk = __builtin_fma(g, __builtin_fma(-h, g, 0.5), g);
    const double tz = __builtin_fma(az, kk, -(ay * P.sr));
    const double ty = __builtin_fma(ay, kk, az * P.sr);
    const double y0 = __builtin_amdgcn_rcp(ty);
    const double y1 = __builtin_fma(y0, __builtin_fma(-ty, y0, 1.0), y0);
    const double num = __builtin_fma(cy, tz, __builtin_fma(P.sr, q, P.srrr));
    const double t = __builtin_fma(-num, y1, cz);
    return __builtin_fma(t, P.scale, P.offs);
}

}  // namespace dr
