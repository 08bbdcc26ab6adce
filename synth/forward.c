/*
 * Seeded forward model for wire-scan image stacks (input generator).
 *
 * This file builds SYNTHETIC INPUTS ONLY.  It is shared by the tests, the
 * benchmark and the smoke check, and holds none of the reconstruction
 * arithmetic: it never computes a tangent depth, a bin index or an overlap
 * fraction.  What it models is the physics the reconstruction inverts
 * (wire-scan depth resolution, Sec. I): point sources on the incident beam
 * send rays to detector pixels; a ray is blocked at wire step k when the wire
 * (a cylinder of radius r around an axis line) comes closer than r to it;
 * every pixel records Poisson counts.
 *
 * Frame: micrometres, beam along +z through x = y = 0, depth = z.  For a wire
 * along the lab x axis only the (y, z) projection matters; other axes use the
 * 3D distance between the axis line and the ray segment.
 *
 * Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011), used as a pure
 * function of (key, counter), so the output does not depend on the number of
 * threads.  Poisson variates use inversion of a tabulated CDF when the rate
 * equals the dark level, Knuth's multiplication method below rate 10, and
 * Hoermann's transformed rejection with squeeze ("PTRS", Insurance:
 * Mathematics and Economics 12, 1993) otherwise.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox */

typedef struct { uint32_t v[4]; } ctr4;

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static ctr4 philox4x32_10(ctr4 c, uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(M0, c.v[0], &hi0, &lo0);
        mulhilo32(M1, c.v[2], &hi1, &lo1);
        ctr4 n;
        n.v[0] = hi1 ^ c.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ c.v[3] ^ k1;
        n.v[3] = lo0;
        c = n;
        k0 += W0;
        k1 += W1;
    }
    return c;
}

/* uniform in (0, 1) from two 32-bit words: 53 random bits, offset by half an ulp */
static inline double u01(uint32_t a, uint32_t b)
{
    uint64_t m = (((uint64_t)a << 32) | (uint64_t)b) >> 11;
    return ((double)m + 0.5) * 0x1.0p-53;
}

/* A small stream of uniforms drawn from consecutive Philox blocks. */
typedef struct {
    uint32_t k0, k1;
    ctr4 ctr;
    ctr4 out;
    int used; /* number of doubles consumed from out (0, 1 or 2) */
} ustream;

static void us_init(ustream* s, uint64_t seed, uint64_t a, uint64_t b)
{
    s->k0 = (uint32_t)seed;
    s->k1 = (uint32_t)(seed >> 32);
    s->ctr.v[0] = (uint32_t)a;
    s->ctr.v[1] = (uint32_t)(a >> 32);
    s->ctr.v[2] = (uint32_t)b;
    s->ctr.v[3] = 0; /* block counter inside this stream */
    s->used = 2;
}

static inline double us_next(ustream* s)
{
    if (s->used == 2) {
        s->out = philox4x32_10(s->ctr, s->k0, s->k1);
        s->ctr.v[3] += 1u;
        s->used = 0;
    }
    double r = u01(s->out.v[2 * s->used], s->out.v[2 * s->used + 1]);
    s->used += 1;
    return r;
}

/* Fill n uniforms in (0,1) for stream (seed, a, b): used by the Python side to
 * draw source parameters with the same generator. */
void synth_uniforms(uint64_t seed, uint64_t a, uint64_t b, int64_t n, double* out)
{
    ustream s;
    us_init(&s, seed, a, b);
    for (int64_t i = 0; i < n; ++i) out[i] = us_next(&s);
}

/* --------------------------------------------------------------- Poisson */

static int64_t poisson_knuth(double lam, ustream* s)
{
    double lim = exp(-lam), p = 1.0;
    int64_t k = 0;
    for (;;) {
        p *= us_next(s);
        if (p <= lim) return k;
        ++k;
    }
}

static int64_t poisson_ptrs(double lam, ustream* s)
{
    const double slam = sqrt(lam), loglam = log(lam);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    const double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (;;) {
        double U = us_next(s) - 0.5;
        double V = us_next(s);
        double us = 0.5 - fabs(U);
        double kd = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return (int64_t)kd;
        if (kd < 0.0 || (us < 0.013 && V > us)) continue;
        int sg;
        double lg = lgamma_r(kd + 1.0, &sg);
        if (log(V) + log(invalpha) - log(a / (us * us) + b) <= -lam + kd * loglam - lg)
            return (int64_t)kd;
    }
}

/* CDF table of Poisson(lam) for inversion; returns length, 0 if not usable. */
static int build_cdf(double lam, double** out)
{
    *out = NULL;
    if (!(lam > 0.0) || lam > 600.0) return 0;
    int n = (int)(lam + 40.0 * sqrt(lam) + 64.0);
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    double p = exp(-lam), acc = 0.0;
    for (int m = 0; m < n; ++m) {
        if (m > 0) p = p * lam / (double)m;
        acc += p;
        c[m] = acc;
    }
    *out = c;
    return n;
}

static int64_t poisson_table(const double* cdf, int n, ustream* s)
{
    double u = us_next(s);
    int lo = 0, hi = n - 1;
    if (u >= cdf[hi]) return hi;
    while (lo < hi) { /* smallest m with cdf[m] > u */
        int mid = (lo + hi) >> 1;
        if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* ------------------------------------------------------------- occlusion */

/* True when the wire disc (centre (cy, cz), radius r) overlaps the ray segment
 * from the source (y = 0, z = zs) to the pixel (py, pz): the distance from the
 * disc centre to the segment is strictly below r. */
static inline int occluded(double zs, double py, double pz, double cy, double cz, double rr)
{
    double dy = py, dz = pz - zs;       /* segment direction */
    double wy = cy, wz = cz - zs;       /* disc centre relative to the source */
    double dd = dy * dy + dz * dz;
    double t = (wy * dy + wz * dz) / dd;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double qy = wy - t * dy, qz = wz - t * dz;
    return qy * qy + qz * qz < rr;
}

int synth_occluded(double zs, double py, double pz, double cy, double cz, double r)
{
    return occluded(zs, py, pz, cy, cz, r * r);
}

/* General wire axis: true when the 3D distance between the axis line
 * C + t*a (a unit) and the segment from the source (0, 0, zs) to the pixel P
 * is strictly below r (closest points of the two lines, segment parameter
 * clamped to [0, 1]). */
static inline int occluded3(double zs, const double* P, const double* C, const double* a,
                            double rr)
{
    const double d[3] = {P[0], P[1], P[2] - zs};
    const double w[3] = {-C[0], -C[1], zs - C[2]};
    const double B = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
    const double Cq = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double D = a[0] * w[0] + a[1] * w[1] + a[2] * w[2];
    const double E = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
    const double den = Cq - B * B;
    double s = den > 0.0 ? (B * D - E) / den : 0.0;
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    double q[3], t = 0.0;
    for (int i = 0; i < 3; ++i) q[i] = (i == 2 ? zs : 0.0) + s * d[i];
    for (int i = 0; i < 3; ++i) t += (q[i] - C[i]) * a[i];
    double dist2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double e = C[i] + t * a[i] - q[i];
        dist2 += e * e;
    }
    return dist2 < rr;
}

/* -------------------------------------------------------------- renderer */

/*
 * Render images[k][j][i] (uint16, step slowest) for an ny x nx detector.
 *   px, py, pz    [ny*nx] pixel-centre x, y and z in um
 *   cx, cy, cz    [n_steps] wire-centre x, y and z in um; radius r
 *   axis          unit wire axis; (1,0,0) uses the (y, z) projection
 *   cptr          [ny*nx + 1] CSR offsets into the contribution arrays
 *   cgain, czs    per contribution: expected counts when the ray is clear,
 *                 and the depth of the source it comes from
 *   dark          dark level added to every pixel
 *   noise         0: write round(rate) (noise free); 1: Poisson(rate)
 *   seed          Philox key for the noise
 * Counts are clipped to [0, 65535].  Returns 0.
 */
int synth_render(int32_t nx, int32_t ny, const double* px, const double* py, const double* pz,
                 int32_t n_steps, const double* cx, const double* cy, const double* cz,
                 const double* axis, double r, const int64_t* cptr, const double* cgain,
                 const double* czs, double dark, int32_t noise, uint64_t seed, uint16_t* images,
                 int32_t nthreads)
{
    const double rr = r * r;
    const int xaxis = axis[0] == 1.0 && axis[1] == 0.0 && axis[2] == 0.0;
    const int64_t plane = (int64_t)nx * (int64_t)ny;
    double* cdf = NULL;
    int ncdf = noise ? build_cdf(dark, &cdf) : 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < ny; ++j) {
        for (int32_t k = 0; k < n_steps; ++k) {
            uint16_t* row = images + (int64_t)k * plane + (int64_t)j * nx;
            for (int32_t i = 0; i < nx; ++i) {
                const int64_t p = (int64_t)j * nx + i;
                double lam = dark;
                for (int64_t c = cptr[p]; c < cptr[p + 1]; ++c) {
                    int occ;
                    if (xaxis) {
                        occ = occluded(czs[c], py[p], pz[p], cy[k], cz[k], rr);
                    } else {
                        const double P[3] = {px[p], py[p], pz[p]};
                        const double C[3] = {cx[k], cy[k], cz[k]};
                        occ = occluded3(czs[c], P, C, axis, rr);
                    }
                    if (!occ) lam += cgain[c];
                }
                int64_t n;
                if (!noise) {
                    n = (int64_t)floor(lam + 0.5);
                } else if (lam <= 0.0) {
                    n = 0;
                } else {
                    ustream s;
                    us_init(&s, seed, (uint64_t)p, (uint64_t)k);
                    if (ncdf > 0 && lam == dark) n = poisson_table(cdf, ncdf, &s);
                    else if (lam < 10.0) n = poisson_knuth(lam, &s);
                    else n = poisson_ptrs(lam, &s);
                }
                if (n < 0) n = 0;
                if (n > 65535) n = 65535;
                row[i] = (uint16_t)n;
            }
        }
    }
    free(cdf);
    return 0;
}
