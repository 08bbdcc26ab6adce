/*
 * ORACLE - test infrastructure only.
 *
 * A plain, slow, FP64 CPU implementation of wire-scan depth reconstruction,
 * used by the tests, the smoke check and the benchmark's CPU baseline to
 * check the GPU library.  It shares no code, header, table or helper with the
 * GPU path, and the product never calls it.
 *
 * What it computes (paper Sec. I and Sec. III-C: the per-pixel reconstruction
 * takes the intensity difference at each pixel between consecutive wire
 * positions and adds the differences into depth arrays; the paper defers the
 * geometry to the differential-aperture method it cites, so the geometry below
 * is the reading written down with the tests):
 *
 *   frame      um, beam along +z through x = y = 0, depth = z.  The wire is a
 *              cylinder of radius r around an axis of unit direction a (the
 *              lab x axis in the standard set-up).  Everything is projected
 *              onto the plane normal to a, with coordinates
 *                xi  = X . e1,  e1 = (z - (z.a) a) / |z - (z.a) a|
 *                eta = X . e2,  e2 = e1 x a
 *              in which the beam is the xi axis (beam point d -> xi = c d,
 *              c = e1.z) and the wire is a disc; for a = x this is
 *              (xi, eta) = (z, y) exactly.
 *   pixel      P = (origin + i*u) + j*v for column i and row j, or an explicit
 *              per-pixel table, then projected.
 *   depth      for projected pixel P, wire centre C_k and radius r, the ray
 *              from P tangent to the disc on side s (+1: the +xi side) meets
 *              the xi axis at
 *                xi* = C_xi - (C_eta*t_xi + s*r*L2) / t_eta
 *              with a = C - P, L2 = |a|^2, kk = sqrt(L2 - r^2),
 *              t_xi = a_xi*kk - a_eta*s*r, t_eta = a_eta*kk + a_xi*s*r,
 *              and depth d = xi* / c.
 *   edge       s_p = +1 when that +z-side depth moves toward +z over the scan
 *              (last step vs first step), else -1.  The leading edge uses
 *              side s_p and dI_k = I_k - I_{k+1} (intensity lost as the edge
 *              covers the slice); the trailing edge uses side -s_p and
 *              dI_k = I_{k+1} - I_k (intensity regained as it uncovers it);
 *              "both" is the average 0.5 * (L + T) of the leading (L) and
 *              trailing (T) reconstructions, each built on its own.
 *   binning    u_k = (d_k - e0) * (1/width), e0 = first_center - width/2.
 *              For k = 0..N-2 the difference dI_k is spread over
 *              [lo, hi] = [min, max](u_k, u_{k+1}): bin b gets
 *              dI_k * (ov/len) with ov = min(hi, b+1) - max(lo, b) > 0 and
 *              len = hi - lo; parts outside [0, n_bins) are dropped; a
 *              zero-length interval puts dI_k into bin floor(lo).
 *   weights    optional per-step weights w_k (beam-monitor normalisation, a
 *              reading: the paper has none): every sample becomes I_k * w_k
 *              (one FP64 rounding) before the differences are taken.
 *   totals     tot[b] = sum over pixels of out[b][p].
 *   selection  (the paper's second experiment processes a percentage of the
 *              pixels, Sec. IV, without stating which; the reading used
 *              here): the activity of pixel p is A_p = sum_k |I_k - I_{k+1}|
 *              over its N samples, and the top-k selection keeps the k
 *              pixels of largest A_p, ties going to the lower pixel index,
 *              listed in increasing pixel index.
 *
 * Every operation is one IEEE binary64 operation in the order written; build
 * with -ffp-contract=off.  Pins (tests/test_oracle_*.py): the tangent depth
 * against a similar-triangles closed form, the zero-radius line intersection,
 * bisection on an independent occlusion predicate and mirror symmetry; the
 * binning against hand-computed profiles and intensity conservation; the
 * whole chain against brute-force sub-sampled ray integration and against
 * depths planted by the forward model.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)

#define EDGE_LEADING 0
#define EDGE_TRAILING 1
#define EDGE_BOTH 2

/* In the plane normal to the wire axis: the xi coordinate at which the ray
 * from (py, pz) = (eta, xi) of the pixel, tangent to the wire disc centred at
 * (cy, cz) on side s, meets the xi axis.  Returns NAN when the pixel is inside
 * the disc. */
double oracle_tangent_depth(double py, double pz, double cy, double cz, double r, int s)
{
    double sr = (double)s * r;
    double ay = cy - py;
    double az = cz - pz;
    double L2 = az * az + ay * ay;
    double q = L2 - r * r;
    if (!(q > 0.0)) return NAN;
    double kk = sqrt(q);
    double tz = az * kk - ay * sr;
    double ty = ay * kk + az * sr;
    return cz - (cy * tz + sr * L2) / ty;
}

/* Projection frame of the plane normal to the wire axis: e1 (projected beam
 * direction), e2 = e1 x a, and c = e1.z.  Returns ORACLE_EINVAL for a zero
 * axis or an axis parallel to the beam. */
typedef struct {
    double e1[3], e2[3], c;
} frame_t;

static int axis_frame(const double* axis, frame_t* f)
{
    double n = sqrt((axis[0] * axis[0] + axis[1] * axis[1]) + axis[2] * axis[2]);
    if (!(n > 0.0)) return ORACLE_EINVAL;
    double a[3] = {axis[0] / n, axis[1] / n, axis[2] / n};
    double zp[3] = {0.0 - a[2] * a[0], 0.0 - a[2] * a[1], 1.0 - a[2] * a[2]};
    double m = sqrt((zp[0] * zp[0] + zp[1] * zp[1]) + zp[2] * zp[2]);
    if (!(m > 1e-6)) return ORACLE_EINVAL;
    for (int q = 0; q < 3; ++q) f->e1[q] = zp[q] / m;
    f->e2[0] = f->e1[1] * a[2] - f->e1[2] * a[1];
    f->e2[1] = f->e1[2] * a[0] - f->e1[0] * a[2];
    f->e2[2] = f->e1[0] * a[1] - f->e1[1] * a[0];
    f->c = f->e1[2];
    return ORACLE_OK;
}

/* (eta, xi) of a lab point */
static void project(const frame_t* f, const double* X, double* eta, double* xi)
{
    *xi = (X[0] * f->e1[0] + X[1] * f->e1[1]) + X[2] * f->e1[2];
    *eta = (X[0] * f->e2[0] + X[1] * f->e2[1]) + X[2] * f->e2[2];
}

/* Leading-edge side for one pixel: +1 when the +xi (downstream) tangent
 * point of the last wire position lies beyond that of the first, else -1.
 * wyz: projected wire centres [n_steps][2] as (eta, xi). */
int oracle_edge_sign(double py, double pz, int n_steps, const double* wyz, double r)
{
    double d0 = oracle_tangent_depth(py, pz, wyz[0], wyz[1], r, +1);
    double d1 = oracle_tangent_depth(py, pz, wyz[2 * (n_steps - 1)],
                                     wyz[2 * (n_steps - 1) + 1], r, +1);
    return (d1 > d0) ? +1 : -1;
}

/* Projected (eta, xi) of pixel p. */
static void pixel_center(const frame_t* f, int nx, const double* origin, const double* u,
                         const double* v, const double* pixel_xyz, int64_t p, double* py,
                         double* pz)
{
    double X[3];
    if (pixel_xyz) {
        X[0] = pixel_xyz[3 * p];
        X[1] = pixel_xyz[3 * p + 1];
        X[2] = pixel_xyz[3 * p + 2];
    } else {
        double i = (double)(p % nx);
        double j = (double)(p / nx);
        for (int q = 0; q < 3; ++q) X[q] = (origin[q] + i * u[q]) + j * v[q];
    }
    project(f, X, py, pz);
}

/* Projected wire centres [n_steps][2] (eta, xi); caller frees. */
static double* project_wire(const frame_t* f, int n_steps, const double* centers)
{
    double* w = (double*)malloc(sizeof(double) * 2 * (size_t)n_steps);
    for (int k = 0; k < n_steps; ++k) project(f, centers + 3 * k, &w[2 * k], &w[2 * k + 1]);
    return w;
}

static int32_t floor_to_i32(double x)
{
    double f = floor(x);
    if (f < -2147483648.0) return INT32_MIN;
    if (f > 2147483647.0) return INT32_MAX;
    return (int32_t)f;
}

/* Positions u_k of one edge (leading, or trailing when `trailing` is set) in
 * bin units for one pixel.  Returns ORACLE_EINVAL if the pixel is inside the
 * wire or a value is not finite. */
static int pixel_positions(double py, double pz, int n_steps, const double* wyz, double r,
                           double c, double e0, double invw, int trailing, double* u)
{
    int s = oracle_edge_sign(py, pz, n_steps, wyz, r);
    if (trailing) s = -s;
    for (int k = 0; k < n_steps; ++k) {
        double d = oracle_tangent_depth(py, pz, wyz[2 * k], wyz[2 * k + 1], r, s) / c;
        u[k] = (d - e0) * invw;
        if (!isfinite(u[k])) return ORACLE_EINVAL;
    }
    return ORACLE_OK;
}

/* Spread the intensity differences of one pixel over the depth bins.
 *   u        [n_steps] edge positions in bin units
 *   I        [n_steps] intensities (counts), read as doubles
 *   trailing 0: dI_k = I_k - I_{k+1}; 1: dI_k = I_{k+1} - I_k
 *   out      [n_bins] accumulated in place (caller zeroes it)
 *   stride   distance between consecutive bins of out */
void oracle_bin_profile(const double* u, const double* I, int n_steps, int n_bins, int trailing,
                        double* out, int64_t stride)
{
    for (int k = 0; k + 1 < n_steps; ++k) {
        double dI = trailing ? I[k + 1] - I[k] : I[k] - I[k + 1];
        double lo = u[k] < u[k + 1] ? u[k] : u[k + 1];
        double hi = u[k] < u[k + 1] ? u[k + 1] : u[k];
        double len = hi - lo;
        if (len > 0.0) {
            double first = floor(lo), last = floor(hi);
            if (first < 0.0) first = 0.0;
            if (last > (double)(n_bins - 1)) last = (double)(n_bins - 1);
            for (double bd = first; bd <= last; bd += 1.0) {
                double top = hi < bd + 1.0 ? hi : bd + 1.0;
                double bot = lo > bd ? lo : bd;
                double ov = top - bot;
                if (ov > 0.0) out[(int64_t)bd * stride] += dI * (ov / len);
            }
        } else {
            double bd = floor(lo);
            if (bd >= 0.0 && bd < (double)n_bins) out[(int64_t)bd * stride] += dI;
        }
    }
}

/* Profile of one pixel for edge LEADING, TRAILING or BOTH into o (stride
 * between bins; the caller zeroes it).  uk [n_steps] is scratch; the
 * positions of the reported edge (trailing for TRAILING, else leading) are
 * left in uk.  lt [2 * n_bins] is scratch for BOTH: the leading profile L and
 * the trailing profile T, each accumulated on its own from zero, then
 * o = 0.5 * (L + T) bin by bin. */
static int pixel_profile(double py, double pz, const double* Ik, int n_steps,
                         const double* wyz, double r, double c, double e0, double invw,
                         int n_bins, int edge, double* o, int64_t stride, double* uk, double* lt)
{
    if (edge == EDGE_BOTH) {
        double* L = lt;
        double* T = lt + n_bins;
        for (int b = 0; b < n_bins; ++b) L[b] = T[b] = 0.0;
        if (pixel_positions(py, pz, n_steps, wyz, r, c, e0, invw, 1, uk) != ORACLE_OK)
            return ORACLE_EINVAL;
        oracle_bin_profile(uk, Ik, n_steps, n_bins, 1, T, 1);
        if (pixel_positions(py, pz, n_steps, wyz, r, c, e0, invw, 0, uk) != ORACLE_OK)
            return ORACLE_EINVAL;
        oracle_bin_profile(uk, Ik, n_steps, n_bins, 0, L, 1);
        for (int b = 0; b < n_bins; ++b) o[(int64_t)b * stride] = 0.5 * (L[b] + T[b]);
        return ORACLE_OK;
    }
    const int trailing = edge == EDGE_TRAILING;
    if (pixel_positions(py, pz, n_steps, wyz, r, c, e0, invw, trailing, uk) != ORACLE_OK)
        return ORACLE_EINVAL;
    oracle_bin_profile(uk, Ik, n_steps, n_bins, trailing, o, stride);
    return ORACLE_OK;
}

/*
 * Full reconstruction of detector rows [row0, row0 + nrows).
 *   edge    EDGE_LEADING, EDGE_TRAILING or EDGE_BOTH
 *   step_weight  [n_steps] per-step sample weights, or NULL (all 1)
 *   images  [n_steps][ny][nx] uint16, step slowest
 *   out     [n_bins][nrows][nx] FP64, overwritten
 *   totals  [n_bins] FP64 sums over the processed pixels, or NULL
 *   bins    [nrows*nx][n_steps] int32 floor(u_k) of the reported edge, or NULL
 * Returns ORACLE_OK or ORACLE_EINVAL.
 */
int oracle_reconstruct(int nx, int ny, const double* origin, const double* u, const double* v,
                       const double* pixel_xyz, double radius, const double* axis, int n_steps,
                       const double* centers, int n_bins, double first_center, double width,
                       int edge, const double* step_weight,
                       const uint16_t* images, int row0, int nrows, double* out, double* totals,
                       int32_t* bins, int nthreads)
{
    if (nx <= 0 || ny <= 0 || n_steps < 2 || n_bins <= 0 || !(width > 0.0) || !(radius > 0.0))
        return ORACLE_EINVAL;
    if (edge < EDGE_LEADING || edge > EDGE_BOTH) return ORACLE_EINVAL;
    if (row0 < 0 || nrows < 0 || row0 + nrows > ny) return ORACLE_EINVAL;
    frame_t fr;
    if (axis_frame(axis, &fr) != ORACLE_OK) return ORACLE_EINVAL;
    const double e0 = first_center - width / 2.0;
    const double invw = 1.0 / width;
    const int64_t plane_in = (int64_t)nx * ny;
    const int64_t plane_out = (int64_t)nx * nrows;
    memset(out, 0, sizeof(double) * (size_t)plane_out * (size_t)n_bins);
    double* wyz = project_wire(&fr, n_steps, centers);
    int status = ORACLE_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel
    {
        double* uk = (double*)malloc(sizeof(double) * (size_t)n_steps);
        double* Ik = (double*)malloc(sizeof(double) * (size_t)n_steps);
        double* lt = (double*)malloc(sizeof(double) * 2 * (size_t)n_bins);
#pragma omp for schedule(dynamic, 1)
        for (int jr = 0; jr < nrows; ++jr) {
            for (int i = 0; i < nx; ++i) {
                int64_t p = (int64_t)(row0 + jr) * nx + i;
                int64_t q = (int64_t)jr * nx + i;
                double py, pz;
                pixel_center(&fr, nx, origin, u, v, pixel_xyz, p, &py, &pz);
                for (int k = 0; k < n_steps; ++k) {
                    Ik[k] = (double)images[(int64_t)k * plane_in + p];
                    if (step_weight) Ik[k] = Ik[k] * step_weight[k];
                }
                if (pixel_profile(py, pz, Ik, n_steps, wyz, radius, fr.c, e0, invw, n_bins, edge,
                                  out + q, plane_out, uk, lt) != ORACLE_OK) {
#pragma omp atomic write
                    status = ORACLE_EINVAL;
                    continue;
                }
                if (bins)
                    for (int k = 0; k < n_steps; ++k) bins[q * n_steps + k] = floor_to_i32(uk[k]);
            }
        }
        free(uk);
        free(Ik);
        free(lt);
    }
    free(wyz);
    if (status != ORACLE_OK) return status;
    if (totals) {
        for (int b = 0; b < n_bins; ++b) {
            double t = 0.0;
            for (int64_t q = 0; q < plane_out; ++q) t += out[(int64_t)b * plane_out + q];
            totals[b] = t;
        }
    }
    return ORACLE_OK;
}

/*
 * Reconstruction of an explicit list of pixels (flat indices j*nx + i), for
 * sampled checks of large scans.  Intensities come from `images`
 * ([n_steps][ny][nx]); with NULL images only the positions are computed.
 *   out   [npix][n_bins] FP64 profile of each listed pixel
 *   bins  [npix][n_steps] int32 floor(u_k) of the reported edge, or NULL
 *   upos  [npix][n_steps] FP64 u_k of the reported edge, or NULL
 */
int oracle_reconstruct_pixels(int nx, int ny, const double* origin, const double* u,
                              const double* v, const double* pixel_xyz, double radius,
                              const double* axis, int n_steps, const double* centers, int n_bins,
                              double first_center, double width, int edge,
                              const double* step_weight,
                              const uint16_t* images, const int64_t* pixels, int64_t npix, double* out, int32_t* bins,
                              double* upos, int nthreads)
{
    if (nx <= 0 || ny <= 0 || n_steps < 2 || n_bins <= 0 || !(width > 0.0) || !(radius > 0.0))
        return ORACLE_EINVAL;
    if (edge < EDGE_LEADING || edge > EDGE_BOTH) return ORACLE_EINVAL;
    frame_t fr;
    if (axis_frame(axis, &fr) != ORACLE_OK) return ORACLE_EINVAL;
    const double e0 = first_center - width / 2.0;
    const double invw = 1.0 / width;
    const int64_t plane_in = (int64_t)nx * ny;
    double* wyz = project_wire(&fr, n_steps, centers);
    int status = ORACLE_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double* uk = (double*)malloc(sizeof(double) * (size_t)n_steps);
        double* Ik = (double*)malloc(sizeof(double) * (size_t)n_steps);
        double* lt = (double*)malloc(sizeof(double) * 2 * (size_t)n_bins);
#pragma omp for schedule(dynamic, 16)
        for (int64_t n = 0; n < npix; ++n) {
            int64_t p = pixels[n];
            double* o = out + n * n_bins;
            for (int b = 0; b < n_bins; ++b) o[b] = 0.0;
            if (p < 0 || p >= plane_in) {
#pragma omp atomic write
                status = ORACLE_EINVAL;
                continue;
            }
            double py, pz;
            pixel_center(&fr, nx, origin, u, v, pixel_xyz, p, &py, &pz);
            for (int k = 0; k < n_steps; ++k) {
                Ik[k] = images ? (double)images[(int64_t)k * plane_in + p] : 0.0;
                if (step_weight) Ik[k] = Ik[k] * step_weight[k];
            }
            if (pixel_profile(py, pz, Ik, n_steps, wyz, radius, fr.c, e0, invw, n_bins, edge, o,
                              1, uk, lt) != ORACLE_OK) {
#pragma omp atomic write
                status = ORACLE_EINVAL;
                continue;
            }
            if (!images)
                for (int b = 0; b < n_bins; ++b) o[b] = 0.0;
            if (bins)
                for (int k = 0; k < n_steps; ++k) bins[n * n_steps + k] = floor_to_i32(uk[k]);
            if (upos)
                for (int k = 0; k < n_steps; ++k) upos[n * n_steps + k] = uk[k];
        }
        free(uk);
        free(Ik);
        free(lt);
    }
    free(wyz);
    return status;
}

/* Activity of every pixel of a full stack images[N][npix]:
 * act[p] = sum_k |I_k - I_{k+1}| (exact in 64-bit integers). */
void oracle_activity(const uint16_t* images, int n_steps, int64_t npix, uint64_t* act)
{
    for (int64_t p = 0; p < npix; ++p) {
        uint64_t a = 0;
        for (int k = 0; k + 1 < n_steps; ++k) {
            int64_t d = (int64_t)images[(int64_t)k * npix + p] -
                        (int64_t)images[(int64_t)(k + 1) * npix + p];
            a += (uint64_t)(d < 0 ? -d : d);
        }
        act[p] = a;
    }
}

/* Order of the selection rule: larger activity first, then lower index. */
static const uint64_t* g_sel_act;
static int sel_cmp(const void* x, const void* y)
{
    int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
    if (g_sel_act[a] != g_sel_act[b]) return g_sel_act[a] > g_sel_act[b] ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}
static int idx_cmp(const void* x, const void* y)
{
    int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* The k pixels of largest activity (ties: lower index), written to list[k]
 * in increasing pixel index.  Not thread-safe (qsort comparator state). */
int oracle_select_top(const uint64_t* act, int64_t npix, int64_t k, int64_t* list)
{
    if (npix < 0 || k < 0 || k > npix) return ORACLE_EINVAL;
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(npix > 0 ? npix : 1));
    for (int64_t p = 0; p < npix; ++p) order[p] = p;
    g_sel_act = act;
    qsort(order, (size_t)npix, sizeof(int64_t), sel_cmp);
    for (int64_t i = 0; i < k; ++i) list[i] = order[i];
    qsort(list, (size_t)k, sizeof(int64_t), idx_cmp);
    free(order);
    return ORACLE_OK;
}
