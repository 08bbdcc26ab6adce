/*
 * A plain C11 caller of the reconstruction library: builds a small scan in
 * host memory, reconstructs it through the C ABI (FP32 and the FP64
 * instance), and checks what holds for any input: intensity conservation for
 * pixels whose sweep lies inside the depth grid (the bins of a pixel add up to
 * I_0 - I_{N-1}), the totals, agreement of the two instances, and an argument
 * error reported with a message.  Exit code 0 and "c abi ok" on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "dr.h"

#define CHECK(c)                                                                   \
    do {                                                                           \
        dr_status s_ = (c);                                                        \
        if (s_ != DR_OK) {                                                         \
            fprintf(stderr, "%s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #c, s_,  \
                    dr_last_error());                                              \
            return 1;                                                              \
        }                                                                          \
    } while (0)
#define HIPCHECK(c)                                                                \
    do {                                                                           \
        if ((c) != hipSuccess) {                                                   \
            fprintf(stderr, "%s:%d: %s failed\n", __FILE__, __LINE__, #c);         \
            return 1;                                                              \
        }                                                                          \
    } while (0)

enum { NX = 96, NY = 5, NS = 41, NB = 121 };

int main(void)
{
    /* detector normal to y at 510 mm, 200 um pixels, columns along x, rows along z */
    dr_detector det;
    memset(&det, 0, sizeof det);
    det.nx = NX;
    det.ny = NY;
    det.origin[0] = -(NX - 1) * 100.0;
    det.origin[1] = 510000.0;
    det.origin[2] = -(NY - 1) * 100.0;
    det.u[0] = 200.0;
    det.v[2] = 200.0;
    /* wire of radius 26 um along x, scanned at 45 degrees in 1 um steps */
    static double centers[NS * 3];
    const double h = sqrt(0.5);
    for (int k = 0; k < NS; ++k) {
        const double t = (double)k - (NS - 1) / 2.0;
        centers[3 * k] = 0.0;
        centers[3 * k + 1] = 300.0 + t * h;
        centers[3 * k + 2] = -26.0 + t * h;
    }
    dr_wire wire = {26.0, {1.0, 0.0, 0.0}, NS, centers, DR_EDGE_LEADING};
    dr_depth_grid grid = {NB, -(NB - 1) / 2.0, 1.0};

    static uint16_t img[NS * NY * NX];
    for (int k = 0; k < NS; ++k)
        for (int p = 0; p < NX * NY; ++p)
            img[(size_t)k * NX * NY + p] =
                (uint16_t)(3000 - 40 * k + (p * 37 + k * k * 13) % 97);

    dr_ctx ctx;
    CHECK(dr_ctx_create(0, 0, &ctx));
    dr_geom g;
    dr_wire bad = wire;
    bad.radius = -1.0;
    if (dr_geometry_init(ctx, &det, &bad, &grid, &g) != DR_E_INVAL || !dr_last_error()[0]) {
        fprintf(stderr, "negative radius not rejected\n");
        return 1;
    }
    CHECK(dr_geometry_init(ctx, &det, &wire, &grid, &g));

    void *d_img, *d_out, *d_tot, *d_out64;
    const size_t n_img = sizeof img, n_out = (size_t)NB * NY * NX;
    HIPCHECK(hipMalloc(&d_img, n_img));
    HIPCHECK(hipMalloc(&d_out, n_out * sizeof(float)));
    HIPCHECK(hipMalloc(&d_out64, n_out * sizeof(double)));
    HIPCHECK(hipMalloc(&d_tot, NB * sizeof(float)));
    HIPCHECK(hipMemcpy(d_img, img, n_img, hipMemcpyHostToDevice));
    CHECK(dr_reconstruct(g, (const uint16_t*)d_img, 1, (float*)d_out, (float*)d_tot, NULL));
    CHECK(dr_reconstruct_f64(g, (const uint16_t*)d_img, (double*)d_out64, NULL, NULL));
    HIPCHECK(hipDeviceSynchronize());

    float* out = (float*)malloc(n_out * sizeof(float));
    double* out64 = (double*)malloc(n_out * sizeof(double));
    float tot[NB];
    HIPCHECK(hipMemcpy(out, d_out, n_out * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(out64, d_out64, n_out * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(tot, d_tot, sizeof tot, hipMemcpyDeviceToHost));

    /* bins each pixel's edge visits, to find the sweeps inside the grid */
    static int64_t pix[NX * NY];
    static int32_t bins[NX * NY * NS];
    for (int p = 0; p < NX * NY; ++p) pix[p] = p;
    CHECK(dr_debug_plan(g, pix, NX * NY, DR_EDGE_LEADING, bins, NULL));

    int inside = 0;
    double scale_all = 0.0, sum_all = 0.0;
    for (int p = 0; p < NX * NY; ++p) {
        double scale = 0.0, s32 = 0.0, s64 = 0.0;
        int lo = bins[(size_t)p * NS], hi = lo;
        for (int k = 0; k < NS; ++k) {
            const int b = bins[(size_t)p * NS + k];
            lo = b < lo ? b : lo;
            hi = b > hi ? b : hi;
            if (k + 1 < NS)
                scale += fabs((double)img[(size_t)k * NX * NY + p] -
                              (double)img[(size_t)(k + 1) * NX * NY + p]);
        }
        for (int b = 0; b < NB; ++b) {
            const double v = out[(size_t)b * NX * NY + p], w = out64[(size_t)b * NX * NY + p];
            if (fabs(v - w) > 1e-5 * scale) {
                fprintf(stderr, "pixel %d bin %d: f32 %g vs f64 %g\n", p, b, v, w);
                return 1;
            }
            s32 += v;
            s64 += w;
        }
        scale_all += scale;
        sum_all += s32;
        if (lo >= 0 && hi <= NB - 1) {
            const double want = (double)img[p] - (double)img[(size_t)(NS - 1) * NX * NY + p];
            if (fabs(s64 - want) > 1e-9 * (1.0 + scale) || fabs(s32 - want) > 1e-5 * scale) {
                fprintf(stderr, "pixel %d: sum %g, expected %g\n", p, s64, want);
                return 1;
            }
            ++inside;
        }
    }
    double tsum = 0.0;
    for (int b = 0; b < NB; ++b) tsum += tot[b];
    if (inside < NX * NY / 2 || fabs(tsum - sum_all) > 1e-5 * scale_all) {
        fprintf(stderr, "inside %d, totals %g vs %g\n", inside, tsum, sum_all);
        return 1;
    }
    CHECK(dr_geometry_free(g));
    CHECK(dr_ctx_destroy(ctx));
    HIPCHECK(hipFree(d_img));
    HIPCHECK(hipFree(d_out));
    HIPCHECK(hipFree(d_out64));
    HIPCHECK(hipFree(d_tot));
    free(out);
    free(out64);
    printf("c abi ok: %d of %d pixels conserve intensity, f32 within 1e-5 of f64\n", inside,
           NX * NY);
    return 0;
}
