// Internal declarations shared by the HIP kernels (dr_kernels.hip) and the
// host runtime (dr_runtime.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dr {

// Row classes of the per-row bin plan: how the leading edge moves over the scan.
// kRowNarrow is or-ed into a monotone class when no interval of the row
// touches more than two bins.
enum RowClass : int8_t { kRowGeneric = 0, kRowIncreasing = 1, kRowDecreasing = 2, kRowNarrow = 8 };

// Plan of the FP64 bin positions of one (row, interval k): the interval
// [u_k, u_{k+1}] touches bins bl .. bl+nb-1 with positive overlap; the first
// bin receives fraction f0, the last f1, the ones between fm (= 1/len).
struct PlanTables {
    int32_t* bl;   // [ny][n_steps-1]
    int32_t* nb;
    float* f0;     // FP32 copies for the FP32 kernel
    float* fm;
    float* f1;
    double* d0;    // FP64 fractions for the FP64 kernel
    double* dm;
    double* d1;
    int8_t* row_class;  // [ny]
    int8_t* row_sign;   // [ny] leading-edge side s_p (+1 / -1)
    int32_t* row_lo;    // [ny] first and last bin the row touches (lo > hi: none)
    int32_t* row_hi;
};

// One scan as seen by the reconstruction kernels.  The image buffer holds
// detector rows [row_base, row_base + rows held) of every step.
struct ScanArgs {
    const uint16_t* img;  // element (step 0, buffer row 0, column 0)
    int64_t img_step;     // elements between consecutive steps
    int64_t img_row;      // elements between consecutive rows
    int32_t row_base;     // detector row stored at buffer row 0
    int32_t nx, ny;
    int32_t row_begin, row_end;  // detector rows to process
    int32_t tiles_per_row;
    int32_t n_steps, n_bins;
    void* out;            // element (bin 0, row 0, column 0); float or double
    int64_t out_plane;    // elements between bins (ny*nx)
    void* partials;       // per-wave partial sums of totals, [slots][n_bins]
    int32_t pass;         // 0: single pass; 1, 2: first and second pass of a two-edge
                          // reconstruction (the second adds onto the first's output)
    const double* wk;     // [n_steps] per-step sample weights, or null
    // plan tables (row mode)
    const int32_t* bl;
    const int32_t* nb;
    const float* f0;
    const float* fm;
    const float* f1;
    const double* d0;
    const double* dm;
    const double* d1;
    const int8_t* row_class;
    const int32_t* row_lo;
    const int32_t* row_hi;
};

// Geometry as seen by the table builder, the per-pixel kernels and the debug
// kernel.  Coordinates are projected onto the plane normal to the wire axis:
// (eta, xi), xi along the projected beam (see axis_frame in dr_kernels.hip).
struct GeomArgs {
    int32_t nx, ny, n_steps, n_bins;
    double radius, first_center, width;
    double axis[3];         // wire axis as given (normalised on the device)
    const double* wire_raw; // [n_steps][3] wire centres as given
    const double* wire_yz;  // [n_steps + 2][2] projected (eta, xi), built on the device;
                            // entries n_steps and n_steps + 1 repeat the last
    const double* pix_xyz;  // [ny][nx][3] explicit pixel centres, or null (affine map)
    double origin[3], u[3], v[3];
    // per-pixel path: bound (bin units) on the difference between the fast
    // and the exact FP64 edge position at any pixel and step; positions of
    // the fast form within it of an integer are recomputed exactly (>= 1:
    // every position exact, as for geometries whose bound is not small or
    // whose shortest step is too short for the fractions to stay exact)
    double pos_margin = 1.0;
};

// A pixel list as seen by the list kernels: entries sorted by pixel index and
// cut into tiles that lie in one detector row: wave tiles of at most 64
// entries for the per-row plan path, 256-entry tiles for the per-pixel path
// (which ignores the row).
struct ListArgs {
    const int64_t* pixels;      // [n] flat pixel indices j*nx + i, increasing
    const int32_t* tile_row;    // [n_tiles]
    const int64_t* tile_start;  // [n_tiles] first entry of the tile
    const int32_t* tile_count;  // [n_tiles] entries in the tile
    int64_t n;
    int64_t tile_first;         // first tile of this launch
    int64_t tile_end;           // one past its last tile
    int32_t compact;            // images are [N][entries] in list order, else full frames
    int64_t entry_base;         // first entry held by a compact image buffer
};

struct BatchArgs {
    const ScanArgs* scans;     // [n_scans] in work order
    const int64_t* tile_start; // [n_scans + 1] prefix sums of tile counts
    int32_t n_scans;
    int64_t total_tiles;
    unsigned long long* counter;  // queue head, reset before each launch
};

struct TileCfg {
    int ppl, waves, prefetch;
};

// Totals of one scan of a batch: partial rows [slots][n_bins] summed into
// totals[n_bins] through the workspace work[kTotalsWorkRows][n_bins].
struct TotalsJob {
    const float* parts;
    int64_t slots;  // partial rows of all passes
    int32_t n_bins;
    int32_t first1; // first block of this job in the stage-1 grid (64 bins per block)
    int32_t first2; // first block of this job in the stage-2 grid (256 bins per block)
    double* work;
    float* totals;
};

// Launch wrappers (dr_kernels.hip).  All return the launch status.
bool tile_supported(const TileCfg& t);
int tile_width(const TileCfg& t);
int num_tile_variants();
TileCfg tile_variant(int i);

// side: 0 = leading edge, 1 = trailing edge; scale multiplies every fraction
// (-1 turns I_k - I_{k+1} into I_{k+1} - I_k; 1/2 averages two edges).
hipError_t launch_build_plans(const GeomArgs& g, const PlanTables& t, int side, double scale,
                              int* d_status, hipStream_t s);
// rows generic in either of two plans become generic in both
hipError_t launch_unify_classes(int8_t* a, int8_t* b, int ny, hipStream_t s);
hipError_t launch_rows_f32(const TileCfg& t, const ScanArgs& a, hipStream_t s);
// FP64 instance: a.pass must not be 2 (each pass of a two-edge reconstruction
// is launched as a pass of its own, the second into a buffer of its own)
hipError_t launch_rows_f64(const ScanArgs& a, hipStream_t s);
// out[i] = out[i] + other[i], i < n (adds the FP64 second pass onto the first)
hipError_t launch_add_f64(double* out, const double* other, int64_t n, hipStream_t s);
// add: every scan of the launch is the second pass of two (pass 2)
hipError_t launch_batch_f32(const TileCfg& t, const BatchArgs& b, bool add, int groups,
                            hipStream_t s);
hipError_t launch_reset_counter(unsigned long long* counter, hipStream_t s);
// the launch-shape dispatch of each template set, one translation unit each
hipError_t launch_rows_f32_single(const TileCfg& t, const ScanArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_rows_f32_add(const TileCfg& t, const ScanArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_batch_f32_single(const TileCfg& t, const BatchArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_batch_f32_add(const TileCfg& t, const BatchArgs& a, dim3 grid, hipStream_t s);
// totals[b] = sum over slots of partials[slot][b] (FP64 sum, stored as T)
hipError_t launch_totals_f32(const float* partials, int64_t slots, int n_bins, double* work,
                             int work_rows, float* totals, hipStream_t s);
hipError_t launch_totals_f64(const double* partials, int64_t slots, int n_bins, double* work,
                             int work_rows, double* totals, hipStream_t s);
// the totals of n jobs of one batch in two launches (the same sums, in the
// same order, as launch_totals_f32 per job); blocks1 / blocks2: the jobs'
// stage-1 / stage-2 block counts summed
hipError_t launch_totals_multi_f32(const TotalsJob* jobs, int n, int blocks1, int blocks2,
                                   hipStream_t s);
// totals[b] = sum over p of out[b][p] (out FP64 [n_bins][P]) in a fixed order;
// work: work_rows * n_bins doubles
hipError_t launch_plane_totals_f64(const double* out, int64_t P, int n_bins, double* work,
                                  int work_rows, double* totals, hipStream_t s);
hipError_t launch_debug_plan(const GeomArgs& g, const int64_t* pixels, int n, int side,
                             int32_t* bins, double* upos, hipStream_t s);
// scans with per-step sample weights: launch shape (1, 4, 16) only
hipError_t launch_rows_norm_f32(const ScanArgs& a, hipStream_t s);
// projected wire table; status bit 4 when the axis is zero or along the beam
hipError_t launch_project_wire(const GeomArgs& g, double* wire_yz, int* d_status, hipStream_t s);
// flags[j] = 1 when every pixel of row j has the row's first (eta, xi) bit for
// bit (flags must be preset to 1)
hipError_t launch_row_uniform(const GeomArgs& g, int* flags, hipStream_t s);
// per-pixel geometry checks (status bits as in build_plans_kernel)
// sides: bit 0 leading edge, bit 1 trailing edge (the sides the passes use)
// bounds[3], bin units as the bits of non-negative doubles, over every pixel
// and step: [0] the largest bound on the fast positions' error (0 before the
// launch), [1] the shortest non-zero step |u_{k+1} - u_k| (at least every
// step before the launch), [2] the largest error found (0 before the launch)
hipError_t launch_validate_pixels(const GeomArgs& g, int sides, int* d_status,
                                  unsigned long long* bounds, hipStream_t s);
// per-pixel path: one lane per pixel, positions and bins computed in FP64 on
// the fly.  side 0/1 = leading/trailing, scale as for the plan tables.
hipError_t launch_pixels_f32(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                             hipStream_t s);
hipError_t launch_pixels_f64(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                             hipStream_t s);
constexpr int kPixelTile = 256;  // pixels per workgroup of the per-pixel path
// partial-total rows per workgroup of the per-pixel FP32 path: one per wave
// (its ring sums, each bin written once) and one for the closes that fall
// outside a ring (device atomics)
constexpr int kPixelPartialRows = kPixelTile / 64 + 1;
// largest partial-total row the FP64 per-pixel instance sums in LDS (larger
// rows are summed with device atomics in the partials buffer itself)
constexpr size_t kPixelLdsBytes = 64 * 1024;

// Top-k selection state, kept on the device between the radix passes:
// after the last pass `prefix` is the k-th largest activity T, `above` the
// number of activities above T and `need` how many equal to T are taken.
struct SelectState {
    uint64_t prefix, mask;
    int64_t need, above;
    unsigned long long bits;  // OR of all keys: digits above its top bit are 0 in every key
    unsigned long long hist[256];
};
constexpr int64_t kSelectBlock = 4096;  // keys per workgroup of the selection scan

// pixel activity sum_k |I_k - I_{k+1}| of a full stack [N][npix]; vec4: 8-byte
// loads of 4 pixels (img 8-byte aligned and npix % 4 == 0)
hipError_t launch_activity(const uint16_t* img, int64_t npix, int n_steps, uint64_t* act,
                           bool vec4, hipStream_t s);
// the k (1 <= k <= npix) largest activities, ties to the lower index, as an
// increasing index list; bsum holds ceil(npix / kSelectBlock) entries
hipError_t launch_select_top(const uint64_t* act, int64_t npix, int64_t k, SelectState* st,
                             uint64_t* bsum, int64_t* list, hipStream_t s);
// status bit 1: an entry outside [0, npix); bit 2: not strictly increasing
hipError_t launch_list_check(const int64_t* list, int64_t n, int64_t npix, int* status,
                             hipStream_t s);
// starts[j] = number of entries below j*nx, j = 0..ny
hipError_t launch_list_rows(const int64_t* list, int64_t n, int nx, int ny, int64_t* starts,
                            hipStream_t s);
// pixel-list reconstruction, one workgroup per list tile (tiles l.tile_first
// .. l.tile_first + n_tiles - 1): per-row plan path and per-pixel path
hipError_t launch_list_f32(const ScanArgs& a, const ListArgs& l, int64_t n_tiles, hipStream_t s);
hipError_t launch_list_f64(const ScanArgs& a, const ListArgs& l, int64_t n_tiles, hipStream_t s);
hipError_t launch_list_pixels_f32(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                                  const ListArgs& l, int64_t n_tiles, hipStream_t s);
hipError_t launch_list_pixels_f64(const ScanArgs& a, const GeomArgs& g, int side, double scale,
                                  const ListArgs& l, int64_t n_tiles, hipStream_t s);
constexpr int kListTile = 256;  // lanes per list tile
// list tiles map lane i to entry (start rounded down to kListAlign) + i; a tile
// spans at most kListTile entries from that base
constexpr int64_t kListAlign = 64;

constexpr int kPlanChunk = 1024;  // intervals staged in LDS at a time
constexpr int kTotalsWorkRows = 64;

}  // namespace dr
