/*
 * dr.h - C ABI of the MI355X (gfx950) wire-scan depth-reconstruction library.
 *
 * The library reconstructs depth-resolved intensity from a stack of detector
 * images taken at successive wire positions: p images of m rows x n columns
 * (paper Sec. III-B), each pixel's intensity differences between consecutive
 * images being added into depth arrays (paper Sec. III-C).  For every pixel
 * and wire step it computes, in FP64, the depth at which the ray from the
 * pixel that grazes the wire's leading edge meets the incident beam, and it
 * spreads I_k - I_{k+1} over the depth interval [d_k, d_{k+1}] into fixed
 * bins in proportion to the overlap.  Geometry conventions:
 *
 *   - lengths in micrometres; the beam is the line x = y = 0 travelling +z;
 *     depth is the z coordinate of a point on the beam;
 *   - the wire is a cylinder of radius `radius` around an axis line of any
 *     direction not along the beam; positions are projected onto the plane
 *     normal to the axis, with coordinates (eta, xi): xi along the beam's
 *     projection, eta = xi x axis (for the lab x axis, (eta, xi) = (y, z)),
 *     and the tangent construction runs in that plane; the depth is the
 *     projected beam coordinate divided by the cosine between beam and plane;
 *   - pixel (row j, column i) has centre (origin + i*u) + j*v unless an
 *     explicit per-pixel table is given;
 *   - bin b of the depth grid is centred at first_center + b*width and covers
 *     [first_center + (b - 1/2) width, first_center + (b + 1/2) width);
 *   - the leading edge is the wire side whose shadow on the beam advances with
 *     the scan: the +z side when the +z tangent depth of the last step exceeds
 *     that of the first, otherwise the -z side; the intensity difference
 *     I_k - I_{k+1} is spread over [u_k, u_{k+1}] (bin units), parts outside
 *     the grid are dropped, and a zero-length interval adds into floor(u_k).
 *
 * Data layout (all row-major, flat one-dimensional buffers as in the paper's
 * Sec. III-B choice of a 1D array over a pointer-based 3D array):
 *   images  uint16 [n_steps][ny][nx]   (step slowest)
 *   out     float  [n_bins][ny][nx]    (depth slowest; every element written)
 *   totals  float  [n_bins]            (sum of out over all pixels)
 *
 * Precision: tangent depths, bin positions and overlap fractions in FP64;
 * intensity differences and bin accumulation in FP32 (dr_reconstruct) or
 * FP64 (dr_reconstruct_f64).  Bin indices floor(u_k) are exact FP64 results
 * (IEEE operations in a fixed order, no contraction).
 *
 * Errors: every entry point returns a dr_status; negative values are errors
 * and dr_last_error() returns a message for the calling thread.  Nothing is
 * thrown across the ABI.  Arguments are checked before any device work.
 *
 * Threads: a dr_ctx may be used from several host threads; calls that enqueue
 * work on one dr_geom must not overlap in time on different streams, because
 * each geometry owns one scratch area (per-wave partial sums of the totals);
 * the same holds for calls on one pixel list.
 */
#ifndef DR_H
#define DR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dr_status;
#define DR_OK 0
#define DR_PENDING 1
#define DR_E_INVAL (-1)
#define DR_E_NOMEM (-2)
#define DR_E_UNSUPPORTED (-3)
#define DR_E_DEVICE (-4)
#define DR_E_BUSY (-5)
#define DR_E_NOTFOUND (-6)

/* Wire edges (dr_wire.edge).  Leading: the side whose shadow advances with
 * the scan, I_k - I_{k+1} spread over its interval (intensity lost as the edge
 * covers a depth slice).  Trailing: the opposite side, I_{k+1} - I_k
 * (intensity regained as it uncovers the slice).  Both: the average
 * (L + T)/2 of the two reconstructions, each formed on its own (a true source
 * keeps its amplitude, the mirrored negative ghosts of the two edges are
 * halved).  The FP32 path stores L/2 in a first pass and adds T/2, summed
 * from zero, in a second; the FP64 instance forms T/2 in a buffer of its own
 * and adds the two buffers. */
#define DR_EDGE_LEADING 0
#define DR_EDGE_TRAILING 1
#define DR_EDGE_BOTH 2

typedef struct dr_ctx_s* dr_ctx;     /* one GPU: streams, slab buffers, scheduler */
typedef struct dr_geom_s* dr_geom;   /* device-resident tables of one geometry */
typedef struct dr_batch_s* dr_batch; /* a captured, tuned launch over many scans */
typedef struct dr_list_s* dr_list;   /* a sorted pixel list of one geometry, tiled by row */

/* Detector: pixel (j, i) centre = (origin + i*u) + j*v (um), any orientation.
 * pixel_xyz, when not NULL, is a host array [ny][nx][3] of explicit centres
 * that overrides the affine map.  When every pixel of each row projects to
 * the row's first (eta, xi) bit for bit (a detector whose rows run along the
 * wire axis), rows share one set of FP64 bin positions built once; otherwise
 * each pixel computes its own positions on the fly (the per-pixel path: the
 * same positions and bins, FP32 fractions from one reciprocal of the interval
 * length, so FP32 outputs agree within the FP32 tolerance and the FP64
 * instance exactly; ALU-bound instead of HBM-bound). */
typedef struct {
    int32_t nx, ny;
    double origin[3], u[3], v[3];
    const double* pixel_xyz;
} dr_detector;

/* Wire: a cylinder of `radius` um around the direction `axis` (any length > 0,
 * not along the beam; normalised inside); centers is a host array
 * [n_steps][3] of a point of the axis line at each step (only its projection
 * matters).  edge: DR_EDGE_LEADING, _TRAILING or _BOTH. */
typedef struct {
    double radius;
    double axis[3];
    int32_t n_steps;
    const double* centers;
    int32_t edge;
} dr_wire;

/* Depth grid: n_bins bins of `width` um, bin b centred at first_center + b*width. */
typedef struct {
    int32_t n_bins;
    double first_center, width;
} dr_depth_grid;

/* Launch shape of the reconstruction kernel.  pixels_per_lane in {1,2,4,8},
 * waves_per_group in {2,4}, prefetch (wire steps in flight per lane) in
 * {4,8,16}; groups_per_cu only matters for persistent (batched) launches.
 * A zero field means "choose". */
typedef struct {
    int32_t pixels_per_lane, waves_per_group, prefetch, groups_per_cu;
} dr_tile_config;

/* ------------------------------------------------------------- context */

/* Create a context on HIP device `device`, with its own compute and copy
 * streams (used by dr_geometry_init, dr_autotune, dr_debug_plan and the
 * serving scheduler).  hbm_budget_bytes bounds the device
 * memory the serving scheduler may hold for admitted requests (0 = 90% of the
 * free memory at creation).  Errors: DR_E_INVAL (bad device or NULL out),
 * DR_E_DEVICE (HIP failure). */
dr_status dr_ctx_create(int device, size_t hbm_budget_bytes, dr_ctx* out);

/* Stop the scheduler, wait for outstanding work and free the context.  Every
 * geometry and batch created on it must have been freed first
 * (DR_E_BUSY otherwise). */
dr_status dr_ctx_destroy(dr_ctx ctx);

/* ------------------------------------------------------------ geometry */

/* Build the device tables of one (detector, wire, depth grid) - the
 * per-pixel geometry the paper's kernel reads for each pixel (Sec. III-C) -
 * and check it on the device.  Copies every input, so the caller may free its
 * arrays on return; the library owns *out until dr_geometry_free.
 * Errors: DR_E_INVAL for NULL pointers, nx/ny/n_bins < 1, nx * ny >= 2^32,
 * n_bins > 2^30, n_steps < 2, radius <= 0, width <= 0, an unknown edge, a
 * zero or non-finite axis or one along the beam, a pixel inside the wire, a
 * wire position not strictly between beam and pixel in eta
 * (0 < eta_wire < eta_pixel), or any non-finite depth on the wire edge(s)
 * that wire->edge reconstructs; for geometries on the per-pixel path also a
 * pixel within 2^-383 um of the wire surface (L2 - r^2 < 2^-767) or an edge
 * position 2^30 bins or more from the grid's first bin;
 * DR_E_NOMEM / DR_E_DEVICE for allocation or HIP failures.
 * Synchronous. */
dr_status dr_geometry_init(dr_ctx ctx, const dr_detector* det, const dr_wire* wire,
                           const dr_depth_grid* grid, dr_geom* out);

/* Per-step sample weights (beam-monitor normalisation; the paper describes
 * none): with weights w[n_steps] set, every sample becomes I_k * w_k (FP64)
 * before the differences are taken, I_k*w_k - I_{k+1}*w_{k+1} formed in FP64
 * and rounded once for the FP32 accumulation; w_k = mean(m)/m_k normalises
 * by monitor counts m_k.  NULL removes them.  Copied; waits for the device
 * work already enqueued.  With weights the reconstruction uses one launch
 * shape (1 pixel per lane, 4 waves, prefetch 16; dr_set_tile and dr_autotune
 * do not change it).
 * Errors: DR_E_INVAL (NULL geometry, a non-finite weight), DR_E_BUSY
 * (serving requests in flight, or a batch built on the geometry: batches
 * keep the launch plan they were built with). */
dr_status dr_geometry_set_step_weights(dr_geom geom, const double* weights);

/* Which path a geometry takes: DR_PATH_ROWS (per-row FP64 bin tables built
 * once, HBM-bound kernel) or DR_PATH_PIXELS (positions computed per pixel on
 * the fly).  Errors: DR_E_INVAL for NULL arguments. */
#define DR_PATH_ROWS 0
#define DR_PATH_PIXELS 1
dr_status dr_geometry_path(dr_geom geom, int32_t* path);

/* Per-pixel path diagnostic: the margin (bin units) within which a position
 * of the shorter FP64 form (hardware reciprocal square root and reciprocal,
 * each refined by one Newton step) must not come to an integer for its floor
 * to be taken as the bin; closer positions are evaluated in the exact form,
 * so bins always follow the exact positions.  max_error (may be NULL)
 * receives the largest distance between the two forms, which the geometry
 * check finds by evaluating both at every pixel and step the kernel
 * evaluates (bin units; 0 for the per-row path).  The shorter form is used
 * only while that distance is below half the margin and every non-zero step
 * is at least 2^28 times it long; otherwise, or when the geometry's bound is
 * not small, *margin >= 1 and every position is evaluated in the exact form.
 * 0 for the per-row path.  Errors: DR_E_INVAL for NULL geom or margin. */
dr_status dr_geometry_position_margin(dr_geom geom, double* margin, double* max_error);

/* Free a geometry.  Waits for the device work already enqueued on it.
 * DR_E_BUSY while serving requests that use it are in flight, or while
 * pixel lists or batches built on it exist. */
dr_status dr_geometry_free(dr_geom geom);

/* Force a launch shape for this geometry (tile-invariance tests, manual
 * tuning); NULL restores the automatic choice.  DR_E_INVAL for values outside
 * the sets listed at dr_tile_config or a shape that does not fit nx or the
 * buffer alignment at launch time; DR_E_UNSUPPORTED for a geometry on the
 * per-pixel path, which has a single launch shape. */
dr_status dr_set_tile(dr_geom geom, const dr_tile_config* tile);

/* Time the available launch shapes on this geometry with the caller's device
 * buffers and keep the fastest for later calls (autotuner; results are cached
 * per device architecture and size class, and in the JSON file named by the
 * environment variable DR_TUNE_CACHE when set).  `out` is overwritten.
 * Synchronous.  *chosen (if not NULL) receives the winner.  On the per-pixel
 * path nothing is timed and *chosen receives its one shape (1, 4, 8, 0). */
dr_status dr_autotune(dr_geom geom, const uint16_t* images_dev, float* out_dev,
                      dr_tile_config* chosen);

/* -------------------------------------------------------- reconstruction */

/* Reconstruct one scan (paper Sec. III-C) into out[n_bins][ny][nx] (device,
 * FP32) and, when totals is not NULL, totals[n_bins] (device, FP32).
 *   images_on_device != 0: images is a device pointer [n_steps][ny][nx].
 *   images_on_device == 0: images is host memory (pinned for full speed);
 *     it is streamed to the device in row slabs, each slab's copy on the
 *     context's copy stream overlapping the kernel of the previous slab - the
 *     paper's pass-per-row-slab scheme (Sec. III-B) with double buffering.
 * stream is a hipStream_t (NULL = the HIP null stream).  The call
 * returns after enqueueing; buffers must stay valid and unchanged until the
 * stream reaches the end of the enqueued work.  Errors: DR_E_INVAL for NULL
 * or misaligned pointers, DR_E_DEVICE for HIP failures. */
dr_status dr_reconstruct(dr_geom geom, const uint16_t* images, int images_on_device,
                         float* out, float* totals, void* stream);

/* Same operation with FP64 intensity differences and FP64 accumulation into
 * out[n_bins][ny][nx] and totals[n_bins] (both device, double).  Validation
 * instance of the same kernel: it performs the oracle's operations in the
 * oracle's order.  images must be on the device. */
dr_status dr_reconstruct_f64(dr_geom geom, const uint16_t* images_dev, double* out,
                             double* totals, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * operation of dr_reconstruct on device-resident images, with its scratch
 * (the per-wave partial totals and the totals workspace) taken from one fixed
 * device array of 128 MiB that the library holds on each GPU it runs on until
 * the process ends, instead of the geometry's scratch buffers that
 * dr_reconstruct grows on demand.  No hipMalloc, hipFree or other allocating
 * call is made; images_dev, out and totals are the caller's, as in
 * dr_reconstruct (out [n_bins][ny][nx] FP32, totals [n_bins] FP32 or NULL;
 * stream NULL = the HIP null stream; returns after enqueueing).  Every call on
 * one GPU shares that GPU's array, so calls whose work overlaps in time on one
 * GPU (other streams, other host threads) race and must be serialized by the
 * caller; each call writes every scratch element it reads before reading it.
 * The array holds the totals scratch of a 2048 x 2048 scan with 1001 bins
 * and one edge on the per-row path; per-pixel geometries need five rows of
 * n_bins floats per 256 pixels, so a per-pixel 2048 x 2048 scan with totals
 * does not fit.
 * Errors: DR_E_INVAL for NULL or misaligned pointers, and for a scan whose
 * totals need more scratch than the array holds (the message gives both
 * sizes; pass totals = NULL, which needs none, or use dr_reconstruct);
 * DR_E_DEVICE for HIP failures. */
dr_status dr_reconstruct_noalloc(dr_geom geom, const uint16_t* images_dev, float* out,
                                 float* totals, void* stream);

/* Positions of one wire edge (edge: DR_EDGE_LEADING or DR_EDGE_TRAILING),
 * computed by the device code the kernels use, for a host list of pixels
 * (flat indices j*nx + i): bins_out[n][n_steps] receives floor(u_k) as int32
 * (saturated) and u_out[n][n_steps] the FP64 positions in bin units,
 * u_k = (d_k - e0) * (1/width) with e0 = first_center - width/2; either output
 * may be NULL.  Positions of an edge the geometry does not reconstruct were
 * not checked at dr_geometry_init and may be non-finite.  Host buffers;
 * synchronous.  DR_E_INVAL for an out-of-range pixel or edge. */
dr_status dr_debug_plan(dr_geom geom, const int64_t* pixels, int32_t n, int32_t edge,
                        int32_t* bins_out, double* u_out);

/* Device time in milliseconds of the last reconstruction kernel launched by
 * dr_reconstruct on this geometry (HIP events on the launch stream; waits for
 * them), and of the totals reduction after it.  Timing is recorded only after
 * dr_enable_timing(geom, 1). */
dr_status dr_enable_timing(dr_geom geom, int enable);
dr_status dr_last_timing(dr_geom geom, double* kernel_ms, double* totals_ms);

/* -------------------------------------------------------------- batches */

/* One scan of a batch: device images [n_steps][ny][nx], device out, device
 * totals (or NULL), each scan with its own geometry. */
typedef struct {
    dr_geom geom;
    const uint16_t* images;
    float* out;
    float* totals;
} dr_batch_item;

#define DR_BATCH_AUTOTUNE 1 /* time launch shapes on the batch and keep the best */
#define DR_BATCH_GRAPH 2    /* capture the launch sequence in a hipGraph */

/* Plan one persistent launch over many scans of uneven size: work items are
 * (scan, row tile) pairs ordered by cost and pulled by workgroups from a
 * device queue.  The plan keeps the item pointers, so the buffers must stay
 * allocated while the batch exists; their contents may change between runs.
 * With DR_BATCH_AUTOTUNE the outputs are overwritten while tuning.
 * Scans on the per-pixel path or with step weights are not in the persistent
 * launch: each of their passes is one launch of its own kernel after it (in
 * the graph too).
 * Errors: DR_E_INVAL (n < 1, NULL items, geometries of another context),
 * DR_E_NOMEM, DR_E_DEVICE. */
dr_status dr_batch_create(dr_ctx ctx, int32_t n, const dr_batch_item* items, int32_t flags,
                          dr_batch* out);

/* Run the batch on `stream` (a hipStream_t; NULL = the HIP null stream):
 * replays the captured graph when the batch has one.  Returns after
 * enqueueing. */
dr_status dr_batch_run(dr_batch batch, void* stream);

/* The launch shape the batch uses. */
dr_status dr_batch_tile(dr_batch batch, dr_tile_config* tile);

dr_status dr_batch_free(dr_batch batch);

/* ---------------------------------------------------------- pixel lists */

/* Reconstructing a chosen part of the detector (the paper's second
 * experiment, Sec. IV, processes a percentage of the pixels without saying
 * which).  Selection rule: the activity of pixel p is
 * A_p = sum_k |I_k - I_{k+1}| over its samples, and the top-k list keeps the k
 * pixels of largest A_p, ties going to the lower index.  Every list is held
 * on the device in increasing pixel index (p = j*nx + i) and cut into tiles:
 * with per-row plans, windows of at most 64 entries (one wave each) inside one
 * detector row; on the per-pixel path, runs of 256 consecutive entries.
 * Results for a listed pixel are
 * bitwise those of dr_reconstruct / dr_reconstruct_f64 for that pixel. */

/* Image layouts for list reconstruction. */
#define DR_LAYOUT_FULL 0 /* full frames uint16 [n_steps][ny][nx], gathered by pixel */
#define DR_LAYOUT_LIST 1 /* compact uint16 [n_steps][n], column e = list entry e */

/* activity_dev[p] = A_p for every pixel of a device stack [n_steps][ny][nx]
 * (uint64, exact).  Asynchronous on `stream` (NULL = the HIP null stream);
 * one pass over the stack.  Errors: DR_E_INVAL (NULL or misaligned). */
dr_status dr_pixel_activity(dr_geom geom, const uint16_t* images_dev, uint64_t* activity_dev,
                            void* stream);

/* The top-k list from device activities [nx*ny] (0 <= k <= nx*ny), selected
 * on the device on the context's stream: the activities must be complete
 * (synchronize the stream that computed them).  Synchronous; the library owns
 * *out until dr_list_free.
 * Errors: DR_E_INVAL (NULL, k out of range, misaligned), DR_E_NOMEM. */
dr_status dr_select_top(dr_geom geom, const uint64_t* activity_dev, int64_t k, dr_list* out);

/* A list from the caller's pixel indices (host or device array of n int64,
 * strictly increasing, each in [0, nx*ny)), copied and checked on the device.
 * Synchronous.  Errors: DR_E_INVAL for an index out of range or an order that
 * is not strictly increasing. */
dr_status dr_list_create(dr_geom geom, const int64_t* pixels, int64_t n, int pixels_on_device,
                         dr_list* out);

dr_status dr_list_size(dr_list list, int64_t* n);

/* Copy the list's n pixel indices to a host array (synchronous). */
dr_status dr_list_pixels(dr_list list, int64_t* pixels_host);

/* Free a list (waits for the device).  Lists must be freed before their
 * geometry (dr_geometry_free returns DR_E_BUSY while any is alive). */
dr_status dr_list_free(dr_list list);

/* Reconstruct the listed pixels: out float [n_bins][n] on the device, column
 * e for list entry e, every element written; totals float [n_bins] (or NULL)
 * = sum of out over the list.  images: device, either layout; or host
 * (pinned for overlap) in DR_LAYOUT_LIST only, streamed in runs of whole
 * tiles through the context's two slab buffers, so the bytes sent over PCIe
 * are n/(nx*ny) of a full stack.  Edges as set for the geometry.  Errors:
 * DR_E_INVAL (NULL, misaligned, unknown layout, host images in full layout). */
dr_status dr_reconstruct_list(dr_list list, const uint16_t* images, int32_t layout,
                              int images_on_device, float* out, float* totals, void* stream);

/* FP64 instance of dr_reconstruct_list (device images): out double
 * [n_bins][n], in the oracle's operation order, bit for bit. */
dr_status dr_reconstruct_list_f64(dr_list list, const uint16_t* images_dev, int32_t layout,
                                  double* out, double* totals, void* stream);

/* ---------------------------------------------------------------- serving */

/* Queue one reconstruction request with the context's scheduler and return
 * at once with a ticket.  Requests are admitted in arrival order while the
 * device memory they need (image staging for host images, plus scratch) fits
 * the context budget; admitted requests are continuously batched: each
 * scheduling epoch is one persistent launch over row tiles of every admitted
 * request whose images are resident, so requests that arrive while others
 * run join the next epoch.  Each pixel's result is bitwise the same as with
 * dr_reconstruct.  images: host (pinned) or device per images_on_device;
 * out/totals: device, as in dr_reconstruct.  The request's device work is
 * not ordered after any stream of the caller: work that writes images, out
 * or totals (an initialising fill, the copy that produces the images) must
 * have completed when dr_submit is called.  The caller keeps every buffer
 * valid until dr_poll reports DR_OK or an error for the ticket.
 * Requests on the per-pixel path or with step weights get launches of their
 * own kernel in each epoch.
 * Errors: DR_E_INVAL, DR_E_NOMEM (the request can never fit the budget). */
dr_status dr_submit(dr_ctx ctx, dr_geom geom, const uint16_t* images, int images_on_device,
                    float* out, float* totals, uint64_t* ticket);

/* DR_PENDING while the request is queued or running, DR_OK once its results
 * are complete in device memory, a negative error if it failed (sticky),
 * DR_E_NOTFOUND for an unknown or already-collected ticket.  A ticket is
 * forgotten after dr_poll has returned DR_OK or an error for it once. */
dr_status dr_poll(dr_ctx ctx, uint64_t ticket);

/* Block until the ticket completes; same results as dr_poll. */
dr_status dr_wait(dr_ctx ctx, uint64_t ticket);

/* Scheduler counters. */
typedef struct {
    uint64_t submitted, admitted, completed, epochs, tiles_launched;
    uint64_t bytes_h2d;
    size_t hbm_in_use, hbm_budget;
} dr_stats;
dr_status dr_ctx_stats(dr_ctx ctx, dr_stats* out);

/* Message of the last error on the calling thread ("" if none). */
const char* dr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DR_H */
