// Pixel lists behind the C ABI: activity, top-k selection, caller lists and
// the reconstruction of the listed pixels only (device images gathered from
// full frames, or compact [N][n] stacks that a host streams in chunks, so
// that the bytes sent scale with the fraction of pixels kept).
#include "dr_runtime.h"

#include <algorithm>
#include <cstdlib>
#include <vector>

struct dr_list_s {
    ~dr_list_s()
    {
        if (g) g->lists--;
    }
    dr_geom g = nullptr;
    int64_t n = 0;
    int64_t n_tiles = 0;
    dr::DevBuf pixels;  // int64 [n]
    dr::DevBuf tiles;   // int32 row [n_tiles], int64 start [n_tiles], int32 count [n_tiles]
    std::vector<int64_t> h_start;  // tile starts and counts, for host chunking
    std::vector<int32_t> h_count;
    dr::DevBuf part32, part64, work;
    std::mutex mu;
};

namespace dr {

static bool aligned_to(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// host runs of a compact stack start and end on multiples of this many
// entries (128 bytes), the last one at the end of the list
constexpr int64_t kRunAlign = kListAlign;

// Tile table of a validated list held in l->pixels: per-row plan path, wave
// tiles inside one detector row, each ending at the next multiple of
// kListAlign entries; per-pixel path, aligned runs of kListTile consecutive
// entries.  Synchronous (reads the row starts back).
static dr_status build_tiles(dr_list l, hipStream_t s)
{
    const dr_geom g = l->g;
    std::vector<int32_t> rows;
    l->h_start.clear();
    l->h_count.clear();
    if (g->row_mode) {
        DevBuf starts;
        DR_HIP(starts.reserve((size_t)(g->ny + 1) * sizeof(int64_t)));
        DR_HIP(launch_list_rows(l->pixels.as<int64_t>(), l->n, g->nx, g->ny,
                                starts.as<int64_t>(), s));
        std::vector<int64_t> h(g->ny + 1);
        DR_HIP(hipMemcpyAsync(h.data(), starts.p, h.size() * sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
        DR_HIP(hipStreamSynchronize(s));
        // wave tiles: a tile ends at the next multiple of kListAlign entries
        // (at most 64 lanes from its start rounded down), so all but a row's
        // first start aligned
        for (int j = 0; j < g->ny; ++j)
            for (int64_t e = h[j]; e < h[j + 1];) {
                const int64_t end = std::min<int64_t>(h[j + 1], e - e % kListAlign + kListAlign);
                rows.push_back(j);
                l->h_start.push_back(e);
                l->h_count.push_back((int32_t)(end - e));
                e = end;
            }
    } else {
        for (int64_t e = 0; e < l->n; e += kListTile) {
            rows.push_back(0);
            l->h_start.push_back(e);
            l->h_count.push_back((int32_t)std::min<int64_t>(kListTile, l->n - e));
        }
    }
    l->n_tiles = (int64_t)rows.size();
    const size_t T = std::max<size_t>(1, rows.size());
    DR_HIP(l->tiles.reserve(up256(T * 4) + up256(T * 8) + T * 4));
    char* b = l->tiles.as<char>();
    if (l->n_tiles) {
        DR_HIP(hipMemcpyAsync(b, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, s));
        DR_HIP(hipMemcpyAsync(b + up256(T * 4), l->h_start.data(), rows.size() * 8,
                              hipMemcpyHostToDevice, s));
        DR_HIP(hipMemcpyAsync(b + up256(T * 4) + up256(T * 8), l->h_count.data(), rows.size() * 4,
                              hipMemcpyHostToDevice, s));
        DR_HIP(hipStreamSynchronize(s));
    }
    return DR_OK;
}

static ListArgs list_args(const dr_list l, int32_t compact)
{
    const size_t T = std::max<size_t>(1, (size_t)l->n_tiles);
    const char* b = l->tiles.as<char>();
    ListArgs la{};
    la.pixels = l->pixels.as<int64_t>();
    la.tile_row = (const int32_t*)b;
    la.tile_start = (const int64_t*)(b + up256(T * 4));
    la.tile_count = (const int32_t*)(b + up256(T * 4) + up256(T * 8));
    la.n = l->n;
    la.tile_first = 0;
    la.compact = compact;
    la.entry_base = 0;
    return la;
}

// workgroups of one pass, and partial-total rows of one pass
static int64_t list_groups(const dr_list l) { return l->n_tiles; }
// partial-total rows of one pass: one per wave tile on the row path,
// kPixelPartialRows per tile on the per-pixel path
static int64_t list_slots(const dr_list l)
{
    return l->n_tiles * (l->g->row_mode ? 1 : kPixelPartialRows);
}

// Scan arguments of pass p over a list: images img (full frames: step stride
// nx*ny; compact: step stride `img_step` entries), output [n_bins][n].
static ScanArgs list_scan_args(const dr_list l, int p, const uint16_t* img, int64_t img_step,
                               void* out, void* partials, size_t elem, int64_t slots)
{
    const dr_geom g = l->g;
    ScanArgs a{};
    a.pass = g->passes == 1 ? 0 : p + 1;
    a.img = img;
    a.img_step = img_step;
    a.img_row = g->nx;
    a.row_base = 0;
    a.nx = g->nx;
    a.ny = g->ny;
    a.row_begin = 0;
    a.row_end = g->ny;
    a.tiles_per_row = 1;
    a.n_steps = g->n_steps;
    a.n_bins = g->n_bins;
    a.out = out;
    a.out_plane = l->n;
    a.partials = partials ? (char*)partials + (size_t)p * slots * g->n_bins * elem : nullptr;
    a.wk = g->weighted ? g->wbuf.as<double>() : nullptr;
    if (g->row_mode) {
        const PlanTables& pt = g->t[p];
        a.bl = pt.bl;
        a.nb = pt.nb;
        a.f0 = pt.f0;
        a.fm = pt.fm;
        a.f1 = pt.f1;
        a.d0 = pt.d0;
        a.dm = pt.dm;
        a.d1 = pt.d1;
        a.row_class = pt.row_class;
        a.row_lo = pt.row_lo;
        a.row_hi = pt.row_hi;
    }
    return a;
}

static hipError_t launch_list_pass(const dr_list l, int p, const ScanArgs& a, const ListArgs& la,
                                   int64_t n_tiles, bool f64, hipStream_t s)
{
    const dr_geom g = l->g;
    if (g->row_mode)
        return f64 ? launch_list_f64(a, la, n_tiles, s) : launch_list_f32(a, la, n_tiles, s);
    return f64 ? launch_list_pixels_f64(a, g->g, g->side[p], g->scale[p], la, n_tiles, s)
               : launch_list_pixels_f32(a, g->g, g->side[p], g->scale[p], la, n_tiles, s);
}

static dr_status new_list(dr_geom g, int64_t n, dr_list* out)
{
    auto l = std::make_unique<dr_list_s>();
    l->g = g;
    g->lists++;  // the destructor gives it back
    l->n = n;
    DR_HIP(l->pixels.reserve(std::max<size_t>(8, (size_t)n * sizeof(int64_t))));
    *out = l.release();
    return DR_OK;
}

}  // namespace dr

using namespace dr;

extern "C" {

dr_status dr_pixel_activity(dr_geom g, const uint16_t* images_dev, uint64_t* activity_dev,
                            void* stream)
{
    if (!g || !images_dev || !activity_dev)
        return set_error(DR_E_INVAL, "dr_pixel_activity: NULL argument");
    if (!aligned_to(images_dev, 2) || !aligned_to(activity_dev, 8))
        return set_error(DR_E_INVAL, "dr_pixel_activity: misaligned buffer");
    DR_HIP(hipSetDevice(g->ctx->device));
    const int64_t npix = (int64_t)g->nx * g->ny;
    const bool vec4 = aligned_to(images_dev, 8) && npix % 4 == 0;
    DR_HIP(launch_activity(images_dev, npix, g->n_steps, activity_dev, vec4, (hipStream_t)stream));
    set_error(DR_OK, "");
    return DR_OK;
}

dr_status dr_select_top(dr_geom g, const uint64_t* activity_dev, int64_t k, dr_list* out)
{
    if (!g || !activity_dev || !out) return set_error(DR_E_INVAL, "dr_select_top: NULL argument");
    *out = nullptr;
    const int64_t npix = (int64_t)g->nx * g->ny;
    if (k < 0 || k > npix) return set_error(DR_E_INVAL, "dr_select_top: k outside [0, nx*ny]");
    if (!aligned_to(activity_dev, 8)) return set_error(DR_E_INVAL, "dr_select_top: misaligned");
    DR_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = g->ctx->stream;
    dr_list l = nullptr;
    dr_status st = new_list(g, k, &l);
    if (st != DR_OK) return st;
    std::unique_ptr<dr_list_s> own(l);
    {
        // selection state and block sums in the geometry's buffer (kept
        // between calls), held under its lock; build_tiles reads the list
        // back on the same stream and waits, so the kernels are done before
        // the lock is released
        std::lock_guard<std::mutex> lk(g->mu);
        if (k > 0) {
            const size_t nb = (size_t)((npix + kSelectBlock - 1) / kSelectBlock);
            DR_HIP(g->sel.reserve(up256(sizeof(SelectState)) + nb * sizeof(uint64_t)));
            char* base = g->sel.as<char>();
            DR_HIP(launch_select_top(activity_dev, npix, k, (SelectState*)base,
                                     (uint64_t*)(base + up256(sizeof(SelectState))),
                                     l->pixels.as<int64_t>(), s));
        }
        st = build_tiles(l, s);
        if (st != DR_OK) {
            (void)hipStreamSynchronize(s);
            return st;
        }
    }
    *out = own.release();
    set_error(DR_OK, "");
    return DR_OK;
}

dr_status dr_list_create(dr_geom g, const int64_t* pixels, int64_t n, int pixels_on_device,
                         dr_list* out)
{
    if (!g || !out || (n > 0 && !pixels))
        return set_error(DR_E_INVAL, "dr_list_create: NULL argument");
    *out = nullptr;
    const int64_t npix = (int64_t)g->nx * g->ny;
    if (n < 0 || n > npix) return set_error(DR_E_INVAL, "dr_list_create: n outside [0, nx*ny]");
    DR_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = g->ctx->stream;
    dr_list l = nullptr;
    dr_status st = new_list(g, n, &l);
    if (st != DR_OK) return st;
    std::unique_ptr<dr_list_s> own(l);
    if (n > 0) {
        DR_HIP(hipMemcpyAsync(l->pixels.p, pixels, (size_t)n * sizeof(int64_t),
                              pixels_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              s));
        DevBuf status;
        DR_HIP(status.reserve(sizeof(int)));
        DR_HIP(hipMemsetAsync(status.p, 0, sizeof(int), s));
        DR_HIP(launch_list_check(l->pixels.as<int64_t>(), n, npix, status.as<int>(), s));
        int h = 0;
        DR_HIP(hipMemcpyAsync(&h, status.p, sizeof(int), hipMemcpyDeviceToHost, s));
        DR_HIP(hipStreamSynchronize(s));
        if (h & 1) return set_error(DR_E_INVAL, "dr_list_create: pixel index outside the detector");
        if (h & 2) return set_error(DR_E_INVAL, "dr_list_create: pixels not strictly increasing");
    }
    st = build_tiles(l, s);
    if (st != DR_OK) return st;
    *out = own.release();
    set_error(DR_OK, "");
    return DR_OK;
}

dr_status dr_list_size(dr_list l, int64_t* n)
{
    if (!l || !n) return set_error(DR_E_INVAL, "dr_list_size: NULL argument");
    *n = l->n;
    return DR_OK;
}

dr_status dr_list_pixels(dr_list l, int64_t* pixels_host)
{
    if (!l || (l->n > 0 && !pixels_host))
        return set_error(DR_E_INVAL, "dr_list_pixels: NULL argument");
    if (l->n == 0) return DR_OK;
    DR_HIP(hipSetDevice(l->g->ctx->device));
    DR_HIP(hipMemcpy(pixels_host, l->pixels.p, (size_t)l->n * sizeof(int64_t),
                     hipMemcpyDeviceToHost));
    set_error(DR_OK, "");
    return DR_OK;
}

dr_status dr_list_free(dr_list l)
{
    if (!l) return set_error(DR_E_INVAL, "dr_list_free: NULL list");
    DR_HIP(hipSetDevice(l->g->ctx->device));
    DR_HIP(hipDeviceSynchronize());
    delete l;
    return DR_OK;
}

dr_status dr_reconstruct_list(dr_list l, const uint16_t* images, int32_t layout,
                              int images_on_device, float* out, float* totals, void* stream)
{
    if (!l || !images || !out) return set_error(DR_E_INVAL, "dr_reconstruct_list: NULL argument");
    if (layout != DR_LAYOUT_FULL && layout != DR_LAYOUT_LIST)
        return set_error(DR_E_INVAL, "dr_reconstruct_list: unknown image layout");
    if (!images_on_device && layout != DR_LAYOUT_LIST)
        return set_error(DR_E_INVAL, "dr_reconstruct_list: host images must be in list layout");
    if (!aligned_to(out, 4) || (totals && !aligned_to(totals, 4)) || !aligned_to(images, 2))
        return set_error(DR_E_INVAL, "dr_reconstruct_list: misaligned buffer");
    const dr_geom g = l->g;
    dr_ctx c = g->ctx;
    DR_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    float* part = nullptr;
    const int32_t compact = layout == DR_LAYOUT_LIST;
    const int64_t slots = list_slots(l), groups = list_groups(l);
    if (totals) {
        std::lock_guard<std::mutex> lk(l->mu);
        DR_HIP(l->part32.reserve(std::max<size_t>(4, (size_t)g->passes * slots * g->n_bins * 4)));
        DR_HIP(l->work.reserve((size_t)kTotalsWorkRows * g->n_bins * sizeof(double)));
        part = l->part32.as<float>();
    }
    if (images_on_device) {
        const int64_t step = compact ? l->n : (int64_t)g->nx * g->ny;
        const ListArgs la = list_args(l, compact);
        for (int p = 0; p < g->passes; ++p) {
            const ScanArgs a = list_scan_args(l, p, images, step, out, part, 4, slots);
            DR_HIP(launch_list_pass(l, p, a, la, groups, false, s));
        }
    } else {
        // compact host stack: runs of whole tiles copied into the context's
        // two slab buffers on its copy stream, each run's kernels overlapping
        // the next run's copy.  A run's window is widened to multiples of
        // kRunAlign entries so that every copied line starts aligned.
        size_t target = (size_t)256 << 20;
        if (const char* e = std::getenv("DR_SLAB_MB")) target = (size_t)std::max(1, atoi(e)) << 20;
        const size_t per_entry = (size_t)g->n_steps * sizeof(uint16_t);
        int64_t cap = std::max<int64_t>(kListTile, (int64_t)(target / per_entry));
        if (const char* e = std::getenv("DR_LIST_RUN_ENTRIES"))  // smaller runs (tests)
            cap = std::max<int64_t>(kListTile, atoll(e));
        std::lock_guard<std::mutex> lk(c->mu);
        const size_t slab_bytes = (size_t)(cap + 2 * kRunAlign) * per_entry;
        for (int i = 0; i < 2; ++i)
            if (c->slab[i].bytes < slab_bytes) {
                DR_HIP(hipStreamSynchronize(c->copy));
                DR_HIP(hipStreamSynchronize(c->stream));
                DR_HIP(hipDeviceSynchronize());
                DR_HIP(c->slab[i].reserve(slab_bytes));
            }
        int run = 0;
        for (int64_t t0 = 0; t0 < l->n_tiles; ++run) {
            const int64_t e0 = l->h_start[t0];
            int64_t t1 = t0 + 1;
            while (t1 < l->n_tiles && l->h_start[t1] + l->h_count[t1] - e0 <= cap) ++t1;
            const int64_t e1 = l->h_start[t1 - 1] + l->h_count[t1 - 1];
            const int64_t a0 = e0 - e0 % kRunAlign;
            const int64_t a1 = std::min<int64_t>(l->n, (e1 + kRunAlign - 1) / kRunAlign * kRunAlign);
            const int b = run & 1;
            DR_HIP(hipStreamWaitEvent(c->copy, c->slab_free[b], 0));
            DR_HIP(hipMemcpy2DAsync(c->slab[b].p, (size_t)(a1 - a0) * sizeof(uint16_t),
                                    images + a0, (size_t)l->n * sizeof(uint16_t),
                                    (size_t)(a1 - a0) * sizeof(uint16_t), (size_t)g->n_steps,
                                    hipMemcpyHostToDevice, c->copy));
            DR_HIP(hipEventRecord(c->slab_ready[b], c->copy));
            DR_HIP(hipStreamWaitEvent(s, c->slab_ready[b], 0));
            ListArgs la = list_args(l, 1);
            la.tile_first = t0;
            la.entry_base = a0;
            for (int p = 0; p < g->passes; ++p) {
                const ScanArgs a = list_scan_args(l, p, c->slab[b].as<uint16_t>(), a1 - a0, out,
                                                  part, 4, slots);
                DR_HIP(launch_list_pass(l, p, a, la, t1 - t0, false, s));
            }
            DR_HIP(hipEventRecord(c->slab_free[b], s));
            t0 = t1;
        }
    }
    if (totals) {
        if (groups == 0) {
            DR_HIP(hipMemsetAsync(totals, 0, (size_t)g->n_bins * sizeof(float), s));
        } else {
            DR_HIP(launch_totals_f32(part, slots * g->passes, g->n_bins, l->work.as<double>(),
                                     kTotalsWorkRows, totals, s));
        }
    }
    set_error(DR_OK, "");
    return DR_OK;
}

dr_status dr_reconstruct_list_f64(dr_list l, const uint16_t* images_dev, int32_t layout,
                                  double* out, double* totals, void* stream)
{
    if (!l || !images_dev || !out)
        return set_error(DR_E_INVAL, "dr_reconstruct_list_f64: NULL argument");
    if (layout != DR_LAYOUT_FULL && layout != DR_LAYOUT_LIST)
        return set_error(DR_E_INVAL, "dr_reconstruct_list_f64: unknown image layout");
    if (!aligned_to(out, 8) || (totals && !aligned_to(totals, 8)) || !aligned_to(images_dev, 2))
        return set_error(DR_E_INVAL, "dr_reconstruct_list_f64: misaligned buffer");
    const dr_geom g = l->g;
    DR_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    double* part = nullptr;
    const int32_t compact = layout == DR_LAYOUT_LIST;
    const int64_t slots = list_slots(l), groups = list_groups(l);
    // totals: per-tile partial rows on the row path; on the per-pixel path the
    // column sums of the finished output, in a fixed order
    if (totals) {
        std::lock_guard<std::mutex> lk(l->mu);
        if (g->row_mode) {
            DR_HIP(l->part64.reserve(
                std::max<size_t>(8, (size_t)g->passes * slots * g->n_bins * 8)));
            part = l->part64.as<double>();
        }
        DR_HIP(l->work.reserve((size_t)kTotalsWorkRows * g->n_bins * sizeof(double)));
    }
    const int64_t step = compact ? l->n : (int64_t)g->nx * g->ny;
    const ListArgs la = list_args(l, compact);
    // two edges: the second pass is formed in a buffer of its own and added
    // onto the first (as in dr_reconstruct_f64)
    const int64_t n_out = (int64_t)g->n_bins * l->n;
    double* second = nullptr;
    if (g->passes == 2 && n_out > 0)
        DR_HIP(hipMallocAsync((void**)&second, (size_t)n_out * sizeof(double), s));
    hipError_t e = hipSuccess;
    for (int p = 0; p < g->passes && e == hipSuccess; ++p) {
        ScanArgs a = list_scan_args(l, p, images_dev, step, p == 0 ? out : second, part, 8,
                                    slots);
        a.pass = 0;
        e = launch_list_pass(l, p, a, la, groups, true, s);
    }
    if (e == hipSuccess && second) e = launch_add_f64(out, second, n_out, s);
    if (second) {
        const hipError_t ef = hipFreeAsync(second, s);
        if (e == hipSuccess) e = ef;
    }
    DR_HIP(e);
    if (totals) {
        if (groups == 0) {
            DR_HIP(hipMemsetAsync(totals, 0, (size_t)g->n_bins * sizeof(double), s));
        } else if (g->row_mode) {
            DR_HIP(launch_totals_f64(part, slots * g->passes, g->n_bins, l->work.as<double>(),
                                     kTotalsWorkRows, totals, s));
        } else {
            DR_HIP(launch_plane_totals_f64(out, l->n, g->n_bins, l->work.as<double>(),
                                           kTotalsWorkRows, totals, s));
        }
    }
    set_error(DR_OK, "");
    return DR_OK;
}

}  // extern "C"
