// Host runtime behind the C ABI: contexts, geometries, single-scan and
// slab-streamed reconstruction, the autotuner and captured batch launches.
#include "dr_runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace dr {

static thread_local std::string g_last_error;

dr_status set_error(dr_status code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

dr_status hip_error(hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return set_error(DR_E_NOMEM, m);
    return set_error(DR_E_DEVICE, m);
}

static dr_status ok()
{
    g_last_error.clear();
    return DR_OK;
}

static bool finite3(const double* v)
{
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// ------------------------------------------------------------ launch shapes

bool tile_fits(const dr_geom g, const TileCfg& t, const void* img, const void* out)
{
    if (!tile_supported(t)) return false;
    if (g->nx % t.ppl != 0) return false;
    if (img && !aligned(img, 2 * (size_t)t.ppl)) return false;
    if (out && !aligned(out, std::min<size_t>(16, 4 * (size_t)t.ppl))) return false;
    return true;
}

TileCfg default_tile(const dr_geom g, const void* img, const void* out)
{
    static const TileCfg prefs[] = {{2, 4, 16}, {1, 4, 16}};
    for (const TileCfg& t : prefs)
        if (tile_fits(g, t, img, out)) return t;
    return TileCfg{1, 4, 16};
}

static int tiles_per_row(const dr_geom g, const TileCfg& t)
{
    const int tw = g->row_mode ? tile_width(t) : kPixelTile;
    return (g->nx + tw - 1) / tw;
}

int64_t partial_slots(const dr_geom g, const TileCfg& t)
{
    // row path: one partial row per wave; per-pixel path: kPixelPartialRows
    // per workgroup of the FP32 kernel (the FP64 instance takes its totals
    // from its finished output)
    return (int64_t)g->ny * tiles_per_row(g, t) * (g->row_mode ? t.waves : kPixelPartialRows);
}

ScanArgs scan_args(const dr_geom g, const TileCfg& t, int pass, const uint16_t* img,
                   int64_t img_step, int row_base, int row_begin, int row_end, float* out,
                   float* partials)
{
    ScanArgs a{};
    a.pass = g->passes == 1 ? 0 : pass + 1;
    a.img = img;
    a.img_step = img_step;
    a.img_row = g->nx;
    a.row_base = row_base;
    a.nx = g->nx;
    a.ny = g->ny;
    a.row_begin = row_begin;
    a.row_end = row_end;
    a.tiles_per_row = tiles_per_row(g, t);
    a.n_steps = g->n_steps;
    a.n_bins = g->n_bins;
    a.out = out;
    a.out_plane = (int64_t)g->nx * g->ny;
    a.partials = partials ? partials + (size_t)pass * partial_slots(g, t) * g->n_bins : nullptr;
    a.wk = g->weighted ? g->wbuf.as<double>() : nullptr;
    if (!g->row_mode) return a;
    const PlanTables& pt = g->t[pass];
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
    return a;
}

hipError_t enqueue_totals(const dr_geom g, const float* partials, int64_t slots, double* work,
                          float* totals, hipStream_t s)
{
    // slots: partial rows of one pass; the partial rows of every pass are summed
    return launch_totals_f32(partials, slots * g->passes, g->n_bins, work, kTotalsWorkRows,
                             totals, s);
}

bool batch_solo(const dr_geom g) { return !g->row_mode || g->weighted; }

TileCfg solo_tile(const dr_geom) { return TileCfg{1, 4, 16}; }

// pass p of any path: the per-row plan kernel (weighted or not) or the
// per-pixel kernel
hipError_t launch_scan_f32(const dr_geom g, const TileCfg& t, int p, const ScanArgs& a,
                           hipStream_t s)
{
    if (g->row_mode) return a.wk ? launch_rows_norm_f32(a, s) : launch_rows_f32(t, a, s);
    return launch_pixels_f32(a, g->g, g->side[p], g->scale[p], s);
}

TileCfg choose_tile(dr_geom g, const void* img, const void* out)
{
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->weighted) return TileCfg{1, 4, 16};  // the weighted kernel's one shape
    if ((g->forced || g->tuned) && tile_fits(g, g->tile, img, out)) return g->tile;
    return default_tile(g, img, out);
}

static dr_status ensure_scratch(dr_geom g, const TileCfg& t, float** part)
{
    std::lock_guard<std::mutex> lk(g->mu);
    const size_t need = (size_t)g->passes * partial_slots(g, t) * g->n_bins * sizeof(float);
    DR_HIP(g->part32.reserve(need));
    DR_HIP(g->work.reserve((size_t)kTotalsWorkRows * g->n_bins * sizeof(double)));
    *part = g->part32.as<float>();
    return DR_OK;
}

size_t partials_bytes(const dr_geom g, const TileCfg& t)
{
    const size_t b = (size_t)g->passes * partial_slots(g, t) * g->n_bins * sizeof(float);
    return (b + 255) & ~(size_t)255;
}

size_t totals_work_bytes(const dr_geom g)
{
    return (size_t)kTotalsWorkRows * g->n_bins * sizeof(double);
}

dr_status reconstruct_device_into(dr_geom g, const TileCfg& t, const uint16_t* images, float* out,
                                  float* totals, float* part, double* work, hipStream_t s)
{
    if (g->timing) DR_HIP(hipEventRecord(g->ev[0], s));
    for (int p = 0; p < g->passes; ++p) {
        ScanArgs a = scan_args(g, t, p, images, (int64_t)g->nx * g->ny, 0, 0, g->ny, out,
                               totals ? part : nullptr);
        DR_HIP(launch_scan_f32(g, t, p, a, s));
    }
    if (g->timing) DR_HIP(hipEventRecord(g->ev[1], s));
    if (totals) DR_HIP(enqueue_totals(g, part, partial_slots(g, t), work, totals, s));
    if (g->timing) {
        DR_HIP(hipEventRecord(g->ev[2], s));
        g->timed = true;
    }
    return DR_OK;
}

// ------------------------------------------------------------- tune cache

static std::string size_class(const dr_ctx c, const char* kind, int nx, int64_t pixels, int n,
                              int b)
{
    auto p2 = [](int64_t x) {
        int64_t r = 1;
        while (r < x) r <<= 1;
        return r;
    };
    std::ostringstream os;
    os << c->arch << "|" << kind << "|nx=" << nx << "|px=" << p2(pixels) << "|N=" << p2(n)
       << "|B=" << p2(b);
    return os.str();
}

static void load_tune_file(dr_ctx c)
{
    if (c->tune_file.empty()) return;
    std::ifstream f(c->tune_file);
    if (!f) return;
    std::string line;
    // one entry per line: "key": [ppl, waves, prefetch, gpc],
    while (std::getline(f, line)) {
        size_t q0 = line.find('"');
        size_t q1 = line.find('"', q0 + 1);
        size_t b0 = line.find('[', q1);
        if (q0 == std::string::npos || q1 == std::string::npos || b0 == std::string::npos)
            continue;
        TileCfg t{0, 0, 0};
        int gpc = 0;
        if (sscanf(line.c_str() + b0, "[%d, %d, %d, %d]", &t.ppl, &t.waves, &t.prefetch, &gpc) >= 3
            && tile_supported(t))
            c->tune_cache[line.substr(q0 + 1, q1 - q0 - 1)] = t;
    }
}

static void save_tune_file(dr_ctx c)
{
    if (c->tune_file.empty()) return;
    std::ofstream f(c->tune_file + ".tmp");
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (auto& kv : c->tune_cache) {
        f << "  \"" << kv.first << "\": [" << kv.second.ppl << ", " << kv.second.waves << ", "
          << kv.second.prefetch << ", 0]" << (++i < c->tune_cache.size() ? "," : "") << "\n";
    }
    f << "}\n";
    f.close();
    std::rename((c->tune_file + ".tmp").c_str(), c->tune_file.c_str());
}

}  // namespace dr

using namespace dr;

// ================================================================== C ABI

extern "C" {

const char* dr_last_error(void) { return g_last_error.c_str(); }

dr_status dr_ctx_create(int device, size_t hbm_budget_bytes, dr_ctx* out)
{
    if (!out) return set_error(DR_E_INVAL, "dr_ctx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    DR_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return set_error(DR_E_INVAL, "dr_ctx_create: bad device");
    DR_HIP(hipSetDevice(device));
    auto c = std::make_unique<dr_ctx_s>();
    c->device = device;
    hipDeviceProp_t prop;
    DR_HIP(hipGetDeviceProperties(&prop, device));
    c->arch = prop.gcnArchName;
    size_t colon = c->arch.find(':');
    if (colon != std::string::npos) c->arch = c->arch.substr(0, colon);
    c->cus = prop.multiProcessorCount;
    size_t free_b = 0, total_b = 0;
    DR_HIP(hipMemGetInfo(&free_b, &total_b));
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
    DR_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    DR_HIP(hipStreamCreateWithFlags(&c->copy, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
        DR_HIP(hipEventCreateWithFlags(&c->slab_ready[i], hipEventDisableTiming));
        DR_HIP(hipEventCreateWithFlags(&c->slab_free[i], hipEventDisableTiming));
    }
    {
        const dr_status st = noalloc_scratch_init(device);
        if (st != DR_OK) return st;
    }
    if (const char* f = std::getenv("DR_TUNE_CACHE")) c->tune_file = f;
    load_tune_file(c.get());
    *out = c.release();
    return ok();
}

dr_status dr_ctx_destroy(dr_ctx c)
{
    if (!c) return set_error(DR_E_INVAL, "dr_ctx_destroy: NULL context");
    if (c->sched) {
        destroy_scheduler(c->sched);
        c->sched = nullptr;
    }
    if (c->live_geoms.load() != 0 || c->live_batches.load() != 0)
        return set_error(DR_E_BUSY, "dr_ctx_destroy: geometries or batches still alive");
    DR_HIP(hipSetDevice(c->device));
    DR_HIP(hipDeviceSynchronize());
    for (int i = 0; i < 2; ++i) {
        c->slab[i].release();
        (void)hipEventDestroy(c->slab_ready[i]);
        (void)hipEventDestroy(c->slab_free[i]);
    }
    (void)hipStreamDestroy(c->stream);
    (void)hipStreamDestroy(c->copy);
    delete c;
    return ok();
}

dr_status dr_geometry_init(dr_ctx c, const dr_detector* det, const dr_wire* wire,
                           const dr_depth_grid* grid, dr_geom* out)
{
    if (!c || !det || !wire || !grid || !out)
        return set_error(DR_E_INVAL, "dr_geometry_init: NULL argument");
    *out = nullptr;
    if (det->nx < 1 || det->ny < 1) return set_error(DR_E_INVAL, "detector nx, ny must be >= 1");
    if ((int64_t)det->nx * det->ny >= ((int64_t)1 << 32))
        return set_error(DR_E_INVAL, "detector nx * ny must be below 2^32");
    if (wire->n_steps < 2 || !wire->centers)
        return set_error(DR_E_INVAL, "wire needs n_steps >= 2 and centers");
    if (grid->n_bins < 1) return set_error(DR_E_INVAL, "depth grid needs n_bins >= 1");
    if (grid->n_bins > (1 << 30)) return set_error(DR_E_INVAL, "depth grid needs n_bins <= 2^30");
    if (!(wire->radius > 0.0) || !std::isfinite(wire->radius))
        return set_error(DR_E_INVAL, "wire radius must be > 0");
    if (!(grid->width > 0.0) || !std::isfinite(grid->width) || !std::isfinite(grid->first_center))
        return set_error(DR_E_INVAL, "depth grid width must be > 0 and finite");
    if (!finite3(det->origin) || !finite3(det->u) || !finite3(det->v))
        return set_error(DR_E_INVAL, "detector origin/u/v must be finite");
    if (!finite3(wire->axis)) return set_error(DR_E_INVAL, "wire axis must be finite");
    if (wire->edge != DR_EDGE_LEADING && wire->edge != DR_EDGE_TRAILING &&
        wire->edge != DR_EDGE_BOTH)
        return set_error(DR_E_INVAL, "wire edge must be DR_EDGE_LEADING, _TRAILING or _BOTH");
    const int nx = det->nx, ny = det->ny, N = wire->n_steps, B = grid->n_bins;
    if ((int64_t)nx * ny > (int64_t)1 << 31)
        return set_error(DR_E_INVAL, "detector larger than 2^31 pixels");
    for (int k = 0; k < N; ++k)
        if (!finite3(wire->centers + 3 * k))
            return set_error(DR_E_INVAL, "wire centers must be finite");
    if (det->pixel_xyz)
        for (int64_t p = 0; p < (int64_t)nx * ny; ++p)
            if (!finite3(det->pixel_xyz + 3 * p))
                return set_error(DR_E_INVAL, "pixel_xyz must be finite");

    DR_HIP(hipSetDevice(c->device));
    auto g = std::make_unique<dr_geom_s>();
    g->ctx = c;
    g->nx = nx;
    g->ny = ny;
    g->n_steps = N;
    g->n_bins = B;
    g->radius = wire->radius;
    g->first_center = grid->first_center;
    g->width = grid->width;
    g->edge = wire->edge;
    g->passes = wire->edge == DR_EDGE_BOTH ? 2 : 1;
    for (int p = 0; p < g->passes; ++p) {
        // leading: side s_p, fractions as they are; trailing: side -s_p,
        // fractions negated (I_{k+1} - I_k); both: leading then trailing at 1/2
        g->side[p] = 0;
        g->scale[p] = 1.0;
        if (g->edge == DR_EDGE_TRAILING) {
            g->side[p] = 1;
            g->scale[p] = -1.0;
        } else if (g->edge == DR_EDGE_BOTH) {
            g->side[p] = p;
            g->scale[p] = p == 0 ? 0.5 : -0.5;
        }
    }

    // wire: raw centres [N][3], then the projected (eta, xi) [N + 2][2] (the
    // last position repeated twice, so that kernels reading one or two steps
    // ahead need no clamp); pixel centres [ny][nx][3] when given explicitly;
    // one status word and one row-uniformity flag per row
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t w_raw = 0, w_yz = up((size_t)N * 3 * 8),
                 w_st = w_yz + up((size_t)(N + 2) * 2 * 8),
                 w_fl = w_st + 256, w_total = w_fl + up((size_t)ny * 4);
    DR_HIP(g->wire.reserve(w_total));
    char* wb = g->wire.as<char>();
    double* d_wraw = (double*)(wb + w_raw);
    double* d_wyz = (double*)(wb + w_yz);
    int* d_status = (int*)(wb + w_st);
    int* d_flags = (int*)(wb + w_fl);
    DR_HIP(hipMemcpyAsync(d_wraw, wire->centers, (size_t)N * 3 * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
    if (det->pixel_xyz) {
        DR_HIP(g->pix.reserve((size_t)nx * ny * 3 * sizeof(double)));
        DR_HIP(hipMemcpyAsync(g->pix.p, det->pixel_xyz, (size_t)nx * ny * 3 * sizeof(double),
                              hipMemcpyHostToDevice, c->stream));
    }
    DR_HIP(hipMemsetAsync(d_status, 0, sizeof(int), c->stream));
    DR_HIP(hipMemsetAsync(d_flags, 1, (size_t)ny * sizeof(int), c->stream));

    GeomArgs& ga = g->g;
    ga.nx = nx;
    ga.ny = ny;
    ga.n_steps = N;
    ga.n_bins = B;
    ga.radius = wire->radius;
    ga.first_center = grid->first_center;
    ga.width = grid->width;
    for (int i = 0; i < 3; ++i) {
        ga.axis[i] = wire->axis[i];
        ga.origin[i] = det->origin[i];
        ga.u[i] = det->u[i];
        ga.v[i] = det->v[i];
    }
    ga.wire_raw = d_wraw;
    ga.wire_yz = d_wyz;
    ga.pix_xyz = det->pixel_xyz ? g->pix.as<double>() : nullptr;
    DR_HIP(launch_project_wire(ga, d_wyz, d_status, c->stream));
    for (int k = N; k < N + 2; ++k)
        DR_HIP(hipMemcpyAsync(d_wyz + 2 * k, d_wyz + 2 * (N - 1), 2 * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    DR_HIP(launch_row_uniform(ga, d_flags, c->stream));
    int status = 0;
    std::vector<int> flags(ny);
    DR_HIP(hipMemcpyAsync(&status, d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    DR_HIP(hipMemcpyAsync(flags.data(), d_flags, (size_t)ny * sizeof(int),
                          hipMemcpyDeviceToHost, c->stream));
    DR_HIP(hipStreamSynchronize(c->stream));
    if (status & 4)
        return set_error(DR_E_INVAL, "wire axis is zero or along the beam");
    // Rows whose pixels all share one projected (eta, xi), bit for bit, take
    // the per-row plan tables; any other geometry takes the per-pixel path.
    bool row_mode = true;
    for (int j = 0; j < ny; ++j) row_mode = row_mode && flags[j] != 0;
    g->row_mode = row_mode;

    if (!row_mode) {
        int sides = 0;  // only the edge sides the passes use
        for (int p = 0; p < g->passes; ++p) sides |= 1 << g->side[p];
        // [0] the largest fast-position bound, [1] the shortest non-zero step,
        // [2] the largest fast-position error found
        unsigned long long* d_bounds = (unsigned long long*)(wb + w_st + 8);
        unsigned long long bounds[3] = {0, 0, 0};
        DR_HIP(hipMemsetAsync(d_bounds, 0, 3 * sizeof(unsigned long long), c->stream));
        // 0x7f in every byte: 1.4e306, above every step
        DR_HIP(hipMemsetAsync(d_bounds + 1, 0x7f, sizeof(unsigned long long), c->stream));
        DR_HIP(launch_validate_pixels(ga, sides, d_status, d_bounds, c->stream));
        DR_HIP(hipMemcpyAsync(&status, d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        DR_HIP(hipMemcpyAsync(bounds, d_bounds, sizeof(bounds), hipMemcpyDeviceToHost,
                              c->stream));
        DR_HIP(hipStreamSynchronize(c->stream));
        double bound = 1.0, min_step = 0.0;
        std::memcpy(&bound, &bounds[0], sizeof(bound));
        std::memcpy(&min_step, &bounds[1], sizeof(min_step));
        std::memcpy(&g->pos_max_error, &bounds[2], sizeof(double));
        // The margin is twice the largest bound (taken 2^9 above the errors
        // it models).  The check has also evaluated the fast form itself at
        // every pixel and step the kernel will evaluate, with the same
        // operations on the same inputs, so its largest error e is exact for
        // this geometry, not an estimate: e < margin / 2 makes every floor the
        // kernel takes from a fast position (one at least a margin away from
        // an integer) the exact position's floor.  A fraction (an overlap over
        // the step's length len, both ends within e) moves by at most
        // 4e / len; steps of at least 2^28 e keep that below 2^-26, far under
        // the FP32 accumulation's rounding.  Otherwise (a large bound, an
        // error not well inside it, or a step too short for it) every
        // position is evaluated exactly (margin 1).
        const double margin = 2.0 * bound, e = g->pos_max_error;
        ga.pos_margin = (std::isfinite(margin) && margin < 0x1p-12 && e < 0.5 * margin &&
                         min_step >= e * 0x1p28)
                            ? margin
                            : 1.0;
        if (status & 1)
            return set_error(DR_E_INVAL, "geometry gives a non-finite depth (pixel inside the "
                                         "wire or a ray parallel to the beam)");
        if (status & 2)
            return set_error(DR_E_INVAL,
                             "wire not strictly between the beam and the detector in y");
        if (status & 8)
            return set_error(DR_E_INVAL, "an edge position lies 2^30 bins or more from the "
                                         "grid's first bin (depth grid too fine for the sweep)");
        for (int i = 0; i < 3; ++i) DR_HIP(hipEventCreate(&g->ev[i]));
        c->live_geoms++;
        *out = g.release();
        return ok();
    }

    // plan tables per pass: bl, nb (int32), f0, fm, f1 (float), d0, dm, d1 (double),
    // class, side, touched-bin range
    const size_t ent = (size_t)ny * (N - 1);
    const size_t o_bl = 0, o_nb = o_bl + up(ent * 4), o_f0 = o_nb + up(ent * 4),
                 o_fm = o_f0 + up(ent * 4), o_f1 = o_fm + up(ent * 4), o_d0 = o_f1 + up(ent * 4),
                 o_dm = o_d0 + up(ent * 8), o_d1 = o_dm + up(ent * 8), o_cls = o_d1 + up(ent * 8),
                 o_sgn = o_cls + up(ny), o_lo = o_sgn + up(ny), o_hi = o_lo + up((size_t)ny * 4),
                 total = o_hi + up((size_t)ny * 4);
    for (int p = 0; p < g->passes; ++p) {
        DR_HIP(g->plan[p].reserve(total));
        char* base = g->plan[p].as<char>();
        PlanTables& t = g->t[p];
        t.bl = (int32_t*)(base + o_bl);
        t.nb = (int32_t*)(base + o_nb);
        t.f0 = (float*)(base + o_f0);
        t.fm = (float*)(base + o_fm);
        t.f1 = (float*)(base + o_f1);
        t.d0 = (double*)(base + o_d0);
        t.dm = (double*)(base + o_dm);
        t.d1 = (double*)(base + o_d1);
        t.row_class = (int8_t*)(base + o_cls);
        t.row_sign = (int8_t*)(base + o_sgn);
        t.row_lo = (int32_t*)(base + o_lo);
        t.row_hi = (int32_t*)(base + o_hi);
        DR_HIP(launch_build_plans(ga, t, g->side[p], g->scale[p], d_status, c->stream));
    }
    if (g->passes == 2)
        DR_HIP(launch_unify_classes(g->t[0].row_class, g->t[1].row_class, ny, c->stream));
    DR_HIP(hipMemcpyAsync(&status, d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    DR_HIP(hipStreamSynchronize(c->stream));
    if (status & 1)
        return set_error(DR_E_INVAL, "geometry gives a non-finite depth (pixel inside the wire "
                                     "or a ray parallel to the beam)");
    if (status & 2)
        return set_error(DR_E_INVAL, "wire not strictly between the beam and the detector in y");
    for (int i = 0; i < 3; ++i) DR_HIP(hipEventCreate(&g->ev[i]));
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->tune_cache.find(size_class(c, "rows", nx, (int64_t)nx * ny, N, B));
        if (it != c->tune_cache.end()) {
            g->tile = it->second;
            g->tuned = true;
        }
    }
    c->live_geoms++;
    *out = g.release();
    return ok();
}

dr_status dr_geometry_set_step_weights(dr_geom g, const double* weights)
{
    if (!g) return set_error(DR_E_INVAL, "dr_geometry_set_step_weights: NULL geometry");
    if (g->inflight.load() != 0)
        return set_error(DR_E_BUSY, "dr_geometry_set_step_weights: serving requests use it");
    if (g->batches.load() != 0)  // batches keep the launch plan they were built with
        return set_error(DR_E_BUSY, "dr_geometry_set_step_weights: a batch uses it");
    if (!weights) {
        g->weighted = false;
        return ok();
    }
    for (int k = 0; k < g->n_steps; ++k)
        if (!std::isfinite(weights[k]))
            return set_error(DR_E_INVAL, "dr_geometry_set_step_weights: weights must be finite");
    DR_HIP(hipSetDevice(g->ctx->device));
    DR_HIP(hipDeviceSynchronize());  // earlier launches may still read the old weights
    DR_HIP(g->wbuf.reserve((size_t)g->n_steps * sizeof(double)));
    DR_HIP(hipMemcpy(g->wbuf.p, weights, (size_t)g->n_steps * sizeof(double),
                     hipMemcpyHostToDevice));
    g->weighted = true;
    return ok();
}

dr_status dr_geometry_path(dr_geom g, int32_t* path)
{
    if (!g || !path) return set_error(DR_E_INVAL, "dr_geometry_path: NULL argument");
    *path = g->row_mode ? DR_PATH_ROWS : DR_PATH_PIXELS;
    return ok();
}

dr_status dr_geometry_position_margin(dr_geom g, double* margin, double* max_error)
{
    if (!g || !margin) return set_error(DR_E_INVAL, "dr_geometry_position_margin: NULL argument");
    *margin = g->row_mode ? 0.0 : g->g.pos_margin;
    if (max_error) *max_error = g->row_mode ? 0.0 : g->pos_max_error;
    return ok();
}

dr_status dr_geometry_free(dr_geom g)
{
    if (!g) return set_error(DR_E_INVAL, "dr_geometry_free: NULL geometry");
    if (g->inflight.load() != 0)
        return set_error(DR_E_BUSY, "dr_geometry_free: serving requests still use it");
    if (g->lists.load() != 0)
        return set_error(DR_E_BUSY, "dr_geometry_free: pixel lists still use it");
    if (g->batches.load() != 0)
        return set_error(DR_E_BUSY, "dr_geometry_free: batches still use it");
    DR_HIP(hipSetDevice(g->ctx->device));
    DR_HIP(hipDeviceSynchronize());
    for (int i = 0; i < 3; ++i)
        if (g->ev[i]) (void)hipEventDestroy(g->ev[i]);
    g->ctx->live_geoms--;
    delete g;
    return ok();
}

dr_status dr_set_tile(dr_geom g, const dr_tile_config* tile)
{
    if (!g) return set_error(DR_E_INVAL, "dr_set_tile: NULL geometry");
    if (!g->row_mode && tile)
        return set_error(DR_E_UNSUPPORTED, "dr_set_tile: a per-pixel geometry has one launch shape");
    std::lock_guard<std::mutex> lk(g->mu);
    if (!tile) {
        g->forced = false;
        return ok();
    }
    TileCfg t{tile->pixels_per_lane, tile->waves_per_group, tile->prefetch};
    if (!tile_supported(t) || g->nx % t.ppl != 0)
        return set_error(DR_E_INVAL, "dr_set_tile: unsupported launch shape for this geometry");
    g->tile = t;
    g->forced = true;
    return ok();
}

static dr_status reconstruct_device(dr_geom g, const TileCfg& t, const uint16_t* images,
                                    float* out, float* totals, hipStream_t s)
{
    float* part = nullptr;
    if (totals) {
        dr_status st = ensure_scratch(g, t, &part);
        if (st != DR_OK) return st;
    }
    return reconstruct_device_into(g, t, images, out, totals, part, g->work.as<double>(), s);
}

static int slab_rows(const dr_geom g)
{
    size_t target = (size_t)256 << 20;
    if (const char* e = std::getenv("DR_SLAB_MB")) target = (size_t)std::max(1, atoi(e)) << 20;
    const size_t row_bytes = (size_t)g->nx * g->n_steps * sizeof(uint16_t);
    int r = (int)std::max<size_t>(1, target / row_bytes);
    if (const char* e = std::getenv("DR_SLAB_ROWS")) r = std::max(1, atoi(e));
    return std::min(r, g->ny);
}

// Host images: row slabs of every step copied on the copy stream into two
// alternating buffers; the kernel of slab s overlaps the copy of slab s+1.
static dr_status reconstruct_streamed(dr_geom g, const TileCfg& t, const uint16_t* images,
                                      float* out, float* totals, hipStream_t s)
{
    dr_ctx c = g->ctx;
    float* part = nullptr;
    if (totals) {
        dr_status st = ensure_scratch(g, t, &part);
        if (st != DR_OK) return st;
    }
    const int R = slab_rows(g);
    const size_t slab_bytes = (size_t)R * g->nx * g->n_steps * sizeof(uint16_t);
    std::lock_guard<std::mutex> lk(c->mu);
    for (int i = 0; i < 2; ++i) {
        if (c->slab[i].bytes < slab_bytes) {
            DR_HIP(hipStreamSynchronize(c->copy));
            DR_HIP(hipStreamSynchronize(c->stream));
            DR_HIP(hipDeviceSynchronize());
            DR_HIP(c->slab[i].reserve(slab_bytes));
        }
    }
    const int64_t plane_in = (int64_t)g->nx * g->ny;
    int n = 0;
    for (int r0 = 0; r0 < g->ny; r0 += R, ++n) {
        const int rs = std::min(R, g->ny - r0);
        const int b = n & 1;
        DR_HIP(hipStreamWaitEvent(c->copy, c->slab_free[b], 0));
        DR_HIP(hipMemcpy2DAsync(c->slab[b].p, (size_t)R * g->nx * sizeof(uint16_t),
                                images + (int64_t)r0 * g->nx, (size_t)plane_in * sizeof(uint16_t),
                                (size_t)rs * g->nx * sizeof(uint16_t), (size_t)g->n_steps,
                                hipMemcpyHostToDevice, c->copy));
        DR_HIP(hipEventRecord(c->slab_ready[b], c->copy));
        DR_HIP(hipStreamWaitEvent(s, c->slab_ready[b], 0));
        if (g->timing && n == 0) DR_HIP(hipEventRecord(g->ev[0], s));
        for (int p = 0; p < g->passes; ++p) {
            ScanArgs a = scan_args(g, t, p, c->slab[b].as<uint16_t>(), (int64_t)R * g->nx, r0,
                                   r0, r0 + rs, out, part);
            DR_HIP(launch_scan_f32(g, t, p, a, s));
        }
        DR_HIP(hipEventRecord(c->slab_free[b], s));
    }
    if (g->timing) DR_HIP(hipEventRecord(g->ev[1], s));
    if (totals)
        DR_HIP(enqueue_totals(g, part, partial_slots(g, t), g->work.as<double>(), totals, s));
    if (g->timing) {
        DR_HIP(hipEventRecord(g->ev[2], s));
        g->timed = true;
    }
    return DR_OK;
}

dr_status dr_reconstruct(dr_geom g, const uint16_t* images, int images_on_device, float* out,
                         float* totals, void* stream)
{
    if (!g || !images || !out) return set_error(DR_E_INVAL, "dr_reconstruct: NULL argument");
    if (!aligned(out, 4) || (totals && !aligned(totals, 4)) || !aligned(images, 2))
        return set_error(DR_E_INVAL, "dr_reconstruct: misaligned buffer");
    DR_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = (hipStream_t)stream;  // NULL is the null stream
    if (images_on_device) {
        const TileCfg t = choose_tile(g, images, out);
        dr_status st = reconstruct_device(g, t, images, out, totals, s);
        return st == DR_OK ? ok() : st;
    }
    // slab buffers are our own allocations, aligned for every shape
    const TileCfg t = choose_tile(g, nullptr, out);
    dr_status st = reconstruct_streamed(g, t, images, out, totals, s);
    return st == DR_OK ? ok() : st;
}

dr_status dr_reconstruct_f64(dr_geom g, const uint16_t* images, double* out, double* totals,
                             void* stream)
{
    if (!g || !images || !out) return set_error(DR_E_INVAL, "dr_reconstruct_f64: NULL argument");
    if (!aligned(out, 8) || (totals && !aligned(totals, 8)) || !aligned(images, 2))
        return set_error(DR_E_INVAL, "dr_reconstruct_f64: misaligned buffer");
    DR_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = (hipStream_t)stream;  // NULL is the null stream
    const TileCfg t{1, 4, 4};
    // totals: per-wave partial rows on the row path; on the per-pixel path
    // the column sums of the finished output, in a fixed order
    double* part = nullptr;
    if (totals) {
        std::lock_guard<std::mutex> lk(g->mu);
        if (g->row_mode) {
            DR_HIP(g->part64.reserve((size_t)g->passes * partial_slots(g, t) * g->n_bins *
                                     sizeof(double)));
            part = g->part64.as<double>();
        }
        DR_HIP(g->work.reserve((size_t)kTotalsWorkRows * g->n_bins * sizeof(double)));
    }
    const int64_t slots = partial_slots(g, t);
    // two edges: each pass is a reconstruction of its own (halved fractions),
    // the second formed in a stream-ordered buffer of its own and then added
    // onto the first, so that out = L/2 + T/2
    const int64_t n_out = (int64_t)g->n_bins * g->nx * g->ny;
    double* second = nullptr;
    if (g->passes == 2)
        DR_HIP(hipMallocAsync((void**)&second, (size_t)n_out * sizeof(double), s));
    hipError_t e = hipSuccess;
    for (int p = 0; p < g->passes && e == hipSuccess; ++p) {
        ScanArgs a = scan_args(g, t, p, images, (int64_t)g->nx * g->ny, 0, 0, g->ny, nullptr,
                               nullptr);
        a.pass = 0;
        a.out = p == 0 ? (void*)out : (void*)second;
        a.partials = part ? part + (size_t)p * slots * g->n_bins : nullptr;
        e = g->row_mode ? launch_rows_f64(a, s)
                        : launch_pixels_f64(a, g->g, g->side[p], g->scale[p], s);
    }
    if (e == hipSuccess && second) e = launch_add_f64(out, second, n_out, s);
    if (second) {
        const hipError_t ef = hipFreeAsync(second, s);
        if (e == hipSuccess) e = ef;
    }
    DR_HIP(e);
    if (totals && g->row_mode)
        DR_HIP(launch_totals_f64(part, slots * g->passes, g->n_bins, g->work.as<double>(),
                                 kTotalsWorkRows, totals, s));
    else if (totals)
        DR_HIP(launch_plane_totals_f64(out, (int64_t)g->nx * g->ny, g->n_bins,
                                       g->work.as<double>(), kTotalsWorkRows, totals, s));
    return ok();
}

dr_status dr_debug_plan(dr_geom g, const int64_t* pixels, int32_t n, int32_t edge,
                        int32_t* bins_out, double* u_out)
{
    if (!g || (n > 0 && !pixels)) return set_error(DR_E_INVAL, "dr_debug_plan: NULL argument");
    if (n < 0) return set_error(DR_E_INVAL, "dr_debug_plan: n < 0");
    if (edge != DR_EDGE_LEADING && edge != DR_EDGE_TRAILING)
        return set_error(DR_E_INVAL, "dr_debug_plan: edge must be leading or trailing");
    if (n == 0) return ok();
    const int64_t np = (int64_t)g->nx * g->ny;
    for (int32_t i = 0; i < n; ++i)
        if (pixels[i] < 0 || pixels[i] >= np)
            return set_error(DR_E_INVAL, "dr_debug_plan: pixel index out of range");
    DR_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = g->ctx->stream;
    DevBuf dp, db, du;
    const size_t cnt = (size_t)n * g->n_steps;
    DR_HIP(dp.reserve((size_t)n * sizeof(int64_t)));
    if (bins_out) DR_HIP(db.reserve(cnt * sizeof(int32_t)));
    if (u_out) DR_HIP(du.reserve(cnt * sizeof(double)));
    DR_HIP(hipMemcpyAsync(dp.p, pixels, (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    DR_HIP(launch_debug_plan(g->g, dp.as<int64_t>(), n, edge == DR_EDGE_TRAILING ? 1 : 0,
                             db.as<int32_t>(), du.as<double>(), s));
    if (bins_out)
        DR_HIP(hipMemcpyAsync(bins_out, db.p, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (u_out) DR_HIP(hipMemcpyAsync(u_out, du.p, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    DR_HIP(hipStreamSynchronize(s));
    return ok();
}

dr_status dr_enable_timing(dr_geom g, int enable)
{
    if (!g) return set_error(DR_E_INVAL, "dr_enable_timing: NULL geometry");
    g->timing = enable != 0;
    g->timed = false;
    return ok();
}

dr_status dr_last_timing(dr_geom g, double* kernel_ms, double* totals_ms)
{
    if (!g) return set_error(DR_E_INVAL, "dr_last_timing: NULL geometry");
    if (!g->timed) return set_error(DR_E_INVAL, "dr_last_timing: no timed launch yet");
    DR_HIP(hipEventSynchronize(g->ev[2]));
    float a = 0.f, b = 0.f;
    DR_HIP(hipEventElapsedTime(&a, g->ev[0], g->ev[1]));
    DR_HIP(hipEventElapsedTime(&b, g->ev[1], g->ev[2]));
    if (kernel_ms) *kernel_ms = a;
    if (totals_ms) *totals_ms = b;
    return ok();
}

dr_status dr_autotune(dr_geom g, const uint16_t* images, float* out, dr_tile_config* chosen)
{
    if (!g || !images || !out) return set_error(DR_E_INVAL, "dr_autotune: NULL argument");
    if (!g->row_mode) {  // one launch shape: a pixel per lane, four waves, prefetch 8
        if (chosen) *chosen = dr_tile_config{1, kPixelTile / 64, 8, 0};
        return ok();
    }
    if (g->weighted) {  // one launch shape with step weights
        if (chosen) *chosen = dr_tile_config{1, 4, 16, 0};
        return ok();
    }
    dr_ctx c = g->ctx;
    DR_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    hipEvent_t e0, e1;
    DR_HIP(hipEventCreate(&e0));
    DR_HIP(hipEventCreate(&e1));
    // totals are part of every call that asks for them; tune with them on
    DevBuf tot;
    DR_HIP(tot.reserve((size_t)g->n_bins * sizeof(float)));
    // every fitting shape, timed (median of 5); among shapes within 1% of the
    // fastest the earliest in the preference order wins, so that the choice
    // does not follow run-to-run noise
    std::vector<std::pair<TileCfg, float>> timed;
    const bool was_timing = g->timing;
    g->timing = false;
    for (int i = 0; i < num_tile_variants(); ++i) {
        const TileCfg t = tile_variant(i);
        if (!tile_fits(g, t, images, out)) continue;
        dr_status st = reconstruct_device(g, t, images, out, tot.as<float>(), s);  // warm-up
        if (st != DR_OK) return st;
        float ms[5];
        for (int r = 0; r < 5; ++r) {
            DR_HIP(hipEventRecord(e0, s));
            st = reconstruct_device(g, t, images, out, tot.as<float>(), s);
            if (st != DR_OK) return st;
            DR_HIP(hipEventRecord(e1, s));
            DR_HIP(hipEventSynchronize(e1));
            DR_HIP(hipEventElapsedTime(&ms[r], e0, e1));
        }
        std::sort(ms, ms + 5);
        timed.push_back({t, ms[2]});
    }
    TileCfg best_t = default_tile(g, images, out);
    float best = 1e30f;
    for (auto& c : timed) best = std::min(best, c.second);
    auto rank = [](const TileCfg& t) {
        static const TileCfg order[] = {{2, 4, 16}, {2, 4, 8}, {2, 4, 4}, {1, 4, 16}, {4, 2, 8}};
        for (int i = 0; i < 5; ++i)
            if (order[i].ppl == t.ppl && order[i].waves == t.waves && order[i].prefetch == t.prefetch)
                return i;
        return 100;
    };
    int best_rank = 1 << 30;
    for (auto& c : timed)
        if (c.second <= best * 1.01f) {
            const int r = rank(c.first) * 1000 + (int)(c.second * 1000.0f / best);
            if (r < best_rank) {
                best_rank = r;
                best_t = c.first;
            }
        }
    g->timing = was_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> lk(g->mu);
        g->tile = best_t;
        g->tuned = true;
    }
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->tune_cache[size_class(c, "rows", g->nx, (int64_t)g->nx * g->ny, g->n_steps,
                                 g->n_bins)] = best_t;
        save_tune_file(c);
    }
    if (chosen) *chosen = dr_tile_config{best_t.ppl, best_t.waves, best_t.prefetch, 0};
    return ok();
}

// ----------------------------------------------------------------- batches

static dr_status batch_build_args(dr_batch b, const TileCfg& t, int gpc)
{
    dr_ctx c = b->ctx;
    const int n = (int)b->items.size();
    // work order: most expensive tiles first (longest-processing-time rule);
    // a tile's cost is its pixels times (steps read + bins written)
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const dr_geom gx = b->geoms[x], gy = b->geoms[y];
        const int64_t cx = (int64_t)std::min(tile_width(t), gx->nx) * (gx->n_steps + gx->n_bins);
        const int64_t cy = (int64_t)std::min(tile_width(t), gy->nx) * (gy->n_steps + gy->n_bins);
        return cx > cy;
    });
    b->part_off.assign(n, 0);
    b->slots.assign(n, 0);
    int64_t poff = 0;
    for (int i = 0; i < n; ++i) {
        const TileCfg ti = batch_solo(b->geoms[i]) ? solo_tile(b->geoms[i]) : t;
        b->slots[i] = b->items[i].totals ? partial_slots(b->geoms[i], ti) : 0;  // per pass
        b->part_off[i] = poff;
        poff += b->slots[i] * b->geoms[i]->passes * b->geoms[i]->n_bins;
    }
    DR_HIP(b->parts.reserve(std::max<size_t>(4, (size_t)poff * sizeof(float))));
    int maxB = 1;
    for (int i = 0; i < n; ++i) maxB = std::max(maxB, b->geoms[i]->n_bins);
    b->max_bins = maxB;
    DR_HIP(b->work.reserve((size_t)n * kTotalsWorkRows * maxB * sizeof(double)));
    // first launch: every scan's first (or only) pass; second launch: the
    // second passes of two-edge scans, which add onto the first launch's output
    std::vector<ScanArgs> args;
    std::vector<int64_t> start1(1, 0), start2(1, 0);
    for (int pass = 0; pass < 2; ++pass) {
        for (int w = 0; w < n; ++w) {
            const int i = order[w];
            const dr_geom g = b->geoms[i];
            if (pass >= g->passes || batch_solo(g)) continue;
            float* part = b->items[i].totals ? b->parts.as<float>() + b->part_off[i] : nullptr;
            ScanArgs a = scan_args(g, t, pass, b->items[i].images, (int64_t)g->nx * g->ny, 0, 0,
                                   g->ny, b->items[i].out, part);
            args.push_back(a);
            std::vector<int64_t>& st = pass == 0 ? start1 : start2;
            st.push_back(st.back() + (int64_t)g->ny * a.tiles_per_row);
        }
    }
    b->n_args1 = (int)start1.size() - 1;
    b->n_args2 = (int)start2.size() - 1;
    // per-pixel and weighted scans: their own launches after the persistent ones
    b->solos.clear();
    for (int i = 0; i < n; ++i) {
        const dr_geom g = b->geoms[i];
        if (!batch_solo(g)) continue;
        float* part = b->items[i].totals ? b->parts.as<float>() + b->part_off[i] : nullptr;
        for (int pass = 0; pass < g->passes; ++pass)
            b->solos.push_back({i, pass, scan_args(g, solo_tile(g), pass, b->items[i].images,
                                                   (int64_t)g->nx * g->ny, 0, 0, g->ny,
                                                   b->items[i].out, part)});
    }
    // the totals of every scan in two launches after the scans
    std::vector<TotalsJob> jobs;
    int blocks1 = 0, blocks2 = 0;
    for (int i = 0; i < n; ++i) {
        if (!b->items[i].totals) continue;
        const dr_geom g = b->geoms[i];
        TotalsJob j{};
        j.parts = b->parts.as<float>() + b->part_off[i];
        j.slots = b->slots[i] * g->passes;
        j.n_bins = g->n_bins;
        j.first1 = blocks1;
        j.first2 = blocks2;
        j.work = b->work.as<double>() + (size_t)i * kTotalsWorkRows * b->max_bins;
        j.totals = b->items[i].totals;
        blocks1 += (g->n_bins + 63) / 64;
        blocks2 += (g->n_bins + 255) / 256;
        jobs.push_back(j);
    }
    b->n_jobs = (int)jobs.size();
    b->jblocks1 = blocks1;
    b->jblocks2 = blocks2;
    if (!jobs.empty()) {
        DR_HIP(b->tjobs.reserve(sizeof(TotalsJob) * jobs.size()));
        DR_HIP(hipMemcpy(b->tjobs.p, jobs.data(), sizeof(TotalsJob) * jobs.size(),
                         hipMemcpyHostToDevice));
    }
    std::vector<int64_t> starts(start1);
    starts.insert(starts.end(), start2.begin(), start2.end());
    DR_HIP(b->scans.reserve(sizeof(ScanArgs) * args.size()));
    DR_HIP(b->starts.reserve(sizeof(int64_t) * starts.size()));
    DR_HIP(b->counter.reserve(2 * sizeof(unsigned long long)));
    DR_HIP(hipMemcpy(b->scans.p, args.data(), sizeof(ScanArgs) * args.size(),
                     hipMemcpyHostToDevice));
    DR_HIP(hipMemcpy(b->starts.p, starts.data(), sizeof(int64_t) * starts.size(),
                     hipMemcpyHostToDevice));
    b->total_tiles = start1.back();
    b->total_tiles2 = start2.back();
    b->tile = t;
    b->gpc = gpc;
    // gpc == 0: one workgroup per tile (no persistent loop)
    b->groups = gpc == 0 ? (int)std::min<int64_t>(b->total_tiles, INT32_MAX)
                         : (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)c->cus * gpc,
                                                                       b->total_tiles));
    return DR_OK;
}

static dr_status batch_enqueue(dr_batch b, hipStream_t s)
{
    for (int launch = 0; launch < 2; ++launch) {
        const int na = launch == 0 ? b->n_args1 : b->n_args2;
        if (na == 0) continue;
        BatchArgs ba{};
        ba.scans = b->scans.as<ScanArgs>() + (launch == 0 ? 0 : b->n_args1);
        ba.tile_start = b->starts.as<int64_t>() + (launch == 0 ? 0 : b->n_args1 + 1);
        ba.n_scans = na;
        ba.total_tiles = launch == 0 ? b->total_tiles : b->total_tiles2;
        ba.counter = b->counter.as<unsigned long long>() + launch;
        const int64_t groups =
            b->gpc == 0 ? ba.total_tiles
                        : std::max<int64_t>(1, std::min<int64_t>((int64_t)b->ctx->cus * b->gpc,
                                                                 ba.total_tiles));
        DR_HIP(launch_reset_counter(ba.counter, s));
        DR_HIP(launch_batch_f32(b->tile, ba, launch == 1,
                                (int)std::min<int64_t>(groups, INT32_MAX), s));
    }
    for (const BatchSolo& so : b->solos) {
        const dr_geom g = b->geoms[so.item];
        DR_HIP(launch_scan_f32(g, solo_tile(g), so.pass, so.args, s));
    }
    DR_HIP(launch_totals_multi_f32(b->tjobs.as<TotalsJob>(), b->n_jobs, b->jblocks1,
                                   b->jblocks2, s));
    return DR_OK;
}

dr_status dr_batch_create(dr_ctx c, int32_t n, const dr_batch_item* items, int32_t flags,
                          dr_batch* out)
{
    if (!c || !items || !out || n < 1) return set_error(DR_E_INVAL, "dr_batch_create: bad argument");
    *out = nullptr;
    auto b = std::make_unique<dr_batch_s>();
    b->ctx = c;
    for (int i = 0; i < n; ++i) {
        const dr_batch_item& it = items[i];
        if (!it.geom || !it.images || !it.out)
            return set_error(DR_E_INVAL, "dr_batch_create: NULL item field");
        if (it.geom->ctx != c)
            return set_error(DR_E_INVAL, "dr_batch_create: geometry of another context");
        b->items.push_back(it);
        b->geoms.push_back(it.geom);
        it.geom->batches++;  // given back when the batch is deleted
    }
    DR_HIP(hipSetDevice(c->device));
    // launch shapes valid for every scan
    std::vector<TileCfg> cands;
    for (int v = 0; v < num_tile_variants(); ++v) {
        const TileCfg t = tile_variant(v);
        bool okall = true;
        for (int i = 0; i < n && okall; ++i)  // scans launched on their own take any
            okall = batch_solo(b->geoms[i]) || tile_fits(b->geoms[i], t, items[i].images,
                                                         items[i].out);
        if (okall) cands.push_back(t);
    }
    if (cands.empty()) return set_error(DR_E_INVAL, "dr_batch_create: no launch shape fits");
    TileCfg t = cands.back();
    for (const TileCfg& x : cands)
        if (x.ppl == 2 && x.waves == 4 && x.prefetch == 16) t = x;
    int gpc = 8;  // persistent workgroups per CU (2048 threads of 4-wave groups)
    hipStream_t s = c->stream;
    if (flags & DR_BATCH_AUTOTUNE) {
        hipEvent_t e0, e1;
        DR_HIP(hipEventCreate(&e0));
        DR_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        TileCfg bt = t;
        int bg = gpc;
        for (const TileCfg& x : cands) {
            for (int g : {0, 1, 2, 4, 8}) {
                if (64 * x.waves * g > 2048) continue;  // CU thread limit
                dr_status st = batch_build_args(b.get(), x, g);
                if (st != DR_OK) return st;
                st = batch_enqueue(b.get(), s);  // warm-up
                if (st != DR_OK) return st;
                float ms[3];
                for (int r = 0; r < 3; ++r) {
                    DR_HIP(hipEventRecord(e0, s));
                    st = batch_enqueue(b.get(), s);
                    if (st != DR_OK) return st;
                    DR_HIP(hipEventRecord(e1, s));
                    DR_HIP(hipEventSynchronize(e1));
                    DR_HIP(hipEventElapsedTime(&ms[r], e0, e1));
                }
                std::sort(ms, ms + 3);
                if (ms[1] < best) {
                    best = ms[1];
                    bt = x;
                    bg = g;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        t = bt;
        gpc = bg;
    }
    dr_status st = batch_build_args(b.get(), t, gpc);
    if (st != DR_OK) return st;
    if (flags & DR_BATCH_GRAPH) {
        hipStream_t cs;
        DR_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        DR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        st = batch_enqueue(b.get(), cs);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &graph);
        (void)hipStreamDestroy(cs);
        if (st != DR_OK) return st;
        if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
        b->graph = graph;
        DR_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    DR_HIP(hipStreamSynchronize(s));
    c->live_batches++;
    *out = b.release();
    return ok();
}

dr_status dr_batch_run(dr_batch b, void* stream)
{
    if (!b) return set_error(DR_E_INVAL, "dr_batch_run: NULL batch");
    DR_HIP(hipSetDevice(b->ctx->device));
    hipStream_t s = (hipStream_t)stream;  // NULL is the null stream
    if (b->exec) {
        DR_HIP(hipGraphLaunch(b->exec, s));
        return ok();
    }
    dr_status st = batch_enqueue(b, s);
    return st == DR_OK ? ok() : st;
}

dr_status dr_batch_tile(dr_batch b, dr_tile_config* tile)
{
    if (!b || !tile) return set_error(DR_E_INVAL, "dr_batch_tile: NULL argument");
    *tile = dr_tile_config{b->tile.ppl, b->tile.waves, b->tile.prefetch, b->gpc};
    return ok();
}

dr_status dr_batch_free(dr_batch b)
{
    if (!b) return set_error(DR_E_INVAL, "dr_batch_free: NULL batch");
    DR_HIP(hipSetDevice(b->ctx->device));
    DR_HIP(hipDeviceSynchronize());
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->ctx->live_batches--;
    delete b;
    return ok();
}

}  // extern "C"
