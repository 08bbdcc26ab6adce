// Host-side objects behind the C ABI (not public).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "dr.h"
#include "dr_internal.h"

namespace dr {

struct Scheduler;  // dr_serve.cpp

dr_status set_error(dr_status code, const std::string& msg);
dr_status hip_error(hipError_t e, const char* what);

#define DR_HIP(call)                                                    \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::dr::hip_error(_e, #call);        \
    } while (0)

// Device allocation owned by a host object.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow to at least n bytes (contents are not kept)
    hipError_t reserve(size_t n)
    {
        if (n <= bytes) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = n;
        return hipSuccess;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace dr

struct dr_ctx_s {
    int device = 0;
    std::string arch;
    int cus = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;  // compute stream (default priority)
    hipStream_t copy = nullptr;    // host-to-device copies
    std::mutex mu;                 // guards the slab buffers and the tune cache
    dr::DevBuf slab[2];
    hipEvent_t slab_ready[2] = {nullptr, nullptr};
    hipEvent_t slab_free[2] = {nullptr, nullptr};
    std::map<std::string, dr::TileCfg> tune_cache;
    std::string tune_file;
    std::atomic<int> live_geoms{0};
    std::atomic<int> live_batches{0};
    dr::Scheduler* sched = nullptr;  // created on the first dr_submit
};

struct dr_geom_s {
    dr_ctx ctx = nullptr;
    int nx = 0, ny = 0, n_steps = 0, n_bins = 0;
    double radius = 0, first_center = 0, width = 0;
    bool row_mode = true;
    int edge = DR_EDGE_LEADING;
    int passes = 1;  // 2 for DR_EDGE_BOTH: leading, then trailing added on
    int side[2] = {0, 0};         // per pass: 0 leading side s_p, 1 trailing side -s_p
    double scale[2] = {1.0, 1.0};  // per pass: factor on every fraction
    dr::GeomArgs g{};
    // per-pixel path: the largest distance between fast and exact positions
    // found at init, over every pixel and step of the passes' sides (bins)
    double pos_max_error = 0.0;
    dr::PlanTables t[2]{};
    // wire: raw and projected centres, status and row flags; pix: explicit
    // pixel centres; plan[p]: all plan tables of pass p in one allocation
    dr::DevBuf wire, pix, plan[2];
    dr::DevBuf part32, part64, work;
    dr::DevBuf sel;  // dr_select_top's state and block sums, kept between calls
    std::mutex mu;
    bool forced = false, tuned = false;
    dr::TileCfg tile{0, 0, 0};
    bool timing = false, timed = false;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    std::atomic<int> inflight{0};  // serving requests using this geometry
    std::atomic<int> lists{0};     // pixel lists built on this geometry
    std::atomic<int> batches{0};   // batch items that use this geometry
    bool weighted = false;         // per-step sample weights set (wbuf holds them)
    dr::DevBuf wbuf;
};

struct BatchSolo {  // one pass of a scan that the persistent kernel does not take
    int item, pass;
    dr::ScanArgs args;
};

struct dr_batch_s {
    ~dr_batch_s()
    {
        for (dr_geom g : geoms) g->batches--;
    }
    dr_ctx ctx = nullptr;
    std::vector<dr_batch_item> items;
    std::vector<dr_geom> geoms;
    dr::TileCfg tile{0, 0, 0};
    int groups = 0;
    int gpc = 0;
    int max_bins = 1;
    dr::DevBuf scans, starts, counter, parts, work;
    dr::DevBuf tjobs;               // TotalsJob per scan with totals
    int n_jobs = 0, jblocks1 = 0, jblocks2 = 0;
    int64_t total_tiles2 = 0;       // tiles of second passes (launched after the first)
    int n_args1 = 0, n_args2 = 0;   // ScanArgs entries of each launch
    std::vector<int64_t> part_off;  // per item offset into parts (floats)
    std::vector<int64_t> slots;     // per item partial slots (all passes)
    std::vector<BatchSolo> solos;   // per-pixel and weighted scans, launched on their own
    int64_t total_tiles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace dr {

// Shared helpers (dr_runtime.cpp) used by the scheduler.
bool tile_fits(const dr_geom g, const TileCfg& t, const void* img, const void* out);
TileCfg default_tile(const dr_geom g, const void* img, const void* out);
// partial-total rows of one pass; a geometry with two passes uses twice as many
int64_t partial_slots(const dr_geom g, const TileCfg& t);
// arguments of pass `pass` (0 or 1); partials points at the base of all passes'
// partial rows, the pass's own rows are selected here
ScanArgs scan_args(const dr_geom g, const TileCfg& t, int pass, const uint16_t* img,
                   int64_t img_step, int row_base, int row_begin, int row_end, float* out,
                   float* partials);
hipError_t enqueue_totals(const dr_geom g, const float* partials, int64_t slots, double* work,
                          float* totals, hipStream_t s);
// scans the persistent row-tile kernel does not take (per-pixel path, step
// weights) are launched on their own, with this launch shape
bool batch_solo(const dr_geom g);
TileCfg solo_tile(const dr_geom g);
// pass `pass` of any path (per-row plans, weighted rows, per-pixel)
hipError_t launch_scan_f32(const dr_geom g, const TileCfg& t, int pass, const ScanArgs& a,
                           hipStream_t s);

// launch shape dr_reconstruct uses for these buffers (forced, tuned or default)
TileCfg choose_tile(dr_geom g, const void* img, const void* out);
// scratch of a device-image reconstruction with totals: the partial-total rows
// of every pass (rounded up to 256 bytes), then the totals reduction workspace
size_t partials_bytes(const dr_geom g, const TileCfg& t);
size_t totals_work_bytes(const dr_geom g);
// every pass of a device-image reconstruction and its totals, with the
// caller's scratch (part and work are unused when totals is null)
dr_status reconstruct_device_into(dr_geom g, const TileCfg& t, const uint16_t* images, float* out,
                                  float* totals, float* part, double* work, hipStream_t s);

// fixed device scratch of dr_reconstruct_noalloc (dr_noalloc.hip): its size,
// the per-device address lookup (called with `device` current), and the bytes
// a reconstruction with this launch shape takes from it
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
dr_status noalloc_scratch_init(int device);
size_t noalloc_scratch_need(const dr_geom g, const TileCfg& t, bool totals);

Scheduler* make_scheduler(dr_ctx ctx);
void destroy_scheduler(Scheduler* s);

}  // namespace dr
