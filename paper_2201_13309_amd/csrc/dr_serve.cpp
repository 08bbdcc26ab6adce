// Serving: dr_submit / dr_poll / dr_wait.  The scheduling policy (admission
// by footprint, slab interleaving, epochs, failure handling) is the Core of
// dr_sched.cpp; this file is its executor on one GPU and the thread that
// drives it.
//
//   allocate   stream-ordered allocations: the staging copy of host images on
//              the copy stream (its first user), partial totals on the compute
//              stream;
//   copy       rows [r0, r0 + rows) of every step with one 2D copy on the copy
//              stream, then an event;
//   epoch      per pass and pixels-per-lane group, one persistent launch of
//              the batch kernel over the epoch's row segments (the same tile
//              code as dr_reconstruct); requests on the per-pixel path or with
//              step weights get launches of their own kernel; then the totals
//              of the finishing requests and an event on the compute stream;
//   release    stream-ordered frees once the core has seen every copy and
//              epoch of the request complete.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <thread>

#include "dr_runtime.h"
#include "dr_sched.h"

namespace dr {

namespace {

constexpr int kMaxSegs = sched::kMaxActive;  // segments per epoch and group
constexpr int kGroups = 6;                   // (pass 1 or 2) x (4, 2 or 1 pixels per lane)

// HIP state of one request
struct Work {
    dr_geom g = nullptr;
    const uint16_t* images = nullptr;  // caller's (host or device)
    bool on_device = false;
    float* out = nullptr;
    float* totals = nullptr;
    TileCfg tile{4, 4, 16};
    uint16_t* staged = nullptr;  // device copy of host images
    float* parts = nullptr;
    double* work = nullptr;
};

Work* work_of(sched::Req& r) { return static_cast<Work*>(r.user); }

size_t image_bytes(const dr_geom g) { return (size_t)g->nx * g->ny * g->n_steps * sizeof(uint16_t); }

size_t parts_bytes(const dr_geom g, const TileCfg& t)
{
    return (size_t)g->passes * partial_slots(g, t) * g->n_bins * sizeof(float);
}

struct EpochArgs {
    DevBuf args;  // ScanArgs[kGroups][kMaxSegs], starts[kGroups][kMaxSegs+1], counters[kGroups]
    ScanArgs* h_args = nullptr;  // pinned staging
    int64_t* h_starts = nullptr;
};

class HipExecutor : public sched::Executor {
public:
    explicit HipExecutor(dr_ctx c) : ctx_(c) {}
    ~HipExecutor() override
    {
        for (auto& es : slots_) {
            if (es.h_args) (void)hipHostFree(es.h_args);
            if (es.h_starts) (void)hipHostFree(es.h_starts);
        }
        for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
    }

    bool init()
    {
        for (auto& es : slots_) {
            const size_t bytes = sizeof(ScanArgs) * kGroups * kMaxSegs +
                                 sizeof(int64_t) * kGroups * (kMaxSegs + 1) +
                                 sizeof(unsigned long long) * kGroups;
            if (es.args.reserve(bytes) != hipSuccess ||
                hipHostMalloc((void**)&es.h_args, sizeof(ScanArgs) * kGroups * kMaxSegs, 0) !=
                    hipSuccess ||
                hipHostMalloc((void**)&es.h_starts, sizeof(int64_t) * kGroups * (kMaxSegs + 1),
                              0) != hipSuccess)
                return false;
        }
        return true;
    }

    uint64_t tiles_launched = 0;

    dr_status allocate(sched::Req& r) override
    {
        Work* w = work_of(r);
        hipError_t e = hipSuccess;
        if (!w->on_device) e = hipMallocAsync((void**)&w->staged, image_bytes(w->g), ctx_->copy);
        if (e == hipSuccess && w->totals) {
            e = hipMallocAsync((void**)&w->parts, parts_bytes(w->g, w->tile), ctx_->stream);
            if (e == hipSuccess)
                e = hipMallocAsync((void**)&w->work,
                                   (size_t)kTotalsWorkRows * w->g->n_bins * sizeof(double),
                                   ctx_->stream);
        }
        if (e != hipSuccess) {  // nothing stays allocated
            free_buffers(*w);
            return e == hipErrorOutOfMemory ? DR_E_NOMEM : DR_E_DEVICE;
        }
        return DR_OK;
    }

    dr_status copy_rows(sched::Req& r, int r0, int rows, sched::Event* ev) override
    {
        Work* w = work_of(r);
        const dr_geom g = w->g;
        const size_t plane = (size_t)g->nx * g->ny;
        hipEvent_t he = get_event();
        if (!he) return DR_E_DEVICE;
        // rows [r0, r0+rows) of every step, into the same place of the device copy
        hipError_t e = hipMemcpy2DAsync(w->staged + (size_t)r0 * g->nx, plane * 2,
                                        w->images + (size_t)r0 * g->nx, plane * 2,
                                        (size_t)rows * g->nx * 2, (size_t)g->n_steps,
                                        hipMemcpyHostToDevice, ctx_->copy);
        if (e == hipSuccess) e = hipEventRecord(he, ctx_->copy);
        if (e != hipSuccess) {
            put_event(he);
            // a copy already enqueued before the failure may still run
            (void)hipStreamSynchronize(ctx_->copy);
            return DR_E_DEVICE;
        }
        *ev = reinterpret_cast<sched::Event>(he);
        return DR_OK;
    }

    dr_status launch_epoch(int slot, const std::vector<sched::Segment>& segs,
                           const std::vector<sched::Req*>& finishing, sched::Event* ev) override
    {
        EpochArgs& es = slots_[slot];
        hipStream_t s = ctx_->stream;
        static const int kPpl[3] = {4, 2, 1};
        int nseg[kGroups] = {0, 0, 0, 0, 0, 0};
        int64_t tiles[kGroups] = {0, 0, 0, 0, 0, 0};
        std::vector<const sched::Segment*> solos;  // per-pixel and weighted requests
        for (const sched::Segment& sg : segs) {
            Work* w = work_of(*sg.r);
            if (batch_solo(w->g)) {
                solos.push_back(&sg);
                continue;
            }
            const int pi = w->tile.ppl == 4 ? 0 : (w->tile.ppl == 2 ? 1 : 2);
            const uint16_t* img = w->on_device ? w->images : w->staged;
            for (int p = 0; p < w->g->passes; ++p) {
                const int gi = p * 3 + pi;
                if (nseg[gi] >= kMaxSegs) return DR_E_DEVICE;  // cannot happen: one per request
                const ScanArgs a = scan_args(w->g, w->tile, p, img,
                                             (int64_t)w->g->nx * w->g->ny, 0, sg.row_begin,
                                             sg.row_end, w->out, w->parts);
                const int k = nseg[gi]++;
                es.h_args[gi * kMaxSegs + k] = a;
                int64_t* st = es.h_starts + gi * (kMaxSegs + 1);
                if (k == 0) st[0] = 0;
                st[k + 1] = st[k] + (int64_t)(sg.row_end - sg.row_begin) * a.tiles_per_row;
                tiles[gi] = st[k + 1];
            }
        }
        char* dbase = es.args.as<char>();
        ScanArgs* d_args = (ScanArgs*)dbase;
        int64_t* d_starts = (int64_t*)(dbase + sizeof(ScanArgs) * kGroups * kMaxSegs);
        unsigned long long* d_cnt =
            (unsigned long long*)(dbase + sizeof(ScanArgs) * kGroups * kMaxSegs +
                                  sizeof(int64_t) * kGroups * (kMaxSegs + 1));
        // the pinned staging of this slot was last read by an epoch that has
        // completed (the core reuses a slot only then)
        hipError_t e = hipMemcpyAsync(d_args, es.h_args, sizeof(ScanArgs) * kGroups * kMaxSegs,
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_starts, es.h_starts, sizeof(int64_t) * kGroups * (kMaxSegs + 1),
                               hipMemcpyHostToDevice, s);
        // rows are handed out only after the host has seen their copy event
        // complete, so the kernels below read finished copies
        for (int gi = 0; gi < kGroups && e == hipSuccess; ++gi) {
            if (!nseg[gi]) continue;
            BatchArgs ba{};
            ba.scans = d_args + gi * kMaxSegs;
            ba.tile_start = d_starts + gi * (kMaxSegs + 1);
            ba.n_scans = nseg[gi];
            ba.total_tiles = tiles[gi];
            ba.counter = d_cnt + gi;
            const TileCfg t{kPpl[gi % 3], 4, 16};
            // 8 persistent 4-wave workgroups per CU (2048 threads)
            const int groups =
                (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)ctx_->cus * 8, tiles[gi]));
            e = launch_reset_counter(ba.counter, s);
            // groups 3..5 hold second passes, which add onto the first
            if (e == hipSuccess) e = launch_batch_f32(t, ba, gi >= 3, groups, s);
            tiles_launched += (uint64_t)tiles[gi];
        }
        for (const sched::Segment* sg : solos) {
            Work* w = work_of(*sg->r);
            const uint16_t* img = w->on_device ? w->images : w->staged;
            for (int p = 0; p < w->g->passes && e == hipSuccess; ++p) {
                const ScanArgs a = scan_args(w->g, w->tile, p, img,
                                             (int64_t)w->g->nx * w->g->ny, 0, sg->row_begin,
                                             sg->row_end, w->out, w->parts);
                e = launch_scan_f32(w->g, w->tile, p, a, s);
                tiles_launched += (uint64_t)(sg->row_end - sg->row_begin) * a.tiles_per_row;
            }
        }
        for (sched::Req* r : finishing) {
            if (e != hipSuccess) break;
            Work* w = work_of(*r);
            if (w->totals)
                e = enqueue_totals(w->g, w->parts, partial_slots(w->g, w->tile), w->work,
                                   w->totals, s);
        }
        hipEvent_t he = nullptr;
        if (e == hipSuccess) {
            he = get_event();
            if (!he) e = hipErrorOutOfMemory;
        }
        if (e == hipSuccess) e = hipEventRecord(he, s);
        if (e != hipSuccess) {
            if (he) put_event(he);
            // what this call enqueued before the failure has finished
            (void)hipStreamSynchronize(s);
            return DR_E_DEVICE;
        }
        *ev = reinterpret_cast<sched::Event>(he);
        return DR_OK;
    }

    sched::Poll query(sched::Event ev) override
    {
        const hipError_t q = hipEventQuery(reinterpret_cast<hipEvent_t>(ev));
        if (q == hipErrorNotReady) return sched::kPending;
        return q == hipSuccess ? sched::kDone : sched::kFailed;
    }

    void forget(sched::Event ev) override { put_event(reinterpret_cast<hipEvent_t>(ev)); }

    void release(sched::Req& r) override { free_buffers(*work_of(r)); }

    void finished(sched::Req& r) override { work_of(r)->g->inflight--; }

private:
    // stream-ordered frees: the staging buffer on the copy stream, the partial
    // totals on the compute stream (each after its last user there)
    void free_buffers(Work& w)
    {
        if (w.staged) (void)hipFreeAsync(w.staged, ctx_->copy);
        if (w.parts) (void)hipFreeAsync(w.parts, ctx_->stream);
        if (w.work) (void)hipFreeAsync(w.work, ctx_->stream);
        w.staged = nullptr;
        w.parts = nullptr;
        w.work = nullptr;
    }
    hipEvent_t get_event()
    {
        if (!pool_.empty()) {
            hipEvent_t e = pool_.back();
            pool_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    void put_event(hipEvent_t e)
    {
        if (e) pool_.push_back(e);
    }

    dr_ctx ctx_;
    EpochArgs slots_[sched::kEpochSlots];
    std::vector<hipEvent_t> pool_;
};

}  // namespace

struct Scheduler {
    explicit Scheduler(dr_ctx c) : ctx(c), ex(c), core(ex, c->budget) {}
    dr_ctx ctx;
    HipExecutor ex;
    sched::Core core;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler thread
    std::condition_variable done_cv;  // wakes dr_wait
    bool stop = false;
    uint64_t next_id = 1;
    std::thread th;

    void run()
    {
        (void)hipSetDevice(ctx->device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            const uint64_t ended = core.counters().completed + core.counters().failed;
            const bool busy = core.step();
            if (core.counters().completed + core.counters().failed != ended)
                done_cv.notify_all();
            if (stop && core.idle()) break;
            if (busy)
                cv.wait_for(lk, std::chrono::microseconds(100));
            else
                cv.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
};

Scheduler* make_scheduler(dr_ctx ctx)
{
    auto* s = new Scheduler(ctx);
    if (!s->ex.init()) {
        delete s;
        return nullptr;
    }
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, ctx->device) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    s->th = std::thread([s] { s->run(); });
    return s;
}

void destroy_scheduler(Scheduler* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    (void)hipStreamSynchronize(s->ctx->stream);
    (void)hipStreamSynchronize(s->ctx->copy);
    // requests never collected by dr_poll / dr_wait
    for (;;) {
        sched::Req* r = nullptr;
        for (uint64_t id = 1; id < s->next_id && !r; ++id) r = s->core.take(id);
        if (!r) break;
        delete work_of(*r);
        delete r;
    }
    delete s;
}

}  // namespace dr

using namespace dr;

extern "C" {

dr_status dr_submit(dr_ctx c, dr_geom g, const uint16_t* images, int images_on_device,
                    float* out, float* totals, uint64_t* ticket)
{
    if (!c || !g || !images || !out || !ticket)
        return set_error(DR_E_INVAL, "dr_submit: NULL argument");
    if (g->ctx != c) return set_error(DR_E_INVAL, "dr_submit: geometry of another context");
    auto w = std::make_unique<Work>();
    w->g = g;
    w->images = images;
    w->on_device = images_on_device != 0;
    w->out = out;
    w->totals = totals;
    if (batch_solo(g)) {
        w->tile = solo_tile(g);
    } else {
        w->tile = default_tile(g, w->on_device ? (const void*)images : nullptr, out);
        w->tile.waves = 4;
        w->tile.prefetch = 16;
    }
    if (!tile_fits(g, w->tile, w->on_device ? (const void*)images : nullptr, out))
        return set_error(DR_E_INVAL, "dr_submit: misaligned buffer");
    auto r = std::make_unique<sched::Req>();
    r->ny = g->ny;
    r->row_bytes = (size_t)g->nx * g->n_steps * sizeof(uint16_t);
    r->on_device = w->on_device;
    // device bytes the request occupies while in flight: its images (the
    // caller's on the device, or the staging copy), its output, and the
    // partial totals with their reduction workspace
    r->footprint = image_bytes(g) + (size_t)g->n_bins * g->nx * g->ny * sizeof(float) +
                   (totals ? parts_bytes(g, w->tile) +
                                 (size_t)kTotalsWorkRows * g->n_bins * sizeof(double)
                           : 0);
    if (!c->sched) {
        std::lock_guard<std::mutex> lk(c->mu);
        if (!c->sched) c->sched = make_scheduler(c);
        if (!c->sched) return set_error(DR_E_DEVICE, "dr_submit: cannot start the scheduler");
    }
    Scheduler* s = c->sched;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id;
        r->user = w.get();
        const dr_status st = s->core.submit(r.get());
        if (st != DR_OK)
            return set_error(st, "dr_submit: request larger than the device-memory budget");
        s->next_id++;
        *ticket = r->id;
        g->inflight++;
        w.release();
        r.release();
    }
    s->cv.notify_all();
    return DR_OK;
}

static dr_status collect(Scheduler* s, uint64_t ticket, bool wait)
{
    std::unique_lock<std::mutex> lk(s->mu);
    sched::Req* r = s->core.find(ticket);
    if (!r) return set_error(DR_E_NOTFOUND, "unknown or collected ticket");
    if (wait) s->done_cv.wait(lk, [r] { return r->state >= sched::kComplete; });
    if (r->state < sched::kComplete) return DR_PENDING;
    r = s->core.take(ticket);
    const dr_status res = r->result;
    delete work_of(*r);
    delete r;
    if (res != DR_OK) return set_error(res, "request failed on the device");
    return DR_OK;
}

dr_status dr_poll(dr_ctx c, uint64_t ticket)
{
    if (!c) return set_error(DR_E_INVAL, "dr_poll: NULL context");
    if (!c->sched) return set_error(DR_E_NOTFOUND, "unknown ticket");
    return collect(c->sched, ticket, false);
}

dr_status dr_wait(dr_ctx c, uint64_t ticket)
{
    if (!c) return set_error(DR_E_INVAL, "dr_wait: NULL context");
    if (!c->sched) return set_error(DR_E_NOTFOUND, "unknown ticket");
    return collect(c->sched, ticket, true);
}

dr_status dr_ctx_stats(dr_ctx c, dr_stats* out)
{
    if (!c || !out) return set_error(DR_E_INVAL, "dr_ctx_stats: NULL argument");
    *out = dr_stats{};
    out->hbm_budget = c->budget;
    if (!c->sched) return DR_OK;
    std::lock_guard<std::mutex> lk(c->sched->mu);
    const sched::Counters& k = c->sched->core.counters();
    out->submitted = k.submitted;
    out->admitted = k.admitted;
    out->completed = k.completed;
    out->epochs = k.epochs;
    out->tiles_launched = c->sched->ex.tiles_launched;
    out->bytes_h2d = k.bytes_h2d;
    out->hbm_in_use = k.in_use;
    out->hbm_budget = c->budget;
    return DR_OK;
}

}  // extern "C"
