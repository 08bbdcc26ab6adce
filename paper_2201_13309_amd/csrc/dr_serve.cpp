// Serving: a request queue with admission by device-memory footprint and
// continuous batching.  One scheduler thread per context:
//
//   admit    FIFO; the head request is admitted when the memory it needs
//            (device copy of host images, partial totals) fits the budget;
//   copy     host images travel in row slabs on the copy stream, slabs of all
//            admitted requests interleaved (shortest remaining first), at most
//            two slabs in flight, so a small request never queues behind a
//            full-frame copy;
//   epoch    every pass launches one persistent kernel (per pixels-per-lane
//            group) over the resident, not yet processed row tiles of every
//            admitted request; at most two epochs are in flight, so requests
//            that arrive while others run join the next one;
//   finish   after a request's last rows: totals, a completion event and the
//            stream-ordered release of its buffers.
//
// Each output element is produced by the same tile code as dr_reconstruct.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "dr_runtime.h"

namespace dr {

namespace {

constexpr int kEpochSlots = 3;     // epoch argument buffers in rotation
constexpr int kEpochsInFlight = 2;
constexpr int kCopiesInFlight = 2;
constexpr int kMaxActive = 64;     // admitted requests at a time
constexpr int kMaxSegs = 256;      // request segments per epoch and group
constexpr int kGroups = 6;         // (pass 1 or 2) x (4, 2 or 1 pixels per lane)

struct Request {
    uint64_t id = 0;
    dr_geom g = nullptr;
    const uint16_t* images = nullptr;  // caller's (host or device)
    bool on_device = false;
    float* out = nullptr;
    float* totals = nullptr;
    size_t footprint = 0;
    TileCfg tile{4, 4, 16};
    uint16_t* staged = nullptr;        // device copy of host images
    float* parts = nullptr;
    double* work = nullptr;
    int rows_copied = 0;               // rows whose copy has been enqueued
    int rows_ready = 0;                // rows resident on the device
    int rows_next = 0;                 // rows handed to an epoch
    std::deque<std::pair<hipEvent_t, int>> copies;  // in-flight slab copies
    hipEvent_t done = nullptr;
    bool finishing = false;            // totals/done enqueued
    int state = 0;                     // 0 queued, 1 admitted, 2 complete, 3 failed
    dr_status result = DR_PENDING;
};

struct EpochSlot {
    DevBuf args;   // ScanArgs[kGroups][kMaxSegs] + starts[kGroups][kMaxSegs+1] + counters
    ScanArgs* h_args = nullptr;  // pinned staging
    int64_t* h_starts = nullptr;
    hipEvent_t uploaded = nullptr;
    hipEvent_t finished = nullptr;
    bool busy = false;
};

}  // namespace

struct Scheduler {
    dr_ctx ctx;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler thread
    std::condition_variable done_cv;  // wakes dr_wait
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<Request*> queue;       // not yet admitted
    std::vector<Request*> active;     // admitted, not complete
    std::unordered_map<uint64_t, Request*> all;
    size_t in_use = 0;
    int copies_in_flight = 0;
    EpochSlot slots[kEpochSlots];
    int slot_next = 0;
    dr_stats stats{};
    std::thread th;
    std::vector<hipEvent_t> event_pool;

    hipEvent_t get_event()
    {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    void put_event(hipEvent_t e)
    {
        if (e) event_pool.push_back(e);
    }

    void fail(Request* r, dr_status code)
    {
        r->state = 3;
        r->result = code;
        done_cv.notify_all();
    }

    static size_t staging_bytes(const Request* r)
    {
        return r->on_device ? 0
                            : (size_t)r->g->nx * r->g->ny * r->g->n_steps * sizeof(uint16_t);
    }
    static size_t parts_bytes(const Request* r)
    {
        return r->totals ? (size_t)r->g->passes * partial_slots(r->g, r->tile) * r->g->n_bins *
                                   sizeof(float) +
                               (size_t)kTotalsWorkRows * r->g->n_bins * sizeof(double)
                         : 0;
    }

    // ---------------------------------------------------------------- steps

    void admit()
    {
        while (!queue.empty() && (int)active.size() < kMaxActive) {
            Request* r = queue.front();
            if (in_use + r->footprint > ctx->budget) break;
            const size_t sb = staging_bytes(r);
            hipError_t e = hipSuccess;
            if (sb) e = hipMallocAsync((void**)&r->staged, sb, ctx->copy);
            if (e == hipSuccess && r->totals) {
                const size_t pb =
                    (size_t)r->g->passes * partial_slots(r->g, r->tile) * r->g->n_bins * sizeof(float);
                e = hipMallocAsync((void**)&r->parts, pb, ctx->copy);
                if (e == hipSuccess)
                    e = hipMallocAsync((void**)&r->work,
                                       (size_t)kTotalsWorkRows * r->g->n_bins * sizeof(double),
                                       ctx->copy);
            }
            queue.pop_front();
            if (e != hipSuccess) {
                fail(r, e == hipErrorOutOfMemory ? DR_E_NOMEM : DR_E_DEVICE);
                r->g->inflight--;
                continue;
            }
            in_use += r->footprint;
            r->state = 1;
            if (r->on_device) {
                r->rows_copied = r->rows_ready = r->g->ny;
            } else {
                // buffers allocated on the copy stream are ready for its copies;
                // the compute stream sees them through the slab events
            }
            active.push_back(r);
            stats.admitted++;
        }
    }

    void issue_copies()
    {
        while (copies_in_flight < kCopiesInFlight) {
            Request* best = nullptr;
            int64_t best_left = 0;
            for (Request* r : active) {
                if (r->on_device || r->rows_copied >= r->g->ny) continue;
                const int64_t left = (int64_t)(r->g->ny - r->rows_copied) * r->g->nx * r->g->n_steps;
                if (!best || left < best_left) {
                    best = r;
                    best_left = left;
                }
            }
            if (!best) return;
            Request* r = best;
            const size_t row_bytes = (size_t)r->g->nx * r->g->n_steps * sizeof(uint16_t);
            const int R = std::max(1, std::min(r->g->ny, (int)(((size_t)64 << 20) / row_bytes)));
            const int r0 = r->rows_copied, rs = std::min(R, r->g->ny - r0);
            const size_t plane = (size_t)r->g->nx * r->g->ny;
            // rows [r0, r0+rs) of every step, into the same place of the device copy
            hipError_t e = hipMemcpy2DAsync(r->staged + (size_t)r0 * r->g->nx, plane * 2,
                                            r->images + (size_t)r0 * r->g->nx, plane * 2,
                                            (size_t)rs * r->g->nx * 2, (size_t)r->g->n_steps,
                                            hipMemcpyHostToDevice, ctx->copy);
            hipEvent_t ev = get_event();
            if (e == hipSuccess && ev) e = hipEventRecord(ev, ctx->copy);
            if (e != hipSuccess || !ev) {
                fail(r, DR_E_DEVICE);
                return;
            }
            r->copies.push_back({ev, r0 + rs});
            r->rows_copied = r0 + rs;
            copies_in_flight++;
            stats.bytes_h2d += (uint64_t)rs * row_bytes;
        }
    }

    void poll_copies()
    {
        for (Request* r : active) {
            while (!r->copies.empty()) {
                hipError_t q = hipEventQuery(r->copies.front().first);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    fail(r, DR_E_DEVICE);
                    break;
                }
                r->rows_ready = r->copies.front().second;
                put_event(r->copies.front().first);
                r->copies.pop_front();
                copies_in_flight--;
            }
        }
    }

    int epochs_in_flight()
    {
        int n = 0;
        for (auto& s : slots)
            if (s.busy) {
                hipError_t q = hipEventQuery(s.finished);
                if (q == hipErrorNotReady) n++;
                else s.busy = false;
            }
        return n;
    }

    bool launch_epoch()
    {
        if (epochs_in_flight() >= kEpochsInFlight) return false;
        EpochSlot* es = nullptr;
        for (int i = 0; i < kEpochSlots && !es; ++i) {
            EpochSlot& s = slots[(slot_next + i) % kEpochSlots];
            if (!s.busy) {
                es = &s;
                slot_next = (slot_next + i + 1) % kEpochSlots;
            }
        }
        if (!es) return false;
        // segments: resident, unprocessed rows of every admitted request,
        // grouped by pass and pixels per lane (one launch per group; every
        // second-pass launch follows every first-pass launch of the epoch)
        static const int kPpl[3] = {4, 2, 1};
        int nseg[kGroups] = {0, 0, 0, 0, 0, 0};
        int64_t tiles[kGroups] = {0, 0, 0, 0, 0, 0};
        std::vector<Request*> finishing;
        struct Solo {
            Request* r;
            int row_begin, row_end;
        };
        std::vector<Solo> solos;  // per-pixel and weighted requests: launched on their own
        for (Request* r : active) {
            if (r->state != 1 || r->finishing) continue;
            if (batch_solo(r->g)) {
                if (r->rows_ready > r->rows_next) {
                    solos.push_back({r, r->rows_next, r->rows_ready});
                    r->rows_next = r->rows_ready;
                }
                if (r->rows_next == r->g->ny) finishing.push_back(r);
                continue;
            }
            const int pi = r->tile.ppl == 4 ? 0 : (r->tile.ppl == 2 ? 1 : 2);
            const int passes = r->g->passes;
            bool room = true;
            for (int p = 0; p < passes; ++p) room = room && nseg[p * 3 + pi] < kMaxSegs;
            if (r->rows_ready > r->rows_next && room) {
                const uint16_t* img = r->on_device ? r->images : r->staged;
                for (int p = 0; p < passes; ++p) {
                    const int gi = p * 3 + pi;
                    ScanArgs a = scan_args(r->g, r->tile, p, img, (int64_t)r->g->nx * r->g->ny,
                                           0, r->rows_next, r->rows_ready, r->out, r->parts);
                    const int sg = nseg[gi]++;
                    es->h_args[gi * kMaxSegs + sg] = a;
                    int64_t* st = es->h_starts + gi * (kMaxSegs + 1);
                    if (sg == 0) st[0] = 0;
                    st[sg + 1] = st[sg] + (int64_t)(r->rows_ready - r->rows_next) * a.tiles_per_row;
                    tiles[gi] = st[sg + 1];
                }
                r->rows_next = r->rows_ready;
            }
            if (r->rows_next == r->g->ny) finishing.push_back(r);
        }
        int nall = (int)solos.size();
        for (int gi = 0; gi < kGroups; ++gi) nall += nseg[gi];
        if (nall == 0 && finishing.empty()) return false;
        hipStream_t s = ctx->stream;
        char* dbase = es->args.as<char>();
        ScanArgs* d_args = (ScanArgs*)dbase;
        int64_t* d_starts = (int64_t*)(dbase + sizeof(ScanArgs) * kGroups * kMaxSegs);
        unsigned long long* d_cnt =
            (unsigned long long*)(dbase + sizeof(ScanArgs) * kGroups * kMaxSegs +
                                  sizeof(int64_t) * kGroups * (kMaxSegs + 1));
        hipError_t e = hipSuccess;
        // the pinned staging of this slot was last read by an upload that has
        // completed (the slot is not busy), so it can be rewritten and sent
        e = hipMemcpyAsync(d_args, es->h_args, sizeof(ScanArgs) * kGroups * kMaxSegs,
                           hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_starts, es->h_starts, sizeof(int64_t) * kGroups * (kMaxSegs + 1),
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
            // 8 persistent 4-wave workgroups per CU (2048 threads); 2 left the GPU a third idle
            const int groups = (int)std::max<int64_t>(1, std::min<int64_t>(ctx->cus * 8, tiles[gi]));
            e = launch_reset_counter(ba.counter, s);
            // groups 3..5 hold second passes, which add onto the first
            if (e == hipSuccess) e = launch_batch_f32(t, ba, gi >= 3, groups, s);
            stats.tiles_launched += (uint64_t)tiles[gi];
        }
        for (const Solo& so : solos) {
            Request* r = so.r;
            const uint16_t* img = r->on_device ? r->images : r->staged;
            for (int p = 0; p < r->g->passes && e == hipSuccess; ++p) {
                const ScanArgs a = scan_args(r->g, r->tile, p, img, (int64_t)r->g->nx * r->g->ny,
                                             0, so.row_begin, so.row_end, r->out, r->parts);
                e = launch_scan_f32(r->g, r->tile, p, a, s);
                stats.tiles_launched += (uint64_t)(so.row_end - so.row_begin) * a.tiles_per_row;
            }
        }
        for (Request* r : finishing) {
            if (e != hipSuccess) break;
            if (r->totals)
                e = enqueue_totals(r->g, r->parts, partial_slots(r->g, r->tile), r->work,
                                   r->totals, s);
            r->done = get_event();
            if (e == hipSuccess && r->done) e = hipEventRecord(r->done, s);
            if (e == hipSuccess && r->staged) e = hipFreeAsync(r->staged, s);
            if (e == hipSuccess && r->parts) e = hipFreeAsync(r->parts, s);
            if (e == hipSuccess && r->work) e = hipFreeAsync(r->work, s);
            r->staged = nullptr;
            r->parts = nullptr;
            r->work = nullptr;
            r->finishing = true;
        }
        if (e == hipSuccess) e = hipEventRecord(es->finished, s);
        if (e != hipSuccess) {
            for (Request* r : active) fail(r, DR_E_DEVICE);
            return false;
        }
        es->busy = true;
        stats.epochs++;
        return true;
    }

    void poll_done()
    {
        for (size_t i = 0; i < active.size();) {
            Request* r = active[i];
            bool remove = false;
            if (r->state == 3) {
                remove = true;
            } else if (r->finishing && r->done) {
                hipError_t q = hipEventQuery(r->done);
                if (q == hipSuccess) {
                    r->state = 2;
                    r->result = DR_OK;
                    stats.completed++;
                    remove = true;
                } else if (q != hipErrorNotReady) {
                    fail(r, DR_E_DEVICE);
                    remove = true;
                }
            }
            if (remove) {
                in_use -= r->footprint;
                for (void* p : {(void*)r->staged, (void*)r->parts, (void*)r->work})
                    if (p) (void)hipFreeAsync(p, ctx->stream);
                r->staged = nullptr;
                r->parts = nullptr;
                r->work = nullptr;
                put_event(r->done);
                r->done = nullptr;
                r->g->inflight--;
                active.erase(active.begin() + i);
                done_cv.notify_all();
            } else {
                ++i;
            }
        }
    }

    bool busy_gpu()
    {
        if (copies_in_flight > 0) return true;
        for (auto& s : slots)
            if (s.busy) return true;
        for (Request* r : active)
            if (r->finishing) return true;
        return false;
    }

    void run()
    {
        (void)hipSetDevice(ctx->device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop || !queue.empty() || !active.empty()) {
            admit();
            // copies must follow the allocations made on the copy stream
            issue_copies();
            poll_copies();
            while (launch_epoch()) {
            }
            poll_done();
            if (stop && queue.empty() && active.empty()) break;
            if (busy_gpu())
                cv.wait_for(lk, std::chrono::microseconds(100));
            else
                cv.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
};

Scheduler* make_scheduler(dr_ctx ctx)
{
    auto* s = new Scheduler();
    s->ctx = ctx;
    for (auto& es : s->slots) {
        const size_t bytes = sizeof(ScanArgs) * kGroups * kMaxSegs +
                             sizeof(int64_t) * kGroups * (kMaxSegs + 1) +
                             sizeof(unsigned long long) * kGroups;
        if (es.args.reserve(bytes) != hipSuccess ||
            hipHostMalloc((void**)&es.h_args, sizeof(ScanArgs) * kGroups * kMaxSegs, 0) != hipSuccess ||
            hipHostMalloc((void**)&es.h_starts, sizeof(int64_t) * kGroups * (kMaxSegs + 1), 0) != hipSuccess ||
            hipEventCreateWithFlags(&es.uploaded, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&es.finished, hipEventDisableTiming) != hipSuccess) {
            destroy_scheduler(s);
            return nullptr;
        }
    }
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, ctx->device) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    s->stats.hbm_budget = ctx->budget;
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
    for (auto& kv : s->all) delete kv.second;
    for (auto& es : s->slots) {
        if (es.h_args) (void)hipHostFree(es.h_args);
        if (es.h_starts) (void)hipHostFree(es.h_starts);
        if (es.uploaded) (void)hipEventDestroy(es.uploaded);
        if (es.finished) (void)hipEventDestroy(es.finished);
    }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
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
    auto r = std::make_unique<Request>();
    r->g = g;
    r->images = images;
    r->on_device = images_on_device != 0;
    r->out = out;
    r->totals = totals;
    if (batch_solo(g)) {
        r->tile = solo_tile(g);
    } else {
        r->tile = default_tile(g, r->on_device ? (const void*)images : nullptr, out);
        r->tile.waves = 4;
        r->tile.prefetch = 16;
    }
    if (!tile_fits(g, r->tile, r->on_device ? (const void*)images : nullptr, out))
        return set_error(DR_E_INVAL, "dr_submit: misaligned buffer");
    r->footprint = Scheduler::staging_bytes(r.get()) + Scheduler::parts_bytes(r.get());
    if (!c->sched) {
        std::lock_guard<std::mutex> lk(c->mu);
        if (!c->sched) c->sched = make_scheduler(c);
        if (!c->sched) return set_error(DR_E_DEVICE, "dr_submit: cannot start the scheduler");
    }
    Scheduler* s = c->sched;
    if (r->footprint > c->budget)
        return set_error(DR_E_NOMEM, "dr_submit: request larger than the device-memory budget");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        *ticket = r->id;
        g->inflight++;
        s->stats.submitted++;
        s->all[r->id] = r.get();
        s->queue.push_back(r.release());
    }
    s->cv.notify_all();
    return DR_OK;
}

static dr_status collect(Scheduler* s, uint64_t ticket, bool wait)
{
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(DR_E_NOTFOUND, "unknown or collected ticket");
    Request* r = it->second;
    if (wait) s->done_cv.wait(lk, [r] { return r->state >= 2; });
    if (r->state < 2) return DR_PENDING;
    const dr_status res = r->result;
    s->all.erase(it);
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
    *out = c->sched->stats;
    out->hbm_in_use = c->sched->in_use;
    out->hbm_budget = c->budget;
    return DR_OK;
}

}  // extern "C"
