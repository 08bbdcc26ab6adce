// The serving scheduler's policy (dr_sched.cpp) driven on the CPU by a
// simulated executor with a fake clock: a copy engine and a compute engine
// that finish work after modelled times, allocations that are counted, and
// failures injected on request.  Built with g++ (ASan/UBSan in the tests) and
// run by tests/test_sched_cpu.py; prints one line per scenario and exits
// non-zero if any fails.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <map>
#include <memory>
#include <random>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "dr_sched.h"

using namespace dr::sched;

namespace {

struct SimReq {
    size_t staging = 0, parts = 0;  // device bytes the executor allocates for it
    std::vector<int> rows_done;     // epochs that processed each row
    bool totals = false;            // its totals were enqueued
    double last_use = 0.0;          // completion time of the last work that touches it
    bool allocated = false, released = false;
    int finished = 0;
    std::vector<double> row_ready_at;        // completion time of the copy of each row (inf: none)
    std::vector<std::pair<int, int>> copied;  // row ranges copied, in order
};

struct Sim : Executor {
    double now = 0.0;
    double copy_bw = 50e9;      // bytes/s of the copy engine
    double row_cost = 2e-6;     // s per detector row on the compute engine
    double epoch_cost = 20e-6;  // s per epoch launch
    int copy_channels = 1;      // >1: copies may complete out of order
    bool shuffle_epochs = false;  // epochs complete out of order
    std::mt19937_64 rng{1};
    std::vector<double> copy_free;
    double compute_free = 0.0;
    uint64_t next_ev = 1;
    std::map<Event, double> done_at;
    std::set<Event> fails;
    size_t allocated = 0, peak_allocated = 0;
    std::vector<std::string> violations;
    int64_t epochs = 0;
    // failure injection
    std::set<uint64_t> fail_alloc, fail_copy_enqueue, fail_copy_event;
    std::set<int64_t> fail_epoch_launch, fail_epoch_event;
    std::map<uint64_t, int> copies_seen;
    std::set<uint64_t> in_failed_epoch;  // requests with work in an epoch that failed
    double slot_busy_until[kEpochSlots] = {0.0, 0.0, 0.0};

    Sim() { copy_free.assign(4, 0.0); }
    SimReq& S(Req& r) { return *static_cast<SimReq*>(r.user); }
    void bad(const std::string& m)
    {
        if (violations.size() < 20) violations.push_back(m);
    }

    dr_status allocate(Req& r) override
    {
        SimReq& s = S(r);
        if (s.allocated) bad("allocated twice");
        if (fail_alloc.count(r.id)) return DR_E_NOMEM;
        s.allocated = true;
        allocated += s.staging + s.parts;
        peak_allocated = std::max(peak_allocated, allocated);
        return DR_OK;
    }
    dr_status copy_rows(Req& r, int r0, int rows, Event* ev) override
    {
        SimReq& s = S(r);
        if (r.on_device) bad("copy of a device-image request");
        if (!s.allocated || s.released) bad("copy into a buffer not held");
        const int n = copies_seen[r.id]++;
        if (fail_copy_enqueue.count(r.id) && n == 1) return DR_E_DEVICE;
        int expect = s.copied.empty() ? 0 : s.copied.back().second;
        if (r0 != expect) bad("copy rows out of order");
        s.copied.push_back({r0, r0 + rows});
        // least-loaded channel
        auto it = std::min_element(copy_free.begin(), copy_free.begin() + copy_channels);
        const double t = std::max(now, *it) + (double)rows * (double)r.row_bytes / copy_bw;
        *it = t;
        *ev = next_ev++;
        done_at[*ev] = t;
        if (fail_copy_event.count(r.id) && n == 1) fails.insert(*ev);
        for (int j = r0; j < r0 + rows; ++j) s.row_ready_at[j] = t;
        s.last_use = std::max(s.last_use, t);
        return DR_OK;
    }
    dr_status launch_epoch(int slot, const std::vector<Segment>& segs,
                           const std::vector<Req*>& finishing, Event* ev) override
    {
        if (slot < 0 || slot >= kEpochSlots) {
            bad("slot out of range");
            return DR_E_DEVICE;
        }
        if (slot_busy_until[slot] > now) bad("epoch slot reused while its epoch runs");
        int running = 0;
        for (double b : slot_busy_until) running += b > now ? 1 : 0;
        if (running >= kEpochsInFlight) bad("more epochs in flight than the limit");
        const int64_t seq = epochs++;
        if (fail_epoch_launch.count(seq) || fail_epoch_event.count(seq)) {
            for (const Segment& sg : segs) in_failed_epoch.insert(sg.r->id);
            for (Req* r : finishing) in_failed_epoch.insert(r->id);
        }
        if (fail_epoch_launch.count(seq)) return DR_E_DEVICE;  // nothing enqueued
        const double start = std::max(now, compute_free);
        double cost = epoch_cost;
        for (const Segment& sg : segs) {
            SimReq& s = S(*sg.r);
            if (!s.allocated || s.released) bad("epoch on a buffer not held");
            if (sg.row_begin < 0 || sg.row_end > sg.r->ny || sg.row_begin >= sg.row_end)
                bad("bad segment");
            // every row of the segment was copied, and the copy completed
            // before the epoch was enqueued (the host saw its event)
            if (!sg.r->on_device)
                for (int j = sg.row_begin; j < sg.row_end; ++j)
                    if (!(s.row_ready_at[j] <= now)) {
                        bad("epoch reads rows whose copy has not completed");
                        break;
                    }
            for (int j = sg.row_begin; j < sg.row_end; ++j) s.rows_done[j]++;
            cost += row_cost * (sg.row_end - sg.row_begin);
        }
        for (Req* r : finishing) {
            SimReq& s = S(*r);
            for (int j = 0; j < r->ny; ++j)
                if (s.rows_done[j] != 1) {
                    bad("totals before every row was launched once");
                    break;
                }
            if (s.totals) bad("totals enqueued twice");
            s.totals = true;
        }
        double t = start + cost;
        compute_free = t;
        if (shuffle_epochs) t = start + cost * std::uniform_real_distribution<double>(0.1, 3.0)(rng);
        *ev = next_ev++;
        done_at[*ev] = t;
        slot_busy_until[slot] = t;
        if (fail_epoch_event.count(seq)) fails.insert(*ev);
        for (const Segment& sg : segs) S(*sg.r).last_use = std::max(S(*sg.r).last_use, t);
        for (Req* r : finishing) S(*r).last_use = std::max(S(*r).last_use, t);
        return DR_OK;
    }
    Poll query(Event ev) override
    {
        auto it = done_at.find(ev);
        if (it == done_at.end()) {
            bad("query of an unknown or forgotten event");
            return kFailed;
        }
        if (it->second > now) return kPending;
        return fails.count(ev) ? kFailed : kDone;
    }
    void forget(Event ev) override
    {
        auto it = done_at.find(ev);
        if (it == done_at.end()) bad("forget of an unknown event");
        else if (it->second > now) bad("forget of an event still pending");
        else done_at.erase(it);
    }
    void release(Req& r) override
    {
        SimReq& s = S(r);
        if (!s.allocated) bad("release of a request never allocated");
        if (s.released) bad("released twice");
        if (s.last_use > now + 1e-15) bad("release while device work still uses the buffers");
        s.released = true;
        allocated -= s.staging + s.parts;
    }
    void finished(Req& r) override { S(r).finished++; }
};

struct Arrival {
    double t;
    int ny, nx, steps;
    bool on_device, totals;
};

struct Run {
    Sim sim;
    std::unique_ptr<Core> core;
    std::vector<std::unique_ptr<Req>> reqs;
    std::vector<std::unique_ptr<SimReq>> sreqs;
    std::vector<dr_status> submit_status;
    std::vector<double> completed_at;
    std::vector<uint64_t> order;  // ids in completion order
    size_t budget;
    size_t max_in_use = 0;
    int max_active_seen = 0;
    explicit Run(size_t b) : budget(b) { core.reset(new Core(sim, b)); }

    static size_t footprint(const Arrival& a)
    {
        const size_t img = (size_t)a.ny * a.nx * a.steps * 2, out = (size_t)a.ny * a.nx * 64 * 4;
        return img + out + (a.totals ? (size_t)a.ny * 16 * 64 * 4 : 0);
    }

    // drive the core until every request is final; false on a stall
    // drive the core until every request is final; false on a stall.  The
    // clock jumps to the next event or arrival once a step changes nothing.
    bool drive(const std::vector<Arrival>& arr, double limit = 600.0)
    {
        size_t next = 0;
        uint64_t id = 1;
        for (long it = 0; next < arr.size() || !core->idle(); ++it) {
            if (it > 20000000L || sim.now > limit) return false;
            while (next < arr.size() && arr[next].t <= sim.now) {
                const Arrival& a = arr[next++];
                auto r = std::make_unique<Req>();
                auto s = std::make_unique<SimReq>();
                r->id = id++;
                r->ny = a.ny;
                r->row_bytes = (size_t)a.nx * a.steps * 2;
                r->on_device = a.on_device;
                r->footprint = footprint(a);
                s->staging = a.on_device ? 0 : (size_t)a.ny * r->row_bytes;
                s->parts = a.totals ? (size_t)a.ny * 16 * 64 * 4 : 0;
                s->rows_done.assign(a.ny, 0);
                s->row_ready_at.assign(a.ny, INFINITY);
                r->user = s.get();
                submit_status.push_back(core->submit(r.get()));
                reqs.push_back(std::move(r));
                sreqs.push_back(std::move(s));
                completed_at.push_back(-1.0);
            }
            const auto sig = [&] {
                const Counters& k = core->counters();
                return std::make_tuple(k.admitted, k.completed, k.failed, k.epochs, k.bytes_h2d,
                                       sim.done_at.size(), core->copies_in_flight());
            };
            const auto before = sig();
            core->step();
            max_in_use = std::max(max_in_use, core->counters().in_use);
            for (size_t i = 0; i < reqs.size(); ++i)
                if (submit_status[i] == DR_OK && completed_at[i] < 0 &&
                    reqs[i]->state >= kComplete) {
                    completed_at[i] = sim.now;
                    order.push_back(reqs[i]->id);
                }
            if (sig() != before) continue;  // something happened: step again now
            double t = INFINITY;
            for (auto& e : sim.done_at)
                if (e.second > sim.now) t = std::min(t, e.second);
            if (next < arr.size()) t = std::min(t, arr[next].t);
            if (!(t < INFINITY)) return !(next < arr.size() || !core->idle()) ? true : false;
            sim.now = std::max(t, sim.now + 1e-9);
        }
        return true;
    }
    std::string check_common()
    {
        if (!sim.violations.empty()) return sim.violations[0];
        if (core->counters().in_use != 0) return "footprint left in use";
        if (max_in_use > budget) return "in use above the budget";
        if (sim.allocated != 0) return "device bytes left allocated";
        if (core->copies_in_flight() != 0) return "copies left in flight";
        for (size_t i = 0; i < reqs.size(); ++i) {
            if (submit_status[i] != DR_OK) continue;
            Req& r = *reqs[i];
            SimReq& s = *sreqs[i];
            if (s.finished != 1) return "finished() not called exactly once";
            if (r.state == kComplete) {
                if (!s.totals) return "completed without totals";
                for (int j = 0; j < r.ny; ++j)
                    if (s.rows_done[j] != 1) return "a row not processed exactly once";
                if (!s.released) return "completed but not released";
            } else if (r.state == kFailedState) {
                if (s.allocated && !s.released) return "failed but not released";
            } else {
                return "request not final";
            }
        }
        return "";
    }
};

std::vector<Arrival> mix(int n, uint64_t seed, double rate, double big_frac = 0.0)
{
    std::mt19937_64 g(seed);
    std::exponential_distribution<double> gap(rate);
    std::uniform_int_distribution<int> side(0, 3), steps(101, 801);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::vector<Arrival> a;
    double t = 0.0;
    for (int i = 0; i < n; ++i) {
        t += gap(g);
        Arrival x;
        x.t = t;
        const bool big = u(g) < big_frac;
        const int s = big ? 2048 : 256 * (1 + side(g));
        x.ny = s;
        x.nx = s;
        x.steps = big ? 1001 : steps(g);
        x.on_device = u(g) < 0.3;
        x.totals = u(g) < 0.8;
        a.push_back(x);
    }
    return a;
}

int g_failures = 0;
void report(const char* name, const std::string& err)
{
    if (err.empty()) {
        std::printf("%s ok\n", name);
    } else {
        std::printf("%s FAIL: %s\n", name, err.c_str());
        g_failures++;
    }
}

// -------------------------------------------------------------- scenarios

std::string poisson_mix()
{
    Run run((size_t)200 << 30);
    auto arr = mix(120, 5, 20.0, 0.05);
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (run.core->counters().completed != arr.size()) return "not every request completed";
    // continuous batching: far fewer epochs than requests x slabs would need
    if (run.core->counters().epochs < 10) return "too few epochs";
    return "";
}

std::string budget_refusal_and_queueing()
{
    // a budget that holds about one 1024^2 request: the larger one is refused
    // at submission, the others wait for admission and all complete in order
    Arrival a{0.0, 1024, 1024, 401, false, true};
    const size_t one = Run::footprint(a);
    Run run(one + one / 2);
    std::vector<Arrival> arr;
    for (int i = 0; i < 6; ++i) arr.push_back({1e-4 * i, 1024, 1024, 401, i % 2 == 0, true});
    arr.push_back({1e-3, 2048, 2048, 1001, false, true});  // larger than the budget
    if (!run.drive(arr)) return "stalled";
    if (run.submit_status.back() != DR_E_NOMEM) return "oversized request not refused";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (run.max_in_use > one + one / 2 || run.max_in_use < one) return "in-use bound wrong";
    for (size_t k = 0; k < run.order.size(); ++k)
        if (run.order[k] != k + 1) return "FIFO admission violated";
    return "";
}

std::string output_counted_in_footprint()
{
    // images alone would fit twice; with their outputs only one at a time
    Arrival a{0.0, 512, 512, 101, false, false};
    const size_t img = (size_t)512 * 512 * 101 * 2;
    const size_t fp = Run::footprint(a);
    if (fp <= img) return "footprint does not count the output";
    Run run(fp + img);
    std::vector<Arrival> arr(4, a);
    for (int i = 0; i < 4; ++i) arr[i].t = 1e-5 * i;
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (run.max_in_use != fp) return "two requests admitted beside each other";
    return "";
}

std::string slot_exhaustion()
{
    // more device-image requests than active slots at once
    Run run((size_t)1 << 40);
    std::vector<Arrival> arr;
    for (int i = 0; i < 3 * kMaxActive; ++i) arr.push_back({0.0, 64, 64, 41, true, true});
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (run.core->counters().completed != arr.size()) return "not every request completed";
    return "";
}

std::string small_not_behind_full_frame()
{
    // a full frame arrives first; a small request arriving just after is
    // copied and completed long before the full frame's copy is over
    Run run((size_t)200 << 30);
    std::vector<Arrival> arr = {{0.0, 2048, 2048, 1001, false, true},
                                {1e-3, 256, 256, 201, false, true}};
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (!(run.completed_at[1] < 0.5 * run.completed_at[0])) return "small request queued behind";
    return "";
}

std::string out_of_order_completion()
{
    Run run((size_t)200 << 30);
    run.sim.copy_channels = 3;
    run.sim.shuffle_epochs = true;
    auto arr = mix(80, 9, 40.0, 0.0);
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (run.core->counters().completed != arr.size()) return "not every request completed";
    return "";
}

std::string copy_enqueue_failure()
{
    // request 2's second copy fails to enqueue: it fails alone, after its
    // first copy drained; later host-image requests are still copied
    Run run((size_t)200 << 30);
    run.sim.fail_copy_enqueue = {2};
    std::vector<Arrival> arr;
    for (int i = 0; i < 8; ++i) arr.push_back({2e-3 * i, 1024, 1024, 401, false, true});
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (run.reqs[1]->state != kFailedState || run.reqs[1]->result != DR_E_DEVICE)
        return "failing request not reported";
    if (run.core->counters().completed != 7) return "other requests did not complete";
    return "";
}

std::string copy_event_failure()
{
    // two requests see a copy fail on the device: both fail, the rest
    // complete (no copy slot stays taken)
    Run run((size_t)200 << 30);
    run.sim.fail_copy_event = {1, 3};
    std::vector<Arrival> arr;
    for (int i = 0; i < 8; ++i) arr.push_back({1e-3 * i, 1024, 1024, 401, false, true});
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (run.core->counters().failed != 2 || run.core->counters().completed != 6)
        return "wrong requests failed";
    return "";
}

std::string alloc_failure()
{
    Run run((size_t)200 << 30);
    run.sim.fail_alloc = {3};
    std::vector<Arrival> arr;
    for (int i = 0; i < 6; ++i) arr.push_back({1e-4 * i, 512, 512, 201, i % 2 == 1, true});
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    if (run.reqs[2]->result != DR_E_NOMEM) return "allocation failure not reported";
    if (run.core->counters().completed != 5) return "other requests did not complete";
    return "";
}

std::string epoch_failures()
{
    // the third epoch fails to launch and the fifth fails on the device: only
    // the requests with work in those epochs fail
    Run run((size_t)200 << 30);
    run.sim.fail_epoch_launch = {2};
    run.sim.fail_epoch_event = {4};
    auto arr = mix(40, 13, 200.0, 0.0);
    if (!run.drive(arr)) return "stalled";
    std::string e = run.check_common();
    if (!e.empty()) return e;
    const auto& k = run.core->counters();
    if (k.failed == 0 || k.completed == 0) return "failures not confined";
    if (k.failed + k.completed != arr.size()) return "requests lost";
    // exactly the requests with work in a failed epoch fail
    for (auto& r : run.reqs)
        if ((r->state == kFailedState) != (run.sim.in_failed_epoch.count(r->id) > 0))
            return "a request failed that had no work in a failed epoch, or the reverse";
    return "";
}

}  // namespace

int main()
{
    report("poisson_mix", poisson_mix());
    report("budget_refusal_and_queueing", budget_refusal_and_queueing());
    report("output_counted_in_footprint", output_counted_in_footprint());
    report("slot_exhaustion", slot_exhaustion());
    report("small_not_behind_full_frame", small_not_behind_full_frame());
    report("out_of_order_completion", out_of_order_completion());
    report("copy_enqueue_failure", copy_enqueue_failure());
    report("copy_event_failure", copy_event_failure());
    report("alloc_failure", alloc_failure());
    report("epoch_failures", epoch_failures());
    return g_failures ? 1 : 0;
}
