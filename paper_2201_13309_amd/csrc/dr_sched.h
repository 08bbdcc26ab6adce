// Scheduling policy of the serving loop (dr_submit / dr_poll), kept apart from
// the device so that it can be driven on the CPU by a simulated executor with
// a fake clock.  Plain C++17, no HIP.
//
//   admit    FIFO; the head request is admitted when its footprint (device
//            bytes it occupies while in flight: images, output, partial
//            totals) fits the budget beside the admitted ones, and fewer than
//            kMaxActive requests are admitted;
//   copy     host images travel in row slabs, slabs of all admitted requests
//            interleaved (least remaining bytes first), at most
//            kCopiesInFlight slabs in flight, so a small request never queues
//            behind a full-frame copy;
//   epoch    at most kEpochsInFlight epochs in flight; each launches the
//            resident, not yet launched rows of every admitted request, so a
//            request that arrives while others run joins the next epoch; a
//            request whose rows have all been launched is finished (totals)
//            in the same epoch, and completes when that epoch does;
//   failure  a failed copy, allocation, launch or epoch fails only the
//            requests it concerns; a failing request waits until its copies
//            and the epochs that read its buffers have completed, then its
//            buffers are released and it is reported failed.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <unordered_map>
#include <vector>

#include "dr.h"

namespace dr {
namespace sched {

typedef uint64_t Event;  // an executor's handle of a point in a device queue; 0: none

enum Poll { kPending = 0, kDone = 1, kFailed = 2 };
enum State { kQueued = 0, kAdmitted = 1, kComplete = 2, kFailedState = 3 };

constexpr int kEpochsInFlight = 2;
constexpr int kEpochSlots = 3;  // argument buffers of the executor, in rotation
constexpr int kCopiesInFlight = 2;
constexpr int kMaxActive = 64;

struct Req {
    uint64_t id = 0;
    int ny = 0;              // detector rows
    size_t row_bytes = 0;    // bytes of one detector row over all steps
    bool on_device = false;  // images already on the device (no copies)
    size_t footprint = 0;    // bytes counted against the budget
    void* user = nullptr;    // the executor's own state of the request
    // progress
    int state = kQueued;
    dr_status result = DR_PENDING;
    bool failing = false;    // failed; waiting for its device work to drain
    dr_status fail_code = DR_OK;
    int rows_copied = 0;     // rows whose copy has been enqueued
    int rows_ready = 0;      // rows resident on the device
    int rows_next = 0;       // rows handed to an epoch
    std::deque<std::pair<Event, int>> copies;  // in flight: event, rows ready once it completes
    int epochs_open = 0;     // epochs in flight that read or write its buffers
    bool finishing = false;  // its totals are enqueued (in the last epoch that has it)
    bool totals_done = false;  // that epoch has completed
    bool released = false;   // buffers handed back
};

// Rows [row_begin, row_end) of one request, launched in one epoch.
struct Segment {
    Req* r;
    int row_begin, row_end;
};

// What the scheduler asks of the device.  Every call returns at once; device
// work is ordered by the executor's queues (a copy queue and a compute queue)
// and observed through events.
struct Executor {
    virtual ~Executor() = default;
    // Allocate the request's device buffers (staging of host images, partial
    // totals).  On failure nothing stays allocated.
    virtual dr_status allocate(Req& r) = 0;
    // Enqueue the copy of rows [r0, r0 + rows) of every step of a host-image
    // request and return an event for its completion.
    virtual dr_status copy_rows(Req& r, int r0, int rows, Event* ev) = 0;
    // Enqueue one epoch in argument slot `slot`: the segments, then the
    // totals of the finishing requests; *ev completes after all of it.  On
    // failure, work this call already enqueued has completed when it returns.
    virtual dr_status launch_epoch(int slot, const std::vector<Segment>& segs,
                                   const std::vector<Req*>& finishing, Event* ev) = 0;
    virtual Poll query(Event ev) = 0;
    virtual void forget(Event ev) = 0;  // the event is not used again
    // Release the request's device buffers; called once per admitted request,
    // after every copy and epoch that uses them has been seen complete.
    virtual void release(Req& r) = 0;
    // The request reached its final state (complete or failed), admitted or
    // not; called once per request.
    virtual void finished(Req& r) = 0;
};

struct Counters {
    uint64_t submitted = 0, admitted = 0, completed = 0, failed = 0, epochs = 0;
    uint64_t rows_launched = 0, bytes_h2d = 0;
    size_t in_use = 0, peak_in_use = 0;
};

class Core {
public:
    Core(Executor& ex, size_t budget) : ex_(ex), budget_(budget) {}

    // Queue a request (its id, shape and footprint set); DR_E_NOMEM when it
    // can never fit the budget.  The core owns r until take() returns it.
    dr_status submit(Req* r);
    // One pass of the loop: admit, copy, launch, complete.  Returns true when
    // device work is in flight (the caller polls again soon).
    bool step();
    // The request of a ticket: nullptr if unknown; *state its state.
    Req* find(uint64_t id);
    // Hand a completed or failed request back to the caller (removed).
    Req* take(uint64_t id);
    bool idle() const { return queue_.empty() && active_.empty(); }
    const Counters& counters() const { return c_; }
    size_t budget() const { return budget_; }
    int copies_in_flight() const { return copies_in_flight_; }
    int epochs_in_flight() const;

private:
    struct Epoch {
        Event ev = 0;
        bool busy = false;
        int64_t seq = -1;
        std::vector<Req*> reqs;       // requests with segments or totals in it
        std::vector<Req*> finishing;  // requests completing with it
    };
    void admit();
    void issue_copies();
    void poll_copies();
    void poll_epochs();
    bool launch_epoch();
    void fail(Req* r, dr_status code);
    void retire();

    Executor& ex_;
    size_t budget_;
    std::deque<Req*> queue_;
    std::vector<Req*> active_;
    std::unordered_map<uint64_t, Req*> all_;
    Epoch slots_[kEpochSlots];
    int slot_next_ = 0;
    int64_t epoch_seq_ = 0;
    int copies_in_flight_ = 0;
    Counters c_;
};

}  // namespace sched
}  // namespace dr
