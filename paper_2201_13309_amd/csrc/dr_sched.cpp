// Scheduling policy of the serving loop (see dr_sched.h).  Plain C++17.
#include "dr_sched.h"

#include <algorithm>

namespace dr {
namespace sched {

namespace {
constexpr size_t kSlabBytes = (size_t)64 << 20;  // host-image bytes per copy
}

dr_status Core::submit(Req* r)
{
    if (r->footprint > budget_) return DR_E_NOMEM;
    r->state = kQueued;
    r->result = DR_PENDING;
    all_[r->id] = r;
    queue_.push_back(r);
    c_.submitted++;
    return DR_OK;
}

Req* Core::find(uint64_t id)
{
    auto it = all_.find(id);
    return it == all_.end() ? nullptr : it->second;
}

Req* Core::take(uint64_t id)
{
    auto it = all_.find(id);
    if (it == all_.end() || it->second->state < kComplete) return nullptr;
    Req* r = it->second;
    all_.erase(it);
    return r;
}

int Core::epochs_in_flight() const
{
    int n = 0;
    for (const Epoch& e : slots_) n += e.busy ? 1 : 0;
    return n;
}

void Core::fail(Req* r, dr_status code)
{
    if (r->failing || r->state >= kComplete) return;
    r->failing = true;
    r->fail_code = code;
}

void Core::admit()
{
    while (!queue_.empty() && (int)active_.size() < kMaxActive) {
        Req* r = queue_.front();
        if (c_.in_use + r->footprint > budget_) break;
        queue_.pop_front();
        const dr_status st = ex_.allocate(*r);
        if (st != DR_OK) {  // the executor keeps nothing allocated
            r->released = true;
            r->state = kFailedState;
            r->result = st;
            c_.failed++;
            ex_.finished(*r);
            continue;
        }
        c_.in_use += r->footprint;
        c_.peak_in_use = std::max(c_.peak_in_use, c_.in_use);
        r->state = kAdmitted;
        if (r->on_device) r->rows_copied = r->rows_ready = r->ny;
        active_.push_back(r);
        c_.admitted++;
    }
}

void Core::issue_copies()
{
    while (copies_in_flight_ < kCopiesInFlight) {
        Req* best = nullptr;
        size_t best_left = 0;
        for (Req* r : active_) {
            if (r->on_device || r->failing || r->rows_copied >= r->ny) continue;
            const size_t left = (size_t)(r->ny - r->rows_copied) * r->row_bytes;
            if (!best || left < best_left) {
                best = r;
                best_left = left;
            }
        }
        if (!best) return;
        Req* r = best;
        const int R = (int)std::max<size_t>(
            1, std::min<size_t>((size_t)r->ny, kSlabBytes / std::max<size_t>(1, r->row_bytes)));
        const int r0 = r->rows_copied, rs = std::min(R, r->ny - r0);
        Event ev = 0;
        const dr_status st = ex_.copy_rows(*r, r0, rs, &ev);
        if (st != DR_OK) {  // this request only; others may still copy
            fail(r, st);
            continue;
        }
        r->copies.push_back({ev, r0 + rs});
        r->rows_copied = r0 + rs;
        copies_in_flight_++;
        c_.bytes_h2d += (uint64_t)rs * r->row_bytes;
    }
}

void Core::poll_copies()
{
    for (Req* r : active_) {
        // completed copies, oldest first; a failing request's copies still drain
        while (!r->copies.empty()) {
            const Poll q = ex_.query(r->copies.front().first);
            if (q == kPending) break;
            if (q == kDone && !r->failing) r->rows_ready = r->copies.front().second;
            if (q == kFailed) fail(r, DR_E_DEVICE);
            ex_.forget(r->copies.front().first);
            r->copies.pop_front();
            copies_in_flight_--;
        }
    }
}

void Core::poll_epochs()
{
    for (Epoch& e : slots_) {
        if (!e.busy) continue;
        const Poll q = ex_.query(e.ev);
        if (q == kPending) continue;
        for (Req* r : e.reqs) r->epochs_open--;
        if (q == kFailed)
            for (Req* r : e.reqs) fail(r, DR_E_DEVICE);
        else
            for (Req* r : e.finishing) r->totals_done = true;
        ex_.forget(e.ev);
        e.busy = false;
        e.ev = 0;
        e.reqs.clear();
        e.finishing.clear();
    }
}

bool Core::launch_epoch()
{
    if (epochs_in_flight() >= kEpochsInFlight) return false;
    int si = -1;
    for (int i = 0; i < kEpochSlots && si < 0; ++i) {
        const int k = (slot_next_ + i) % kEpochSlots;
        if (!slots_[k].busy) si = k;
    }
    if (si < 0) return false;
    // rows are handed to an epoch only after their copy was seen complete
    std::vector<Segment> segs;
    std::vector<Req*> finishing, reqs;
    for (Req* r : active_) {
        if (r->state != kAdmitted || r->failing || r->finishing) continue;
        bool in = false;
        if (r->rows_ready > r->rows_next) {
            segs.push_back({r, r->rows_next, r->rows_ready});
            in = true;
        }
        if (r->rows_ready == r->ny) {  // every row launched by the end of this epoch
            finishing.push_back(r);
            in = true;
        }
        if (in) reqs.push_back(r);
    }
    if (reqs.empty()) return false;
    Event ev = 0;
    const dr_status st = ex_.launch_epoch(si, segs, finishing, &ev);
    if (st != DR_OK) {  // the executor has drained what it enqueued
        for (Req* r : reqs) fail(r, st);
        return false;
    }
    for (const Segment& s : segs) {
        s.r->rows_next = s.row_end;
        c_.rows_launched += (uint64_t)(s.row_end - s.row_begin);
    }
    Epoch& e = slots_[si];
    e.busy = true;
    e.ev = ev;
    e.seq = epoch_seq_++;
    e.reqs = reqs;
    e.finishing = finishing;
    for (Req* r : reqs) r->epochs_open++;
    for (Req* r : finishing) r->finishing = true;
    slot_next_ = (si + 1) % kEpochSlots;
    c_.epochs++;
    return true;
}

void Core::retire()
{
    for (size_t i = 0; i < active_.size();) {
        Req* r = active_[i];
        // nothing of it in flight: no copy, no epoch that reads its buffers
        const bool drained = r->copies.empty() && r->epochs_open == 0;
        const bool done = r->finishing && r->totals_done;
        if (drained && (r->failing || done)) {
            if (!r->released) {
                ex_.release(*r);
                r->released = true;
            }
            c_.in_use -= r->footprint;
            if (r->failing) {
                r->state = kFailedState;
                r->result = r->fail_code;
                c_.failed++;
            } else {
                r->state = kComplete;
                r->result = DR_OK;
                c_.completed++;
            }
            ex_.finished(*r);
            active_.erase(active_.begin() + (long)i);
        } else {
            ++i;
        }
    }
}

bool Core::step()
{
    admit();
    issue_copies();
    poll_copies();
    poll_epochs();
    while (launch_epoch()) {
    }
    retire();
    return copies_in_flight_ > 0 || epochs_in_flight() > 0;
}

}  // namespace sched
}  // namespace dr
