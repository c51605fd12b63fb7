// Host-side scheduling of a serving session (rs_session_* of include/rs.h):
// request states, the partial-sum arena, admission, the work of each time
// slice and retirement.  Plain C++17 with no HIP: rs_session.hip drives it
// from its scheduler thread with the device's completions, and the host
// tests drive it with synthetic ones (under AddressSanitizer and
// UndefinedBehaviorSanitizer).  Not thread-safe: the caller serialises every
// call (the session holds its mutex).
//
// Model.  A request is an amount of work made of `items` work items (pixel
// chunk x channel x tile), each `steps` 16-pixel steps long; a slice gives a
// request a segment of steps [seg_begin, seg_end) of all its items, with
// segments starting on 256-pixel (16-step) boundaries.  The session runs a
// slice as persistent launches, then calls retire(); a request whose last
// segment is in a slice completes with it.
//
// Policies.
//   Admission: requests are admitted in arrival order while a slot is free
//   and their partial sums fit the arena (first fit).  A request that does
//   not fit may be overtaken by later ones that do, at most `max_bypass`
//   times; after that nothing is admitted past it until it fits, so it
//   cannot starve (max_bypass = 0 is strict arrival order).
//   Shares: a slice carries at most `slice_terms` terms.  EQUAL gives every
//   admitted request with work left an equal share of slice_terms (a slice
//   is shorter when the requests' remaining work is smaller than their
//   shares).  SHORTEST makes the slice as large as EQUAL would and gives it
//   to the requests with the least work left first (shortest remaining
//   processing time), after a floor of `min_share` of an equal share for
//   every request so that none stalls.
#pragma once

#include "../../include/rs.h"

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

namespace rs_sched {

enum { SHORTEST = RS_SCHED_SHORTEST, EQUAL = RS_SCHED_EQUAL };

constexpr int32_t kBlockSteps = 16;  // steps per 256-pixel parameter block

struct Options {
    size_t budget = 0;          // arena bytes
    int32_t max_slots = 1;      // requests admitted at once
    int32_t queue_cap = 1;      // requests queued before submit gives RS_E_BUSY
    int32_t slice_items = 0;    // > 0: each request's segment covers about this many item-blocks
    int32_t policy = SHORTEST;  // EQUAL or SHORTEST
    int32_t max_bypass = 64;    // admissions that may overtake a request that does not fit
    double slice_terms = 1.2e11;
    double min_share = 0.125;   // SHORTEST: floor per request, as a fraction of an equal share
};

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
  public:
    void init(size_t size)
    {
        free_.clear();
        size_ = size;
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round(n);
        if (!n) return;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const
    {
        size_t t = 0;
        for (const auto &f : free_) t += f.second;
        return t;
    }
    size_t size() const { return size_; }
    static size_t round(size_t n) { return (n + 255) & ~(size_t)255; }
    const std::map<size_t, size_t> &free_list() const { return free_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    int32_t state = RS_REQ_QUEUED;
    rs_timing tm{};
    // work
    int64_t items = 0;          // work items
    int32_t steps = 0;          // 16-pixel steps of a full chunk
    int32_t cursor = 0;         // next step to give out
    double step_terms = 0;      // terms of one step of one work item
    double terms = 0;           // whole request
    size_t footprint = 0;       // arena bytes (partial sums, chunk scales)
    size_t request_bytes = 0;   // pixels + cube + partial sums in HBM (reported)
    size_t arena_off = 0;
    int32_t bypassed = 0;       // admissions that overtook it
    int32_t slot = -1;          // while admitted: its slot, 0 .. max_slots-1
    bool started = false;       // a segment of it has been given out
    bool issued_all = false;    // every segment given out
    bool failed = false;
    // the session's payload (not used by the scheduler)
    const rs_plan *plan = nullptr;
    rs_pixels px{};
    void *cube = nullptr;
    int32_t S = 0, chunk = 0;   // pixel chunks and pixels per chunk

    double remaining_terms() const { return (double)(steps - cursor) * step_terms * (double)items; }
};

struct Part {
    Request *r;
    int32_t seg_begin, seg_end;  // steps of every work item
    bool first;                  // the request's first segment
};

struct Slice {
    std::vector<Part> parts;
    std::vector<Request *> completing;  // requests whose last segment is in the slice
};

struct Stats {
    int64_t submitted = 0, admitted = 0, done = 0, failed = 0, cancelled = 0, slices = 0;
    size_t footprint_now = 0, footprint_peak = 0;
    size_t request_bytes_now = 0, request_bytes_peak = 0;
    double terms_done = 0;
};

class Scheduler {
  public:
    explicit Scheduler(const Options &o) : opt_(o), slot_used_((size_t)std::max(o.max_slots, 1), false)
    {
        arena_.init(o.budget);
    }

    const Options &options() const { return opt_; }
    const Stats &stats() const { return st_; }
    size_t queued() const { return queue_.size(); }
    size_t running() const { return active_.size(); }
    const Arena &arena() const { return arena_; }
    const std::vector<Request *> &active() const { return active_; }
    bool stopped() const { return !error_.empty(); }
    const std::string &error() const { return error_; }

    // Queue a request (ticket assigned here).  RS_E_INVALID: its footprint
    // can never fit the budget; RS_E_BUSY: queue full; RS_E_DEVICE: the
    // session stopped after a device error.
    rs_status submit(std::unique_ptr<Request> r, int64_t now, uint64_t *ticket)
    {
        if (!error_.empty()) return RS_E_DEVICE;
        if (Arena::round(r->footprint) > opt_.budget) return RS_E_INVALID;
        if ((int64_t)queue_.size() >= opt_.queue_cap) return RS_E_BUSY;
        r->ticket = next_ticket_++;
        r->state = RS_REQ_QUEUED;
        r->tm.t_submit_ns = now;
        *ticket = r->ticket;
        queue_.push_back(r.get());
        all_[r->ticket] = std::move(r);
        st_.submitted++;
        return RS_OK;
    }

    Request *find(uint64_t ticket)
    {
        auto it = all_.find(ticket);
        return it == all_.end() ? nullptr : it->second.get();
    }

    // RS_E_NOT_FOUND, or RS_E_BUSY when it is no longer queued.
    rs_status cancel(uint64_t ticket, int64_t now)
    {
        Request *r = find(ticket);
        if (!r) return RS_E_NOT_FOUND;
        if (r->state != RS_REQ_QUEUED) return RS_E_BUSY;
        queue_.erase(std::find(queue_.begin(), queue_.end(), r));
        r->state = RS_REQ_CANCELLED;
        r->tm.t_done_ns = now;
        st_.cancelled++;
        return RS_OK;
    }

    // Admission (see the policy above).
    void admit(int64_t now)
    {
        if (!error_.empty()) return;
        for (auto it = queue_.begin(); it != queue_.end() && (int32_t)active_.size() < opt_.max_slots;) {
            Request *r = *it;
            size_t off = 0;
            if (r->footprint > 0 && !arena_.alloc(r->footprint, &off)) {
                // r waits; later requests may overtake it a bounded number of times
                if (r->bypassed >= opt_.max_bypass) break;
                bool overtaken = false;
                for (auto jt = std::next(it); jt != queue_.end() && (int32_t)active_.size() < opt_.max_slots;) {
                    Request *q = *jt;
                    size_t o2 = 0;
                    if (q->footprint == 0 || arena_.alloc(q->footprint, &o2)) {
                        jt = queue_.erase(jt);
                        start(q, o2, now);
                        overtaken = true;
                        if (++r->bypassed >= opt_.max_bypass) break;
                    } else {
                        ++jt;
                    }
                }
                (void)overtaken;
                break;
            }
            it = queue_.erase(it);
            start(r, off, now);
        }
    }

    bool has_work() const
    {
        for (const Request *r : active_)
            if (!r->issued_all) return true;
        return false;
    }

    // The next slice: segments of the admitted requests with work left.
    Slice next_slice()
    {
        Slice sl;
        std::vector<Request *> pend;
        for (Request *r : active_)
            if (!r->issued_all) pend.push_back(r);
        if (pend.empty()) return sl;
        std::vector<int64_t> seg(pend.size(), 0);  // steps given to each
        if (opt_.slice_items > 0) {
            for (size_t i = 0; i < pend.size(); ++i)
                seg[i] = (int64_t)opt_.slice_items * kBlockSteps / std::max<int64_t>(1, pend[i]->items);
        } else if (opt_.policy == EQUAL) {
            const double share = opt_.slice_terms / (double)pend.size();
            for (size_t i = 0; i < pend.size(); ++i) seg[i] = steps_for(pend[i], share);
        } else {
            // The slice is as large as equal shares would make it (so a slice
            // with little work left in it stays short and the next one starts
            // soon); a floor for everyone, then the rest to the least work
            // left first.
            const double share = opt_.slice_terms / (double)pend.size();
            double budget = 0.0;
            for (const Request *r : pend) budget += std::min(r->remaining_terms(), share);
            const double floor_terms = opt_.min_share * share;
            double left = budget;
            for (size_t i = 0; i < pend.size(); ++i) {
                seg[i] = clamp_steps(pend[i], steps_for(pend[i], floor_terms));
                left -= given_terms(pend[i], seg[i]);
            }
            std::vector<size_t> order(pend.size());
            for (size_t i = 0; i < order.size(); ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
                return pend[a]->remaining_terms() < pend[b]->remaining_terms();
            });
            for (size_t k = 0; k < order.size() && left > 0; ++k) {
                const size_t i = order[k];
                const int32_t room = pend[i]->steps - pend[i]->cursor;
                if (seg[i] >= room) continue;
                const int64_t before = seg[i];
                seg[i] = clamp_steps(pend[i], seg[i] + steps_for(pend[i], left));
                left -= given_terms(pend[i], seg[i]) - given_terms(pend[i], before);
            }
        }
        for (size_t i = 0; i < pend.size(); ++i) {
            Request *r = pend[i];
            const int64_t s = clamp_steps(r, seg[i]);
            Part p{r, r->cursor, (int32_t)(r->cursor + s), !r->started};
            r->started = true;
            r->cursor += (int32_t)s;
            if (r->items > 0 && s > 0) sl.parts.push_back(p);
            if (r->cursor >= r->steps) {  // includes P = 0 (no items, zero cube)
                r->issued_all = true;
                sl.completing.push_back(r);
            }
        }
        st_.slices++;
        return sl;
    }

    // The slice's work failed to launch: every request with a part in it
    // fails, gets no further slices and completes with this slice.
    void fail_slice(Slice &sl)
    {
        for (auto &p : sl.parts) {
            p.r->failed = true;
            if (!p.r->issued_all) {
                p.r->issued_all = true;
                p.r->cursor = p.r->steps;
                sl.completing.push_back(p.r);
            }
        }
        for (Request *r : sl.completing) r->failed = true;
    }

    // The device finished the slice: its completing requests end DONE (or
    // FAILED) and free their arena ranges.
    void retire(const Slice &sl, int64_t now)
    {
        for (Request *r : sl.completing) finish(r, r->failed ? RS_REQ_FAILED : RS_REQ_DONE, now);
    }

    // A device error: every admitted and queued request ends FAILED, the
    // arena is released, and nothing more is admitted or accepted.  Slices
    // still counted in flight are then retired as no-ops by the caller.
    void fail_all(const std::string &why, int64_t now)
    {
        if (error_.empty()) error_ = why.empty() ? std::string("device error") : why;
        std::vector<Request *> act = active_;
        for (Request *r : act) {
            r->failed = true;
            r->issued_all = true;
            finish(r, RS_REQ_FAILED, now);
        }
        while (!queue_.empty()) {
            Request *r = queue_.front();
            queue_.pop_front();
            r->state = RS_REQ_FAILED;
            r->tm.t_done_ns = now;
            st_.failed++;
        }
    }

  private:
    void start(Request *r, size_t off, int64_t now)
    {
        r->slot = (int32_t)(std::find(slot_used_.begin(), slot_used_.end(), false) - slot_used_.begin());
        slot_used_[(size_t)r->slot] = true;
        r->arena_off = off;
        r->state = RS_REQ_RUNNING;
        r->tm.t_admit_ns = now;
        active_.push_back(r);
        st_.admitted++;
        st_.footprint_now += Arena::round(r->footprint);
        st_.footprint_peak = std::max(st_.footprint_peak, st_.footprint_now);
        st_.request_bytes_now += r->request_bytes;
        st_.request_bytes_peak = std::max(st_.request_bytes_peak, st_.request_bytes_now);
    }

    void finish(Request *r, int32_t state, int64_t now)
    {
        auto it = std::find(active_.begin(), active_.end(), r);
        if (it == active_.end()) return;  // already finished
        active_.erase(it);
        slot_used_[(size_t)r->slot] = false;
        r->slot = -1;
        r->state = state;
        r->tm.t_done_ns = now;
        arena_.release(r->arena_off, r->footprint);
        st_.footprint_now -= Arena::round(r->footprint);
        st_.request_bytes_now -= r->request_bytes;
        if (state == RS_REQ_FAILED) {
            st_.failed++;
        } else {
            st_.done++;
            st_.terms_done += r->terms;
        }
    }

    // whole 16-step blocks worth about `terms` (at least one block)
    static int64_t steps_for(const Request *r, double terms)
    {
        const double per_step = std::max(1.0, r->step_terms * (double)r->items);
        int64_t s = (int64_t)(terms / per_step);
        return std::max<int64_t>(kBlockSteps, (s / kBlockSteps) * kBlockSteps);
    }
    static int64_t clamp_steps(const Request *r, int64_t s)
    {
        const int64_t room = r->steps - r->cursor;
        s = std::max<int64_t>(kBlockSteps, (s / kBlockSteps) * kBlockSteps);
        return s >= room ? room : s;
    }
    static double given_terms(const Request *r, int64_t s) { return (double)s * r->step_terms * (double)r->items; }

    Options opt_;
    Arena arena_;
    std::deque<Request *> queue_;
    std::vector<Request *> active_;
    std::vector<bool> slot_used_;
    std::map<uint64_t, std::unique_ptr<Request>> all_;
    uint64_t next_ticket_ = 1;
    Stats st_;
    std::string error_;
};

}  // namespace rs_sched
