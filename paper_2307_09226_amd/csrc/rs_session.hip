// Serving loop with continuous batching (rs_session_* of include/rs.h).
//
// A scheduler thread owns one HIP stream and a device arena for the split-K
// partial sums of admitted requests.  Each iteration it
//   1. admits queued requests in arrival order while a slot is free and the
//      request's partial-sum footprint fits in the arena (first fit);
//   2. takes a time slice of work items from every admitted request (round
//      robin, an equal share of the slice's terms each, enough items to fill
//      the chip) and runs them as persistent matrix-core launches that mix
//      the requests (one launch per tile shape present);
//   3. enqueues the split-K reduction of every request whose last items are
//      in the slice, records an event, and keeps up to two slices in flight
//      so that the device never waits for the host;
//   4. retires finished slices: requests become DONE, their arena range is
//      freed and the next queued requests can be admitted.
// A request's chunking depends on its own plan and pixel count only and the
// reduction sums chunks in a fixed order, so its cube is bitwise identical
// to rs_beat_synthesize of the same request, whatever runs beside it.
#include "rs_api_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct request {
    uint64_t ticket = 0;
    const rs_plan *plan = nullptr;
    rs_pixels px{};
    void *cube = nullptr;
    int32_t state = RS_REQ_QUEUED;
    rs_timing tm{};
    int32_t S = 0, chunk = 0;
    int64_t items = 0, cursor = 0;
    size_t footprint = 0, arena_off = 0;
    bool failed = false;
    bool issued_all = false;  // every work item (and the reduction) enqueued
    double terms = 0;
    double item_terms = 0;
};

// First-fit allocator over [0, size) in 256-byte units.
struct arena_alloc {
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t size) { free_.clear(); if (size) free_[0] = size; }
    bool alloc(size_t n, size_t *off)
    {
        n = (n + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                size_t rest = it->second - n, o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + 255) & ~(size_t)255;
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
};

constexpr int kRing = 3;         // job-table slots (at most 2 slices in flight)
constexpr int kMaxVariants = 8;  // tile shapes per slice

struct ring_slot {
    rs_job *h_jobs = nullptr;  // pinned host job tables
    rs_job *d_jobs = nullptr;  // device job tables
    int *d_counter = nullptr;  // one counter per launch
    hipEvent_t done = nullptr;
};

struct inflight {
    int slot = 0;
    std::vector<request *> completing;
};

}  // namespace

struct rs_session {
    int device = 0;
    int ncu = 0;
    size_t budget = 0;
    int max_slots = 1, queue_cap = 1, slice_items = 0;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    arena_alloc alloc;
    ring_slot ring[kRing];
    int ring_next = 0;
    int jobs_cap = 0;  // job entries per ring slot

    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<request *> queue;
    std::vector<request *> active;
    std::map<uint64_t, std::unique_ptr<request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    int inject_fail = 0;
    int busy_iters = 0;  // slices enqueued but not retired
    rs_session_stats st{};
    std::thread worker;
    std::string worker_error;
};

namespace {

void retire(rs_session *s, inflight &f)
{
    const int64_t t = now_ns();
    for (request *r : f.completing) {
        r->state = r->failed ? RS_REQ_FAILED : RS_REQ_DONE;
        r->tm.t_done_ns = t;
        s->alloc.release(r->arena_off, r->footprint);
        s->st.footprint_now -= r->footprint;
        s->active.erase(std::find(s->active.begin(), s->active.end(), r));
        if (r->failed) s->st.failed++;
        else {
            s->st.done++;
            s->st.terms_done += r->terms;
        }
    }
    s->busy_iters--;
    s->cv_done.notify_all();
}

void admit(rs_session *s)
{
    while (!s->queue.empty() && (int)s->active.size() < s->max_slots) {
        request *r = s->queue.front();
        size_t off = 0;
        if (r->footprint > 0 && !s->alloc.alloc(r->footprint, &off)) break;  // head-of-line waits
        s->queue.pop_front();
        r->arena_off = off;
        r->state = RS_REQ_RUNNING;
        r->tm.t_admit_ns = now_ns();
        s->active.push_back(r);
        s->st.admitted++;
        s->st.footprint_now += r->footprint;
        s->st.footprint_peak = std::max(s->st.footprint_peak, s->st.footprint_now);
    }
}

struct slice_part {
    request *r;
    int64_t first, count;
};

// Work items of every admitted request for one slice (caller holds mu).
std::vector<slice_part> build_slice(rs_session *s, std::vector<request *> &completing)
{
    std::vector<slice_part> parts;
    std::vector<request *> pend;
    for (request *r : s->active)
        if (!r->issued_all) pend.push_back(r);
    if (pend.empty()) return parts;
    const double target_terms = 1.2e11;  // ~2 ms of matrix-core work
    const double share = target_terms / pend.size();
    const int64_t min_items = std::max<int64_t>(1, (s->ncu + pend.size() - 1) / pend.size());
    int64_t total = 0;
    for (request *r : pend) {
        int64_t q = (int64_t)(share / std::max(1.0, r->item_terms));
        q = std::max(q, min_items);
        if (s->slice_items > 0)
            q = std::min<int64_t>(q, std::max<int64_t>(1, s->slice_items / (int64_t)pend.size()));
        q = std::min(q, r->items - r->cursor);
        if (q > 0) parts.push_back({r, r->cursor, q});
        r->cursor += q;
        total += q;
        if (r->cursor >= r->items) {  // includes P = 0 (no items, zero cube)
            r->issued_all = true;
            completing.push_back(r);
        }
    }
    return parts;
}

void worker_main(rs_session *s)
{
    (void)hipSetDevice(s->device);
    std::deque<inflight> fly;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // retire slices the device has finished
        while (!fly.empty() && hipEventQuery(s->ring[fly.front().slot].done) == hipSuccess) {
            retire(s, fly.front());
            fly.pop_front();
        }
        admit(s);
        bool work = false;
        for (request *r : s->active)
            if (!r->issued_all) work = true;
        if (!work || fly.size() >= 2) {
            if (!fly.empty()) {
                hipEvent_t ev = s->ring[fly.front().slot].done;
                lk.unlock();
                (void)hipEventSynchronize(ev);
                lk.lock();
                continue;
            }
            if (s->stop && s->queue.empty() && s->active.empty()) break;
            s->cv.wait(lk);
            continue;
        }
        std::vector<request *> completing;
        std::vector<slice_part> parts = build_slice(s, completing);
        bool fail = false;
        if (s->inject_fail > 0) {
            s->inject_fail--;
            fail = true;
            for (auto &p : parts) {
                p.r->failed = true;
                if (!p.r->issued_all) {
                    p.r->cursor = p.r->items;
                    p.r->issued_all = true;
                    completing.push_back(p.r);
                }
            }
            for (request *r : completing) r->failed = true;
        }
        const int slot = s->ring_next;
        s->ring_next = (s->ring_next + 1) % kRing;
        s->busy_iters++;
        s->st.launches++;
        lk.unlock();

        // ---- enqueue the slice (no lock held) --------------------------------
        ring_slot &rg = s->ring[slot];
        int nj = 0;
        hipError_t err = hipSuccess;
        if (!fail) {
            // group parts by tile shape: one persistent launch per shape
            std::vector<std::pair<int, int>> shapes;
            for (auto &p : parts) {
                std::pair<int, int> k(p.r->plan->wn, p.r->plan->tl);
                if (std::find(shapes.begin(), shapes.end(), k) == shapes.end()) shapes.push_back(k);
            }
            int launch = 0;
            for (auto &shp : shapes) {
                const int j0 = nj;
                int64_t items = 0;
                for (auto &p : parts) {
                    if (p.r->plan->wn != shp.first || p.r->plan->tl != shp.second) continue;
                    rs_job j = rs_make_job(p.r->plan, &p.r->px, p.r->cube, s->arena + p.r->arena_off,
                                           p.r->S, p.r->chunk);
                    j.item_begin = items;
                    j.item_first = p.first;
                    j.item_count = p.count;
                    items += p.count;
                    rg.h_jobs[nj++] = j;
                }
                rs_launch L;
                std::memset(&L, 0, sizeof L);
                L.jobs = rg.d_jobs + j0;
                L.njobs = nj - j0;
                L.total = items;
                L.counter = rg.d_counter + launch;
                const rs_plan *pl = parts[0].r->plan;
                for (auto &p : parts)
                    if (p.r->plan->wn == shp.first && p.r->plan->tl == shp.second) pl = p.r->plan;
                err = hipMemcpyAsync(rg.d_jobs + j0, rg.h_jobs + j0, (size_t)(nj - j0) * sizeof(rs_job),
                                     hipMemcpyHostToDevice, s->stream);
                if (err != hipSuccess) break;
                rs_launch_zero_int(L.counter, 1, s->stream);
                int64_t grid = std::min<int64_t>(items, (int64_t)s->ncu * pl->occupancy);
                if (rs_launch_main(pl, L, (int)grid, s->stream) != RS_OK) {
                    err = hipErrorLaunchFailure;
                    break;
                }
                launch++;
            }
            // reduction of the requests completed by this slice
            if (err == hipSuccess && !completing.empty()) {
                const int j0 = nj;
                int64_t outs = 0;
                for (request *r : completing) {
                    rs_job j = rs_make_job(r->plan, &r->px, r->cube, s->arena + r->arena_off, r->S,
                                           r->chunk);
                    j.out_begin = outs;
                    outs += (int64_t)r->plan->C * r->plan->L * r->plan->Ns;
                    rg.h_jobs[nj++] = j;
                }
                err = hipMemcpyAsync(rg.d_jobs + j0, rg.h_jobs + j0, (size_t)(nj - j0) * sizeof(rs_job),
                                     hipMemcpyHostToDevice, s->stream);
                if (err == hipSuccess) {
                    rs_launch R;
                    std::memset(&R, 0, sizeof R);
                    R.jobs = rg.d_jobs + j0;
                    R.njobs = nj - j0;
                    R.total = outs;
                    if (rs_launch_reduce_checked(completing[0]->plan, R, s->stream) != RS_OK)
                        err = hipErrorLaunchFailure;
                }
            }
        }
        if (err != hipSuccess) {
            for (auto &p : parts) {
                p.r->failed = true;
                if (!p.r->issued_all) {
                    completing.push_back(p.r);
                    p.r->cursor = p.r->items;
                    p.r->issued_all = true;
                }
            }
        }
        (void)hipEventRecord(rg.done, s->stream);
        lk.lock();
        fly.push_back(inflight{slot, completing});
    }
}

}  // namespace

extern "C" rs_status rs_session_create(const rs_session_opts *o, rs_session **out)
{
    if (!out) return rs_fail(RS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!o) return rs_fail(RS_E_INVALID, "opts is NULL");
    if (o->max_slots < 1 || o->max_slots > 4096) return rs_fail(RS_E_INVALID, "max_slots out of range");
    if (o->queue_cap < 1) return rs_fail(RS_E_INVALID, "queue_cap < 1");
    if (o->slice_items < 0) return rs_fail(RS_E_INVALID, "slice_items < 0");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || o->device < 0 || o->device >= ndev)
        return rs_fail(RS_E_INVALID, "bad device %d", o->device);
    std::unique_ptr<rs_session> s(new (std::nothrow) rs_session());
    if (!s) return rs_fail(RS_E_NOMEM, "host allocation failed");
    s->device = o->device;
    s->budget = (o->hbm_budget + 255) & ~(size_t)255;
    s->max_slots = o->max_slots;
    s->queue_cap = o->queue_cap;
    s->slice_items = o->slice_items;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(s->device) != hipSuccess) return rs_fail(RS_E_DEVICE, "hipSetDevice failed");
    rs_status status = RS_OK;
    do {
        if (hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess) {
            status = rs_fail(RS_E_DEVICE, "cannot query compute units");
            break;
        }
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            status = rs_fail(RS_E_DEVICE, "stream creation failed");
            break;
        }
        if (s->budget && hipMalloc(&s->arena, s->budget) != hipSuccess) {
            status = rs_fail(RS_E_NOMEM, "arena allocation of %zu bytes failed", s->budget);
            break;
        }
        s->alloc.init(s->budget);
        s->jobs_cap = s->max_slots * (kMaxVariants + 1);
        for (auto &rg : s->ring) {
            if (hipHostMalloc(reinterpret_cast<void **>(&rg.h_jobs), sizeof(rs_job) * s->jobs_cap,
                              hipHostMallocDefault) != hipSuccess ||
                hipMalloc(&rg.d_jobs, sizeof(rs_job) * s->jobs_cap) != hipSuccess ||
                hipMalloc(&rg.d_counter, sizeof(int) * 64) != hipSuccess ||
                hipEventCreateWithFlags(&rg.done, hipEventDisableTiming) != hipSuccess) {
                status = rs_fail(RS_E_NOMEM, "session ring allocation failed");
                break;
            }
        }
    } while (0);
    if (status == RS_OK) {
        rs_session *raw = s.get();
        try {
            s->worker = std::thread(worker_main, raw);
        } catch (...) {
            status = rs_fail(RS_E_NOMEM, "cannot start the scheduler thread");
        }
    }
    if (status != RS_OK) {
        for (auto &rg : s->ring) {
            if (rg.h_jobs) (void)hipHostFree(rg.h_jobs);
            if (rg.d_jobs) (void)hipFree(rg.d_jobs);
            if (rg.d_counter) (void)hipFree(rg.d_counter);
            if (rg.done) (void)hipEventDestroy(rg.done);
        }
        if (s->arena) (void)hipFree(s->arena);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        (void)hipSetDevice(prev);
        return status;
    }
    (void)hipSetDevice(prev);
    *out = s.release();
    return RS_OK;
}

extern "C" rs_status rs_session_submit(rs_session *s, const rs_plan *pl, const rs_pixels *px,
                                       void *cube, uint64_t *ticket)
{
    if (!s || !pl || !cube || !ticket) return rs_fail(RS_E_INVALID, "NULL argument");
    if (pl->form != RS_FORM_MFMA_SPLIT16)
        return rs_fail(RS_E_UNSUPPORTED, "sessions serve RS_FORM_MFMA_SPLIT16 plans");
    if (pl->device != s->device) return rs_fail(RS_E_INVALID, "plan is on another device");
    rs_status st = rs_check_pixels(pl, px);
    if (st != RS_OK) return st;
    auto r = std::make_unique<request>();
    r->plan = pl;
    r->px = *px;
    r->cube = cube;
    if ((st = rs_plan_chunking(pl, px->P, &r->S, &r->chunk)) != RS_OK) return st;
    r->items = (int64_t)r->S * pl->C * pl->n_tiles * pl->l_tiles;
    r->footprint = rs_partial_bytes(pl, r->S);
    r->terms = (double)px->P * pl->C * pl->L * pl->Ns;
    r->item_terms = (double)r->chunk * pl->tn * pl->tl;
    if (r->footprint > s->budget)
        return rs_fail(RS_E_INVALID, "request needs %zu bytes of workspace, session budget is %zu",
                       r->footprint, s->budget);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return rs_fail(RS_E_INVALID, "session is shutting down");
    if ((int)s->queue.size() >= s->queue_cap) return rs_fail(RS_E_BUSY, "queue full");
    r->ticket = s->next_ticket++;
    r->tm.t_submit_ns = now_ns();
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->all[r->ticket] = std::move(r);
    s->st.submitted++;
    s->cv.notify_all();
    return RS_OK;
}

extern "C" rs_status rs_session_poll(rs_session *s, uint64_t ticket, int32_t *state, rs_timing *tm)
{
    if (!s || !state) return rs_fail(RS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return rs_fail(RS_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    *state = it->second->state;
    if (tm) *tm = it->second->tm;
    return RS_OK;
}

extern "C" rs_status rs_session_cancel(rs_session *s, uint64_t ticket)
{
    if (!s) return rs_fail(RS_E_INVALID, "NULL session");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return rs_fail(RS_E_NOT_FOUND, "unknown ticket");
    request *r = it->second.get();
    if (r->state != RS_REQ_QUEUED) return rs_fail(RS_E_BUSY, "request already admitted or finished");
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
    r->state = RS_REQ_CANCELLED;
    r->tm.t_done_ns = now_ns();
    s->st.cancelled++;
    s->cv.notify_all();
    s->cv_done.notify_all();
    return RS_OK;
}

extern "C" rs_status rs_session_drain(rs_session *s)
{
    if (!s) return rs_fail(RS_E_INVALID, "NULL session");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->queue.empty() && s->active.empty() && s->busy_iters == 0; });
    return RS_OK;
}

extern "C" rs_status rs_session_stats_get(rs_session *s, rs_session_stats *out)
{
    if (!s || !out) return rs_fail(RS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->st;
    out->queued_now = (int64_t)s->queue.size();
    out->running_now = (int64_t)s->active.size();
    return RS_OK;
}

extern "C" rs_status rs_session_inject_failure(rs_session *s, int32_t count)
{
    if (!s || count < 0) return rs_fail(RS_E_INVALID, "bad argument");
    std::lock_guard<std::mutex> g(s->mu);
    s->inject_fail += count;
    return RS_OK;
}

extern "C" void rs_session_destroy(rs_session *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto &rg : s->ring) {
        if (rg.h_jobs) (void)hipHostFree(rg.h_jobs);
        if (rg.d_jobs) (void)hipFree(rg.d_jobs);
        if (rg.d_counter) (void)hipFree(rg.d_counter);
        if (rg.done) (void)hipEventDestroy(rg.done);
    }
    if (s->arena) (void)hipFree(s->arena);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    (void)hipSetDevice(prev);
    delete s;
}
