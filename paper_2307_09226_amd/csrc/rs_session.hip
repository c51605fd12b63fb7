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
    int64_t items = 0;
    int32_t steps = 0;        // 16-pixel steps of a full chunk
    int32_t cursor = 0;       // next step segment to enqueue
    bool scaled = false;      // per-chunk strength scales enqueued
    size_t footprint = 0, arena_off = 0;
    bool failed = false;
    bool issued_all = false;  // every work item (and the reduction) enqueued
    double terms = 0;
    double step_terms = 0;    // terms of one 16-pixel step of one work item
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
    int32_t seg_begin, seg_end;  // 16-pixel steps of every chunk
    bool scale;                  // enqueue the request's chunk scales first
};

// Work of every admitted request for one slice (caller holds mu): all work
// items of a request over a segment of steps sized to an equal share of the
// slice (segments start at 256-pixel boundaries).
std::vector<slice_part> build_slice(rs_session *s, std::vector<request *> &completing)
{
    constexpr int kBlockSteps = 16;
    std::vector<slice_part> parts;
    std::vector<request *> pend;
    for (request *r : s->active)
        if (!r->issued_all) pend.push_back(r);
    if (pend.empty()) return parts;
    const double target_terms = s->slice_items > 0 ? 0.0 : 1.2e11;  // ~2 ms of matrix-core work
    const double share = target_terms / pend.size();
    for (request *r : pend) {
        const int32_t left = r->steps - r->cursor;
        int64_t seg;
        if (s->slice_items > 0) {
            seg = (int64_t)s->slice_items * kBlockSteps / std::max<int64_t>(1, r->items);
        } else {
            const double per_step = std::max(1.0, r->step_terms * (double)r->items);
            seg = (int64_t)(share / per_step);
        }
        seg = std::max<int64_t>(kBlockSteps, (seg / kBlockSteps) * kBlockSteps);
        if (seg >= left) seg = left;
        slice_part p{r, r->cursor, (int32_t)(r->cursor + seg), !r->scaled};
        r->scaled = true;
        r->cursor += (int32_t)seg;
        if (r->items > 0 && seg > 0) parts.push_back(p);
        if (r->cursor >= r->steps) {  // includes P = 0 (no items, zero cube)
            r->issued_all = true;
            completing.push_back(r);
        }
    }
    return parts;
}

// Enqueue one slice on the session stream: chunk scales of newly started
// requests, one persistent launch per tile shape, reductions of the requests
// completed by the slice.  One host-to-device copy carries all job tables.
hipError_t enqueue_slice(rs_session *s, ring_slot &rg, const std::vector<slice_part> &parts,
                         const std::vector<request *> &completing)
{
    int nj = 0;
    // chunk-scale jobs
    const int js = nj;
    int64_t chunks = 0;
    bool scale_bs = false;  // some new request has strengths per block
    for (const auto &p : parts) {
        // chunk scales of requests with strengths per block (the main kernel
        // finds the others itself)
        if (!p.scale || !(p.r->plan->model & RS_MODEL_BLOCK_STRENGTH)) continue;
        rs_job j = rs_make_job(p.r->plan, &p.r->px, p.r->cube, s->arena + p.r->arena_off, p.r->S,
                               p.r->chunk);
        j.chunk_begin = chunks;
        chunks += p.r->S;
        if (j.amp_lstride) scale_bs = true;
        rg.h_jobs[nj++] = j;
    }
    const int nscale = nj - js;
    // main jobs grouped by tile shape
    struct group {
        int wn, tl, nw, il, j0, n;
        int64_t items;
        const rs_plan *pl;
        bool block_strength;  // some request of the group has strengths per block
    };
    std::vector<group> groups;
    for (const auto &p : parts) {
        bool found = false;
        for (auto &g : groups)
            if (g.wn == p.r->plan->wn && g.tl == p.r->plan->tl && g.nw == p.r->plan->nw &&
                g.il == p.r->plan->interleave)
                found = true;
        if (!found)
            groups.push_back(group{p.r->plan->wn, p.r->plan->tl, p.r->plan->nw, p.r->plan->interleave, 0, 0, 0,
                                   p.r->plan, false});
    }
    for (auto &g : groups) {
        g.j0 = nj;
        for (const auto &p : parts) {
            if (p.r->plan->wn != g.wn || p.r->plan->tl != g.tl || p.r->plan->nw != g.nw ||
                p.r->plan->interleave != g.il)
                continue;
            rs_job j = rs_make_job(p.r->plan, &p.r->px, p.r->cube, s->arena + p.r->arena_off,
                                   p.r->S, p.r->chunk);
            j.item_begin = g.items;
            j.item_first = 0;
            j.item_count = p.r->items;
            j.seg_begin = p.seg_begin;
            j.seg_end = p.seg_end;
            g.items += p.r->items;
            if (j.amp_lstride) g.block_strength = true;
            rg.h_jobs[nj++] = j;
        }
        g.n = nj - g.j0;
    }
    // reduction jobs
    const int jr = nj;
    int64_t outs = 0;
    for (request *r : completing) {
        rs_job j = rs_make_job(r->plan, &r->px, r->cube, s->arena + r->arena_off, r->S, r->chunk);
        j.out_begin = outs;
        outs += (int64_t)r->plan->C * r->plan->L * r->plan->Ns;
        rg.h_jobs[nj++] = j;
    }
    const int nred = nj - jr;
    if (nj == 0) return hipSuccess;
    hipError_t err = hipMemcpyAsync(rg.d_jobs, rg.h_jobs, (size_t)nj * sizeof(rs_job),
                                    hipMemcpyHostToDevice, s->stream);
    if (err != hipSuccess) return err;
    if (nscale > 0) {
        rs_launch Sc;
        std::memset(&Sc, 0, sizeof Sc);
        Sc.jobs = rg.d_jobs + js;
        Sc.njobs = nscale;
        Sc.total = chunks;
        if (rs_launch_scale_checked(Sc, scale_bs, s->stream) != RS_OK) return hipErrorLaunchFailure;
    }
    int launch = 0;
    for (auto &g : groups) {
        if (g.items <= 0) continue;
        rs_launch L;
        std::memset(&L, 0, sizeof L);
        L.jobs = rg.d_jobs + g.j0;
        L.njobs = g.n;
        L.total = g.items;
        L.counter = rg.d_counter + launch++;
        rs_launch_zero_int(L.counter, 1, s->stream);
        const int64_t grid = std::min<int64_t>(g.items, (int64_t)s->ncu * g.pl->occupancy);
        if (rs_launch_main(g.pl, L, g.block_strength, (int)grid, s->stream) != RS_OK) return hipErrorLaunchFailure;
    }
    if (nred > 0) {
        rs_launch R;
        std::memset(&R, 0, sizeof R);
        R.jobs = rg.d_jobs + jr;
        R.njobs = nred;
        R.total = outs;
        if (rs_launch_reduce_checked(completing[0]->plan, R, s->stream) != RS_OK)
            return hipErrorLaunchFailure;
    }
    return hipSuccess;
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
        }
        const int slot = s->ring_next;
        s->ring_next = (s->ring_next + 1) % kRing;
        s->busy_iters++;
        s->st.launches++;
        lk.unlock();

        ring_slot &rg = s->ring[slot];
        hipError_t err = fail ? hipErrorLaunchFailure : enqueue_slice(s, rg, parts, completing);
        (void)hipEventRecord(rg.done, s->stream);

        lk.lock();
        if (err != hipSuccess) {
            // every request with work in this slice fails; it retires with
            // this slice (no further work of it is enqueued)
            for (auto &p : parts) {
                p.r->failed = true;
                if (!p.r->issued_all) {
                    p.r->issued_all = true;
                    p.r->cursor = p.r->steps;
                    completing.push_back(p.r);
                }
            }
            for (request *r : completing) r->failed = true;
        }
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
    r->steps = r->S > 0 ? rs_steps_per_chunk(pl, r->chunk) : 0;
    r->footprint = rs_workspace_bytes(pl, r->S);
    r->terms = (double)px->P * pl->C * pl->L * pl->Ns;
    r->step_terms = 16.0 * pl->tn * pl->tl;
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
