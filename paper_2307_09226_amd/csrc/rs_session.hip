// Serving loop with continuous batching (rs_session_* of include/rs.h).
//
// A scheduler thread owns one HIP stream and a device arena for the split-K
// partial sums of admitted requests; the policy decisions (admission, the
// shares of each time slice, retirement, failure) live in rs_sched.h, plain
// C++ that the host tests drive with synthetic completions.  Each iteration
// the thread
//   1. retires the slices the device has finished (their completing
//      requests become DONE, their arena ranges are freed);
//   2. admits queued requests (rs_sched::Scheduler::admit);
//   3. takes the next slice of work from the admitted requests and runs it
//      as persistent matrix-core launches that mix the requests (one launch
//      per tile configuration present), then the split-K reduction of every
//      request whose last segment is in the slice, and records an event --
//      keeping up to two slices in flight so that the device never waits
//      for the host.
// A device error seen at a completion check stops the session: every
// admitted and queued request fails, and later submits are refused.
// A request's chunking depends on its own plan and pixel count only and the
// reduction sums chunks in a fixed order, so its cube is bitwise identical
// to rs_beat_synthesize of the same request, whatever runs beside it.
#include "rs_api_internal.h"
#include "rs_sched.h"

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

constexpr int kRing = 3;         // job-table slots (at most 2 slices in flight)
constexpr int kMaxVariants = 8;  // job entries per request and slot: room for scale, main and reduce jobs
constexpr int kMaxGroups = 16;   // tile configurations per slice (the library builds 11)
constexpr int kSide = 3;         // streams on which a slice's configurations run side by side

struct ring_slot {
    rs_job *h_jobs = nullptr;  // pinned host job tables
    rs_job *d_jobs = nullptr;  // device job tables
    int *d_counter = nullptr;  // one counter per launch
    hipEvent_t done = nullptr;
    hipEvent_t start = nullptr;            // job tables and chunk scales of the slice ready
    hipEvent_t grp[kMaxGroups] = {};       // a configuration's launch finished
};

struct inflight {
    int slot = 0;
    rs_sched::Slice slice;
};

}  // namespace

struct rs_session {
    int device = 0;
    int ncu = 0;
    hipStream_t stream = nullptr;
    hipStream_t side[kSide] = {};
    int32_t *scales = nullptr;  // chunk-scale pool: max_slots rows of scale_row exponents
    size_t scale_row = 0;
    char *arena = nullptr;
    ring_slot ring[kRing];
    int ring_next = 0;
    int jobs_cap = 0;  // job entries per ring slot

    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::unique_ptr<rs_sched::Scheduler> sched;
    bool stop = false;
    int inject_fail = 0;
    bool inject_device_error = false;
    int busy_iters = 0;  // slices enqueued but not retired
    int64_t launches = 0;
    std::thread worker;
};

namespace {

// A request's job: its partial sums in its arena range and its chunk scales
// in its slot's row of the scale pool.  In a session every request's chunk
// scales come from one k_chunk_scale pass when it starts (a work item would
// otherwise find its chunk's scale again in every segment).
rs_job session_job(rs_session *s, const rs_sched::Request *r)
{
    rs_job j = rs_make_job(r->plan, &r->px, r->cube, s->arena + r->arena_off, r->S, r->chunk);
    j.scale = s->scales + (size_t)r->slot * s->scale_row;
    return j;
}

// Enqueue one slice on the session stream: chunk scales of newly started
// requests, one persistent launch per tile shape, reductions of the requests
// completed by the slice.  One host-to-device copy carries all job tables.
hipError_t enqueue_slice(rs_session *s, ring_slot &rg, const rs_sched::Slice &sl)
{
    const std::vector<rs_sched::Part> &parts = sl.parts;
    const std::vector<rs_sched::Request *> &completing = sl.completing;
    int nj = 0;
    // chunk-scale jobs
    const int js = nj;
    int64_t chunks = 0;
    bool scale_bs = false;  // some new request has strengths per block
    for (const auto &p : parts) {
        // chunk scales of the requests that start in this slice
        if (!p.first) continue;
        rs_job j = session_job(s, p.r);
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
            rs_job j = session_job(s, p.r);
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
    for (rs_sched::Request *r : completing) {
        rs_job j = session_job(s, r);
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
    // Several tile configurations in one slice run side by side on the side
    // streams (each launch's tail, where its last work items leave compute
    // units idle, overlaps the others' work); each starts after the slice's
    // job tables and chunk scales, and the reductions wait for all of them.
    // The next slice starts behind those reductions on the session stream,
    // so a request's segments stay in order.
    int ngroups = 0;
    for (auto &g : groups) ngroups += g.items > 0;
    const bool side = ngroups > 1;
    if (side && (err = hipEventRecord(rg.start, s->stream)) != hipSuccess) return err;
    int launch = 0;
    for (auto &g : groups) {
        if (g.items <= 0) continue;
        if (launch >= kMaxGroups) return hipErrorLaunchFailure;
        hipStream_t st = side ? s->side[launch % kSide] : s->stream;
        if (side && (err = hipStreamWaitEvent(st, rg.start, 0)) != hipSuccess) return err;
        rs_launch L;
        std::memset(&L, 0, sizeof L);
        L.jobs = rg.d_jobs + g.j0;
        L.njobs = g.n;
        L.total = g.items;
        L.counter = rg.d_counter + launch;
        rs_launch_zero_int(L.counter, 1, st);
        const int64_t grid = std::min<int64_t>(g.items, (int64_t)s->ncu * g.pl->occupancy);
        if (rs_launch_main(g.pl, L, g.block_strength, (int)grid, st) != RS_OK) return hipErrorLaunchFailure;
        if (side) {
            if ((err = hipEventRecord(rg.grp[launch], st)) != hipSuccess) return err;
            if ((err = hipStreamWaitEvent(s->stream, rg.grp[launch], 0)) != hipSuccess) return err;
        }
        ++launch;
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

// The device's verdict on a slice's completion event: done, not yet, or a
// device error (any status other than success or not-ready; the injected
// test error counts as one).
enum class ev_state { done, pending, error };

ev_state query(rs_session *s, hipEvent_t ev, hipError_t *err)
{
    if (s->inject_device_error) {
        *err = hipErrorLaunchFailure;
        return ev_state::error;
    }
    *err = hipEventQuery(ev);
    if (*err == hipSuccess) return ev_state::done;
    if (*err == hipErrorNotReady) return ev_state::pending;
    return ev_state::error;
}

void device_failed(rs_session *s, std::unique_lock<std::mutex> &lk, std::deque<inflight> &fly, hipError_t err)
{
    // nothing of the abandoned slices may still run once their requests'
    // buffers are handed back as FAILED
    lk.unlock();
    (void)hipStreamSynchronize(s->stream);
    for (auto &st : s->side) (void)hipStreamSynchronize(st);
    lk.lock();
    char why[160];
    snprintf(why, sizeof why, "session stopped by a device error: %s",
             s->inject_device_error ? "injected for a test" : hipGetErrorString(err));
    s->sched->fail_all(why, now_ns());
    s->busy_iters -= (int)fly.size();
    fly.clear();
    s->cv_done.notify_all();
}

void worker_main(rs_session *s)
{
    (void)hipSetDevice(s->device);
    std::deque<inflight> fly;
    std::unique_lock<std::mutex> lk(s->mu);
    rs_sched::Scheduler &sc = *s->sched;
    for (;;) {
        // retire slices the device has finished; stop at a device error
        bool dead = sc.stopped();
        while (!dead && !fly.empty()) {
            hipError_t err = hipSuccess;
            const ev_state e = query(s, s->ring[fly.front().slot].done, &err);
            if (e == ev_state::pending) break;
            if (e == ev_state::error) {
                device_failed(s, lk, fly, err);
                dead = true;
                break;
            }
            sc.retire(fly.front().slice, now_ns());
            fly.pop_front();
            s->busy_iters--;
            s->cv_done.notify_all();
        }
        if (dead) {
            // nothing runs any more; requests already failed
            if (s->stop) break;
            s->cv.wait(lk);
            continue;
        }
        sc.admit(now_ns());
        if (!sc.has_work() || fly.size() >= 2) {
            if (!fly.empty()) {
                hipEvent_t ev = s->ring[fly.front().slot].done;
                lk.unlock();
                const hipError_t err = hipEventSynchronize(ev);
                lk.lock();
                if (err != hipSuccess || s->inject_device_error) device_failed(s, lk, fly, err);
                continue;
            }
            if (s->stop && sc.queued() == 0 && sc.running() == 0) break;
            s->cv.wait(lk);
            continue;
        }
        inflight f;
        f.slice = sc.next_slice();
        bool fail = false;
        if (s->inject_fail > 0) {
            s->inject_fail--;
            fail = true;
        }
        f.slot = s->ring_next;
        s->ring_next = (s->ring_next + 1) % kRing;
        s->busy_iters++;
        s->launches++;
        lk.unlock();

        ring_slot &rg = s->ring[f.slot];
        hipError_t err = fail ? hipErrorLaunchFailure : enqueue_slice(s, rg, f.slice);
        (void)hipEventRecord(rg.done, s->stream);

        lk.lock();
        // a slice that could not be launched fails the requests with work in
        // it; they retire with this slice
        if (err != hipSuccess) sc.fail_slice(f.slice);
        fly.push_back(std::move(f));
    }
}

}  // namespace

// Frees what rs_session_create allocated (anything not allocated is null).
static void release_resources(rs_session *s)
{
    for (auto &rg : s->ring) {
        if (rg.h_jobs) (void)hipHostFree(rg.h_jobs);
        if (rg.d_jobs) (void)hipFree(rg.d_jobs);
        if (rg.d_counter) (void)hipFree(rg.d_counter);
        if (rg.done) (void)hipEventDestroy(rg.done);
        if (rg.start) (void)hipEventDestroy(rg.start);
        for (auto &e : rg.grp)
            if (e) (void)hipEventDestroy(e);
    }
    if (s->arena) (void)hipFree(s->arena);
    if (s->scales) (void)hipFree(s->scales);
    for (auto &st : s->side)
        if (st) (void)hipStreamDestroy(st);
    if (s->stream) (void)hipStreamDestroy(s->stream);
}

extern "C" rs_status rs_session_create(const rs_session_opts *o, rs_session **out)
{
    if (!out) return rs_fail(RS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!o) return rs_fail(RS_E_INVALID, "opts is NULL");
    if (o->max_slots < 1 || o->max_slots > 4096) return rs_fail(RS_E_INVALID, "max_slots out of range");
    if (o->queue_cap < 1) return rs_fail(RS_E_INVALID, "queue_cap < 1");
    if (o->slice_items < 0) return rs_fail(RS_E_INVALID, "slice_items < 0");
    if (o->policy != RS_SCHED_SHORTEST && o->policy != RS_SCHED_EQUAL)
        return rs_fail(RS_E_INVALID, "unknown policy %d", o->policy);
    if (!(o->slice_terms >= 0.0) || o->slice_terms > 1e18) return rs_fail(RS_E_INVALID, "slice_terms out of range");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || o->device < 0 || o->device >= ndev)
        return rs_fail(RS_E_INVALID, "bad device %d", o->device);
    std::unique_ptr<rs_session> s(new (std::nothrow) rs_session());
    if (!s) return rs_fail(RS_E_NOMEM, "host allocation failed");
    s->device = o->device;
    rs_sched::Options so;
    so.budget = (o->hbm_budget + 255) & ~(size_t)255;
    so.max_slots = o->max_slots;
    so.queue_cap = o->queue_cap;
    so.slice_items = o->slice_items;
    so.policy = o->policy;
    so.max_bypass = o->strict_fifo ? 0 : 64;
    if (o->slice_terms > 0.0) so.slice_terms = o->slice_terms;
    s->sched.reset(new (std::nothrow) rs_sched::Scheduler(so));
    if (!s->sched) return rs_fail(RS_E_NOMEM, "host allocation failed");
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
        for (auto &st : s->side)
            if (status == RS_OK && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
                status = rs_fail(RS_E_DEVICE, "stream creation failed");
        if (status != RS_OK) break;
        if (so.budget && hipMalloc(&s->arena, so.budget) != hipSuccess) {
            status = rs_fail(RS_E_NOMEM, "arena allocation of %zu bytes failed", so.budget);
            break;
        }
        // a matrix-core plan has at most one chunk per compute unit
        s->scale_row = (size_t)s->ncu;
        if (hipMalloc(reinterpret_cast<void **>(&s->scales), sizeof(int32_t) * s->scale_row * so.max_slots) !=
            hipSuccess) {
            status = rs_fail(RS_E_NOMEM, "scale pool allocation failed");
            break;
        }
        s->jobs_cap = so.max_slots * (kMaxVariants + 1);
        for (auto &rg : s->ring) {
            if (hipHostMalloc(reinterpret_cast<void **>(&rg.h_jobs), sizeof(rs_job) * s->jobs_cap,
                              hipHostMallocDefault) != hipSuccess ||
                hipMalloc(&rg.d_jobs, sizeof(rs_job) * s->jobs_cap) != hipSuccess ||
                hipMalloc(&rg.d_counter, sizeof(int) * 64) != hipSuccess ||
                hipEventCreateWithFlags(&rg.done, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&rg.start, hipEventDisableTiming) != hipSuccess) {
                status = rs_fail(RS_E_NOMEM, "session ring allocation failed");
                break;
            }
            for (auto &e : rg.grp)
                if (status == RS_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                    status = rs_fail(RS_E_NOMEM, "session ring allocation failed");
            if (status != RS_OK) break;
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
        release_resources(s.get());
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
    auto r = std::make_unique<rs_sched::Request>();
    r->plan = pl;
    r->px = *px;
    r->cube = cube;
    if ((st = rs_plan_chunking(pl, px->P, &r->S, &r->chunk)) != RS_OK) return st;
    r->items = (int64_t)r->S * pl->C * pl->n_tiles * pl->l_tiles;
    r->steps = r->S > 0 ? rs_steps_per_chunk(pl, r->chunk) : 0;
    r->footprint = rs_workspace_bytes(pl, r->S);
    if ((size_t)r->S > s->scale_row)
        return rs_fail(RS_E_UNSUPPORTED, "request has %d pixel chunks, the session's scale rows hold %zu", r->S,
                       s->scale_row);
    r->terms = (double)px->P * pl->C * pl->L * pl->Ns;
    r->step_terms = 16.0 * pl->tn * pl->tl;
    const size_t amp_bytes = (pl->model & RS_MODEL_BLOCK_STRENGTH) ? (size_t)4 * pl->L : 4;
    r->request_bytes = (size_t)px->P * (16 + amp_bytes) +
                       (size_t)pl->C * pl->L * pl->Ns * (pl->dtype == RS_C128 ? 16 : 8) + r->footprint;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return rs_fail(RS_E_INVALID, "session is shutting down");
    const size_t need = r->footprint;
    switch (s->sched->submit(std::move(r), now_ns(), ticket)) {
    case RS_OK:
        break;
    case RS_E_INVALID:
        return rs_fail(RS_E_INVALID, "request needs %zu bytes of workspace, session budget is %zu", need,
                       s->sched->options().budget);
    case RS_E_BUSY:
        return rs_fail(RS_E_BUSY, "queue full");
    default:
        return rs_fail(RS_E_DEVICE, "%s", s->sched->error().c_str());
    }
    s->cv.notify_all();
    return RS_OK;
}

extern "C" rs_status rs_session_poll(rs_session *s, uint64_t ticket, int32_t *state, rs_timing *tm)
{
    if (!s || !state) return rs_fail(RS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    rs_sched::Request *r = s->sched->find(ticket);
    if (!r) return rs_fail(RS_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    *state = r->state;
    if (tm) *tm = r->tm;
    return RS_OK;
}

extern "C" rs_status rs_session_cancel(rs_session *s, uint64_t ticket)
{
    if (!s) return rs_fail(RS_E_INVALID, "NULL session");
    std::lock_guard<std::mutex> g(s->mu);
    const rs_status st = s->sched->cancel(ticket, now_ns());
    if (st == RS_E_NOT_FOUND) return rs_fail(RS_E_NOT_FOUND, "unknown ticket");
    if (st == RS_E_BUSY) return rs_fail(RS_E_BUSY, "request already admitted or finished");
    s->cv.notify_all();
    s->cv_done.notify_all();
    return RS_OK;
}

extern "C" rs_status rs_session_drain(rs_session *s)
{
    if (!s) return rs_fail(RS_E_INVALID, "NULL session");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->sched->queued() == 0 && s->sched->running() == 0 && s->busy_iters == 0; });
    return RS_OK;
}

extern "C" rs_status rs_session_stats_get(rs_session *s, rs_session_stats *out)
{
    if (!s || !out) return rs_fail(RS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    const rs_sched::Stats &t = s->sched->stats();
    std::memset(out, 0, sizeof *out);
    out->submitted = t.submitted;
    out->admitted = t.admitted;
    out->done = t.done;
    out->failed = t.failed;
    out->cancelled = t.cancelled;
    out->launches = s->launches;
    out->queued_now = (int64_t)s->sched->queued();
    out->running_now = (int64_t)s->sched->running();
    out->footprint_now = t.footprint_now;
    out->footprint_peak = t.footprint_peak;
    out->terms_done = t.terms_done;
    out->request_bytes_now = t.request_bytes_now;
    out->request_bytes_peak = t.request_bytes_peak;
    out->device_error = s->sched->stopped() ? 1 : 0;
    return RS_OK;
}

extern "C" rs_status rs_session_inject_failure(rs_session *s, int32_t count)
{
    if (!s || count < 0) return rs_fail(RS_E_INVALID, "bad argument");
    std::lock_guard<std::mutex> g(s->mu);
    s->inject_fail += count;
    return RS_OK;
}

extern "C" rs_status rs_session_inject_device_error(rs_session *s)
{
    if (!s) return rs_fail(RS_E_INVALID, "NULL session");
    std::lock_guard<std::mutex> g(s->mu);
    s->inject_device_error = true;
    s->cv.notify_all();
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
    for (auto &st : s->side)
        if (st) (void)hipStreamSynchronize(st);
    release_resources(s);
    (void)hipSetDevice(prev);
    delete s;
}
