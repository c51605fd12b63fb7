// Host tests of the serving scheduler (paper_2307_09226_amd/csrc/rs_sched.h)
// with synthetic completions: no GPU, built with g++ under AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_scheduler_host.py.  Each
// scenario checks its own expectations; the randomised run checks the
// invariants after every event.  Prints "ALL OK" and exits 0 on success.
#include "rs_sched.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>

using rs_sched::Arena;
using rs_sched::Options;
using rs_sched::Request;
using rs_sched::Scheduler;
using rs_sched::Slice;

static int g_checks = 0;

#define CHECK(cond)                                                                 \
    do {                                                                            \
        ++g_checks;                                                                 \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                           \
        }                                                                           \
    } while (0)

// A request of `items` work items x `steps` steps, each step worth
// `step_terms` terms per item, holding `footprint` arena bytes.
static std::unique_ptr<Request> make_req(int64_t items, int32_t steps, double step_terms, size_t footprint)
{
    auto r = std::make_unique<Request>();
    r->items = items;
    r->steps = steps;
    r->step_terms = step_terms;
    r->terms = (double)items * steps * step_terms;
    r->footprint = footprint;
    r->request_bytes = footprint + 1000;
    return r;
}

static uint64_t submit(Scheduler &s, std::unique_ptr<Request> r, int64_t now = 0, rs_status want = RS_OK)
{
    uint64_t t = 0;
    CHECK(s.submit(std::move(r), now, &t) == want);
    return t;
}

// Runs slices until nothing is left, retiring each at once; returns the
// number of slices.
static int run_to_end(Scheduler &s, int64_t &now)
{
    int n = 0;
    for (;;) {
        s.admit(now);
        if (!s.has_work()) {
            if (s.queued() == 0) return n;
            CHECK(s.running() > 0);  // otherwise the queue could never move
        }
        Slice sl = s.next_slice();
        ++now;
        s.retire(sl, now);
        ++n;
        CHECK(n < 1000000);
    }
}

static void test_arena()
{
    Arena a;
    a.init(4096);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(1000, &o1) && o1 == 0);      // rounds to 1024
    CHECK(a.alloc(256, &o2) && o2 == 1024);
    CHECK(a.alloc(2048, &o3) && o3 == 1280);
    CHECK(!a.alloc(1024, &o4));                // 768 left
    CHECK(a.free_bytes() == 768);
    a.release(o2, 256);
    CHECK(a.alloc(200, &o4) && o4 == 1024);    // first fit reuses the hole
    a.release(o1, 1000);
    a.release(o3, 2048);
    a.release(o4, 200);
    CHECK(a.free_bytes() == 4096 && a.free_list().size() == 1);  // fully coalesced
    // random stress: no overlap, everything coalesces back
    std::mt19937_64 rng(1);
    a.init(1 << 20);
    std::vector<std::pair<size_t, size_t>> held;
    for (int i = 0; i < 20000; ++i) {
        if (!held.empty() && (rng() % 2)) {
            const size_t k = rng() % held.size();
            a.release(held[k].first, held[k].second);
            held.erase(held.begin() + (long)k);
        } else {
            const size_t n = 1 + rng() % 40000;
            size_t off;
            if (a.alloc(n, &off)) held.push_back({off, n});
        }
        size_t used = 0;
        for (auto &h : held) used += Arena::round(h.second);
        CHECK(used + a.free_bytes() == a.size());
    }
    std::sort(held.begin(), held.end());
    for (size_t k = 1; k < held.size(); ++k) CHECK(held[k - 1].first + Arena::round(held[k - 1].second) <= held[k].first);
    for (auto &h : held) a.release(h.first, h.second);
    CHECK(a.free_bytes() == a.size() && a.free_list().size() == 1);
}

static void test_submit_limits_and_cancel()
{
    Options o;
    o.budget = 10000;
    o.max_slots = 1;
    o.queue_cap = 2;
    Scheduler s(o);
    submit(s, make_req(4, 32, 1e6, 20000), 0, RS_E_INVALID);  // can never fit
    const uint64_t a = submit(s, make_req(4, 32, 1e6, 1000));
    const uint64_t b = submit(s, make_req(4, 32, 1e6, 1000));
    CHECK(b == a + 1);
    submit(s, make_req(4, 32, 1e6, 1000), 0, RS_E_BUSY);      // queue full: back-pressure
    s.admit(5);
    CHECK(s.find(a)->state == RS_REQ_RUNNING && s.find(a)->tm.t_admit_ns == 5);
    CHECK(s.find(b)->state == RS_REQ_QUEUED);                 // one slot
    CHECK(s.cancel(a, 6) == RS_E_BUSY);                       // already admitted
    CHECK(s.cancel(b, 6) == RS_OK && s.find(b)->state == RS_REQ_CANCELLED);
    CHECK(s.cancel(b, 6) == RS_E_BUSY);
    CHECK(s.cancel(987654, 6) == RS_E_NOT_FOUND);
    const uint64_t c = submit(s, make_req(4, 32, 1e6, 1000));  // room again after the cancel
    int64_t now = 10;
    run_to_end(s, now);
    CHECK(s.find(a)->state == RS_REQ_DONE && s.find(c)->state == RS_REQ_DONE);
    CHECK(s.stats().done == 2 && s.stats().cancelled == 1 && s.stats().submitted == 3);
    CHECK(s.stats().footprint_now == 0 && s.arena().free_bytes() == o.budget);
}

static void test_admission_bypass()
{
    // arena for one big request; a big one runs, a second big one waits;
    // small ones overtake it at most max_bypass times
    Options o;
    o.budget = 1 << 20;
    o.max_slots = 64;
    o.queue_cap = 64;
    o.max_bypass = 3;
    Scheduler s(o);
    const uint64_t big1 = submit(s, make_req(8, 64, 1e6, 900 << 10));
    const uint64_t big2 = submit(s, make_req(8, 64, 1e6, 900 << 10));
    std::vector<uint64_t> small;
    for (int i = 0; i < 6; ++i) small.push_back(submit(s, make_req(1, 16, 1e6, 10 << 10)));
    s.admit(1);
    CHECK(s.find(big1)->state == RS_REQ_RUNNING);
    CHECK(s.find(big2)->state == RS_REQ_QUEUED);
    int admitted_small = 0;
    for (uint64_t t : small) admitted_small += s.find(t)->state == RS_REQ_RUNNING;
    CHECK(admitted_small == 3);                   // three overtook big2, then it blocks
    CHECK(s.find(big2)->bypassed == 3);
    s.admit(2);                                   // nothing new while big2 waits
    admitted_small = 0;
    for (uint64_t t : small) admitted_small += s.find(t)->state == RS_REQ_RUNNING;
    CHECK(admitted_small == 3);
    int64_t now = 3;
    run_to_end(s, now);
    for (uint64_t t : small) CHECK(s.find(t)->state == RS_REQ_DONE);
    CHECK(s.find(big2)->state == RS_REQ_DONE);
    for (int i = 3; i < 6; ++i) CHECK(s.find(big2)->tm.t_admit_ns <= s.find(small[i])->tm.t_admit_ns);  // not overtaken again
    // strict arrival order
    Options f = o;
    f.max_bypass = 0;
    Scheduler t(f);
    submit(t, make_req(8, 64, 1e6, 900 << 10));
    const uint64_t b2 = submit(t, make_req(8, 64, 1e6, 900 << 10));
    const uint64_t s1 = submit(t, make_req(1, 16, 1e6, 10 << 10));
    t.admit(1);
    CHECK(t.find(b2)->state == RS_REQ_QUEUED && t.find(s1)->state == RS_REQ_QUEUED);
}

static void test_slices_equal_and_shortest()
{
    for (int policy : {rs_sched::EQUAL, rs_sched::SHORTEST}) {
        Options o;
        o.budget = 1 << 30;
        o.max_slots = 8;
        o.queue_cap = 8;
        o.policy = policy;
        o.slice_terms = 64.0 * 16 * 1e6;  // 64 item-blocks of 16 steps at 1e6 terms per step
        Scheduler s(o);
        // a: 1 item x 64 steps (4 blocks); b: 8 items x 1024 steps; z: no items (P = 0)
        const uint64_t a = submit(s, make_req(1, 64, 1e6, 4096));
        const uint64_t b = submit(s, make_req(8, 1024, 1e6, 4096));
        const uint64_t z = submit(s, make_req(0, 0, 1e6, 0));
        s.admit(0);
        Slice sl = s.next_slice();
        // z completes in its first slice without any part
        CHECK(std::find(sl.completing.begin(), sl.completing.end(), s.find(z)) != sl.completing.end());
        for (auto &p : sl.parts) CHECK(p.r != s.find(z));
        for (auto &p : sl.parts) {
            CHECK(p.first && p.seg_begin == 0 && p.seg_end > p.seg_begin);
            CHECK(p.seg_end % rs_sched::kBlockSteps == 0 || p.seg_end == p.r->steps);
        }
        const Request *ra = s.find(a), *rb = s.find(b);
        if (policy == rs_sched::SHORTEST) {
            CHECK(ra->cursor == ra->steps);         // the small one gets all its work first
            CHECK(rb->cursor >= rs_sched::kBlockSteps);  // the floor keeps the big one moving
        } else {
            CHECK(ra->cursor == 64 && rb->cursor < 1024);  // equal terms: a's share covers it
        }
        s.retire(sl, 1);
        CHECK(s.find(a)->state == RS_REQ_DONE && s.find(z)->state == RS_REQ_DONE);
        int64_t now = 2;
        run_to_end(s, now);
        CHECK(s.find(b)->state == RS_REQ_DONE && s.find(b)->cursor == 1024);
    }
}

static void test_failures()
{
    Options o;
    o.budget = 1 << 20;
    o.max_slots = 4;
    o.queue_cap = 16;
    Scheduler s(o);
    const uint64_t a = submit(s, make_req(4, 256, 1e6, 4096));
    const uint64_t b = submit(s, make_req(4, 256, 1e6, 4096));
    s.admit(0);
    Slice sl = s.next_slice();
    s.fail_slice(sl);                       // the launch of this slice failed
    s.retire(sl, 1);
    CHECK(s.find(a)->state == RS_REQ_FAILED && s.find(b)->state == RS_REQ_FAILED);
    CHECK(s.stats().failed == 2 && s.stats().footprint_now == 0);
    const uint64_t c = submit(s, make_req(4, 64, 1e6, 4096));  // the session goes on
    int64_t now = 2;
    run_to_end(s, now);
    CHECK(s.find(c)->state == RS_REQ_DONE);
    // a device error: admitted and queued requests fail, nothing more runs
    Options o2 = o;
    o2.max_slots = 1;
    Scheduler t(o2);
    const uint64_t d = submit(t, make_req(4, 256, 1e6, 4096));
    const uint64_t e = submit(t, make_req(4, 256, 1e6, 4096));
    t.admit(0);
    Slice s1 = t.next_slice();
    (void)s1;                                // in flight when the error is seen
    t.fail_all("injected", 5);
    CHECK(t.find(d)->state == RS_REQ_FAILED && t.find(e)->state == RS_REQ_FAILED);
    CHECK(t.find(e)->tm.t_done_ns == 5);
    CHECK(t.running() == 0 && t.queued() == 0 && t.stats().footprint_now == 0);
    CHECK(t.arena().free_bytes() == o2.budget);
    CHECK(t.stopped() && t.error() == "injected");
    uint64_t tk = 0;
    CHECK(t.submit(make_req(1, 16, 1e6, 0), 6, &tk) == RS_E_DEVICE);
    t.retire(s1, 7);                         // a late retire of the failed slice is harmless
    CHECK(t.stats().failed == 2 && t.stats().done == 0);
    t.admit(8);
    CHECK(!t.has_work());
}

// Randomised arrivals, sizes, cancellations and launch failures with
// completions in order; invariants after every event.
static void test_random(int policy, uint64_t seed)
{
    std::mt19937_64 rng(seed);
    Options o;
    o.budget = 64 << 20;
    o.max_slots = 12;
    o.queue_cap = 40;
    o.policy = policy;
    o.max_bypass = 8;
    o.slice_terms = 4e9;
    Scheduler s(o);
    std::vector<uint64_t> tickets;
    std::map<uint64_t, int64_t> given;        // steps handed out per request
    std::map<uint64_t, int32_t> last_end;     // contiguity of segments
    std::deque<Slice> fly;
    int64_t now = 0;
    for (int ev = 0; ev < 6000; ++ev) {
        now += 1 + (int64_t)(rng() % 5);
        const unsigned dice = (unsigned)(rng() % 100);
        if (dice < 30) {
            const int64_t items = (int64_t)(rng() % 64);
            const int32_t steps = items ? 16 * (1 + (int32_t)(rng() % 40)) - (int32_t)(rng() % 8) : 0;
            const size_t fp = 256 + (size_t)(rng() % (20 << 20));
            uint64_t t = 0;
            const rs_status st = s.submit(make_req(items, steps, 1e6, fp), now, &t);
            CHECK(st == RS_OK || st == RS_E_BUSY);
            if (st == RS_OK) tickets.push_back(t);
        } else if (dice < 33 && !tickets.empty()) {
            const uint64_t t = tickets[rng() % tickets.size()];
            const int32_t before = s.find(t)->state;
            const rs_status st = s.cancel(t, now);
            CHECK(st == (before == RS_REQ_QUEUED ? RS_OK : RS_E_BUSY));
        } else if (dice < 70) {
            s.admit(now);
            if (s.has_work() && fly.size() < 2) {
                Slice sl = s.next_slice();
                for (auto &p : sl.parts) {
                    CHECK(p.seg_begin == (last_end.count(p.r->ticket) ? last_end[p.r->ticket] : 0));
                    CHECK(p.seg_end > p.seg_begin && p.seg_end <= p.r->steps);
                    CHECK(p.seg_begin % rs_sched::kBlockSteps == 0);
                    last_end[p.r->ticket] = p.seg_end;
                    given[p.r->ticket] += p.seg_end - p.seg_begin;
                }
                if (rng() % 200 == 0) s.fail_slice(sl);
                fly.push_back(std::move(sl));
            }
        } else if (!fly.empty()) {
            s.retire(fly.front(), now);
            fly.pop_front();
        }
        // invariants
        const auto &st = s.stats();
        CHECK(st.footprint_now <= o.budget);
        CHECK(st.footprint_now + s.arena().free_bytes() == o.budget);
        CHECK((int)s.running() <= o.max_slots && (int)s.queued() <= o.queue_cap);
        std::vector<std::pair<size_t, size_t>> ranges;
        std::set<int32_t> slots;
        for (const Request *r : s.active()) {
            CHECK(r->state == RS_REQ_RUNNING);
            CHECK(r->slot >= 0 && r->slot < o.max_slots && slots.insert(r->slot).second);  // distinct slots
            if (r->footprint) ranges.push_back({r->arena_off, Arena::round(r->footprint)});
        }
        std::sort(ranges.begin(), ranges.end());
        for (size_t k = 1; k < ranges.size(); ++k) CHECK(ranges[k - 1].first + ranges[k - 1].second <= ranges[k].first);
        for (uint64_t t : tickets) CHECK(s.find(t)->bypassed <= o.max_bypass);
    }
    // drain
    while (!fly.empty()) {
        s.retire(fly.front(), ++now);
        fly.pop_front();
    }
    for (;;) {
        s.admit(++now);
        if (!s.has_work() && s.queued() == 0) break;
        Slice sl = s.next_slice();
        for (auto &p : sl.parts) given[p.r->ticket] += p.seg_end - p.seg_begin;
        s.retire(sl, ++now);
    }
    const auto &st = s.stats();
    CHECK(st.done + st.failed + st.cancelled == st.submitted);
    CHECK(st.footprint_now == 0 && s.arena().free_bytes() == o.budget && s.arena().free_list().size() == 1);
    for (uint64_t t : tickets) {
        const Request *r = s.find(t);
        CHECK(r->state == RS_REQ_DONE || r->state == RS_REQ_FAILED || r->state == RS_REQ_CANCELLED);
        if (r->state == RS_REQ_DONE) {
            CHECK(given[t] == r->steps);         // every step given out exactly once
            CHECK(r->tm.t_submit_ns <= r->tm.t_admit_ns && r->tm.t_admit_ns <= r->tm.t_done_ns);
        }
        if (r->state == RS_REQ_CANCELLED) CHECK(given[t] == 0);
    }
}

// Mean completion time of a fixed mix under both policies: shortest
// remaining first completes the small requests sooner.
static void test_policy_mean_latency()
{
    double mean[2] = {0, 0};
    for (int policy : {rs_sched::EQUAL, rs_sched::SHORTEST}) {
        Options o;
        o.budget = 1 << 30;
        o.max_slots = 64;
        o.queue_cap = 64;
        o.policy = policy;
        o.slice_terms = 64 * 16 * 1e6;  // 64 blocks of one item
        Scheduler s(o);
        std::vector<uint64_t> t;
        for (int i = 0; i < 20; ++i) t.push_back(submit(s, make_req(1, 16 * (1 + (i * 7) % 40), 1e6, 256)));
        int64_t now = 0;
        run_to_end(s, now);
        double sum = 0;
        for (uint64_t k : t) sum += (double)s.find(k)->tm.t_done_ns;
        mean[policy == rs_sched::SHORTEST] = sum / t.size();
    }
    std::printf("mean completion (slices): equal %.2f, shortest %.2f\n", mean[0], mean[1]);
    CHECK(mean[1] < mean[0]);
}

int main()
{
    test_arena();
    test_submit_limits_and_cancel();
    test_admission_bypass();
    test_slices_equal_and_shortest();
    test_failures();
    for (uint64_t seed = 1; seed <= 4; ++seed) {
        test_random(rs_sched::EQUAL, seed);
        test_random(rs_sched::SHORTEST, seed + 100);
    }
    test_policy_mean_latency();
    std::printf("ALL OK (%d checks)\n", g_checks);
    return 0;
}
