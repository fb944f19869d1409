// Host test of the server's scheduling core (rkc_server_core.h) with a fake
// backend: no device, a fake clock, and batches that "complete" after a
// chosen number of polls.  The fake marks every cell it processes, so the test
// can check that each cell of each request is processed exactly once, that
// in-flight arena regions never overlap and stay inside the budget, that no
// more batches run than there are slots, that batches only merge compatible
// requests and start from the oldest waiting request, and the latency
// statistics.  Prints "OK" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "rkc_server_core.h"

using namespace rkcsrv;

static int failures = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);        \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

struct Fake {
    double t = 0.0;                      // fake clock, seconds
    size_t budget = 0;
    int n_slots = 0;
    int delay_polls = 1;                 // polls until a batch completes
    bool fail_next_start = false;
    std::vector<Batch *> inflight;
    std::vector<int> polls_left;         // by slot
    std::vector<std::vector<uint64_t>> started;   // request ids per started batch
    size_t max_inflight = 0;
    std::mt19937 rng{7};
    bool random_delay = false;

    double now() { return t; }

    int start(Batch &b) {
        if (fail_next_start) { fail_next_start = false; return RKC_EDEVICE; }
        // region inside the budget and disjoint from every in-flight region
        CHECK(b.offset + b.bytes <= budget);
        for (Batch *o : inflight) {
            CHECK(b.slot != o->slot);
            CHECK(b.offset + b.bytes <= o->offset || o->offset + o->bytes <= b.offset);
        }
        // one compatible key, contiguous cells, footprint of the whole batch
        size_t c = 0;
        for (Request *r : b.reqs) {
            CHECK(r->cell0 == c);
            c += r->n;
            const Request &h = *b.reqs[0];
            CHECK(r->mech == h.mech && r->dt == h.dt && r->rtol == h.rtol &&
                  r->atol == h.atol && r->method == h.method);
        }
        CHECK(c == b.cells);
        CHECK(b.bytes == footprint(b.cells, b.reqs[0]->n_species));
        inflight.push_back(&b);
        max_inflight = std::max(max_inflight, inflight.size());
        if ((int)polls_left.size() < n_slots) polls_left.resize(n_slots, 0);
        polls_left[b.slot] = random_delay ? 1 + (int)(rng() % 5) : delay_polls;
        std::vector<uint64_t> ids;
        for (Request *r : b.reqs) ids.push_back(r->id);
        started.push_back(ids);
        return RKC_OK;
    }

    int poll(Batch &b) {
        if (--polls_left[b.slot] > 0) return 0;
        for (Request *r : b.reqs) {
            for (size_t i = 0; i < r->n; ++i) r->T[i] += 1.0;   // processed once
            r->n_failed = 0;
            r->rc = RKC_OK;
        }
        for (size_t i = 0; i < inflight.size(); ++i)
            if (inflight[i] == &b) { inflight.erase(inflight.begin() + (long)i); break; }
        return 1;
    }
};

struct Owned {
    std::vector<double> T, P, Y;
};

static Request make(Owned &o, int mech, size_t n, size_t nS, double dt) {
    o.T.assign(n, 0.0);
    o.P.assign(n, 1.0);
    o.Y.assign(n * nS, 0.5);
    Request r;
    r.mech = mech;
    r.n = n;
    r.n_species = nS;
    r.T = o.T.data();
    r.P = o.P.data();
    r.Y = o.Y.data();
    r.dt = dt;
    r.rtol = 1e-6;
    r.atol = 1e-10;
    return r;
}

static void drain(Core<Fake> &c, Fake &f, int max_rounds = 100000) {
    for (int i = 0; i < max_rounds && !c.idle(); ++i) {
        c.pump();
        f.t += 1e-3;
    }
    CHECK(c.idle());
}

static void test_batching_and_order() {
    Fake f;
    f.budget = 1 << 24;
    f.n_slots = 1;
    Core<Fake> c(&f, f.budget, 1, 1 << 20);
    Owned a, b, d, e;
    uint64_t ia, ib, id, ie;
    CHECK(c.submit(make(a, 0, 100, 9, 1e-6), &ia) == RKC_OK);
    CHECK(c.submit(make(b, 1, 50, 13, 1e-6), &ib) == RKC_OK);
    CHECK(c.submit(make(d, 0, 200, 9, 1e-6), &id) == RKC_OK);
    CHECK(c.submit(make(e, 0, 10, 9, 1e-5), &ie) == RKC_OK);   // other dt
    drain(c, f);
    CHECK(f.started.size() == 3);
    CHECK((f.started[0] == std::vector<uint64_t>{ia, id}));   // oldest plus compatible
    CHECK((f.started[1] == std::vector<uint64_t>{ib}));
    CHECK((f.started[2] == std::vector<uint64_t>{ie}));
    for (Owned *o : {&a, &b, &d, &e})
        for (double v : o->T) CHECK(v == 1.0);
    CHECK(c.state(ia) == RQ_DONE && c.state(ib) == RQ_DONE);
    const CoreStats s = c.stats();
    CHECK(s.submitted == 4 && s.completed == 4 && s.launches == 3 && s.cells == 360);
}

static void test_budget_and_cell_limit() {
    const size_t nS = 13;
    Fake f;
    f.budget = footprint(1000, nS) + footprint(10, nS);   // room for one big request at a time
    f.n_slots = 4;
    Core<Fake> c(&f, f.budget, 4, 1500);
    Owned big[6], huge;
    uint64_t id;
    CHECK(c.submit(make(huge, 0, 4000, nS, 1e-6), &id) == RKC_ENOMEM);   // never fits
    for (auto &o : big) CHECK(c.submit(make(o, 0, 1000, nS, 1e-6), &id) == RKC_OK);
    drain(c, f);
    for (auto &v : f.started) CHECK(v.size() == 1);   // 2 x 1000 cells exceeds the limit
    CHECK(f.max_inflight == 1);                        // the arena holds one at a time
    CHECK(c.stats().peak_bytes <= (int64_t)f.budget);
    CHECK(c.arena().used() == 0);
    for (auto &o : big)
        for (double v : o.T) CHECK(v == 1.0);
}

static void test_slots_limit_and_concurrency() {
    Fake f;
    f.budget = 1 << 26;
    f.n_slots = 3;
    f.delay_polls = 4;
    Core<Fake> c(&f, f.budget, 3, 1 << 20);
    Owned o[8];
    uint64_t id;
    for (int i = 0; i < 8; ++i) CHECK(c.submit(make(o[i], i, 64, 9, 1e-6), &id) == RKC_OK);
    drain(c, f);
    CHECK(f.max_inflight == 3);
    CHECK(f.started.size() == 8);
}

static void test_latency_statistics() {
    Fake f;
    f.budget = 1 << 24;
    f.n_slots = 1;
    f.delay_polls = 1;
    Core<Fake> c(&f, f.budget, 1, 1 << 20);
    Owned o[4];
    uint64_t id;
    // submitted at t = 0, 0, 0, 0 with distinct mechanisms: batches run one
    // after another, completing at the 1st, 2nd, 3rd and 4th pump (+1 ms each)
    for (int i = 0; i < 4; ++i) CHECK(c.submit(make(o[i], i, 8, 9, 1e-6), &id) == RKC_OK);
    for (int i = 0; i < 6; ++i) {
        c.pump();
        f.t += 1e-3;
    }
    const CoreStats s = c.stats();
    CHECK(s.completed == 4);
    // completion times 1, 2, 3, 4 ms (a batch started at pump k completes at pump k+1)
    CHECK(std::abs(s.max_ms - 4.0) < 1e-9);
    CHECK(std::abs(s.p50_ms - 2.0) < 1e-9);
    CHECK(std::abs(s.p99_ms - 4.0) < 1e-9);
    CHECK(std::abs(s.mean_ms - 2.5) < 1e-9);
    CHECK(percentile({5, 1, 3, 2, 4}, 0.5) == 3);
    CHECK(percentile({5, 1, 3, 2, 4}, 0.99) == 5);
    CHECK(percentile({7}, 0.01) == 7);
}

static void test_empty_request_and_start_failure() {
    Fake f;
    f.budget = 1 << 24;
    f.n_slots = 2;
    Core<Fake> c(&f, f.budget, 2, 1 << 20);
    Owned e, a, b;
    uint64_t ie, ia, ib;
    CHECK(c.submit(make(e, 0, 0, 9, 1e-6), &ie) == RKC_OK);
    CHECK(c.state(ie) == RQ_DONE);
    f.fail_next_start = true;
    CHECK(c.submit(make(a, 0, 10, 9, 1e-6), &ia) == RKC_OK);
    CHECK(c.submit(make(b, 1, 10, 9, 1e-6), &ib) == RKC_OK);
    drain(c, f);
    CHECK(c.get(ia)->rc == RKC_EDEVICE);
    CHECK(c.get(ib)->rc == RKC_OK);
    CHECK(c.arena().used() == 0);
    for (double v : b.T) CHECK(v == 1.0);
}

static void test_random_stress() {
    std::mt19937 rng(11);
    Fake f;
    f.budget = 3 << 20;
    f.n_slots = 4;
    f.random_delay = true;
    Core<Fake> c(&f, f.budget, 4, 20000);
    const int R = 600;
    std::vector<Owned> own(R);
    std::vector<uint64_t> ids;
    std::vector<int> mech(R);
    std::vector<int> accepted;
    for (int i = 0; i < R; ++i) {
        const size_t n = 1 + rng() % 6000;
        mech[i] = (int)(rng() % 3);
        const size_t nS = mech[i] == 0 ? 9 : (mech[i] == 1 ? 13 : 53);
        uint64_t id;
        const int rc = c.submit(make(own[i], mech[i], n, nS, (rng() % 2) ? 1e-6 : 1e-5), &id);
        if (footprint(n, nS) > f.budget) { CHECK(rc == RKC_ENOMEM); continue; }
        CHECK(rc == RKC_OK);
        ids.push_back(id);
        accepted.push_back(i);
        if (rng() % 3 == 0) { c.pump(); f.t += 1e-4; }
    }
    drain(c, f);
    std::set<uint64_t> seen;
    for (auto &v : f.started)
        for (uint64_t x : v) { CHECK(!seen.count(x)); seen.insert(x); }
    CHECK(seen.size() == ids.size());
    for (uint64_t x : ids) CHECK(c.state(x) == RQ_DONE);
    for (int i : accepted)
        for (double v : own[i].T) CHECK(v == 1.0);
    CHECK(f.max_inflight <= 4);
    CHECK(c.arena().used() == 0);
    CHECK(c.stats().peak_bytes <= (int64_t)f.budget);
}

static void test_arena_coalescing() {
    Arena a(4096);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(1000, &o1) && a.alloc(1000, &o2) && a.alloc(1000, &o3));
    CHECK(o1 == 0 && o2 == 1024 && o3 == 2048);
    CHECK(!a.alloc(2000, &o4));
    a.release(o2, 1000);
    a.release(o1, 1000);
    CHECK(a.largest_free() == 2048);
    CHECK(a.alloc(2000, &o4) && o4 == 0);
    a.release(o3, 1000);
    a.release(o4, 2000);
    CHECK(a.used() == 0 && a.largest_free() == 4096);
}

int main() {
    test_arena_coalescing();
    test_batching_and_order();
    test_budget_and_cell_limit();
    test_slots_limit_and_concurrency();
    test_latency_statistics();
    test_empty_request_and_start_failure();
    test_random_stress();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("OK\n");
    return 0;
}
