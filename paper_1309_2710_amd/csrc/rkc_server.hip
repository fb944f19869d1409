// Integration server (include/rkc_server.h): the scheduling core of
// rkc_server_core.h driven by a dispatcher thread, with a backend that stages
// requests through a pinned host mirror of the device arena and launches the
// integrator kernels on a pool of streams.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "rkc.h"
#include "rkc_internal.h"
#include "rkc_server.h"
#include "rkc_server_core.h"

namespace {

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    unsigned long long *agg_d = nullptr;
    int *queue_d = nullptr;
    unsigned long long *agg_h = nullptr;   // pinned
};

// Byte offsets of a batch's arrays inside its arena region.
struct Layout {
    size_t T, P, Y, S;
};

Layout layout(size_t cells, size_t nS) {
    Layout l;
    l.T = 0;
    l.P = rkcsrv::align256(8 * cells);
    l.Y = 2 * rkcsrv::align256(8 * cells);
    l.S = l.Y + rkcsrv::align256(8 * cells * nS);
    return l;
}

struct HipBackend {
    int device = 0;
    char *arena_d = nullptr;
    char *mirror_h = nullptr;   // pinned, same size and offsets as the arena
    std::vector<Slot> slots;
    std::vector<rkc_mech *> mechs;
    int lanes = 0, placement = RKC_PARAMS_AUTO;
    int64_t n_rhs = 0;

    double now() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }

    int start(rkcsrv::Batch &b) {
        Slot &sl = slots[(size_t)b.slot];
        const rkcsrv::Request &h = *b.reqs[0];
        rkc_mech *m = mechs[(size_t)h.mech];
        const size_t nS = h.n_species, n = b.cells;
        const Layout L = layout(n, nS);
        char *hb = mirror_h + b.offset;
        char *db = arena_d + b.offset;
        for (const rkcsrv::Request *r : b.reqs) {
            std::memcpy(hb + L.T + 8 * r->cell0, r->T, 8 * r->n);
            std::memcpy(hb + L.P + 8 * r->cell0, r->P, 8 * r->n);
            std::memcpy(hb + L.Y + 8 * nS * r->cell0, r->Y, 8 * nS * r->n);
        }
        if (hipMemcpyAsync(db, hb, L.Y + 8 * nS * n, hipMemcpyHostToDevice, sl.st) != hipSuccess)
            return RKC_EDEVICE;
        rkc_opts o;
        rkc_opts_default(&o);
        o.method = h.method;
        o.lanes_per_cell = lanes;
        o.param_placement = placement;
        o.device_ptrs = 1;
        o.stream = sl.st;
        rkchost::LaunchInfo li;
        int rc = rkchost::enqueue_integrate(m, n, (double *)(db + L.T), (const double *)(db + L.P),
                                            (double *)(db + L.Y), h.dt, h.rtol, h.atol, o,
                                            (int32_t *)(db + L.S), nullptr, sl.agg_d, sl.queue_d,
                                            sl.st, &li);
        if (rc) return rc;
        if (hipMemcpyAsync(hb + L.T, db + L.T, 8 * n, hipMemcpyDeviceToHost, sl.st) != hipSuccess ||
            hipMemcpyAsync(hb + L.Y, db + L.Y, L.S - L.Y + 4 * n, hipMemcpyDeviceToHost,
                           sl.st) != hipSuccess ||
            hipMemcpyAsync(sl.agg_h, sl.agg_d, rkchost::AGG_N * 8, hipMemcpyDeviceToHost,
                           sl.st) != hipSuccess ||
            hipEventRecord(sl.ev, sl.st) != hipSuccess)
            return RKC_EDEVICE;
        return RKC_OK;
    }

    int poll(rkcsrv::Batch &b) {
        Slot &sl = slots[(size_t)b.slot];
        const hipError_t e = hipEventQuery(sl.ev);
        if (e == hipErrorNotReady) return 0;
        if (e != hipSuccess) return RKC_EDEVICE;
        const size_t nS = b.reqs[0]->n_species;
        const Layout L = layout(b.cells, nS);
        const char *hb = mirror_h + b.offset;
        const int32_t *st = (const int32_t *)(hb + L.S);
        for (rkcsrv::Request *r : b.reqs) {
            std::memcpy(r->T, hb + L.T + 8 * r->cell0, 8 * r->n);
            std::memcpy(r->Y, hb + L.Y + 8 * nS * r->cell0, 8 * nS * r->n);
            int32_t failed = 0;
            for (size_t i = 0; i < r->n; ++i) failed += st[r->cell0 + i] != RKC_CELL_OK;
            if (r->status) std::memcpy(r->status, st + r->cell0, 4 * r->n);
            r->n_failed = failed;
            r->rc = failed ? RKC_ECELLS : RKC_OK;
        }
        n_rhs += (int64_t)sl.agg_h[0];
        return 1;
    }
};

}  // namespace

struct rkc_server {
    HipBackend be;
    rkcsrv::Core<HipBackend> *core = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;
};

namespace {

void dispatcher(rkc_server *s) {
    (void)hipSetDevice(s->be.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->core->pump();
        s->cv_done.notify_all();
        if (s->stop && s->core->idle()) break;
        if (s->core->busy()) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            s->cv_work.wait(lk, [s] { return s->stop || s->core->queued(); });
        }
    }
}

void release(rkc_server *s) {
    for (Slot &sl : s->be.slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.agg_d) (void)hipFree(sl.agg_d);
        if (sl.queue_d) (void)hipFree(sl.queue_d);
        if (sl.agg_h) (void)hipHostFree(sl.agg_h);
    }
    for (rkc_mech *m : s->be.mechs) rkc_mech_destroy(m);
    if (s->be.arena_d) (void)hipFree(s->be.arena_d);
    if (s->be.mirror_h) (void)hipHostFree(s->be.mirror_h);
    delete s->core;
    delete s;
}

}  // namespace

extern "C" {

int rkc_server_opts_default(rkc_server_opts *o) {
    if (!o) return RKC_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->budget_bytes = (size_t)1 << 30;
    o->n_streams = 4;
    o->max_batch_cells = 1 << 20;
    o->param_placement = RKC_PARAMS_AUTO;
    return RKC_OK;
}

int rkc_server_create(const rkc_server_opts *opts, rkc_server **out) {
    if (!out) return RKC_EINVAL;
    *out = nullptr;
    rkc_server_opts o;
    if (opts) o = *opts; else rkc_server_opts_default(&o);
    if (o.n_streams < 1 || o.n_streams > 16 || o.budget_bytes < ((size_t)1 << 20) ||
        o.max_batch_cells < 1 || o.param_placement < 0 || o.param_placement > 3)
        return RKC_EINVAL;
    if (o.lanes_per_cell != 0 && o.lanes_per_cell != 1 && o.lanes_per_cell != 8 && o.lanes_per_cell != 16 &&
        o.lanes_per_cell != 32 && o.lanes_per_cell != 64)
        return RKC_EINVAL;
    rkc_server *s = new (std::nothrow) rkc_server();
    if (!s) return RKC_ENOMEM;
    HipBackend &be = s->be;
    be.lanes = o.lanes_per_cell;
    be.placement = o.param_placement;
    int rc = RKC_OK;
    const size_t budget = o.budget_bytes / 256 * 256;
    if (hipGetDevice(&be.device) != hipSuccess) rc = RKC_EDEVICE;
    if (rc == RKC_OK && (hipMalloc(&be.arena_d, budget) != hipSuccess ||
                         hipHostMalloc(&be.mirror_h, budget, hipHostMallocDefault) != hipSuccess))
        rc = RKC_ENOMEM;
    be.slots.resize((size_t)o.n_streams);
    for (Slot &sl : be.slots) {
        if (rc) break;
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess)
            rc = RKC_EDEVICE;
        else if (hipMalloc(&sl.agg_d, rkchost::AGG_N * 8) != hipSuccess ||
                 hipMalloc(&sl.queue_d, sizeof(int)) != hipSuccess ||
                 hipHostMalloc(&sl.agg_h, rkchost::AGG_N * 8, hipHostMallocDefault) != hipSuccess)
            rc = RKC_ENOMEM;
    }
    if (rc) {
        release(s);
        return rc;
    }
    s->core = new (std::nothrow) rkcsrv::Core<HipBackend>(&be, budget, o.n_streams,
                                                          (size_t)o.max_batch_cells);
    if (!s->core) {
        release(s);
        return RKC_ENOMEM;
    }
    try {
        s->th = std::thread(dispatcher, s);
    } catch (...) {
        release(s);
        return RKC_ENOMEM;
    }
    *out = s;
    return RKC_OK;
}

int rkc_server_destroy(rkc_server *s) {
    if (!s) return RKC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(s->be.device);
    for (Slot &sl : s->be.slots)
        if (sl.st) (void)hipStreamSynchronize(sl.st);
    release(s);
    return RKC_OK;
}

int rkc_server_register_mech(rkc_server *s, const rkc_mech_desc *desc, int32_t *mech_id) {
    if (!s || !desc || !mech_id) return RKC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return RKC_EDEVICE;
    if (cur != s->be.device && hipSetDevice(s->be.device) != hipSuccess) return RKC_EDEVICE;
    rkc_mech *m = nullptr;
    int rc = rkc_mech_create(desc, &m);
    if (rc == RKC_OK) {
        rkc_opts o;
        rkc_opts_default(&o);
        o.lanes_per_cell = s->be.lanes;
        o.param_placement = s->be.placement;
        rc = rkchost::prepare(m, o, 0);
        if (rc) rkc_mech_destroy(m);
    }
    if (cur != s->be.device) (void)hipSetDevice(cur);
    if (rc) return rc;
    s->be.mechs.push_back(m);
    *mech_id = (int32_t)(s->be.mechs.size() - 1);
    return RKC_OK;
}

int rkc_server_submit(rkc_server *s, int32_t mech_id, size_t n, double *T, const double *P,
                      double *Y, double dt, double rtol, double atol, int32_t method,
                      int32_t *cell_status, uint64_t *req_id) {
    if (!s || !req_id) return RKC_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop || mech_id < 0 || (size_t)mech_id >= s->be.mechs.size()) return RKC_EINVAL;
    rkc_opts o;
    rkc_opts_default(&o);
    o.method = method;
    int rc = rkchost::check_integrate_args(dt, rtol, atol, o);
    if (rc) return rc;
    if (n > RKC_MAX_CELLS) return RKC_ENOTSUP;
    if (n > 0 && (!T || !P || !Y)) return RKC_EINVAL;
    rkcsrv::Request r;
    r.mech = mech_id;
    r.n = n;
    r.n_species = (size_t)rkchost::mech_species(s->be.mechs[(size_t)mech_id]);
    r.T = T; r.P = P; r.Y = Y; r.status = cell_status;
    r.dt = dt; r.rtol = rtol; r.atol = atol; r.method = method;
    rc = s->core->submit(r, req_id);
    if (rc) return rc;
    lk.unlock();
    s->cv_work.notify_one();
    return RKC_OK;
}

int rkc_server_poll(rkc_server *s, uint64_t id, int32_t *done) {
    if (!s || !done) return RKC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const int st = s->core->state(id);
    if (st < 0) return RKC_EINVAL;
    *done = st == rkcsrv::RQ_DONE;
    return RKC_OK;
}

int rkc_server_wait(rkc_server *s, uint64_t id, int32_t *n_failed) {
    if (!s) return RKC_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->core->state(id) < 0) return RKC_EINVAL;
    s->cv_done.wait(lk, [&] { return s->core->state(id) == rkcsrv::RQ_DONE; });
    const rkcsrv::Request *r = s->core->get(id);
    const int rc = r->rc;
    if (n_failed) *n_failed = r->n_failed;
    s->core->forget(id);
    return rc;
}

int rkc_server_get_stats(rkc_server *s, rkc_server_stats *out) {
    if (!s || !out) return RKC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const rkcsrv::CoreStats c = s->core->stats();
    std::memset(out, 0, sizeof(*out));
    out->submitted = c.submitted;
    out->completed = c.completed;
    out->failed_requests = c.failed_requests;
    out->launches = c.launches;
    out->cells = c.cells;
    out->n_rhs = s->be.n_rhs;
    out->peak_bytes = c.peak_bytes;
    out->peak_queue = c.peak_queue;
    out->mean_ms = c.mean_ms;
    out->p50_ms = c.p50_ms;
    out->p99_ms = c.p99_ms;
    out->max_ms = c.max_ms;
    return RKC_OK;
}

int rkc_server_reset_stats(rkc_server *s) {
    if (!s) return RKC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->core->reset_stats();
    s->be.n_rhs = 0;
    return RKC_OK;
}

}  // extern "C"
