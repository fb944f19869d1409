// Scheduling core of the integration server: request queue, admission by
// device-memory footprint, batching of compatible requests into one launch,
// launch slots, completion and latency bookkeeping.
//
// The core holds no device code and no HIP types; everything that touches a
// device goes through the Backend, which provides
//   int  start(Batch &b);   enqueue copies in, the launch and copies out of a
//                           batch whose arena region and slot are assigned;
//                           RKC_OK or a negative code
//   int  poll(Batch &b);    1 when the batch's work has completed (it then sets
//                           each request's rc and n_failed), 0 while pending,
//                           a negative code on failure
//   double now();           seconds on a monotonic clock
// Methods of Core are not thread-safe by themselves: the server wraps them in
// its own lock.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "rkc.h"

namespace rkcsrv {

enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct Request {
    uint64_t id = 0;
    int mech = 0;
    size_t n = 0;          // cells
    size_t n_species = 0;
    size_t bytes = 0;      // device footprint
    double *T = nullptr;
    const double *P = nullptr;
    double *Y = nullptr;
    int32_t *status = nullptr;
    double dt = 0, rtol = 0, atol = 0;
    int method = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int state = RQ_QUEUED;
    int rc = RKC_OK;
    int32_t n_failed = 0;
    size_t cell0 = 0;      // first cell inside its batch
};

struct Batch {
    std::vector<Request *> reqs;
    size_t cells = 0, bytes = 0, offset = 0;
    int slot = -1;
    void *backend_state = nullptr;   // owned by the backend between start and poll
};

// Device bytes of a request's state: T, P, Y and per-cell status, each array
// aligned to 256 bytes.
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
inline size_t footprint(size_t n, size_t n_species) {
    return align256(8 * n) * 2 + align256(8 * n * n_species) + align256(4 * n);
}

// First-fit allocator over [0, size) in 256-byte units, coalescing on free.
class Arena {
 public:
    explicit Arena(size_t size = 0) { reset(size); }
    void reset(size_t size) {
        size_ = size / 256 * 256;
        free_.clear();
        if (size_) free_[0] = size_;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    void reset_peak() { peak_ = used_; }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &f : free_) m = std::max(m, f.second);
        return m;
    }

 private:
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
};

struct CoreStats {
    int64_t submitted = 0, completed = 0, failed_requests = 0, launches = 0, cells = 0;
    int64_t peak_bytes = 0, peak_queue = 0;
    double mean_ms = 0, p50_ms = 0, p99_ms = 0, max_ms = 0;
};

// Nearest-rank percentile (the ceil(q n)-th smallest) of a sample.
inline double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t r = (size_t)std::ceil(q * (double)v.size());
    r = std::min(std::max<size_t>(r, 1), v.size());
    return v[r - 1];
}

template <class Backend>
class Core {
 public:
    Core(Backend *be, size_t budget, int n_slots, size_t max_batch_cells)
        : be_(be), arena_(budget), slots_(std::max(1, n_slots), false),
          max_batch_(std::max<size_t>(1, max_batch_cells)) {}

    // Queue a request.  RKC_ENOMEM for a request larger than the whole arena
    // (it could never be admitted).
    int submit(const Request &r0, uint64_t *id) {
        Request r = r0;
        r.bytes = footprint(r.n, r.n_species);
        if (r.bytes > arena_.size()) return RKC_ENOMEM;
        r.id = ++last_id_;
        r.t_submit = be_->now();
        r.state = RQ_QUEUED;
        ++st_.submitted;
        auto up = std::make_unique<Request>(r);
        if (r.n == 0) {   // nothing to integrate: complete at once
            up->state = RQ_DONE;
            up->t_start = up->t_done = r.t_submit;
            ++st_.completed;
            lat_ms_.push_back(0.0);
            *id = r.id;
            reqs_[r.id] = std::move(up);
            return RKC_OK;
        }
        queue_.push_back(up.get());
        reqs_[r.id] = std::move(up);
        st_.peak_queue = std::max<int64_t>(st_.peak_queue, (int64_t)queue_.size());
        *id = r.id;
        return RKC_OK;
    }

    // One round: retire completed batches, then admit queued requests while a
    // slot and arena space are free.  Returns a negative code if the backend
    // failed (the affected requests carry it as their rc).
    int pump() {
        int err = RKC_OK;
        for (size_t i = 0; i < running_.size();) {
            Batch &b = *running_[i];
            const int p = be_->poll(b);
            if (p == 0) { ++i; continue; }
            if (p < 0) {
                err = p;
                for (Request *r : b.reqs) r->rc = p;
            }
            finish(b);
            running_.erase(running_.begin() + (long)i);
        }
        while (!queue_.empty()) {
            int slot = -1;
            for (size_t s = 0; s < slots_.size(); ++s)
                if (!slots_[s]) { slot = (int)s; break; }
            if (slot < 0) break;
            auto b = std::make_unique<Batch>();
            if (!form_batch(b.get())) break;
            b->slot = slot;
            slots_[slot] = true;
            const double t = be_->now();
            for (Request *r : b->reqs) { r->state = RQ_RUNNING; r->t_start = t; }
            ++st_.launches;
            st_.cells += (int64_t)b->cells;
            const int rc = be_->start(*b);
            if (rc != RKC_OK) {
                err = rc;
                for (Request *r : b->reqs) r->rc = rc;
                finish(*b);
                continue;
            }
            running_.push_back(std::move(b));
        }
        return err;
    }

    bool idle() const { return queue_.empty() && running_.empty(); }
    bool queued() const { return !queue_.empty(); }
    bool busy() const { return !running_.empty(); }

    // State of a request: RQ_* or -1 for an unknown id.
    int state(uint64_t id) const {
        auto it = reqs_.find(id);
        return it == reqs_.end() ? -1 : it->second->state;
    }
    const Request *get(uint64_t id) const {
        auto it = reqs_.find(id);
        return it == reqs_.end() ? nullptr : it->second.get();
    }
    void forget(uint64_t id) { reqs_.erase(id); }

    CoreStats stats() const {
        CoreStats s = st_;
        s.peak_bytes = (int64_t)arena_.peak();
        if (!lat_ms_.empty()) {
            double sum = 0, mx = 0;
            for (double v : lat_ms_) { sum += v; mx = std::max(mx, v); }
            s.mean_ms = sum / (double)lat_ms_.size();
            s.max_ms = mx;
            s.p50_ms = percentile(lat_ms_, 0.50);
            s.p99_ms = percentile(lat_ms_, 0.99);
        }
        return s;
    }
    void reset_stats() {
        st_ = CoreStats();
        lat_ms_.clear();
        arena_.reset_peak();
    }
    const Arena &arena() const { return arena_; }

 private:
    static bool compatible(const Request &a, const Request &b) {
        return a.mech == b.mech && a.dt == b.dt && a.rtol == b.rtol && a.atol == b.atol &&
               a.method == b.method;
    }

    // The queue head plus any later compatible requests (queue order) that fit
    // the batch's cell limit; followers are dropped from the end until the
    // batch's region fits the arena.  False when not even the head fits now.
    bool form_batch(Batch *b) {
        Request *head = queue_.front();
        std::vector<Request *> pick{head};
        size_t cells = head->n;
        for (size_t i = 1; i < queue_.size(); ++i) {
            Request *r = queue_[i];
            if (compatible(*r, *head) && cells + r->n <= max_batch_) {
                pick.push_back(r);
                cells += r->n;
            }
        }
        for (;;) {
            size_t total = 0;
            for (Request *r : pick) total += r->n;
            const size_t bytes = footprint(total, head->n_species);
            size_t off = 0;
            if (arena_.alloc(bytes, &off)) {
                b->reqs = pick;
                b->cells = total;
                b->bytes = bytes;
                b->offset = off;
                size_t c0 = 0;
                for (Request *r : pick) { r->cell0 = c0; c0 += r->n; }
                // remove the picked requests from the queue, keeping the order of the rest
                std::deque<Request *> rest;
                size_t k = 0;
                for (Request *r : queue_) {
                    if (k < pick.size() && r == pick[k]) { ++k; continue; }
                    rest.push_back(r);
                }
                queue_.swap(rest);
                return true;
            }
            if (pick.size() == 1) return false;
            pick.pop_back();
        }
    }

    void finish(Batch &b) {
        arena_.release(b.offset, b.bytes);
        slots_[b.slot] = false;
        const double t = be_->now();
        for (Request *r : b.reqs) {
            r->t_done = t;
            r->state = RQ_DONE;
            ++st_.completed;
            if (r->rc != RKC_OK || r->n_failed > 0) ++st_.failed_requests;
            lat_ms_.push_back((r->t_done - r->t_submit) * 1e3);
        }
    }

    Backend *be_;
    Arena arena_;
    std::vector<bool> slots_;
    size_t max_batch_;
    uint64_t last_id_ = 0;
    std::deque<Request *> queue_;
    std::vector<std::unique_ptr<Batch>> running_;
    std::map<uint64_t, std::unique_ptr<Request>> reqs_;
    std::vector<double> lat_ms_;
    CoreStats st_;
};

}  // namespace rkcsrv
