// Admission and completion logic of the continuous-batching server, independent of the device: the
// server (serve.cpp) runs it with its HIP backend, the tests with a host-only one.
//
// Requests wait in arrival order.  Whenever an arena (one in-flight batch's share of the HBM budget and
// a stream) is idle, it takes, in arrival order, every pending request that (a) fits the arena's bytes,
// (b) touches no env slot that an in-flight batch or an earlier request of this batch touches, and
// (c) keeps the batch within max_batch_agents.  A request that does not fit the arena stops the scan
// (requests behind it wait: no starvation); a request that conflicts on an env slot keeps its place, and
// so does every later request that shares a slot with it, so requests on one slot run in arrival order.
//
// When the backend reports a batch failed (a launch error, or an error forced from the host), the
// backend first restores the batch's env slots to their states before the batch; the requests then go
// back to the front of the queue in their order and run again, at most max_attempts times in all, after
// which they fail.  Requests touching one slot therefore run in arrival order, and a request's result is
// the same whether its batch failed before or not.  Data errors a batch's kernels flag fail that batch's
// requests (running them again would flag them again).
#pragma once

#include <stdint.h>

#include <deque>
#include <string>
#include <unordered_set>
#include <vector>

namespace vf {
namespace sched {

enum : int32_t { kOk = 0, kFailed = -4 /* VF_EHIP */, kDataError = -6 /* VF_EDEVICE */, kNoMemory = -2 };

// What the scheduler needs of a request (the server's request type derives from it).
struct Item {
    std::vector<int32_t> slots;   // env slots the request steps (distinct)
    int32_t n_env = 0;
    int64_t bytes = 0;            // arena bytes it needs
    int32_t attempts = 0;         // batches it was launched in
    bool done = false;
    int32_t status = kOk;
    std::string why;
};

struct Arena {
    bool busy = false;
    int64_t bytes = 0;
    std::vector<Item*> items;
};

struct Stats {
    int64_t batches = 0, agents = 0, requests = 0, max_batch = 0, requeued = 0, failed_batches = 0;
};

// Backend: bool launch(int arena, std::vector<Item*>& items)  -- enqueue the batch (false: it did not start)
//          int poll(int arena)        -- 1 finished, 0 still running, -1 failed
//          uint32_t finish(int arena, std::vector<Item*>& items)   -- deliver results; the data-error bits
//          bool restore(int arena, std::vector<Item*>& items)      -- undo the batch's step (false: cannot)
//          void on_done(Item*)        -- a request reached its final status
template <class Backend>
class Scheduler {
public:
    Scheduler(Backend& be, int n_arenas, int64_t arena_bytes, int64_t max_batch_agents, int32_t max_attempts)
        : be_(be), arenas_(n_arenas), max_batch_(max_batch_agents), max_attempts_(max_attempts) {
        for (auto& a : arenas_) a.bytes = arena_bytes;
    }

    void submit(Item* r) { pending_.push_back(r); }
    // forced backend errors: the next n batches that finish are treated as failed
    void inject_faults(int64_t n) { inject_ += n; }
    bool idle() const {
        if (!pending_.empty()) return false;
        for (const auto& a : arenas_)
            if (a.busy) return false;
        return true;
    }
    bool any_busy() const {
        for (const auto& a : arenas_)
            if (a.busy) return true;
        return false;
    }
    size_t pending() const { return pending_.size(); }
    int64_t in_flight() const {
        int64_t k = 0;
        for (const auto& a : arenas_) k += a.busy ? 1 : 0;
        return k;
    }
    const Stats& stats() const { return st_; }
    std::vector<Arena>& arenas() { return arenas_; }

    // One pass over completions and admissions; true when something changed.
    bool step() {
        bool progressed = false;
        for (int i = 0; i < (int)arenas_.size(); ++i) {
            Arena& a = arenas_[i];
            if (!a.busy) continue;
            const int q = be_.poll(i);
            if (q == 0) continue;
            progressed = true;
            bool failed = q < 0;
            if (!failed && inject_ > 0) {
                --inject_;
                failed = true;
            }
            if (failed) {
                fail_batch(i);
            } else {
                const uint32_t err = be_.finish(i, a.items);
                for (Item* r : a.items) {
                    if (err) {
                        r->status = kDataError;
                        if (r->why.empty()) r->why = "a kernel of the batch flagged bad data";
                    }
                    complete(r);
                }
                st_.requests += (int64_t)a.items.size();
                release(a);
            }
        }
        for (int i = 0; i < (int)arenas_.size(); ++i) {
            Arena& a = arenas_[i];
            if (a.busy || pending_.empty()) continue;
            int64_t used = 0, agents = 0;
            std::unordered_set<int32_t> batch_slots, held;   // held: slots of requests left waiting
            for (auto it = pending_.begin(); it != pending_.end();) {
                Item* r = *it;
                if (used + r->bytes > a.bytes || agents + r->n_env > max_batch_) break;
                bool conflict = false;
                for (int32_t sl : r->slots)
                    if (busy_slots_.count(sl) || batch_slots.count(sl) || held.count(sl)) {
                        conflict = true;
                        break;
                    }
                if (conflict) {
                    for (int32_t sl : r->slots) held.insert(sl);
                    ++it;
                    continue;
                }
                for (int32_t sl : r->slots) batch_slots.insert(sl);
                used += r->bytes;
                agents += r->n_env;
                a.items.push_back(r);
                it = pending_.erase(it);
            }
            if (a.items.empty()) continue;
            for (int32_t sl : batch_slots) busy_slots_.insert(sl);
            for (Item* r : a.items) ++r->attempts;
            progressed = true;
            if (be_.launch(i, a.items)) {
                a.busy = true;
                st_.batches += 1;
                st_.agents += agents;
                if (agents > st_.max_batch) st_.max_batch = agents;
            } else {
                fail_batch(i);
            }
        }
        return progressed;
    }

    // Fail every request still queued or in flight (server shutdown with work left, or a lost device).
    void fail_everything(const std::string& why) {
        for (auto& a : arenas_) {
            for (Item* r : a.items) {
                r->status = kFailed;
                r->why = why;
                complete(r);
            }
            release(a);
        }
        for (Item* r : pending_) {
            r->status = kFailed;
            r->why = why;
            complete(r);
        }
        pending_.clear();
    }

private:
    void complete(Item* r) {
        r->done = true;
        be_.on_done(r);
    }
    void release(Arena& a) {
        for (Item* r : a.items)
            for (int32_t sl : r->slots) busy_slots_.erase(sl);
        a.items.clear();
        a.busy = false;
    }
    // A batch that did not start or did not finish: restore its slots and queue its requests again at the
    // front (in their order), or fail them after max_attempts.
    void fail_batch(int i) {
        Arena& a = arenas_[i];
        st_.failed_batches += 1;
        const bool restored = be_.restore(i, a.items);
        std::vector<Item*> again;
        for (Item* r : a.items) {
            if (restored && r->attempts < max_attempts_) {
                again.push_back(r);
            } else {
                r->status = kFailed;
                r->why = restored ? "batch failed on every attempt" : "batch failed and its env slots could not be restored";
                complete(r);
            }
        }
        st_.requeued += (int64_t)again.size();
        release(a);
        for (auto it = again.rbegin(); it != again.rend(); ++it) pending_.push_front(*it);
    }

    Backend& be_;
    std::vector<Arena> arenas_;
    std::deque<Item*> pending_;
    std::unordered_set<int32_t> busy_slots_;
    int64_t max_batch_;
    int32_t max_attempts_;
    int64_t inject_ = 0;
    Stats st_;
};

}  // namespace sched
}  // namespace vf
