// serve_core.h -- continuous-batching scheduler for resize / warp requests
// (host logic only; the device side is an Exec policy, see serve.hip).
//
// Requests arrive over time and wait in a FIFO queue.  Whenever one of the
// `slots` in-flight batch slots is free, the scheduler admits queued requests
// in arrival order into a new batch while their output blocks fit in the
// output arena (the HBM budget) and the batch has room, and hands the batch to
// the executor.  Batches of different slots run concurrently on the device.
// When a batch completes, its requests complete and their slot is reused;
// output blocks stay allocated until the caller releases them.  Admission
// stops at the first request that does not fit (strict FIFO: a large request
// is never starved by smaller ones behind it).
//
// Plain C++: no HIP types, so the scheduler is tested on the CPU with a fake
// executor.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace kr {
namespace serve {

// First-fit allocator of offsets in [0, size), aligned blocks, coalescing free.
class Arena {
public:
    explicit Arena(size_t size = 0, size_t align = 256) : size_(size), align_(align)
    {
        if (size_ > 0)
            free_[0] = size_;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t round(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

    bool alloc(size_t bytes, size_t *off)
    {
        const size_t need = round(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need;
                const size_t start = it->first + need;
                free_.erase(it);
                if (rest > 0)
                    free_[start] = rest;
                taken_[*off] = need;
                used_ += need;
                return true;
            }
        }
        return false;
    }

    bool release(size_t off)
    {
        auto t = taken_.find(off);
        if (t == taken_.end())
            return false;
        size_t start = off, len = t->second;
        taken_.erase(t);
        used_ -= len;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                prev->second += len;
                return true;
            }
        }
        free_[start] = len;
        return true;
    }

    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &f : free_)
            m = std::max(m, f.second);
        return m;
    }

private:
    size_t size_, align_, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> taken_;  // offset -> length
};

struct Request {
    uint64_t id = 0;
    int op = 0;             // 0 resize, 1 warp
    const void *src = nullptr;
    int sh = 0, sw = 0, dh = 0, dw = 0;
    double m[6] = {0, 0, 0, 0, 0, 0};
    int flags = 0;
    size_t dst_bytes = 0;   // output block size
    double t_arrival = 0;   // scheduled arrival (caller's clock)
};

struct Admitted {
    Request req;
    size_t dst_off = 0;     // output block offset in the arena
};

struct Completion {
    uint64_t id;
    size_t dst_off;
    size_t dst_bytes;
    double t_done;
};

// Exec must provide:
//   bool launch(int slot, const std::vector<Admitted> &batch)  -- enqueue, true on success
//   bool done(int slot)                                          -- the slot's batch has finished
template <class Exec>
class Scheduler {
public:
    Scheduler(Exec &exec, size_t budget, int slots, int max_batch)
        : exec_(exec), arena_(budget), slots_(slots), max_batch_(max_batch), inflight_(slots)
    {
    }

    const Arena &arena() const { return arena_; }
    size_t queued() const { return queue_.size(); }
    int busy_slots() const
    {
        int n = 0;
        for (const auto &s : inflight_)
            n += s.busy ? 1 : 0;
        return n;
    }
    bool idle() const { return queue_.empty() && busy_slots() == 0; }

    // false if the request can never fit the budget
    bool submit(const Request &r)
    {
        if (arena_.round(r.dst_bytes) > arena_.size())
            return false;
        queue_.push_back(r);
        return true;
    }

    // Harvest finished batches (appending their requests to `out` with
    // t_done = now), then admit queued requests into free slots.  Returns
    // false if the executor failed to launch a batch (its requests are
    // returned to the front of the queue, their blocks released).
    bool step(double now, std::vector<Completion> &out)
    {
        for (int s = 0; s < slots_; s++) {
            Slot &sl = inflight_[s];
            if (sl.busy && exec_.done(s)) {
                for (const Admitted &a : sl.batch)
                    out.push_back(Completion{a.req.id, a.dst_off, a.req.dst_bytes, now});
                sl.batch.clear();
                sl.busy = false;
            }
        }
        for (int s = 0; s < slots_ && !queue_.empty(); s++) {
            Slot &sl = inflight_[s];
            if (sl.busy)
                continue;
            while (!queue_.empty() && (int)sl.batch.size() < max_batch_) {
                size_t off = 0;
                if (!arena_.alloc(queue_.front().dst_bytes, &off))
                    break;
                sl.batch.push_back(Admitted{queue_.front(), off});
                queue_.pop_front();
            }
            if (sl.batch.empty())
                break;  // the head of the queue waits for memory
            if (!exec_.launch(s, sl.batch)) {
                for (auto it = sl.batch.rbegin(); it != sl.batch.rend(); ++it) {
                    arena_.release(it->dst_off);
                    queue_.push_front(it->req);
                }
                sl.batch.clear();
                return false;
            }
            sl.busy = true;
        }
        return true;
    }

    bool release(size_t dst_off) { return arena_.release(dst_off); }

private:
    struct Slot {
        bool busy = false;
        std::vector<Admitted> batch;
    };
    Exec &exec_;
    Arena arena_;
    int slots_, max_batch_;
    std::deque<Request> queue_;
    std::vector<Slot> inflight_;
};

}  // namespace serve
}  // namespace kr
