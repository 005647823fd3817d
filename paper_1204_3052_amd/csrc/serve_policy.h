// Request-server policy, kept free of HIP so that it can be exercised on a CPU
// against a simulated executor.
//
//  - Arena: first-fit allocator over the server's device-memory budget; every
//    admitted request that runs on its own stream holds one workspace region
//    (operands and partial powers stay on the device) until it completes.
//  - Scheduler: two FIFO queues.  Small float32 requests (n <= 256) need no
//    arena memory; whenever no batch is in flight, all of them that are
//    waiting (up to the batch capacity) leave together as one ragged batch,
//    so requests that arrive while others run join the next batch
//    (continuous batching).  Other requests are admitted in strict arrival
//    order when their workspace fits the remaining budget and a stream has
//    room; a request that does not fit blocks the ones behind it, so none
//    can starve.  A request larger than the whole budget is rejected at
//    submission.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace mpow {
namespace serve {

struct Req {
    uint64_t id = 0;
    int n = 0;
    int64_t p = 0;
    int mode = 0;
    size_t ws_bytes = 0;  // arena bytes (0 on the batched route)
    bool batched = false;
    double work = 0.0;    // (G(p) + 1) n^3, for stream choice
    double t_submit = 0.0, t_start = 0.0, t_end = 0.0;
    // payload (opaque to the policy)
    const float *A = nullptr;
    float *out = nullptr;
    double *scale = nullptr;
    // assigned by the scheduler
    size_t arena_off = 0;
    int stream = -1;
};

class Arena {
   public:
    static constexpr size_t kGranule = 256;
    explicit Arena(size_t capacity = 0) { reset(capacity); }
    void reset(size_t capacity) {
        cap_ = capacity / kGranule * kGranule;
        free_.clear();
        if (cap_) free_[0] = cap_;
        used_ = peak_ = 0;
    }
    static size_t granules(size_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }
    bool alloc(size_t bytes, size_t *off) {
        const size_t need = granules(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need;
                const size_t at = it->first + need;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += need;
                if (used_ > peak_) peak_ = used_;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        const size_t len = granules(bytes ? bytes : 1);
        auto it = free_.emplace(off, len).first;
        used_ -= len;
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
    size_t capacity() const { return cap_; }
    size_t in_use() const { return used_; }
    size_t peak() const { return peak_; }

   private:
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Launch {
    bool batched = false;
    int stream = -1;
    std::vector<Req *> reqs;
};

class Scheduler {
   public:
    Scheduler(size_t budget, int n_streams, int depth, int batch_cap)
        : arena_(budget), depth_(depth), batch_cap_(batch_cap),
          stream_depth_(n_streams, 0), stream_work_(n_streams, 0.0) {}

    // false: the request can never fit the budget (rejected)
    bool submit(Req *r) {
        if (!r->batched && Arena::granules(r->ws_bytes) > arena_.capacity()) return false;
        (r->batched ? small_ : large_).push_back(r);
        return true;
    }

    std::vector<Launch> next(bool batch_free) {
        std::vector<Launch> out;
        while (!large_.empty()) {
            Req *r = large_.front();
            int best = -1;
            for (int s = 0; s < (int)stream_depth_.size(); ++s)
                if (stream_depth_[s] < depth_ && (best < 0 || stream_work_[s] < stream_work_[best]))
                    best = s;
            if (best < 0) break;
            size_t off = 0;
            if (!arena_.alloc(r->ws_bytes, &off)) break;  // head of line waits for memory
            large_.pop_front();
            r->arena_off = off;
            r->stream = best;
            stream_depth_[best] += 1;
            stream_work_[best] += r->work;
            Launch l;
            l.stream = best;
            l.reqs.push_back(r);
            out.push_back(l);
        }
        if (batch_free && !small_.empty()) {
            Launch l;
            l.batched = true;
            while (!small_.empty() && (int)l.reqs.size() < batch_cap_) {
                l.reqs.push_back(small_.front());
                small_.pop_front();
            }
            out.push_back(l);
        }
        return out;
    }

    void finish_plain(Req *r) {
        arena_.release(r->arena_off, r->ws_bytes);
        stream_depth_[r->stream] -= 1;
        stream_work_[r->stream] -= r->work;
        if (stream_depth_[r->stream] == 0) stream_work_[r->stream] = 0.0;
    }

    size_t queued() const { return large_.size() + small_.size(); }
    const Arena &arena() const { return arena_; }
    int streams() const { return (int)stream_depth_.size(); }

   private:
    Arena arena_;
    int depth_, batch_cap_;
    std::vector<int> stream_depth_;
    std::vector<double> stream_work_;
    std::deque<Req *> large_, small_;
};

}  // namespace serve
}  // namespace mpow
