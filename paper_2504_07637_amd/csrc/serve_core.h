// serve_core.h -- host-side core of the serving loop (no HIP calls).
//
// Requests (one argument array each: n arguments, an order n_max, a precision class)
// arrive at any time.  The core
//   * admits them in arrival order while their device footprint fits the memory budget
//     (a first-fit pool over one device allocation); a request that does not fit waits
//     at the head of the queue until releases free enough memory (no reordering, so no
//     request starves);
//   * launches every admitted request at the next opportunity: whenever one of the K
//     execution slots (one HIP stream each) is free, all admitted, not yet launched
//     requests (up to a batch limit) go out as one batch.  Batches on different slots
//     overlap on the device; requests that arrive while others run join the next batch
//     (continuous batching);
//   * marks a batch's requests complete when the executor reports the slot done, and
//     keeps each result in the pool until the client releases it;
//   * fails a batch's requests, instead of completing them, when its launch could not be
//     enqueued or its completion reports a device error: a failed request is reported by
//     poll like a completed one, has no result, and is released like one (no retries);
//   * keeps a released request's memory allocated until every read of its result that
//     the client enqueued through the server (a "read token", an event on the client's
//     stream) has completed, so that a later request cannot overwrite a result that is
//     still being copied out.
// The executor is a template parameter: the library uses a HIP executor (streams, events,
// the batched kernel); the tests drive the same core with a fake executor on a simulated
// clock, which can also inject failed launches and failed completions.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

namespace boys_serve {

constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t v)
{
    return (v + kAlign - 1) / kAlign * kAlign;
}

// First-fit allocator over [0, capacity); free blocks are coalesced on release.
class Pool {
  public:
    explicit Pool(uint64_t capacity) : cap_(capacity / kAlign * kAlign)
    {
        if (cap_ > 0)
            free_[0] = cap_;
    }

    bool alloc(uint64_t bytes, uint64_t *off)
    {
        const uint64_t need = align_up(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const uint64_t o = it->first, sz = it->second;
                free_.erase(it);
                if (sz > need)
                    free_[o + need] = sz - need;
                used_[o] = need;
                in_use_ += need;
                *off = o;
                return true;
            }
        }
        return false;
    }

    bool release(uint64_t off)
    {
        auto u = used_.find(off);
        if (u == used_.end())
            return false;
        uint64_t o = off, sz = u->second;
        used_.erase(u);
        in_use_ -= sz;
        auto next = free_.lower_bound(o);
        if (next != free_.end() && o + sz == next->first) {
            sz += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == o) {
                o = prev->first;
                sz += prev->second;
                free_.erase(prev);
            }
        }
        free_[o] = sz;
        return true;
    }

    uint64_t capacity() const { return cap_; }
    uint64_t in_use() const { return in_use_; }
    size_t free_blocks() const { return free_.size(); }
    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (auto &kv : free_)
            m = std::max(m, kv.second);
        return m;
    }

  private:
    uint64_t cap_;
    uint64_t in_use_ = 0;
    std::map<uint64_t, uint64_t> free_;
    std::map<uint64_t, uint64_t> used_;
};

enum class State : int { Queued = 0, Admitted = 1, Launched = 2, Done = 3, Failed = 4,
                         Releasing = 5 };

// what the executor reports for a slot
enum class SlotStatus : int { Running = 0, Done = 1, Failed = 2 };

struct Request {
    uint64_t id = 0;
    int64_t n = 0;
    int32_t n_max = 0;
    int32_t prec = 0;
    const double *x_host = nullptr;
    uint64_t off = 0;      // pool offset: x at off, output at off + x_bytes
    uint64_t x_bytes = 0;  // aligned size of the x copy
    int64_t ld = 0;        // output row stride (elements)
    uint64_t bytes = 0;    // whole footprint
    int slot = -1;
    State state = State::Queued;
    std::vector<void *> reads;  // executor tokens of enqueued reads of the result
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
};

// precision classes: 0 binary64, 1 mixed (binary32 output), 2 binary64 (order n+1 trick),
// 3 binary32 output computed in binary64, 4 all binary32
inline uint64_t elem_size(int32_t prec)
{
    return prec == 1 || prec == 3 || prec == 4 ? 4u : 8u;
}

// row stride of a request's output: every row starts on a 128-byte boundary
inline int64_t padded_ld(int64_t n, int32_t prec)
{
    const int64_t q = 128 / (int64_t)elem_size(prec);
    return (n + q - 1) / q * q;
}

inline uint64_t out_bytes(int64_t n, int32_t n_max, int32_t prec)
{
    return (uint64_t)(n_max + 1) * (uint64_t)padded_ld(n, prec) * elem_size(prec);
}

inline uint64_t footprint(int64_t n, int32_t n_max, int32_t prec)
{
    return align_up((uint64_t)n * 8u) + align_up(out_bytes(n, n_max, prec));
}

struct Stats {
    uint64_t submitted = 0, admitted = 0, launched = 0, completed = 0, released = 0;
    uint64_t failed = 0;  // requests whose batch failed (also counted in completed)
    uint64_t batches = 0;
    uint64_t queued_now = 0, admitted_now = 0, inflight_now = 0;
    uint64_t max_queued = 0, max_inflight_requests = 0;
    uint64_t bytes_in_use = 0, max_bytes_in_use = 0;
};

// Exec must provide:
//   SlotStatus status(int slot)                           -- the slot's last batch: running,
//                                                            finished, or failed on the device
//   bool launch(int slot, const std::vector<Request*>&)   -- enqueue a batch on the slot; on
//                                                            false nothing of it is pending
//   bool read_done(void *token), void read_free(void *token) -- read tokens (see above)
//   int64_t tile_args() const, int64_t max_tiles() const  -- per-batch tile capacity
template <class Exec>
class Core {
  public:
    Core(uint64_t budget, int slots, int max_batch, Exec *ex)
        : pool_(budget), slots_(slots), busy_(slots), max_batch_(max_batch), ex_(ex)
    {
    }

    // 0 ok, 1 invalid, 3 larger than the whole budget or the per-batch tile capacity
    int submit(int64_t n, int32_t n_max, int32_t prec, const double *x_host, double now,
               uint64_t *id)
    {
        if (n <= 0 || n_max < 0 || prec < 0 || prec > 4 || x_host == nullptr)
            return 1;
        const uint64_t fp = footprint(n, n_max, prec);
        const int64_t tiles = (n + ex_->tile_args() - 1) / ex_->tile_args();
        if (fp > pool_.capacity() || tiles > ex_->max_tiles())
            return 3;
        Request r;
        r.id = next_id_++;
        r.n = n;
        r.n_max = n_max;
        r.prec = prec;
        r.x_host = x_host;
        r.bytes = fp;
        r.x_bytes = align_up((uint64_t)n * 8u);
        r.ld = padded_ld(n, prec);
        r.t_submit = now;
        reqs_[r.id] = r;
        queue_.push_back(r.id);
        ++st_.submitted;
        st_.max_queued = std::max<uint64_t>(st_.max_queued, queue_.size());
        *id = r.id;
        return 0;
    }

    // poll completions and pending reads, admit by memory, launch on free slots
    void step(double now)
    {
        for (int s = 0; s < slots_; ++s) {
            if (busy_[s].empty())
                continue;
            const SlotStatus ss = ex_->status(s);
            if (ss == SlotStatus::Running)
                continue;
            for (uint64_t id : busy_[s]) {
                finish(reqs_[id], ss == SlotStatus::Done ? State::Done : State::Failed, now);
                --inflight_;
            }
            busy_[s].clear();
        }
        for (auto it = releasing_.begin(); it != releasing_.end();) {
            Request &r = reqs_[*it];
            drop_finished_reads(r);
            if (r.reads.empty()) {
                free_request(*it);
                it = releasing_.erase(it);
            } else {
                ++it;
            }
        }
        while (!queue_.empty()) {
            Request &r = reqs_[queue_.front()];
            uint64_t off = 0;
            if (!pool_.alloc(r.bytes, &off))
                break;  // head waits for memory; arrival order is kept
            r.off = off;
            r.state = State::Admitted;
            r.t_admit = now;
            admitted_.push_back(r.id);
            queue_.pop_front();
            ++st_.admitted;
        }
        for (int s = 0; s < slots_ && !admitted_.empty(); ++s) {
            if (!busy_[s].empty())
                continue;
            std::vector<Request *> batch;
            int64_t tiles = 0;
            while (!admitted_.empty() && (int)batch.size() < max_batch_) {
                Request &r = reqs_[admitted_.front()];
                const int64_t t = (r.n + ex_->tile_args() - 1) / ex_->tile_args();
                if (!batch.empty() && tiles + t > ex_->max_tiles())
                    break;
                tiles += t;
                batch.push_back(&r);
                admitted_.pop_front();
            }
            if (!ex_->launch(s, batch)) {
                // the batch fails as a whole (no retry: a launch that failed once, for a
                // reason the core cannot see, would most likely fail again); the slot
                // stays free, since the executor left nothing of the batch pending
                for (Request *r : batch) {
                    r->t_launch = now;
                    finish(*r, State::Failed, now);
                }
                launch_failures_++;
                continue;
            }
            for (Request *r : batch) {
                r->state = State::Launched;
                r->t_launch = now;
                r->slot = s;
                busy_[s].push_back(r->id);
            }
            st_.launched += batch.size();
            ++st_.batches;
            inflight_ += batch.size();
            st_.max_inflight_requests = std::max<uint64_t>(st_.max_inflight_requests, inflight_);
        }
        st_.bytes_in_use = pool_.in_use();
        st_.max_bytes_in_use = std::max(st_.max_bytes_in_use, st_.bytes_in_use);
    }

    std::vector<uint64_t> take_completed(size_t max)
    {
        std::vector<uint64_t> out;
        while (!completed_.empty() && out.size() < max) {
            out.push_back(completed_.front());
            completed_.pop_front();
        }
        return out;
    }

    const Request *find(uint64_t id) const
    {
        auto it = reqs_.find(id);
        return it == reqs_.end() ? nullptr : &it->second;
    }

    // record a read of a completed request's result enqueued by the client (the token
    // is the executor's); false if the request is not completed or was released
    bool add_read(uint64_t id, void *token)
    {
        auto it = reqs_.find(id);
        if (it == reqs_.end() || it->second.state != State::Done)
            return false;
        it->second.reads.push_back(token);
        return true;
    }

    // only completed (or failed) requests can be released; their device memory is freed
    // at once, or, while reads of the result are pending, once the last of them completes
    bool release(uint64_t id)
    {
        auto it = reqs_.find(id);
        if (it == reqs_.end() ||
            (it->second.state != State::Done && it->second.state != State::Failed))
            return false;
        Request &r = it->second;
        ++st_.released;
        drop_finished_reads(r);
        if (r.reads.empty()) {
            free_request(id);
        } else {
            r.state = State::Releasing;
            releasing_.push_back(id);
        }
        return true;
    }

    // nothing admitted and waiting for a slot, nothing running, no released memory
    // waiting for reads, and the queue is empty or its head does not fit the free memory
    // (only releases by the client can admit it)
    bool quiescent() const
    {
        if (!admitted_.empty() || !releasing_.empty())
            return false;
        for (auto &b : busy_)
            if (!b.empty())
                return false;
        if (queue_.empty())
            return true;
        const Request &head = reqs_.at(queue_.front());
        return pool_.largest_free() < align_up(head.bytes);
    }

    bool idle() const
    {
        if (!queue_.empty() || !admitted_.empty() || !releasing_.empty())
            return false;
        for (auto &b : busy_)
            if (!b.empty())
                return false;
        return true;
    }

    Stats stats() const
    {
        Stats s = st_;
        s.queued_now = queue_.size();
        s.admitted_now = admitted_.size();
        s.inflight_now = inflight_;
        s.bytes_in_use = pool_.in_use();
        return s;
    }

    const Pool &pool() const { return pool_; }
    uint64_t launch_failures() const { return launch_failures_; }

  private:
    void finish(Request &r, State st, double now)
    {
        r.state = st;
        r.t_done = now;
        completed_.push_back(r.id);
        ++st_.completed;
        if (st == State::Failed)
            ++st_.failed;
    }

    void drop_finished_reads(Request &r)
    {
        auto &v = r.reads;
        for (size_t k = 0; k < v.size();) {
            if (ex_->read_done(v[k])) {
                ex_->read_free(v[k]);
                v[k] = v.back();
                v.pop_back();
            } else {
                ++k;
            }
        }
    }

    void free_request(uint64_t id)
    {
        auto it = reqs_.find(id);
        pool_.release(it->second.off);
        reqs_.erase(it);
        st_.bytes_in_use = pool_.in_use();
    }

    Pool pool_;
    int slots_;
    std::vector<std::vector<uint64_t>> busy_;
    int max_batch_;
    Exec *ex_;
    uint64_t next_id_ = 1;
    std::unordered_map<uint64_t, Request> reqs_;
    std::deque<uint64_t> queue_;
    std::deque<uint64_t> admitted_;
    std::deque<uint64_t> completed_;
    std::vector<uint64_t> releasing_;
    uint64_t inflight_ = 0;
    uint64_t launch_failures_ = 0;
    Stats st_;
};

}  // namespace boys_serve
