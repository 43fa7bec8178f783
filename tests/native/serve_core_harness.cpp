// CPU harness for serve_core.h: the serving loop's pool, admission and batching policy
// driven by a fake executor on a simulated clock (no GPU), which can also fail chosen
// launches and chosen completions and hold results under pending reads.  Built by
// tests/test_serve_core.py.
#include <cstdint>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "serve_core.h"

using boys_serve::Core;
using boys_serve::Request;
using boys_serve::SlotStatus;
using boys_serve::State;

namespace {

struct FakeExec {
    const double *clock = nullptr;
    double bytes_per_s = 1e12;  // simulated device throughput
    double launch_overhead = 5e-6;
    int64_t tile = 2048;
    int64_t cap = 65536;
    std::vector<double> busy_until;
    int concurrent_max = 0;
    // failure injection: launch attempts (counted from 0) that fail, and launched batches
    // (counted from 0) whose completion reports a device error
    std::set<int> fail_launch, fail_done;
    int launches = 0, batches = 0;
    std::vector<int> slot_batch;  // batch number running on each slot
    // read tokens: each is the simulated time at which the read completes
    std::vector<double *> tokens_live;
    int tokens_freed = 0;

    int64_t tile_args() const { return tile; }
    int64_t max_tiles() const { return cap; }
    SlotStatus status(int s)
    {
        if (*clock < busy_until[s])
            return SlotStatus::Running;
        if (!slot_batch.empty() && fail_done.count(slot_batch[s]))
            return SlotStatus::Failed;
        return SlotStatus::Done;
    }
    bool read_done(void *t) { return *clock >= *static_cast<double *>(t); }
    void read_free(void *t)
    {
        for (size_t k = 0; k < tokens_live.size(); ++k)
            if (tokens_live[k] == t) {
                delete tokens_live[k];
                tokens_live.erase(tokens_live.begin() + k);
                ++tokens_freed;
                return;
            }
        std::abort();  // a token freed twice or never issued
    }
    void *read_token(double due)
    {
        tokens_live.push_back(new double(due));
        return tokens_live.back();
    }
    bool launch(int s, const std::vector<Request *> &b)
    {
        if (fail_launch.count(launches++))
            return false;
        if (slot_batch.empty())
            slot_batch.assign(busy_until.size(), -1);
        slot_batch[s] = batches++;
        double bytes = 0;
        for (const Request *r : b)
            bytes += (double)r->bytes;
        busy_until[s] = *clock + launch_overhead + bytes / bytes_per_s;
        int c = 0;
        for (double u : busy_until)
            c += u > *clock;
        if (c > concurrent_max)
            concurrent_max = c;
        return true;
    }
};

}  // namespace

extern "C" {

// Simulate requests arriving at t_arr[i] (sorted); every completed request is released at
// once.  Outputs per request: admit, launch, done times and slot; and global maxima.
int sim_run(int nreq, const double *t_arr, const int64_t *len, const int *nmax, const int *prec,
            int64_t budget, int slots, int max_batch, double bytes_per_s, double dt,
            double *t_admit, double *t_launch, double *t_done, int *slot, int *rc_submit,
            int64_t *max_in_use, int *max_inflight, int *max_concurrent, int *batches)
{
    double now = 0;
    FakeExec ex;
    ex.clock = &now;
    ex.bytes_per_s = bytes_per_s;
    ex.busy_until.assign(slots, -1.0);
    Core<FakeExec> core((uint64_t)budget, slots, max_batch, &ex);
    std::vector<uint64_t> ids(nreq, 0);
    std::vector<int> idx_of(nreq + 1, -1);
    static const double dummy = 0.0;
    int next = 0, done = 0, refused = 0;
    for (int guard = 0; guard < 50000000 && done + refused < nreq; ++guard) {
        while (next < nreq && t_arr[next] <= now) {
            uint64_t id = 0;
            rc_submit[next] = core.submit(len[next], nmax[next], prec[next], &dummy, now, &id);
            if (rc_submit[next] == 0) {
                ids[next] = id;
                if (id < idx_of.size())
                    idx_of[id] = next;
            } else {
                ++refused;
            }
            ++next;
        }
        core.step(now);
        for (uint64_t id : core.take_completed(1u << 20)) {
            const Request *r = core.find(id);
            const int i = idx_of[id];
            t_admit[i] = r->t_admit;
            t_launch[i] = r->t_launch;
            t_done[i] = r->t_done;
            slot[i] = r->slot;
            core.release(id);
            ++done;
        }
        now += dt;
    }
    const boys_serve::Stats st = core.stats();
    *max_in_use = (int64_t)st.max_bytes_in_use;
    *max_inflight = (int)st.max_inflight_requests;
    *max_concurrent = ex.concurrent_max;
    *batches = (int)st.batches;
    return done;
}

// Failure handling.  nreq requests of n arguments arrive at t = 0, 1e-4, 2e-4, ... on a
// core with `slots` slots and batches of at most max_batch requests; launch attempts in
// fail_launch[] fail, completions of batches in fail_done[] report a device error.  Every
// completed request is released at once.  Outputs per request: final state (3 done,
// 4 failed) and how many times poll reported it; returns the number of launch attempts,
// or a negative code when an invariant breaks (-1 a request reported twice or never,
// -2 memory left in the pool, -3 a failed request whose result was readable, -4 the
// simulation did not finish).
int sim_failures(int nreq, int64_t n, int slots, int max_batch, const int *fail_launch,
                 int nfl, const int *fail_done, int nfd, int *state_out, int *reports_out,
                 int *failed_stat)
{
    double now = 0;
    FakeExec ex;
    ex.clock = &now;
    ex.bytes_per_s = 1e11;
    ex.busy_until.assign(slots, -1.0);
    for (int k = 0; k < nfl; ++k)
        ex.fail_launch.insert(fail_launch[k]);
    for (int k = 0; k < nfd; ++k)
        ex.fail_done.insert(fail_done[k]);
    Core<FakeExec> core(1ull << 32, slots, max_batch, &ex);
    static const double dummy = 0.0;
    std::vector<uint64_t> ids(nreq);
    for (int i = 0; i < nreq; ++i) {
        state_out[i] = -1;
        reports_out[i] = 0;
    }
    int next = 0, reported = 0;
    for (int guard = 0; guard < 10000000 && reported < nreq; ++guard) {
        while (next < nreq && next * 1e-4 <= now) {
            if (core.submit(n, 4, 0, &dummy, now, &ids[next]) != 0)
                return -4;
            ++next;
        }
        core.step(now);
        for (uint64_t id : core.take_completed(1u << 20)) {
            const Request *r = core.find(id);
            const int i = (int)(id - ids[0]);
            if (r == nullptr || i < 0 || i >= nreq)
                return -1;
            state_out[i] = (int)r->state;
            reports_out[i]++;
            ++reported;
            // a failed request is not Done, so no read of it can be recorded
            if (r->state == State::Failed && core.add_read(id, &ex))
                return -3;
            core.release(id);
        }
        now += 1e-6;
    }
    for (int i = 0; i < nreq; ++i)
        if (reports_out[i] != 1)
            return -1;
    core.step(now);
    if (core.pool().in_use() != 0 || !core.idle())
        return -2;
    *failed_stat = (int)core.stats().failed;
    return ex.launches;
}

// Pending reads.  Request A (n arguments) completes; the client enqueues a read of its
// result that completes at t_read, then releases A at once.  Request B, submitted right
// after the release, fits the budget only once A's memory is free.  Outputs: the time A's
// memory was freed as seen by B's admission, pool bytes in use right after the release,
// and whether the token was freed exactly once.  Returns 0, or a negative code.
int sim_pending_read(int64_t n, double t_read, double *t_admit_b, uint64_t *in_use_after_release,
                     int *tokens_freed)
{
    double now = 0;
    FakeExec ex;
    ex.clock = &now;
    ex.bytes_per_s = 1e12;
    ex.busy_until.assign(1, -1.0);
    const uint64_t fp = boys_serve::footprint(n, 4, 0);
    Core<FakeExec> core(fp + fp / 2, 1, 16, &ex);  // room for one request, not two
    static const double dummy = 0.0;
    uint64_t a = 0, b = 0;
    if (core.submit(n, 4, 0, &dummy, now, &a) != 0)
        return -1;
    bool released = false;
    *t_admit_b = -1;
    for (int guard = 0; guard < 10000000; ++guard) {
        core.step(now);
        for (uint64_t id : core.take_completed(16)) {
            if (id == a) {
                void *tok = ex.read_token(t_read);
                if (!core.add_read(a, tok))
                    return -2;
                if (!core.release(a))
                    return -3;
                if (core.release(a))
                    return -4;  // a second release of the same request must fail
                if (core.add_read(a, ex.read_token(0.0)))
                    return -5;  // no reads after the release
                ex.read_free(ex.tokens_live.back());
                *in_use_after_release = core.pool().in_use();
                released = true;
                if (core.submit(n, 4, 0, &dummy, now, &b) != 0)
                    return -6;
            } else if (id == b) {
                *t_admit_b = core.find(b)->t_admit;
                core.release(b);
            }
        }
        if (*t_admit_b >= 0)
            break;
        now += 1e-6;
    }
    if (!released || *t_admit_b < 0)
        return -7;
    core.step(now);
    if (core.pool().in_use() != 0 || !ex.tokens_live.empty())
        return -8;
    *tokens_freed = ex.tokens_freed;
    return 0;
}

// Random alloc/free against the pool; checks no overlap, exact accounting, and full
// coalescing at the end.  Returns 0 when every invariant held.
int pool_fuzz(uint64_t seed, int ops, uint64_t capacity)
{
    std::mt19937_64 g(seed);
    boys_serve::Pool pool(capacity);
    struct Blk {
        uint64_t off, size;
    };
    std::vector<Blk> live;
    uint64_t acc = 0;
    for (int k = 0; k < ops; ++k) {
        if (live.empty() || (g() % 3) != 0) {
            const uint64_t want = 1 + g() % (capacity / 16);
            uint64_t off = 0;
            if (pool.alloc(want, &off)) {
                const uint64_t sz = boys_serve::align_up(want);
                for (const Blk &b : live)
                    if (off < b.off + b.size && b.off < off + sz)
                        return 1;  // overlap
                if (off % boys_serve::kAlign != 0 || off + sz > pool.capacity())
                    return 2;
                live.push_back({off, sz});
                acc += sz;
            } else if (pool.largest_free() >= boys_serve::align_up(want)) {
                return 3;  // refused although a block was large enough
            }
        } else {
            const size_t i = g() % live.size();
            if (!pool.release(live[i].off))
                return 4;
            acc -= live[i].size;
            live.erase(live.begin() + i);
        }
        if (pool.in_use() != acc)
            return 5;
    }
    for (const Blk &b : live)
        pool.release(b.off);
    if (pool.in_use() != 0 || pool.free_blocks() != 1 || pool.largest_free() != pool.capacity())
        return 6;
    if (pool.release(12345))
        return 7;  // releasing an unknown offset must fail
    return 0;
}

}  // extern "C"
