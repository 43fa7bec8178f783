// CPU harness for serve_core.h: the serving loop's pool, admission and batching policy
// driven by a fake executor on a simulated clock (no GPU).  Built by tests/test_serve_core.py.
#include <cstdint>
#include <cstdlib>
#include <random>
#include <vector>

#include "serve_core.h"

using boys_serve::Core;
using boys_serve::Request;

namespace {

struct FakeExec {
    const double *clock = nullptr;
    double bytes_per_s = 1e12;  // simulated device throughput
    double launch_overhead = 5e-6;
    int64_t tile = 2048;
    int64_t cap = 65536;
    std::vector<double> busy_until;
    int concurrent_max = 0;

    int64_t tile_args() const { return tile; }
    int64_t max_tiles() const { return cap; }
    bool done(int s) { return *clock >= busy_until[s]; }
    bool launch(int s, const std::vector<Request *> &b)
    {
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
