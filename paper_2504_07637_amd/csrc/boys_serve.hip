// boys_serve.hip -- the serving loop of libboys.so (boys_server_* in boys.h).
//
// A scheduler thread drives serve_core.h's Core with a HIP executor:
//   * one device allocation of the budget is the pool; an admitted request owns a
//     contiguous piece of it: its x copy, then its (n_max+1) output rows, each starting
//     on a 128-byte boundary (ld = n rounded up to 16 binary64 / 32 binary32 elements);
//   * K execution slots, each a HIP stream with its own pinned staging and device
//     buffers for the descriptor and tile tables;
//   * a launch on a slot enqueues, in stream order, the host-to-device copies of the
//     batch's arguments and tables, then the batched kernel with one workgroup per tile
//     (the same per-argument bodies as boys_eval), then an event; the slot is free again
//     when the event has completed, which is also the completion time of its requests.
//     A launch that cannot be enqueued completely waits for what it did enqueue and
//     fails its batch; an event that reports a device error fails its batch too;
//   * boys_server_copy_result records an event on the client's stream after its copy;
//     a released request keeps its memory until those events have completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "boys.h"
#include "boys_internal.h"
#include "serve_core.h"

namespace {

using boys_internal::Desc;
using boys_serve::Request;

struct HipExec {
    int slots = 0;
    int64_t tile = 256;
    int64_t cap_tiles = 65536;
    int max_batch = 256;
    int grid = 1024;
    int block = 256;
    int schedule = 1;  // one workgroup per tile (tile = block x 1, 2 or 4)
    char *pool_base = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<Desc *> h_desc;
    std::vector<int2 *> h_tiles;
    std::vector<Desc *> d_desc;
    std::vector<int2 *> d_tiles;
    std::vector<hipEvent_t> read_events;       // every read event created
    std::vector<hipEvent_t> read_events_free;  // those not in use
    std::atomic<uint64_t> errors{0};

    int64_t tile_args() const { return tile; }
    int64_t max_tiles() const { return cap_tiles; }

    boys_serve::SlotStatus status(int s)
    {
        const hipError_t e = hipEventQuery(events[s]);
        if (e == hipSuccess)
            return boys_serve::SlotStatus::Done;
        if (e == hipErrorNotReady)
            return boys_serve::SlotStatus::Running;
        errors++;
        return boys_serve::SlotStatus::Failed;
    }

    // an event recorded on the client's stream after a read of a result (nullptr if none
    // could be recorded)
    void *read_token(hipStream_t client)
    {
        hipEvent_t ev = nullptr;
        if (!read_events_free.empty()) {
            ev = read_events_free.back();
            read_events_free.pop_back();
        } else {
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
                return nullptr;
            read_events.push_back(ev);
        }
        if (hipEventRecord(ev, client) != hipSuccess) {
            read_events_free.push_back(ev);
            return nullptr;
        }
        return ev;
    }

    // a read that reports a device error will never complete: its memory is given back
    bool read_done(void *t)
    {
        const hipError_t e = hipEventQuery(static_cast<hipEvent_t>(t));
        if (e == hipErrorNotReady)
            return false;
        if (e != hipSuccess)
            errors++;
        return true;
    }

    void read_free(void *t) { read_events_free.push_back(static_cast<hipEvent_t>(t)); }

    bool launch(int s, const std::vector<Request *> &batch)
    {
        const int nb = (int)batch.size();
        if (nb == 0 || nb > max_batch)
            return false;
        struct T {
            double cost;
            int32_t a, k;
        };
        std::vector<T> ts;
        int maxn = 0;
        for (int a = 0; a < nb; ++a) {
            const Request &r = *batch[a];
            char *base = pool_base + r.off;
            h_desc[s][a] = Desc{reinterpret_cast<const double *>(base), base + r.x_bytes, r.n, r.ld,
                                r.n_max, r.prec};
            maxn = std::max(maxn, r.n_max);
            const int64_t nt = (r.n + tile - 1) / tile;
            const double per = 8.0 + (r.n_max + 1) * (double)boys_serve::elem_size(r.prec);
            for (int64_t k = 0; k < nt; ++k) {
                const int64_t cnt = std::min<int64_t>(tile, r.n - k * tile);
                ts.push_back({per * (double)cnt, a, (int32_t)k});
            }
        }
        if ((int64_t)ts.size() > cap_tiles)
            return false;
        std::stable_sort(ts.begin(), ts.end(), [](const T &l, const T &r) { return l.cost > r.cost; });
        for (size_t i = 0; i < ts.size(); ++i)
            h_tiles[s][i] = make_int2(ts[i].a, ts[i].k);
        hipStream_t st = streams[s];
        bool ok = true;
        for (int a = 0; a < nb && ok; ++a) {
            const Request &r = *batch[a];
            ok = hipMemcpyAsync(pool_base + r.off, r.x_host, (size_t)r.n * 8, hipMemcpyHostToDevice,
                                st) == hipSuccess;
        }
        ok = ok && hipMemcpyAsync(d_desc[s], h_desc[s], sizeof(Desc) * nb, hipMemcpyHostToDevice,
                                  st) == hipSuccess;
        ok = ok && hipMemcpyAsync(d_tiles[s], h_tiles[s], sizeof(int2) * ts.size(),
                                  hipMemcpyHostToDevice, st) == hipSuccess;
        const boys_internal::Launch L{schedule, (int)tile, block, grid};
        ok = ok && boys_internal::launch_batched(d_desc[s], d_tiles[s], (int32_t)ts.size(),
                                                 nullptr, maxn, L, st) == hipSuccess;
        ok = ok && hipEventRecord(events[s], st) == hipSuccess;
        if (!ok) {
            // wait for whatever part of the batch was enqueued (copies from the slot's
            // staging and into the requests' memory), so that nothing of it is pending
            (void)hipStreamSynchronize(st);
            (void)hipGetLastError();
            errors++;
        }
        return ok;
    }
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct boys_server {
    int device = 0;
    HipExec ex;
    boys_serve::Core<HipExec> *core = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop = false;
    std::chrono::steady_clock::time_point t0;
};

namespace {

void scheduler(boys_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        s->core->step(now_s(s->t0));
        if (s->core->idle()) {
            s->cv.wait_for(lk, std::chrono::microseconds(200));
        } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

void destroy_exec(HipExec &ex)
{
    // reads of results that clients enqueued and have not finished
    for (hipEvent_t ev : ex.read_events) {
        (void)hipEventSynchronize(ev);
        (void)hipEventDestroy(ev);
    }
    ex.read_events.clear();
    ex.read_events_free.clear();
    for (size_t i = 0; i < ex.streams.size(); ++i) {
        if (ex.streams[i]) {
            (void)hipStreamSynchronize(ex.streams[i]);
            (void)hipStreamDestroy(ex.streams[i]);
        }
        if (ex.events[i])
            (void)hipEventDestroy(ex.events[i]);
        if (ex.h_desc[i])
            (void)hipHostFree(ex.h_desc[i]);
        if (ex.h_tiles[i])
            (void)hipHostFree(ex.h_tiles[i]);
        if (ex.d_desc[i])
            (void)hipFree(ex.d_desc[i]);
        if (ex.d_tiles[i])
            (void)hipFree(ex.d_tiles[i]);
    }
    if (ex.pool_base)
        (void)hipFree(ex.pool_base);
    ex.pool_base = nullptr;
}

}  // namespace

extern "C" {

boys_status boys_server_create(boys_server **out, const boys_server_config *cfg)
{
    if (out == nullptr || cfg == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    const int streams = cfg->streams > 0 ? cfg->streams : 4;
    const int max_batch = cfg->max_batch > 0 ? cfg->max_batch : 256;
    const int tile = cfg->tile > 0 ? cfg->tile : 256;
    const int max_tiles = cfg->max_tiles > 0 ? cfg->max_tiles : 65536;
    if (cfg->budget_bytes <= 0 || streams > 32 || max_batch > 65536 ||
        !(tile == 256 || tile == 512 || tile == 1024) || max_tiles > (1 << 24))
        return BOYS_ERR_INVALID_ARGUMENT;
    boys_server *s = new (std::nothrow) boys_server();
    if (!s)
        return BOYS_ERR_OUT_OF_MEMORY;
    (void)hipGetDevice(&s->device);
    HipExec &ex = s->ex;
    ex.slots = streams;
    ex.tile = tile;
    ex.cap_tiles = max_tiles;
    ex.max_batch = max_batch;
    ex.block = 256;
    ex.grid = boys_internal::cu_count() * 4;
    ex.streams.assign(streams, nullptr);
    ex.events.assign(streams, nullptr);
    ex.h_desc.assign(streams, nullptr);
    ex.h_tiles.assign(streams, nullptr);
    ex.d_desc.assign(streams, nullptr);
    ex.d_tiles.assign(streams, nullptr);
    bool ok = hipMalloc(&ex.pool_base, (size_t)cfg->budget_bytes) == hipSuccess;
    boys_status st = ok ? BOYS_OK : BOYS_ERR_OUT_OF_MEMORY;
    for (int i = 0; i < streams && ok; ++i) {
        ok = hipStreamCreateWithFlags(&ex.streams[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&ex.events[i], hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc((void **)&ex.h_desc[i], sizeof(Desc) * max_batch, hipHostMallocDefault) ==
                 hipSuccess &&
             hipHostMalloc((void **)&ex.h_tiles[i], sizeof(int2) * max_tiles, hipHostMallocDefault) ==
                 hipSuccess &&
             hipMalloc(&ex.d_desc[i], sizeof(Desc) * max_batch) == hipSuccess &&
             hipMalloc(&ex.d_tiles[i], sizeof(int2) * max_tiles) == hipSuccess;
        if (!ok)
            st = BOYS_ERR_OUT_OF_MEMORY;
    }
    if (!ok) {
        (void)hipGetLastError();
        destroy_exec(ex);
        delete s;
        return st;
    }
    s->core = new (std::nothrow) boys_serve::Core<HipExec>((uint64_t)cfg->budget_bytes, streams,
                                                           max_batch, &s->ex);
    if (!s->core) {
        destroy_exec(ex);
        delete s;
        return BOYS_ERR_OUT_OF_MEMORY;
    }
    s->t0 = std::chrono::steady_clock::now();
    try {
        s->th = std::thread(scheduler, s);
    } catch (...) {
        delete s->core;
        destroy_exec(ex);
        delete s;
        return BOYS_ERR_DEVICE;
    }
    *out = s;
    return BOYS_OK;
}

boys_status boys_server_submit(boys_server *s, const double *x_host, int64_t n, int32_t n_max,
                               int32_t precision, uint64_t *id)
{
    if (s == nullptr || id == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    if (boys_max_nmax(precision) < 0)
        return BOYS_ERR_INVALID_ARGUMENT;
    if (n_max < 0 || n_max > boys_max_nmax(precision))
        return BOYS_ERR_UNSUPPORTED_NMAX;
    int rc;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        rc = s->core->submit(n, n_max, precision, x_host, now_s(s->t0), id);
    }
    s->cv.notify_one();
    if (rc == 1)
        return BOYS_ERR_INVALID_ARGUMENT;
    if (rc == 3)
        return BOYS_ERR_OUT_OF_MEMORY;
    return BOYS_OK;
}

int32_t boys_server_poll(boys_server *s, uint64_t *ids, int32_t max)
{
    if (s == nullptr || ids == nullptr || max <= 0)
        return 0;
    std::lock_guard<std::mutex> lk(s->mu);
    const std::vector<uint64_t> done = s->core->take_completed((size_t)max);
    std::copy(done.begin(), done.end(), ids);
    return (int32_t)done.size();
}

boys_status boys_server_result(boys_server *s, uint64_t id, const void **out, int64_t *ld,
                               double *t_submit, double *t_done)
{
    if (s == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(s->mu);
    const Request *r = s->core->find(id);
    if (r != nullptr && r->state == boys_serve::State::Failed)
        return BOYS_ERR_DEVICE;
    if (r == nullptr || r->state != boys_serve::State::Done)
        return BOYS_ERR_INVALID_ARGUMENT;
    if (out)
        *out = s->ex.pool_base + r->off + r->x_bytes;
    if (ld)
        *ld = r->ld;
    if (t_submit)
        *t_submit = r->t_submit;
    if (t_done)
        *t_done = r->t_done;
    return BOYS_OK;
}

boys_status boys_server_copy_result(boys_server *s, uint64_t id, void *dst, int64_t ld_dst,
                                    void *stream)
{
    if (s == nullptr || dst == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    const void *src;
    size_t width, rows, spitch;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const Request *r = s->core->find(id);
        if (r != nullptr && r->state == boys_serve::State::Failed)
            return BOYS_ERR_DEVICE;
        if (r == nullptr || r->state != boys_serve::State::Done || ld_dst < r->n)
            return BOYS_ERR_INVALID_ARGUMENT;
        const size_t es = boys_serve::elem_size(r->prec);
        src = s->ex.pool_base + r->off + r->x_bytes;
        width = (size_t)r->n * es;
        spitch = (size_t)r->ld * es;
        rows = (size_t)r->n_max + 1;
        const size_t dpitch = (size_t)ld_dst * es;
        const hipStream_t cs = static_cast<hipStream_t>(stream);
        if (hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, hipMemcpyDeviceToDevice,
                             cs) != hipSuccess)
            return BOYS_ERR_DEVICE;
        // the request's memory must outlive this copy, even if it is released at once
        void *tok = s->ex.read_token(cs);
        if (tok == nullptr || !s->core->add_read(id, tok)) {
            if (tok != nullptr)
                s->ex.read_free(tok);
            // no event to track the copy: let it finish before returning
            if (hipStreamSynchronize(cs) != hipSuccess)
                return BOYS_ERR_DEVICE;
        }
    }
    return BOYS_OK;
}

boys_status boys_server_release(boys_server *s, uint64_t id)
{
    if (s == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    bool ok;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        ok = s->core->release(id);
    }
    s->cv.notify_one();
    return ok ? BOYS_OK : BOYS_ERR_INVALID_ARGUMENT;
}

boys_status boys_server_get_stats(boys_server *s, boys_server_stats *out)
{
    if (s == nullptr || out == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(s->mu);
    const boys_serve::Stats st = s->core->stats();
    out->submitted = st.submitted;
    out->admitted = st.admitted;
    out->launched = st.launched;
    out->completed = st.completed;
    out->released = st.released;
    out->batches = st.batches;
    out->queued_now = st.queued_now;
    out->inflight_now = st.inflight_now;
    out->max_queued = st.max_queued;
    out->max_inflight = st.max_inflight_requests;
    out->bytes_in_use = st.bytes_in_use;
    out->max_bytes_in_use = st.max_bytes_in_use;
    out->device_errors = s->ex.errors.load();
    out->failed = st.failed;
    return BOYS_OK;
}

boys_status boys_server_drain(boys_server *s, double timeout_s)
{
    if (s == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    const auto t_end = std::chrono::steady_clock::now() +
                       std::chrono::microseconds((int64_t)(timeout_s * 1e6));
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->core->quiescent())
                return s->ex.errors.load() ? BOYS_ERR_DEVICE : BOYS_OK;
        }
        if (std::chrono::steady_clock::now() > t_end)
            return BOYS_ERR_DEVICE;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

void boys_server_destroy(boys_server *s)
{
    if (s == nullptr)
        return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_one();
    if (s->th.joinable())
        s->th.join();
    destroy_exec(s->ex);
    delete s->core;
    delete s;
}

}  // extern "C"
