// boys_lib.hip -- host side and C ABI of libboys.so (see include/boys.h): argument
// checks, dispatch to the kernels (boys_kernels.h, instantiated in plain_inst.hip,
// batched_inst.hip, split_inst.hip and eri_inst.hip), batch schedules, plans with HIP
// graphs, the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <new>
#include <utility>
#include <vector>

#include "boys.h"
#include "boys_device.h"
#include "boys_internal.h"

namespace {

using boys_internal::Desc;
using boys_tab::kMaxN32;
using boys_tab::kMaxN32x;
using boys_tab::kMaxN64;

// n_max buckets of the batched kernels (the same list as boys_kernels.h's kBuckets)
constexpr int kMaxN = kMaxN64 > kMaxN32 ? (kMaxN64 > kMaxN32x ? kMaxN64 : kMaxN32x)
                                        : (kMaxN32 > kMaxN32x ? kMaxN32 : kMaxN32x);
constexpr int kBuckets[] = {4, 8, 16, 24, kMaxN};
constexpr int kNumBuckets = 5;


// ---------------------------------------------------------------------------------
// host helpers

int g_cu_count[64];
std::once_flag g_cu_once[64];

int cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    std::call_once(g_cu_once[dev], [dev] {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        g_cu_count[dev] = v;
    });
    return g_cu_count[dev];
}

using boys_internal::PlainLaunch;

PlainLaunch plain_launcher(int32_t prec, int n, bool select_rows)
{
    switch (prec) {
    case BOYS_FP64:
        return boys_internal::plain_launcher<BOYS_FP64>(n, select_rows);
    case BOYS_FP32:
        return boys_internal::plain_launcher<BOYS_FP32>(n, select_rows);
    case BOYS_FP64_PLUS:
        return boys_internal::plain_launcher<BOYS_FP64_PLUS>(n, select_rows);
    case BOYS_FP32X:
        return boys_internal::plain_launcher<BOYS_FP32X>(n, select_rows);
    case BOYS_FP32_SINGLE:
        return boys_internal::plain_launcher<BOYS_FP32_SINGLE>(n, select_rows);
    }
    return nullptr;
}

int max_nmax(int32_t prec)
{
    if (prec == BOYS_FP64)
        return kMaxN64;
    if (prec == BOYS_FP32)
        return kMaxN32;
    if (prec == BOYS_FP64_PLUS)
        return kMaxN64 - 1;
    if (prec == BOYS_FP32X)
        return kMaxN32x;
    if (prec == BOYS_FP32_SINGLE)
        return kMaxN32;
    return -1;
}

int elem_bytes(int32_t prec)
{
    return prec == BOYS_FP32 || prec == BOYS_FP32X || prec == BOYS_FP32_SINGLE ? 4 : 8;
}

boys_status check_array(const double *x, int64_t n, int32_t n_max, const void *out,
                        int64_t ld, int32_t prec)
{
    if (max_nmax(prec) < 0)
        return BOYS_ERR_INVALID_ARGUMENT;
    if (n < 0)
        return BOYS_ERR_INVALID_ARGUMENT;
    if (n_max < 0 || n_max > max_nmax(prec))
        return BOYS_ERR_UNSUPPORTED_NMAX;
    if (n == 0)
        return BOYS_OK;
    if (x == nullptr || out == nullptr || ld < n)
        return BOYS_ERR_INVALID_ARGUMENT;
    // the last output element must be addressable
    const int64_t lim = INT64_MAX / 8;
    if (ld > lim / (int64_t)(n_max + 1))
        return BOYS_ERR_INVALID_ARGUMENT;
    return BOYS_OK;
}

int bucket_of(int maxn)
{
    for (int b = 0; b < kNumBuckets; ++b)
        if (maxn <= kBuckets[b])
            return b;
    return kNumBuckets - 1;
}

using BucketLaunch = hipError_t (*)(const Desc *, const int2 *, int32_t, uint32_t *,
                                    const boys_internal::Launch &, hipStream_t);

template <int S, int K, int... B>
constexpr std::array<BucketLaunch, sizeof...(B)> bucket_table(std::integer_sequence<int, B...>)
{
    return {&boys_internal::launch_bucket<B, S, K>...};
}

// [shape][bucket]; shape 0 persistent, 1..3 one workgroup per tile with K = 1, 2, 4,
// 4 one wave per tile with K = 4
const std::array<std::array<BucketLaunch, kNumBuckets>, 5> kBucketLaunch = {
    bucket_table<0, 0>(std::make_integer_sequence<int, kNumBuckets>{}),
    bucket_table<1, 1>(std::make_integer_sequence<int, kNumBuckets>{}),
    bucket_table<1, 2>(std::make_integer_sequence<int, kNumBuckets>{}),
    bucket_table<1, 4>(std::make_integer_sequence<int, kNumBuckets>{}),
    bucket_table<2, 4>(std::make_integer_sequence<int, kNumBuckets>{})};

// row of kBucketLaunch for a tuning, -1 if that shape is not built
int shape_row(int schedule, int tile, int block)
{
    if (schedule == 0)
        return 0;
    if (schedule == 1 && tile % block == 0) {
        const int k = tile / block;
        return k == 1 ? 1 : k == 2 ? 2 : k == 4 ? 3 : -1;
    }
    if (schedule == 2)
        return tile == 256 ? 4 : -1;  // 64 lanes x 4 arguments
    return -1;
}

}  // namespace

hipError_t boys_internal::launch_batched(const Desc *d_desc, const int2 *d_tiles, int32_t ntiles,
                                         uint32_t *d_counter, int maxn, const Launch &L,
                                         hipStream_t s)
{
    const int row = shape_row(L.schedule, L.tile, L.block);
    if (row < 0)
        return hipErrorInvalidValue;
    return kBucketLaunch[row][bucket_of(maxn)](d_desc, d_tiles, ntiles, d_counter, L, s);
}

int boys_internal::cu_count()
{
    return ::cu_count();
}

// ---------------------------------------------------------------------------------
// plans

struct boys_plan {
    int device = 0;
    int32_t count = 0;
    std::vector<boys_array> arrays;   // shapes, for update checks
    std::vector<Desc> host_desc;
    Desc *d_desc = nullptr;
    int2 *d_tiles = nullptr;
    uint32_t *d_counter = nullptr;
    int32_t ntiles = 0;
    int32_t ntiles_hi = 0;  // split_nmax > 0: the first ntiles_hi tiles form their own launch
    boys_tuning tuning{};
    int grid = 0;
    int maxn = 0;     // largest n_max of the (other) tiles
    int maxn_hi = 0;  // largest n_max of the first ntiles_hi tiles
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // one event per stream the plan was executed on, recorded behind each execute, so
    // that update and destroy can wait for replays still reading the plan's tables
    std::vector<std::pair<hipStream_t, hipEvent_t>> exec_events;
};

namespace {

constexpr int kDefaultTile = 256;
constexpr int kDefaultBlock = 256;
constexpr int kDefaultGridPerCU = 4;
// with no tuning: one wave per 256-argument tile, array by array, in one launch (on the
// 8,192-array batch within 0.5% of the best shape measured, and 2-3% ahead of putting the
// store-bound arrays in a launch of their own)
constexpr int kDefaultSchedule = 2;
constexpr int kDefaultOrder = 1;
constexpr int kDefaultSplit = 0;

boys_tuning resolve(const boys_tuning *t)
{
    boys_tuning r{kDefaultTile, kDefaultBlock, kDefaultGridPerCU, kDefaultSchedule, kDefaultOrder,
                  kDefaultSplit};
    if (t) {
        if (t->tile > 0)
            r.tile = t->tile;
        if (t->block > 0)
            r.block = t->block;
        if (t->grid_per_cu > 0)
            r.grid_per_cu = t->grid_per_cu;
        r.schedule = t->schedule;
        r.order = t->order;
        r.split_nmax = t->split_nmax;
    }
    return r;
}

bool tuning_ok(const boys_tuning &t)
{
    const bool block_ok = t.block == 64 || t.block == 128 || t.block == 256;
    if (!block_ok || t.tile <= 0 || t.tile > (1 << 24))
        return false;
    if (t.order < 0 || t.order > 2)
        return false;
    if (t.split_nmax < 0 || t.split_nmax > 64 || (t.split_nmax != 0 && t.schedule != 2))
        return false;
    if (t.schedule == 0)
        return t.tile == 256 && t.grid_per_cu >= 1 && t.grid_per_cu <= 64;
    return shape_row(t.schedule, t.tile, t.block) >= 0;  // schedule 1: tile = block x K
}

boys_internal::Launch launch_of(const boys_plan *p)
{
    return boys_internal::Launch{p->tuning.schedule, p->tuning.tile, p->tuning.block, p->grid};
}

double tile_cost(const boys_array &a, int64_t cnt)
{
    const double bytes = 8.0 + (a.n_max + 1) * (elem_bytes(a.precision) * 1.0);
    return bytes * (double)cnt;
}

// wait for every execute of the plan enqueued so far
hipError_t wait_executes(boys_plan *p)
{
    hipError_t r = hipSuccess;
    for (auto &se : p->exec_events) {
        const hipError_t e = hipEventSynchronize(se.second);
        if (e != hipSuccess && r == hipSuccess)
            r = e;
    }
    return r;
}

void free_plan_buffers(boys_plan *p)
{
    (void)wait_executes(p);
    for (auto &se : p->exec_events)
        (void)hipEventDestroy(se.second);
    p->exec_events.clear();
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    if (p->d_desc)
        (void)hipFree(p->d_desc);
    if (p->d_tiles)
        (void)hipFree(p->d_tiles);
    if (p->d_counter)
        (void)hipFree(p->d_counter);
    p->exec = nullptr;
    p->graph = nullptr;
    p->d_desc = nullptr;
    p->d_tiles = nullptr;
    p->d_counter = nullptr;
}

boys_status build_schedule(boys_plan *p, const boys_array *arrays, int32_t count,
                           std::vector<int2> &tiles)
{
    p->arrays.assign(arrays, arrays + count);
    p->host_desc.resize(count);
    struct T {
        double cost;
        int32_t array;
        int32_t slice;
        bool hi;  // in the one-argument-per-lane launch (split_nmax > 0)
    };
    std::vector<T> all;
    int maxn = 0, maxn_hi = 0;
    const int split = p->tuning.split_nmax;
    for (int32_t a = 0; a < count; ++a) {
        const boys_array &A = arrays[a];
        p->host_desc[a] = Desc{A.x, A.out, A.n, A.ld_out, A.n_max, A.precision};
        const int64_t nt = (A.n + p->tuning.tile - 1) / p->tuning.tile;
        if (nt > INT32_MAX || (int64_t)all.size() + nt > INT32_MAX)
            return BOYS_ERR_INVALID_ARGUMENT;
        const bool hi =
            split > 0 && A.n_max >= split + (elem_bytes(A.precision) == 4 ? 4 : 0);
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t cnt = std::min<int64_t>(p->tuning.tile, A.n - t * p->tuning.tile);
            all.push_back({tile_cost(A, cnt), a, (int32_t)t, hi});
        }
        if (A.n > 0) {
            if (hi)
                maxn_hi = std::max(maxn_hi, A.n_max);
            else
                maxn = std::max(maxn, A.n_max);
        }
    }
    if (p->tuning.order == 0) {
        // longest processing time first (ties keep array order)
        std::stable_sort(all.begin(), all.end(),
                         [](const T &l, const T &r) { return l.cost > r.cost; });
    } else if (p->tuning.order == 2) {
        // by (precision, n_max) class, heavier classes first, then array by array
        std::stable_sort(all.begin(), all.end(), [arrays](const T &l, const T &r) {
            const boys_array &A = arrays[l.array], &B = arrays[r.array];
            const double ca = tile_cost(A, 1), cb = tile_cost(B, 1);
            if (ca != cb)
                return ca > cb;
            if (A.precision != B.precision)
                return A.precision < B.precision;
            return A.n_max > B.n_max;
        });
    }
    // order 1: as built, array by array with each array's tiles consecutive, so the
    // workgroups running at one time write neighbouring pieces of the same output rows.
    // The tiles of the store-bound arrays go first, in the same order, for their own launch.
    const auto mid = std::stable_partition(all.begin(), all.end(), [](const T &t) { return t.hi; });
    p->ntiles_hi = (int32_t)(mid - all.begin());
    p->maxn_hi = maxn_hi;
    tiles.resize(all.size());
    for (size_t i = 0; i < all.size(); ++i)
        tiles[i] = make_int2(all[i].array, all[i].slice);
    p->maxn = maxn;
    p->ntiles = (int32_t)all.size();
    return BOYS_OK;
}

boys_status capture_graph(boys_plan *p)
{
    if (p->ntiles == 0)
        return BOYS_OK;  // nothing to launch: execute is a no-op
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return BOYS_ERR_DEVICE;
    boys_status st = BOYS_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return BOYS_ERR_DEVICE;
    }
    // split plans: the store-bound arrays first, one workgroup of 256 threads per tile of
    // 256 arguments (the plan's tile size), then the rest per wave
    if (p->ntiles_hi > 0 &&
        boys_internal::launch_batched(p->d_desc, p->d_tiles, p->ntiles_hi, p->d_counter,
                                      p->maxn_hi, boys_internal::Launch{1, p->tuning.tile, 256, p->grid},
                                      s) != hipSuccess)
        st = BOYS_ERR_DEVICE;
    if (st == BOYS_OK && p->ntiles > p->ntiles_hi &&
        boys_internal::launch_batched(p->d_desc, p->d_tiles + p->ntiles_hi,
                                      p->ntiles - p->ntiles_hi, p->d_counter, p->maxn,
                                      launch_of(p), s) != hipSuccess)
        st = BOYS_ERR_DEVICE;
    if (hipStreamEndCapture(s, &p->graph) != hipSuccess)
        st = BOYS_ERR_DEVICE;
    if (st == BOYS_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        st = BOYS_ERR_DEVICE;
    (void)hipStreamDestroy(s);
    return st;
}

boys_status validate_batch(const boys_array *arrays, int32_t count)
{
    if (count < 0 || (count > 0 && arrays == nullptr))
        return BOYS_ERR_INVALID_ARGUMENT;
    for (int32_t a = 0; a < count; ++a) {
        const boys_array &A = arrays[a];
        const boys_status st = check_array(A.x, A.n, A.n_max, A.out, A.ld_out, A.precision);
        if (st != BOYS_OK)
            return st;
    }
    return BOYS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------
// C ABI

extern "C" {

boys_status boys_eval(const double *x, int64_t n, int32_t n_max, void *out, int64_t ld_out,
                      int32_t precision, void *stream)
{
    const boys_status st = check_array(x, n, n_max, out, ld_out, precision);
    if (st != BOYS_OK || n == 0)
        return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const PlainLaunch launch = plain_launcher(precision, n_max, false);
    if (launch == nullptr)
        return BOYS_ERR_UNSUPPORTED_NMAX;
    return launch(x, n, out, ld_out, 0, s) == hipSuccess ? BOYS_OK : BOYS_ERR_DEVICE;
}

boys_status boys_eval_rows(const double *x, int64_t n, int32_t n_max, uint64_t rows, void *out,
                           int64_t ld_out, int32_t precision, void *stream)
{
    // the selected rows are written as rows 0..k-1 of out: check the array as one of
    // k - 1 orders
    if (n_max < 0 || n_max > max_nmax(precision))
        return max_nmax(precision) < 0 ? BOYS_ERR_INVALID_ARGUMENT : BOYS_ERR_UNSUPPORTED_NMAX;
    if (rows == 0 || (n_max < 63 && (rows >> (n_max + 1)) != 0))
        return BOYS_ERR_INVALID_ARGUMENT;
    const int k = __builtin_popcountll(rows);
    const boys_status st = check_array(x, n, k - 1, out, ld_out, precision);
    if (st != BOYS_OK || n == 0)
        return st;
    const PlainLaunch launch = plain_launcher(precision, n_max, true);
    if (launch == nullptr)
        return BOYS_ERR_UNSUPPORTED_NMAX;
    return launch(x, n, out, ld_out, rows, static_cast<hipStream_t>(stream)) == hipSuccess
               ? BOYS_OK
               : BOYS_ERR_DEVICE;
}

boys_status boys_eval_split(const double *x, int64_t n, int32_t n_bar, int32_t n_max, void *out,
                            int64_t ld_out, void *stream)
{
    const boys_status st = check_array(x, n, n_max, out, ld_out, BOYS_FP64);
    if (st != BOYS_OK)
        return st;
    if (n_bar < 0 || n_bar >= n_max)
        return BOYS_ERR_UNSUPPORTED_NMAX;
    if (n == 0)
        return BOYS_OK;
    const boys_internal::SplitLaunch launch = boys_internal::split_launcher(n_max);
    if (launch == nullptr)
        return BOYS_ERR_UNSUPPORTED_NMAX;
    return launch(x, n, static_cast<double *>(out), ld_out, n_bar,
                  static_cast<hipStream_t>(stream)) == hipSuccess
               ? BOYS_OK
               : BOYS_ERR_DEVICE;
}

boys_status boys_eri_ssss(const boys_pair_list *bra, const boys_pair_list *ket, int32_t n_max,
                          double *out, int64_t ld_out, void *stream)
{
    if (bra == nullptr || ket == nullptr || bra->count < 0 || ket->count < 0)
        return BOYS_ERR_INVALID_ARGUMENT;
    if (n_max < 0 || n_max > kMaxN64)
        return BOYS_ERR_UNSUPPORTED_NMAX;
    const int64_t total = (int64_t)bra->count * ket->count;
    if (total == 0)
        return BOYS_OK;
    for (const boys_pair_list *l : {bra, ket})
        if (!l->p || !l->px || !l->py || !l->pz || !l->w || !l->start)
            return BOYS_ERR_INVALID_ARGUMENT;
    if (out == nullptr || ld_out < total || ld_out > INT64_MAX / 8 / (int64_t)(n_max + 1))
        return BOYS_ERR_INVALID_ARGUMENT;
    if ((total + 255) / 256 > INT32_MAX)
        return BOYS_ERR_INVALID_ARGUMENT;
    return boys_internal::launch_eri_ssss(*bra, *ket, n_max, out, ld_out,
                                          static_cast<hipStream_t>(stream)) == hipSuccess
               ? BOYS_OK
               : BOYS_ERR_DEVICE;
}

boys_status boys_plan_create(boys_plan **plan, const boys_array *arrays, int32_t count,
                             const boys_tuning *tuning)
{
    if (plan == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    *plan = nullptr;
    boys_status st = validate_batch(arrays, count);
    if (st != BOYS_OK)
        return st;
    const boys_tuning tn = resolve(tuning);
    if (!tuning_ok(tn))
        return BOYS_ERR_INVALID_ARGUMENT;
    boys_plan *p = new (std::nothrow) boys_plan();
    if (!p)
        return BOYS_ERR_OUT_OF_MEMORY;
    p->tuning = tn;
    p->count = count;
    (void)hipGetDevice(&p->device);
    std::vector<int2> tiles;
    st = build_schedule(p, arrays, count, tiles);
    if (st != BOYS_OK) {
        delete p;
        return st;
    }
    // schedule 0: grid_per_cu resident workgroups per compute unit, no more than one wave
    // per tile, at least one workgroup per work queue (8)
    const int64_t waves_per_wg = tn.block / 64;
    p->grid = (int)std::max<int64_t>(
        8, std::min<int64_t>((int64_t)cu_count() * tn.grid_per_cu,
                             (std::max(p->ntiles, 1) + waves_per_wg - 1) / waves_per_wg));
    const size_t desc_bytes = sizeof(Desc) * std::max<int32_t>(count, 1);
    const size_t tile_bytes = sizeof(int2) * std::max<int32_t>(p->ntiles, 1);
    if (hipMalloc(&p->d_desc, desc_bytes) != hipSuccess ||
        hipMalloc(&p->d_tiles, tile_bytes) != hipSuccess ||
        hipMalloc(&p->d_counter, boys_internal::kCounterBytes) != hipSuccess) {
        (void)hipGetLastError();
        free_plan_buffers(p);
        delete p;
        return BOYS_ERR_OUT_OF_MEMORY;
    }
    if ((count > 0 &&
         hipMemcpy(p->d_desc, p->host_desc.data(), sizeof(Desc) * count, hipMemcpyHostToDevice) !=
             hipSuccess) ||
        (p->ntiles > 0 && hipMemcpy(p->d_tiles, tiles.data(), sizeof(int2) * p->ntiles,
                                    hipMemcpyHostToDevice) != hipSuccess)) {
        free_plan_buffers(p);
        delete p;
        return BOYS_ERR_DEVICE;
    }
    st = capture_graph(p);
    if (st != BOYS_OK) {
        free_plan_buffers(p);
        delete p;
        return st;
    }
    *plan = p;
    return BOYS_OK;
}

boys_status boys_plan_update(boys_plan *p, const boys_array *arrays, int32_t count)
{
    if (p == nullptr || count != p->count)
        return BOYS_ERR_INVALID_ARGUMENT;
    boys_status st = validate_batch(arrays, count);
    if (st != BOYS_OK)
        return st;
    for (int32_t a = 0; a < count; ++a) {
        const boys_array &o = p->arrays[a], &A = arrays[a];
        if (o.n != A.n || o.n_max != A.n_max || o.precision != A.precision)
            return BOYS_ERR_INVALID_ARGUMENT;
    }
    // replays enqueued before this call may still be reading the descriptors
    if (wait_executes(p) != hipSuccess)
        return BOYS_ERR_DEVICE;
    for (int32_t a = 0; a < count; ++a) {
        p->arrays[a] = arrays[a];
        p->host_desc[a].x = arrays[a].x;
        p->host_desc[a].out = arrays[a].out;
        p->host_desc[a].ld = arrays[a].ld_out;
    }
    if (count > 0 && hipMemcpy(p->d_desc, p->host_desc.data(), sizeof(Desc) * count,
                               hipMemcpyHostToDevice) != hipSuccess)
        return BOYS_ERR_DEVICE;
    return BOYS_OK;
}

boys_status boys_plan_execute(boys_plan *p, void *stream)
{
    if (p == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    if (p->exec == nullptr)
        return BOYS_OK;  // empty batch
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipGraphLaunch(p->exec, s) != hipSuccess)
        return BOYS_ERR_DEVICE;
    hipEvent_t ev = nullptr;
    for (auto &se : p->exec_events)
        if (se.first == s)
            ev = se.second;
    if (ev == nullptr) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return BOYS_ERR_DEVICE;
        p->exec_events.emplace_back(s, ev);
    }
    return hipEventRecord(ev, s) == hipSuccess ? BOYS_OK : BOYS_ERR_DEVICE;
}

void boys_plan_destroy(boys_plan *p)
{
    if (p == nullptr)
        return;
    free_plan_buffers(p);
    delete p;
}

boys_status boys_eval_batched(const boys_array *arrays, int32_t count, void *stream)
{
    boys_plan *p = nullptr;
    boys_status st = boys_plan_create(&p, arrays, count, nullptr);
    if (st != BOYS_OK)
        return st;
    st = boys_plan_execute(p, stream);
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess && st == BOYS_OK)
        st = BOYS_ERR_DEVICE;
    boys_plan_destroy(p);
    return st;
}

boys_status boys_autotune(const boys_array *arrays, int32_t count, const boys_tuning *candidates,
                          int32_t ncand, int32_t warmup, int32_t reps, void *stream,
                          boys_tuning *best, float *times_ms)
{
    if (candidates == nullptr || ncand <= 0 || reps <= 0 || warmup < 0 || best == nullptr)
        return BOYS_ERR_INVALID_ARGUMENT;
    boys_status st = validate_batch(arrays, count);
    if (st != BOYS_OK)
        return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return BOYS_ERR_DEVICE;
    float best_t = INFINITY;
    int best_i = -1;
    for (int32_t c = 0; c < ncand; ++c) {
        float t_ms = INFINITY;
        boys_plan *p = nullptr;
        if (boys_plan_create(&p, arrays, count, &candidates[c]) == BOYS_OK) {
            bool ok = true;
            for (int32_t w = 0; w < warmup && ok; ++w)
                ok = boys_plan_execute(p, stream) == BOYS_OK;
            ok = ok && hipEventRecord(e0, s) == hipSuccess;
            for (int32_t r = 0; r < reps && ok; ++r)
                ok = boys_plan_execute(p, stream) == BOYS_OK;
            ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float el = 0.f;
            if (ok && hipEventElapsedTime(&el, e0, e1) == hipSuccess)
                t_ms = el / reps;
            boys_plan_destroy(p);
        }
        if (times_ms)
            times_ms[c] = t_ms;
        if (t_ms < best_t) {
            best_t = t_ms;
            best_i = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_i < 0)
        return BOYS_ERR_DEVICE;
    *best = resolve(&candidates[best_i]);
    return BOYS_OK;
}

int32_t boys_max_nmax(int32_t precision)
{
    return max_nmax(precision);
}

double boys_cutoff(int32_t n, int32_t precision)
{
    if (precision == BOYS_FP64 && n >= 0 && n <= kMaxN64)
        return boys_tab::kCut64[n];
    if (precision == BOYS_FP32 && n >= 0 && n <= kMaxN32)
        return boys_tab::kCut32[n];
    if (precision == BOYS_FP64_PLUS && n >= 0 && n < kMaxN64)
        return boys_tab::kCut64[n + 1];
    if (precision == BOYS_FP32X && n >= 0 && n <= kMaxN32x)
        return boys_tab::kCut32x[n];
    if (precision == BOYS_FP32_SINGLE && n >= 0 && n <= kMaxN32)
        return boys_tab::kCut32[n];
    return NAN;
}

const char *boys_status_string(boys_status status)
{
    switch (status) {
    case BOYS_OK:
        return "ok";
    case BOYS_ERR_INVALID_ARGUMENT:
        return "invalid argument";
    case BOYS_ERR_UNSUPPORTED_NMAX:
        return "unsupported n_max";
    case BOYS_ERR_OUT_OF_MEMORY:
        return "out of device memory";
    case BOYS_ERR_DEVICE:
        return "device error";
    case BOYS_ERR_TOO_LARGE:
        return "batch too large for the fixed scratch array";
    }
    return "unknown status";
}

}  // extern "C"
