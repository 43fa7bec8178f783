// boys_batched.h -- the batched kernels (included by batched_inst.hip, one n_max bucket and
// one launch shape per unit).
//
//   k_batched<MAXN>  persistent waves: each wave on its own takes 256-argument tiles from
//                    one of eight work counters and loads the next tile's arguments before
//                    it stores the current one's rows; a tile is one slice of one array, so
//                    (precision, n_max) is uniform per tile and the per-tile dispatch is a
//                    scalar branch to the same unrolled bodies that k_plain uses, which
//                    makes batched results equal to solo ones bit for bit.
//   k_batched_wg<MAXN, K>  one workgroup per tile of K * blockDim arguments.
//   k_batched_wave<MAXN, K>  one wave per tile of K * 64 arguments.
//   k_reset          zeroes the work counters (a kernel rather than a memset node, so the
//                    plan's graph replays correctly).
#pragma once

#include "boys_kernels.h"

namespace {

// one argument of class C (a boys_precision value) at order N, its x already loaded: the
// tile functions below load a tile's arguments before any of its stores.  Every wait for
// a vector load here is a wait for all of the wave's outstanding vector memory operations
// (loads and stores share one counter), so a load issued after stores would hold the
// wave until those stores have drained.
template <int C, int N>
__device__ __forceinline__ void body_x(const Desc &d, int64_t i, double xi, const double2 *tab)
{
    if constexpr (C == BOYS_FP64) {
        double F[N + 1];
        boys::eval_f64<N>(xi, tab, F);
        store_rows<N>(F, static_cast<double *>(d.out) + i, d.ld);
    } else if constexpr (C == BOYS_FP64_PLUS) {
        double F[N + 2];
        boys::eval_f64<N + 1>(xi, tab, F);
        store_rows<N>(F, static_cast<double *>(d.out) + i, d.ld);
    } else if constexpr (C == BOYS_FP32X) {
        double F[N + 1];
        boys::eval_f32r<N>(xi, tab, F);
        store_rows_f32<N>(F, static_cast<float *>(d.out) + i, d.ld);
    } else if constexpr (C == BOYS_FP32_SINGLE) {
        float F[N + 1];
        boys::eval_f32s<N>(xi, tab, F);
        store_rows<N>(F, static_cast<float *>(d.out) + i, d.ld);
    } else {
        float F[N + 1];
        boys::eval_f32<N>(xi, tab, F);
        store_rows<N>(F, static_cast<float *>(d.out) + i, d.ld);
    }
}

// The batched kernels inline all 4 x 37 (class, order) bodies, times the unroll factor K.
// Calling them as functions instead (once per tile) cut the compile time but cost
// occupancy and scratch (callee-saved registers, no occupancy target in the callees),
// so they stay inlined and the build compiles each (bucket, K) kernel in a unit of its
// own, in parallel.

// The exp table, staged in LDS by every batched kernel, for every class: a table read
// through L1 is a vector load, and its wait would also wait for the rows that the
// previous argument of the tile has stored (see body_x); an LDS read has a counter of its
// own.
__shared__ double2 s_exp_tab[256];

// One 256-argument tile of the persistent schedule (4 arguments per lane, their values xv
// loaded by the caller).  Before it stores anything, it loads the next tile's arguments
// into xn (nx: the next tile's first argument, nn >= 1 arguments from there on; nx null:
// no next tile), so that waiting for them later does not wait for these stores.
template <int C, int N>
__device__ __forceinline__ void tile_persistent(const Desc &d, int64_t start,
                                                const double (&xv)[4], const double *nx,
                                                int64_t nn, double (&xn)[4])
{
    const int lane = (int)(threadIdx.x & 63u);
    if (nx != nullptr) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int64_t i = (int64_t)a * 64 + lane;
            xn[a] = load_nt(nx + (i < nn ? i : nn - 1));
        }
    }
    const Desc e{d.x, d.out, d.n, d.ld, N, C};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t i = start + (int64_t)a * 64 + lane;
        if (i < d.n)
            body_x<C, N>(e, i, xv[a], s_exp_tab);
    }
}

// K guarded iterations, fully unrolled (no loop): a tile of K * blockDim arguments, all K
// arguments loaded first (Wave: a tile of K * 64 arguments owned by one wave)
template <int C, int N, int K, bool Wave>
__device__ __forceinline__ void tile_unrolled(const double *x, void *out, int64_t n, int64_t ld,
                                           int64_t start)
{
    const Desc d{x, out, n, ld, N, C};
    const double2 *tab = s_exp_tab;
    const int stride = Wave ? 64 : (int)blockDim.x;
    const int lane = Wave ? (int)(threadIdx.x & 63u) : (int)threadIdx.x;
    // unconditional loads (a lane past the end reads the array's last argument): the wait
    // for each argument then counts only the operations issued after it
    double xv[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const int64_t i = start + (int64_t)a * stride + lane;
        xv[a] = load_nt(x + (i < n ? i : n - 1));
    }
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const int64_t i = start + (int64_t)a * stride + lane;
        if (i < n)
            body_x<C, N>(d, i, xv[a], tab);
    }
}

// scalar dispatch over n (wave-uniform) to the tile functions of orders N, N-1, ..., 0;
// S: 1 one workgroup per tile, 2 one wave per tile
template <int C, int N, int S, int K>
__device__ __forceinline__ void dispatch(int n, const Desc &d, int64_t start, int64_t cnt)
{
    if (n == N)
        tile_unrolled<C, N, K, S == 2>(d.x, d.out, d.n, d.ld, start);
    else if constexpr (N > 0)
        dispatch<C, N - 1, S, K>(n, d, start, cnt);
}

// the same dispatch for the persistent schedule's tiles
template <int C, int N>
__device__ __forceinline__ void dispatch_p(int n, const Desc &d, int64_t start,
                                           const double (&xv)[4], const double *nx, int64_t nn,
                                           double (&xn)[4])
{
    if (n == N)
        tile_persistent<C, N>(d, start, xv, nx, nn, xn);
    else if constexpr (N > 0)
        dispatch_p<C, N - 1>(n, d, start, xv, nx, nn, xn);
}

template <int MAXN>
__device__ __forceinline__ void dispatch_class_p(int prec, int n, const Desc &d, int64_t start,
                                                 const double (&xv)[4], const double *nx,
                                                 int64_t nn, double (&xn)[4])
{
    if (prec == BOYS_FP64)
        dispatch_p<BOYS_FP64, cmin(MAXN, class_max<BOYS_FP64>())>(n, d, start, xv, nx, nn, xn);
    else if (prec == BOYS_FP32)
        dispatch_p<BOYS_FP32, cmin(MAXN, class_max<BOYS_FP32>())>(n, d, start, xv, nx, nn, xn);
    else if (prec == BOYS_FP32X)
        dispatch_p<BOYS_FP32X, cmin(MAXN, class_max<BOYS_FP32X>())>(n, d, start, xv, nx, nn,
                                                                    xn);
    else if (prec == BOYS_FP32_SINGLE)
        dispatch_p<BOYS_FP32_SINGLE, cmin(MAXN, class_max<BOYS_FP32_SINGLE>())>(n, d, start, xv,
                                                                                nx, nn, xn);
    else
        dispatch_p<BOYS_FP64_PLUS, cmin(MAXN, class_max<BOYS_FP64_PLUS>())>(n, d, start, xv, nx,
                                                                            nn, xn);
}

template <int MAXN, int S, int K>
__device__ __forceinline__ void dispatch_class(int prec, int n, const Desc &d, int64_t start,
                                               int64_t cnt)
{
    if (prec == BOYS_FP64)
        dispatch<BOYS_FP64, cmin(MAXN, class_max<BOYS_FP64>()), S, K>(n, d, start, cnt);
    else if (prec == BOYS_FP32)
        dispatch<BOYS_FP32, cmin(MAXN, class_max<BOYS_FP32>()), S, K>(n, d, start, cnt);
    else if (prec == BOYS_FP32X)
        dispatch<BOYS_FP32X, cmin(MAXN, class_max<BOYS_FP32X>()), S, K>(n, d, start, cnt);
    else if (prec == BOYS_FP32_SINGLE)
        dispatch<BOYS_FP32_SINGLE, cmin(MAXN, class_max<BOYS_FP32_SINGLE>()), S, K>(n, d, start,
                                                                                     cnt);
    else
        dispatch<BOYS_FP64_PLUS, cmin(MAXN, class_max<BOYS_FP64_PLUS>()), S, K>(n, d, start,
                                                                                 cnt);
}

// Persistent waves (schedule 0): a grid of resident workgroups whose waves work on their
// own, with no barrier after the exp table is staged.  The tile list is dealt to 8 queues,
// queue q holding tiles q, q + 8, q + 16, ... (an even share of every part of the list);
// workgroup b serves queue b mod 8 (the dispatcher places workgroup b on XCD b mod 8, so
// the waves of one XCD share a counter), and its waves take kPersistentChunk tiles at a
// time from that queue's counter until the queue is empty.  Every queue q < ntiles needs
// a workgroup with b mod 8 = q: the host launches at least 8.
__device__ __forceinline__ int32_t grab(uint32_t *ctr)
{
    uint32_t k = 0;
    if ((threadIdx.x & 63u) == 0)
        k = atomicAdd(ctr, (uint32_t)boys_internal::kPersistentChunk);
    // every lane is active again here, so the first active lane is lane 0
    return (int32_t)__builtin_amdgcn_readfirstlane(k);
}

template <int MAXN>
__global__ __launch_bounds__(256) void k_batched(const Desc *__restrict__ descs,
                                                 const int2 *__restrict__ tiles,
                                                 int32_t ntiles, uint32_t *__restrict__ counters)
{
    using boys_internal::kPersistentChunk;
    load_exp_table(s_exp_tab);  // every thread reaches its barrier before any leaves
    const int32_t q = (int32_t)(blockIdx.x & 7u);
    if (q >= ntiles)
        return;
    const int32_t nq = (ntiles - q + 7) / 8;  // tiles in queue q
    uint32_t *ctr = counters + boys_internal::kCounterStride * q;
    const int lane = (int)(threadIdx.x & 63u);
    int32_t k = grab(ctr);
    if (k >= nq)
        return;
    int32_t kend = k + kPersistentChunk < nq ? k + kPersistentChunk : nq;
    int2 ts = tiles[q + 8 * k];
    Desc d = descs[__builtin_amdgcn_readfirstlane(ts.x)];
    int64_t start = (int64_t)__builtin_amdgcn_readfirstlane(ts.y) * 256;
    double xv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t i = start + (int64_t)a * 64 + lane;
        xv[a] = load_nt(d.x + (i < d.n ? i : d.n - 1));
    }
    for (;;) {
        int32_t kn = k + 1;
        if (kn >= kend) {
            kn = grab(ctr);
            kend = kn + kPersistentChunk < nq ? kn + kPersistentChunk : nq;
        }
        Desc dn{};
        int64_t sn = 0;
        const double *nx = nullptr;
        int64_t nn = 0;
        if (kn < nq) {
            ts = tiles[q + 8 * kn];
            dn = descs[__builtin_amdgcn_readfirstlane(ts.x)];
            sn = (int64_t)__builtin_amdgcn_readfirstlane(ts.y) * 256;
            nx = dn.x + sn;
            nn = dn.n - sn;
        }
        double xn[4] = {0.0, 0.0, 0.0, 0.0};
        dispatch_class_p<MAXN>(__builtin_amdgcn_readfirstlane(d.prec),
                               __builtin_amdgcn_readfirstlane(d.n_max), d, start, xv, nx, nn, xn);
        if (nx == nullptr)
            break;
        d = dn;
        start = sn;
        xv[0] = xn[0];
        xv[1] = xn[1];
        xv[2] = xn[2];
        xv[3] = xn[3];
        k = kn;
    }
}

// one workgroup per tile: the hardware dispatcher hands out the tiles in table order, no
// work counter
template <int MAXN, int K>
__global__ __launch_bounds__(256) void k_batched_wg(const Desc *__restrict__ descs,
                                                    const int2 *__restrict__ tiles,
                                                    int32_t tile_args)
{
    const int2 ts = tiles[blockIdx.x];
    const int32_t a = __builtin_amdgcn_readfirstlane(ts.x);
    const Desc d = descs[a];
    const int64_t start = (int64_t)__builtin_amdgcn_readfirstlane(ts.y) * tile_args;
    const int prec = __builtin_amdgcn_readfirstlane(d.prec);
    load_exp_table(s_exp_tab);
    dispatch_class<MAXN, 1, K>(prec, __builtin_amdgcn_readfirstlane(d.n_max), d, start, 0);
}

// one wave per tile: each wave of a workgroup takes its own tile of K * 64 arguments, so
// one workgroup can serve several short arrays (a tile never spans two arrays)
template <int MAXN, int K>
__global__ __launch_bounds__(256) void k_batched_wave(const Desc *__restrict__ descs,
                                                      const int2 *__restrict__ tiles,
                                                      int32_t ntiles, int32_t tile_args)
{
    // every thread reaches the barrier in load_exp_table before any leaves
    load_exp_table(s_exp_tab);
    const int32_t w = __builtin_amdgcn_readfirstlane(
        (int32_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    if (w >= ntiles)
        return;
    const int2 ts = tiles[w];
    const int32_t a = __builtin_amdgcn_readfirstlane(ts.x);
    const Desc d = descs[a];
    const int64_t start = (int64_t)__builtin_amdgcn_readfirstlane(ts.y) * tile_args;
    dispatch_class<MAXN, 2, K>(__builtin_amdgcn_readfirstlane(d.prec),
                               __builtin_amdgcn_readfirstlane(d.n_max), d, start, 0);
}

// one wave: zero the 8 work counters of k_batched
__global__ void k_reset(uint32_t *counters)
{
    if (threadIdx.x < 8)
        counters[boys_internal::kCounterStride * threadIdx.x] = 0u;
}

}  // namespace
