// boys_batched.h -- the batched kernels (included by batched_inst.hip, one n_max bucket and
// one launch shape per unit).
//
//   k_batched<MAXN>  persistent workgroups pull tiles from a device counter; a tile is
//                    one slice of one array, so (precision, n_max) is uniform per tile and
//                    the per-tile dispatch is a scalar branch to the same unrolled bodies
//                    that k_plain uses, which makes batched results equal to solo ones
//                    bit for bit.
//   k_batched_wg<MAXN, K>  one workgroup per tile of K * blockDim arguments.
//   k_batched_wave<MAXN, K>  one wave per tile of K * 64 arguments.
//   k_reset          zeroes the tile counter (a kernel rather than a memset node, so the
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

// arguments [start, start + cnt) of one array, blockDim-strided; each thread loads its
// next argument before it stores the current one's rows
template <int C, int N>
__device__ __forceinline__ void tile_strided(const double *x, void *out, int64_t ld, int64_t start,
                                          int64_t cnt)
{
    const Desc d{x, out, start + cnt, ld, N, C};
    const double2 *tab = s_exp_tab;
    int64_t j = threadIdx.x;
    double xn = j < cnt ? load_nt(x + start + j) : 0.0;
    for (; j < cnt; j += blockDim.x) {
        const double xc = xn;
        if (j + blockDim.x < cnt)
            xn = load_nt(x + start + j + blockDim.x);
        body_x<C, N>(d, start + j, xc, tab);
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
// S: 0 the strided form (persistent schedule), 1 one workgroup per tile, 2 one wave per tile
template <int C, int N, int S, int K>
__device__ __forceinline__ void dispatch(int n, const Desc &d, int64_t start, int64_t cnt)
{
    if (n == N) {
        if constexpr (S == 0)
            tile_strided<C, N>(d.x, d.out, d.ld, start, cnt);
        else
            tile_unrolled<C, N, K, S == 2>(d.x, d.out, d.n, d.ld, start);
    } else if constexpr (N > 0) {
        dispatch<C, N - 1, S, K>(n, d, start, cnt);
    }
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

template <int MAXN>
__global__ __launch_bounds__(256) void k_batched(const Desc *__restrict__ descs,
                                                 const int2 *__restrict__ tiles,
                                                 int32_t ntiles, int32_t tile_args,
                                                 uint32_t *__restrict__ counter)
{
    __shared__ int32_t s_tile;
    load_exp_table(s_exp_tab);
    for (;;) {
        if (threadIdx.x == 0)
            s_tile = (int32_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int32_t t = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t >= ntiles)
            break;
        const int2 ts = tiles[t];
        const int32_t a = __builtin_amdgcn_readfirstlane(ts.x);
        const Desc d = descs[a];
        const int64_t start = (int64_t)__builtin_amdgcn_readfirstlane(ts.y) * tile_args;
        const int64_t rem = d.n - start;
        const int64_t cnt = rem < tile_args ? rem : tile_args;
        dispatch_class<MAXN, 0, 0>(__builtin_amdgcn_readfirstlane(d.prec),
                                __builtin_amdgcn_readfirstlane(d.n_max), d, start, cnt);
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

__global__ void k_reset(uint32_t *counter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *counter = 0u;
}

}  // namespace
