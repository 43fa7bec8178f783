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

// one argument of class C (a boys_precision value) at order N
template <int C, int N>
__device__ __forceinline__ void body(const Desc &d, int64_t i, const double2 *tab)
{
    if constexpr (C == BOYS_FP64)
        body_f64<N>(d.x, static_cast<double *>(d.out), d.ld, i, tab);
    else if constexpr (C == BOYS_FP64_PLUS)
        body_f64plus<N>(d.x, static_cast<double *>(d.out), d.ld, i, tab);
    else if constexpr (C == BOYS_FP32X)
        body_f32x<N>(d.x, static_cast<float *>(d.out), d.ld, i, tab);
    else if constexpr (C == BOYS_FP32_SINGLE)
        body_f32s<N>(d.x, static_cast<float *>(d.out), d.ld, i, tab);
    else
        body_f32<N>(d.x, static_cast<float *>(d.out), d.ld, i, tab);
}

// The batched kernels inline all 4 x 37 (class, order) bodies, times the unroll factor K.
// Calling them as functions instead (once per tile) cut the compile time but cost
// occupancy and scratch (callee-saved registers, no occupancy target in the callees),
// so they stay inlined and the build compiles each (bucket, K) kernel in a unit of its
// own, in parallel.

// the exp table as the bodies of class C read it: binary64 classes from global memory
// through L1, the mixed class from the LDS copy that the kernel stages in s_exp_tab
__shared__ double2 s_exp_tab[256];

template <int C>
__device__ __forceinline__ const double2 *exp_tab()
{
    if constexpr (C == BOYS_FP32)
        return s_exp_tab;
    else
        return reinterpret_cast<const double2 *>(boys_tab::kExp2Tab);
}

// arguments [start, start + cnt) of one array, blockDim-strided
template <int C, int N>
__device__ __forceinline__ void tile_strided(const double *x, void *out, int64_t ld, int64_t start,
                                          int64_t cnt)
{
    const Desc d{x, out, start + cnt, ld, N, C};
    const double2 *tab = exp_tab<C>();
    for (int64_t j = threadIdx.x; j < cnt; j += blockDim.x)
        body<C, N>(d, start + j, tab);
}

// K guarded iterations, fully unrolled (no loop): a tile of K * blockDim arguments
// (Wave: a tile of K * 64 arguments owned by one wave, the exp table read through L1 for
// every class, so that the waves of a workgroup need no barrier)
template <int C, int N, int K, bool Wave>
__device__ __forceinline__ void tile_unrolled(const double *x, void *out, int64_t n, int64_t ld,
                                           int64_t start)
{
    const Desc d{x, out, n, ld, N, C};
    const double2 *tab =
        Wave ? reinterpret_cast<const double2 *>(boys_tab::kExp2Tab) : exp_tab<C>();
    const int stride = Wave ? 64 : (int)blockDim.x;
    const int lane = Wave ? (int)(threadIdx.x & 63u) : (int)threadIdx.x;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const int64_t i = start + (int64_t)a * stride + lane;
        if (i < n)
            body<C, N>(d, i, tab);
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

// one workgroup per tile: the hardware dispatcher hands out the tiles in table order
// (longest first), no work counter; binary64 bodies read the exp table through L1,
// binary32 bodies stage it in LDS, as the plain kernels do
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
    if (prec == BOYS_FP32)
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
