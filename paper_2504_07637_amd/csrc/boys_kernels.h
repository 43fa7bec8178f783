// boys_kernels.h -- the device code of libboys.so: per-argument bodies and kernels.
//
// Included by the instantiation units (plain_inst.hip: the plain kernels of one precision
// class; batched_inst.hip: the batched kernels of one n_max bucket and one launch shape;
// split_inst.hip and eri_inst.hip), which the build compiles in parallel.  Everything here has internal linkage, so each
// unit holds only the kernels it instantiates.
//
// Kernels (gfx950, wave64):
//   k_plain<C, N, Sel>  one lane per argument, one argument per lane (a full grid: for the
//                    (n_max+1)-row output this launch shape keeps the HBM write streams
//                    densest; Sel: only selected rows are stored, boys_eval_rows);
//                    x is read and the output rows are written with coalesced
//                    non-temporal accesses (for a wave, 512 contiguous bytes per binary64
//                    row).  The binary64-output classes read the 4 KiB exp table through
//                    the L1 cache with 128-thread workgroups; the binary32-output classes
//                    stage it in LDS with 512-thread workgroups (the faster shape for each,
//                    by measurement).  Outputs of 25+ binary64 rows take an XCD-contiguous
//                    block order (xcd_contiguous below).
//   k_batched<MAXN>  persistent workgroups pull tiles from a device counter; a tile is
//                    one slice of one array, so (precision, n_max) is uniform per tile and
//                    the per-tile dispatch is a scalar branch to the same unrolled bodies
//                    that k_plain uses, which makes batched results equal to solo ones
//                    bit for bit.
//   k_batched_wg<MAXN, K>  one workgroup per tile of K * blockDim arguments.
//   k_batched_wave<MAXN, K>  one wave per tile of K * 64 arguments.
//   k_split<N>       the two-approximation option (binary64, lower order a launch argument),
//                    shaped as k_plain.
//   k_eri_ssss<N>    a consumer: contracted (ss|ss)^(m) integrals, F_m never leave registers.
//   k_reset          zeroes the tile counter (a kernel rather than a memset node, so the
//                    plan's graph replays correctly).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "boys.h"
#include "boys_device.h"
#include "boys_internal.h"

namespace {

using boys_tab::kMaxN32;
using boys_tab::kMaxN32x;
using boys_tab::kMaxN64;

constexpr int kMaxN = kMaxN64 > kMaxN32 ? (kMaxN64 > kMaxN32x ? kMaxN64 : kMaxN32x)
                                        : (kMaxN32 > kMaxN32x ? kMaxN32 : kMaxN32x);

// n_max buckets of the batched kernels: a batch runs the smallest MAXN >= its largest n_max
constexpr int kBuckets[] = {4, 8, 16, 24, kMaxN};
constexpr int kNumBuckets = 5;

using boys_internal::Desc;

// Every array the kernels read or write lives in global memory.  A pointer that reaches a
// kernel through a descriptor in memory carries no address space, and the compiler would
// access it with flat instructions (which also count against the LDS/scalar wait
// counter); these access through a global-address-space pointer instead.
template <typename T>
__device__ __forceinline__ T load_nt(const T *p)
{
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T *)p);
}

template <typename T>
__device__ __forceinline__ void store_nt(T v, T *p)
{
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T *)p);
}

// F_0..F_N of one argument to rows 0..N of the output (row stride ld), non-temporal.  The
// address walks by ld: written as out + m*ld + i, the compiler forms each row address with
// two 64-bit vector multiply-adds, which costs the VALU-bound classes measurably.
template <int N, typename T>
__device__ __forceinline__ void store_rows(const T *F, T *p, int64_t ld)
{
#pragma unroll
    for (int m = 0; m <= N; ++m) {
        store_nt(F[m], p);
        p += ld;
    }
}

// the same, each binary64 value rounded once to binary32
template <int N>
__device__ __forceinline__ void store_rows_f32(const double *F, float *p, int64_t ld)
{
#pragma unroll
    for (int m = 0; m <= N; ++m) {
        store_nt((float)F[m], p);
        p += ld;
    }
}

// Row selection (boys_eval_rows): only the orders whose bit is set in `rows` (a kernel
// argument, so every test is a scalar branch) are stored, the k-th selected one to row k.
// Every F_m is still computed: the recursion and the upward chain pass through all orders.
template <int N, typename T>
__device__ __forceinline__ void store_rows_sel(const T *F, T *p, int64_t ld, uint64_t rows)
{
#pragma unroll
    for (int m = 0; m <= N; ++m) {
        if ((rows >> m) & 1u) {
            store_nt(F[m], p);
            p += ld;
        }
    }
}

template <int N>
__device__ __forceinline__ void store_rows_sel_f32(const double *F, float *p, int64_t ld,
                                                   uint64_t rows)
{
#pragma unroll
    for (int m = 0; m <= N; ++m) {
        if ((rows >> m) & 1u) {
            store_nt((float)F[m], p);
            p += ld;
        }
    }
}

// every row (Sel = false) or the selected ones
template <bool Sel, int N, typename T>
__device__ __forceinline__ void store_out(const T *F, T *p, int64_t ld, uint64_t rows)
{
    if constexpr (Sel)
        store_rows_sel<N>(F, p, ld, rows);
    else
        store_rows<N>(F, p, ld);
}

template <bool Sel, int N>
__device__ __forceinline__ void store_out_f32(const double *F, float *p, int64_t ld, uint64_t rows)
{
    if constexpr (Sel)
        store_rows_sel_f32<N>(F, p, ld, rows);
    else
        store_rows_f32<N>(F, p, ld);
}

__device__ __forceinline__ void load_exp_table(double2 *tab)
{
    for (int t = threadIdx.x; t < 256; t += blockDim.x)
        tab[t] = make_double2(boys_tab::kExp2Tab[2 * t], boys_tab::kExp2Tab[2 * t + 1]);
    __syncthreads();
}

template <int N, bool Sel = false>
__device__ __forceinline__ void body_f64(const double *__restrict__ x, double *__restrict__ out,
                                         int64_t ld, int64_t i, const double2 *tab,
                                         uint64_t rows = 0)
{
    double F[N + 1];
    boys::eval_f64<N>(load_nt(x + i), tab, F);
    store_out<Sel, N>(F, out + i, ld, rows);
}

// binary64, F_0..F_N from the order N+1 approximant and one more recursion step
template <int N, bool Sel = false>
__device__ __forceinline__ void body_f64plus(const double *__restrict__ x,
                                             double *__restrict__ out, int64_t ld, int64_t i,
                                             const double2 *tab, uint64_t rows = 0)
{
    double F[N + 2];
    boys::eval_f64<N + 1>(load_nt(x + i), tab, F);
    store_out<Sel, N>(F, out + i, ld, rows);
}

// binary32 output from binary64 arithmetic with the ~28-bit approximants; each value is
// rounded once to binary32 at the store
template <int N, bool Sel = false>
__device__ __forceinline__ void body_f32x(const double *__restrict__ x, float *__restrict__ out,
                                          int64_t ld, int64_t i, const double2 *tab,
                                          uint64_t rows = 0)
{
    double F[N + 1];
    boys::eval_f32r<N>(load_nt(x + i), tab, F);
    store_out_f32<Sel, N>(F, out + i, ld, rows);
}

// one argument of class C (a boys_precision value) at order N
template <int C, int N>
__device__ __forceinline__ void body(const Desc &d, int64_t i, const double2 *tab);

template <int N, bool Sel = false>
__device__ __forceinline__ void body_f32(const double *__restrict__ x, float *__restrict__ out,
                                         int64_t ld, int64_t i, const double2 *tab,
                                         uint64_t rows = 0)
{
    float F[N + 1];
    boys::eval_f32<N>(load_nt(x + i), tab, F);
    store_out<Sel, N>(F, out + i, ld, rows);
}

// all binary32 below the cut-off (Table 1's binary32 arithmetic)
template <int N, bool Sel = false>
__device__ __forceinline__ void body_f32s(const double *__restrict__ x, float *__restrict__ out,
                                          int64_t ld, int64_t i, const double2 *tab,
                                          uint64_t rows = 0)
{
    float F[N + 1];
    boys::eval_f32s<N>(load_nt(x + i), tab, F);
    store_out<Sel, N>(F, out + i, ld, rows);
}

constexpr int cmin(int a, int b)
{
    return a < b ? a : b;
}

// block size of the plain kernel per class
template <int C>
constexpr int plain_block()
{
    return C == BOYS_FP32 || C == BOYS_FP32X || C == BOYS_FP32_SINGLE ? 512 : 128;
}

// largest order of a class
template <int C>
constexpr int class_max()
{
    return C == BOYS_FP32 || C == BOYS_FP32_SINGLE ? kMaxN32
           : C == BOYS_FP64                       ? kMaxN64
           : C == BOYS_FP32X                      ? kMaxN32x
                                                  : kMaxN64 - 1;
}

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

// Block order across the 8 XCDs: the dispatcher hands workgroup b to XCD b mod 8.  For
// binary64 outputs of 25 rows or more, remapping so that each XCD takes a contiguous
// eighth of the grid measured 1% (n_max 24) to 5% (n_max 36) faster; for fewer rows and
// for binary32 outputs it was neutral or slower, so those keep the hardware order.
template <int C, int N>
constexpr bool xcd_contiguous()
{
    return (C == BOYS_FP64 || C == BOYS_FP64_PLUS) && N >= 24;
}

template <bool Remap>
__device__ __forceinline__ unsigned block_index()
{
    unsigned b = blockIdx.x;
    if constexpr (Remap) {
        const unsigned per = gridDim.x / 8u;
        if (b < per * 8u)
            b = (b % 8u) * per + b / 8u;
    }
    return b;
}

// Where the plain kernel reads the exp table: the binary64 classes through L1; binary32
// outputs computed in binary64 from a copy staged in LDS; the classes with binary32
// arithmetic from LDS at orders 11..20 and through L1 otherwise (measured at 2^26
// arguments, 512-thread workgroups: LDS 5-7% faster at n_max 12..18, L1 3-8% faster at
// n_max <= 8 and 3-7% at n_max >= 22, the two even at 10 and 20).
template <int C, int N>
constexpr bool plain_lds_table()
{
    if constexpr (C == BOYS_FP32X)
        return true;
    else if constexpr (C == BOYS_FP32 || C == BOYS_FP32_SINGLE)
        return N >= 11 && N <= 20;
    else
        return false;
}

// Sel: store only the rows selected by `rows` (boys_eval_rows); otherwise `rows` is unused
template <int C, int N, bool Sel>
__global__ __launch_bounds__(plain_block<C>()) void k_plain(const double *__restrict__ x, int64_t n,
                                                            void *__restrict__ out, int64_t ld,
                                                            uint64_t rows)
{
    constexpr int BS = plain_block<C>();
    const double2 *tab;
    if constexpr (!plain_lds_table<C, N>()) {
        tab = reinterpret_cast<const double2 *>(boys_tab::kExp2Tab);
    } else {
        __shared__ double2 lds_tab[256];
        load_exp_table(lds_tab);
        tab = lds_tab;
    }
    // one argument per lane and no loop: a grid-stride loop, even one that runs once,
    // costs about 10% here (measured); the host splits arrays too long for one grid
    const int64_t i = (int64_t)block_index<xcd_contiguous<C, N>()>() * BS + threadIdx.x;
    if (i < n) {
        if constexpr (C == BOYS_FP64)
            body_f64<N, Sel>(x, static_cast<double *>(out), ld, i, tab, rows);
        else if constexpr (C == BOYS_FP64_PLUS)
            body_f64plus<N, Sel>(x, static_cast<double *>(out), ld, i, tab, rows);
        else if constexpr (C == BOYS_FP32X)
            body_f32x<N, Sel>(x, static_cast<float *>(out), ld, i, tab, rows);
        else if constexpr (C == BOYS_FP32_SINGLE)
            body_f32s<N, Sel>(x, static_cast<float *>(out), ld, i, tab, rows);
        else
            body_f32<N, Sel>(x, static_cast<float *>(out), ld, i, tab, rows);
    }
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

// the two-approximation option (binary64): one lane per argument, as k_plain<BOYS_FP64, N>;
// nbar is wave-uniform (a kernel argument)
template <int N>
__global__ __launch_bounds__(128) void k_split(const double *__restrict__ x, int64_t n,
                                               double *__restrict__ out, int64_t ld, int nbar)
{
    const int64_t i = (int64_t)block_index<xcd_contiguous<BOYS_FP64, N>()>() * 128 + threadIdx.x;
    if (i < n) {
        double F[N + 1];
        boys::eval_split<N>(load_nt(x + i), nbar,
                            reinterpret_cast<const double2 *>(boys_tab::kExp2Tab), F);
        // indexed row addresses here, not store_rows: with the pointer walk the compiler
        // turns the branches on nbar into selects (static VALU count 812 against 755)
#pragma unroll
        for (int m = 0; m <= N; ++m)
            store_nt(F[m], out + (int64_t)m * ld + i);
    }
}

// a consumer of F_m: contracted (ss|ss)^(m) auxiliary integrals (the arithmetic and its
// order are fixed by the declaration of boys_eri_ssss).  One lane per contracted
// (bra, ket) pair; T = rho |PQ|^2 is formed in registers, F_0..F_N are consumed there,
// only the N+1 contracted sums are stored.
using boys::PairList;

template <int N>
__global__ __launch_bounds__(256) void k_eri_ssss(PairList bra, PairList ket, double K,
                                                  double *__restrict__ out, int64_t ld)
{
    // the exp table in LDS (2-3% faster than through L1 here, measured); every thread
    // reaches the barrier in load_exp_table before any leaves
    load_exp_table(s_exp_tab);
    const int64_t ij = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (ij >= (int64_t)bra.count * ket.count)
        return;
    const int32_t i = (int32_t)(ij / ket.count);
    const int32_t j = (int32_t)(ij - (int64_t)i * ket.count);
    double acc[N + 1];
    boys::eri_ssss_one<N>(bra, ket, i, j, K, s_exp_tab, acc);
#pragma unroll
    for (int m = 0; m <= N; ++m)
        store_nt(acc[m], out + (int64_t)m * ld + ij);
}

__global__ void k_reset(uint32_t *counter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *counter = 0u;
}

}  // namespace
