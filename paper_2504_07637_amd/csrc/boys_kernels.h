// boys_kernels.h -- the device code of libboys.so shared by every kernel (per-argument
// bodies, loads and stores), the plain kernels and the two-approximation kernels.
//
// Included by the instantiation units (plain_inst.hip: the plain kernels of one precision
// class; split_inst.hip), and through boys_batched.h (the batched kernels, batched_inst.hip)
// and boys_eri.h (the consumer, eri_inst.hip).  Everything here has internal linkage, so
// each unit holds only the kernels it instantiates; the build compiles the units in
// parallel.
//
// Kernels here (gfx950, wave64):
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
//   k_split<N>       the two-approximation option (binary64, lower order a launch argument),
//                    shaped as k_plain.
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

}  // namespace
