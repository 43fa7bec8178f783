// boys_internal.h -- library-internal interface between the kernel instantiation units
// (plain_inst.hip, batched_inst.hip, split_inst.hip, eri_inst.hip), the host side (boys_lib.hip) and the serving
// executor (boys_serve.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "boys.h"

namespace boys_internal {

// one argument array of a batched launch (device-side descriptor)
struct Desc {
    const double *x;
    void *out;
    int64_t n;
    int64_t ld;
    int32_t n_max;
    int32_t prec;
};

// schedule 0 (persistent waves): 8 work counters, one per 128-byte line, and the tiles a
// wave takes from its counter at a time
constexpr int kCounterStride = 32;                     // uint32 elements between counters
constexpr int kCounterBytes = 8 * kCounterStride * 4;  // 1 KiB
constexpr int kPersistentChunk = 4;

// how a batch is launched
struct Launch {
    int schedule;  // 0: persistent waves + work counters; 1: one workgroup per tile;
                   // 2: one wave per tile
    int tile;      // arguments per tile (schedule 1: block x 1, 2 or 4; schedules 0 and 2: 256)
    int block;     // threads per workgroup (64, 128, 256)
    int grid;      // schedule 0: number of persistent workgroups (at least 8)
};

// Enqueue a batch on stream s: schedule 0 = [zero the counters, persistent kernel],
// schedule 1 = [one workgroup per tile], schedule 2 = [one wave per tile].  tiles holds
// (array index, slice index) pairs; slice k of array a covers arguments [k * tile,
// min((k+1) * tile, n_a)).  d_counter: kCounterBytes of device memory (schedule 0 only).
// maxn is the largest n_max in the batch.
hipError_t launch_batched(const Desc *d_desc, const int2 *d_tiles, int32_t ntiles,
                          uint32_t *d_counter, int maxn, const Launch &L, hipStream_t s);

int cu_count();

// the plain launch of precision class C at order n (nullptr outside 0..the class's largest
// order); with select_rows, the form that stores only the rows whose bit is set in `rows`
// (boys_eval_rows), otherwise `rows` is ignored; defined per class in plain_inst.hip
using PlainLaunch = hipError_t (*)(const double *x, int64_t n, void *out, int64_t ld,
                                   uint64_t rows, hipStream_t s);
template <int C>
PlainLaunch plain_launcher(int n, bool select_rows);

// the two-approximation launch at order n (1..the binary64 maximum; nullptr otherwise);
// defined in split_inst.hip
using SplitLaunch = hipError_t (*)(const double *x, int64_t n, double *out, int64_t ld,
                                   int nbar, hipStream_t s);
SplitLaunch split_launcher(int n);

// the consumer kernels (contracted (ss|ss)^(m) integrals) at order n_max; defined in
// eri_inst.hip.  Arguments are checked by the caller.
hipError_t launch_eri_ssss(const boys_pair_list &bra, const boys_pair_list &ket, int n_max,
                           double *out, int64_t ld, hipStream_t s);

// the batched kernel of n_max bucket B with schedule S (0: persistent waves, [zero the
// counters, kernel]; 1: one workgroup per tile of K * L.block arguments, K = 1, 2, 4; 2: one wave
// per tile of K * 64 arguments, K = 4); defined per (B, S, K) in batched_inst.hip
template <int B, int S, int K>
hipError_t launch_bucket(const Desc *d_desc, const int2 *d_tiles, int32_t ntiles,
                         uint32_t *d_counter, const Launch &L, hipStream_t s);

}  // namespace boys_internal
