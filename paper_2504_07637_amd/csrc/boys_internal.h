// boys_internal.h -- library-internal interface between the kernels (boys_lib.hip) and
// the serving executor (boys_serve.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Enqueue [zero the counter, persistent batched kernel] on stream s.  tiles holds
// (array index, slice index) pairs; slice k of array a covers arguments
// [k * tile_args, min((k+1) * tile_args, n_a)).  maxn is the largest n_max in the batch.
hipError_t launch_batched(const Desc *d_desc, const int2 *d_tiles, int32_t ntiles,
                          int32_t tile_args, uint32_t *d_counter, int maxn, int grid,
                          int block, hipStream_t s);

int cu_count();

}  // namespace boys_internal
