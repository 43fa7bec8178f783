// batched_inst.hip -- one batched kernel and its launcher: n_max bucket B (the largest
// order it dispatches is kBuckets[B]), schedule S (0: persistent waves with work
// counters; 1: one workgroup per tile of K * blockDim arguments, K = 1, 2, 4; 2: one wave
// per tile of K * 64 arguments, K = 4).
// Compiled once per (B, S, K) with -DBOYS_BUCKET=<B> -DBOYS_SCHED=<S> -DBOYS_K=<K>.
#include <algorithm>

#include "boys_batched.h"

#if !defined(BOYS_BUCKET) || !defined(BOYS_SCHED) || !defined(BOYS_K)
#error "compile with -DBOYS_BUCKET=<bucket> -DBOYS_SCHED=<0, 1, 2> -DBOYS_K=<tile factor>"
#endif

template <int B, int S, int K>
hipError_t boys_internal::launch_bucket(const Desc *d_desc, const int2 *d_tiles, int32_t ntiles,
                                        uint32_t *d_counter, const Launch &L, hipStream_t s)
{
    static_assert(B >= 0 && B < kNumBuckets, "bucket out of range");
    constexpr int kMax = kBuckets[B];
    if constexpr (S == 2) {
        static_assert(K == 4, "unsupported tile factor");
        const int waves = L.block / 64;
        if (ntiles > 0)
            hipLaunchKernelGGL((k_batched_wave<kMax, K>), dim3((ntiles + waves - 1) / waves),
                               dim3(L.block), 0, s, d_desc, d_tiles, ntiles, L.tile);
    } else if constexpr (S == 0) {
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, d_counter);
        // at least 8 workgroups: one per work queue
        if (ntiles > 0)
            hipLaunchKernelGGL((k_batched<kMax>), dim3(std::max(8, L.grid)), dim3(L.block), 0, s,
                               d_desc, d_tiles, ntiles, d_counter);
    } else {
        static_assert(K == 1 || K == 2 || K == 4, "unsupported tile factor");
        if (ntiles > 0)
            hipLaunchKernelGGL((k_batched_wg<kMax, K>), dim3(ntiles), dim3(L.block), 0, s,
                               d_desc, d_tiles, L.tile);
    }
    return hipGetLastError();
}

template hipError_t boys_internal::launch_bucket<BOYS_BUCKET, BOYS_SCHED, BOYS_K>(
    const Desc *, const int2 *, int32_t, uint32_t *, const Launch &, hipStream_t);
