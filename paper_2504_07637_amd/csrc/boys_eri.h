// boys_eri.h -- a consumer of F_m that never stores them: the contracted (ss|ss)^(m)
// auxiliary two-electron integrals (included by eri_inst.hip).  The arithmetic and its
// order are those that the declaration of boys_eri_ssss in boys.h states.
#pragma once

#include "boys_kernels.h"

namespace boys {
namespace {

struct PairList {
    const double *p, *px, *py, *pz, *w;  // primitive pairs: p, product centre P, weight
    const int32_t *start;                // contracted pair c: primitive pairs [start[c], start[c+1])
    int32_t count;
};

// the contracted (ss|ss)^(m) of bra contracted pair i and ket contracted pair j
template <int N>
__host__ __device__ __forceinline__ void eri_ssss_one(const PairList &bra, const PairList &ket,
                                                      int32_t i, int32_t j, double K,
                                                      const double2 *__restrict__ tab,
                                                      double (&acc)[N + 1])
{
#pragma unroll
    for (int m = 0; m <= N; ++m)
        acc[m] = 0.0;
    const int32_t a1 = bra.start[i + 1], b0 = ket.start[j], b1 = ket.start[j + 1];
    for (int32_t a = bra.start[i]; a < a1; ++a) {
        const double p = bra.p[a], px = bra.px[a], py = bra.py[a], pz = bra.pz[a];
        const double wa = bra.w[a];
        for (int32_t b = b0; b < b1; ++b) {
            const double q = ket.p[b];
            const double pq = p * q;
            const double spq = p + q;
            const double rho = pq / spq;
            const double dx = px - ket.px[b], dy = py - ket.py[b], dz = pz - ket.pz[b];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double T = rho * r2;
            const double s = (wa * ket.w[b]) * (K / (pq * __builtin_sqrt(spq)));
            double F[N + 1];
            eval_f64<N>(T, tab, F);
#pragma unroll
            for (int m = 0; m <= N; ++m)
                acc[m] = __builtin_fma(s, F[m], acc[m]);
        }
    }
}

}  // namespace
}  // namespace boys

namespace {

// a consumer of F_m: contracted (ss|ss)^(m) auxiliary integrals (the arithmetic and its
// order are fixed by the declaration of boys_eri_ssss).  One lane per contracted
// (bra, ket) pair; T = rho |PQ|^2 is formed in registers, F_0..F_N are consumed there,
// only the N+1 contracted sums are stored.
using boys::PairList;

__shared__ double2 s_eri_exp_tab[256];

// at most 128 VGPRs, 4 waves per SIMD: left alone the compiler takes 129-133 (3 waves);
// the bound costs 4 spilled VGPRs (20 bytes per lane) and measured 1% faster (3.837
// against 3.88 ms on the benchmark's 2048 x 2048 pairs; 5 waves spill 38 and lose 23%)
template <int N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_eri_ssss(PairList bra, PairList ket, double K,
                                                  double *__restrict__ out, int64_t ld)
{
    // the exp table in LDS (2-3% faster than through L1 here, measured); every thread
    // reaches the barrier in load_exp_table before any leaves
    load_exp_table(s_eri_exp_tab);
    const int64_t ij = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (ij >= (int64_t)bra.count * ket.count)
        return;
    const int32_t i = (int32_t)(ij / ket.count);
    const int32_t j = (int32_t)(ij - (int64_t)i * ket.count);
    double acc[N + 1];
    boys::eri_ssss_one<N>(bra, ket, i, j, K, s_eri_exp_tab, acc);
#pragma unroll
    for (int m = 0; m <= N; ++m)
        store_nt(acc[m], out + (int64_t)m * ld + ij);
}

}  // namespace
