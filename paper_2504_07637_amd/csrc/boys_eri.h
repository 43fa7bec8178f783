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

}  // namespace
}  // namespace boys

namespace {

// A consumer of F_m: contracted (ss|ss)^(m) auxiliary integrals.  One lane per contracted
// (bra, ket) pair; each lane walks its primitive quartets in the order the contract fixes
// (bra primitives outer, ket primitives inner) and keeps its N+1 sums in registers; only
// the sums are stored.
//
// The Boys evaluation differs in cost by side of the cut-off: the rational branch (exp,
// the factored Q~, the power, the downward recursion) costs several times the long-range
// branch, and in lockstep a wave runs it whenever one of its 64 lanes needs it (on the
// benchmark's lists in 2 of 3 wave-steps, for 15% of the quartets).  So a wave works
// in windows: it forms the arguments T and prefactors s of up to kEriWindow quartet steps
// of every lane, queues in LDS the arguments below the cut-off (at most 64 per window; a
// step whose arguments would not fit opens the next window), evaluates the queue in one
// pass with one argument per lane, and then replays the window's steps in order: a lane
// whose quartet lies below the cut-off takes F_0..F_N from the queue's results, the others
// evaluate the long-range branch in lockstep.  Each sum still adds the same terms in the
// same order, and each F_m comes from the same operations (eval_f64 with its side named),
// so the results are those of the plain per-lane loop bit for bit.
// windows of 4 steps: 2 measured 14% slower at n_max = 16, 6 or 8 no faster (more registers)
constexpr int kEriWindow = 4;
constexpr int kEriBlock = 256;  // threads per workgroup: 4 waves, each with its LDS rows

// At the orders where it buys a wave per SIMD, the values go straight from the evaluation
// into the sums and into the LDS rows (eval_f64_each), with no array of N+1 values, and the
// exp table is read through L1: 20-24 run 3 waves per SIMD instead of 2 (146-162 VGPRs
// instead of 172-196; 7% faster at 20 and 24), 34-36 run 2 instead of 1 (37% faster at
// 36).  Elsewhere the occupancy is the same either way and the array form with the table in
// LDS is ahead (2% at 16, 4% at 28 and 30).
constexpr bool eri_streams(int n)
{
    return (n >= 20 && n <= 24) || n >= 34;
}

using boys::PairList;

__shared__ double2 s_eri_exp_tab[256];

// the waves of a workgroup each use their own LDS rows; the order of a wave's LDS writes
// and reads needs only the compiler's (LDS operations of one wave complete in order)
__device__ __forceinline__ void wave_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N>
__global__ __launch_bounds__(kEriBlock) void k_eri_ssss(PairList bra, PairList ket, double K,
                                                        double *__restrict__ out, int64_t ld)
{
    // per wave: the window's below-cut-off arguments and their F_0..F_N
    __shared__ double s_arg[kEriBlock / 64][64];
    __shared__ double s_val[kEriBlock / 64][N + 1][64];
    constexpr bool stream = eri_streams(N);
    // otherwise the exp table in LDS (2-3% faster than through L1 there, measured); every
    // thread reaches the barrier in load_exp_table before any leaves
    const double2 *tab = reinterpret_cast<const double2 *>(boys_tab::kExp2Tab);
    if constexpr (!stream) {
        load_exp_table(s_eri_exp_tab);
        tab = s_eri_exp_tab;
    }
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63u);
    double *arg = s_arg[wave];
    double(*val)[64] = s_val[wave];
    const int64_t ij = (int64_t)blockIdx.x * kEriBlock + threadIdx.x;
    const bool live = ij < (int64_t)bra.count * ket.count;
    // this lane's next quartet (a, b); a == a1 once it has none left
    int32_t a = 0, a1 = 0, b0 = 0, b1 = 0;
    if (live) {
        const int32_t i = (int32_t)(ij / ket.count);
        const int32_t j = (int32_t)(ij - (int64_t)i * ket.count);
        a = bra.start[i];
        a1 = bra.start[i + 1];
        b0 = ket.start[j];
        b1 = ket.start[j + 1];
        if (b0 >= b1)
            a = a1;  // a ket pair without primitives: no quartets
    }
    int32_t b = b0;
    double acc[N + 1];
#pragma unroll
    for (int m = 0; m <= N; ++m)
        acc[m] = 0.0;
    constexpr double z = boys_tab::F64Set<N>::z;
    // a step formed but not taken by the previous window (it would have overfilled the
    // queue): it is the next window's first step
    bool carry = false;  // the same in every lane
    bool c_has = false;
    double c_T = 0.0, c_s = 0.0;
    // every lane of the wave takes part in every window (the ballots), so the loop ends
    // for the whole wave at once
    while (carry || __builtin_amdgcn_ballot_w64(a < a1) != 0) {
        double T[kEriWindow], S[kEriWindow];
        bool has[kEriWindow], below[kEriWindow];
        int slot[kEriWindow];
        int queued = 0, steps = 0;
        bool full = false;
#pragma unroll
        for (int t = 0; t < kEriWindow; ++t) {
            has[t] = below[t] = false;
            slot[t] = 0;
            T[t] = S[t] = 0.0;
            if (full)
                continue;
            bool h = false;
            double x = 0.0, s = 0.0;
            if (t == 0 && carry) {
                h = c_has;
                x = c_T;
                s = c_s;
            } else if (a < a1) {
                h = true;
                const double p = bra.p[a], px = bra.px[a], py = bra.py[a], pz = bra.pz[a];
                const double wa = bra.w[a];
                const double q = ket.p[b];
                const double pq = p * q;
                const double spq = p + q;
                const double rho = pq / spq;
                const double dx = px - ket.px[b], dy = py - ket.py[b], dz = pz - ket.pz[b];
                const double r2 = dx * dx + dy * dy + dz * dz;
                x = rho * r2;
                s = (wa * ket.w[b]) * (K / (pq * __builtin_sqrt(spq)));
                if (++b == b1) {
                    b = b0;
                    ++a;
                }
            }
            // the cut-off test of eval_f64 (NaN and x < 0 count as below)
            const bool bl = h && !(x > z);
            const uint64_t mask = __builtin_amdgcn_ballot_w64(bl);
            const int cnt = __builtin_popcountll(mask);
            if (queued + cnt > 64) {  // the same in every lane: this step opens the next window
                full = true;
                c_has = h;
                c_T = x;
                c_s = s;
                continue;
            }
            if (bl) {
                slot[t] = queued + (int)__builtin_amdgcn_mbcnt_hi(
                                       (uint32_t)(mask >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                arg[slot[t]] = x;
            }
            has[t] = h;
            below[t] = bl;
            T[t] = x;
            S[t] = s;
            queued += cnt;
            steps = t + 1;
        }
        carry = full;
        wave_order();
        // the queue, one argument per lane, all below the cut-off
        if (lane < queued) {
            if constexpr (stream) {
                auto put = [&](int m, double v) { val[m][lane] = v; };
                boys::eval_f64_each<N, boys::kBelowCut>(arg[lane], tab, put);
            } else {
                double F[N + 1];
                boys::eval_f64<N, boys::kBelowCut>(arg[lane], tab, F);
#pragma unroll
                for (int m = 0; m <= N; ++m)
                    val[m][lane] = F[m];
            }
        }
        wave_order();
        // the window's steps in order
#pragma unroll
        for (int t = 0; t < kEriWindow; ++t) {
            if (t < steps && has[t]) {
                if constexpr (stream) {
                    const double st = S[t];
                    if (below[t]) {
#pragma unroll
                        for (int m = 0; m <= N; ++m)
                            acc[m] = __builtin_fma(st, val[m][slot[t]], acc[m]);
                    } else {
                        auto add = [&](int m, double v) { acc[m] = __builtin_fma(st, v, acc[m]); };
                        boys::eval_f64_each<N, boys::kPastCut>(T[t], tab, add);
                    }
                } else {
                    double F[N + 1];
                    if (below[t]) {
#pragma unroll
                        for (int m = 0; m <= N; ++m)
                            F[m] = val[m][slot[t]];
                    } else {
                        boys::eval_f64<N, boys::kPastCut>(T[t], tab, F);
                    }
#pragma unroll
                    for (int m = 0; m <= N; ++m)
                        acc[m] = __builtin_fma(S[t], F[m], acc[m]);
                }
            }
        }
        wave_order();  // the next window rewrites the queue
    }
    if (live) {
#pragma unroll
        for (int m = 0; m <= N; ++m)
            store_nt(acc[m], out + (int64_t)m * ld + ij);
    }
}

}  // namespace
