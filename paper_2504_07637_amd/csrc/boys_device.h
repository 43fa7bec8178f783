// boys_device.h -- per-lane evaluation of the Boys functions F_0..F_n for gfx950.
//
// One lane evaluates one argument x.  For the order n = n_max (a compile-time constant,
// so every loop below is unrolled and every coefficient is an immediate) the lane
// computes, following Laikov, arXiv 2504.07637, section "Methodology":
//
//   e   = exp(-x)                                   correctly rounded binary64
//   u,v = products of the factors of Eqs. pz, qz      (negative-real-part roots gathered
//                                                     into one Horner polynomial)
//   Q   = q0 + q1 x + q2 (u/v) x^2                   Eq. pqz
//   W   = Q^n sqrt(Q) e,  G = x + W                   Eq. fq
//   F_n = c_n / (G^n sqrt(G))                         Eq. fq
//   F_{m-1} = (2x F_m + e) / (2m-1), m = n..1         Eq. r (divisor 2m-1, see below)
//
// and, past the cut-off x > z_nb, the long-range limit c_m / x^(m+1/2) of Eq. limf1 for
// every m, generated upward from c_0 / sqrt(x).
//
// Arithmetic contract (the results are reproducible bit for bit on any IEEE machine
// that follows the same steps):
//   * every +, -, *, / and sqrt is a single correctly rounded IEEE operation; nothing is
//     contracted into an fma except where an fma is written out;
//   * exp(-x) is the correctly rounded binary64 value (Tang's table method with a
//     double-only fast path and Ziv's rounding test; when the test cannot decide, a
//     double-double evaluation with error below 2^-95 before its one rounding, so a
//     misrounding needs exp(-x) within 2^-95 of a rounding boundary); the classes with
//     binary32 arithmetic use that value rounded to binary32, which a shorter evaluation
//     decides whenever it is safely away from a binary32 rounding midpoint (exp_rn32);
//   * y^n is left-to-right binary powering, y^(n+1/2) = y^n * sqrt(y);
//   * the recursion F_{m-1} = RN(RN(RN(2x) F_m) + e) / (2m-1)) divides by the odd
//     constant d = 2m-1 as q = t*r, r = RN(1/d),
//     q' = fma(fma(-q, d, t), r, q).  This is the correctly rounded t/d: the exact t/d
//     is at least ulp/(2d) away from a rounding midpoint (t has a 53-bit or 24-bit
//     significand and d is odd, so t/d cannot be a midpoint and differs from one by a
//     multiple of ulp/(2d)), while q + (t - q d) r differs from t/d by less than
//     2^-51 ulp.  The classes with binary32 outputs take the step as one product
//     RN(t * RN(1/d)) instead (recurse_down_rcp); their values need far less than the
//     working precision;
//   * x < 0 becomes NaN on entry, and NaN reaches every row through the arithmetic.
//
// The recursion divisor: the paper prints Eq. r with 2m+1; integrating
// d/dt (t^(2m-1) exp(-x t^2)) over [0, 1] gives exp(-x) = (2m-1) F_{m-1} - 2x F_m.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "boys_tables.inc"

#pragma clang fp contract(off)

namespace boys {
// internal linkage, like the coefficient tables these functions read
namespace {

// ---------------------------------------------------------------------------------
// double-double helpers (error-free transformations)

struct dd {
    double hi, lo;
};

__host__ __device__ __forceinline__ dd two_prod(double a, double b)
{
    const double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}

// requires |a| >= |b| (or a == 0)
__host__ __device__ __forceinline__ dd fast_two_sum(double a, double b)
{
    const double s = a + b;
    return {s, b - (s - a)};
}

__host__ __device__ __forceinline__ dd two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

// (a.hi + a.lo) * (b.hi + b.lo), relative error about 2^-104
__host__ __device__ __forceinline__ dd mul_dd(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    double lo = __builtin_fma(a.hi, b.lo, p.lo);
    lo = __builtin_fma(a.lo, b.hi, lo);
    return fast_two_sum(p.hi, lo);
}

// a + b for |a.hi| >= |b.hi|
__host__ __device__ __forceinline__ dd add_dd_fast(dd a, dd b)
{
    dd s = fast_two_sum(a.hi, b.hi);
    const double lo = s.lo + (a.lo + b.lo);
    return fast_two_sum(s.hi, lo);
}

// ---------------------------------------------------------------------------------
// correctly rounded exp(a) for a in [-120, 0]
//
// tab: the 256 pairs (hi, lo) of 2^(j/256) (kept in L1 or LDS by the kernels).
// a = k ln2/256 + r with |r| <= ln2/512 and r a double-double (k * L1 exact), then
// exp(a) = 2^m 2^(j/256) exp(r), k = 256 m + j.
//
// Fast path (Ziv's strategy): exp(r) - 1 = r_hi + w with w = r_lo + r_hi r_lo +
// r_hi^2 P(r_hi), P the Taylor polynomial 1/2 + r/6 + .. + r^4/720 (truncation below
// 2^-78); the result S + e = T (1 + r_hi + w) as an unevaluated sum has a relative
// error below 2^-70.  If S + 1.0000152 e still rounds to S (|e| stays 2^-16 of a
// half-ulp away from a rounding boundary, more than the error can cover) then S is the
// correctly rounded value.  Otherwise, about once in 2^16 arguments, the slow path
// recomputes exp(r) in double-double (error below 2^-95) and rounds once.

__host__ __device__ __forceinline__ double exp_rn_slow(dd r, double2 T, int m)
{
    using namespace boys_tab;
    const double rh = r.hi;
    // exp(r) - 1 = r + r^2 s2, s2 = 1/2 + r s3, s3 = 1/6 + r s4, s4 = 1/24 + r s5
    const double s5 = kInvFact5_hi + rh * (kInvFact6_hi + rh * (kInvFact7_hi + rh * kInvFact8_hi));
    dd s4 = fast_two_sum(kInvFact4_hi, rh * s5);
    s4.lo += kInvFact4_lo;
    const dd s3 = add_dd_fast(dd{kInvFact3_hi, kInvFact3_lo}, mul_dd(r, s4));
    const dd s2 = add_dd_fast(dd{0.5, 0.0}, mul_dd(r, s3));
    const dd pm1 = add_dd_fast(r, mul_dd(r, mul_dd(r, s2)));
    dd q = two_prod(T.x, pm1.hi);
    double lo = __builtin_fma(T.x, pm1.lo, q.lo);
    lo = __builtin_fma(T.y, pm1.hi, lo);
    lo = lo + T.y;
    const dd s = fast_two_sum(T.x, q.hi);
    const double v = s.hi + (s.lo + lo);
    return __builtin_ldexp(v, m);
}

__host__ __device__ __forceinline__ double exp_rn(double a, const double2 *__restrict__ tab)
{
    using namespace boys_tab;
    const double kd = __builtin_rint(a * kInvLn2x256);
    const int k = (int)kd;
    const int j = k & 255;
    const int m = (k - j) / 256;
    const double t = __builtin_fma(-kd, kLn2d256_1, a);
    const dd p2 = two_prod(kd, kLn2d256_2);
    dd r = two_sum(t, -p2.hi);
    r = fast_two_sum(r.hi, (r.lo - p2.lo) - kd * kLn2d256_3);
    const double2 T = tab[j];
    const double rh = r.hi;
    double P = __builtin_fma(rh, kInvFact6_hi, kInvFact5_hi);
    P = __builtin_fma(rh, P, kInvFact4_hi);
    P = __builtin_fma(rh, P, kInvFact3_hi);
    P = __builtin_fma(rh, P, 0.5);
    const double w = __builtin_fma(rh * rh, P, __builtin_fma(rh, r.lo, r.lo));
    const dd q = two_prod(T.x, rh);
    double lo = __builtin_fma(T.x, w, q.lo);
    lo = __builtin_fma(T.y, rh, lo) + T.y;
    const dd s = fast_two_sum(T.x, q.hi);
    const double e = s.lo + lo;
    if (s.hi + e * 0x1.0001p+0 == s.hi)
        return __builtin_ldexp(s.hi, m);
    return exp_rn_slow(r, T, m);
}

// RN32(exp_rn(a)) for a in [-120, 0]: the binary32 rounding of the correctly rounded
// binary64 exp, as the classes with binary32 arithmetic use it.  A short evaluation
// usually decides it: v = T_hi * P(r), P the degree-4 Taylor polynomial of exp(r) (|r| <=
// ln2/512, truncation below 2^-54.5), r from the two-part reduction, so that v differs
// from exp(a) 2^-m by less than 2^-51 relative and from RN64(exp(a)) 2^-m by less than
// 2^-50.9.
// When v lies farther than 2^-47 (absolute, v < 2) from every binary32 rounding midpoint,
// exp(a) and its binary64 rounding round to the same binary32 value as v.  Otherwise, or
// when the result would fall below the binary32 normal range, the full exp_rn decides.
__host__ __device__ __forceinline__ float exp_rn32(double a, const double2 *__restrict__ tab)
{
    using namespace boys_tab;
    const double kd = __builtin_rint(a * kInvLn2x256);
    const int k = (int)kd;
    const int m = k >> 8;  // floor(k / 256)
    double r = __builtin_fma(-kd, kLn2d256_1, a);
    r = __builtin_fma(-kd, kLn2d256_2, r);
    double P = __builtin_fma(r, kInvFact4_hi, kInvFact3_hi);
    P = __builtin_fma(r, P, 0.5);
    P = __builtin_fma(r, P, 1.0);
    P = __builtin_fma(r, P, 1.0);
    const double v = tab[k & 255].x * P;
    const float f = (float)v;
    const double d = v - (double)f;  // exact
    // half a binary32 ulp below 1 and above it, less the error bound
    const double h = v < 1.0 ? 0x1p-25 - 0x1p-47 : 0x1p-24 - 0x1p-47;
    if (__builtin_fabs(d) < h && m >= -125)
        return __builtin_ldexpf(f, m);
    return (float)exp_rn(a, tab);
}

// ---------------------------------------------------------------------------------
// small building blocks

// y^K by left-to-right binary powering
template <int K, typename T>
__host__ __device__ __forceinline__ T powi(T y)
{
    if constexpr (K == 0) {
        return T(1);
    } else {
        constexpr int top = 31 - __builtin_clz((unsigned)K);
        T r = y;
#pragma unroll
        for (int b = top - 1; b >= 0; --b) {
            r = r * r;
            if ((K >> b) & 1)
                r = r * y;
        }
        return r;
    }
}

// RN(1/(2m-1)) for m = 1..kRcpSize-1, folded at compile time
constexpr int kRcpSize = 64;
struct OddReciprocals {
    double d[kRcpSize];
    float f[kRcpSize];
    constexpr OddReciprocals() : d(), f()
    {
        for (int m = 1; m < kRcpSize; ++m) {
            d[m] = 1.0 / (double)(2 * m - 1);
            f[m] = 1.0f / (float)(2 * m - 1);
        }
    }
};
constexpr OddReciprocals kOddRcp{};

// correctly rounded t / (2m-1) for a compile-time m (see the header comment)
template <int M>
__host__ __device__ __forceinline__ double div_odd(double t)
{
    static_assert(M >= 1 && M < kRcpSize, "recursion order out of range");
    if constexpr (M == 1) {
        return t;
    } else {
        constexpr double d = (double)(2 * M - 1);
        constexpr double r = kOddRcp.d[M];
        const double q = t * r;
        const double rem = __builtin_fma(-q, d, t);
        return __builtin_fma(rem, r, q);
    }
}

template <int M>
__host__ __device__ __forceinline__ float div_odd(float t)
{
    static_assert(M >= 1 && M < kRcpSize, "recursion order out of range");
    if constexpr (M == 1) {
        return t;
    } else {
        constexpr float d = (float)(2 * M - 1);
        constexpr float r = kOddRcp.f[M];
        const float q = t * r;
        const float rem = __builtin_fmaf(-q, d, t);
        return __builtin_fmaf(rem, r, q);
    }
}

// The evaluations below hand each F_m to put(m, F_m) as they form it; the forms that fill
// an array F are the same code with put storing into F.  A consumer that adds the values
// into sums as they come then holds no array of N+1 values.

// downward recursion of Eq. r from F[M] to F[0], unrolled at compile time
template <int M, typename T, class Put>
__host__ __device__ __forceinline__ void recurse_down_each(T x2, T e, T f, Put &put)
{
    if constexpr (M >= 1) {
        const T g = div_odd<M>(x2 * f + e);
        put(M - 1, g);
        recurse_down_each<M - 1, T>(x2, e, g, put);
    }
}

// the same recursion with each step a multiplication by RN(1/(2m-1)) instead of a
// correctly rounded division: one operation instead of three, for the classes with
// binary32 outputs, whose values need far less than the working precision (the downward
// recursion damps the extra rounding)
template <int M, typename T, class Put>
__host__ __device__ __forceinline__ void recurse_down_rcp_each(T x2, T e, T f, Put &put)
{
    if constexpr (M >= 1) {
        T g = x2 * f + e;
        if constexpr (M > 1) {
            if constexpr (sizeof(T) == 8)
                g = g * kOddRcp.d[M];
            else
                g = g * kOddRcp.f[M];
        }
        put(M - 1, g);
        recurse_down_rcp_each<M - 1, T>(x2, e, g, put);
    }
}

template <int M, typename T>
__host__ __device__ __forceinline__ void recurse_down_rcp(T x2, T e, T f, T *F)
{
    auto put = [F](int m, T v) { F[m] = v; };
    recurse_down_rcp_each<M, T>(x2, e, f, put);
}

// one of u, v: gathered monic polynomial (Horner), then quadratic, then linear factors
template <typename T, int NG, int NQ, int NL>
__host__ __device__ __forceinline__ T factors(T x, const T (&g)[NG > 0 ? NG : 1],
                                              const T (&q)[NQ > 0 ? 2 * NQ : 1],
                                              const T (&l)[NL > 0 ? NL : 1])
{
    T p = T(1);
#pragma unroll
    for (int k = NG - 1; k >= 0; --k)
        p = p * x + g[k];
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        p = p * ((x - q[2 * k]) * (x - q[2 * k]) + q[2 * k + 1]);
#pragma unroll
    for (int k = 0; k < NL; ++k)
        p = p * (x - l[k]);
    return p;
}

// ---------------------------------------------------------------------------------
// F_0..F_N for one argument, binary64 class

// The two sides of the cut-off share one division and one square root, at the same place
// in the code: below it u/v and c_n / (G^n sqrt(G)), past it 1/x and c_0 / (1 sqrt(x)).  Each
// lane performs exactly the correctly rounded operations of its own side on the operands
// that side selects (a product with 1 is exact), so the values are those of two separate
// branches bit for bit; a wave with lanes on both sides (on the integral workload nearly
// every wave) issues the division and the square root once instead of once per side.
//
// Side: a caller whose lanes all lie on one side of the cut-off (it has tested
// !(x > z) itself, the same test) names that side, and the other side's code is not
// generated; the operations of the side taken are the same.
enum : int { kBothSides = 0, kBelowCut = 1, kPastCut = 2 };

template <class S, int N, bool RcpRecursion = false, int Side = kBothSides, class Put>
__host__ __device__ __forceinline__ void eval_f64_set_each(double x,
                                                           const double2 *__restrict__ tab,
                                                           Put &put)
{
    // outside the domain (x < 0) the argument becomes NaN, which every step below carries
    // into every row (fmax keeps the exponential's argument finite)
    x = x >= 0.0 ? x : __builtin_nan("");
    // below the cut-off, and NaN
    const bool below = Side == kBelowCut || (Side == kBothSides && !(x > S::z));
    double e = 0.0, num = 1.0, den = x;
    if (below) {
        e = exp_rn(__builtin_fmax(-x, -120.0), tab);
        num = factors<double, S::ug_n, S::uq_n, S::ul_n>(x, S::ug, S::uq, S::ul);
        den = factors<double, S::vg_n, S::vq_n, S::vl_n>(x, S::vg, S::vq, S::vl);
    }
    const double d = num / den;  // u/v below the cut-off, 1/x past it
    double C = boys_tab::kC0, G = x, Gn = 1.0;
    if (below) {
        const double Q = S::q0 + S::q1 * x + S::q2 * d * x * x;
        const double W = powi<N>(Q) * __builtin_sqrt(Q) * e;
        G = x + W;
        Gn = powi<N>(G);
        C = S::c;
    }
    // F_n below the cut-off; past it F_0 of Eq. limf1 (x = +inf gives 0 everywhere)
    const double f = C / (Gn * __builtin_sqrt(G));
    if (below) {
        put(N, f);
        if constexpr (RcpRecursion)
            recurse_down_rcp_each<N, double>(2.0 * x, e, f, put);
        else
            recurse_down_each<N, double>(2.0 * x, e, f, put);
    } else {
        // Eq. limf1 for every m, generated upward with d = 1/x
        double g = f;
        put(0, g);
#pragma unroll
        for (int m = 1; m <= N; ++m) {
            g = g * (m - 0.5) * d;
            put(m, g);
        }
    }
}

template <class S, int N, bool RcpRecursion = false, int Side = kBothSides>
__host__ __device__ __forceinline__ void eval_f64_set(double x, const double2 *__restrict__ tab,
                                                      double (&F)[N + 1])
{
    auto put = [&F](int m, double v) { F[m] = v; };
    eval_f64_set_each<S, N, RcpRecursion, Side>(x, tab, put);
}

// the binary64 class: Table 1's binary64 approximants, cut-off z_{n,53}
template <int N, int Side = kBothSides>
__host__ __device__ __forceinline__ void eval_f64(double x, const double2 *__restrict__ tab,
                                                  double (&F)[N + 1])
{
    eval_f64_set<boys_tab::F64Set<N>, N, false, Side>(x, tab, F);
}

// the same, each F_m handed to put(m, F_m)
template <int N, int Side = kBothSides, class Put>
__host__ __device__ __forceinline__ void eval_f64_each(double x, const double2 *__restrict__ tab,
                                                       Put &put)
{
    eval_f64_set_each<boys_tab::F64Set<N>, N, false, Side>(x, tab, put);
}

// the binary32-output class computed in binary64: approximants of about 28 bits with the
// cut-off z_{n,28}, the recursion by reciprocals, every value rounded once to binary32
// (by the caller)
template <int N>
__host__ __device__ __forceinline__ void eval_f32r(double x, const double2 *__restrict__ tab,
                                                   double (&F)[N + 1])
{
    eval_f64_set<boys_tab::F32xSet<N>, N, true>(x, tab, F);
}

// ---------------------------------------------------------------------------------
// The two-approximation option of section "Computations" (binary64): F_nbar and F_N from
// their own best approximants (order nbar given at run time, nbar < N), the downward
// recursion from N to nbar+1 and from nbar to 0, one exp(-x) for both.  Every value is
// the one the plain evaluation of its own order gives: rows 0..nbar those of order nbar,
// rows nbar+1..N those of order N.

// factors() for a set read at run time: the same operations in the same order
__host__ __device__ __forceinline__ double factors_rt(double x, const double *c, int ng, int nq,
                                                      int nl)
{
    double p = 1.0;
    for (int k = ng - 1; k >= 0; --k)
        p = p * x + c[k];
    c += ng;
    for (int k = 0; k < nq; ++k)
        p = p * ((x - c[2 * k]) * (x - c[2 * k]) + c[2 * k + 1]);
    c += 2 * nq;
    for (int k = 0; k < nl; ++k)
        p = p * (x - c[k]);
    return p;
}

// powi<K>() for a run-time K >= 0: the same left-to-right binary powering
__host__ __device__ __forceinline__ double powi_rt(double y, int k)
{
    if (k == 0)
        return 1.0;
    const int top = 31 - __builtin_clz((unsigned)k);
    double r = y;
    for (int b = top - 1; b >= 0; --b) {
        r = r * r;
        if ((k >> b) & 1)
            r = r * y;
    }
    return r;
}

// F[M-1] .. F[nbar+1] by Eq. r from f = F[M] (steps at or below nbar skipped)
template <int M>
__host__ __device__ __forceinline__ void recurse_down_to(int nbar, double x2, double e, double f,
                                                         double *F)
{
    if constexpr (M >= 1) {
        if (M - 1 > nbar) {
            const double g = div_odd<M>(x2 * f + e);
            F[M - 1] = g;
            recurse_down_to<M - 1>(nbar, x2, e, g, F);
        }
    }
}

// F[M] for M = nbar..0 by Eq. r, starting from g = F[nbar]; M runs down from a
// compile-time bound so that every divisor is a constant
template <int M>
__host__ __device__ __forceinline__ void recurse_low(int nbar, double x2, double e, double &g,
                                                     double *F)
{
    if (M <= nbar) {
        if (M < nbar)
            g = div_odd<M + 1>(x2 * g + e);
        F[M] = g;
    }
    if constexpr (M > 0)
        recurse_low<M - 1>(nbar, x2, e, g, F);
}

// the upward product of Eq. limf1 for F[1..lim] from f = F[0]
template <int N>
__host__ __device__ __forceinline__ void chain_up(int lim, double ix, double f, double *F)
{
#pragma unroll
    for (int m = 1; m <= N; ++m) {
        if (m <= lim) {
            f = f * (m - 0.5) * ix;
            F[m] = f;
        }
    }
}

template <int N>
__host__ __device__ __forceinline__ void eval_split(double x, int nbar,
                                                    const double2 *__restrict__ tab,
                                                    double (&F)[N + 1])
{
    static_assert(N >= 1, "the two-approximation option needs nbar < N");
    x = x >= 0.0 ? x : __builtin_nan("");  // as in eval_f64_set
    using S = boys_tab::F64Set<N>;
    const boys_tab::RtSet &B = boys_tab::kRt64[nbar];
    const bool below_n = !(x > S::z);  // z_nbar < z_N: below_b implies below_n
    const bool below_b = !(x > B.z);
    double e = 0.0, num = 1.0, den = x;
    if (below_n) {
        e = exp_rn(__builtin_fmax(-x, -120.0), tab);
        const double u = factors<double, S::ug_n, S::uq_n, S::ul_n>(x, S::ug, S::uq, S::ul);
        const double v = factors<double, S::vg_n, S::vq_n, S::vl_n>(x, S::vg, S::vq, S::vl);
        const double Q = S::q0 + S::q1 * x + S::q2 * (u / v) * x * x;
        const double W = powi<N>(Q) * __builtin_sqrt(Q) * e;
        const double G = x + W;
        const double f = S::c / (powi<N>(G) * __builtin_sqrt(G));
        F[N] = f;
        recurse_down_to<N>(nbar, 2.0 * x, e, f, F);
        if (below_b) {
            const double *cu = boys_tab::kRtCoef64 + B.off;
            const double *cv = cu + B.ug_n + 2 * B.uq_n + B.ul_n;
            num = factors_rt(x, cu, B.ug_n, B.uq_n, B.ul_n);
            den = factors_rt(x, cv, B.vg_n, B.vq_n, B.vl_n);
        }
    }
    // the order-nbar approximant below z_nbar and Eq. limf1 past it share one division and
    // one square root, as in eval_f64_set: ub/vb or 1/x, then F_nbar or F_0
    const double d = num / den;
    double C = boys_tab::kC0, G = x, Gn = 1.0;
    if (below_b) {
        const double Qb = B.q0 + B.q1 * x + B.q2 * d * x * x;
        const double Wb = powi_rt(Qb, nbar) * __builtin_sqrt(Qb) * e;
        G = x + Wb;
        Gn = powi_rt(G, nbar);
        C = B.c;
    }
    double g = C / (Gn * __builtin_sqrt(G));
    if (below_b) {
        recurse_low<N - 1>(nbar, 2.0 * x, e, g, F);
    } else {
        // Eq. limf1 for rows 0..nbar (z_nbar < x <= z_N) or for every row (x > z_N)
        F[0] = g;
        chain_up<N>(below_n ? nbar : N, d, g, F);
    }
}

// ---------------------------------------------------------------------------------
// F_0..F_N for one argument, mixed binary32/binary64 class

// Separate branches here: sharing the binary64 division and square root between the two
// sides, as eval_f64_set does, measured 3.6% slower for this class's full-row kernel
// (0.897 against 0.866 ms at n_max = 16, 2^26 arguments), though fewer instructions.
template <int N>
__host__ __device__ __forceinline__ void eval_f32(double x, const double2 *__restrict__ tab,
                                                  float (&F)[N + 1])
{
    using S = boys_tab::F32Set<N>;
    x = x >= 0.0 ? x : __builtin_nan("");  // as in eval_f64_set
    if (!(x > S::z)) {
        const float xf = (float)x;
        const float e = exp_rn32(__builtin_fmax(-x, -120.0), tab);
        const float u = factors<float, S::ug_n, S::uq_n, S::ul_n>(xf, S::ug, S::uq, S::ul);
        const float v = factors<float, S::vg_n, S::vq_n, S::vl_n>(xf, S::vg, S::vq, S::vl);
        const float Q = S::q0 + S::q1 * xf + S::q2 * (u / v) * xf * xf;
        const float W = powi<N>(Q) * __builtin_sqrtf(Q) * e;
        const double G = x + (double)W;
        const float f = (float)(S::c / (powi<N>(G) * __builtin_sqrt(G)));
        F[N] = f;
        recurse_down_rcp<N, float>(2.0f * xf, e, f, F);
    } else {
        const double ix = 1.0 / x;
        double f = boys_tab::kC0 / __builtin_sqrt(x);
        F[0] = (float)f;
#pragma unroll
        for (int m = 1; m <= N; ++m) {
            f = f * (m - 0.5) * ix;
            F[m] = (float)f;
        }
    }
}

// ---------------------------------------------------------------------------------
// F_0..F_N for one argument, all binary32 below the cut-off (the arithmetic of Table 1's
// binary32 columns): G = x + W in binary32 and F_N = (kappa_N / G)^(N+1/2) with kappa_N =
// c_N^(1/(N+1/2)) in binary32 (c_N itself leaves the binary32 range beyond N = 27); the
// recursion by reciprocals; past the cut-off the same long-range limit as eval_f32

template <int N>
__host__ __device__ __forceinline__ void eval_f32s(double x, const double2 *__restrict__ tab,
                                                   float (&F)[N + 1])
{
    using S = boys_tab::F32Set<N>;
    x = x >= 0.0 ? x : __builtin_nan("");  // as in eval_f64_set
    if (!(x > S::z)) {
        const float xf = (float)x;
        const float e = exp_rn32(__builtin_fmax(-x, -120.0), tab);
        const float u = factors<float, S::ug_n, S::uq_n, S::ul_n>(xf, S::ug, S::uq, S::ul);
        const float v = factors<float, S::vg_n, S::vq_n, S::vl_n>(xf, S::vg, S::vq, S::vl);
        const float Q = S::q0 + S::q1 * xf + S::q2 * (u / v) * xf * xf;
        const float W = powi<N>(Q) * __builtin_sqrtf(Q) * e;
        const float G = xf + W;
        const float t = boys_tab::kKappa32[N] / G;
        const float f = powi<N>(t) * __builtin_sqrtf(t);
        F[N] = f;
        recurse_down_rcp<N, float>(2.0f * xf, e, f, F);
    } else {
        const double ix = 1.0 / x;
        double f = boys_tab::kC0 / __builtin_sqrt(x);
        F[0] = (float)f;
#pragma unroll
        for (int m = 1; m <= N; ++m) {
            f = f * (m - 0.5) * ix;
            F[m] = (float)f;
        }
    }
}

}  // namespace
}  // namespace boys
