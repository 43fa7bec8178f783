/*
 * CPU oracle for the Boys functions and for Laikov's closed-form approximant
 * (arXiv 2504.07637).  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark are its only users.  Nothing on the product
 * path may call, link or load it, and it shares no code with the GPU library.
 *
 * It is deliberately plain and slow:
 *
 *   1. oracle_boys_exact: the Boys function itself, F_m(x) = int_0^1 t^2m exp(-x t^2) dt
 *      (section "Introduction", Eq. fn), in binary128, for each m independently:
 *        - x = 0: the integral is 1/(2m+1);
 *        - 0 < x <= X_m: the Kummer-transformed series
 *              F_m(x) = exp(-x) sum_{k>=0} (2x)^k / ((2m+1)(2m+3)...(2m+2k+1)),
 *          whose terms are all positive (no cancellation);
 *        - x > X_m: F_m(x) = (Gamma(m+1/2) - Gamma(m+1/2, x)) / (2 x^(m+1/2)), with
 *          Gamma(1/2, x) = sqrt(pi) erfc(sqrt x) and the upward recurrence
 *          Gamma(a+1, x) = a Gamma(a, x) + x^a exp(-x); the leading term is the
 *          long-range limit of Eq. limf1.
 *      The result is returned as an unevaluated double-double hi + lo.
 *
 *   2. oracle_boys_approx_f64: the approximant of section "Methodology", evaluated in
 *      IEEE binary64 step by step in the paper's order and notation:
 *        e   = exp(-x)                                  (one exponential, shared)
 *        u,v = products of factors (Eqs. pz, qz), the negative-real-part factors
 *              gathered into one polynomial evaluated by Horner's rule
 *        Q   = q0 + q1 x + q2 (u/v) x^2                 (Eq. pqz)
 *        F_n = c_n / (x + Q^(n+1/2) e)^(n+1/2)          (Eq. fq)
 *        F_{m-1} = (2x F_m + e) / (2m-1), m = n..1       (Eq. r; see below)
 *      and, past the cut-off x > z_nb, the long-range limit (Eq. limf1) for every m.
 *
 *   3. oracle_boys_approx_mixed: the same approximant with the rational function, the
 *      power Q^(n+1/2) and the recursion in binary32 and only x + W and
 *      c_n / G^(n+1/2) in binary64.  The classes with binary32 outputs (this one and
 *      oracle_boys_approx_f64r for the ~28-bit sets) take each recursion step as a
 *      multiplication by RN(1/(2m-1)) rather than a division: their outputs need far
 *      less than the working precision, and the downward recursion damps the extra
 *      rounding (the accuracy pins hold them to the same bounds).
 *      oracle_boys_approx_single is the all-binary32 evaluation that Table 1's binary32
 *      columns describe, with F_n = (kappa_n / G)^(n+1/2) to stay in range.
 *
 *   4. oracle_boys_approx_q: F~_n alone in binary128 from extended-precision
 *      coefficients, i.e. the approximant in (nearly) exact arithmetic, for the
 *      exact-arithmetic error E_n of Eq. e.
 *
 *   5. oracle_eri_ssss: a consumer of F_m, the contracted (ss|ss)^(m) auxiliary
 *      two-electron integrals of s-type Gaussians (the application the paper names),
 *      with x = rho |PQ|^2 formed from the pair data and every sum in a fixed order.
 *
 * Readings where the paper leaves the arithmetic open or is misprinted (all also used by
 * the GPU library, which implements them independently):
 *   - Eq. r is printed with the divisor 2m+1; integrating d/dt(t^(2m-1) exp(-x t^2)) over
 *     [0,1] gives e^-x = (2m-1) F_{m-1} - 2x F_m, so the divisor used is 2m-1 (this is
 *     also the only choice with F_{m-1}(0) = 1/(2m-1));
 *   - exp(-x) is the correctly rounded binary64 value (here: binary128 expq, rounded);
 *     the binary32 class rounds that binary64 value to binary32;
 *   - y^(n+1/2) = y^n * sqrt(y), with y^n by left-to-right binary powering
 *     (square, then multiply when the next exponent bit is set);
 *   - past the cut-off every F_m is the long-range limit c_m / x^(m+1/2), generated
 *     upward from F_0 = c_0 / sqrt(x) by F_m = F_{m-1} (m - 1/2) / x, with 1/x rounded once;
 *   - x < 0 or NaN gives NaN for every m; x = +inf gives 0 for every m.
 * Built with -ffp-contract=off: every + - * / sqrt is one IEEE operation, no fusion.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------------------ */
/* 1. the Boys function by its definition                                           */

static __float128 boys_exact_q(__float128 x, int m)
{
    const __float128 two_m1 = (__float128)(2 * m + 1);
    if (x == 0)
        return 1 / two_m1;
    /* crossover between the series and the incomplete-gamma form */
    const double Xm = (2.0 * m + 20.0 > 30.0) ? 2.0 * m + 20.0 : 30.0;
    if (x <= (__float128)Xm) {
        /* Kummer series: all terms positive */
        __float128 term = 1 / two_m1;
        __float128 sum = term;
        for (int k = 1; k < 100000; ++k) {
            term = term * (2 * x) / (__float128)(2 * m + 2 * k + 1);
            sum += term;
            if ((__float128)k > x && term < sum * 1e-36Q)
                break;
        }
        return expq(-x) * sum;
    }
    /* F_m = (Gamma(m+1/2) - Gamma(m+1/2, x)) / (2 x^(m+1/2)) */
    const __float128 sqrtpi = sqrtq(M_PIq);
    __float128 gam = sqrtpi;                       /* Gamma(1/2) */
    __float128 ugam = sqrtpi * erfcq(sqrtq(x));    /* Gamma(1/2, x) */
    const __float128 lx = logq(x);
    for (int j = 0; j < m; ++j) {
        const __float128 a = (__float128)j + 0.5Q;
        ugam = a * ugam + expq(a * lx - x);        /* Gamma(a+1, x) */
        gam = a * gam;                             /* Gamma(a+1) */
    }
    return (gam - ugam) / (2 * expq(((__float128)m + 0.5Q) * lx));
}

/* F_m(x_i) for m = 0..mmax; hi/lo are (mmax+1) x n, row m at offset m*n. */
int oracle_boys_exact(const double *x, int64_t n, int mmax, double *hi, double *lo)
{
    if (n < 0 || mmax < 0)
        return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const double xi = x[i];
        for (int m = 0; m <= mmax; ++m) {
            double h, l;
            if (!(xi >= 0)) {
                h = NAN;
                l = 0;
            } else if (isinf(xi)) {
                h = 0;
                l = 0;
            } else {
                const __float128 f = boys_exact_q((__float128)xi, m);
                h = (double)f;
                l = (double)(f - (__float128)h);
            }
            hi[(int64_t)m * n + i] = h;
            lo[(int64_t)m * n + i] = l;
        }
    }
    return 0;
}

/* F_m(x_i) for one order m only */
int oracle_boys_exact_one(const double *x, int64_t n, int m, double *hi, double *lo)
{
    if (n < 0 || m < 0)
        return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const double xi = x[i];
        if (!(xi >= 0)) {
            hi[i] = NAN;
            lo[i] = 0;
        } else if (isinf(xi)) {
            hi[i] = 0;
            lo[i] = 0;
        } else {
            const __float128 f = boys_exact_q((__float128)xi, m);
            hi[i] = (double)f;
            lo[i] = (double)(f - (__float128)hi[i]);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* coefficient records, passed flat from the Python side                            */
/*
 * rec[] layout (all doubles; counts are small integers held exactly):
 *   [0] n   [1] c_n   [2] z_nb   [3] q0   [4] q1   [5] q2   [6] c_0
 *   then for u and then for v:
 *     kg, g_0 .. g_{kg-1}            gathered monic factor, ascending, leading 1 implied
 *     kq, y_1, a_1, .., y_kq, a_kq   quadratic factors (x - y)^2 + a
 *     kl, y_1 .. y_kl                linear factors (x - y)
 * For the binary32 class every coefficient except c_n, z_nb and c_0 is a binary32 value.
 */
typedef struct {
    int n;
    double c, z, q0, q1, q2, c0;
    int ug, uq, ul, vg, vq, vl;
    const double *pug, *puq, *pul, *pvg, *pvq, *pvl;
} record;

static int parse_record(const double *rec, int len, record *r)
{
    int p = 7;
    if (len < 13)
        return 1;
    r->n = (int)rec[0];
    r->c = rec[1];
    r->z = rec[2];
    r->q0 = rec[3];
    r->q1 = rec[4];
    r->q2 = rec[5];
    r->c0 = rec[6];
#define TAKE(cnt, ptr, width)                 \
    do {                                      \
        if (p >= len) return 1;               \
        cnt = (int)rec[p++];                  \
        ptr = rec + p;                        \
        p += (width) * cnt;                   \
        if (p > len) return 1;                \
    } while (0)
    TAKE(r->ug, r->pug, 1);
    TAKE(r->uq, r->puq, 2);
    TAKE(r->ul, r->pul, 1);
    TAKE(r->vg, r->pvg, 1);
    TAKE(r->vq, r->pvq, 2);
    TAKE(r->vl, r->pvl, 1);
#undef TAKE
    return 0;
}

/* y^k by left-to-right binary powering (k >= 0) */
static double powi_d(double y, int k)
{
    if (k == 0)
        return 1.0;
    int top = 30;
    while (!((k >> top) & 1))
        --top;
    double r = y;
    for (int b = top - 1; b >= 0; --b) {
        r = r * r;
        if ((k >> b) & 1)
            r = r * y;
    }
    return r;
}

static float powi_f(float y, int k)
{
    if (k == 0)
        return 1.0f;
    int top = 30;
    while (!((k >> top) & 1))
        --top;
    float r = y;
    for (int b = top - 1; b >= 0; --b) {
        r = r * r;
        if ((k >> b) & 1)
            r = r * y;
    }
    return r;
}

/* correctly rounded exp in binary64 (binary128 evaluation, one final rounding) */
static double exp_rn(double a)
{
    return (double)expq((__float128)a);
}

/* u(x) or v(x) of Eqs. pz / qz in binary64 */
static double factors_d(double x, int kg, const double *g, int kq, const double *q, int kl,
                        const double *l)
{
    double p = 1.0;
    for (int k = kg - 1; k >= 0; --k)
        p = p * x + g[k];
    for (int k = 0; k < kq; ++k) {
        const double y = q[2 * k], a = q[2 * k + 1];
        p = p * ((x - y) * (x - y) + a);
    }
    for (int k = 0; k < kl; ++k)
        p = p * (x - l[k]);
    return p;
}

static float factors_f(float x, int kg, const double *g, int kq, const double *q, int kl,
                       const double *l)
{
    float p = 1.0f;
    for (int k = kg - 1; k >= 0; --k)
        p = p * x + (float)g[k];
    for (int k = 0; k < kq; ++k) {
        const float y = (float)q[2 * k], a = (float)q[2 * k + 1];
        p = p * ((x - y) * (x - y) + a);
    }
    for (int k = 0; k < kl; ++k)
        p = p * (x - (float)l[k]);
    return p;
}

/* past the cut-off: F_m = c_m / x^(m+1/2) for every m (Eq. limf1), generated upward */
static void asymptote_d(double x, double c0, int nmax, double *F, int64_t stride)
{
    const double ix = 1.0 / x;
    double f = c0 / sqrt(x);
    F[0] = f;
    for (int m = 1; m <= nmax; ++m) {
        f = f * (m - 0.5) * ix;
        F[(int64_t)m * stride] = f;
    }
}

/* F~_m(xi), m = 0..r->n, in binary64 into F[m * stride]; rcp != 0 takes the recursion
   step as a multiplication by the rounded reciprocal of 2m-1 instead of a division */
static void approx_one_d_(const record *r, double xi, double *F, int64_t stride, int rcp)
{
    const int n = r->n;
    if (!(xi >= 0)) {
        for (int m = 0; m <= n; ++m)
            F[(int64_t)m * stride] = NAN;
        return;
    }
    if (isinf(xi)) {
        for (int m = 0; m <= n; ++m)
            F[(int64_t)m * stride] = 0.0;
        return;
    }
    if (xi > r->z) {
        asymptote_d(xi, r->c0, n, F, stride);
        return;
    }
    const double e = exp_rn(-xi);
    const double u = factors_d(xi, r->ug, r->pug, r->uq, r->puq, r->ul, r->pul);
    const double v = factors_d(xi, r->vg, r->pvg, r->vq, r->pvq, r->vl, r->pvl);
    const double Q = r->q0 + r->q1 * xi + r->q2 * (u / v) * xi * xi;
    const double W = powi_d(Q, n) * sqrt(Q) * e;
    const double G = xi + W;
    double Fm = r->c / (powi_d(G, n) * sqrt(G));
    F[(int64_t)n * stride] = Fm;
    for (int m = n; m >= 1; --m) {
        if (rcp)
            Fm = (2.0 * xi * Fm + e) * (1.0 / (2 * m - 1));
        else
            Fm = (2.0 * xi * Fm + e) / (2 * m - 1);
        F[(int64_t)(m - 1) * stride] = Fm;
    }
}

static void approx_one_d(const record *r, double xi, double *F, int64_t stride)
{
    approx_one_d_(r, xi, F, stride, 0);
}

/* 2. F~_m, m = 0..n, in binary64; out is (n+1) x count, row m at offset m*ld */
int oracle_boys_approx_f64(const double *x, int64_t count, const double *rec, int reclen,
                           double *out, int64_t ld)
{
    record r;
    if (parse_record(rec, reclen, &r) || count < 0 || ld < count)
        return 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        approx_one_d(&r, x[i], out + i, ld);
    return 0;
}

/* 2'. the same in binary64 with the recursion step by the rounded reciprocal: the
   evaluation of the ~28-bit sets for binary32 outputs (rounded by the caller) */
int oracle_boys_approx_f64r(const double *x, int64_t count, const double *rec, int reclen,
                            double *out, int64_t ld)
{
    record r;
    if (parse_record(rec, reclen, &r) || count < 0 || ld < count)
        return 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        approx_one_d_(&r, x[i], out + i, ld, 1);
    return 0;
}

/* 3. the mixed binary32/binary64 class; out is float, (n+1) x count, row stride ld */
int oracle_boys_approx_mixed(const double *x, int64_t count, const double *rec, int reclen,
                             float *out, int64_t ld)
{
    record r;
    if (parse_record(rec, reclen, &r) || count < 0 || ld < count)
        return 1;
    const int n = r.n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        const double xi = x[i];
        float *F = out + i;
        if (!(xi >= 0)) {
            for (int m = 0; m <= n; ++m)
                F[(int64_t)m * ld] = NAN;
            continue;
        }
        if (isinf(xi)) {
            for (int m = 0; m <= n; ++m)
                F[(int64_t)m * ld] = 0.0f;
            continue;
        }
        if (xi > r.z) {
            const double ix = 1.0 / xi;
            double f = r.c0 / sqrt(xi);
            F[0] = (float)f;
            for (int m = 1; m <= n; ++m) {
                f = f * (m - 0.5) * ix;
                F[(int64_t)m * ld] = (float)f;
            }
            continue;
        }
        const float xf = (float)xi;
        const float e = (float)exp_rn(-xi);
        const float u = factors_f(xf, r.ug, r.pug, r.uq, r.puq, r.ul, r.pul);
        const float v = factors_f(xf, r.vg, r.pvg, r.vq, r.pvq, r.vl, r.pvl);
        const float Q = (float)r.q0 + (float)r.q1 * xf + (float)r.q2 * (u / v) * xf * xf;
        const float W = powi_f(Q, n) * sqrtf(Q) * e;
        const double G = xi + (double)W;
        float Fm = (float)(r.c / (powi_d(G, n) * sqrt(G)));
        F[(int64_t)n * ld] = Fm;
        for (int m = n; m >= 1; --m) {
            /* multiplication by the rounded reciprocal of 2m-1 (see the header) */
            Fm = (2.0f * xf * Fm + e) * (1.0f / (float)(2 * m - 1));
            F[(int64_t)(m - 1) * ld] = Fm;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* 3'. the all-binary32 evaluation (the arithmetic of Table 1's binary32 columns) with
   the binary32 sets: x, e, u/v, Q, W, G and F_n = (kappa_n / G)^(n+1/2) in binary32,
   kappa_n = c_n^(1/(n+1/2)) rounded once to binary32 (c_n itself leaves the binary32
   range beyond n = 27); the recursion by RN(1/(2m-1)) as in the mixed class; past the
   cut-off the same long-range limit as the mixed class.  out is float.                */
float oracle_kappa32(int n)
{
    const __float128 s = (__float128)n + 0.5Q;
    const __float128 c = tgammaq(s) / 2;
    return (float)powq(c, 1 / s);
}

int oracle_boys_approx_single(const double *x, int64_t count, const double *rec, int reclen,
                              float *out, int64_t ld)
{
    record r;
    if (parse_record(rec, reclen, &r) || count < 0 || ld < count)
        return 1;
    const int n = r.n;
    const float kappa = oracle_kappa32(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        const double xi = x[i];
        float *F = out + i;
        if (!(xi >= 0)) {
            for (int m = 0; m <= n; ++m)
                F[(int64_t)m * ld] = NAN;
            continue;
        }
        if (isinf(xi)) {
            for (int m = 0; m <= n; ++m)
                F[(int64_t)m * ld] = 0.0f;
            continue;
        }
        if (xi > r.z) {
            const double ix = 1.0 / xi;
            double f = r.c0 / sqrt(xi);
            F[0] = (float)f;
            for (int m = 1; m <= n; ++m) {
                f = f * (m - 0.5) * ix;
                F[(int64_t)m * ld] = (float)f;
            }
            continue;
        }
        const float xf = (float)xi;
        const float e = (float)exp_rn(-xi);
        const float u = factors_f(xf, r.ug, r.pug, r.uq, r.puq, r.ul, r.pul);
        const float v = factors_f(xf, r.vg, r.pvg, r.vq, r.pvq, r.vl, r.pvl);
        const float Q = (float)r.q0 + (float)r.q1 * xf + (float)r.q2 * (u / v) * xf * xf;
        const float W = powi_f(Q, n) * sqrtf(Q) * e;
        const float G = xf + W;
        const float t = kappa / G;
        float Fm = powi_f(t, n) * sqrtf(t);
        F[(int64_t)n * ld] = Fm;
        for (int m = n; m >= 1; --m) {
            Fm = (2.0f * xf * Fm + e) * (1.0f / (float)(2 * m - 1));
            F[(int64_t)(m - 1) * ld] = Fm;
        }
    }
    return 0;
}

/* 4. F~_n in binary128 from double-double coefficients                             */
/*
 * recx[] layout: [0] n, then pairs (hi, lo) for q0, q1, q2, then for u and then v:
 *   kg, kg pairs; kq, 2*kq pairs (y, a); kl, kl pairs.
 * c_n is Gamma(n+1/2)/2 computed here in binary128.
 */
static __float128 dd(const double *p)
{
    return (__float128)p[0] + (__float128)p[1];
}

static __float128 factors_q(__float128 x, const double **pp)
{
    const double *p = *pp;
    __float128 r = 1;
    int kg = (int)*p++;
    const double *g = p;
    p += 2 * kg;
    for (int k = kg - 1; k >= 0; --k)
        r = r * x + dd(g + 2 * k);
    int kq = (int)*p++;
    for (int k = 0; k < kq; ++k) {
        const __float128 y = dd(p), a = dd(p + 2);
        p += 4;
        r = r * ((x - y) * (x - y) + a);
    }
    int kl = (int)*p++;
    for (int k = 0; k < kl; ++k) {
        r = r * (x - dd(p));
        p += 2;
    }
    *pp = p;
    return r;
}

int oracle_boys_approx_q(const double *x, int64_t count, const double *recx, double *hi,
                         double *lo)
{
    const int n = (int)recx[0];
    const __float128 s = (__float128)n + 0.5Q;
    __float128 c = sqrtq(M_PIq) / 2;
    for (int j = 0; j < n; ++j)
        c *= (__float128)j + 0.5Q;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        const __float128 xq = (__float128)x[i];
        const double *p = recx + 1;
        const __float128 q0 = dd(p), q1 = dd(p + 2), q2 = dd(p + 4);
        p += 6;
        const __float128 u = factors_q(xq, &p);
        const __float128 v = factors_q(xq, &p);
        const __float128 Q = q0 + q1 * xq + q2 * (u / v) * xq * xq;
        const __float128 W = powq(Q, s) * expq(-xq);
        const __float128 F = c / powq(xq + W, s);
        hi[i] = (double)F;
        lo[i] = (double)(F - (__float128)hi[i]);
    }
    return 0;
}

/* exp(-x) as used by both approximant evaluators, for direct checks */
int oracle_exp_neg(const double *x, int64_t count, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        out[i] = exp_rn(-x[i]);
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* 5. a consumer of F_m: contracted (ss|ss)^(m) auxiliary integrals                 */
/*
 * Two-electron repulsion integrals over s-type Gaussians (the paper's context: the
 * Boys functions are the special functions of Gaussian-basis one- and two-electron
 * integrals).  A primitive pair of exponents a, b at centres A, B is its Gaussian
 * product: p = a + b, P = (a A + b B)/p, and a weight w that carries the contraction
 * coefficients and exp(-ab/p |AB|^2).  For a bra pair (p, P, w_a) and a ket pair
 * (q, Q, w_b), with rho = pq/(p+q) and T = rho |P - Q|^2,
 *     (ss|ss)^(m) = w_a w_b 2 pi^(5/2) / (p q sqrt(p + q)) F_m(T),
 * and a contracted pair sums over its primitive pairs.  The arithmetic, in this order:
 *     pq = p*q;  spq = p+q;  rho = pq/spq;  d = P - Q (per component);
 *     r2 = (dx*dx + dy*dy) + dz*dz;  T = rho*r2;  s = (w_a*w_b) * (K / (pq*sqrt(spq)));
 *     acc_m = acc_m + s*F_m(T)   for bra primitives in order, ket primitives inner,
 * K = 2 pi^(5/2) rounded once to binary64 and F_m the binary64 evaluation above.
 *
 * Pair lists: pairs[k*ldp + j] holds component k = (p, Px, Py, Pz, w) of primitive pair
 * j; contracted pair c owns primitive pairs start[c] .. start[c+1]-1.  out[m*ld + i*nket
 * + j] is the integral of bra contracted pair i with ket contracted pair j.
 */
double oracle_eri_prefactor(void)
{
    return (double)(2.0Q * M_PIq * M_PIq * sqrtq(M_PIq));
}

int oracle_eri_ssss(const double *rec, int reclen, const double *bra, int64_t ldb,
                    const int32_t *bstart, int32_t nbra, const double *ket, int64_t ldk,
                    const int32_t *kstart, int32_t nket, double *out, int64_t ld)
{
    record r;
    if (parse_record(rec, reclen, &r) || nbra < 0 || nket < 0 || ld < (int64_t)nbra * nket)
        return 1;
    const int n = r.n;
    const double K = oracle_eri_prefactor();
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ij = 0; ij < (int64_t)nbra * nket; ++ij) {
        const int32_t i = (int32_t)(ij / nket), j = (int32_t)(ij % nket);
        double acc[64], F[64];
        for (int m = 0; m <= n; ++m)
            acc[m] = 0.0;
        for (int32_t a = bstart[i]; a < bstart[i + 1]; ++a) {
            const double p = bra[a], px = bra[ldb + a], py = bra[2 * ldb + a],
                         pz = bra[3 * ldb + a], wa = bra[4 * ldb + a];
            for (int32_t b = kstart[j]; b < kstart[j + 1]; ++b) {
                const double q = ket[b], qx = ket[ldk + b], qy = ket[2 * ldk + b],
                             qz = ket[3 * ldk + b], wb = ket[4 * ldk + b];
                const double pq = p * q;
                const double spq = p + q;
                const double rho = pq / spq;
                const double dx = px - qx, dy = py - qy, dz = pz - qz;
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double T = rho * r2;
                const double sc = (wa * wb) * (K / (pq * sqrt(spq)));
                approx_one_d(&r, T, F, 1);
                for (int m = 0; m <= n; ++m)
                    acc[m] = fma(sc, F[m], acc[m]);
            }
        }
        for (int m = 0; m <= n; ++m)
            out[(int64_t)m * ld + ij] = acc[m];
    }
    return 0;
}
