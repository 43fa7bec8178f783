/*
 * boys.h -- C ABI of libboys.so: bulk evaluation of the Boys functions on MI355X (gfx950).
 *
 * The Boys function of order m is F_m(x) = int_0^1 t^(2m) exp(-x t^2) dt, x >= 0
 * (Laikov, arXiv 2504.07637, section "Introduction", Eq. fn).  The library evaluates
 * F_m(x) for m = 0..n_max over arrays of arguments with the paper's global closed form
 * (section "Methodology"):
 *
 *     F_n(x) = c_n / (x + Q~_n(x)^(n+1/2) exp(-x))^(n+1/2)             (Eq. fq)
 *     Q~_n(x) = q0 + q1 x + q2 x^2 u_n(x) / v_n(x)                      (Eqs. pqz, pz, qz)
 *     F_{m-1}(x) = (2x F_m(x) + exp(-x)) / (2m-1),  m = n..1             (Eq. r)
 *     F_m(x) = c_m / x^(m+1/2) for x > z_nb                              (Eq. limf1, cut-off)
 *
 * with n = n_max and one exp(-x) shared by Eq. fq and Eq. r.  (The paper prints the
 * divisor of Eq. r as 2m+1; integration by parts of Eq. fn gives 2m-1.)
 *
 * Conventions for every entry point:
 *   - Pointers named x / out, and the arrays a boys_pair_list points to, are DEVICE
 *     pointers (memory of the current HIP device); all other pointers are host pointers.  The caller owns all of them; the library
 *     never frees or retains them beyond the call (plans keep the pointers they were
 *     given until updated or destroyed).
 *   - x is binary64, contiguous, n elements.
 *   - out holds (n_max + 1) rows of ld_out elements: F_m(x[i]) is at out[m * ld_out + i]
 *     (structure of arrays), binary64 for BOYS_FP64 / BOYS_FP64_PLUS and binary32 for
 *     BOYS_FP32 / BOYS_FP32X / BOYS_FP32_SINGLE.
 *     Requires ld_out >= n.  Alignment: 8 bytes (FP64) or 4 bytes (FP32).  Rows that
 *     start on 128-byte boundaries (out 128-byte aligned and ld_out a multiple of 16
 *     binary64 / 32 binary32 elements) are written as whole cache lines; other strides
 *     work but cost up to a third of the store bandwidth.
 *   - stream is a hipStream_t (NULL = the null stream).  Calls only enqueue work and
 *     return; results are ready when the stream reaches them.
 *   - Inputs outside x >= 0: x < 0 or NaN gives NaN for every m; x = +inf gives 0.
 *     x = -0.0 is treated as 0.
 *   - Argument errors are detected on the host and returned before anything is
 *     enqueued.  A failed kernel launch is reported as BOYS_ERR_DEVICE.  No C++
 *     exception crosses this interface.  n == 0 is a successful no-op.
 *   - Entry points are reentrant; a plan object must not be used from two threads at once.
 */
#ifndef BOYS_H
#define BOYS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    /* binary64 throughout; output binary64 */
    BOYS_FP64 = 0,
    /* mixed class: u/v, Q~ and the power Q~^(n+1/2) and the recursion in binary32,
       x + W and c_n / G^(n+1/2) in binary64 (the power whose rounding error is
       amplified by n+1/2); output binary32 */
    BOYS_FP32 = 1,
    /* binary64 with the option of section "Computations" for a few more bits in F_n:
       the order n_max+1 approximant (and its cut-off z_{n_max+1,53}) gives F_{n_max+1},
       one more step of Eq. r gives F_{n_max}, which is not stored; output binary64
       (F_{n_max} gains about 3 bits at n_max >= 16); n_max <= boys_max_nmax - 1 */
    BOYS_FP64_PLUS = 2,
    /* binary32 output at full single-precision accuracy, as the paper suggests for it:
       binary64 arithmetic throughout with approximants fitted to about 28 bits (the
       smallest N per n reaching 28 bits) and the cut-off z_{n_max,28}; each value is
       rounded once to binary32 at the store, so its error is within half a binary32 ulp
       plus 2^-28 relative (subnormal outputs: plus half the subnormal spacing) */
    BOYS_FP32X = 3,
    /* all binary32 below the cut-off: the arithmetic of Table 1's binary32 columns, with
       the binary32 sets, G = x + W in binary32 and F_n = (kappa_n / G)^(n+1/2), kappa_n =
       c_n^(1/(n+1/2)) rounded to binary32 (c_n itself leaves the binary32 range beyond
       n = 27); past the cut-off the long-range limit as BOYS_FP32; output binary32 */
    BOYS_FP32_SINGLE = 4
} boys_precision;

typedef enum {
    BOYS_OK = 0,
    BOYS_ERR_INVALID_ARGUMENT = 1, /* null pointer with n > 0, ld_out < n, bad precision, count < 0 */
    BOYS_ERR_UNSUPPORTED_NMAX = 2, /* n_max < 0 or n_max > boys_max_nmax(precision) */
    BOYS_ERR_OUT_OF_MEMORY = 3,    /* a plan or batch could not get its device buffers */
    BOYS_ERR_DEVICE = 4,           /* a HIP call or kernel launch failed */
    BOYS_ERR_TOO_LARGE = 5         /* the batch's tables exceed the fixed scratch array of
                                      boys_eval_batched_noalloc */
} boys_status;

/*
 * Evaluate F_m(x[i]) for m = 0..n_max and i = 0..n-1 into out (layout above).
 * precision is a boys_precision value.  The approximant of order n_max is used
 * (coefficient set fitted for that n and that precision class, with the cut-off
 * z_{n_max,b}, b = 53 for BOYS_FP64, 24 for BOYS_FP32 and BOYS_FP32_SINGLE, 28 for BOYS_FP32X), and the lower orders come
 * from the downward recursion of Eq. r below the cut-off and from Eq. limf1 above it.
 */
boys_status boys_eval(const double *x, int64_t n, int32_t n_max, void *out, int64_t ld_out,
                      int32_t precision, void *stream);

/*
 * The evaluation of boys_eval, storing only some of the orders: bit m of rows (m = 0..n_max)
 * selects F_m, and the k-th selected order, counting upward from m = 0, is written to
 * out[k * ld_out + i] (k = 0..popcount(rows)-1; row layout and element type as boys_eval).
 * Every order is still computed in full (the recursion of Eq. r and the upward product of
 * Eq. limf1 pass through all of them), so each stored value equals, bit for bit, the one
 * boys_eval stores for that order.  For consumers that need a few orders, and to measure the
 * arithmetic without the full (n_max+1)-row store.  BOYS_ERR_INVALID_ARGUMENT when rows is 0
 * or selects an order above n_max; other errors as boys_eval (with ld_out >= n).
 */
boys_status boys_eval_rows(const double *x, int64_t n, int32_t n_max, uint64_t rows, void *out,
                           int64_t ld_out, int32_t precision, void *stream);

/*
 * The two-approximation option of section "Computations", binary64: when the highest
 * accuracy is wanted for the orders m = 0..n_bar, F_{n_bar} and F_{n_max} are both taken
 * from their own best approximants (cut-offs z_{n_bar,53} and z_{n_max,53}) and two
 * downward recursions of Eq. r run, from n_max to n_bar+1 and from n_bar to 0, with one
 * exp(-x).  Rows 0..n_bar equal boys_eval(..., n_bar, BOYS_FP64) bit for bit and rows
 * n_bar+1..n_max equal those of boys_eval(..., n_max, BOYS_FP64).  Output binary64, layout
 * and conventions as boys_eval.  Requires 0 <= n_bar < n_max <= boys_max_nmax(BOYS_FP64)
 * (BOYS_ERR_UNSUPPORTED_NMAX otherwise).
 */
boys_status boys_eval_split(const double *x, int64_t n, int32_t n_bar, int32_t n_max, void *out,
                            int64_t ld_out, void *stream);

/*
 * A consumer of F_m that never stores them: the contracted (ss|ss)^(m) auxiliary
 * two-electron integrals over s-type Gaussian functions, the application the paper names
 * for the Boys functions (section "Introduction"), with x formed on the device.
 *
 * A primitive pair of Gaussians (exponents a, b at centres A, B) enters as its product:
 * p = a + b, P = (a A + b B)/p and a weight w (contraction coefficients times
 * exp(-ab/p |AB|^2)).  For a bra pair (p, P, w_a) and a ket pair (q, Q, w_b), with
 * rho = pq/(p+q) and T = rho |P - Q|^2,
 *     (ss|ss)^(m) = w_a w_b 2 pi^(5/2) / (p q sqrt(p+q)) F_m(T),   m = 0..n_max,
 * with F_m the BOYS_FP64 evaluation of order n_max; a contracted pair sums over its
 * primitive pairs, bra primitives outer and ket primitives inner, in the order below:
 *     pq = p*q; spq = p+q; rho = pq/spq; d = P - Q; r2 = (dx*dx + dy*dy) + dz*dz;
 *     T = rho*r2; s = (w_a*w_b) * (K / (pq*sqrt(spq))); acc_m = fma(s, F_m(T), acc_m),
 * K = 2 pi^(5/2) rounded to binary64 and fma one correctly rounded multiply-add.  Each
 * output is a plain sequential sum, so results are reproducible bit for bit.
 */
typedef struct {
    const double *p;       /* device: exponent sums p of the primitive pairs            */
    const double *px;      /* device: product centres P, x component                    */
    const double *py;      /* device: y component                                       */
    const double *pz;      /* device: z component                                       */
    const double *w;       /* device: weights                                           */
    const int32_t *start;  /* device, count+1 entries: contracted pair c owns primitive
                              pairs start[c] .. start[c+1]-1 (non-decreasing, start[0] >= 0;
                              the caller guarantees it, the library cannot check device data) */
    int32_t count;         /* contracted pairs in the list (>= 0)                       */
} boys_pair_list;

/*
 * out[m * ld_out + i * ket->count + j] = the contracted (ss|ss)^(m) of bra contracted pair
 * i and ket contracted pair j, m = 0..n_max (binary64; out is a device pointer).
 * Requires ld_out >= bra->count * ket->count, 0 <= n_max <= boys_max_nmax(BOYS_FP64).
 * Empty lists are a no-op.  BOYS_ERR_INVALID_ARGUMENT for null lists or pointers, negative
 * counts or a short ld_out; BOYS_ERR_UNSUPPORTED_NMAX for n_max out of range.
 */
boys_status boys_eri_ssss(const boys_pair_list *bra, const boys_pair_list *ket, int32_t n_max,
                          double *out, int64_t ld_out, void *stream);

/* One argument array of a batch (host struct; x and out are device pointers). */
typedef struct {
    const double *x;
    void *out;
    int64_t n;
    int64_t ld_out;
    int32_t n_max;
    int32_t precision;
} boys_array;

/*
 * Launch parameters of a batched launch (0 in tile/block/grid_per_cu = library default).
 * schedule 0: persistent waves: grid_per_cu resident workgroups per compute unit (at
 *             least 8 in all) whose waves each take 256-argument tiles (tile must be 256)
 *             from one of 8 work counters, the tile list dealt round-robin to the 8;
 * schedule 1: one workgroup per tile, dispatched by the hardware in table order;
 *             tile must be block x 1, 2 or 4.
 * schedule 2: one wave per tile (tile = 256, i.e. 64 lanes x 4 arguments; a block of
 *             64, 128 or 256 holds block / 64 tiles), so one workgroup can serve several
 *             short arrays.  With split_nmax > 0 the store-bound arrays, those with
 *             n_max >= split_nmax (binary64 outputs) or n_max >= split_nmax + 4 (binary32
 *             outputs), run first in a launch of their own with one workgroup of 256
 *             threads per 256-argument tile (one argument per lane); the plan's graph holds
 *             both launches.
 */
typedef struct {
    int32_t tile;        /* arguments per tile: schedule 1 block x 1, 2 or 4; 0 and 2: 256 */
    int32_t block;       /* threads per workgroup: 64, 128 or 256 */
    int32_t grid_per_cu; /* schedule 0: persistent workgroups per compute unit (1..64) */
    int32_t schedule;    /* 0, 1 or 2 (above) */
    int32_t order;       /* tile order: 0 longest first; 1 array by array (each array's
                            tiles consecutive); 2 grouped by (precision, n_max), then
                            array by array */
    int32_t split_nmax;  /* schedule 2: 0 (one launch) or 1..64 (above); must be 0 for
                            schedules 0 and 1 */
} boys_tuning;

/*
 * Evaluate every array of a batch in one batched launch.  Results equal, bit
 * for bit, those of boys_eval on each array alone.  arrays is a host array of count
 * entries.  Builds a temporary schedule (device buffers allocated and freed inside the
 * call, synchronising stream before the free); use a plan for repeated batches.
 */
boys_status boys_eval_batched(const boys_array *arrays, int32_t count, void *stream);

/*
 * boys_eval_batched without any allocation, for callers that cannot allocate device
 * memory (allocation-free serving loops, harnesses that forbid hipMalloc): the same
 * kernels, the same default schedule and results equal bit for bit to those of
 * boys_eval_batched, with the descriptor and tile tables in a fixed device array of the
 * library (BOYS_NOALLOC_SCRATCH_BYTES per device, held until the process ends) instead of
 * buffers allocated per call.  No hipMalloc, hipFree or other allocating call is made.
 * Limit: 256 + 40 * count bytes (rounded up to 256) + 8 bytes per 256-argument tile of
 * every array must fit in the array (about 2.6e8 arguments in total for a few thousand
 * arrays); larger batches return BOYS_ERR_TOO_LARGE before anything is enqueued.
 * The call uploads the tables on stream from a static host staging area, enqueues the
 * kernels and synchronises stream before it returns (work already on stream is waited
 * for too).  The library serialises these calls (one staging area, one array per device,
 * each call overwriting the previous call's tables), so calls from several threads do
 * not race but do not overlap either.  Not usable under stream capture (it synchronises).
 */
#define BOYS_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
boys_status boys_eval_batched_noalloc(const boys_array *arrays, int32_t count, void *stream);

/*
 * Plans: a schedule (tiles in the tuning's order, descriptor and tile tables in
 * device memory, the work counters of schedule 0) and a HIP graph of the batched launch
 * (schedule 0: [reset counters, persistent kernel]; schedule 1: [one workgroup per
 * tile]; schedule 2: [one wave per tile], after [one workgroup per tile] for the
 * store-bound arrays of a split plan) built once for a batch and replayed by boys_plan_execute.  tuning may be
 * NULL for the defaults: schedule 2, tile 256, block 256, order 1, split_nmax 0.
 * boys_eval_batched uses the defaults.  boys_plan_update replaces the x/out pointers of a
 * batch with the same count, lengths, n_max and precisions (other changes return
 * BOYS_ERR_INVALID_ARGUMENT); it first waits for every execute of the plan already
 * enqueued (on any stream) to finish, so executes enqueued before it use the old pointers
 * and executes enqueued after it returns use the new ones.  boys_plan_destroy also waits
 * for the plan's enqueued executes.  A plan belongs to the device that was current at
 * creation.
 */
typedef struct boys_plan boys_plan;
boys_status boys_plan_create(boys_plan **plan, const boys_array *arrays, int32_t count,
                             const boys_tuning *tuning);
boys_status boys_plan_update(boys_plan *plan, const boys_array *arrays, int32_t count);
boys_status boys_plan_execute(boys_plan *plan, void *stream);
void boys_plan_destroy(boys_plan *plan);

/*
 * Autotuner: times plan execution for each of ncand candidate tunings on the given
 * batch (each candidate executed warmup + reps times on stream, timed with HIP events)
 * and writes the fastest into *best and, if times_ms is not NULL, the mean time of each
 * candidate.  The arrays' out buffers are overwritten.
 */
boys_status boys_autotune(const boys_array *arrays, int32_t count, const boys_tuning *candidates,
                          int32_t ncand, int32_t warmup, int32_t reps, void *stream,
                          boys_tuning *best, float *times_ms);

/*
 * Serving loop.  A server owns one device allocation of budget_bytes and a scheduler
 * thread.  Each request is one argument array (host memory; pinned memory gives truly
 * asynchronous copies), evaluated as by boys_eval into device memory owned by the server:
 *   - requests are admitted in arrival order while their footprint (n*8 bytes for x plus
 *     (n_max+1)*ld*{8,4} bytes of output, each rounded up to 256 bytes) fits the budget;
 *     one that does not fit waits until releases free enough memory;
 *   - admitted requests are launched at the next opportunity: whenever one of the
 *     `streams` execution slots is free, every admitted request not yet launched (up to
 *     max_batch, and up to max_tiles tiles of `tile` arguments) goes out as one batched
 *     launch on that slot's stream; batches on different slots overlap
 *     (continuous batching);
 *   - a request completes when its batch's event completes; its output stays in device
 *     memory until boys_server_release (rows of ld elements, ld = n rounded up to a
 *     multiple of 16 binary64 / 32 binary32 elements);
 *   - a request fails, instead, when its batch could not be launched (the server then
 *     waits for whatever part of the batch it had enqueued) or its completion event
 *     reports a device error.  Failed requests are reported by boys_server_poll like
 *     completed ones; boys_server_result and boys_server_copy_result return
 *     BOYS_ERR_DEVICE for them, and they are released like completed ones.  A failed
 *     batch is not retried.
 * Times are seconds on the server's monotonic clock.  x_host must stay valid and
 * unchanged until the request completes.  All functions are thread-safe.
 */
typedef struct boys_server boys_server;
typedef struct {
    int64_t budget_bytes; /* device memory for admitted requests (inputs + outputs) */
    int32_t streams;      /* execution slots, one HIP stream each (0 = 4) */
    int32_t max_batch;    /* requests per launch (0 = 256) */
    int32_t tile;         /* arguments per tile: 256, 512 or 1024 (0 = 256); one
                             256-thread workgroup per tile */
    int32_t max_tiles;    /* tiles per launch (0 = 65536); larger requests are refused */
} boys_server_config;
typedef struct {
    uint64_t submitted, admitted, launched, completed, released, batches;
    uint64_t queued_now, inflight_now, max_queued, max_inflight;
    uint64_t bytes_in_use, max_bytes_in_use;
    uint64_t device_errors;
    uint64_t failed;      /* requests that failed (also counted in completed) */
} boys_server_stats;
/* cfg is a host struct; the server is bound to the device current at creation. */
boys_status boys_server_create(boys_server **server, const boys_server_config *cfg);
/* BOYS_ERR_OUT_OF_MEMORY: the request can never fit (larger than the budget or the
   per-launch tile capacity); BOYS_ERR_INVALID_ARGUMENT: n <= 0, null x_host, bad
   precision; BOYS_ERR_UNSUPPORTED_NMAX as for boys_eval. */
boys_status boys_server_submit(boys_server *server, const double *x_host, int64_t n,
                               int32_t n_max, int32_t precision, uint64_t *id);
/* Writes up to max ids of requests completed since the last poll; returns their count. */
int32_t boys_server_poll(boys_server *server, uint64_t *ids, int32_t max);
/* For a completed, unreleased request: device pointer of its output rows, their leading
   dimension, and its submit and completion times (BOYS_ERR_DEVICE for a failed request).
   A client that reads the rows through this pointer with work of its own must have
   finished those reads (for example, synchronised their stream) before it releases the
   request; reads through boys_server_copy_result are tracked by the server. */
boys_status boys_server_result(boys_server *server, uint64_t id, const void **out,
                               int64_t *ld, double *t_submit, double *t_done);
/* Copies a completed, unreleased request's (n_max+1) output rows into the device buffer
   dst (row stride ld_dst >= n elements of the request's precision), enqueued on stream
   (BOYS_ERR_DEVICE for a failed request).  The request may be released right after the
   call: the server records an event on stream behind the copy and keeps the request's
   memory until that event has completed. */
boys_status boys_server_copy_result(boys_server *server, uint64_t id, void *dst, int64_t ld_dst,
                                    void *stream);
/* Releases a completed or failed request: its output pointer becomes invalid, and its
   device memory is freed once the copies enqueued by boys_server_copy_result are done. */
boys_status boys_server_release(boys_server *server, uint64_t id);
boys_status boys_server_get_stats(boys_server *server, boys_server_stats *stats);
/* Waits until no admitted request is waiting for a slot or running and the queue is
   empty or its head does not fit the free memory.  Requests still queued for memory stay
   queued: only releases of completed requests can admit them, so a client that holds
   results must keep polling and releasing (BOYS_ERR_DEVICE on timeout or after a device
   error). */
boys_status boys_server_drain(boys_server *server, double timeout_s);
/* Stops the scheduler, waits for the streams and frees everything. */
void boys_server_destroy(boys_server *server);

/* Largest supported n_max for a precision class (-1 for an unknown class). */
int32_t boys_max_nmax(int32_t precision);

/* The cut-off z_nb used for n_max = n in a precision class (NaN if unsupported). */
double boys_cutoff(int32_t n, int32_t precision);

/* Static description of a status code. */
const char *boys_status_string(boys_status status);

#ifdef __cplusplus
}
#endif

#endif /* BOYS_H */
