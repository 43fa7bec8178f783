// A standalone driver of the serving policy core for sanitizer builds: the pool fuzz, a
// simulated Poisson stream, injected launch and completion failures and a release under a
// pending read, run under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_serve_core.py.  Exit status 0 when every check passes.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" int pool_fuzz(uint64_t seed, int ops, uint64_t capacity);
extern "C" int sim_run(int nreq, const double *t_arr, const int64_t *len, const int *nmax,
                       const int *prec, int64_t budget, int slots, int max_batch, double bw,
                       double dt, double *t_admit, double *t_launch, double *t_done, int *slot,
                       int *rc, int64_t *max_in_use, int *max_inflight, int *max_concurrent,
                       int *batches);
extern "C" int sim_failures(int nreq, int64_t n, int slots, int max_batch,
                            const int *fail_launch, int nfl, const int *fail_done, int nfd,
                            int *state_out, int *reports_out, int *failed_stat);
extern "C" int sim_pending_read(int64_t n, double t_read, double *t_admit_b,
                                uint64_t *in_use_after_release, int *tokens_freed);

int main()
{
    for (uint64_t seed = 0; seed < 4; ++seed)
        if (pool_fuzz(seed, 20000, 1ull << 30) != 0) {
            std::printf("pool_fuzz failed for seed %llu\n", (unsigned long long)seed);
            return 1;
        }
    const int n = 3000;
    std::mt19937_64 g(7);
    std::exponential_distribution<double> gap(20000.0);
    std::uniform_real_distribution<double> u(std::log(64.0), std::log(262144.0));
    std::vector<double> t(n), ta(n), tl(n), td(n);
    std::vector<int64_t> len(n);
    std::vector<int> nm(n), pr(n), sl(n), rc(n);
    double now = 0.0;
    for (int i = 0; i < n; ++i) {
        now += gap(g);
        t[i] = now;
        len[i] = (int64_t)std::llround(std::exp(u(g)));
        nm[i] = (int)(g() % 21);
        pr[i] = (int)(g() % 5);
    }
    int64_t mu = 0;
    int mi = 0, mc = 0, nb = 0;
    const int done = sim_run(n, t.data(), len.data(), nm.data(), pr.data(), 64ll << 20, 4, 256,
                             3e10, 2e-6, ta.data(), tl.data(), td.data(), sl.data(), rc.data(),
                             &mu, &mi, &mc, &nb);
    if (done != n || mu > (64ll << 20)) {
        std::printf("sim_run: %d of %d done, max in use %lld\n", done, n, (long long)mu);
        return 1;
    }
    const int fl[] = {0, 3, 9}, fd[] = {1, 5, 6};
    std::vector<int> st(200), rep(200);
    int failed = 0;
    for (int64_t len : {1000LL, 3000000LL}) {
        const int launches = sim_failures(200, len, 3, 8, fl, 3, fd, 3, st.data(), rep.data(),
                                          &failed);
        if (launches < 0 || failed <= 0) {
            std::printf("sim_failures: %d (n = %lld)\n", launches, (long long)len);
            return 1;
        }
    }
    double tb = 0;
    uint64_t in_use = 0;
    int freed = 0;
    const int prc = sim_pending_read(100000, 0.01, &tb, &in_use, &freed);
    if (prc != 0 || tb < 0.01 || freed != 2) {
        std::printf("sim_pending_read: %d, admit %g, freed %d\n", prc, tb, freed);
        return 1;
    }
    std::printf("ok: %d requests, %d batches\n", done, nb);
    return 0;
}
