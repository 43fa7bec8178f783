// A standalone driver of the serving policy core for sanitizer builds: the pool fuzz and a
// simulated Poisson stream, run under AddressSanitizer and UndefinedBehaviorSanitizer by
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
    std::printf("ok: %d requests, %d batches\n", done, nb);
    return 0;
}
