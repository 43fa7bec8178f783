// eri_inst.hip -- the consumer kernels k_eri_ssss<0..max> and their launchers.
#include <array>
#include <utility>

#include "boys_eri.h"

namespace {

template <int N>
hipError_t launch_eri(const PairList &bra, const PairList &ket, double K, double *out, int64_t ld,
                      hipStream_t s)
{
    const int64_t total = (int64_t)bra.count * ket.count;
    const int64_t grid = (total + kEriBlock - 1) / kEriBlock;
    if (grid > INT32_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_eri_ssss<N>), dim3((unsigned)grid), dim3(kEriBlock), 0, s, bra, ket,
                       K, out, ld);
    return hipGetLastError();
}

using EriLaunch = hipError_t (*)(const PairList &, const PairList &, double, double *, int64_t,
                                 hipStream_t);

template <int... Ns>
constexpr std::array<EriLaunch, sizeof...(Ns)> eri_table(std::integer_sequence<int, Ns...>)
{
    return {&launch_eri<Ns>...};
}

PairList pair_list(const boys_pair_list &l)
{
    return PairList{l.p, l.px, l.py, l.pz, l.w, l.start, l.count};
}

}  // namespace

hipError_t boys_internal::launch_eri_ssss(const boys_pair_list &bra, const boys_pair_list &ket,
                                          int n_max, double *out, int64_t ld, hipStream_t s)
{
    static constexpr auto kTable = eri_table(std::make_integer_sequence<int, kMaxN64 + 1>{});
    if (n_max < 0 || n_max > kMaxN64)
        return hipErrorInvalidValue;
    return kTable[n_max](pair_list(bra), pair_list(ket), boys_tab::kTwoPi52, out, ld, s);
}
