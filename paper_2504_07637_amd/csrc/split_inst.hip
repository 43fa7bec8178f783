// split_inst.hip -- the kernels k_split<1..max> of the two-approximation option and their
// launchers.
#include <algorithm>
#include <array>
#include <utility>

#include "boys_kernels.h"

namespace {

template <int N>
hipError_t launch_split(const double *x, int64_t n, double *out, int64_t ld, int nbar,
                        hipStream_t s)
{
    if constexpr (N == 0) {
        return hipErrorInvalidValue;  // no order below 0
    } else {
        constexpr int kBlock = 128;
        constexpr int64_t kChunk = (int64_t)INT32_MAX / kBlock * kBlock;
        for (int64_t off = 0; off < n; off += kChunk) {
            const int64_t cnt = std::min(kChunk, n - off);
            const int grid = (int)((cnt + kBlock - 1) / kBlock);
            hipLaunchKernelGGL((k_split<N>), dim3(grid), dim3(kBlock), 0, s, x + off, cnt,
                               out + off, ld, nbar);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
}

template <int... Ns>
constexpr std::array<boys_internal::SplitLaunch, sizeof...(Ns)>
split_table(std::integer_sequence<int, Ns...>)
{
    return {&launch_split<Ns>...};
}

}  // namespace

boys_internal::SplitLaunch boys_internal::split_launcher(int n)
{
    static constexpr auto kTable = split_table(std::make_integer_sequence<int, kMaxN64 + 1>{});
    return n >= 1 && n <= kMaxN64 ? kTable[n] : nullptr;
}
