// plain_inst.hip -- the plain kernels k_plain<C, 0..max, Sel> of one precision class C and
// their launchers (Sel: the row-selecting form of boys_eval_rows).  Compiled once per class
// with -DBOYS_CLASS=<boys_precision value>.
#include <algorithm>
#include <array>
#include <type_traits>
#include <utility>

#include "boys_kernels.h"

#ifndef BOYS_CLASS
#error "compile with -DBOYS_CLASS=<precision class>"
#endif

namespace {

template <int C, int N, bool Sel>
hipError_t launch_plain(const double *x, int64_t n, void *out, int64_t ld, uint64_t rows,
                        hipStream_t s)
{
    constexpr int kBlock = plain_block<C>();
    constexpr int64_t kChunk = (int64_t)INT32_MAX / kBlock * kBlock;  // one grid's worth
    using T = std::conditional_t<C == BOYS_FP32 || C == BOYS_FP32X || C == BOYS_FP32_SINGLE,
                                 float, double>;
    for (int64_t off = 0; off < n; off += kChunk) {
        const int64_t cnt = std::min(kChunk, n - off);
        const int grid = (int)((cnt + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((k_plain<C, N, Sel>), dim3(grid), dim3(kBlock), 0, s, x + off, cnt,
                           static_cast<void *>(static_cast<T *>(out) + off), ld, rows);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <int C, bool Sel, int... Ns>
constexpr std::array<boys_internal::PlainLaunch, sizeof...(Ns)>
plain_table(std::integer_sequence<int, Ns...>)
{
    return {&launch_plain<C, Ns, Sel>...};
}

}  // namespace

template <int C>
boys_internal::PlainLaunch boys_internal::plain_launcher(int n, bool select_rows)
{
    static constexpr auto kAll =
        plain_table<C, false>(std::make_integer_sequence<int, class_max<C>() + 1>{});
    static constexpr auto kSel =
        plain_table<C, true>(std::make_integer_sequence<int, class_max<C>() + 1>{});
    if (n < 0 || n > class_max<C>())
        return nullptr;
    return select_rows ? kSel[n] : kAll[n];
}

template boys_internal::PlainLaunch boys_internal::plain_launcher<BOYS_CLASS>(int n, bool);
