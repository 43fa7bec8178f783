// boys_noalloc.hip -- boys_eval_batched_noalloc: the batched evaluation of
// boys_eval_batched for callers that cannot allocate device memory.
//
// boys_eval_batched builds a temporary plan: its descriptor and tile tables live in
// device buffers it allocates and frees inside the call.  This entry point runs the same
// kernels with the same default schedule (one wave per 256-argument tile, array by array,
// in one launch) on tables placed in a
// fixed device array of this file, `scratch`, so it calls no hipMalloc or hipFree.
//
// Per device, the first call with that device current looks up the array's device
// address once (hipGetSymbolAddress); the host name of a __device__ array is only a
// host-side stand-in, so kernels and copies are given that looked-up address.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "boys.h"
#include "boys_internal.h"

namespace {

using boys_internal::Desc;

constexpr size_t kScratchBytes = size_t(8) << 20;  // BOYS_NOALLOC_SCRATCH_BYTES in boys.h
constexpr int kTile = 256;                         // arguments per tile
constexpr size_t kDescOff = 256;

static_assert(BOYS_NOALLOC_SCRATCH_BYTES == kScratchBytes, "boys.h states the scratch size");

}  // namespace

// the tables of one call: descriptors at kDescOff, then the tile list
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
unsigned char *g_ptr[kMaxDevices];  // the device address of scratch, per device
hipError_t g_err[kMaxDevices];

// host staging of the tables (static, so a call allocates no host memory either); one
// call at a time uses it, and with it the device array of its device
alignas(256) unsigned char g_host[kScratchBytes];
std::mutex g_mu;

unsigned char *scratch_ptr(int dev)
{
    std::call_once(g_once[dev], [dev] {
        void *p = nullptr;
        g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_err[dev] == hipSuccess ? static_cast<unsigned char *>(p) : nullptr;
    });
    return g_ptr[dev];
}

}  // namespace

extern "C" boys_status boys_eval_batched_noalloc(const boys_array *arrays, int32_t count,
                                                 void *stream)
{
    if (count < 0 || (count > 0 && arrays == nullptr))
        return BOYS_ERR_INVALID_ARGUMENT;
    // the same argument checks as every batched entry point (boys_eval on each array)
    for (int32_t a = 0; a < count; ++a) {
        const boys_array &A = arrays[a];
        const int32_t mx = boys_max_nmax(A.precision);
        if (mx < 0 || A.n < 0)
            return BOYS_ERR_INVALID_ARGUMENT;
        if (A.n_max < 0 || A.n_max > mx)
            return BOYS_ERR_UNSUPPORTED_NMAX;
        if (A.n > 0 && (A.x == nullptr || A.out == nullptr || A.ld_out < A.n ||
                        A.ld_out > INT64_MAX / 8 / (int64_t)(A.n_max + 1)))
            return BOYS_ERR_INVALID_ARGUMENT;
    }
    // table sizes against the fixed array
    int64_t ntiles = 0;
    int maxn = 0;
    for (int32_t a = 0; a < count; ++a) {
        const int64_t t = (arrays[a].n + kTile - 1) / kTile;
        ntiles += t;
        if (t > 0)
            maxn = std::max(maxn, (int)arrays[a].n_max);
        if (ntiles > INT32_MAX)
            return BOYS_ERR_TOO_LARGE;
    }
    const size_t tiles_off = (kDescOff + sizeof(Desc) * (size_t)count + 255) / 256 * 256;
    if ((size_t)count > kScratchBytes / sizeof(Desc) ||
        tiles_off + sizeof(int2) * (size_t)ntiles > kScratchBytes)
        return BOYS_ERR_TOO_LARGE;
    if (ntiles == 0)
        return BOYS_OK;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return BOYS_ERR_DEVICE;
    unsigned char *base = scratch_ptr(dev);
    if (base == nullptr)
        return BOYS_ERR_DEVICE;

    std::lock_guard<std::mutex> lock(g_mu);
    // descriptors, then the tiles, each array's consecutive (the order of boys_eval_batched's
    // default schedule)
    Desc *hd = reinterpret_cast<Desc *>(g_host + kDescOff);
    for (int32_t a = 0; a < count; ++a) {
        const boys_array &A = arrays[a];
        hd[a] = Desc{A.x, A.out, A.n, A.ld_out, A.n_max, A.precision};
    }
    int2 *ht = reinterpret_cast<int2 *>(g_host + tiles_off);
    int64_t k = 0;
    for (int32_t a = 0; a < count; ++a) {
        const int64_t t = (arrays[a].n + kTile - 1) / kTile;
        for (int64_t s = 0; s < t; ++s)
            ht[k++] = make_int2(a, (int32_t)s);
    }
    const size_t used = tiles_off + sizeof(int2) * (size_t)ntiles - kDescOff;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const Desc *d_desc = reinterpret_cast<const Desc *>(base + kDescOff);
    const int2 *d_tiles = reinterpret_cast<const int2 *>(base + tiles_off);
    if (hipMemcpyAsync(base + kDescOff, g_host + kDescOff, used, hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return BOYS_ERR_DEVICE;
    // schedule 2 uses no work counter
    boys_status st = BOYS_OK;
    if (boys_internal::launch_batched(d_desc, d_tiles, (int32_t)ntiles, nullptr, maxn,
                                      boys_internal::Launch{2, kTile, 256, 0}, s) != hipSuccess)
        st = BOYS_ERR_DEVICE;
    // whatever was enqueued must have read the tables before the next call rewrites them
    if (hipStreamSynchronize(s) != hipSuccess)
        st = BOYS_ERR_DEVICE;
    return st;
}
