// fd_probe.hip -- STREAM-style triad a = b + s c: the measured bandwidth
// ceiling of section 3.1 (STREAM TRIAD as the practical limit), and a kernel
// of exactly known traffic (8 bytes read + 4 written per element) for
// calibrating hardware byte counters.
#include "fd.h"
#include "fd_internal.h"

namespace fd {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void triad_kernel(v4f* __restrict__ a,
                                                    const v4f* __restrict__ b,
                                                    const v4f* __restrict__ c, float s,
                                                    int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * 256) {
        const v4f x = __builtin_nontemporal_load(b + i);
        const v4f y = __builtin_nontemporal_load(c + i);
        v4f r;
        r.x = fmaf(s, y.x, x.x);
        r.y = fmaf(s, y.y, x.y);
        r.z = fmaf(s, y.z, x.z);
        r.w = fmaf(s, y.w, x.w);
        __builtin_nontemporal_store(r, a + i);
    }
}

__global__ void triad_tail(float* a, const float* b, const float* c, float s, int64_t from,
                           int64_t n) {
    const int64_t i = from + threadIdx.x;
    if (i < n) a[i] = fmaf(s, c[i], b[i]);
}

}  // namespace
}  // namespace fd

extern "C" int32_t fd_triad(float* a, const float* b, const float* c, float s, int64_t n,
                            void* stream) {
    if (!a || !b || !c || n < 0) return FD_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
         reinterpret_cast<uintptr_t>(c)) % 16)
        return FD_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n4 = n / 4;
    if (n4 > 0) {
        // 8 blocks per CU on 256 CUs, grid-stride
        hipLaunchKernelGGL(fd::triad_kernel, dim3(2048), dim3(256), 0, st,
                           reinterpret_cast<fd::v4f*>(a), reinterpret_cast<const fd::v4f*>(b),
                           reinterpret_cast<const fd::v4f*>(c), s, n4);
    }
    if (n4 * 4 < n)
        hipLaunchKernelGGL(fd::triad_tail, dim3(1), dim3(64), 0, st, a, b, c, s, n4 * 4, n);
    return hipGetLastError() == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}
