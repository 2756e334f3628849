// fd_probe.hip -- STREAM-style triad a = b + s c: the measured bandwidth
// ceiling of section 3.1 (STREAM TRIAD as the practical limit), and a kernel
// of exactly known traffic (8 bytes read + 4 written per element) for
// calibrating hardware byte counters.
//
// Each thread moves U 16-byte vectors of every array per iteration: a wave
// reads U whole kilobytes of b and of c before it computes, so that enough
// bytes are in flight to cover HBM latency.  The grid either gives every
// block one chunk of 256 U vectors (blocks = 0) or a fixed number of blocks
// strides over the chunks; loads and stores are non-temporal unless the
// caller asks for ordinary ones.
#include "fd.h"
#include "fd_internal.h"

namespace fd {
namespace {

// fd_triad's configuration (the best of the measured sweep).
constexpr int kTriadUnroll = 1;
constexpr int kTriadBlocks = 0;

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ v4f ld(const v4f* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT>
__device__ __forceinline__ void st(v4f* p, v4f v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int U, bool NT>
__global__ __launch_bounds__(256) void triad_kernel(v4f* __restrict__ a,
                                                    const v4f* __restrict__ b,
                                                    const v4f* __restrict__ c, float s,
                                                    int64_t n4, int64_t chunks) {
    for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int64_t i0 = ch * (256 * U) + threadIdx.x;
        v4f x[U], y[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t i = i0 + k * 256;
            if (i < n4) {
                x[k] = ld<NT>(b + i);
                y[k] = ld<NT>(c + i);
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t i = i0 + k * 256;
            if (i < n4) {
                v4f r;
                r.x = fmaf(s, y[k].x, x[k].x);
                r.y = fmaf(s, y[k].y, x[k].y);
                r.z = fmaf(s, y[k].z, x[k].z);
                r.w = fmaf(s, y[k].w, x[k].w);
                st<NT>(a + i, r);
            }
        }
    }
}

__global__ void triad_tail(float* a, const float* b, const float* c, float s, int64_t from,
                           int64_t n) {
    const int64_t i = from + threadIdx.x;
    if (i < n) a[i] = fmaf(s, c[i], b[i]);
}

template <int U>
hipError_t launch_u(v4f* a, const v4f* b, const v4f* c, float s, int64_t n4, int blocks,
                    bool nt, hipStream_t st) {
    const int64_t chunks = (n4 + 256 * U - 1) / (256 * U);
    int64_t grid = blocks > 0 ? blocks : chunks;
    if (grid > chunks) grid = chunks;
    if (grid > 0x7fffffff) grid = 0x7fffffff;  // the blocks then stride over the chunks
    if (nt)
        hipLaunchKernelGGL((triad_kernel<U, true>), dim3((unsigned)grid), dim3(256), 0, st, a, b, c,
                           s, n4, chunks);
    else
        hipLaunchKernelGGL((triad_kernel<U, false>), dim3((unsigned)grid), dim3(256), 0, st, a, b,
                           c, s, n4, chunks);
    return hipGetLastError();
}

}  // namespace
}  // namespace fd

extern "C" int32_t fd_triad_config(float* a, const float* b, const float* c, float s, int64_t n,
                                   int32_t unroll, int32_t blocks, int32_t flags, void* stream) {
    if (!a || !b || !c || n < 0 || blocks < 0 || (flags & ~FD_TRIAD_TEMPORAL))
        return FD_ERR_INVALID_ARG;
    if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) return FD_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
         reinterpret_cast<uintptr_t>(c)) % 16)
        return FD_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n4 = n / 4;
    const bool nt = !(flags & FD_TRIAD_TEMPORAL);
    using fd::v4f;
    v4f* a4 = reinterpret_cast<v4f*>(a);
    const v4f* b4 = reinterpret_cast<const v4f*>(b);
    const v4f* c4 = reinterpret_cast<const v4f*>(c);
    hipError_t e = hipSuccess;
    if (n4 > 0) {
        switch (unroll) {
            case 1: e = fd::launch_u<1>(a4, b4, c4, s, n4, blocks, nt, st); break;
            case 2: e = fd::launch_u<2>(a4, b4, c4, s, n4, blocks, nt, st); break;
            case 4: e = fd::launch_u<4>(a4, b4, c4, s, n4, blocks, nt, st); break;
            default: e = fd::launch_u<8>(a4, b4, c4, s, n4, blocks, nt, st); break;
        }
    }
    if (e == hipSuccess && n4 * 4 < n) {
        hipLaunchKernelGGL(fd::triad_tail, dim3(1), dim3(64), 0, st, a, b, c, s, n4 * 4, n);
        e = hipGetLastError();
    }
    return e == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}

extern "C" int32_t fd_triad(float* a, const float* b, const float* c, float s, int64_t n,
                            void* stream) {
    return fd_triad_config(a, b, c, s, n, fd::kTriadUnroll, fd::kTriadBlocks, 0,
                           stream);
}
