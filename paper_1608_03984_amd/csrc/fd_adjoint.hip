// fd_adjoint.hip -- imaging-condition kernels of libfd (gfx950).
//
// The velocity gradient of a misfit of the traces of Eq. (Acou) is a
// correlation in time of the adjoint wavefield with the forward wavefield's
// second time difference.  With mu^k = dt^2 v^2 lambda^k (lambda the adjoint
// state) and a^k = A L u^{k-1} + injected source (the acceleration term the
// forward step stores), the gradient with respect to m = 1/v^2 is
//   dJ/dm = -(1/dt^2) sum_k mu^k a^k.
// The per-step correlation is summed in FP32 in two levels: into a partial
// sum on the padded layout of the fields (16 bytes per point and step: mu and
// the acceleration read, the partial sum read and written), flushed every few
// tens of steps into a dense total, which keeps the rounding of long sums
// bounded without FP64 on the device.  A
// final pass scales the total and, for the gradient with respect to v,
// applies dm/dv = -2/v^3.
#include "fd_internal.h"

namespace fd {

namespace {

constexpr int kRows = 4;  // rows of 64 points per 256-thread block

// grid: x = ceil(nx / 64) * ceil(ny / kRows) tiles of one plane, y = planes
// (strided when nz exceeds the grid).
__global__ __launch_bounds__(256) void image_kernel(const float* __restrict__ mu,
                                                    const float* __restrict__ acc,
                                                    float* __restrict__ gpart, Layout L, int ntx) {
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int x = tx * kTileX + (threadIdx.x & 63);
    const int y = ty * kRows + (threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    for (int z = blockIdx.y; z < L.nz; z += gridDim.y) {
        const int64_t v = L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
        gpart[v] = fmaf(mu[v], acc[v], gpart[v]);
    }
}

__global__ __launch_bounds__(256) void flush_kernel(float* __restrict__ gpart,
                                                    float* __restrict__ gsum, Layout L, int ntx) {
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int x = tx * kTileX + (threadIdx.x & 63);
    const int y = ty * kRows + (threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    for (int z = blockIdx.y; z < L.nz; z += gridDim.y) {
        const int64_t v = L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
        const int64_t d = ((int64_t)z * L.ny + y) * L.nx + x;
        gsum[d] += gpart[v];
        gpart[v] = 0.f;
    }
}

__global__ __launch_bounds__(256) void finish_kernel(const float* __restrict__ gsum,
                                                     const float* __restrict__ A,
                                                     float* __restrict__ out, Layout L, int ntx,
                                                     float dt, float inv_dt2, int wrt_vel,
                                                     int accumulate) {
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int x = tx * kTileX + (threadIdx.x & 63);
    const int y = ty * kRows + (threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    for (int z = blockIdx.y; z < L.nz; z += gridDim.y) {
        const int64_t v = L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
        const int64_t d = ((int64_t)z * L.ny + y) * L.nx + x;
        if (wrt_vel) {
            // dJ/dv = dJ/dm * (-2 / v^3), v = sqrt(A) / dt
            const float a = A[v];
            const float g = gsum[d] * (2.f * dt) / (a * sqrtf(a));
            out[d] = accumulate ? out[d] + g : g;
        } else {
            const float g = -gsum[d] * inv_dt2;
            out[d] = accumulate ? out[d] + g : g;
        }
    }
}

// res = d - d_obs and 1/2 sum res^2 in FP64 (the misfit is what the
// finite-difference checks of the gradient difference), in two passes with
// a fixed grid, so the sum is the same bits on every run: block b sums the
// elements b*256 + t + k*kMisfitBlocks*256 of each thread t in a fixed tree
// into J[1 + b]; one block then adds J[1..kMisfitBlocks] (four consecutive
// partials per thread, then a fixed tree) to J[0].
__global__ __launch_bounds__(256) void misfit_kernel(const float* __restrict__ d,
                                                     const float* __restrict__ dobs, int64_t n,
                                                     float* res, double* __restrict__ J) {
    __shared__ double part[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const float r = d[i] - dobs[i];
        res[i] = r;
        acc += 0.5 * (double)r * (double)r;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) J[1 + blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ __launch_bounds__(256) void misfit_sum_kernel(double* __restrict__ J, int nblocks) {
    __shared__ double part[4];
    double acc = 0.0;  // thread t: partials 4t .. 4t+3 in order
    for (int k = 0; k < 4; ++k)
        if (4 * (int)threadIdx.x + k < nblocks) acc += J[1 + 4 * threadIdx.x + k];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) J[0] += (part[0] + part[1]) + (part[2] + part[3]);
}

dim3 plane_grid(const Layout& L, int& ntx) {
    ntx = (L.nx + kTileX - 1) / kTileX;
    const int nty = (L.ny + kRows - 1) / kRows;
    return dim3(ntx * nty, L.nz < 65535 ? L.nz : 65535);
}

}  // namespace

hipError_t launch_image(const float* mu, const float* acc, float* gpart, const Layout& L,
                        hipStream_t s) {
    int ntx;
    const dim3 grid = plane_grid(L, ntx);
    hipLaunchKernelGGL(image_kernel, grid, dim3(256), 0, s, mu, acc, gpart, L, ntx);
    return hipGetLastError();
}

hipError_t launch_flush_gradient(float* gpart, float* gsum, const Layout& L, hipStream_t s) {
    int ntx;
    const dim3 grid = plane_grid(L, ntx);
    hipLaunchKernelGGL(flush_kernel, grid, dim3(256), 0, s, gpart, gsum, L, ntx);
    return hipGetLastError();
}

hipError_t launch_finish_gradient(const float* gsum, const float* A, float* out, const Layout& L,
                                  double dt, int wrt_vel, int accumulate, hipStream_t s) {
    int ntx;
    const dim3 grid = plane_grid(L, ntx);
    hipLaunchKernelGGL(finish_kernel, grid, dim3(256), 0, s, gsum, A, out, L, ntx, (float)dt,
                       (float)(1.0 / (dt * dt)), wrt_vel, accumulate);
    return hipGetLastError();
}

hipError_t launch_misfit(const float* d, const float* dobs, int64_t n, float* res, double* J,
                         hipStream_t s) {
    static_assert(kMisfitBlocks <= 4 * 256, "one block of the second pass sums the partials");
    hipLaunchKernelGGL(misfit_kernel, dim3(kMisfitBlocks), dim3(256), 0, s, d, dobs, n, res, J);
    hipLaunchKernelGGL(misfit_sum_kernel, dim3(1), dim3(256), 0, s, J, kMisfitBlocks);
    return hipGetLastError();
}

}  // namespace fd
