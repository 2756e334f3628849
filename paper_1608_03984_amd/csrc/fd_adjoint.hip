// fd_adjoint.hip -- imaging-condition kernels of libfd (gfx950).
//
// The velocity gradient of a misfit of the traces of Eq. (Acou) is a
// correlation in time of the adjoint wavefield with the forward wavefield's
// second time difference.  With mu^k = dt^2 v^2 lambda^k (lambda the adjoint
// state) and a^k = A L u^{k-1} + injected source (the acceleration term the
// forward step stores), the gradient with respect to m = 1/v^2 is
//   dJ/dm = -(1/dt^2) sum_k mu^k a^k.
// The per-step correlation is accumulated in FP64 over a dense array; a final
// pass scales it and, for the gradient with respect to v, applies
// dm/dv = -2/v^3.  Both kernels stream (no reuse): 16 bytes per point per step
// for the correlation (two FP32 reads, one FP64 read and write).
#include "fd_internal.h"

namespace fd {

namespace {

constexpr int kRows = 4;  // rows of 64 points per 256-thread block

// grid: x = ceil(nx / 64) * ceil(ny / kRows) tiles of one plane, y = planes
// (strided when nz exceeds the grid).
__global__ __launch_bounds__(256) void image_kernel(const float* __restrict__ mu,
                                                    const float* __restrict__ acc,
                                                    double* __restrict__ g, Layout L, int ntx) {
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int x = tx * kTileX + (threadIdx.x & 63);
    const int y = ty * kRows + (threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    for (int z = blockIdx.y; z < L.nz; z += gridDim.y) {
        const int64_t v = L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
        const int64_t d = ((int64_t)z * L.ny + y) * L.nx + x;
        g[d] += (double)mu[v] * (double)acc[v];  // exact product, no FP32 underflow
    }
}

__global__ __launch_bounds__(256) void finish_kernel(const double* __restrict__ g,
                                                     const float* __restrict__ A,
                                                     float* __restrict__ out, Layout L, int ntx,
                                                     double dt, int wrt_vel) {
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int x = tx * kTileX + (threadIdx.x & 63);
    const int y = ty * kRows + (threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    for (int z = blockIdx.y; z < L.nz; z += gridDim.y) {
        const int64_t v = L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
        const int64_t d = ((int64_t)z * L.ny + y) * L.nx + x;
        if (wrt_vel) {
            // dJ/dv = dJ/dm * (-2 / v^3), v = sqrt(A) / dt
            const double a = (double)A[v];
            out[d] = (float)(g[d] * 2.0 * dt / (a * sqrt(a)));
        } else {
            out[d] = (float)(-g[d] / (dt * dt));
        }
    }
}

dim3 plane_grid(const Layout& L, int& ntx) {
    ntx = (L.nx + kTileX - 1) / kTileX;
    const int nty = (L.ny + kRows - 1) / kRows;
    return dim3(ntx * nty, L.nz < 65535 ? L.nz : 65535);
}

}  // namespace

hipError_t launch_image(const float* mu, const float* acc, double* g, const Layout& L,
                        hipStream_t s) {
    int ntx;
    const dim3 grid = plane_grid(L, ntx);
    hipLaunchKernelGGL(image_kernel, grid, dim3(256), 0, s, mu, acc, g, L, ntx);
    return hipGetLastError();
}

hipError_t launch_finish_gradient(const double* g, const float* A, float* out, const Layout& L,
                                  double dt, int wrt_vel, hipStream_t s) {
    int ntx;
    const dim3 grid = plane_grid(L, ntx);
    hipLaunchKernelGGL(finish_kernel, grid, dim3(256), 0, s, g, A, out, L, ntx, dt, wrt_vel);
    return hipGetLastError();
}

}  // namespace fd
