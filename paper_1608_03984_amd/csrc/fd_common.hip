// fd_common.hip -- layout, setup and sparse-point kernels of libfd (gfx950).
#include "fd_internal.h"

namespace fd {

namespace {

constexpr int kBlock = 256;

__device__ inline int64_t vol_index(const Layout& L, int x, int y, int z) {
    return L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
}

__global__ __launch_bounds__(kBlock) void fill_zero_kernel(float4* p, int64_t n4) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = z;
}

// dense [nz][ny][nx] <-> padded volume
__global__ __launch_bounds__(kBlock) void pack_kernel(const float* __restrict__ vol,
                                                      float* __restrict__ dense, Layout L) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int x = (int)(i % L.nx);
        const int64_t r = i / L.nx;
        const int y = (int)(r % L.ny);
        const int z = (int)(r / L.ny);
        dense[i] = vol[vol_index(L, x, y, z)];
    }
}

__global__ __launch_bounds__(kBlock) void unpack_kernel(const float* __restrict__ dense,
                                                        float* __restrict__ vol, Layout L) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int x = (int)(i % L.nx);
        const int64_t r = i / L.nx;
        const int y = (int)(r % L.ny);
        const int z = (int)(r / L.ny);
        vol[vol_index(L, x, y, z)] = dense[i];
    }
}

// Damping profiles through the centre point (xc, yc, zc): sx[x] = sig(x, yc,
// zc), sy[y] = sig(xc, y, zc), sz[z] = sig(xc, yc, z).  For a field that is a
// sum of per-axis profiles vanishing at the centre (the usual absorbing
// layer), (sx[x] + sy[y]) + sz[z] reproduces it.
__global__ __launch_bounds__(kBlock) void damping_profile_kernel(const float* __restrict__ sig,
                                                                 Layout L, float* sx, float* sy,
                                                                 float* sz) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int xc = L.nx / 2, yc = L.ny / 2, zc = L.nz / 2;
    if (i < L.nx) sx[i] = sig[vol_index(L, i, yc, zc)];
    if (i < L.ny) sy[i] = sig[vol_index(L, xc, i, zc)];
    if (i < L.nz) sz[i] = sig[vol_index(L, xc, yc, i)];
}

// red[0] = max |sig - ((sx + sy) + sz)|, red[1] = max sig (float bits; both
// non-negative, so integer order is float order).
__global__ __launch_bounds__(kBlock) void damping_check_kernel(const float* __restrict__ sig,
                                                               Layout L,
                                                               const float* __restrict__ sx,
                                                               const float* __restrict__ sy,
                                                               const float* __restrict__ sz,
                                                               uint32_t* red) {
    __shared__ float sd[kBlock / 64], sm[kBlock / 64];
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    float dmax = 0.f, smx = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int x = (int)(i % L.nx);
        const int64_t r = i / L.nx;
        const int y = (int)(r % L.ny);
        const int z = (int)(r / L.ny);
        const float v = sig[vol_index(L, x, y, z)];
        const float sep = (sx[x] + sy[y]) + sz[z];
        dmax = fmaxf(dmax, fabsf(v - sep));
        smx = fmaxf(smx, fabsf(v));
    }
    for (int off = 32; off > 0; off >>= 1) {
        dmax = fmaxf(dmax, __shfl_xor(dmax, off));
        smx = fmaxf(smx, __shfl_xor(smx, off));
    }
    if ((threadIdx.x & 63) == 0) {
        sd[threadIdx.x >> 6] = dmax;
        sm[threadIdx.x >> 6] = smx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float d = sd[0], m = sm[0];
        for (int i = 1; i < kBlock / 64; ++i) {
            d = fmaxf(d, sd[i]);
            m = fmaxf(m, sm[i]);
        }
        atomicMax(&red[0], __float_as_uint(d));
        atomicMax(&red[1], __float_as_uint(m));
    }
}

// flags[(z * nty + ty) * ntx + tx] = 1 when any damping coefficient in the
// 64 x tile_y tile (tx, ty) of plane z is non-zero.
__global__ __launch_bounds__(kBlock) void damping_flags_kernel(const float* __restrict__ sig,
                                                               int32_t* flags, Layout L,
                                                               int tile_y, int ntx, int nty) {
    const int tile = blockIdx.x;
    const int z = blockIdx.y;
    const int tx = tile % ntx, ty = tile / ntx;
    int any = 0;
    for (int e = threadIdx.x; e < kTileX * tile_y; e += kBlock) {
        const int x = tx * kTileX + (e & (kTileX - 1));
        const int y = ty * tile_y + e / kTileX;
        if (x < L.nx && y < L.ny && sig[vol_index(L, x, y, z)] != 0.f) any = 1;
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) flags[((int64_t)z * nty + ty) * ntx + tx] = any ? 1 : 0;
}

// One thread per target corner of the plan: u[corner] += w A q scale / (1 + s)
// for each contribution (point, corner weight w) in point order, in the
// volume of the target's shot.  A corner reached by one point gets exactly
// the single addition of that point.
__global__ __launch_bounds__(kBlock) void inject_kernel(float* u, const float* __restrict__ A,
                                                        const float* __restrict__ sig,
                                                        const SparsePoint* __restrict__ pts,
                                                        InjectPlan plan,
                                                        const float* __restrict__ q, float scale,
                                                        Layout L, int ndim, int64_t shot_stride) {
    const int m = blockIdx.x * kBlock + threadIdx.x;
    if (m >= plan.ntarget) return;
    const int64_t i = plan.target[m];
    float* up = u + plan.shot[m] * shot_stride + i;
    const float a = A[i];
    const float sg = sig ? sig[i] : 0.f;
    *up = inject_target(*up, plan, m, pts, q, scale, a, sg, ndim);
}

__global__ __launch_bounds__(kBlock) void record_kernel(const float* __restrict__ u,
                                                        const SparsePoint* __restrict__ pts,
                                                        int n, float* __restrict__ out,
                                                        float scale, Layout L, int ndim,
                                                        int64_t shot_stride) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const SparsePoint P = pts[j];
    out[j] = sample_point(u + P.shot * shot_stride, P, L, ndim) * scale;
}

// Blocks [0, ninj) inject into un, the others record from uc (a different
// level, so the two parts are independent).
__global__ __launch_bounds__(kBlock) void inject_record_kernel(
    float* un, float* un2, int un2_damped, const float* __restrict__ A, const float* __restrict__ sig,
    const SparsePoint* __restrict__ spts, InjectPlan plan, const float* __restrict__ q,
    float scale, int ninj, const float* __restrict__ uc, const SparsePoint* __restrict__ rpts,
    int nrec, float* __restrict__ out, Layout L, int ndim, int64_t shot_stride) {
    if ((int)blockIdx.x < ninj) {
        const int m = blockIdx.x * kBlock + threadIdx.x;
        if (m >= plan.ntarget) return;
        const int64_t i = plan.target[m];
        const int64_t o = plan.shot[m] * shot_stride + i;
        const float a = A[i];
        const float sg = sig ? sig[i] : 0.f;
        un[o] = inject_target(un[o], plan, m, spts, q, scale, a, sg, ndim);
        if (un2)
            un2[o] = inject_target(un2[o], plan, m, spts, q, scale, a, un2_damped ? sg : 0.f, ndim);
        return;
    }
    const int j = (blockIdx.x - ninj) * kBlock + threadIdx.x;
    if (j >= nrec) return;
    const SparsePoint P = rpts[j];
    out[j] = sample_point(uc + P.shot * shot_stride, P, L, ndim) * 1.f;
}

int grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
    const int64_t n4 = n / 4;  // volumes and regions are multiples of 64 floats
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n4)), dim3(kBlock), 0, s,
                       reinterpret_cast<float4*>(p), n4);
    return hipGetLastError();
}

hipError_t launch_pack(const float* vol, float* dense, const Layout& L, hipStream_t s) {
    hipLaunchKernelGGL(pack_kernel, dim3(grid_for((int64_t)L.nx * L.ny * L.nz)), dim3(kBlock), 0,
                       s, vol, dense, L);
    return hipGetLastError();
}

hipError_t launch_unpack(const float* dense, float* vol, const Layout& L, hipStream_t s) {
    hipLaunchKernelGGL(unpack_kernel, dim3(grid_for((int64_t)L.nx * L.ny * L.nz)), dim3(kBlock),
                       0, s, dense, vol, L);
    return hipGetLastError();
}

hipError_t launch_damping_profiles(const float* sig, const Layout& L, float* sx, float* sy,
                                   float* sz, uint32_t* red, hipStream_t s) {
    const int nmax = L.nx > L.ny ? (L.nx > L.nz ? L.nx : L.nz) : (L.ny > L.nz ? L.ny : L.nz);
    hipLaunchKernelGGL(damping_profile_kernel, dim3((nmax + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       s, sig, L, sx, sy, sz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t g = grid_for((int64_t)L.nx * L.ny * L.nz);
    hipLaunchKernelGGL(damping_check_kernel, dim3(g < 1024 ? g : 1024), dim3(kBlock), 0, s, sig,
                       L, sx, sy, sz, red);
    return hipGetLastError();
}

hipError_t launch_damping_flags(const float* sig, int32_t* flags, const Layout& L, int tile_y,
                                int ntx, int nty, hipStream_t s) {
    hipLaunchKernelGGL(damping_flags_kernel, dim3(ntx * nty, L.nz), dim3(kBlock), 0, s, sig,
                       flags, L, tile_y, ntx, nty);
    return hipGetLastError();
}

hipError_t launch_inject(float* u, const float* A, const float* sig, const SparsePoint* pts,
                         const InjectPlan& plan, const float* q, float scale, const Layout& L,
                         int ndim, int64_t shot_stride, hipStream_t s) {
    if (plan.ntarget <= 0) return hipSuccess;
    hipLaunchKernelGGL(inject_kernel, dim3((plan.ntarget + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       s, u, A, sig, pts, plan, q, scale, L, ndim, shot_stride);
    return hipGetLastError();
}

hipError_t launch_inject_record(float* un, float* un2, bool un2_damped, const float* A,
                                const float* sig,
                                const SparsePoint* spts, const InjectPlan& plan, const float* q,
                                float scale, const float* uc, const SparsePoint* rpts, int nrec,
                                float* out, const Layout& L, int ndim, int64_t shot_stride,
                                hipStream_t s) {
    const int ninj = plan.ntarget > 0 ? (plan.ntarget + kBlock - 1) / kBlock : 0;
    const int nrb = nrec > 0 ? (nrec + kBlock - 1) / kBlock : 0;
    if (ninj + nrb == 0) return hipSuccess;
    hipLaunchKernelGGL(inject_record_kernel, dim3(ninj + nrb), dim3(kBlock), 0, s, un, un2,
                       un2_damped ? 1 : 0, A, sig,
                       spts, plan, q, scale, ninj, uc, rpts, nrec, out, L, ndim, shot_stride);
    return hipGetLastError();
}

hipError_t launch_record(const float* u, const SparsePoint* pts, int n, float* out, float scale,
                         const Layout& L, int ndim, int64_t shot_stride, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(record_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, u, pts,
                       n, out, scale, L, ndim, shot_stride);
    return hipGetLastError();
}

}  // namespace fd
