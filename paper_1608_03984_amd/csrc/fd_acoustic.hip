// fd_acoustic.hip -- acoustic leapfrog stencil kernels of libfd (gfx950):
// the direct kernel (2D, and a plain 3D variant), the launch dispatch, and
// the tiled 3D kernel of radius 1-4 (radius 5-6 is instantiated in
// fd_acoustic_hi.hip, 7-8 in fd_acoustic_top.hip).  The update and the tiled kernel's design are
// described in fd_acoustic_tiled.h.
#include "fd_acoustic_tiled.h"

namespace fd {

namespace {

// ---------------------------------------------------------------------------
// Direct kernel: one thread per point, every neighbour read from global memory
// (served by the caches).  Used for 2D, where the whole field is cache
// resident, and as a plain 3D variant.
// ---------------------------------------------------------------------------
template <int DIM, int R>
__global__ __launch_bounds__(256) void acoustic_direct(AcousticStep p) {
    if (p.rec_n > 0) {
        // the previous step's receiver samples (u^n is only read here)
        const int64_t nthr = (int64_t)gridDim.x * gridDim.y * gridDim.z * 256;
        const int64_t g = (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 256 +
                          threadIdx.y * 64 + threadIdx.x;
        for (int64_t j = g; j < p.rec_n; j += nthr)
            p.rec_out[j] = sample_point(p.uc, p.rec_pts[j], p.L, DIM);
    }
    const int x = blockIdx.x * kTileX + threadIdx.x;
    const int y = DIM == 3 ? (int)(blockIdx.y * 4 + threadIdx.y) : 0;
    const int z = DIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * 4 + threadIdx.y);
    if (x >= p.L.nx || y >= p.L.ny || z >= p.L.nz) return;
    const int64_t pitch = p.L.pitch, plane = p.L.plane;
    const int64_t i = p.L.origin + z * plane + y * pitch + x;
    const float* __restrict__ u = p.uc;
    const float c = u[i];
    float lx = 0.f, ly = 0.f, lz = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) lx = fmaf(p.cx[j], u[i + j] + u[i - j], lx);
    if (DIM == 3) {
#pragma unroll
        for (int j = 1; j <= R; ++j) ly = fmaf(p.cy[j], u[i + j * pitch] + u[i - j * pitch], ly);
    }
#pragma unroll
    for (int j = 1; j <= R; ++j) lz = fmaf(p.cz[j], u[i + j * plane] + u[i - j * plane], lz);
    const float lap = fmaf(p.c0, c, lx + ly + lz);
    const float s = p.sig ? p.sig[i] : 0.f;
    const float a = p.A[i];
    float un = update(c, p.up[i], a, lap, s);
    if (p.inj.ntarget > 0 && i >= p.inj_lo && i <= p.inj_hi) {
        // a target of the plan (sorted): add its sources as the injection
        // kernel would, to the value about to be stored
        int lo = 0, hi = p.inj.ntarget - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (p.inj.target[mid] < i)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (p.inj.target[lo] == i)
            un = inject_target(un, p.inj, lo, p.inj_pts, p.inj_q, p.inj_scale, a, s, DIM);
    }
    p.up[i] = un;
    if (p.acc) p.acc[i] = a * lap;
}

template <int R>
hipError_t launch_direct(const AcousticStep& p, int ndim, hipStream_t s) {
    const int gx = (p.L.nx + kTileX - 1) / kTileX;
    // one launch per shot (the direct kernel serves 2D and the plain variant)
    for (int shot = 0; shot < p.nshots; ++shot) {
        AcousticStep q = p;
        q.uc = p.uc + shot * p.shot_stride;
        q.up = p.up + shot * p.shot_stride;
        q.acc = p.acc ? p.acc + shot * p.shot_stride : nullptr;
        if (ndim == 2) {
            hipLaunchKernelGGL((acoustic_direct<2, R>), dim3(gx, (p.L.nz + 3) / 4), dim3(64, 4),
                               0, s, q);
        } else {
            hipLaunchKernelGGL((acoustic_direct<3, R>), dim3(gx, (p.L.ny + 3) / 4, p.L.nz),
                               dim3(64, 4), 0, s, q);
        }
    }
    return hipGetLastError();
}

}  // namespace

int acoustic_tile_y(int cfg) {
    return cfg >= 0 && cfg < 5 ? kAcousticTiles[cfg].height() : kAcousticTiles[0].height();
}

hipError_t launch_acoustic(const AcousticStep& p, int ndim, int radius, int variant, int cfg,
                           int shots_per_block, hipStream_t s) {
    const bool tiled = ndim == 3 && variant == 0;
    if (tiled && (radius == 5 || radius == 6))
        return launch_acoustic_tiled_r56(p, radius, cfg, shots_per_block, s);
    if (tiled && (radius == 7 || radius == 8))
        return launch_acoustic_tiled_r78(p, radius, cfg, shots_per_block, s);
    switch (radius) {
        case 1:
            return tiled ? launch_tiled_cfg<1>(p, cfg, shots_per_block, s)
                         : launch_direct<1>(p, ndim, s);
        case 2:
            return tiled ? launch_tiled_cfg<2>(p, cfg, shots_per_block, s)
                         : launch_direct<2>(p, ndim, s);
        case 3:
            return tiled ? launch_tiled_cfg<3>(p, cfg, shots_per_block, s)
                         : launch_direct<3>(p, ndim, s);
        case 4:
            return tiled ? launch_tiled_cfg<4>(p, cfg, shots_per_block, s)
                         : launch_direct<4>(p, ndim, s);
        case 5: return launch_direct<5>(p, ndim, s);
        case 6: return launch_direct<6>(p, ndim, s);
        case 7: return launch_direct<7>(p, ndim, s);
        case 8: return launch_direct<8>(p, ndim, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fd
