// fd_tti.hip -- TTI pseudo-acoustic stencil kernels of libfd (gfx950).
//
// One launch advances p and r by one step of Eq. (TTI):
//   p+ = [2p - (1-s)p- + A(e H p + d Gz r)]/(1+s)
//   r+ = [2r - (1-s)r- + A(d H p + Gz r)]/(1+s)
// with Gz = G_zbar_zbar = c1 Dxx + c2 Dyy + c3 Dzz + c4 Dxy + c5 Dyz + c6 Dxz
// (Eq. (DiffOp)), H = G_xbar_xbar + G_ybar_ybar = Laplacian - Gz, pure second
// derivatives from the 2R+1-point second-derivative stencil and mixed ones as
// the product of two first-derivative stencils (section 4.1).  Algorithmic
// traffic: 15 fields x 4 bytes = 60 bytes per point (section 4.2).
#include "fd_internal.h"

namespace fd {

namespace {

struct Derivs {
    float xx, yy, zz, xy, yz, xz;
};

// All six second derivatives of f at flat index i, straight from global
// memory.  Mixed terms use the antisymmetry w1[-a] = -w1[a]:
//   Dab f = sum_{a,b>0} w1a w1b (f[+a,+b] - f[+a,-b] - f[-a,+b] + f[-a,-b]).
template <int R>
__device__ inline Derivs derivs_direct(const float* __restrict__ f, int64_t i, int64_t sy,
                                       int64_t sz, const TTIStep& p) {
    Derivs d;
    const float c = f[i];
    float xx = 0.f, yy = 0.f, zz = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        xx = fmaf(p.w2x[j], f[i + j] + f[i - j], xx);
        yy = fmaf(p.w2y[j], f[i + j * sy] + f[i - j * sy], yy);
        zz = fmaf(p.w2z[j], f[i + j * sz] + f[i - j * sz], zz);
    }
    d.xx = fmaf(p.w2x[0], c, xx);
    d.yy = fmaf(p.w2y[0], c, yy);
    d.zz = fmaf(p.w2z[0], c, zz);
    float xy = 0.f, yz = 0.f, xz = 0.f;
#pragma unroll
    for (int a = 1; a <= R; ++a) {
        float sxy = 0.f, syz = 0.f, sxz = 0.f;
#pragma unroll
        for (int b = 1; b <= R; ++b) {
            sxy = fmaf(p.w1y[b], (f[i + a + b * sy] - f[i + a - b * sy]) -
                                     (f[i - a + b * sy] - f[i - a - b * sy]), sxy);
            syz = fmaf(p.w1z[b], (f[i + a * sy + b * sz] - f[i + a * sy - b * sz]) -
                                     (f[i - a * sy + b * sz] - f[i - a * sy - b * sz]), syz);
            sxz = fmaf(p.w1z[b], (f[i + a + b * sz] - f[i + a - b * sz]) -
                                     (f[i - a + b * sz] - f[i - a - b * sz]), sxz);
        }
        xy = fmaf(p.w1x[a], sxy, xy);
        yz = fmaf(p.w1y[a], syz, yz);
        xz = fmaf(p.w1x[a], sxz, xz);
    }
    d.xy = xy;
    d.yz = yz;
    d.xz = xz;
    return d;
}

template <int R>
__global__ __launch_bounds__(256) void tti_direct(TTIStep p) {
    const int x = blockIdx.x * kTileX + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= p.L.nx || y >= p.L.ny || z >= p.L.nz) return;
    const int64_t sy = p.L.pitch, sz = p.L.plane;
    const int64_t i = p.L.origin + z * sz + y * sy + x;
    const Derivs dp = derivs_direct<R>(p.pc, i, sy, sz, p);
    const Derivs dr = derivs_direct<R>(p.rc, i, sy, sz, p);
    const float c1 = p.c[0][i], c2 = p.c[1][i], c3 = p.c[2][i];
    const float c4 = p.c[3][i], c5 = p.c[4][i], c6 = p.c[5][i];
    const float gzp = c1 * dp.xx + c2 * dp.yy + c3 * dp.zz + c4 * dp.xy + c5 * dp.yz + c6 * dp.xz;
    const float gzr = c1 * dr.xx + c2 * dr.yy + c3 * dr.zz + c4 * dr.xy + c5 * dr.yz + c6 * dr.xz;
    const float hp = (dp.xx + dp.yy + dp.zz) - gzp;
    const float a = p.A[i], e = p.e[i], d = p.d[i];
    const float s = p.sig ? p.sig[i] : 0.f;
    const float pc = p.pc[i], rc = p.rc[i];
    const float fp = a * (e * hp + d * gzr);
    const float fr = a * (d * hp + gzr);
    float pn, rn;
    if (s == 0.f) {
        pn = (2.f * pc - p.pp[i]) + fp;
        rn = (2.f * rc - p.rp[i]) + fr;
    } else {
        pn = (2.f * pc - (1.f - s) * p.pp[i] + fp) / (1.f + s);
        rn = (2.f * rc - (1.f - s) * p.rp[i] + fr) / (1.f + s);
    }
    p.pp[i] = pn;
    p.rp[i] = rn;
}

template <int R>
hipError_t launch_direct(const TTIStep& p, hipStream_t s) {
    const dim3 grid((p.L.nx + kTileX - 1) / kTileX, (p.L.ny + 3) / 4, p.L.nz);
    hipLaunchKernelGGL((tti_direct<R>), grid, dim3(64, 4), 0, s, p);
    return hipGetLastError();
}

}  // namespace

int tti_tile_y(int radius) {
    (void)radius;
    return 16;
}

hipError_t launch_tti(const TTIStep& p, int radius, int variant, hipStream_t s) {
    (void)variant;
    switch (radius) {
        case 1: return launch_direct<1>(p, s);
        case 2: return launch_direct<2>(p, s);
        case 3: return launch_direct<3>(p, s);
        case 4: return launch_direct<4>(p, s);
        case 5: return launch_direct<5>(p, s);
        case 6: return launch_direct<6>(p, s);
        case 7: return launch_direct<7>(p, s);
        case 8: return launch_direct<8>(p, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fd
