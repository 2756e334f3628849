// fd_acoustic.hip -- acoustic leapfrog stencil kernels of libfd (gfx950).
//
// One launch advances every point of the padded volume by one step of
// Algorithm 1 for Eq. (Acou) with the damping layer:
//   u^{n+1} = [2 u^n - (1 - s) u^{n-1} + A L u^n] / (1 + s),  A = dt^2 v^2,
// written over u^{n-1}.  L is the star-shaped Laplacian of radius R whose
// per-axis weights arrive pre-divided by h^2; symmetric neighbours are summed
// before they are weighted.  Algorithmic traffic per point: read u^n, u^{n-1}
// and A, write u^{n+1} = 16 bytes (section 4.2); s is read only in tiles that
// hold damping.
#include "fd_internal.h"

namespace fd {

namespace {

__device__ inline float update(float c, float prev, float a, float lap, float s) {
    if (s == 0.f) return fmaf(a, lap, 2.f * c - prev);
    return (2.f * c - (1.f - s) * prev + a * lap) / (1.f + s);
}

// ---------------------------------------------------------------------------
// Direct kernel: one thread per point, every neighbour read from global memory
// (served by the caches).  Used for 2D, where the whole field is cache
// resident, and as a plain 3D variant.
// ---------------------------------------------------------------------------
template <int DIM, int R>
__global__ __launch_bounds__(256) void acoustic_direct(AcousticStep p) {
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
    p.up[i] = update(c, p.up[i], p.A[i], lap, s);
}

// ---------------------------------------------------------------------------
// Tiled 3D kernel (2.5D blocking).
//
// A block owns a 64 x TY column of (x, y) and marches over a chunk of z
// planes.  Each lane holds one x position and VY consecutive rows; the 2R+1
// planes around the current one live in a per-lane register queue (the z
// derivative never touches LDS).  The current plane, with an R-wide halo in x
// and y, is staged in a double-buffered LDS tile (one barrier per plane);
// x and y neighbours are read from LDS.  The loads for plane z+1 (queue
// head, halo, u^{n-1}, A and, in damped tiles, s) are issued before plane z
// is computed, so their latency overlaps the arithmetic.
//
// Blocks are numbered so that the 8 XCDs (which receive blocks round-robin)
// each get a contiguous run of tiles: neighbours that share halo rows run on
// the same XCD and find them in its L2.
// ---------------------------------------------------------------------------
template <int R, int NW, int VY>
__global__ __launch_bounds__(64 * NW) void acoustic3d_tiled(AcousticStep p) {
    constexpr int TY = NW * VY;
    constexpr int LW = kTileX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int NYH = (2 * R + NW - 1) / NW;               // y-halo rows per wave
    constexpr int NXH = (2 * R * TY + 64 * NW - 1) / (64 * NW);  // x-halo values per thread
    __shared__ float lds[2][LH][LW];

    const int b = blockIdx.x;
    const int t = (b & 7) * (p.nblocks >> 3) + (b >> 3);
    if (t >= p.ntiles) return;
    const int tx = t % p.ntx;
    const int t2 = t / p.ntx;
    const int ty = t2 % p.nty;
    const int zc = t2 / p.nty;
    const int x0 = tx * kTileX, y0 = ty * TY;
    const int z0 = zc * p.zchunk;
    const int z1 = min(z0 + p.zchunk, p.L.nz);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int64_t pitch = p.L.pitch, plane = p.L.plane;
    const int64_t col = p.L.origin + (int64_t)(y0 + w * VY) * pitch + x0 + lane;
    const bool xin = x0 + lane < p.L.nx;
    const float* __restrict__ u = p.uc;

    // halo sources (offsets within a plane) and LDS destinations
    int64_t hy_off[NYH];
    int hy_row[NYH];
#pragma unroll
    for (int k = 0; k < NYH; ++k) {
        const int hr = w + k * NW;
        const int yy = hr < R ? y0 - R + hr : y0 + TY + (hr - R);
        hy_row[k] = hr < R ? hr : TY + hr;
        hy_off[k] = p.L.origin + (int64_t)yy * pitch + x0 + lane;
    }
    int64_t hx_off[NXH];
    int hx_lds[NXH];
#pragma unroll
    for (int k = 0; k < NXH; ++k) {
        const int e = tid + k * 64 * NW;
        const int row = e / (2 * R), cc = e % (2 * R);
        const int xx = cc < R ? x0 - R + cc : x0 + kTileX + (cc - R);
        hx_lds[k] = (R + row) * LW + (cc < R ? cc : kTileX + cc);
        hx_off[k] = p.L.origin + (int64_t)(y0 + row) * pitch + xx;
    }

    float q[2 * R + 1][VY];
    float nxt[VY], prv[VY], aa[VY], sg[VY], hyv[NYH], hxv[NXH];
    int damp;

    auto load_plane_extras = [&](int z, float* prv_, float* aa_, float* sg_, int& damp_) {
        const int64_t zo = (int64_t)z * plane;
#pragma unroll
        for (int k = 0; k < NYH; ++k)
            if (w + k * NW < 2 * R) hyv[k] = u[hy_off[k] + zo];
#pragma unroll
        for (int k = 0; k < NXH; ++k)
            if (tid + k * 64 * NW < 2 * R * TY) hxv[k] = u[hx_off[k] + zo];
#pragma unroll
        for (int v = 0; v < VY; ++v) {
            prv_[v] = __builtin_nontemporal_load(p.up + col + v * pitch + zo);
            aa_[v] = __builtin_nontemporal_load(p.A + col + v * pitch + zo);
        }
        damp_ = 0;
        if (p.dflag) damp_ = __builtin_amdgcn_readfirstlane(
                         (int)p.dflag[((int64_t)z * p.nty + ty) * p.ntx + tx]);
        if (damp_) {
#pragma unroll
            for (int v = 0; v < VY; ++v) sg_[v] = p.sig[col + v * pitch + zo];
        } else {
#pragma unroll
            for (int v = 0; v < VY; ++v) sg_[v] = 0.f;
        }
    };

    // prime the queue with planes z0-R .. z0+R-1 and fetch plane z0+R
#pragma unroll
    for (int k = 0; k < 2 * R; ++k)
#pragma unroll
        for (int v = 0; v < VY; ++v) q[k + 1][v] = u[col + v * pitch + (int64_t)(z0 - R + k) * plane];
#pragma unroll
    for (int v = 0; v < VY; ++v) nxt[v] = u[col + v * pitch + (int64_t)(z0 + R) * plane];
    load_plane_extras(z0, prv, aa, sg, damp);

    int buf = 0;
    for (int z = z0; z < z1; ++z) {
#pragma unroll
        for (int k = 0; k < 2 * R; ++k)
#pragma unroll
            for (int v = 0; v < VY; ++v) q[k][v] = q[k + 1][v];
#pragma unroll
        for (int v = 0; v < VY; ++v) q[2 * R][v] = nxt[v];

        float* tile = &lds[buf][0][0];
#pragma unroll
        for (int v = 0; v < VY; ++v) tile[(R + w * VY + v) * LW + R + lane] = q[R][v];
#pragma unroll
        for (int k = 0; k < NYH; ++k)
            if (w + k * NW < 2 * R) tile[hy_row[k] * LW + R + lane] = hyv[k];
#pragma unroll
        for (int k = 0; k < NXH; ++k)
            if (tid + k * 64 * NW < 2 * R * TY) tile[hx_lds[k]] = hxv[k];
        __syncthreads();

        // keep this plane's operands, prefetch the next plane's
        float prv_c[VY], aa_c[VY], sg_c[VY];
#pragma unroll
        for (int v = 0; v < VY; ++v) {
            prv_c[v] = prv[v];
            aa_c[v] = aa[v];
            sg_c[v] = sg[v];
        }
        const int damp_c = damp;
        if (z + 1 < z1) {
#pragma unroll
            for (int v = 0; v < VY; ++v)
                nxt[v] = u[col + v * pitch + (int64_t)(z + R + 1) * plane];
            load_plane_extras(z + 1, prv, aa, sg, damp);
        }

        // y window of this lane's column: rows w*VY - R .. w*VY + VY + R - 1
        float cw[VY + 2 * R];
#pragma unroll
        for (int k = 0; k < VY + 2 * R; ++k) cw[k] = tile[(w * VY + k) * LW + R + lane];

        const int64_t zo = (int64_t)z * plane;
#pragma unroll
        for (int v = 0; v < VY; ++v) {
            const float* row = tile + (R + w * VY + v) * LW + R + lane;
            const float c = q[R][v];
            float lx = 0.f, ly = 0.f, lz = 0.f;
#pragma unroll
            for (int j = 1; j <= R; ++j) lx = fmaf(p.cx[j], row[j] + row[-j], lx);
#pragma unroll
            for (int j = 1; j <= R; ++j) ly = fmaf(p.cy[j], cw[v + R + j] + cw[v + R - j], ly);
#pragma unroll
            for (int j = 1; j <= R; ++j) lz = fmaf(p.cz[j], q[R + j][v] + q[R - j][v], lz);
            const float lap = fmaf(p.c0, c, lx + ly + lz);
            float nv;
            if (damp_c)
                nv = update(c, prv_c[v], aa_c[v], lap, sg_c[v]);
            else
                nv = fmaf(aa_c[v], lap, 2.f * c - prv_c[v]);
            if (xin && y0 + w * VY + v < p.L.ny)
                __builtin_nontemporal_store(nv, p.up + col + v * pitch + zo);
        }
        buf ^= 1;
    }
}

template <int R>
hipError_t launch_direct(const AcousticStep& p, int ndim, hipStream_t s) {
    const int gx = (p.L.nx + kTileX - 1) / kTileX;
    if (ndim == 2) {
        hipLaunchKernelGGL((acoustic_direct<2, R>), dim3(gx, (p.L.nz + 3) / 4), dim3(64, 4), 0, s,
                           p);
    } else {
        hipLaunchKernelGGL((acoustic_direct<3, R>), dim3(gx, (p.L.ny + 3) / 4, p.L.nz),
                           dim3(64, 4), 0, s, p);
    }
    return hipGetLastError();
}

template <int R, int NW, int VY>
hipError_t launch_tiled(const AcousticStep& p, hipStream_t s) {
    hipLaunchKernelGGL((acoustic3d_tiled<R, NW, VY>), dim3(p.nblocks), dim3(64 * NW), 0, s, p);
    return hipGetLastError();
}

template <int R>
hipError_t launch_tiled_vy(const AcousticStep& p, int vy, hipStream_t s) {
    switch (vy) {
        case 2: return launch_tiled<R, 4, 2>(p, s);
        case 4: return launch_tiled<R, 4, 4>(p, s);
        case 8: return launch_tiled<R, 4, 8>(p, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int acoustic_tile_y(int radius, int vy) {
    (void)radius;
    return 4 * vy;
}

hipError_t launch_acoustic(const AcousticStep& p, int ndim, int radius, int variant, int vy,
                           hipStream_t s) {
    const bool tiled = ndim == 3 && variant == 0;
#define FD_CASE(RR)                                                     \
    case RR:                                                            \
        return tiled ? launch_tiled_vy<RR>(p, vy, s) : launch_direct<RR>(p, ndim, s);
    switch (radius) {
        FD_CASE(1)
        FD_CASE(2)
        FD_CASE(3)
        FD_CASE(4)
        FD_CASE(5)
        FD_CASE(6)
        FD_CASE(7)
        FD_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef FD_CASE
}

}  // namespace fd
