// fd_vti.hip -- VTI pseudo-acoustic stencil kernels of libfd (gfx950).
//
// One launch advances p and r by one step of Eq. (vVTI) with the damping
// layer, the horizontal operator Dh = Dxx (2D) or Dxx + Dyy (3D):
//   p+ = [2p - (1-s)p- + A(e Dh p + d Dzz r)]/(1+s)
//   r+ = [2r - (1-s)r- + A(d Dh p + Dzz r)]/(1+s)
// with A = dt^2 v^2, e = 1 + 2 eps, d = sqrt(1 + 2 delta), written over p- and
// r-.  Only the horizontal derivatives of p and the vertical derivative of r
// enter.  Algorithmic traffic: 9 fields x 4 bytes = 36 bytes per point
// (section 4.2: read A, e, d, p, p-, r, r-; write p+, r+).
#include "fd_internal.h"

#include <utility>

namespace fd {

namespace {

constexpr int kBufNT = 2;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const float* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, 0x7fffffff, 0x00020000);
}
template <int AUX = 0>
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, kBufNT);
}

__device__ __forceinline__ void vti_update(float pc, float pp, float rc, float rp, float a, float e,
                                           float d, float s, float dh, float dzz, float& pn,
                                           float& rn) {
    const float fp = fmaf(e, dh, d * dzz);
    const float fr = fmaf(d, dh, dzz);
    if (s == 0.f) {
        pn = fmaf(a, fp, 2.f * pc - pp);
        rn = fmaf(a, fr, 2.f * rc - rp);
    } else {
        pn = (2.f * pc - (1.f - s) * pp + a * fp) / (1.f + s);
        rn = (2.f * rc - (1.f - s) * rp + a * fr) / (1.f + s);
    }
}

// ---------------------------------------------------------------------------
// Direct kernel: one thread per point, neighbours from global memory (through
// the caches).  2D and the plain 3D variant.
// ---------------------------------------------------------------------------
template <int DIM, int R>
__global__ __launch_bounds__(256) void vti_direct(VTIStep p) {
    const int x = blockIdx.x * kTileX + threadIdx.x;
    const int y = DIM == 3 ? (int)(blockIdx.y * 4 + threadIdx.y) : 0;
    const int z = DIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * 4 + threadIdx.y);
    if (x >= p.L.nx || y >= p.L.ny || z >= p.L.nz) return;
    const int64_t pitch = p.L.pitch, plane = p.L.plane;
    const int64_t i = p.L.origin + z * plane + y * pitch + x;
    const float* __restrict__ P = p.pc;
    const float* __restrict__ Q = p.rc;
    const float pcv = P[i], rcv = Q[i];
    float lx = 0.f, ly = 0.f, lz = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) lx = fmaf(p.cx[j], P[i + j] + P[i - j], lx);
    if (DIM == 3) {
#pragma unroll
        for (int j = 1; j <= R; ++j) ly = fmaf(p.cy[j], P[i + j * pitch] + P[i - j * pitch], ly);
    }
#pragma unroll
    for (int j = 1; j <= R; ++j) lz = fmaf(p.cz[j], Q[i + j * plane] + Q[i - j * plane], lz);
    const float dh = fmaf(p.c0h, pcv, lx + ly);
    const float dzz = fmaf(p.c0z, rcv, lz);
    const float s = p.sig ? p.sig[i] : 0.f;
    float pn, rn;
    vti_update(pcv, p.pp[i], rcv, p.rp[i], p.A[i], p.e[i], p.d[i], s, dh, dzz, pn, rn);
    p.pp[i] = pn;
    p.rp[i] = rn;
}

// ---------------------------------------------------------------------------
// Tiled 3D kernel.
//
// A block owns a 64 x TY column of (x, y) and marches over a chunk of z
// planes; each lane holds one x position and VY rows.  p enters only through
// its in-plane derivatives, so the output plane of p (centre and R-wide x/y
// halo) is staged in LDS at output time; r enters only through Dzz, so its
// centre values stream through a per-lane register queue of 2R+1 planes (the
// head plane R ahead of the output), with no halo at all.  Operands are
// loaded two steps ahead into one of two register slots, the z loop is
// unrolled by the queue period 2R+2, loads and stores are raw buffer
// accesses with 32-bit offsets (ghost points read 0, their stores drop), the
// damping coefficient is read only in tile-planes flagged as damped (and
// not at all when it is a sum of per-axis profiles: SEP adds the three
// profile values), and block numbers are mapped so each XCD streams a
// contiguous run of tiles.
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(4))) int32_t cflag_t;
constexpr uint32_t kOOB = 0x80000000u;

template <int R, int NW, int VY, bool SEP>
struct TiledVTI {
    static constexpr int TY = NW * VY;
    static constexpr int LW = kTileX + 2 * R;
    static constexpr int LH = TY + 2 * R + 1;  // last row: sink for idle halo lanes
    static constexpr int U = 2 * R + 2;
    static constexpr int NYH = (2 * R + NW - 1) / NW;
    static constexpr int NXH = (2 * R * TY + 64 * NW - 1) / (64 * NW);
    static constexpr int LDS_FLOATS = LH * LW;

    const VTIStep& p;
    float* lds;
    const float *pcb, *rcb, *ab, *eb, *db, *sb, *zpl;
    float *ppb, *rpb;
    cflag_t* flags;
    int64_t plane;
    int z0, z1, nz, ty, tx, nty, ntx;
    int lane, w;
    int flagbuf;
    uint32_t oc[VY], ohy[NYH], ohx[NXH];
    int ly_[NYH], lx_[NXH];
    float q[U][VY];  // r centre values, planes z-R .. z+R
    float rh[2][VY], pcn[2][VY], hy[2][NYH], hx[2][NXH];
    float ppv[2][VY], rpv[2][VY], aa[2][VY], ee[2][VY], dd[2][VY], sg[2][VY];
    int damp[2];
    float sxl, syv[VY], ezs[2];  // SEP: profile values (x per lane, y per row, z per step)
    const __attribute__((address_space(4))) float* szc;

    __device__ TiledVTI(const VTIStep& ps, float* l) : p(ps), lds(l) {}

    __device__ __forceinline__ int flag_of(int z) const {
        if (z < 0 || z >= nz) return 0;
        return flags[((int64_t)z * nty + ty) * ntx + tx];
    }

    // Operands of the step whose output plane is zc: the r head plane zc + R,
    // p of plane zc with its halo, and p-, r-, A, e, d (and damping) of plane
    // zc.  Prefetches past the chunk read the all-zero plane.
    template <int S>
    __device__ __forceinline__ void fetch(int zc) {
        const bool out = zc < z1;
        const int64_t zo = (int64_t)zc * plane;
        const auto rr = rsrc(out ? rcb + zo + (int64_t)R * plane : zpl);
#pragma unroll
        for (int v = 0; v < VY; ++v) rh[S][v] = bload(rr, oc[v]);
        const auto rpc = rsrc(out ? pcb + zo : zpl);
#pragma unroll
        for (int v = 0; v < VY; ++v) pcn[S][v] = bload(rpc, oc[v]);
#pragma unroll
        for (int k = 0; k < NYH; ++k) hy[S][k] = bload(rpc, ohy[k]);
#pragma unroll
        for (int k = 0; k < NXH; ++k) hx[S][k] = bload(rpc, ohx[k]);
        const auto r1 = rsrc(out ? ppb + zo : zpl);
        const auto r2 = rsrc(out ? rpb + zo : zpl);
        const auto r3 = rsrc(out ? ab + zo : zpl);
        const auto r4 = rsrc(out ? eb + zo : zpl);
        const auto r5 = rsrc(out ? db + zo : zpl);
#pragma unroll
        for (int v = 0; v < VY; ++v) {
            ppv[S][v] = bload<kBufNT>(r1, oc[v]);
            rpv[S][v] = bload<kBufNT>(r2, oc[v]);
            aa[S][v] = bload<kBufNT>(r3, oc[v]);
            ee[S][v] = bload<kBufNT>(r4, oc[v]);
            dd[S][v] = bload<kBufNT>(r5, oc[v]);
        }
        const int dm = (out && flagbuf != 0) ? 1 : 0;
        flagbuf = flag_of(zc + 1);
        damp[S] = dm;
        if constexpr (SEP) {
            ezs[S] = dm ? szc[zc] : 0.f;
        } else {
            const auto rs = rsrc(dm ? sb + zo : zpl);
#pragma unroll
            for (int v = 0; v < VY; ++v) sg[S][v] = bload(rs, oc[v]);
        }
    }

    template <int K>
    __device__ __forceinline__ bool step(int z) {
        if (z >= z1) return false;
        constexpr int S = K & 1;
        constexpr int H = (K + 2 * R) % U;  // r head plane z + R
        constexpr int C = (K + R) % U;      // output plane z
#pragma unroll
        for (int v = 0; v < VY; ++v) q[H][v] = rh[S][v];
        float* tile = lds + S * LDS_FLOATS;
#pragma unroll
        for (int v = 0; v < VY; ++v) tile[(R + w * VY + v) * LW + R + lane] = pcn[S][v];
#pragma unroll
        for (int k = 0; k < NYH; ++k) tile[ly_[k]] = hy[S][k];
#pragma unroll
        for (int k = 0; k < NXH; ++k) tile[lx_[k]] = hx[S][k];
        __syncthreads();

        float cw[VY + 2 * R];
#pragma unroll
        for (int k = 0; k < VY + 2 * R; ++k) cw[k] = tile[(w * VY + k) * LW + R + lane];
        const auto rop = rsrc(ppb + (int64_t)z * plane);
        const auto ror = rsrc(rpb + (int64_t)z * plane);
        float pn[VY], rn[VY];
#pragma unroll
        for (int v = 0; v < VY; ++v) {
            const float* row = tile + (R + w * VY + v) * LW + R + lane;
            float lx = 0.f, ly = 0.f, lz = 0.f;
#pragma unroll
            for (int j = 1; j <= R; ++j) lx = fmaf(p.cx[j], row[j] + row[-j], lx);
#pragma unroll
            for (int j = 1; j <= R; ++j) ly = fmaf(p.cy[j], cw[v + R + j] + cw[v + R - j], ly);
#pragma unroll
            for (int j = 1; j <= R; ++j)
                lz = fmaf(p.cz[j], q[(C + j) % U][v] + q[(C + U - j) % U][v], lz);
            const float dh = fmaf(p.c0h, pcn[S][v], lx + ly);
            const float dzz = fmaf(p.c0z, q[C][v], lz);
            vti_update(pcn[S][v], ppv[S][v], q[C][v], rpv[S][v], aa[S][v], ee[S][v], dd[S][v],
                       damp[S] ? (SEP ? (sxl + syv[v]) + ezs[S] : sg[S][v]) : 0.f, dh, dzz,
                       pn[v], rn[v]);
        }
#pragma unroll
        for (int v = 0; v < VY; ++v) {
            bstore_nt(rop, oc[v], pn[v]);
            bstore_nt(ror, oc[v], rn[v]);
        }
        fetch<S>(z + 2);
        return true;
    }

    template <int... Ks>
    __device__ __forceinline__ bool period(int zb, std::integer_sequence<int, Ks...>) {
        return (step<Ks>(zb + Ks) && ...);
    }

    __device__ void run() {
        const int b = blockIdx.x;
        const int t = (b & 7) * (p.nblocks >> 3) + (b >> 3);
        if (t >= p.ntiles) return;
        ntx = p.ntx;
        nty = p.nty;
        tx = t % ntx;
        const int t2 = t / ntx;
        ty = t2 % nty;
        const int zc = t2 / nty;
        const int x0 = tx * kTileX, y0 = ty * TY;
        const int nx = p.L.nx, ny = p.L.ny;
        nz = p.L.nz;
        z0 = zc * p.zchunk;
        z1 = min(z0 + p.zchunk, nz);
        const int tid = threadIdx.x;
        lane = tid & 63;
        w = tid >> 6;
        plane = p.L.plane;
        const int pitch = p.L.pitch;
        const int64_t org = p.L.origin + (int64_t)(y0 - R) * pitch + (x0 - R);
        pcb = p.pc + org;
        rcb = p.rc + org;
        ppb = p.pp + org;
        rpb = p.rp + org;
        ab = p.A + org;
        eb = p.e + org;
        db = p.d + org;
        sb = (p.sig ? p.sig : p.A) + org;
        zpl = p.A + org - (int64_t)kGhostYZ * plane;
        flags = (cflag_t*)p.dflag;
        sxl = 0.f;
#pragma unroll
        for (int v = 0; v < VY; ++v) syv[v] = 0.f;
        if constexpr (SEP) {
            // the same sum, in the same order, as the setup's check; lanes and
            // rows past the interior read the last value (their stores drop)
            szc = (const __attribute__((address_space(4))) float*)p.sz;
            sxl = p.sx[min(x0 + lane, nx - 1)];
#pragma unroll
            for (int v = 0; v < VY; ++v) syv[v] = p.sy[min(y0 + w * VY + v, ny - 1)];
        }
        auto off = [&](int r, int c) -> uint32_t {
            const int y = y0 - R + r, x = x0 - R + c;
            return (x >= 0 && x < nx && y >= 0 && y < ny) ? (uint32_t)((r * pitch + c) * 4)
                                                           : kOOB;
        };
#pragma unroll
        for (int v = 0; v < VY; ++v) oc[v] = off(R + w * VY + v, R + lane);
        const int sink = (LH - 1) * LW + lane;
#pragma unroll
        for (int k = 0; k < NYH; ++k) {
            const int hr = w + k * NW;
            const int row = hr < R ? hr : TY + hr;
            const bool on = hr < 2 * R;
            ohy[k] = on ? off(row, R + lane) : kOOB;
            ly_[k] = on ? row * LW + R + lane : sink;
        }
#pragma unroll
        for (int k = 0; k < NXH; ++k) {
            const int e = tid + k * 64 * NW;
            const int row = e / (2 * R), cc = e % (2 * R);
            const int col = cc < R ? cc : kTileX + cc;
            const bool on = e < 2 * R * TY;
            ohx[k] = on ? off(R + row, col) : kOOB;
            lx_[k] = on ? (R + row) * LW + col : (LH - 1) * LW + (tid & 63);
        }
        // queue index i holds r plane z0 - R + i (mod U); planes z0-R ..
        // z0+R-1 are primed here, the loop's first head is z0+R
#pragma unroll
        for (int i = 0; i < U; ++i)
#pragma unroll
            for (int v = 0; v < VY; ++v) q[i][v] = 0.f;
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) {
            const auto r = rsrc(rcb + (int64_t)(z0 - R + i) * plane);
#pragma unroll
            for (int v = 0; v < VY; ++v) q[i][v] = bload(r, oc[v]);
        }
        flagbuf = flag_of(z0);
        fetch<0>(z0);
        fetch<1>(z0 + 1);
        for (int zb_ = z0; period(zb_, std::make_integer_sequence<int, U>{}); zb_ += U) {
        }
    }
};

template <int R, int NW, int VY, bool SEP>
__global__ __launch_bounds__(64 * NW) void vti3d_tiled(VTIStep p) {
    __shared__ float lds[2 * TiledVTI<R, NW, VY, SEP>::LDS_FLOATS];
    TiledVTI<R, NW, VY, SEP> k(p, lds);
    k.run();
}

template <int R>
hipError_t launch_direct(const VTIStep& p, int ndim, hipStream_t s) {
    const int gx = (p.L.nx + kTileX - 1) / kTileX;
    if (ndim == 2)
        hipLaunchKernelGGL((vti_direct<2, R>), dim3(gx, (p.L.nz + 3) / 4), dim3(64, 4), 0, s, p);
    else
        hipLaunchKernelGGL((vti_direct<3, R>), dim3(gx, (p.L.ny + 3) / 4, p.L.nz), dim3(64, 4),
                           0, s, p);
    return hipGetLastError();
}

template <int R>
hipError_t launch_tiled(const VTIStep& p, hipStream_t s) {
    constexpr int NW = kVTITile.waves, VY = kVTITile.rows;
    if (p.sx)
        hipLaunchKernelGGL((vti3d_tiled<R, NW, VY, true>), dim3(p.nblocks), dim3(64 * NW), 0, s,
                           p);
    else
        hipLaunchKernelGGL((vti3d_tiled<R, NW, VY, false>), dim3(p.nblocks), dim3(64 * NW), 0, s,
                           p);
    return hipGetLastError();
}

}  // namespace

int vti_tile_y() { return kVTITile.height(); }

hipError_t launch_vti(const VTIStep& p, int ndim, int radius, int variant, hipStream_t s) {
    const bool tiled = ndim == 3 && variant == 0;
#define FD_VCASE(RR) \
    case RR: return tiled ? launch_tiled<RR>(p, s) : launch_direct<RR>(p, ndim, s);
    switch (radius) {
        FD_VCASE(1)
        FD_VCASE(2)
        FD_VCASE(3)
        FD_VCASE(4)
        FD_VCASE(5)
        FD_VCASE(6)
        FD_VCASE(7)
        FD_VCASE(8)
        default: return hipErrorInvalidValue;
    }
#undef FD_VCASE
}

}  // namespace fd
