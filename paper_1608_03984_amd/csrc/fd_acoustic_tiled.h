// fd_acoustic_tiled.h -- the tiled 3D acoustic leapfrog kernel of libfd
// (gfx950), included by the translation units that instantiate it (space
// orders are split between them so that they compile in parallel).
//
// One launch advances every point of the padded volume by one step of
// Algorithm 1 for Eq. (Acou) with the damping layer:
//   u^{n+1} = [2 u^n - (1 - s) u^{n-1} + A L u^n] / (1 + s),  A = dt^2 v^2,
// written over u^{n-1}.  L is the star-shaped Laplacian of radius R whose
// per-axis weights arrive pre-divided by h^2; symmetric neighbours are summed
// before they are weighted.  Algorithmic traffic per point: read u^n, u^{n-1}
// and A, write u^{n+1} = 16 bytes (section 4.2); s is read only in tiles that
// hold damping, and not at all when it is a sum of per-axis profiles (the
// kernel then adds the three profile values).  For gradients a launch can
// also store the acceleration term A L u^n of every point (4 more bytes
// written), which the imaging condition correlates with the adjoint field.
#pragma once

#include "fd_internal.h"

#include <utility>

namespace fd {

namespace {


__device__ inline float update(float c, float prev, float a, float lap, float s) {
    if (s == 0.f) return fmaf(a, lap, 2.f * c - prev);
    return (2.f * c - (1.f - s) * prev + a * lap) / (1.f + s);
}

// Raw buffer access: a uniform base pointer (one per plane, held in SGPRs)
// plus a per-lane 32-bit byte offset.  aux 2 marks streaming (non-temporal)
// accesses.  The record limit only has to exceed the largest in-tile offset.
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

// ---------------------------------------------------------------------------
// Tiled 3D kernel (2.5D blocking).
//
// A block owns a 64 x TY column of (x, y) and marches over a chunk of z
// planes; each lane holds one x position and VY consecutive rows.
//
// Plane p enters the block once, as the "head" of the z pipeline, R planes
// before it becomes the output plane.  On arrival its centre values and its
// R-wide x/y halo are staged in LDS and the in-plane part of the Laplacian,
// Lx + Ly, is computed for the lane's points; the centre values go into a
// register queue (2R+1 planes, for the z derivative) and Lx + Ly into an LDS
// ring (R+1 planes, each lane reading back only what it wrote) until the
// plane is output.  Loading the halo of the
// head plane -- rather than of the output plane -- means a tile reads its
// neighbours' rows at the moment the neighbours stream the same plane in, so
// the halo re-reads hit in L2 instead of going back to memory.
//
// The operands of a step (head centre and halo, and u^{n-1}, A, damping of
// the output plane) are loaded two steps ahead into one of two register
// slots.  Every step issues the same loads and the z loop is unrolled by the
// queue period U = 2R+2, so queues and slots rotate by compile-time index and
// the compiler waits for exactly the slot it needs.  Loads and stores are
// raw buffer accesses: a uniform per-plane base in SGPRs plus a per-lane
// 32-bit offset.  Offsets of points outside the interior are set past the
// buffer's record limit, so ghost points read as zero without any memory
// traffic and their stores are dropped.  Undamped tiles, and the steps that
// produce no output, read their operands from an all-zero ghost plane that
// stays cached; the per-plane damping flag is a scalar load issued one step
// ahead.
//
// Blocks are numbered so that the 8 XCDs (which receive blocks round-robin)
// each get a contiguous run of tiles: neighbours that share halo rows run on
// the same XCD and find them in its L2.
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(4))) int32_t cflag_t;
constexpr uint32_t kOOB = 0x80000000u;  // any offset at or past the record limit reads 0
constexpr int kRecords = 0x7fffffff;


// Operand buffering of the tiled acoustic kernel: true = two register slots,
// each step's operands loaded two steps ahead; false = one slot, the next
// head plane loaded right after the current one is staged and the next
// output plane's operands right after the update (half the operand
// registers and fewer spilled scalar registers, about one step of latency
// hiding).  Measured at 592^3 (same bits either way): one slot is faster
// for the 64 x 24 tile (so 4: 576 against 585 us) and one shot per block at
// radius 6 and 8 (so 12 / 16: 669 / 709 against 673 / 717 us), two slots
// at radius 4 (so 8: 625 against 655 us, where the deeper prefetch matters
// and the registers do not change the occupancy).
template <int R, int NW, int VY, int SB>
constexpr bool acoustic_double_buffer() { return !(NW == 12 || (SB == 1 && R >= 6)); }

template <int R, int NW, int VY, int SB, bool ACC, bool SEP, bool IMG>
struct TiledAcoustic {
    static_assert(!IMG || !ACC, "fused imaging is an adjoint step (no acceleration output)");
    static constexpr bool DB = acoustic_double_buffer<R, NW, VY, SB>();
    static constexpr int NS = DB ? 2 : 1;  // operand register slots
    static constexpr int TY = NW * VY;
    static constexpr int LW = kTileX + 2 * R;
    static constexpr int LH = TY + 2 * R + 1;  // last row: sink for idle halo lanes
    static constexpr int U = 2 * R + 2;
    static constexpr int NYH = (2 * R + NW - 1) / NW;
    static constexpr int NXH = (2 * R * TY + 64 * NW - 1) / (64 * NW);
    static constexpr int LDS_FLOATS = LH * LW;
    static constexpr int LQ_FLOATS = (R + 1) * TY * kTileX;  // ring of Lx + Ly, R+1 planes
    static constexpr int SMEM_FLOATS = SB * (2 * LDS_FLOATS + LQ_FLOATS);

    const AcousticStep& p;
    float* lds;
    const float* ub[SB];  // tile origin (x0 - R, y0 - R) of u^n, plane 0, per shot
    float* pb[SB];        // same for u^{n-1} / u^{n+1}
    int lim[SB];          // store record limit: 0 for the padding shots of a ragged group
    float* cb[SB];        // same for the acceleration output (ACC), per shot
    const float* iab[SB]; // IMG: the acceleration the output point's u^n images with
    float* igb[SB];       // IMG: the FP32 partial sum of the imaging condition
    float ia[NS][SB][VY], ig[NS][SB][VY];
    const float* ab;      // same for A (shared by the shots)
    const float* sb;      // same for the damping coefficient
    const float* zpl;     // an all-zero plane (ghost plane of A) at the tile origin
    cflag_t* flags;
    int64_t plane;
    int z0, z1, nz, ty, tx, nty, ntx;
    int lane, w;
    int flagbuf;      // damping flag of the next plane to fetch
    uint32_t oc[VY], ohy[NYH], ohx[NXH];  // byte offsets inside the tile (kOOB outside)
    int ly_[NYH], lx_[NXH];
    float q[SB][U][VY];  // centre values, planes z-R .. z+R
    float nxt[NS][SB][VY], prv[NS][SB][VY], hy[NS][SB][NYH], hx[NS][SB][NXH];
    float aa[NS][VY], sg[NS][VY];
    int damp[NS];
    // SEP: damping from the per-axis profiles (p.sx, p.sy, p.sz), evaluated at
    // use; the z value of a step is a scalar load issued with its operands
    float sxl, syv[VY];   // this lane's x profile value and its rows' y values
    float ezs[NS];
    const __attribute__((address_space(4))) float* szc;

    __device__ TiledAcoustic(const AcousticStep& ps, float* l) : p(ps), lds(l) {}

    // staging tile of shot s, buffer T (the step's parity); LDS ring of
    // Lx + Ly of shot s (planes z .. z+R, slot (plane - zs) mod (R+1), each
    // lane reading back only what it wrote)
    __device__ __forceinline__ float* tile_of(int s, int T) const {
        return lds + (2 * s + T) * LDS_FLOATS;
    }
    __device__ __forceinline__ float* ring_of(int s) const {
        return lds + 2 * SB * LDS_FLOATS + s * LQ_FLOATS;
    }

    __device__ __forceinline__ int flag_of(int z) const {
        if (z < 0 || z >= nz) return 0;
        return flags[((int64_t)z * nty + ty) * ntx + tx];
    }

    // Operands of the step whose output plane is zc: the head plane zc + R
    // (centre and halo) of every shot (fetch_head) and u^{n-1} of plane zc,
    // with A and damping of plane zc loaded once for all shots (fetch_out).
    // Head planes beyond the grid are zero ghost planes of the volume; the
    // operands of a step without output come from the all-zero plane.
    template <int S>
    __device__ __forceinline__ void fetch_head(int zc) {
#pragma unroll
        for (int s = 0; s < SB; ++s) {
            const auto rh = rsrc(ub[s] + (int64_t)(zc + R) * plane);
#pragma unroll
            for (int v = 0; v < VY; ++v) nxt[S][s][v] = bload(rh, oc[v]);
#pragma unroll
            for (int k = 0; k < NYH; ++k) hy[S][s][k] = bload(rh, ohy[k]);
#pragma unroll
            for (int k = 0; k < NXH; ++k) hx[S][s][k] = bload(rh, ohx[k]);
        }
    }
    template <int S>
    __device__ __forceinline__ void fetch(int zc) {
        fetch_head<S>(zc);
        fetch_out<S>(zc);
    }
    template <int S>
    __device__ __forceinline__ void fetch_out(int zc) {
        const bool out = zc >= z0 && zc < z1;
        const int64_t zo = (int64_t)zc * plane;
        const auto ra = rsrc(out ? ab + zo : zpl);
#pragma unroll
        for (int v = 0; v < VY; ++v) {
#pragma unroll
            for (int s = 0; s < SB; ++s) {
                const auto rp = rsrc(out ? pb[s] + zo : zpl);
                prv[S][s][v] = bload<kBufNT>(rp, oc[v]);
            }
            aa[S][v] = bload<kBufNT>(ra, oc[v]);
        }
        if constexpr (IMG) {
#pragma unroll
            for (int s = 0; s < SB; ++s) {
                const auto ri = rsrc(out ? iab[s] + zo : zpl), rg = rsrc(out ? igb[s] + zo : zpl);
#pragma unroll
                for (int v = 0; v < VY; ++v) {
                    ia[S][s][v] = bload<kBufNT>(ri, oc[v]);
                    ig[S][s][v] = bload<kBufNT>(rg, oc[v]);
                }
            }
        }
        const int d = (out && flagbuf != 0) ? 1 : 0;
        flagbuf = flag_of(zc + 1);
        damp[S] = d;
        if constexpr (SEP) {
            ezs[S] = d ? szc[zc] : 0.f;
        } else {
            const auto rs = rsrc(d ? sb + zo : zpl);
#pragma unroll
            for (int v = 0; v < VY; ++v) sg[S][v] = bload(rs, oc[v]);
        }
    }

    template <int K>
    __device__ __forceinline__ bool step(int z) {
        if (z >= z1) return false;
        constexpr int S = DB ? (K & 1) : 0;  // operand register slot
        constexpr int T = K & 1;             // LDS staging buffer
        constexpr int H = (K + 2 * R) % U;  // head plane z + R
        constexpr int C = (K + R) % U;      // output plane z
#pragma unroll
        for (int s = 0; s < SB; ++s) {
#pragma unroll
            for (int v = 0; v < VY; ++v) q[s][H][v] = nxt[S][s][v];
            float* tile = tile_of(s, T);
#pragma unroll
            for (int v = 0; v < VY; ++v) tile[(R + w * VY + v) * LW + R + lane] = q[s][H][v];
#pragma unroll
            for (int k = 0; k < NYH; ++k) tile[ly_[k]] = hy[S][s][k];
#pragma unroll
            for (int k = 0; k < NXH; ++k) tile[lx_[k]] = hx[S][s][k];
        }
        // one slot: the next head plane's registers are free once staged
        if constexpr (!DB) fetch_head<0>(z + 1);
        __syncthreads();

        // in-plane Laplacian of the head plane
#pragma unroll
        for (int s = 0; s < SB; ++s) {
            const float* tile = tile_of(s, T);
            float cw[VY + 2 * R];
#pragma unroll
            for (int k = 0; k < VY + 2 * R; ++k) cw[k] = tile[(w * VY + k) * LW + R + lane];
#pragma unroll
            for (int v = 0; v < VY; ++v) {
                const float* row = tile + (R + w * VY + v) * LW + R + lane;
                float lx = 0.f, ly = 0.f;
#pragma unroll
                for (int j = 1; j <= R; ++j) lx = fmaf(p.cx[j], row[j] + row[-j], lx);
#pragma unroll
                for (int j = 1; j <= R; ++j) ly = fmaf(p.cy[j], cw[v + R + j] + cw[v + R - j], ly);
                ring_of(s)[((K + R) % (R + 1)) * TY * kTileX + (w * VY + v) * kTileX + lane] =
                    lx + ly;
            }
        }

        // output plane z; the R steps before the chunk store nothing (their
        // store buffer has a zero record limit), so every step issues the
        // same memory operations
#pragma unroll
        for (int s = 0; s < SB; ++s) {
            const auto ro = __builtin_amdgcn_make_buffer_rsrc(pb[s] + (int64_t)z * plane, 0,
                                                              z >= z0 ? lim[s] : 0, 0x00020000);
            float nv[VY], av[VY];
#pragma unroll
            for (int v = 0; v < VY; ++v) {
                float lz = 0.f;
#pragma unroll
                for (int j = 1; j <= R; ++j)
                    lz = fmaf(p.cz[j], q[s][(C + j) % U][v] + q[s][(C + U - j) % U][v], lz);
                const float lxy =
                    ring_of(s)[(K % (R + 1)) * TY * kTileX + (w * VY + v) * kTileX + lane];
                const float lap = fmaf(p.c0, q[s][C][v], lxy + lz);
                av[v] = aa[S][v] * lap;
                nv[v] = fmaf(aa[S][v], lap, 2.f * q[s][C][v] - prv[S][s][v]);
                if (damp[S]) {
                    // the profile sum in the same order as the setup's check
                    const float sv = SEP ? (sxl + syv[v]) + ezs[S] : sg[S][v];
                    nv[v] = (2.f * q[s][C][v] - (1.f - sv) * prv[S][s][v] + aa[S][v] * lap) /
                            (1.f + sv);
                }
            }
#pragma unroll
            for (int v = 0; v < VY; ++v) bstore_nt(ro, oc[v], nv[v]);
            if constexpr (ACC) {
                const auto rc = __builtin_amdgcn_make_buffer_rsrc(
                    cb[s] + (int64_t)z * plane, 0, z >= z0 ? lim[s] : 0, 0x00020000);
#pragma unroll
                for (int v = 0; v < VY; ++v) bstore_nt(rc, oc[v], av[v]);
            }
            if constexpr (IMG) {
                // the same fmaf as the separate imaging kernel
                const auto rg = __builtin_amdgcn_make_buffer_rsrc(
                    igb[s] + (int64_t)z * plane, 0, z >= z0 ? lim[s] : 0, 0x00020000);
#pragma unroll
                for (int v = 0; v < VY; ++v)
                    bstore_nt(rg, oc[v], fmaf(q[s][C][v], ia[S][s][v], ig[S][s][v]));
            }
        }
        if constexpr (DB)
            fetch<S>(z + 2);
        else
            fetch_out<0>(z + 1);
        return true;
    }

    template <int... Ks>
    __device__ __forceinline__ bool period(int zb, std::integer_sequence<int, Ks...>) {
        return (step<Ks>(zb + Ks) && ...);
    }

    __device__ void run() {
        const int b = blockIdx.x;
        int t, group;
        if (p.slab > 0) {
            // pass-major: XCD b & 7 takes tiles [(b & 7) slab, (b & 7 + 1) slab)
            // of pass (b >> 3) / slab; groups vary fastest over the passes
            const int j = b >> 3, pass = j / p.slab;
            const int txy = (b & 7) * p.slab + j % p.slab;
            if (txy >= p.ntx * p.nty) return;
            group = pass % p.ngroups;
            t = txy + (pass / p.ngroups) * (p.ntx * p.nty);
        } else {
            const int item = (b & 7) * (p.nblocks >> 3) + (b >> 3);
            if (item >= p.ntiles * p.ngroups) return;
            t = item % p.ntiles;
            group = item / p.ntiles;
        }
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
#pragma unroll
        for (int s = 0; s < SB; ++s) {
            // padding shots of a ragged last group re-read the last shot and
            // store nothing
            const int shot = group * SB + s;
            const int se = shot < p.nshots ? shot : p.nshots - 1;
            ub[s] = p.uc + se * p.shot_stride + org;
            pb[s] = p.up + se * p.shot_stride + org;
            lim[s] = shot < p.nshots ? kRecords : 0;
        }
        ab = p.A + org;
#pragma unroll
        for (int s = 0; s < SB; ++s) {
            // shot s of the acceleration and imaging volumes (the padding
            // shots of a ragged group re-read the last shot and store nothing)
            const int shot = group * SB + s;
            const int64_t so = (int64_t)(shot < p.nshots ? shot : p.nshots - 1) * p.shot_stride;
            cb[s] = ACC ? p.acc + so + org : pb[s];
            iab[s] = IMG ? p.img_a + so + org : ab;
            igb[s] = IMG ? p.img_g + so + org : pb[s];
        }
        sb = (p.sig ? p.sig : p.A) + org;
        zpl = p.A + org - (int64_t)kGhostYZ * plane;
        flags = (cflag_t*)p.dflag;
        sxl = 0.f;
#pragma unroll
        for (int v = 0; v < VY; ++v) syv[v] = 0.f;
        if constexpr (SEP) {
            szc = (const __attribute__((address_space(4))) float*)p.sz;
            // lanes and rows past the interior read the last value; their
            // stores are dropped
            sxl = p.sx[min(x0 + lane, nx - 1)];
#pragma unroll
            for (int v = 0; v < VY; ++v) syv[v] = p.sy[min(y0 + w * VY + v, ny - 1)];
        }
        // offsets of tile point (row r, column c), r/c counted from (y0 - R, x0 - R)
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
        // The loop starts R steps before the chunk so that planes z0 .. z0+R-1
        // enter as heads; those steps produce no output.  Queue index i holds
        // plane zs - R + i (mod U); planes z0-R .. z0-1 are primed here.
        const int zs = z0 - R;
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int i = 0; i < U; ++i)
#pragma unroll
                for (int v = 0; v < VY; ++v) q[s][i][v] = 0.f;
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int i = R; i < 2 * R; ++i) {
                const auto r = rsrc(ub[s] + (int64_t)(zs - R + i) * plane);
#pragma unroll
                for (int v = 0; v < VY; ++v) q[s][i][v] = bload(r, oc[v]);
            }
        flagbuf = flag_of(zs);
        fetch<0>(zs);
        if constexpr (DB) fetch<1>(zs + 1);
        for (int zb_ = zs; period(zb_, std::make_integer_sequence<int, U>{}); zb_ += U) {
        }
    }
};

template <int R, int NW, int VY, int SB, bool ACC, bool SEP, bool IMG>
__global__ __launch_bounds__(64 * NW) void acoustic3d_tiled(AcousticStep p) {
    using T = TiledAcoustic<R, NW, VY, SB, ACC, SEP, IMG>;
    __shared__ float lds[T::SMEM_FLOATS];
    T k(p, lds);
    k.run();
}

// Configuration CFG of kAcousticTiles with SB shots per block; the
// acceleration-output and fused-imaging variants exist where acc_built /
// img_built say so.
template <int R, int CFG, int SB, bool SEP>
hipError_t launch_tiled_sep(const AcousticStep& p, hipStream_t s) {
    constexpr int NW = kAcousticTiles[CFG].waves, VY = kAcousticTiles[CFG].rows;
    if (p.acc) {
        if constexpr (acc_built(CFG, SB)) {
            hipLaunchKernelGGL((acoustic3d_tiled<R, NW, VY, SB, true, SEP, false>),
                               dim3(p.nblocks), dim3(64 * NW), 0, s, p);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (p.img_a) {
        if constexpr (img_built(CFG, SB)) {
            hipLaunchKernelGGL((acoustic3d_tiled<R, NW, VY, SB, false, SEP, true>),
                               dim3(p.nblocks), dim3(64 * NW), 0, s, p);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((acoustic3d_tiled<R, NW, VY, SB, false, SEP, false>), dim3(p.nblocks),
                       dim3(64 * NW), 0, s, p);
    return hipGetLastError();
}

// Tile configurations: 0 = 64 x 8 (4 waves x 2 rows), 1 = 64 x 16 (4 x 4),
// 2 = 64 x 8 (8 waves x 1 row), 3 = 64 x 16 (8 x 2), 4 = 64 x 24 (12 x 2).
// Shots per block 2 and 4 are built for configurations 0 and 2.
template <int R, int CFG, int SB>
hipError_t launch_tiled_t(const AcousticStep& p, hipStream_t s) {
    return p.sx ? launch_tiled_sep<R, CFG, SB, true>(p, s)
                : launch_tiled_sep<R, CFG, SB, false>(p, s);
}

template <int R>
hipError_t launch_tiled_cfg(const AcousticStep& p, int cfg, int sb, hipStream_t s) {
    if (sb == 1) {
        switch (cfg) {
            case 0: return launch_tiled_t<R, 0, 1>(p, s);
            case 1: return launch_tiled_t<R, 1, 1>(p, s);
            case 2: return launch_tiled_t<R, 2, 1>(p, s);
            case 3: return launch_tiled_t<R, 3, 1>(p, s);
            case 4: return launch_tiled_t<R, 4, 1>(p, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (cfg == 0 && sb == 2) return launch_tiled_t<R, 0, 2>(p, s);
    if (cfg == 0 && sb == 4) return launch_tiled_t<R, 0, 4>(p, s);
    if (cfg == 2 && sb == 2) return launch_tiled_t<R, 2, 2>(p, s);
    if (cfg == 2 && sb == 4) return launch_tiled_t<R, 2, 4>(p, s);
    return hipErrorInvalidValue;
}

}  // namespace

}  // namespace fd
