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

#include <utility>

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

// ---------------------------------------------------------------------------
// Tiled TTI kernel (2.5D blocking), one row per lane, 64 x NW tiles.
//
// Each plane of p and r enters the block once, as the head of the z pipeline,
// R planes before it is output, staged in LDS with its full R-wide halo
// (corners included: the mixed derivative needs them).  At head time the
// lane computes, for f in {p, r}:
//   Dxx f, Dyy f, gx = D1x f, gy = D1y f (gy also on the x-halo columns, into
//   an LDS tile), then Dxy f = D1x(gy);
//   the in-plane parts  Dxx p + Dyy p  and  c1 Dxx f + c2 Dyy f + c4 Dxy f
//   (c1, c2, c4 of the head plane), parked in an LDS ring until output.
// f, gx and gy go into per-lane register queues of the 2R+1 planes of the
// output plane's z stencil; at output time
//   Dzz f = D2z(f queue),  Dxz f = D1z(gx queue),  Dyz f = D1z(gy queue),
// which is the product-of-first-derivatives form of the mixed terms (the
// same sum the zero-ghost stencil gives).  G_zbar_zbar f adds c3 Dzz + c5 Dyz
// + c6 Dxz (c's of the output plane), H p = Laplacian p - G_zbar_zbar p, and
// the update of Eq. (TTI) writes p^{n+1}, r^{n+1} over p^{n-1}, r^{n-1}.
//
// Registers decide the occupancy of this kernel (six queues of 2R+1 planes
// per lane), so its operands are single-buffered and loaded half a step
// ahead, each group as soon as its registers are free: the next head plane's
// values right after they were staged in LDS, the head plane's c1, c2, c4
// right after the in-plane parts are formed, and the output plane's fields
// and coefficients right after the update.  The z loop is unrolled by the
// queue period 2R+1 so that queue slots are compile-time registers; the LDS
// ring slot is a block-uniform counter.  Loads and stores are raw buffer
// accesses with out-of-range offsets for ghost points, and the 2R steps
// before a chunk only fill the pipeline (their stores have a zero record
// limit).  Two barriers per step: one after staging p and r, one after
// staging gy.  A damping layer that is a sum of per-axis profiles (SEP) is
// evaluated from the three profile values instead of read.
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(4))) int32_t tflag_t;
constexpr uint32_t kOOBt = 0x80000000u;
constexpr int kRecordsT = 0x7fffffff;
constexpr int kNT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t trsrc(const float* base, int rec = kRecordsT) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, rec, 0x00020000);
}
template <int AUX = 0>
__device__ __forceinline__ float tload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
__device__ __forceinline__ void tstore(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, kNT);
}

template <int R, int NW, bool SEP>
struct TiledTTI {
    static constexpr int TY = NW;  // one row per wave
    static constexpr int LW = kTileX + 2 * R;
    static constexpr int LH = TY + 2 * R;
    static constexpr int FT = (LH + 1) * LW;  // staged field tile (+1 sink row)
    static constexpr int GT = TY * LW;        // gy on the x-extended rows
    static constexpr int U = 2 * R + 1;       // queue period: planes z-R .. z+R
    static constexpr int NHALO = LH * LW - TY * kTileX;
    static constexpr int NH = (NHALO + 64 * NW - 1) / (64 * NW);
    static constexpr int NGX = 2 * R * TY;     // x-halo gy points
    static constexpr int RING = (R + 1) * TY * kTileX;
    static constexpr int LDS_FLOATS = 2 * FT + 2 * GT + 3 * RING;

    const TTIStep& p;
    float* fp_t;   // staged p tile
    float* fr_t;   // staged r tile
    float* gp_t;   // gy of p
    float* gr_t;   // gy of r
    float* ring;   // [3][R+1][TY][64]: Dxx p + Dyy p, c1 Dxx p + c2 Dyy p + c4 Dxy p, same for r
    const float *pb, *rb, *ab, *eb, *db, *sb, *zpl;
    const float* cb[6];
    float *ppb, *rpb;
    tflag_t* flags;
    int64_t plane;
    int z0, z1, nz, tx, ty, ntx, nty, lane, w, tid;
    int flagbuf;
    int rslot;              // ring slot of the head plane; the output plane's is rslot + 1
    uint32_t oc;            // own point offset (kOOBt outside the interior)
    uint32_t oh[NH];        // halo element offsets
    int lh[NH];             // halo element LDS index
    bool gx_on;             // this thread computes one x-halo gy point
    int gxf, gxg;           // its f-tile index (row, col) and gy-tile index
    float fqp[U], fqr[U], gxp[U], gxr[U], gyp[U], gyr[U];
    // operands, one buffer each (loaded half a step ahead)
    float hp_c, hr_c, hp_h[NH], hr_h[NH];      // head plane: centre and halo of p, r
    float c1h, c2h, c4h;                        // head plane: in-plane G_zbar_zbar weights
    float opp, orp, oa, oe, od, oc3, oc5, oc6, osg;  // output plane
    int damp;
    float sxy;  // SEP: this lane's x profile value plus its row's y value
    const __attribute__((address_space(4))) float* szc;

    __device__ TiledTTI(const TTIStep& ps, float* lds) : p(ps) {
        fp_t = lds;
        fr_t = lds + FT;
        gp_t = lds + 2 * FT;
        gr_t = lds + 2 * FT + GT;
        ring = lds + 2 * FT + 2 * GT;
    }

    __device__ __forceinline__ int flag_of(int z) const {
        if (z < 0 || z >= nz) return 0;
        return flags[((int64_t)z * nty + ty) * ntx + tx];
    }

    // centre and halo of p and r at head plane zh (beyond the grid: zero
    // ghost planes of the volume)
    __device__ __forceinline__ void fetch_head(int zh) {
        const int64_t o = (int64_t)zh * plane;
        const auto rp = trsrc(pb + o), rr = trsrc(rb + o);
        hp_c = tload(rp, oc);
        hr_c = tload(rr, oc);
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            hp_h[k] = tload(rp, oh[k]);
            hr_h[k] = tload(rr, oh[k]);
        }
    }
    __device__ __forceinline__ void fetch_head_coef(int zh) {
        const int64_t o = (int64_t)zh * plane;
        c1h = tload<kNT>(trsrc(cb[0] + o), oc);
        c2h = tload<kNT>(trsrc(cb[1] + o), oc);
        c4h = tload<kNT>(trsrc(cb[3] + o), oc);
    }
    // fields and coefficients of output plane zc (steps without output read
    // the all-zero plane), and its damping flag
    __device__ __forceinline__ void fetch_out(int zc) {
        const bool out = zc >= z0 && zc < z1;
        const int64_t zo = (int64_t)zc * plane;
        opp = tload<kNT>(trsrc(out ? ppb + zo : zpl), oc);
        orp = tload<kNT>(trsrc(out ? rpb + zo : zpl), oc);
        oa = tload<kNT>(trsrc(out ? ab + zo : zpl), oc);
        oe = tload<kNT>(trsrc(out ? eb + zo : zpl), oc);
        od = tload<kNT>(trsrc(out ? db + zo : zpl), oc);
        oc3 = tload<kNT>(trsrc(out ? cb[2] + zo : zpl), oc);
        oc5 = tload<kNT>(trsrc(out ? cb[4] + zo : zpl), oc);
        oc6 = tload<kNT>(trsrc(out ? cb[5] + zo : zpl), oc);
        const int d = (out && flagbuf != 0) ? 1 : 0;
        flagbuf = flag_of(zc + 1);
        damp = d;
        if constexpr (SEP)
            osg = d ? szc[zc] : 0.f;  // the z value; the sum is formed at use
        else
            osg = tload(trsrc(d ? sb + zo : zpl), oc);
    }

    template <int K>
    __device__ __forceinline__ bool step(int z) {
        if (z >= z1) return false;
        constexpr int H = (K + 2 * R) % U;  // queue slot of the head plane z + R
        constexpr int C = (K + R) % U;      // queue slot of the output plane z
        const int rh = rslot, rc = rslot == R ? 0 : rslot + 1;  // ring slots (head, output)
        const int fc = (R + w) * LW + R + lane;  // own point in the field tile
        // stage the head planes of p and r
        fqp[H] = hp_c;
        fqr[H] = hr_c;
        fp_t[fc] = hp_c;
        fr_t[fc] = hr_c;
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            fp_t[lh[k]] = hp_h[k];
            fr_t[lh[k]] = hr_h[k];
        }
        __syncthreads();
        fetch_head(z + 1 + R);

        // first and second derivatives of the head plane at the own point
        float dxx_p = p.w2x[0] * fp_t[fc], dxx_r = p.w2x[0] * fr_t[fc];
        float dyy_p = p.w2y[0] * fp_t[fc], dyy_r = p.w2y[0] * fr_t[fc];
        float gx_p = 0.f, gx_r = 0.f, gy_p = 0.f, gy_r = 0.f;
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const float ap = fp_t[fc + j], bp = fp_t[fc - j];
            const float ar = fr_t[fc + j], br = fr_t[fc - j];
            dxx_p = fmaf(p.w2x[j], ap + bp, dxx_p);
            dxx_r = fmaf(p.w2x[j], ar + br, dxx_r);
            gx_p = fmaf(p.w1x[j], ap - bp, gx_p);
            gx_r = fmaf(p.w1x[j], ar - br, gx_r);
            const float cp = fp_t[fc + j * LW], dp = fp_t[fc - j * LW];
            const float cr = fr_t[fc + j * LW], dr = fr_t[fc - j * LW];
            dyy_p = fmaf(p.w2y[j], cp + dp, dyy_p);
            dyy_r = fmaf(p.w2y[j], cr + dr, dyy_r);
            gy_p = fmaf(p.w1y[j], cp - dp, gy_p);
            gy_r = fmaf(p.w1y[j], cr - dr, gy_r);
        }
        gxp[H] = gx_p;
        gxr[H] = gx_r;
        gyp[H] = gy_p;
        gyr[H] = gy_r;
        const int gc = w * LW + R + lane;
        gp_t[gc] = gy_p;
        gr_t[gc] = gy_r;
        if (gx_on) {
            float a = 0.f, b = 0.f;
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                a = fmaf(p.w1y[j], fp_t[gxf + j * LW] - fp_t[gxf - j * LW], a);
                b = fmaf(p.w1y[j], fr_t[gxf + j * LW] - fr_t[gxf - j * LW], b);
            }
            gp_t[gxg] = a;
            gr_t[gxg] = b;
        }
        __syncthreads();
        float dxy_p = 0.f, dxy_r = 0.f;
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            dxy_p = fmaf(p.w1x[j], gp_t[gc + j] - gp_t[gc - j], dxy_p);
            dxy_r = fmaf(p.w1x[j], gr_t[gc + j] - gr_t[gc - j], dxy_r);
        }
        const int rw = w * kTileX + lane;
        float* rhp = ring + rh * TY * kTileX + rw;
        rhp[0 * (R + 1) * TY * kTileX] = dxx_p + dyy_p;
        rhp[1 * (R + 1) * TY * kTileX] = fmaf(c1h, dxx_p, fmaf(c2h, dyy_p, c4h * dxy_p));
        rhp[2 * (R + 1) * TY * kTileX] = fmaf(c1h, dxx_r, fmaf(c2h, dyy_r, c4h * dxy_r));
        fetch_head_coef(z + 1 + R);

        // output plane z
        const float* rcp = ring + rc * TY * kTileX + rw;
        const float lap_in = rcp[0 * (R + 1) * TY * kTileX];
        const float gzin_p = rcp[1 * (R + 1) * TY * kTileX];
        const float gzin_r = rcp[2 * (R + 1) * TY * kTileX];
        float dzz_p = p.w2z[0] * fqp[C], dzz_r = p.w2z[0] * fqr[C];
        float dxz_p = 0.f, dxz_r = 0.f, dyz_p = 0.f, dyz_r = 0.f;
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            dzz_p = fmaf(p.w2z[j], fqp[(C + j) % U] + fqp[(C + U - j) % U], dzz_p);
            dzz_r = fmaf(p.w2z[j], fqr[(C + j) % U] + fqr[(C + U - j) % U], dzz_r);
            dxz_p = fmaf(p.w1z[j], gxp[(C + j) % U] - gxp[(C + U - j) % U], dxz_p);
            dxz_r = fmaf(p.w1z[j], gxr[(C + j) % U] - gxr[(C + U - j) % U], dxz_r);
            dyz_p = fmaf(p.w1z[j], gyp[(C + j) % U] - gyp[(C + U - j) % U], dyz_p);
            dyz_r = fmaf(p.w1z[j], gyr[(C + j) % U] - gyr[(C + U - j) % U], dyz_r);
        }
        const float gz_p = gzin_p + oc3 * dzz_p + oc5 * dyz_p + oc6 * dxz_p;
        const float gz_r = gzin_r + oc3 * dzz_r + oc5 * dyz_r + oc6 * dxz_r;
        const float h_p = (lap_in + dzz_p) - gz_p;
        const float fpv = oa * (oe * h_p + od * gz_r);
        const float frv = oa * (od * h_p + gz_r);
        const float pc = fqp[C], rcv = fqr[C];
        float pn = (2.f * pc - opp) + fpv;
        float rn = (2.f * rcv - orp) + frv;
        if (damp) {
            // the profile sum in the same order as the setup's check
            const float sv = SEP ? sxy + osg : osg;
            pn = (2.f * pc - (1.f - sv) * opp + fpv) / (1.f + sv);
            rn = (2.f * rcv - (1.f - sv) * orp + frv) / (1.f + sv);
        }
        const int64_t zo = (int64_t)z * plane;
        const int rec = z >= z0 ? kRecordsT : 0;
        tstore(trsrc(ppb + zo, rec), oc, pn);
        tstore(trsrc(rpb + zo, rec), oc, rn);
        fetch_out(z + 1);
        rslot = rc;  // the head plane of the next step takes the output plane's slot
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
        tid = threadIdx.x;
        lane = tid & 63;
        w = tid >> 6;
        plane = p.L.plane;
        const int pitch = p.L.pitch;
        const int64_t org = p.L.origin + (int64_t)(y0 - R) * pitch + (x0 - R);
        pb = p.pc + org;
        rb = p.rc + org;
        ppb = p.pp + org;
        rpb = p.rp + org;
        ab = p.A + org;
        eb = p.e + org;
        db = p.d + org;
        sb = (p.sig ? p.sig : p.A) + org;
#pragma unroll
        for (int k = 0; k < 6; ++k) cb[k] = p.c[k] + org;
        zpl = p.A + org - (int64_t)kGhostYZ * plane;
        flags = (tflag_t*)p.dflag;
        sxy = 0.f;
        if constexpr (SEP) {
            // lanes and rows past the interior read the last value (their
            // stores drop)
            szc = (const __attribute__((address_space(4))) float*)p.sz;
            sxy = p.sx[min(x0 + lane, nx - 1)] + p.sy[min(y0 + w, ny - 1)];
        }
        auto off = [&](int r, int c) -> uint32_t {
            const int y = y0 - R + r, x = x0 - R + c;
            return (x >= 0 && x < nx && y >= 0 && y < ny) ? (uint32_t)((r * pitch + c) * 4) : kOOBt;
        };
        oc = off(R + w, R + lane);
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            int e = tid + k * 64 * NW;
            int row = LH, col = lane;  // sink row
            if (e < R * LW) {
                row = e / LW;
                col = e % LW;
            } else if ((e -= R * LW) < TY * 2 * R) {
                row = R + e / (2 * R);
                const int cc = e % (2 * R);
                col = cc < R ? cc : kTileX + cc;
            } else if ((e -= TY * 2 * R) < R * LW) {
                row = R + TY + e / LW;
                col = e % LW;
            }
            oh[k] = row < LH ? off(row, col) : kOOBt;
            lh[k] = row * LW + col;
        }
        gx_on = tid < NGX;
        {
            const int g = tid < NGX ? tid : 0;
            const int row = g / (2 * R), cc = g % (2 * R);
            const int col = cc < R ? cc : kTileX + cc;
            gxf = (R + row) * LW + col;
            gxg = row * LW + col;
        }
#pragma unroll
        for (int i = 0; i < U; ++i) fqp[i] = fqr[i] = gxp[i] = gxr[i] = gyp[i] = gyr[i] = 0.f;
        // 2R pipeline-fill steps: planes z0-R .. z0+R-1 enter as heads
        const int zs = z0 - 2 * R;
        rslot = 0;
        flagbuf = flag_of(zs);
        fetch_head(zs + R);
        fetch_head_coef(zs + R);
        fetch_out(zs);
        for (int zb_ = zs; period(zb_, std::make_integer_sequence<int, U>{}); zb_ += U) {
        }
    }
};

// Waves per SIMD the compiler is asked to fit (register budget 512 / waves):
// radius up to 4 with 64 x 8 tiles fits four (128 registers) without
// spilling, so two blocks share a CU and a 464^3 grid's 464 column blocks
// are all resident at once; 64 x 15 tiles (15 waves) need four to fit one
// block; the other shapes keep the compiler's choice.
template <int R, int NW>
constexpr int tti_waves_per_simd() { return (R <= 4 && NW >= 8) ? 4 : 1; }

template <int R, int NW, bool SEP>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(tti_waves_per_simd<R, NW>()))) void tti3d_tiled(TTIStep p) {
    __shared__ float lds[TiledTTI<R, NW, SEP>::LDS_FLOATS];
    TiledTTI<R, NW, SEP> k(p, lds);
    k.run();
}

template <int R, int CFG>
hipError_t launch_tiled(const TTIStep& p, hipStream_t s) {
    static_assert(kTTITiles[CFG].rows == 1, "the tiled TTI kernel gives each lane one row");
    constexpr int NW = kTTITiles[CFG].waves;
    if (p.sx)
        hipLaunchKernelGGL((tti3d_tiled<R, NW, true>), dim3(p.nblocks), dim3(64 * NW), 0, s, p);
    else
        hipLaunchKernelGGL((tti3d_tiled<R, NW, false>), dim3(p.nblocks), dim3(64 * NW), 0, s, p);
    return hipGetLastError();
}

template <int R>
hipError_t launch_tiled_cfg(const TTIStep& p, int cfg, hipStream_t s) {
    switch (cfg) {
        case 0: return launch_tiled<R, 0>(p, s);
        case 1: return launch_tiled<R, 1>(p, s);
        case 2:
            if constexpr (R <= kTTITallMaxRadius) return launch_tiled<R, 2>(p, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <int R>
hipError_t launch_direct(const TTIStep& p, hipStream_t s) {
    const dim3 grid((p.L.nx + kTileX - 1) / kTileX, (p.L.ny + 3) / 4, p.L.nz);
    hipLaunchKernelGGL((tti_direct<R>), grid, dim3(64, 4), 0, s, p);
    return hipGetLastError();
}

}  // namespace

int tti_tile_y(int cfg) {
    return cfg >= 0 && cfg < 3 ? kTTITiles[cfg].height() : kTTITiles[0].height();
}

hipError_t launch_tti(const TTIStep& p, int radius, int variant, int cfg, hipStream_t s) {
#define FD_TCASE(RR) \
    case RR: return variant == 0 ? launch_tiled_cfg<RR>(p, cfg, s) : launch_direct<RR>(p, s);
    switch (radius) {
        FD_TCASE(1)
        FD_TCASE(2)
        FD_TCASE(3)
        FD_TCASE(4)
        FD_TCASE(5)
        FD_TCASE(6)
        FD_TCASE(7)
        FD_TCASE(8)
        default: return hipErrorInvalidValue;
    }
#undef FD_TCASE
}

}  // namespace fd
