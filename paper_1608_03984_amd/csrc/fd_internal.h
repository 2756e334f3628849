// fd_internal.h -- layout and launch parameters shared by the host runtime and
// the gfx950 kernels of libfd.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fd {

constexpr int kMaxRadius = 8;   // space order 16
constexpr int kGhostX = 32;     // zero columns left of x = 0 (128 B: rows start line-aligned)
constexpr int kGhostYZ = 8;     // zero rows / planes beyond each y and z edge (>= kMaxRadius)
constexpr int kGhostZTop = 12;  // zero planes above the last z plane: kMaxRadius plus the
                                // two planes a streaming kernel may prefetch past its end
constexpr int kTileX = 64;      // one wave64 spans the x extent of a tile

// One padded volume in HBM.  Interior point (x, y, z) of the caller's
// [Nz][Ny][Nx] array sits at  origin + z * plane + y * pitch + x.  The ring of
// ghost cells around the interior is zero and never written, so stencil
// reads need no bounds checks (homogeneous Dirichlet boundary).  The pitch
// and the row count are rounded up so that the last, ragged tile of any
// kernel reads only ghost cells past the interior; the planes below z = 0
// are also the all-zero source of the tiled kernels' undamped loads.
struct Layout {
    int32_t nx, ny, nz;   // interior sizes (padded problem shape)
    int32_t pitch;        // floats per row
    int32_t rows;         // rows per plane
    int32_t planes;       // planes per volume
    int64_t plane;        // pitch * rows
    int64_t origin;       // offset of interior (0,0,0)
    int64_t volume;       // floats per volume (multiple of 64)
};

// A sparse point after host-side preprocessing: flat offset of its lowest
// interpolation corner, the fractional position in that cell per axis, and
// the shot (wavefield) it belongs to.
struct SparsePoint {
    int64_t base;
    float fx, fy, fz;
    int32_t shot;
};

// The multilinear sample of field us at point P (2^ndim corners, zero
// weights skipped), with one rounding per corner: every kernel that records
// receivers forms it with this function, so they give the same bits.
__device__ __forceinline__ float sample_point(const float* __restrict__ us, const SparsePoint& P,
                                              const Layout& L, int ndim) {
    const int ncorner = ndim == 3 ? 8 : 4;
    float acc = 0.f;
    for (int c = 0; c < ncorner; ++c) {
        const int dx = c & 1;
        const int dy = ndim == 3 ? (c >> 1) & 1 : 0;
        const int dz = ndim == 3 ? c >> 2 : c >> 1;
        const float w =
            (dx ? P.fx : 1.f - P.fx) * (dy ? P.fy : 1.f - P.fy) * (dz ? P.fz : 1.f - P.fz);
        if (w != 0.f) acc = fmaf(w, us[P.base + dx + (int64_t)dy * L.pitch + (int64_t)dz * L.plane], acc);
    }
    return acc;
}

// Injection plan of one point set: the distinct (shot, corner) targets that
// its points' non-zero multilinear weights reach, each with its
// contributions (point index within the set << 3 | corner) in point order, so
// that one thread adds every contribution to a target in a fixed order: the
// result does not depend on scheduling (no atomics).
struct InjectPlan {
    const int64_t* target;  // [ntarget] flat index of the corner within its volume
    const int32_t* shot;    // [ntarget] volume (shot) of the target
    const int32_t* start;   // [ntarget + 1] first contribution of each target
    const int32_t* entry;   // [start[ntarget]] contributions
    int32_t ntarget;
};

// Value uv of target m's point after its contributions: each point's
// multilinear weight times dt^2 v^2 (a), its wavelet sample q[point] and
// scale, over 1 + sigma (sg), added in point order.  Every kernel that
// injects forms it with this function, so they give the same bits.
__device__ __forceinline__ float inject_target(float uv, const InjectPlan& plan, int m,
                                               const SparsePoint* __restrict__ pts,
                                               const float* __restrict__ q, float scale, float a,
                                               float sg, int ndim) {
    for (int e = plan.start[m]; e < plan.start[m + 1]; ++e) {
        const int s = plan.entry[e] >> 3, c = plan.entry[e] & 7;
        const SparsePoint P = pts[s];
        const int dx = c & 1;
        const int dy = ndim == 3 ? (c >> 1) & 1 : 0;
        const int dz = ndim == 3 ? c >> 2 : c >> 1;
        const float w =
            (dx ? P.fx : 1.f - P.fx) * (dy ? P.fy : 1.f - P.fy) * (dz ? P.fz : 1.f - P.fz);
        uv += w * a * q[s] * scale / (1.f + sg);
    }
    return uv;
}

// Acoustic step: u^{n+1} = [2u^n - (1-s)u^{n-1} + A L u^n]/(1+s), written
// over u^{n-1}.  L u = c0 u + sum_j cx[j](u[x+j]+u[x-j]) + (y) + (z).
struct AcousticStep {
    const float* __restrict__ uc;  // u^n
    float* up;                     // u^{n-1} in, u^{n+1} out
    float* acc;                    // if set, receives A L u^n (the step's acceleration term)
    const float* __restrict__ A;   // dt^2 v^2
    const float* __restrict__ sig; // eta dt / 2, or nullptr
    const int32_t* __restrict__ dflag; // per (z, tile): 1 if the tile-plane holds damping
    // Imaging fused into an adjoint step (tiled kernel, the configurations
    // img_built names): when img_a is set, img_g[p] = fmaf(u^n[p], img_a[p], img_g[p])
    // at every output point (img_a: the step's stored acceleration, img_g: the
    // FP32 partial sum, both padded volumes).
    const float* img_a;
    float* img_g;
    // Separable damping: when set, sig[x][y][z] equals (sx[x] + sy[y]) + sz[z]
    // (checked at setup) and the tiled kernel evaluates that sum instead of
    // reading sig.
    const float* __restrict__ sx;
    const float* __restrict__ sy;
    const float* __restrict__ sz;
    float c0;
    float cx[kMaxRadius + 1], cy[kMaxRadius + 1], cz[kMaxRadius + 1];
    Layout L;
    int32_t ntx, nty, nzc, zchunk;  // tile grid (tiled kernels)
    int32_t ntiles, nblocks;        // ntx*nty*nzc and the launched (multiple of 8) count
    int32_t nshots, ngroups;        // wavefields advanced together; groups of shots per block
    // > 0: pass-major block order (several shot groups): a pass is one
    // (z chunk, shot group) over all x-y tiles, each XCD takes `slab`
    // consecutive x-y tiles of every pass, and passes run in order
    int32_t slab;
    int64_t shot_stride;            // floats between the volumes of consecutive shots
    // Direct kernel only: when rec_n > 0 the launch also records rec_n
    // receivers (rec_pts) from u^n -- the previous step's u^{n+1}, which it
    // only reads -- into rec_out (one sample per receiver).
    const SparsePoint* rec_pts;
    float* rec_out;
    int32_t rec_n;
    // Direct kernel, one shot only: when inj.ntarget > 0 the launch also
    // injects the plan's points (inj_pts, wavelet samples inj_q, scale
    // inj_scale) into the u^{n+1} it writes; the plan's targets, all of
    // shot 0, are sorted and lie in [inj_lo, inj_hi].
    InjectPlan inj;
    const SparsePoint* inj_pts;
    const float* inj_q;
    float inj_scale;
    int64_t inj_lo, inj_hi;
};

// TTI step (3D).  Per point the coefficient fields are
//   A = dt^2 v^2, e = 1 + 2 eps, d = sqrt(1 + 2 delta),
//   c1..c6 the G_zbar_zbar weights of Dxx, Dyy, Dzz, Dxy, Dyz, Dxz;
// H = Laplacian - G_zbar_zbar.
struct TTIStep {
    const float* __restrict__ pc;
    const float* __restrict__ rc;
    float* pp;  // p^{n-1} in, p^{n+1} out
    float* rp;  // r^{n-1} in, r^{n+1} out
    const float* __restrict__ A;
    const float* __restrict__ sig;
    const int32_t* __restrict__ dflag;
    const float* __restrict__ e;
    const float* __restrict__ d;
    const float* __restrict__ c[6];
    // separable damping (as in AcousticStep): sig = (sx[x] + sy[y]) + sz[z]
    const float* __restrict__ sx;
    const float* __restrict__ sy;
    const float* __restrict__ sz;
    float w2x[kMaxRadius + 1], w2y[kMaxRadius + 1], w2z[kMaxRadius + 1];  // 2nd-derivative / h^2
    float w1x[kMaxRadius + 1], w1y[kMaxRadius + 1], w1z[kMaxRadius + 1];  // 1st-derivative / h
    Layout L;
    int32_t ntx, nty, nzc, zchunk;
    int32_t ntiles, nblocks;
};

// VTI step (2D or 3D), Eq. (vVTI): Dh = Dxx (+ Dyy in 3D) of p and Dzz of r,
//   Dh p = c0h p + sum_j cx[j](p[x+j]+p[x-j]) + cy[j](p[y+j]+p[y-j]),
//   Dzz r = c0z r + sum_j cz[j](r[z+j]+r[z-j]).
struct VTIStep {
    const float* __restrict__ pc;
    const float* __restrict__ rc;
    float* pp;  // p^{n-1} in, p^{n+1} out
    float* rp;  // r^{n-1} in, r^{n+1} out
    const float* __restrict__ A;
    const float* __restrict__ sig;
    const int32_t* __restrict__ dflag;
    const float* __restrict__ e;  // 1 + 2 eps
    const float* __restrict__ d;  // sqrt(1 + 2 delta)
    // separable damping (as in AcousticStep): sig = (sx[x] + sy[y]) + sz[z]
    const float* __restrict__ sx;
    const float* __restrict__ sy;
    const float* __restrict__ sz;
    float c0h, c0z;
    float cx[kMaxRadius + 1], cy[kMaxRadius + 1], cz[kMaxRadius + 1];
    Layout L;
    int32_t ntx, nty, nzc, zchunk;
    int32_t ntiles, nblocks;
};

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files), all asynchronous on `s`.
// ---------------------------------------------------------------------------
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
hipError_t launch_pack(const float* vol, float* dense, const Layout& L, hipStream_t s);
hipError_t launch_unpack(const float* dense, float* vol, const Layout& L, hipStream_t s);

// Per-axis damping profiles along the lines through the centre point, then
// the largest |sig - ((sx + sy) + sz)| and the largest sig over the volume into
// red[0] and red[1] (float bits).
hipError_t launch_damping_profiles(const float* sig, const Layout& L, float* sx, float* sy,
                                   float* sz, uint32_t* red, hipStream_t s);
hipError_t launch_damping_flags(const float* sig, int32_t* flags, const Layout& L, int tile_y,
                                int ntx, int nty, hipStream_t s);


// sparse points
// Shot k of a point writes / reads the volume u + k * shot_stride.
hipError_t launch_inject(float* u, const float* A, const float* sig, const SparsePoint* pts,
                         const InjectPlan& plan, const float* q, float scale, const Layout& L,
                         int ndim, int64_t shot_stride, hipStream_t s);
hipError_t launch_record(const float* u, const SparsePoint* pts, int n, float* out, float scale,
                         const Layout& L, int ndim, int64_t shot_stride, hipStream_t s);
// One launch doing both: injection into un, and into un2 when it is not
// null (as launch_inject on each; into un2 without the damping divisor when
// un2_damped is false), and, from the level uc that the injection does not
// touch, recording (as launch_record with scale 1); either part may be
// empty.
hipError_t launch_inject_record(float* un, float* un2, bool un2_damped, const float* A,
                                const float* sig,
                                const SparsePoint* spts, const InjectPlan& plan, const float* q,
                                float scale, const float* uc, const SparsePoint* rpts, int nrec,
                                float* out, const Layout& L, int ndim, int64_t shot_stride,
                                hipStream_t s);

// adjoint / gradient (FP32, two-level summation)
// gpart[vol] += mu[vol] * acc[vol] over the interior.
// res = d - dobs (n values), J[0] += 1/2 sum res^2 (summed in FP64 in a
// fixed order; J[1 .. kMisfitBlocks] hold the per-block partial sums).
constexpr int kMisfitBlocks = 1024;
hipError_t launch_misfit(const float* d, const float* dobs, int64_t n, float* res, double* J,
                         hipStream_t s);
hipError_t launch_image(const float* mu, const float* acc, float* gpart, const Layout& L,
                        hipStream_t s);
// gsum[dense] += gpart[vol]; gpart[vol] = 0 over the interior.
hipError_t launch_flush_gradient(float* gpart, float* gsum, const Layout& L, hipStream_t s);
// out[dense] = gsum * -1/dt^2 (wrt m = 1/v^2) or gsum * 2 dt / A^{3/2} (wrt v);
// with accumulate, that value is added to out.
hipError_t launch_finish_gradient(const float* gsum, const float* A, float* out, const Layout& L,
                                  double dt, int wrt_vel, int accumulate, hipStream_t s);

// correction network (fd_cnn.hip)
constexpr int kCnnWgradZChunk = 32;  // z planes per block of the weight-gradient pass
int cnn_packed_elems(int cin_pad);
int cnn_wgrad_slots(int D, int H, int W, int zchunk);
hipError_t launch_cnn_pack(const float* w, int cin, int cout, int cin_pad, int flip,
                           uint16_t* out, hipStream_t s);
hipError_t launch_cnn_conv(const uint16_t* x, int cin_pad, int D, int H, int W,
                           const uint16_t* packed, const float* bias, int mode,
                           const uint16_t* mask, int cout_store, uint16_t* y, float* yf,
                           hipStream_t s);
hipError_t launch_cnn_wgrad(const uint16_t* x, int cx, const uint16_t* dz, int cz, int D, int H,
                            int W, int zchunk, float* partials, float* out, hipStream_t s);
// loss[0] += the masked loss (loss[1 .. kLossBlocks]: per-block partials,
// summed in a fixed order).
constexpr int kLossBlocks = 256;
hipError_t launch_cnn_loss_grad(const float* out, const float* target, const uint8_t* mask,
                                int64_t nvox, int cout, int cpad, float inv_n, uint16_t* dz,
                                float* loss, hipStream_t s);
hipError_t launch_cnn_adam(float* p, const float* g, float* m, float* v, int64_t n, int t,
                           float lr, float b1, float b2, float eps, hipStream_t s);
hipError_t launch_cnn_features(const float* uc, const float* up, const float* A, const Layout& L,
                               float inv_dt_vref, const uint8_t* mask, uint32_t* bits,
                               uint16_t* xo, hipStream_t s);
hipError_t launch_cnn_correct(float* uc, float* up, const Layout& L, const float* d,
                              const uint8_t* mask, const uint32_t* bits, hipStream_t s);
hipError_t launch_cnn_residual(const float* ref_cur, const float* ref_prev, const float* uc,
                               const float* up, const Layout& L, const uint32_t* bits, float* t,
                               hipStream_t s);
hipError_t launch_restrict(const float* u, const Layout& L, int stride, float* out,
                           hipStream_t s);

// stencils
hipError_t launch_acoustic(const AcousticStep& p, int ndim, int radius, int variant, int tile_cfg,
                           int shots_per_block, hipStream_t s);
// The tiled 3D kernel for radius 5-6 and 7-8 (translation units of their own,
// compiled in parallel).
hipError_t launch_acoustic_tiled_r56(const AcousticStep& p, int radius, int cfg,
                                     int shots_per_block, hipStream_t s);
hipError_t launch_acoustic_tiled_r78(const AcousticStep& p, int radius, int cfg,
                                     int shots_per_block, hipStream_t s);
hipError_t launch_tti(const TTIStep& p, int radius, int variant, int tile_cfg, hipStream_t s);
hipError_t launch_vti(const VTIStep& p, int ndim, int radius, int variant, hipStream_t s);

// Tile shapes of the tiled 3D kernels: the launchers instantiate the kernels
// from these tables and the host sizes its tile grid and damping flags from
// the same entries, so the two cannot disagree.
struct TileShape {
    int waves;  // waves per block (64 x waves threads)
    int rows;   // rows each lane owns
    constexpr int height() const { return waves * rows; }
};
// acoustic FD_OPT_TILE configurations 0..4: 64 x 8, 64 x 16, 64 x 8, 64 x 16,
// 64 x 24
constexpr TileShape kAcousticTiles[5] = {{4, 2}, {4, 4}, {8, 1}, {8, 2}, {12, 2}};
// TTI FD_OPT_TILE configurations 0..2: 64 x 8, 64 x 4, 64 x 15 (radius up to
// 4: a 960-thread block must fit in 128 registers per lane; the default
// there, 64 x 8 above)
constexpr TileShape kTTITiles[3] = {{8, 1}, {4, 1}, {15, 1}};
constexpr int kTTITallMaxRadius = 4;
// VTI: 64 x 16, one row per wave (1024 threads; up to 110 registers per lane
// at radius 8, so the block fits a CU at every order)
constexpr TileShape kVTITile = {16, 1};
// The smallest tile height of any tiled kernel: the damping flags are sized
// for it.
constexpr int kMinTileRows = 4;
// Tiled acoustic variants for gradients (configuration, shots per block):
// the acceleration output is built with one shot per block in every
// configuration and with two in configuration 2; the imaging fused into the
// adjoint step in configurations 0 and 4 (the single-shot defaults) with one
// shot and configuration 2 with two.
constexpr bool acc_built(int cfg, int sb) { return sb == 1 || (cfg == 2 && sb == 2); }
constexpr bool img_built(int cfg, int sb) {
    return ((cfg == 0 || cfg == 4) && sb == 1) || (cfg == 2 && sb == 2);
}

// Tile height (rows) of the tiled kernels for a tile configuration.
int acoustic_tile_y(int tile_cfg);
int tti_tile_y(int tile_cfg);
int vti_tile_y();

}  // namespace fd
