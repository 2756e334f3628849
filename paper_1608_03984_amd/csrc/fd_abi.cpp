// fd_abi.cpp -- host runtime and C ABI of libfd (see include/fd.h).
//
// Validates problems, derives stencil weights (Fornberg's recursion, in
// double, rounded once to float), lays the volumes out in the caller's
// workspace, and enqueues the per-step launch sequence of Algorithm 1:
// stencil update -> source injection -> receiver sampling -> level swap (the
// acoustic forward run merges launches: a step samples the previous step's
// receivers from the level it only reads).
#include "fd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "fd_internal.h"

using fd::Layout;
using fd::SparsePoint;

struct fd_ctx {
    fd_grid g;
    int radius;
    Layout L;
    bool damping;
    bool tti;
    bool vti;
    int32_t nshots;  // wavefields advanced together on the one model
    int32_t max_points;
    // workspace regions
    uint32_t* reduce;
    float* A;
    float* sig;
    float* e;
    float* d;
    float* c[6];
    float* u[2];  // acoustic u / TTI p: two levels (shot k at + k * L.volume)
    float* r[2];  // TTI r: two levels
    int32_t* dflag;
    float* prof;      // damping profiles sx[nx], sy[ny], sz[nz] (3D)
    bool sep_ok;      // the damping field is (sx + sy) + sz to within 2^-20 of its maximum
    bool sep_use;     // FD_OPT_DAMPING_PROFILE
    bool fuse_image;  // FD_OPT_FUSED_IMAGING
    SparsePoint* pts;
    // injection plans (device) of the two point sets of the last upload
    int64_t* plan_target;
    int32_t* plan_shot;
    int32_t* plan_start;
    int32_t* plan_entry;
    fd::InjectPlan plan[2];
    // smallest and largest target of each plan (meaningful for one shot,
    // where the targets are sorted by index)
    int64_t plan_lo[2], plan_hi[2];
    int cur;  // index of the level holding u^n in u[]/r[]
    // derived stencil coefficients (float, already divided by h or h^2)
    float w2[3][fd::kMaxRadius + 1];
    float w1[3][fd::kMaxRadius + 1];
    // launch configuration
    int variant;
    int tile_cfg;
    int zchunk_opt;
    int shots_per_block;
    int tile_y;
    int ncu;  // compute units of the device current at setup (0 if unknown)
    bool flags_stale;
    // cached sparse-point coordinates of the last upload
    std::vector<double> src_coords, rec_coords;
    std::vector<int32_t> src_counts, rec_counts;  // points per shot of the last upload
    int nsrc_dev, nrec_dev;
    // checkpoint store filled by the last fd_forward_checkpointed
    const void* ck_store;
    int32_t ck_nt, ck_interval;
    bool ck_last_acc;  // the last segment's accelerations are still in the store
    std::string err;
};

namespace {

// Runs an entry point's body; a C++ exception from its host-side work (the
// host copies of the FP64 setup, point tables, injection plans) becomes
// FD_ERR_HOST instead of crossing the C boundary.
template <class F>
int32_t guarded(fd_ctx* ctx, F&& body) {
    try {
        return body();
    } catch (const std::exception& ex) {
        if (ctx) {
            try {
                ctx->err = ex.what();
            } catch (...) {
            }
        }
        return FD_ERR_HOST;
    } catch (...) {
        return FD_ERR_HOST;
    }
}

int32_t fail(fd_ctx* ctx, int32_t code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int32_t hip_fail(fd_ctx* ctx, hipError_t e, const char* where) {
    if (ctx) ctx->err = std::string(where) + ": " + hipGetErrorString(e);
    return FD_ERR_DEVICE;
}

// Fornberg (1988) recursion for finite-difference weights at z over nodes
// x[0..n-1], derivatives 0..m.  c[j*(m+1)+k] = weight of node j for d^k/dx^k.
void fornberg(double z, const double* x, int n, int m, double* c) {
    for (int i = 0; i < n * (m + 1); ++i) c[i] = 0.0;
    double c1 = 1.0, c4 = x[0] - z;
    c[0] = 1.0;
    for (int i = 1; i < n; ++i) {
        const int mn = i < m ? i : m;
        double c2 = 1.0;
        const double c5 = c4;
        c4 = x[i] - z;
        for (int j = 0; j < i; ++j) {
            const double c3 = x[i] - x[j];
            c2 *= c3;
            if (j == i - 1) {
                for (int k = mn; k >= 1; --k)
                    c[i * (m + 1) + k] =
                        c1 * (k * c[(i - 1) * (m + 1) + k - 1] - c5 * c[(i - 1) * (m + 1) + k]) / c2;
                c[i * (m + 1)] = -c1 * c5 * c[(i - 1) * (m + 1)] / c2;
            }
            for (int k = mn; k >= 1; --k)
                c[j * (m + 1) + k] = (c4 * c[j * (m + 1) + k] - k * c[j * (m + 1) + k - 1]) / c3;
            c[j * (m + 1)] = c4 * c[j * (m + 1)] / c3;
        }
        c1 = c2;
    }
}

// Central weights w[0..r] of the derivative `deriv` on unit spacing, nodes
// ordered 0, -1, +1, -2, +2, ... so that the recursion adds symmetric pairs.
bool central_weights(int so, int deriv, double* w) {
    if (so < 2 || so > 2 * fd::kMaxRadius || so % 2 || (deriv != 1 && deriv != 2)) return false;
    const int r = so / 2, n = 2 * r + 1;
    double x[2 * fd::kMaxRadius + 1];
    double c[(2 * fd::kMaxRadius + 1) * 3];
    x[0] = 0.0;
    for (int j = 1; j <= r; ++j) {
        x[2 * j - 1] = -j;
        x[2 * j] = j;
    }
    fornberg(0.0, x, n, 2, c);
    w[0] = c[0 * 3 + deriv];
    for (int j = 1; j <= r; ++j) {
        const double wp = c[(2 * j) * 3 + deriv], wm = c[(2 * j - 1) * 3 + deriv];
        // symmetrise against rounding: the exact weights are (anti)symmetric
        w[j] = deriv == 2 ? 0.5 * (wp + wm) : 0.5 * (wp - wm);
    }
    if (deriv == 1) w[0] = 0.0;
    return true;
}

int32_t validate_grid(const fd_grid* g, std::string& msg) {
    if (!g) return msg = "grid is NULL", FD_ERR_INVALID_ARG;
    if (g->ndim != 2 && g->ndim != 3) return msg = "ndim must be 2 or 3", FD_ERR_INVALID_ARG;
    if (g->space_order < 2 || g->space_order % 2)
        return msg = "space_order must be even and >= 2", FD_ERR_INVALID_ARG;
    if (g->space_order > FD_MAX_SPACE_ORDER)
        return msg = "space_order above 16 is not built", FD_ERR_UNSUPPORTED;
    if (g->physics != FD_ACOUSTIC && g->physics != FD_TTI && g->physics != FD_VTI)
        return msg = "unknown physics", FD_ERR_INVALID_ARG;
    if (g->physics == FD_TTI && g->ndim != 3)
        return msg = "TTI is built for 3D grids only", FD_ERR_UNSUPPORTED;
    if (g->nbl < 0 || g->nbl > (1 << 20)) return msg = "nbl out of range", FD_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a)
        if (g->shape[a] < 1 || g->shape[a] > (1 << 20))
            return msg = "shape out of range", FD_ERR_INVALID_ARG;
    if (g->ndim == 2 && g->shape[1] != 1) return msg = "2D grids need shape[1] == 1", FD_ERR_INVALID_ARG;
    {
        // the padded array must stay far from 64-bit byte-count overflow in the
        // workspace plan (2^40 points, 4 TiB per field, is far beyond one GPU)
        const double pad = 2.0 * g->nbl;
        const double pts = (g->shape[0] + pad) * (g->ndim == 3 ? g->shape[1] + pad : 1.0) *
                           (g->shape[2] + pad);
        if (pts > 1099511627776.0) return msg = "grid too large", FD_ERR_INVALID_ARG;
    }
    for (int a = 0; a < 3; ++a) {
        if (g->ndim == 2 && a == 1) continue;
        if (!(g->spacing[a] > 0.0) || !std::isfinite(g->spacing[a]))
            return msg = "spacing must be positive and finite", FD_ERR_INVALID_ARG;
    }
    if (!(g->dt > 0.0) || !std::isfinite(g->dt)) return msg = "dt must be positive", FD_ERR_INVALID_ARG;
    return FD_OK;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

Layout make_layout(const fd_grid* g) {
    Layout L;
    const int64_t nb = g->nbl;
    L.nx = (int32_t)(g->shape[0] + 2 * nb);
    L.ny = g->ndim == 3 ? (int32_t)(g->shape[1] + 2 * nb) : 1;
    L.nz = (int32_t)(g->shape[2] + 2 * nb);
    // x: 32 zero columns before the interior (rows start on a 128-byte line),
    // the interior rounded up to whole 64-wide tiles, 32 zero columns after.
    L.pitch = (int32_t)(fd::kGhostX + round_up(L.nx, fd::kTileX) + 32);
    // y: kGhostYZ zero rows each side of the interior rounded to 64 rows (so
    // any tile height dividing 64 stays inside); 2D has a single row.
    L.rows = g->ndim == 3 ? (int32_t)(fd::kGhostYZ + round_up(L.ny, 64) + fd::kGhostYZ) : 1;
    L.planes = L.nz + fd::kGhostYZ + fd::kGhostZTop;
    L.plane = (int64_t)L.pitch * L.rows;
    L.origin = (int64_t)fd::kGhostYZ * L.plane + (g->ndim == 3 ? (int64_t)fd::kGhostYZ * L.pitch : 0) +
               fd::kGhostX;
    L.volume = round_up(L.plane * L.planes, 64);
    return L;
}

struct Carve {
    uint64_t off = 0;
    uint64_t take(uint64_t bytes) {
        const uint64_t o = off;
        off = (uint64_t)round_up((int64_t)(off + bytes), 256);
        return o;
    }
};

// The damping flags are sized for the smallest tile height of any kernel.
int min_tile_y() { return fd::kMinTileRows; }

constexpr int32_t kMaxShots = 4096;
static_assert(FD_MISFIT_DOUBLES == 1 + fd::kMisfitBlocks, "misfit partial slots");
static_assert(FD_CNN_LOSS_FLOATS == 1 + fd::kLossBlocks, "loss partial slots");
// Sparse points per context: the injection plan codes a point index in the
// upper 29 bits of an int32 (the corner in the lower 3).
constexpr int32_t kMaxPoints = 1 << 27;

// The imaging condition is summed in FP32 in two levels: a partial sum over
// at most this many adjoint steps, then the running total (bounded rounding
// without FP64 on the device).
constexpr int kFlushSteps = 32;

// Workspace plan; when base is non-null the pointers are filled in.
uint64_t plan_workspace(const fd_grid* g, const Layout& L, int32_t nshots, int32_t max_points,
                        fd_ctx* ctx, char* base) {
    Carve cv;
    const uint64_t vol = (uint64_t)L.volume * sizeof(float);
    const bool tti = g->physics == FD_TTI;
    const bool aniso = g->physics != FD_ACOUSTIC;  // two wavefields p, r and e, d
    const uint64_t o_red = cv.take(256);
    const uint64_t o_A = cv.take(vol);
    const uint64_t o_sig = cv.take(vol);
    uint64_t o_e = 0, o_d = 0, o_c[6] = {0, 0, 0, 0, 0, 0}, o_r[2] = {0, 0};
    if (aniso) {
        o_e = cv.take(vol);
        o_d = cv.take(vol);
    }
    if (tti)
        for (int k = 0; k < 6; ++k) o_c[k] = cv.take(vol);
    const uint64_t o_u0 = cv.take(vol * (uint64_t)nshots);
    const uint64_t o_u1 = cv.take(vol * (uint64_t)nshots);
    if (aniso) {
        o_r[0] = cv.take(vol);
        o_r[1] = cv.take(vol);
    }
    const int64_t ntx = (L.nx + fd::kTileX - 1) / fd::kTileX;
    const int64_t nty = (L.ny + min_tile_y() - 1) / min_tile_y();
    const uint64_t o_flag = cv.take((uint64_t)(ntx * nty * L.nz) * sizeof(int32_t));
    const uint64_t o_prof = cv.take((uint64_t)(L.nx + L.ny + L.nz) * sizeof(float));
    const uint64_t o_pts = cv.take((uint64_t)(max_points > 0 ? max_points : 1) * sizeof(SparsePoint));
    // injection plans: at most 8 corners per point, over both point sets
    const uint64_t cap = 8 * (uint64_t)(max_points > 0 ? max_points : 1);
    const uint64_t o_ptg = cv.take(cap * sizeof(int64_t));
    const uint64_t o_psh = cv.take(cap * sizeof(int32_t));
    const uint64_t o_pst = cv.take((cap + 2) * sizeof(int32_t));
    const uint64_t o_pen = cv.take(cap * sizeof(int32_t));
    if (ctx && base) {
        ctx->reduce = reinterpret_cast<uint32_t*>(base + o_red);
        ctx->A = reinterpret_cast<float*>(base + o_A);
        ctx->sig = reinterpret_cast<float*>(base + o_sig);
        ctx->e = aniso ? reinterpret_cast<float*>(base + o_e) : nullptr;
        ctx->d = aniso ? reinterpret_cast<float*>(base + o_d) : nullptr;
        for (int k = 0; k < 6; ++k) ctx->c[k] = tti ? reinterpret_cast<float*>(base + o_c[k]) : nullptr;
        ctx->u[0] = reinterpret_cast<float*>(base + o_u0);
        ctx->u[1] = reinterpret_cast<float*>(base + o_u1);
        ctx->r[0] = aniso ? reinterpret_cast<float*>(base + o_r[0]) : nullptr;
        ctx->r[1] = aniso ? reinterpret_cast<float*>(base + o_r[1]) : nullptr;
        ctx->dflag = reinterpret_cast<int32_t*>(base + o_flag);
        ctx->prof = reinterpret_cast<float*>(base + o_prof);
        ctx->pts = reinterpret_cast<SparsePoint*>(base + o_pts);
        ctx->plan_target = reinterpret_cast<int64_t*>(base + o_ptg);
        ctx->plan_shot = reinterpret_cast<int32_t*>(base + o_psh);
        ctx->plan_start = reinterpret_cast<int32_t*>(base + o_pst);
        ctx->plan_entry = reinterpret_cast<int32_t*>(base + o_pen);
    }
    return cv.off;
}

// S = |w0| + 2 sum |w_j| of the second-derivative stencil (unit spacing).
double abs_weight_sum(int so) {
    double w[fd::kMaxRadius + 1];
    central_weights(so, 2, w);
    double s = std::fabs(w[0]);
    for (int j = 1; j <= so / 2; ++j) s += 2.0 * std::fabs(w[j]);
    return s;
}

double cfl_dt(const fd_grid* g, double vmax) {
    const double S = abs_weight_sum(g->space_order);
    double den = S / (g->spacing[0] * g->spacing[0]) + S / (g->spacing[2] * g->spacing[2]);
    if (g->ndim == 3) den += S / (g->spacing[1] * g->spacing[1]);
    return std::sqrt(4.0 / den) / vmax;
}

// Host preprocessing of one sparse point (see fd.h, Conventions).
bool locate(const fd_ctx* ctx, const double* c, SparsePoint* P) {
    const fd_grid& g = ctx->g;
    const Layout& L = ctx->L;
    int64_t idx[3] = {0, 0, 0};
    double frac[3] = {0.0, 0.0, 0.0};
    const int32_t n[3] = {L.nx, L.ny, L.nz};
    for (int a = 0; a < 3; ++a) {
        if (g.ndim == 2 && a == 1) continue;
        const double coord = g.ndim == 2 ? c[a == 0 ? 0 : 1] : c[a];
        if (!std::isfinite(coord)) return false;
        const double gi = coord / g.spacing[a] + (double)g.nbl;
        if (!(gi >= 0.0) || gi > (double)(n[a] - 1) || n[a] < 2) return false;
        int64_t i = (int64_t)std::floor(gi);
        if (i > n[a] - 2) i = n[a] - 2;
        idx[a] = i;
        frac[a] = gi - (double)i;
    }
    P->base = L.origin + idx[2] * L.plane + idx[1] * L.pitch + idx[0];
    P->fx = (float)frac[0];
    P->fy = (float)frac[1];
    P->fz = (float)frac[2];
    P->shot = 0;
    return true;
}

// Tiles of one block per CU (a whole column each) pay only when their blocks
// fill the chip in one round: between 90 % and 100 % of the device's compute
// units.  Fewer leave CUs idle (500^3, so 2: 168 blocks of 64 x 24 took
// 0.50 s for the cost-to-solution run against 0.41 s with 64 x 8 tiles);
// more run in rounds of lone blocks.
bool fills_chip_once(const fd_ctx* ctx, int tile_y) {
    const int64_t ntx = (ctx->L.nx + fd::kTileX - 1) / fd::kTileX;
    const int64_t nty = (ctx->L.ny + tile_y - 1) / tile_y;
    const int64_t blocks = ntx * nty;
    return ctx->ncu > 0 && 10 * blocks >= 9 * (int64_t)ctx->ncu && blocks <= ctx->ncu;
}

// Tile shape of the tiled acoustic kernel (measured on the 592^3 workload
// with the damping layer evaluated from its profiles, whole columns):
// 64 x 24 with 768 threads up to radius 4 where its blocks fill the chip
// once (250 blocks at 592^3, one per CU, fewer halo rows per point: 582 /
// 576 / 608 / 616 us at so 2 / 4 / 6 / 8 against 621 / 603 / 631 / 626 for
// 64 x 8), else 64 x 8 with 256 threads (740 blocks at 592^3, up to three
// per CU, all resident at once: 668 / 706 us at so 12 / 16 against 668 /
// 746 for 64 x 24, whose single block per CU lines all its waves up at
// every barrier while the longer steps of these orders need independent
// blocks to overlap).
int default_tile(const fd_ctx* ctx) {
    return ctx->radius <= 4 && fills_chip_once(ctx, fd::kAcousticTiles[4].height()) ? 4 : 0;
}

// Several shots (measured with 16 shots on the 336^3 survey grid, three z
// chunks): 4 shots per block up to radius 2, 2 up to radius 6, one above,
// where the register queues of several shots cost more occupancy than the
// shared model reads save; 64 x 8 tiles of 512 threads (configuration 2),
// 64 x 8 of 256 above radius 6.
int default_shots_per_block(int radius, int nshots) {
    if (nshots <= 1) return 1;
    const int sb = radius <= 2 ? 4 : (radius <= 6 ? 2 : 1);
    return nshots < sb ? (nshots >= 2 ? 2 : 1) : sb;
}
int shots_tile(int radius) { return radius <= 6 ? 2 : 0; }

// TTI (measured at 464^3, so 8): 64 x 15 tiles of 960 threads where they
// fit 128 registers per lane (radius up to 4) and fill the chip once, 1.12
// ms per step against 1.33 for 64 x 8 of 512 threads: the y halo is 8 rows
// per 15 instead of per 8, and the 248 column blocks each hold a CU alone,
// so no block is slowed by a neighbour on its CU and neighbouring tiles keep
// marching through the same planes (64 x 16 tiles, 232 blocks, took 1.15
// ms).  64 x 8 otherwise.
int tti_default_tile(const fd_ctx* ctx) {
    return ctx->radius <= fd::kTTITallMaxRadius &&
                   fills_chip_once(ctx, fd::kTTITiles[2].height())
               ? 2
               : 0;
}

void tile_grid(const fd_ctx* ctx, int tile_y, int zchunk_opt, int radius, int ngroups,
               fd::AcousticStep* a, fd::TTIStep* t) {
    const Layout& L = ctx->L;
    const int ntx = (L.nx + fd::kTileX - 1) / fd::kTileX;
    const int nty = (L.ny + tile_y - 1) / tile_y;
    int zc = zchunk_opt;
    if (zc <= 0) {
        // One wavefield: one chunk per column when the x-y tiles already give
        // the chip about 6 waves per CU (1600 waves) -- neighbouring tiles
        // then march through z together from the first plane, sharing halo
        // rows in L2, and no chunk re-reads 2R planes or refills the pipeline
        // (measured best for the acoustic kernel at 592^3 and VTI and TTI at
        // 464^3); otherwise z is split for about 768 blocks, high orders
        // rounding the count down.  Several shots (many more blocks than the
        // chip holds at once): three chunks per column, 4-10 % faster than
        // whole columns for 16 shots at 336^3.
        const int waves = ctx->tti   ? fd::kTTITiles[ctx->tile_cfg].waves
                          : ctx->vti ? fd::kVTITile.waves
                                     : fd::kAcousticTiles[ctx->tile_cfg].waves;
        const int64_t xy = (int64_t)ntx * nty * ngroups;
        int64_t nzc;
        if (ctx->nshots > 1)
            nzc = 3;
        else if (xy * waves >= 1600)
            nzc = 1;
        else
            nzc = radius <= 4 ? (768 + xy / 2) / xy : 768 / xy;
        if (nzc < 1) nzc = 1;
        zc = (int)((L.nz + nzc - 1) / nzc);
        if (zc < 4 * radius) zc = 4 * radius;
    }
    if (zc > L.nz) zc = L.nz;
    const int nzc = (L.nz + zc - 1) / zc;
    const int ntiles = ntx * nty * nzc;
    int nblocks = (int)round_up((int64_t)ntiles * ngroups, 8);
    // Several shot groups give many more blocks than the chip holds: order
    // them by pass (z chunk, group), every pass spread over the 8 XCDs in
    // x-y slabs, so that the blocks running together are whole x-y planes of
    // tiles started at the same time (neighbours share halo rows in L2) and
    // consecutive groups of one chunk read the same A planes together.
    const int slab = ngroups > 1 ? (ntx * nty + 7) / 8 : 0;
    if (slab > 0) nblocks = 8 * slab * nzc * ngroups;
    if (a) {
        a->ntx = ntx; a->nty = nty; a->nzc = nzc; a->zchunk = zc;
        a->ntiles = ntiles; a->nblocks = nblocks; a->ngroups = ngroups;
        a->slab = slab;
    }
    if (t) {
        t->ntx = ntx; t->nty = nty; t->nzc = nzc; t->zchunk = zc;
        t->ntiles = ntiles; t->nblocks = nblocks;
    }
}

// Injection plan of n points (host table pts[0..n)): every non-zero corner
// weight as a contribution (point << 3 | corner) to its target (shot,
// flat index), targets in (shot, index) order and each target's
// contributions in point order.  Appends to the concatenated plan arrays;
// `start` values are offsets into the concatenated entries (entry_base for
// this set's first entry).
void build_plan(const fd_ctx* ctx, const SparsePoint* pts, int n, int32_t entry_base,
                std::vector<int64_t>& tg, std::vector<int32_t>& sh, std::vector<int32_t>& st,
                std::vector<int32_t>& en) {
    struct Contribution {
        int32_t shot;
        int64_t index;
        int32_t code;
    };
    const int nd = ctx->g.ndim, nc = nd == 3 ? 8 : 4;
    std::vector<Contribution> cs;
    cs.reserve((size_t)n * nc);
    for (int i = 0; i < n; ++i) {
        const SparsePoint& P = pts[i];
        for (int c = 0; c < nc; ++c) {
            const int dx = c & 1;
            const int dy = nd == 3 ? (c >> 1) & 1 : 0;
            const int dz = nd == 3 ? c >> 2 : c >> 1;
            // the weight as the injection kernel forms it (FP32 products)
            const float w =
                (dx ? P.fx : 1.f - P.fx) * (dy ? P.fy : 1.f - P.fy) * (dz ? P.fz : 1.f - P.fz);
            if (w == 0.f) continue;
            cs.push_back({P.shot, P.base + dx + (int64_t)dy * ctx->L.pitch +
                                      (int64_t)dz * ctx->L.plane,
                          (i << 3) | c});
        }
    }
    std::stable_sort(cs.begin(), cs.end(), [](const Contribution& a, const Contribution& b) {
        return a.shot != b.shot ? a.shot < b.shot : a.index < b.index;
    });
    for (size_t k = 0; k < cs.size(); ++k) {
        if (k == 0 || cs[k].shot != cs[k - 1].shot || cs[k].index != cs[k - 1].index) {
            tg.push_back(cs[k].index);
            sh.push_back(cs[k].shot);
            st.push_back(entry_base + (int32_t)k);
        }
        en.push_back(cs[k].code);
    }
}

// True when the given points are those of the last upload (compared in
// place: no copy of the coordinates).
bool same_points(const fd_ctx* ctx, int n1, const double* c1, int n2, const double* c2,
                 const int32_t* counts1, const int32_t* counts2) {
    const size_t nd = (size_t)ctx->g.ndim;
    if (n1 != ctx->nsrc_dev || n2 != ctx->nrec_dev) return false;
    if ((size_t)n1 * nd != ctx->src_coords.size() || (size_t)n2 * nd != ctx->rec_coords.size())
        return false;
    if (n1 && std::memcmp(c1, ctx->src_coords.data(), (size_t)n1 * nd * sizeof(double))) return false;
    if (n2 && std::memcmp(c2, ctx->rec_coords.data(), (size_t)n2 * nd * sizeof(double))) return false;
    const size_t ns = counts1 || counts2 ? (size_t)ctx->nshots : 0;
    if ((counts1 ? ns : 0) != ctx->src_counts.size() || (counts2 ? ns : 0) != ctx->rec_counts.size())
        return false;
    if (counts1 && std::memcmp(counts1, ctx->src_counts.data(), ns * sizeof(int32_t))) return false;
    if (counts2 && std::memcmp(counts2, ctx->rec_counts.data(), ns * sizeof(int32_t))) return false;
    return true;
}

// Upload the sparse-point table [first..., second...] when the coordinates
// differ from the last upload.
// counts1 / counts2 give the points per shot (NULL: all in shot 0).
int32_t sync_points(fd_ctx* ctx, int n1, const double* c1, int n2, const double* c2,
                    const char* what1, const char* what2, hipStream_t s,
                    const int32_t* counts1 = nullptr, const int32_t* counts2 = nullptr) {
    if (same_points(ctx, n1, c1, n2, c2, counts1, counts2)) return FD_OK;
    const int nd = ctx->g.ndim;
    std::vector<double> a(n1 ? c1 : nullptr, n1 ? c1 + (size_t)n1 * nd : nullptr);
    std::vector<double> b(n2 ? c2 : nullptr, n2 ? c2 + (size_t)n2 * nd : nullptr);
    const int ns = counts1 || counts2 ? ctx->nshots : 0;
    std::vector<int32_t> k1(counts1 ? counts1 : nullptr, counts1 ? counts1 + ns : nullptr);
    std::vector<int32_t> k2(counts2 ? counts2 : nullptr, counts2 ? counts2 + ns : nullptr);
    std::vector<SparsePoint> host((size_t)n1 + n2);
    for (int i = 0; i < n1; ++i)
        if (!locate(ctx, &a[(size_t)i * nd], &host[i]))
            return fail(ctx, FD_ERR_INVALID_ARG,
                        std::string(what1) + " " + std::to_string(i) + " outside the grid");
    for (int i = 0; i < n2; ++i)
        if (!locate(ctx, &b[(size_t)i * nd], &host[(size_t)n1 + i]))
            return fail(ctx, FD_ERR_INVALID_ARG,
                        std::string(what2) + " " + std::to_string(i) + " outside the grid");
    // shot of each point from the per-shot counts (validated by the caller)
    auto assign = [&](const std::vector<int32_t>& k, size_t first, int n) {
        size_t i = first;
        for (size_t shot = 0; shot < k.size(); ++shot)
            for (int j = 0; j < k[shot]; ++j) host[i++].shot = (int32_t)shot;
        (void)n;
    };
    if (!k1.empty()) assign(k1, 0, n1);
    if (!k2.empty()) assign(k2, (size_t)n1, n2);
    // injection plans of both sets, concatenated: targets of set 1, then set 2
    std::vector<int64_t> tg;
    std::vector<int32_t> sh, st, en;
    int32_t nt1 = 0;
    for (int set = 0; set < 2; ++set) {
        const int first = set == 0 ? 0 : n1, n = set == 0 ? n1 : n2;
        const int t0 = (int)tg.size();
        build_plan(ctx, host.data() + first, n, (int32_t)en.size(), tg, sh, st, en);
        if (set == 0) nt1 = (int32_t)tg.size() - t0;
    }
    st.push_back((int32_t)en.size());
    // the device tables change from here on: until they are complete no later
    // call may take them for the previous upload's
    ctx->nsrc_dev = ctx->nrec_dev = -1;
    if (!host.empty()) {
        hipError_t he = hipMemcpyAsync(ctx->pts, host.data(), host.size() * sizeof(SparsePoint),
                                       hipMemcpyHostToDevice, s);
        if (he == hipSuccess && !tg.empty())
            he = hipMemcpyAsync(ctx->plan_target, tg.data(), tg.size() * sizeof(int64_t),
                                hipMemcpyHostToDevice, s);
        if (he == hipSuccess && !tg.empty())
            he = hipMemcpyAsync(ctx->plan_shot, sh.data(), sh.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s);
        if (he == hipSuccess)
            he = hipMemcpyAsync(ctx->plan_start, st.data(), st.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s);
        if (he == hipSuccess && !en.empty())
            he = hipMemcpyAsync(ctx->plan_entry, en.data(), en.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s);
        if (he == hipSuccess) he = hipStreamSynchronize(s);  // host tables go out of scope
        if (he != hipSuccess) return hip_fail(ctx, he, "point upload");
    }
    const int32_t ntot = (int32_t)tg.size();
    ctx->plan[0] = {ctx->plan_target, ctx->plan_shot, ctx->plan_start, ctx->plan_entry, nt1};
    ctx->plan[1] = {ctx->plan_target + nt1, ctx->plan_shot + nt1, ctx->plan_start + nt1,
                    ctx->plan_entry, ntot - nt1};
    ctx->plan_lo[0] = nt1 > 0 ? tg[0] : 0;
    ctx->plan_hi[0] = nt1 > 0 ? tg[(size_t)nt1 - 1] : -1;
    ctx->plan_lo[1] = ntot > nt1 ? tg[(size_t)nt1] : 0;
    ctx->plan_hi[1] = ntot > nt1 ? tg[(size_t)ntot - 1] : -1;
    ctx->src_coords.swap(a);
    ctx->rec_coords.swap(b);
    ctx->src_counts.swap(k1);
    ctx->rec_counts.swap(k2);
    ctx->nsrc_dev = n1;
    ctx->nrec_dev = n2;
    return FD_OK;
}

// Argument checks shared by the stepping entry points.
// keep: the coordinates are those of the last upload (FD_KEEP_POINTS) and
// may be NULL.
int32_t check_points_arg(fd_ctx* ctx, int nt, const fd_points* p, const char* what,
                         bool keep = false) {
    if (!p) return FD_OK;
    if (p->n < 0) return fail(ctx, FD_ERR_INVALID_ARG, std::string("negative ") + what + " count");
    if (p->n > 0 && ((!p->coords && !keep) || (!p->data && nt > 0)))
        return fail(ctx, FD_ERR_INVALID_ARG, std::string(what) + " coords/data missing");
    return FD_OK;
}

// FD_KEEP_POINTS: reuse the point table of the last upload as it stands; the
// counts must be those of that upload (O(1) host work per call).
int32_t keep_points(fd_ctx* ctx, int n1, int n2) {
    if (ctx->nsrc_dev < 0 || n1 != ctx->nsrc_dev || n2 != ctx->nrec_dev)
        return fail(ctx, FD_ERR_INVALID_ARG,
                    "FD_KEEP_POINTS: the point counts differ from the last upload");
    return FD_OK;
}

double cell_volume(const fd_ctx* ctx) {
    const double* h = ctx->g.spacing;
    return ctx->g.ndim == 3 ? h[0] * h[1] * h[2] : h[0] * h[2];
}

// Shots a block of the tiled kernel advances together in plain stepping.
int ctx_sb(const fd_ctx* ctx) { return ctx->nshots > 1 ? ctx->shots_per_block : 1; }

// Shots per block of the gradient's launches: the context's value, halved
// until the tiled kernel has an acceleration-output variant for it.
int grad_sb(const fd_ctx* ctx) {
    int sb = ctx_sb(ctx);
    while (sb > 1 && !fd::acc_built(ctx->tile_cfg, sb)) sb /= 2;
    return sb;
}

// Coefficient part of an acoustic launch (fields set per step) for sb shots
// per block.
fd::AcousticStep acoustic_params(const fd_ctx* ctx, int sb) {
    fd::AcousticStep p;
    std::memset(&p, 0, sizeof(p));
    p.A = ctx->A;
    p.sig = ctx->damping ? ctx->sig : nullptr;
    p.dflag = ctx->g.ndim == 3 ? ctx->dflag : nullptr;  // all zero without damping
    if (ctx->damping && ctx->sep_ok && ctx->sep_use) {
        p.sx = ctx->prof;
        p.sy = ctx->prof + ctx->L.nx;
        p.sz = ctx->prof + ctx->L.nx + ctx->L.ny;
    }
    p.L = ctx->L;
    double c0 = 0.0;
    for (int a = 0; a < 3; ++a) c0 += ctx->w2[a][0];
    p.c0 = (float)c0;
    for (int j = 0; j <= fd::kMaxRadius; ++j) {
        p.cx[j] = ctx->w2[0][j];
        p.cy[j] = ctx->w2[1][j];
        p.cz[j] = ctx->w2[2][j];
    }
    p.nshots = ctx->nshots;
    p.shot_stride = ctx->L.volume;
    tile_grid(ctx, ctx->tile_y, ctx->zchunk_opt, ctx->radius, (ctx->nshots + sb - 1) / sb, &p,
              nullptr);
    return p;
}

// The sparse-point work of forward step n in one launch: the sources of step
// n into the new level un and, when not null, into rn (the second field of
// the anisotropic equations, damped like un; or the stored acceleration of
// a checkpointed run, which carries the source term without the damping
// divisor: rn_damped false), and the receivers of step n - 1 from uc = u^n,
// which step n only reads (nothing in the loop's first step, n_first).  The
// loop's last step is recorded after it (forward_last_record).
hipError_t forward_points(const fd_ctx* ctx, int n, int n_first, float* un, float* rn,
                          bool rn_damped, const float* uc, const fd_points* src, int nsrc,
                          const fd_points* rec, int nrec, const float* sig, float scale,
                          hipStream_t s) {
    const fd::InjectPlan none{};
    const bool rec_prev = nrec > 0 && n > n_first;
    return fd::launch_inject_record(un, rn, rn_damped, ctx->A, sig, ctx->pts,
                                    nsrc ? ctx->plan[0] : none,
                                    nsrc ? src->data + (size_t)n * nsrc : nullptr, scale, uc,
                                    ctx->pts + nsrc, rec_prev ? nrec : 0,
                                    rec_prev ? rec->data + (size_t)(n - 1) * nrec : nullptr, ctx->L,
                                    ctx->g.ndim, ctx->L.volume, s);
}
// The receivers of step n_end - 1 (the last of a loop over [n_first, n_end))
// from u = u^{n_end}.
hipError_t forward_last_record(const fd_ctx* ctx, int n_first, int n_end, const float* u,
                               const fd_points* rec, int nsrc, int nrec, hipStream_t s) {
    if (n_end <= n_first || nrec <= 0) return hipSuccess;
    return fd::launch_record(u, ctx->pts + nsrc, nrec, rec->data + (size_t)(n_end - 1) * nrec,
                             1.f, ctx->L, ctx->g.ndim, ctx->L.volume, s);
}

// One acoustic stencil launch over every shot: up <- step(uc, up),
// optionally storing A L uc (volumes of shot k at + k * volume).
hipError_t acoustic_stencil(const fd_ctx* ctx, fd::AcousticStep& p, const float* uc, float* up,
                            float* acc, int sb, hipStream_t s) {
    p.uc = uc;
    p.up = up;
    p.acc = acc;
    return fd::launch_acoustic(p, ctx->g.ndim, ctx->radius, ctx->variant, ctx->tile_cfg, sb, s);
}

// Checkpoint store layout for S = nshots wavefields (all regions 256-byte
// aligned):
//   ck[S][2 * nck]  dense fields (u^{n-1}, u^n) at n = 0, I, 2I, ... per shot
//   acc[I][S]       padded volumes: accelerations of one segment, the S
//                   shots of a step one after another
//   mu[2][S]        padded volumes: adjoint levels
//   gpart[S]        padded volumes: partial sums of the imaging condition over
//                   at most kFlushSteps adjoint steps
//   gsum[S]         dense fields: sums of the flushed partial sums
// With S = 1 this is the single-shot store.
struct Store {
    int nck = 0;
    int nshots = 1;
    int64_t dense = 0;       // floats per dense field (rounded to 64)
    float* ck = nullptr;
    float* acc = nullptr;
    float* mu[2] = {nullptr, nullptr};
    float* gpart = nullptr;
    float* gsum = nullptr;
    uint64_t bytes = 0;
    float* ckf(int shot, int k) const { return ck + ((int64_t)shot * 2 * nck + k) * dense; }
    float* slot(const fd_ctx* ctx, int i) const {
        return acc + (int64_t)i * nshots * ctx->L.volume;
    }
};

Store plan_store(const fd_ctx* ctx, int nt, int interval, char* base) {
    Store st;
    const Layout& L = ctx->L;
    const uint64_t S = (uint64_t)ctx->nshots;
    st.nshots = ctx->nshots;
    st.nck = nt > 0 ? (nt + interval - 1) / interval : 0;
    st.dense = round_up((int64_t)L.nx * L.ny * L.nz, 64);
    Carve cv;
    const uint64_t vol = (uint64_t)L.volume * sizeof(float);
    const uint64_t o_ck = cv.take(S * (uint64_t)(2 * st.nck) * st.dense * sizeof(float));
    const uint64_t o_acc = cv.take((uint64_t)interval * S * vol);
    const uint64_t o_mu0 = cv.take(S * vol);
    const uint64_t o_mu1 = cv.take(S * vol);
    const uint64_t o_gp = cv.take(S * vol);
    const uint64_t o_gs = cv.take(S * (uint64_t)st.dense * sizeof(float));
    st.bytes = cv.off;
    if (base) {
        st.ck = reinterpret_cast<float*>(base + o_ck);
        st.acc = reinterpret_cast<float*>(base + o_acc);
        st.mu[0] = reinterpret_cast<float*>(base + o_mu0);
        st.mu[1] = reinterpret_cast<float*>(base + o_mu1);
        st.gpart = reinterpret_cast<float*>(base + o_gp);
        st.gsum = reinterpret_cast<float*>(base + o_gs);
    }
    return st;
}

// interval <= 0: minimise 2 (nt / I) dense + I volume floats.
int resolve_interval(const fd_ctx* ctx, int nt, int interval) {
    if (interval > 0) return interval < nt ? interval : (nt > 0 ? nt : 1);
    const double dense = (double)ctx->L.nx * ctx->L.ny * ctx->L.nz;
    const double best = std::sqrt(2.0 * nt * dense / (double)ctx->L.volume);
    int I = (int)std::lround(best);
    if (I < 1) I = 1;
    if (I > nt) I = nt > 0 ? nt : 1;
    return I;
}

hipError_t refresh_flags(fd_ctx* ctx, hipStream_t s) {
    if (!ctx->damping || ctx->g.ndim != 3) return hipSuccess;
    if (ctx->tile_y < min_tile_y()) return hipErrorInvalidValue;  // flags sized for min_tile_y
    const Layout& L = ctx->L;
    const int ntx = (L.nx + fd::kTileX - 1) / fd::kTileX;
    const int nty = (L.ny + ctx->tile_y - 1) / ctx->tile_y;
    return fd::launch_damping_flags(ctx->sig, ctx->dflag, L, ctx->tile_y, ntx, nty, s);
}

// ---------------------------------------------------------------------------
// Setup on the host: the per-point coefficients are derived in FP64 from the
// FP32 model and rounded once to FP32 (section 4.1 weights aside, these are
// the factors of Eq. (Acou) and Eq. (TTI) with Eq. (DiffOp)).
// ---------------------------------------------------------------------------

// Host threads of the setup passes.
int host_threads(int64_t n) {
    const unsigned hw = std::thread::hardware_concurrency();
    const int nt = (int)std::min<unsigned>(hw ? hw : 1, 32);
    return n < ((int64_t)1 << 16) ? 1 : nt;
}

// Runs f(t, i0, i1) for t = 0 .. host_threads(n) - 1 over consecutive ranges
// covering [0, n), each on a thread of its own; a range whose thread cannot
// be started runs on the calling thread.
template <class F>
void parallel_for(int64_t n, F f) {
    const int nt = host_threads(n);
    if (nt <= 1) {
        f(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)nt);
    const int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a >= b) continue;
        bool started = false;
        try {
            th.emplace_back(f, t, a, b);
            started = true;
        } catch (const std::system_error&) {
        }
        if (!started) f(t, a, b);
    }
    for (auto& t : th) t.join();
}

// Copy one dense FP32 model field (device) to the host.
hipError_t fetch_field(const float* dev, int64_t n, std::vector<float>& host) {
    host.resize((size_t)n);
    return hipMemcpy(host.data(), dev, (size_t)n * sizeof(float), hipMemcpyDeviceToHost);
}

// Upload a dense host field into the padded volume `vol` through the dense
// staging area `stage` (stream-ordered; the caller keeps `host` alive until
// the stream has passed the copy).
hipError_t upload_field(const std::vector<float>& host, float* stage, float* vol, const Layout& L,
                        hipStream_t s) {
    hipError_t e = hipMemcpyAsync(stage, host.data(), host.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = fd::launch_unpack(stage, vol, L, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // stage is reused by the next field
    return e;
}

struct ModelCheck {
    double vmax = 0.0;  // fastest speed: v, or v sqrt(1 + 2 eps) for VTI and TTI
    bool bad = false;   // a non-finite or out-of-range value
    bool dgt = false;   // delta > epsilon somewhere
};

// Derives A = dt^2 v^2, s = eta dt / 2, e = 1 + 2 eps, d = sqrt(1 + 2 delta)
// and the six G_zbar_zbar weights
//   c1 = sin^2(th) cos^2(ph), c2 = sin^2(th) sin^2(ph), c3 = cos^2(th),
//   c4 = sin(2 ph) sin^2(th), c5 = sin(ph) sin(2 th), c6 = cos(ph) sin(2 th)
// in FP64 on the host, rounds each once to FP32 and uploads it into its
// volume.  `stage` is a device area of at least nx ny nz floats.
hipError_t derive_coefficients(fd_ctx* ctx, const fd_model* m, float* stage, hipStream_t s,
                               ModelCheck& chk) {
    const Layout& L = ctx->L;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    const double dt = ctx->g.dt;
    std::vector<float> vel, a, b, out0, out1;
    hipError_t e = fetch_field(m->vel, n, vel);
    if (e != hipSuccess) return e;
    // body(i) returns flag bits for point i; a pass returns their OR
    auto flag_pass = [&](auto body) {
        std::vector<unsigned char> part((size_t)host_threads(n), 0);
        parallel_for(n, [&](int t, int64_t i0, int64_t i1) {
            unsigned char bd = 0;
            for (int64_t i = i0; i < i1; ++i) bd |= body(i);
            part[(size_t)t] = bd;
        });
        unsigned char all = 0;
        for (unsigned char c : part) all |= c;
        return all;
    };
    // A = dt^2 v^2
    out0.resize((size_t)n);
    unsigned char fl = flag_pass([&](int64_t i) -> unsigned char {
        const double v = vel[i];
        out0[i] = (float)(dt * dt * v * v);
        return (v > 0.0 && std::isfinite(v)) ? 0 : 1;
    });
    chk.bad |= fl != 0;
    e = upload_field(out0, stage, ctx->A, L, s);
    if (e != hipSuccess) return e;
    // the largest finite sp(i)
    auto max_speed = [&](auto sp) {
        std::vector<double> part((size_t)host_threads(n), 0.0);
        parallel_for(n, [&](int t, int64_t i0, int64_t i1) {
            double mx = 0.0;
            for (int64_t i = i0; i < i1; ++i) {
                const double v = sp(i);
                if (std::isfinite(v) && v > mx) mx = v;
            }
            part[(size_t)t] = mx;
        });
        double mx = 0.0;
        for (double v : part) mx = std::max(mx, v);
        return mx;
    };
    if (ctx->e) {  // VTI and TTI: e = 1 + 2 eps, d = sqrt(1 + 2 delta)
        e = fetch_field(m->epsilon, n, a);
        if (e == hipSuccess) e = fetch_field(m->delta, n, b);
        if (e != hipSuccess) return e;
        out1.resize((size_t)n);
        fl = flag_pass([&](int64_t i) -> unsigned char {
            const double ep = a[i], de = b[i];
            const double ev = 1.0 + 2.0 * ep, d2 = 1.0 + 2.0 * de;
            out0[i] = (float)ev;
            out1[i] = (float)std::sqrt(std::max(d2, 0.0));
            unsigned char r = 0;
            if (!std::isfinite(ep) || !std::isfinite(de) || !(ev > 0.0) || !(d2 > 0.0)) r |= 1;
            if (de > ep) r |= 2;
            return r;
        });
        chk.bad |= (fl & 1) != 0;
        chk.dgt = (fl & 2) != 0;
        e = upload_field(out0, stage, ctx->e, L, s);
        if (e == hipSuccess) e = upload_field(out1, stage, ctx->d, L, s);
        if (e != hipSuccess) return e;
        chk.vmax = max_speed([&](int64_t i) {
            return (double)vel[i] * std::sqrt(std::max(1.0 + 2.0 * (double)a[i], 0.0));
        });
    } else {
        chk.vmax = max_speed([&](int64_t i) { return (double)vel[i]; });
    }
    vel.clear();
    vel.shrink_to_fit();
    if (ctx->damping) {  // s = eta dt / 2
        e = fetch_field(m->eta, n, a);
        if (e != hipSuccess) return e;
        fl = flag_pass([&](int64_t i) -> unsigned char {
            const double et = a[i];
            out0[i] = (float)(0.5 * dt * et);
            return (et >= 0.0 && std::isfinite(et)) ? 0 : 1;
        });
        chk.bad |= fl != 0;
        e = upload_field(out0, stage, ctx->sig, L, s);
        if (e != hipSuccess) return e;
    }
    if (ctx->tti) {  // the weights of Dxx, Dyy, Dzz, Dxy, Dyz, Dxz in G_zbar_zbar
        e = fetch_field(m->theta, n, a);
        if (e == hipSuccess) e = fetch_field(m->phi, n, b);
        if (e != hipSuccess) return e;
        std::vector<float> c[6];
        for (auto& v : c) v.resize((size_t)n);
        fl = flag_pass([&](int64_t i) -> unsigned char {
            const double th = a[i], ph = b[i];
            const double st = std::sin(th), ct = std::cos(th), sp = std::sin(ph), cp = std::cos(ph);
            const double st2 = st * st;
            c[0][i] = (float)(st2 * cp * cp);
            c[1][i] = (float)(st2 * sp * sp);
            c[2][i] = (float)(ct * ct);
            c[3][i] = (float)(2.0 * sp * cp * st2);
            c[4][i] = (float)(sp * 2.0 * st * ct);
            c[5][i] = (float)(cp * 2.0 * st * ct);
            return (std::isfinite(th) && std::isfinite(ph)) ? 0 : 1;
        });
        chk.bad |= fl != 0;
        for (int k = 0; k < 6 && e == hipSuccess; ++k) e = upload_field(c[k], stage, ctx->c[k], L, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int32_t fd_stencil_weights(int32_t space_order, int32_t deriv, double* w) {
    if (!w) return FD_ERR_INVALID_ARG;
    if (space_order > FD_MAX_SPACE_ORDER && space_order % 2 == 0) return FD_ERR_UNSUPPORTED;
    return central_weights(space_order, deriv, w) ? FD_OK : FD_ERR_INVALID_ARG;
}

int32_t fd_cfl_dt(const fd_grid* grid, double vmax, double* dt_max) {
    std::string msg;
    if (!dt_max || !(vmax > 0.0)) return FD_ERR_INVALID_ARG;
    fd_grid g = *grid;
    g.dt = 1.0;  // dt itself is not validated here
    const int32_t rc = validate_grid(&g, msg);
    if (rc != FD_OK) return rc;
    *dt_max = cfl_dt(grid, vmax);
    return FD_OK;
}

int32_t fd_workspace_bytes_shots(const fd_grid* grid, int32_t nshots, int32_t max_points,
                                 uint64_t* bytes) {
    std::string msg;
    if (!bytes || max_points < 0 || max_points > kMaxPoints || nshots < 1 || nshots > kMaxShots)
        return FD_ERR_INVALID_ARG;
    const int32_t rc = validate_grid(grid, msg);
    if (rc != FD_OK) return rc;
    if (nshots > 1 && grid->physics != FD_ACOUSTIC) return FD_ERR_UNSUPPORTED;
    const Layout L = make_layout(grid);
    *bytes = plan_workspace(grid, L, nshots, max_points, nullptr, nullptr);
    return FD_OK;
}

int32_t fd_workspace_bytes(const fd_grid* grid, int32_t max_points, uint64_t* bytes) {
    return fd_workspace_bytes_shots(grid, 1, max_points, bytes);
}

int32_t fd_setup(const fd_grid* grid, const fd_model* model, void* workspace,
                 uint64_t workspace_bytes, int32_t max_points, void* stream, fd_ctx** out) {
    return fd_setup_shots(grid, model, 1, workspace, workspace_bytes, max_points, stream, out);
}

int32_t fd_setup_shots(const fd_grid* grid, const fd_model* model, int32_t nshots,
                       void* workspace, uint64_t workspace_bytes, int32_t max_points,
                       void* stream, fd_ctx** out) {
    std::string msg;
    if (!out) return FD_ERR_INVALID_ARG;
    *out = nullptr;
    int32_t rc = validate_grid(grid, msg);
    if (rc != FD_OK) return rc;
    if (!model || !model->vel || max_points < 0 || max_points > kMaxPoints || !workspace)
        return FD_ERR_INVALID_ARG;
    if (nshots < 1 || nshots > kMaxShots) return FD_ERR_INVALID_ARG;
    const bool tti = grid->physics == FD_TTI;
    const bool vti = grid->physics == FD_VTI;
    if ((tti || vti) && nshots > 1) return FD_ERR_UNSUPPORTED;
    if (tti && (!model->epsilon || !model->delta || !model->theta || !model->phi))
        return FD_ERR_INVALID_ARG;
    if (vti && (!model->epsilon || !model->delta)) return FD_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return FD_ERR_WORKSPACE;
    const Layout L = make_layout(grid);
    const uint64_t need = plan_workspace(grid, L, nshots, max_points, nullptr, nullptr);
    if (workspace_bytes < need) return FD_ERR_WORKSPACE;

    fd_ctx* ctx = new (std::nothrow) fd_ctx();
    if (!ctx) return FD_ERR_INVALID_ARG;
    ctx->g = *grid;
    ctx->radius = grid->space_order / 2;
    ctx->L = L;
    ctx->tti = tti;
    ctx->vti = vti;
    ctx->nshots = nshots;
    ctx->shots_per_block = default_shots_per_block(ctx->radius, nshots);
    ctx->damping = model->eta != nullptr;
    ctx->max_points = max_points;
    ctx->cur = 1;
    ctx->variant = 0;
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 0;
        ctx->ncu = ncu;
    }
    ctx->tile_cfg = tti ? tti_default_tile(ctx)
                    : vti ? 0
                    : nshots > 1 ? shots_tile(ctx->radius) : default_tile(ctx);
    ctx->zchunk_opt = 0;
    ctx->tile_y = tti ? fd::tti_tile_y(ctx->tile_cfg)
                      : vti ? fd::vti_tile_y() : fd::acoustic_tile_y(ctx->tile_cfg);
    ctx->nsrc_dev = ctx->nrec_dev = -1;
    ctx->flags_stale = false;
    ctx->ck_store = nullptr;
    ctx->ck_nt = ctx->ck_interval = 0;
    ctx->ck_last_acc = false;
    ctx->sep_ok = false;
    ctx->sep_use = true;
    ctx->fuse_image = true;
    plan_workspace(grid, L, nshots, max_points, ctx, static_cast<char*>(workspace));
    hipStream_t s = static_cast<hipStream_t>(stream);

    // zero everything (ghost rings must be zero), then derive coefficients
    hipError_t he = fd::launch_fill_zero(static_cast<float*>(workspace),
                                         (int64_t)(need / sizeof(float)), s);
    if (he != hipSuccess) {
        hip_fail(ctx, he, "fill");
        delete ctx;
        return FD_ERR_DEVICE;
    }
    // coefficients in FP64 on the host (the first wavefield level is the
    // staging area of the uploads and is cleared again afterwards); the
    // host copies of the model are volume-sized
    ModelCheck chk;
    if (guarded(nullptr, [&]() -> int32_t {
            he = derive_coefficients(ctx, model, ctx->u[0], s, chk);
            return FD_OK;
        }) != FD_OK) {
        (void)hipStreamSynchronize(s);  // no upload may still read the host copies
        delete ctx;
        return FD_ERR_HOST;
    }
    if (he == hipSuccess) he = fd::launch_fill_zero(ctx->u[0], L.volume * nshots, s);
    if (he == hipSuccess) he = refresh_flags(ctx, s);
    const bool try_sep = ctx->damping && grid->ndim == 3;
    if (he == hipSuccess && try_sep)
        he = fd::launch_damping_profiles(ctx->sig, L, ctx->prof, ctx->prof + L.nx,
                                         ctx->prof + L.nx + L.ny, ctx->reduce + 4, s);
    uint32_t red[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (he == hipSuccess) he = hipMemcpyAsync(red, ctx->reduce, sizeof(red), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) {
        hip_fail(ctx, he, "setup");
        delete ctx;
        return FD_ERR_DEVICE;
    }
    if (chk.bad) {
        delete ctx;
        return FD_ERR_NONFINITE;
    }
    if (chk.dgt) {
        delete ctx;
        return FD_ERR_INVALID_ARG;  // delta > epsilon: unstable pseudo-acoustic mode
    }
    if (try_sep) {
        float dmax, smax;
        std::memcpy(&dmax, &red[4], sizeof(float));
        std::memcpy(&smax, &red[5], sizeof(float));
        ctx->sep_ok = smax > 0.f && dmax <= std::ldexp(smax, -20);
    }
    const double vmax = chk.vmax;
    if (!(vmax > 0.0)) {
        delete ctx;
        return FD_ERR_NONFINITE;
    }
    if (grid->dt > cfl_dt(grid, vmax) * (1.0 + 1e-12)) {
        delete ctx;
        return FD_ERR_UNSTABLE_DT;
    }
    // stencil weights / h or h^2, rounded once to float
    double w2[fd::kMaxRadius + 1], w1[fd::kMaxRadius + 1];
    central_weights(grid->space_order, 2, w2);
    central_weights(grid->space_order, 1, w1);
    for (int a = 0; a < 3; ++a) {
        const bool used = !(grid->ndim == 2 && a == 1);
        const double h = grid->spacing[a];
        for (int j = 0; j <= fd::kMaxRadius; ++j) {
            ctx->w2[a][j] = (used && j <= ctx->radius) ? (float)(w2[j] / (h * h)) : 0.f;
            ctx->w1[a][j] = (used && j <= ctx->radius) ? (float)(w1[j] / h) : 0.f;
        }
    }
    *out = ctx;
    return FD_OK;
}

int32_t fd_set_option(fd_ctx* ctx, int32_t option, int64_t value) {
    if (!ctx) return FD_ERR_INVALID_ARG;
    switch (option) {
        case FD_OPT_KERNEL:
            if (value != 0 && value != 1) return fail(ctx, FD_ERR_INVALID_ARG, "kernel variant 0 or 1");
            ctx->variant = (int)value;
            return FD_OK;
        case FD_OPT_ZCHUNK:
            if (value < 0 || value > (1 << 20)) return fail(ctx, FD_ERR_INVALID_ARG, "zchunk range");
            ctx->zchunk_opt = (int)value;
            return FD_OK;
        case FD_OPT_TILE: {
            if (ctx->vti) return fail(ctx, FD_ERR_UNSUPPORTED, "the VTI kernel has one tile shape");
            if (ctx->tti) {
                const int v = value < 0 ? tti_default_tile(ctx) : (int)value;
                if (v > 2) return fail(ctx, FD_ERR_INVALID_ARG, "TTI tile configuration is 0..2");
                if (v == 2 && ctx->radius > fd::kTTITallMaxRadius)
                    return fail(ctx, FD_ERR_UNSUPPORTED,
                                "the 64x15 TTI tile is built for space orders up to 8");
                ctx->tile_cfg = v;
                ctx->tile_y = fd::tti_tile_y(v);
                ctx->flags_stale = true;  // rebuilt on the caller's stream by fd_forward
                return FD_OK;
            }
            const int v = value < 0 ? (ctx->nshots > 1 ? shots_tile(ctx->radius)
                                                       : default_tile(ctx))
                                    : (int)value;
            if (v < 0 || v > 4) return fail(ctx, FD_ERR_INVALID_ARG, "tile configuration is 0..4");
            if (ctx->nshots > 1 && ctx->shots_per_block > 1 && v != 0 && v != 2)
                return fail(ctx, FD_ERR_UNSUPPORTED,
                            "several shots per block are built for tile configurations 0 and 2");
            ctx->tile_cfg = v;
            ctx->tile_y = fd::acoustic_tile_y(v);
            ctx->flags_stale = true;  // rebuilt on the caller's stream by fd_forward
            return FD_OK;
        }
        case FD_OPT_FUSED_IMAGING:
            if (value != 0 && value != 1)
                return fail(ctx, FD_ERR_INVALID_ARG, "fused imaging option 0 or 1");
            ctx->fuse_image = value == 1;
            return FD_OK;
        case FD_OPT_DAMPING_PROFILE:
            if (value != 0 && value != 1)
                return fail(ctx, FD_ERR_INVALID_ARG, "damping profile option 0 or 1");
            ctx->sep_use = value == 1;
            return FD_OK;
        case FD_OPT_SHOTS_PER_BLOCK: {
            const int v = value <= 0 ? default_shots_per_block(ctx->radius, ctx->nshots)
                                     : (int)value;
            if (v != 1 && v != 2 && v != 4)
                return fail(ctx, FD_ERR_INVALID_ARG, "shots per block is 1, 2 or 4");
            if (v > 1 && ctx->tile_cfg != 0 && ctx->tile_cfg != 2)
                return fail(ctx, FD_ERR_UNSUPPORTED,
                            "several shots per block are built for tile configurations 0 and 2");
            ctx->shots_per_block = v;
            return FD_OK;
        }
        default: return fail(ctx, FD_ERR_INVALID_ARG, "unknown option");
    }
}

int32_t fd_get_option(const fd_ctx* ctx, int32_t option, int64_t* value) {
    if (!ctx || !value) return FD_ERR_INVALID_ARG;
    switch (option) {
        case FD_OPT_KERNEL: *value = ctx->variant; return FD_OK;
        case FD_OPT_ZCHUNK: *value = ctx->zchunk_opt; return FD_OK;
        case FD_OPT_TILE: *value = ctx->tile_cfg; return FD_OK;
        case FD_OPT_SHOTS_PER_BLOCK: *value = ctx->shots_per_block; return FD_OK;
        case FD_OPT_DAMPING_PROFILE: *value = ctx->sep_use ? 1 : 0; return FD_OK;
        case FD_OPT_FUSED_IMAGING: *value = ctx->fuse_image ? 1 : 0; return FD_OK;
        default: return FD_ERR_INVALID_ARG;
    }
}

int32_t fd_forward(fd_ctx* ctx, int32_t nt, const fd_points* src, const fd_points* rec,
                   int32_t flags, void* stream) {
    return guarded(ctx, [&]() -> int32_t {
        if (!ctx) return FD_ERR_INVALID_ARG;
        ctx->err.clear();
        if (ctx->nshots > 1)
            return fail(ctx, FD_ERR_INVALID_ARG, "a context of several shots steps with fd_forward_shots");
        if (nt < 0) return fail(ctx, FD_ERR_INVALID_ARG, "nt < 0");
        const bool keep = (flags & FD_KEEP_POINTS) != 0;
        int32_t rc = check_points_arg(ctx, nt, src, "source", keep);
        if (rc == FD_OK) rc = check_points_arg(ctx, nt, rec, "receiver", keep);
        if (rc != FD_OK) return rc;
        const int nsrc = src ? src->n : 0, nrec = rec ? rec->n : 0;
        if ((int64_t)nsrc + nrec > ctx->max_points)
            return fail(ctx, FD_ERR_INVALID_ARG, "more points than max_points");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int nd = ctx->g.ndim;
        rc = keep ? keep_points(ctx, nsrc, nrec)
                  : sync_points(ctx, nsrc, src ? src->coords : nullptr, nrec,
                                rec ? rec->coords : nullptr, "source", "receiver", s);
        if (rc != FD_OK) return rc;

        hipError_t he = hipSuccess;
        if (ctx->flags_stale) {
            he = refresh_flags(ctx, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "damping flags");
            ctx->flags_stale = false;
        }
        if (flags & FD_ZERO_STATE) {
            for (int k = 0; k < 2 && he == hipSuccess; ++k) he = fd::launch_fill_zero(ctx->u[k], ctx->L.volume, s);
            if (ctx->r[0])
                for (int k = 0; k < 2 && he == hipSuccess; ++k)
                    he = fd::launch_fill_zero(ctx->r[k], ctx->L.volume, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "zero state");
        }
        const float scale = (float)(1.0 / cell_volume(ctx));
        const SparsePoint* spts = ctx->pts;
        const SparsePoint* rpts = ctx->pts + nsrc;
        const float* sig = ctx->damping ? ctx->sig : nullptr;

        if (ctx->vti) {
            fd::VTIStep p;
            std::memset(&p, 0, sizeof(p));
            p.A = ctx->A;
            p.sig = sig;
            p.dflag = nd == 3 ? ctx->dflag : nullptr;
            p.e = ctx->e;
            p.d = ctx->d;
            if (nd == 3 && ctx->damping && ctx->sep_ok && ctx->sep_use) {
                p.sx = ctx->prof;
                p.sy = ctx->prof + ctx->L.nx;
                p.sz = ctx->prof + ctx->L.nx + ctx->L.ny;
            }
            p.L = ctx->L;
            p.c0h = (float)((double)ctx->w2[0][0] + (nd == 3 ? (double)ctx->w2[1][0] : 0.0));
            p.c0z = ctx->w2[2][0];
            for (int j = 0; j <= fd::kMaxRadius; ++j) {
                p.cx[j] = ctx->w2[0][j];
                p.cy[j] = ctx->w2[1][j];
                p.cz[j] = ctx->w2[2][j];
            }
            fd::TTIStep grid_only;
            tile_grid(ctx, ctx->tile_y, ctx->zchunk_opt, ctx->radius, 1, nullptr, &grid_only);
            p.ntx = grid_only.ntx;
            p.nty = grid_only.nty;
            p.nzc = grid_only.nzc;
            p.zchunk = grid_only.zchunk;
            p.ntiles = grid_only.ntiles;
            p.nblocks = grid_only.nblocks;
            for (int n = 0; n < nt; ++n) {
                float* pn = ctx->u[1 - ctx->cur];
                float* rn = ctx->r[1 - ctx->cur];
                p.pc = ctx->u[ctx->cur];
                p.rc = ctx->r[ctx->cur];
                p.pp = pn;
                p.rp = rn;
                he = fd::launch_vti(p, nd, ctx->radius, ctx->variant, s);
                if (he == hipSuccess)
                    he = forward_points(ctx, n, 0, pn, rn, true, p.pc, src, nsrc, rec, nrec, sig,
                                        scale, s);
                if (he != hipSuccess) return hip_fail(ctx, he, "step");
                ctx->cur = 1 - ctx->cur;
            }
            he = forward_last_record(ctx, 0, nt, ctx->u[ctx->cur], rec, nsrc, nrec, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "step");
        } else if (!ctx->tti) {
            fd::AcousticStep p = acoustic_params(ctx, 1);
            // The receivers of step n - 1 are sampled during step n from the
            // level u^n, which step n only reads, and one launch after the
            // loop samples the last step.  2D (the direct kernel, bound by
            // launches): step n's stencil launch also injects the sources
            // into the u^{n+1} it writes and does that sampling.  3D: one
            // launch after the stencil injects and samples.
            const bool fuse_rec = nrec > 0;
            const bool fuse_inj = nd == 2 && nsrc > 0;
            if (fuse_inj) {
                p.inj = ctx->plan[0];
                p.inj_pts = spts;
                p.inj_scale = scale;
                p.inj_lo = ctx->plan_lo[0];
                p.inj_hi = ctx->plan_hi[0];
            }
            for (int n = 0; n < nt; ++n) {
                float* un = ctx->u[1 - ctx->cur];  // holds u^{n-1}, receives u^{n+1}
                p.rec_n = 0;
                if (nd == 2 && fuse_rec && n > 0) {
                    p.rec_pts = rpts;
                    p.rec_out = rec->data + (size_t)(n - 1) * nrec;
                    p.rec_n = nrec;
                }
                if (fuse_inj) p.inj_q = src->data + (size_t)n * nsrc;
                const float* uc = ctx->u[ctx->cur];
                he = acoustic_stencil(ctx, p, uc, un, nullptr, 1, s);
                if (he == hipSuccess && nd == 3)
                    he = forward_points(ctx, n, 0, un, nullptr, true, uc, src, nsrc, rec, nrec, sig,
                                        scale, s);
                if (he != hipSuccess) return hip_fail(ctx, he, "step");
                ctx->cur = 1 - ctx->cur;
            }
            he = forward_last_record(ctx, 0, nt, ctx->u[ctx->cur], rec, nsrc, nrec, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "step");
        } else {
            fd::TTIStep p;
            std::memset(&p, 0, sizeof(p));
            p.A = ctx->A;
            p.sig = sig;
            p.dflag = ctx->dflag;
            p.e = ctx->e;
            p.d = ctx->d;
            for (int k = 0; k < 6; ++k) p.c[k] = ctx->c[k];
            if (ctx->damping && ctx->sep_ok && ctx->sep_use) {
                p.sx = ctx->prof;
                p.sy = ctx->prof + ctx->L.nx;
                p.sz = ctx->prof + ctx->L.nx + ctx->L.ny;
            }
            p.L = ctx->L;
            for (int j = 0; j <= fd::kMaxRadius; ++j) {
                p.w2x[j] = ctx->w2[0][j];
                p.w2y[j] = ctx->w2[1][j];
                p.w2z[j] = ctx->w2[2][j];
                p.w1x[j] = ctx->w1[0][j];
                p.w1y[j] = ctx->w1[1][j];
                p.w1z[j] = ctx->w1[2][j];
            }
            tile_grid(ctx, ctx->tile_y, ctx->zchunk_opt, ctx->radius, 1, nullptr, &p);
            for (int n = 0; n < nt; ++n) {
                float* pn = ctx->u[1 - ctx->cur];
                float* rn = ctx->r[1 - ctx->cur];
                p.pc = ctx->u[ctx->cur];
                p.rc = ctx->r[ctx->cur];
                p.pp = pn;
                p.rp = rn;
                he = fd::launch_tti(p, ctx->radius, ctx->variant, ctx->tile_cfg, s);
                if (he == hipSuccess)
                    he = forward_points(ctx, n, 0, pn, rn, true, p.pc, src, nsrc, rec, nrec, sig,
                                        scale, s);
                if (he != hipSuccess) return hip_fail(ctx, he, "step");
                ctx->cur = 1 - ctx->cur;
            }
            he = forward_last_record(ctx, 0, nt, ctx->u[ctx->cur], rec, nsrc, nrec, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "step");
        }
        return FD_OK;
    });
}

int32_t fd_checkpoint_bytes(const fd_ctx* ctx, int32_t nt, int32_t interval, uint64_t* bytes,
                            int32_t* interval_out) {
    if (!ctx || !bytes || nt < 0) return FD_ERR_INVALID_ARG;
    if (ctx->tti || ctx->vti) return FD_ERR_UNSUPPORTED;
    const int I = resolve_interval(ctx, nt, interval);
    *bytes = plan_store(ctx, nt, I, nullptr).bytes;
    if (interval_out) *interval_out = I;
    return FD_OK;
}

namespace {

int32_t check_store(fd_ctx* ctx, int nt, int I, void* store, uint64_t store_bytes) {
    if (!store || reinterpret_cast<uintptr_t>(store) % 256)
        return fail(ctx, FD_ERR_WORKSPACE, "checkpoint store missing or not 256-byte aligned");
    if (store_bytes < plan_store(ctx, nt, I, nullptr).bytes)
        return fail(ctx, FD_ERR_WORKSPACE, "checkpoint store smaller than fd_checkpoint_bytes");
    return FD_OK;
}

// Per-shot point counts of a multi-shot call must cover the points exactly;
// a single-shot context takes none (all points in its one shot).
int32_t check_counts(fd_ctx* ctx, const int32_t* k, int n, const char* what) {
    if (ctx->nshots == 1) {
        if (k && n != k[0])
            return fail(ctx, FD_ERR_INVALID_ARG, std::string(what) + " counts do not sum to n");
        return FD_OK;
    }
    if (n == 0) return FD_OK;
    if (!k) return fail(ctx, FD_ERR_INVALID_ARG, std::string(what) + " counts missing");
    int64_t t = 0;
    for (int i = 0; i < ctx->nshots; ++i) {
        if (k[i] < 0) return fail(ctx, FD_ERR_INVALID_ARG, std::string(what) + " count < 0");
        t += k[i];
    }
    if (t != n) return fail(ctx, FD_ERR_INVALID_ARG, std::string(what) + " counts do not sum to n");
    return FD_OK;
}

// Forward steps n0 .. n1-1 of every shot from the held state, storing the
// accelerations of step n into slot n - n0 when `slots` is set and sampling
// receivers when `nrec` > 0.
hipError_t forward_segment(fd_ctx* ctx, fd::AcousticStep& p, int sb, const Store* slots, int n0,
                           int n1, const fd_points* src, int nsrc, const fd_points* rec, int nrec,
                           hipStream_t s) {
    const float scale = (float)(1.0 / cell_volume(ctx));
    const float* sig = ctx->damping ? ctx->sig : nullptr;
    hipError_t he = hipSuccess;
    for (int n = n0; n < n1 && he == hipSuccess; ++n) {
        float* un = ctx->u[1 - ctx->cur];
        const float* uc = ctx->u[ctx->cur];
        float* acc = slots ? slots->slot(ctx, n - n0) : nullptr;
        he = acoustic_stencil(ctx, p, uc, un, acc, sb, s);
        // the acceleration carries the source term without the damping
        // divisor; the receivers of step n - 1 come from u^n (the first
        // step of a segment records nothing: the previous segment's last
        // step is recorded at its end)
        if (he == hipSuccess)
            he = forward_points(ctx, n, n0, un, acc, false, uc, src, nsrc, rec, nrec, sig, scale, s);
        ctx->cur = 1 - ctx->cur;
    }
    if (he == hipSuccess) he = forward_last_record(ctx, n0, n1, ctx->u[ctx->cur], rec, nsrc, nrec, s);
    return he;
}

// One adjoint step in mu = dt^2 v^2 lambda for every shot: mu^k from
// (mu^{k+1}, mu^{k+2}) by the forward stencil, then B R^T d'^{k-1} / (1 + s)
// injected at the receivers (the forward injection without the 1 / prod(h)
// source scaling), and dJ/dq^{k-1} = S mu^k / prod(h) sampled at the sources.
hipError_t adjoint_step(fd_ctx* ctx, fd::AcousticStep& p, int sb, const float* mu1, float* mu2,
                        int k, int nsrc, float* qgrad, const fd_points* adj, int nadj,
                        hipStream_t s) {
    const int nd = ctx->g.ndim;
    const float* sig = ctx->damping ? ctx->sig : nullptr;
    hipError_t he = acoustic_stencil(ctx, p, mu1, mu2, nullptr, sb, s);
    if (he == hipSuccess && nadj)
        he = fd::launch_inject(mu2, ctx->A, sig, ctx->pts + nsrc, ctx->plan[1],
                               adj->data + (size_t)(k - 1) * nadj, 1.f, ctx->L, nd, ctx->L.volume,
                               s);
    if (he == hipSuccess && nsrc && qgrad)
        he = fd::launch_record(mu2, ctx->pts, nsrc, qgrad + (size_t)(k - 1) * nsrc,
                               (float)(1.0 / cell_volume(ctx)), ctx->L, nd, ctx->L.volume, s);
    return he;
}

// Dense checkpoint k of every shot from / into the held level `f`.
hipError_t pack_shots(const fd_ctx* ctx, const float* f, const Store& st, int k, hipStream_t s) {
    hipError_t he = hipSuccess;
    for (int i = 0; i < ctx->nshots && he == hipSuccess; ++i)
        he = fd::launch_pack(f + (int64_t)i * ctx->L.volume, st.ckf(i, k), ctx->L, s);
    return he;
}
hipError_t unpack_shots(const fd_ctx* ctx, const Store& st, int k, float* f, hipStream_t s) {
    hipError_t he = hipSuccess;
    for (int i = 0; i < ctx->nshots && he == hipSuccess; ++i)
        he = fd::launch_unpack(st.ckf(i, k), f + (int64_t)i * ctx->L.volume, ctx->L, s);
    return he;
}

}  // namespace

int32_t fd_forward_checkpointed_shots(fd_ctx* ctx, int32_t nt, const fd_points* src,
                                      const int32_t* src_counts, const fd_points* rec,
                                      const int32_t* rec_counts, int32_t interval, void* store,
                                      uint64_t store_bytes, void* stream) {
    return guarded(ctx, [&]() -> int32_t {
        if (!ctx) return FD_ERR_INVALID_ARG;
        ctx->err.clear();
        if (ctx->tti || ctx->vti)
            return fail(ctx, FD_ERR_UNSUPPORTED, "gradients are built for acoustic only");
        if (nt < 0) return fail(ctx, FD_ERR_INVALID_ARG, "nt < 0");
        int32_t rc = check_points_arg(ctx, nt, src, "source");
        if (rc == FD_OK) rc = check_points_arg(ctx, nt, rec, "receiver");
        if (rc != FD_OK) return rc;
        const int nsrc = src ? src->n : 0, nrec = rec ? rec->n : 0;
        if ((int64_t)nsrc + nrec > ctx->max_points)
            return fail(ctx, FD_ERR_INVALID_ARG, "more points than max_points");
        rc = check_counts(ctx, src_counts, nsrc, "source");
        if (rc == FD_OK) rc = check_counts(ctx, rec_counts, nrec, "receiver");
        if (rc != FD_OK) return rc;
        const int I = resolve_interval(ctx, nt, interval);
        rc = check_store(ctx, nt, I, store, store_bytes);
        if (rc != FD_OK) return rc;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const bool multi = ctx->nshots > 1;
        rc = sync_points(ctx, nsrc, src ? src->coords : nullptr, nrec, rec ? rec->coords : nullptr,
                         "source", "receiver", s, multi && nsrc ? src_counts : nullptr,
                         multi && nrec ? rec_counts : nullptr);
        if (rc != FD_OK) return rc;
        ctx->ck_store = nullptr;
        hipError_t he = hipSuccess;
        if (ctx->flags_stale) {
            he = refresh_flags(ctx, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "damping flags");
            ctx->flags_stale = false;
        }
        for (int k = 0; k < 2 && he == hipSuccess; ++k)
            he = fd::launch_fill_zero(ctx->u[k], ctx->L.volume * ctx->nshots, s);
        const Store st = plan_store(ctx, nt, I, static_cast<char*>(store));
        const int sb = grad_sb(ctx);
        fd::AcousticStep p = acoustic_params(ctx, sb);
        for (int j = 0; j < st.nck && he == hipSuccess; ++j) {
            const int n0 = j * I, n1 = n0 + I < nt ? n0 + I : nt;
            he = pack_shots(ctx, ctx->u[1 - ctx->cur], st, 2 * j, s);
            if (he == hipSuccess) he = pack_shots(ctx, ctx->u[ctx->cur], st, 2 * j + 1, s);
            if (he == hipSuccess)
                he = forward_segment(ctx, p, sb, j == st.nck - 1 ? &st : nullptr, n0, n1, src, nsrc,
                                     rec, nrec, s);
        }
        if (he != hipSuccess) return hip_fail(ctx, he, "checkpointed forward");
        ctx->ck_store = store;
        ctx->ck_nt = nt;
        ctx->ck_interval = I;
        ctx->ck_last_acc = true;
        return FD_OK;
    });
}

int32_t fd_forward_checkpointed(fd_ctx* ctx, int32_t nt, const fd_points* src,
                                const fd_points* rec, int32_t interval, void* store,
                                uint64_t store_bytes, void* stream) {
    if (!ctx) return FD_ERR_INVALID_ARG;
    if (ctx->nshots > 1)
        return fail(ctx, FD_ERR_INVALID_ARG,
                    "a context of several shots uses fd_forward_checkpointed_shots");
    return fd_forward_checkpointed_shots(ctx, nt, src, nullptr, rec, nullptr, interval, store,
                                         store_bytes, stream);
}

int32_t fd_gradient_shots(fd_ctx* ctx, int32_t nt, const fd_points* src,
                          const int32_t* src_counts, const fd_points* adj,
                          const int32_t* adj_counts, int32_t interval, void* store,
                          uint64_t store_bytes, int32_t wrt, float* grad, float* wavelet_grad,
                          void* stream) {
    return guarded(ctx, [&]() -> int32_t {
        if (!ctx) return FD_ERR_INVALID_ARG;
        ctx->err.clear();
        if (ctx->tti || ctx->vti)
            return fail(ctx, FD_ERR_UNSUPPORTED, "gradients are built for acoustic only");
        const bool accumulate = (wrt & FD_GRAD_ACCUMULATE) != 0;
        wrt &= ~FD_GRAD_ACCUMULATE;
        if (wrt != FD_WRT_M && wrt != FD_WRT_VEL) return fail(ctx, FD_ERR_INVALID_ARG, "wrt");
        if (!grad) return fail(ctx, FD_ERR_INVALID_ARG, "grad is NULL");
        const int I = resolve_interval(ctx, nt, interval);
        if (!ctx->ck_store || store != ctx->ck_store || nt != ctx->ck_nt || I != ctx->ck_interval)
            return fail(ctx, FD_ERR_INVALID_ARG,
                        "store, nt and interval must match the last fd_forward_checkpointed");
        int32_t rc = check_points_arg(ctx, nt, src, "source");
        if (rc == FD_OK) rc = check_points_arg(ctx, nt, adj, "adjoint source");
        if (rc != FD_OK) return rc;
        const int nsrc = src ? src->n : 0, nadj = adj ? adj->n : 0;
        if ((int64_t)nsrc + nadj > ctx->max_points)
            return fail(ctx, FD_ERR_INVALID_ARG, "more points than max_points");
        rc = check_counts(ctx, src_counts, nsrc, "source");
        if (rc == FD_OK) rc = check_counts(ctx, adj_counts, nadj, "adjoint source");
        if (rc != FD_OK) return rc;
        rc = check_store(ctx, nt, I, store, store_bytes);
        if (rc != FD_OK) return rc;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const bool multi = ctx->nshots > 1;
        rc = sync_points(ctx, nsrc, src ? src->coords : nullptr, nadj, adj ? adj->coords : nullptr,
                         "source", "adjoint source", s, multi && nsrc ? src_counts : nullptr,
                         multi && nadj ? adj_counts : nullptr);
        if (rc != FD_OK) return rc;
        const Store st = plan_store(ctx, nt, I, static_cast<char*>(store));
        const int S = ctx->nshots;
        const int64_t vol = ctx->L.volume;
        hipError_t he = hipSuccess;
        for (int k = 0; k < 2 && he == hipSuccess; ++k) he = fd::launch_fill_zero(st.mu[k], vol * S, s);
        if (he == hipSuccess) he = fd::launch_fill_zero(st.gpart, vol * S, s);
        if (he == hipSuccess) he = fd::launch_fill_zero(st.gsum, st.dense * S, s);
        int pending = 0;  // adjoint steps accumulated in gpart since the last flush
        auto imaged = [&]() -> hipError_t {  // one more term in gpart: flush every kFlushSteps
            if (++pending < kFlushSteps) return hipSuccess;
            pending = 0;
            hipError_t e = hipSuccess;
            for (int i = 0; i < S && e == hipSuccess; ++i)
                e = fd::launch_flush_gradient(st.gpart + i * vol, st.gsum + i * st.dense, ctx->L, s);
            return e;
        };
        // the separate imaging kernel, shot by shot: gpart += mu a
        auto image = [&](const float* mu, const float* acc) -> hipError_t {
            hipError_t e = hipSuccess;
            for (int i = 0; i < S && e == hipSuccess; ++i)
                e = fd::launch_image(mu + i * vol, acc + i * vol, st.gpart + i * vol, ctx->L, s);
            return e;
        };
        const int sb = grad_sb(ctx);
        fd::AcousticStep p = acoustic_params(ctx, sb);
        // The imaging term mu^{k+1} a^{k+1} is fused into the adjoint step that
        // produces mu^k (its centre field is mu^{k+1}) where the tiled kernel has
        // that variant; the first step of a segment has no a^{k+1} in the
        // segment, so the segment's last term, mu^{n0+1} a^{n0+1}, is imaged by
        // the separate kernel before the next segment's recomputation overwrites
        // the slots.  The terms enter gpart in the same order and with the same
        // fmaf as the unfused loop, so both give the same bits.
        const bool fuse = ctx->fuse_image && ctx->g.ndim == 3 && ctx->variant == 0 &&
                          fd::img_built(ctx->tile_cfg, sb);
        int m = 0;  // st.mu[m] holds mu^{k+1}, st.mu[1-m] mu^{k+2}
        for (int j = st.nck - 1; j >= 0 && he == hipSuccess; --j) {
            const int n0 = j * I, n1 = n0 + I < nt ? n0 + I : nt;
            if (!(j == st.nck - 1 && ctx->ck_last_acc)) {
                he = unpack_shots(ctx, st, 2 * j, ctx->u[1 - ctx->cur], s);
                if (he == hipSuccess) he = unpack_shots(ctx, st, 2 * j + 1, ctx->u[ctx->cur], s);
                if (he == hipSuccess)
                    he = forward_segment(ctx, p, sb, &st, n0, n1, src, nsrc, nullptr, 0, s);
            }
            for (int k = n1; k > n0 && he == hipSuccess; --k) {
                const bool fused = fuse && k < n1;
                if (fused) {
                    p.img_a = st.slot(ctx, k - n0);  // a^{k+1}
                    p.img_g = st.gpart;
                }
                he = adjoint_step(ctx, p, sb, st.mu[m], st.mu[1 - m], k, nsrc, wavelet_grad, adj,
                                  nadj, s);
                p.img_a = nullptr;
                p.img_g = nullptr;
                if (he == hipSuccess && fused) he = imaged();  // mu^{k+1} a^{k+1}
                if (he == hipSuccess && !fuse) {
                    he = image(st.mu[1 - m], st.slot(ctx, k - 1 - n0));
                    if (he == hipSuccess) he = imaged();
                }
                m = 1 - m;
            }
            if (he == hipSuccess && fuse && n1 > n0) {  // mu^{n0+1} a^{n0+1}
                he = image(st.mu[m], st.slot(ctx, 0));
                if (he == hipSuccess) he = imaged();
            }
        }
        ctx->ck_last_acc = false;  // the segment slots now hold the first segment
        if (he == hipSuccess && pending)
            for (int i = 0; i < S && he == hipSuccess; ++i)
                he = fd::launch_flush_gradient(st.gpart + i * vol, st.gsum + i * st.dense, ctx->L, s);
        // shot by shot into grad: the bits of one fd_gradient per shot with
        // FD_GRAD_ACCUMULATE from the second shot on
        for (int i = 0; i < S && he == hipSuccess; ++i)
            he = fd::launch_finish_gradient(st.gsum + i * st.dense, ctx->A, grad, ctx->L, ctx->g.dt,
                                            wrt == FD_WRT_VEL, (accumulate || i > 0) ? 1 : 0, s);
        if (he != hipSuccess) return hip_fail(ctx, he, "gradient");
        return FD_OK;
    });
}

int32_t fd_gradient(fd_ctx* ctx, int32_t nt, const fd_points* src, const fd_points* adj,
                    int32_t interval, void* store, uint64_t store_bytes, int32_t wrt,
                    float* grad, float* wavelet_grad, void* stream) {
    if (!ctx) return FD_ERR_INVALID_ARG;
    if (ctx->nshots > 1)
        return fail(ctx, FD_ERR_INVALID_ARG, "a context of several shots uses fd_gradient_shots");
    return fd_gradient_shots(ctx, nt, src, nullptr, adj, nullptr, interval, store, store_bytes,
                             wrt, grad, wavelet_grad, stream);
}

int32_t fd_misfit(const float* d, const float* d_obs, int64_t n, float* res, double* J,
                  void* stream) {
    if (n < 0 || (n > 0 && (!d || !d_obs || !res || !J))) return FD_ERR_INVALID_ARG;
    if (n == 0) return FD_OK;
    const hipError_t e = fd::launch_misfit(d, d_obs, n, res, J, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}

int32_t fd_adjoint(fd_ctx* ctx, int32_t nt, const fd_points* adj, const fd_points* out,
                   void* stream) {
    return guarded(ctx, [&]() -> int32_t {
        if (!ctx) return FD_ERR_INVALID_ARG;
        ctx->err.clear();
        if (ctx->nshots > 1)
            return fail(ctx, FD_ERR_INVALID_ARG, "a context of several shots steps with fd_forward_shots");
        if (ctx->tti || ctx->vti)
            return fail(ctx, FD_ERR_UNSUPPORTED, "the adjoint is built for acoustic only");
        if (nt < 0) return fail(ctx, FD_ERR_INVALID_ARG, "nt < 0");
        int32_t rc = check_points_arg(ctx, nt, adj, "adjoint source");
        if (rc == FD_OK) rc = check_points_arg(ctx, nt, out, "source");
        if (rc != FD_OK) return rc;
        const int nadj = adj ? adj->n : 0, nsrc = out ? out->n : 0;
        if ((int64_t)nsrc + nadj > ctx->max_points)
            return fail(ctx, FD_ERR_INVALID_ARG, "more points than max_points");
        hipStream_t s = static_cast<hipStream_t>(stream);
        rc = sync_points(ctx, nsrc, out ? out->coords : nullptr, nadj, adj ? adj->coords : nullptr,
                         "source", "adjoint source", s);
        if (rc != FD_OK) return rc;
        hipError_t he = hipSuccess;
        if (ctx->flags_stale) {
            he = refresh_flags(ctx, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "damping flags");
            ctx->flags_stale = false;
        }
        for (int k = 0; k < 2 && he == hipSuccess; ++k) he = fd::launch_fill_zero(ctx->u[k], ctx->L.volume, s);
        fd::AcousticStep p = acoustic_params(ctx, 1);
        for (int k = nt; k >= 1 && he == hipSuccess; --k) {
            he = adjoint_step(ctx, p, 1, ctx->u[ctx->cur], ctx->u[1 - ctx->cur], k, nsrc,
                              out ? out->data : nullptr, adj, nadj, s);
            ctx->cur = 1 - ctx->cur;
        }
        if (he != hipSuccess) return hip_fail(ctx, he, "adjoint");
        return FD_OK;
    });
}

int32_t fd_forward_shots(fd_ctx* ctx, int32_t nt, const fd_points* src, const int32_t* src_counts,
                         const fd_points* rec, const int32_t* rec_counts, int32_t flags,
                         void* stream) {
    return guarded(ctx, [&]() -> int32_t {
        if (!ctx) return FD_ERR_INVALID_ARG;
        ctx->err.clear();
        if (ctx->tti || ctx->vti)
            return fail(ctx, FD_ERR_UNSUPPORTED, "several shots are built for acoustic only");
        if (nt < 0) return fail(ctx, FD_ERR_INVALID_ARG, "nt < 0");
        const bool keep = (flags & FD_KEEP_POINTS) != 0;
        int32_t rc = check_points_arg(ctx, nt, src, "source", keep);
        if (rc == FD_OK) rc = check_points_arg(ctx, nt, rec, "receiver", keep);
        if (rc != FD_OK) return rc;
        const int nsrc = src ? src->n : 0, nrec = rec ? rec->n : 0;
        if ((int64_t)nsrc + nrec > ctx->max_points)
            return fail(ctx, FD_ERR_INVALID_ARG, "more points than max_points");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int nd = ctx->g.ndim;
        if (keep) {
            // the shots of the points are those of the last upload
            rc = keep_points(ctx, nsrc, nrec);
        } else {
            rc = check_counts(ctx, src_counts, nsrc, "source");
            if (rc == FD_OK) rc = check_counts(ctx, rec_counts, nrec, "receiver");
            if (rc == FD_OK)
                rc = sync_points(ctx, nsrc, src ? src->coords : nullptr, nrec,
                                 rec ? rec->coords : nullptr, "source", "receiver", s,
                                 nsrc ? src_counts : nullptr, nrec ? rec_counts : nullptr);
        }
        if (rc != FD_OK) return rc;
        hipError_t he = hipSuccess;
        if (ctx->flags_stale) {
            he = refresh_flags(ctx, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "damping flags");
            ctx->flags_stale = false;
        }
        if (flags & FD_ZERO_STATE)
            for (int k = 0; k < 2 && he == hipSuccess; ++k)
                he = fd::launch_fill_zero(ctx->u[k], ctx->L.volume * ctx->nshots, s);
        if (he != hipSuccess) return hip_fail(ctx, he, "zero state");
        const float scale = (float)(1.0 / cell_volume(ctx));
        const float* sig = ctx->damping ? ctx->sig : nullptr;
        const int sb = ctx_sb(ctx);
        fd::AcousticStep p = acoustic_params(ctx, sb);
        for (int n = 0; n < nt; ++n) {
            float* un = ctx->u[1 - ctx->cur];
            const float* uc = ctx->u[ctx->cur];
            he = acoustic_stencil(ctx, p, uc, un, nullptr, sb, s);
            if (he == hipSuccess)
                he = forward_points(ctx, n, 0, un, nullptr, true, uc, src, nsrc, rec, nrec, sig,
                                    scale, s);
            if (he != hipSuccess) return hip_fail(ctx, he, "step");
            ctx->cur = 1 - ctx->cur;
        }
        he = forward_last_record(ctx, 0, nt, ctx->u[ctx->cur], rec, nsrc, nrec, s);
        if (he != hipSuccess) return hip_fail(ctx, he, "step");
        return FD_OK;
    });
}

static float* field_ptr(fd_ctx* ctx, int32_t shot, int32_t which) {
    if (shot < 0 || shot >= ctx->nshots) return nullptr;
    const int64_t o = (int64_t)shot * ctx->L.volume;
    switch (which) {
        case FD_FIELD_PREV: return ctx->u[1 - ctx->cur] + o;
        case FD_FIELD_CUR: return ctx->u[ctx->cur] + o;
        case FD_FIELD_R_PREV: return ctx->r[0] ? ctx->r[1 - ctx->cur] : nullptr;
        case FD_FIELD_R_CUR: return ctx->r[0] ? ctx->r[ctx->cur] : nullptr;
        default: return nullptr;
    }
}

int32_t fd_get_shot_field(fd_ctx* ctx, int32_t shot, int32_t which, float* dst, void* stream) {
    if (!ctx) return FD_ERR_INVALID_ARG;
    float* f = field_ptr(ctx, shot, which);
    if (!f || !dst) return fail(ctx, FD_ERR_INVALID_ARG, "bad shot, field selector or pointer");
    const hipError_t he = fd::launch_pack(f, dst, ctx->L, static_cast<hipStream_t>(stream));
    return he == hipSuccess ? FD_OK : hip_fail(ctx, he, "get_field");
}

int32_t fd_set_shot_field(fd_ctx* ctx, int32_t shot, int32_t which, const float* src,
                          void* stream) {
    if (!ctx) return FD_ERR_INVALID_ARG;
    float* f = field_ptr(ctx, shot, which);
    if (!f || !src) return fail(ctx, FD_ERR_INVALID_ARG, "bad shot, field selector or pointer");
    const hipError_t he = fd::launch_unpack(src, f, ctx->L, static_cast<hipStream_t>(stream));
    return he == hipSuccess ? FD_OK : hip_fail(ctx, he, "set_field");
}

int32_t fd_get_field(fd_ctx* ctx, int32_t which, float* dst, void* stream) {
    return fd_get_shot_field(ctx, 0, which, dst, stream);
}

int32_t fd_set_field(fd_ctx* ctx, int32_t which, const float* src, void* stream) {
    return fd_set_shot_field(ctx, 0, which, src, stream);
}

int32_t fd_destroy(fd_ctx* ctx) {
    delete ctx;
    return FD_OK;
}

// ---------------------------------------------------------------------------
// correction network
// ---------------------------------------------------------------------------

static bool cnn_shape_ok(const int64_t* shape) {
    if (!shape) return false;
    for (int a = 0; a < 3; ++a)
        if (shape[a] < 1 || shape[a] > 65535) return false;
    return shape[0] * shape[1] * shape[2] < ((int64_t)1 << 40);
}

static bool aligned16(const void* p) { return p && reinterpret_cast<uintptr_t>(p) % 16 == 0; }

int32_t fd_cnn_packed_elems(int32_t cin_pad, int64_t* elems) {
    if (!elems || (cin_pad != 8 && cin_pad != 16)) return FD_ERR_INVALID_ARG;
    *elems = fd::cnn_packed_elems(cin_pad);
    return FD_OK;
}

int32_t fd_cnn_pack(const float* layer, int32_t cin_pad, int32_t transpose, uint16_t* packed,
                    void* stream) {
    if (!layer || !aligned16(packed) || (cin_pad != 8 && cin_pad != 16)) return FD_ERR_INVALID_ARG;
    const hipError_t e = fd::launch_cnn_pack(layer, 16, 16, cin_pad, transpose ? 1 : 0, packed,
                                             static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}

int32_t fd_cnn_conv(const uint16_t* x, int32_t cin_pad, const int64_t* shape,
                    const uint16_t* packed, const float* bias, int32_t mode, const uint16_t* mask,
                    int32_t cout_store, uint16_t* y, float* yf, void* stream) {
    if (!cnn_shape_ok(shape) || !aligned16(x) || !aligned16(packed) ||
        (cin_pad != 8 && cin_pad != 16))
        return FD_ERR_INVALID_ARG;
    if (mode == FD_CNN_RELU && (!bias || !aligned16(y))) return FD_ERR_INVALID_ARG;
    if (mode == FD_CNN_LINEAR && (!bias || !yf || cout_store < 1 || cout_store > 16))
        return FD_ERR_INVALID_ARG;
    if (mode == FD_CNN_MASKED && (!mask || !aligned16(y))) return FD_ERR_INVALID_ARG;
    if (mode == FD_CNN_IDENTITY && (!bias || !aligned16(y))) return FD_ERR_INVALID_ARG;
    if (mode == FD_CNN_UNMASKED && !aligned16(y)) return FD_ERR_INVALID_ARG;
    if (mode < FD_CNN_RELU || mode > FD_CNN_UNMASKED) return FD_ERR_INVALID_ARG;
    const hipError_t e = fd::launch_cnn_conv(x, cin_pad, (int)shape[0], (int)shape[1],
                                             (int)shape[2], packed, bias, mode, mask, cout_store,
                                             y, yf, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}

int32_t fd_cnn_wgrad_scratch(const int64_t* shape, int64_t* floats) {
    if (!cnn_shape_ok(shape) || !floats) return FD_ERR_INVALID_ARG;
    *floats = (int64_t)fd::cnn_wgrad_slots((int)shape[0], (int)shape[1], (int)shape[2],
                                           fd::kCnnWgradZChunk) *
              FD_CNN_LAYER_FLOATS;
    return FD_OK;
}

int32_t fd_cnn_wgrad(const uint16_t* x, int32_t cx, const uint16_t* dz, int32_t cz,
                     const int64_t* shape, float* scratch, int64_t scratch_floats, float* grad,
                     void* stream) {
    int64_t need = 0;
    if (fd_cnn_wgrad_scratch(shape, &need) != FD_OK || !x || !dz || !scratch || !grad)
        return FD_ERR_INVALID_ARG;
    if (!((cx == 8 && cz == 16) || (cx == 16 && cz == 16) || (cx == 16 && cz == 8)))
        return FD_ERR_INVALID_ARG;
    if (scratch_floats < need) return FD_ERR_WORKSPACE;
    const hipError_t e = fd::launch_cnn_wgrad(x, cx, dz, cz, (int)shape[0], (int)shape[1],
                                              (int)shape[2], fd::kCnnWgradZChunk, scratch, grad,
                                              static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}

int32_t fd_cnn_loss_grad(const float* out, const float* target, const uint8_t* mask,
                         int64_t nvox, int32_t cout, int32_t cpad, float inv_n, uint16_t* dz,
                         float* loss, void* stream) {
    if (!out || !target || !mask || !dz || !loss || nvox < 1 || cout < 1 || cpad < cout ||
        cpad > 16)
        return FD_ERR_INVALID_ARG;
    const hipError_t e = fd::launch_cnn_loss_grad(out, target, mask, nvox, cout, cpad, inv_n, dz,
                                                  loss, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}

int32_t fd_cnn_adam(float* param, const float* grad, float* m, float* v, int64_t n, int32_t t,
                    float lr, float beta1, float beta2, float eps, void* stream) {
    if (!param || !grad || !m || !v || n < 1 || t < 1) return FD_ERR_INVALID_ARG;
    const hipError_t e = fd::launch_cnn_adam(param, grad, m, v, n, t, lr, beta1, beta2, eps,
                                             static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}

static int32_t cnn_ctx_ok(fd_ctx* ctx) {
    if (!ctx) return FD_ERR_INVALID_ARG;
    if (ctx->tti || ctx->vti || ctx->nshots != 1)
        return fail(ctx, FD_ERR_UNSUPPORTED, "the correction works on single-shot acoustic contexts");
    return FD_OK;
}

int32_t fd_cnn_features(fd_ctx* ctx, float vref, const uint8_t* mask, uint32_t* scale_bits,
                        uint16_t* x, void* stream) {
    int32_t rc = cnn_ctx_ok(ctx);
    if (rc != FD_OK) return rc;
    if (!scale_bits || !aligned16(x) || !(vref > 0.f))
        return fail(ctx, FD_ERR_INVALID_ARG, "features: bad pointer or vref");
    const hipError_t e = fd::launch_cnn_features(ctx->u[ctx->cur], ctx->u[1 - ctx->cur], ctx->A,
                                                 ctx->L, (float)(1.0 / (ctx->g.dt * vref)), mask,
                                                 scale_bits, x, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : hip_fail(ctx, e, "features");
}

int32_t fd_cnn_correct(fd_ctx* ctx, const float* d, const uint8_t* mask,
                       const uint32_t* scale_bits, void* stream) {
    int32_t rc = cnn_ctx_ok(ctx);
    if (rc != FD_OK) return rc;
    if (!d || !scale_bits) return fail(ctx, FD_ERR_INVALID_ARG, "correct: bad pointer");
    const hipError_t e = fd::launch_cnn_correct(ctx->u[ctx->cur], ctx->u[1 - ctx->cur], ctx->L, d,
                                                mask, scale_bits,
                                                static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : hip_fail(ctx, e, "correct");
}

int32_t fd_cnn_residual(fd_ctx* ctx, const float* ref_cur, const float* ref_prev,
                        const uint32_t* scale_bits, float* target, void* stream) {
    int32_t rc = cnn_ctx_ok(ctx);
    if (rc != FD_OK) return rc;
    if (!ref_cur || !ref_prev || !scale_bits || !target)
        return fail(ctx, FD_ERR_INVALID_ARG, "residual: bad pointer");
    const hipError_t e = fd::launch_cnn_residual(ref_cur, ref_prev, ctx->u[ctx->cur],
                                                 ctx->u[1 - ctx->cur], ctx->L, scale_bits, target,
                                                 static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : hip_fail(ctx, e, "residual");
}

int32_t fd_restrict(fd_ctx* ctx, int32_t which, int32_t stride, float* dst, void* stream) {
    if (!ctx) return FD_ERR_INVALID_ARG;
    float* f = field_ptr(ctx, 0, which);
    if (!f || !dst || stride < 1) return fail(ctx, FD_ERR_INVALID_ARG, "restrict: bad argument");
    const hipError_t e = fd::launch_restrict(f, ctx->L, stride, dst,
                                             static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : hip_fail(ctx, e, "restrict");
}

const char* fd_strerror(int32_t status) {
    switch (status) {
        case FD_OK: return "success";
        case FD_ERR_INVALID_ARG: return "invalid argument";
        case FD_ERR_UNSTABLE_DT: return "dt exceeds the CFL bound";
        case FD_ERR_UNSUPPORTED: return "unsupported space order or physics";
        case FD_ERR_WORKSPACE: return "workspace too small or misaligned";
        case FD_ERR_DEVICE: return "HIP runtime error";
        case FD_ERR_NONFINITE: return "non-finite or non-positive model values";
        case FD_ERR_HOST: return "host memory could not be obtained";
        default: return "unknown status";
    }
}

const char* fd_last_error(const fd_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"
