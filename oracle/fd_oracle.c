/*
 * fd_oracle.c -- plain, slow, FP64 CPU oracle for the explicit
 * finite-difference wave solver (Louboutin et al., "Performance prediction of
 * finite-difference solvers for different computer architectures").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or table with the GPU library; the two are independent statements of
 * the same mathematics.
 *
 * What it computes (all arithmetic in IEEE double, round-to-nearest, scalar
 * loops in a fixed order; build with -O2 -ffp-contract=off):
 *
 *   - central finite-difference weights of maximal order for the second and
 *     first derivative on a symmetric k-point stencil (section 4.1 "Stencil
 *     operators": k points per 1D derivative, order k-1, radius r = (k-1)/2);
 *   - the CFL bound of Eq. (stability), section 6, with a1 = 4 and a2 the sum
 *     of the absolute stencil weights of the discrete Laplacian;
 *   - Algorithm 1 (time stepping) for the acoustic equation of Appendix A,
 *     Eq. (Acou): m u_tt - lap(u) = q, zero initial state, with
 *       * the stencil sweep over every grid point, then
 *       * the source added after the sweep (Algorithm 1, "Add Source"),
 *       * a damping layer (the paper leaves boundary treatment out of the
 *         model, section 2): u_tt + eta u_t = v^2 (lap u + q),
 *       * receivers sampled from the freshly updated field;
 *   - the VTI pseudo-acoustic system, Eq. (vVTI), with the horizontal operator
 *     D_xx (2D) or D_xx + D_yy (3D);
 *   - the TTI pseudo-acoustic system, Eq. (TTI), with the rotated operators of
 *     Eq. (DiffOp) written out term by term (G_xbar_xbar, G_ybar_ybar,
 *     G_zbar_zbar), cross derivatives as products of two first-derivative
 *     stencils (their FLOP count in section 4.1 is that of such a product).
 *
 * Readings where the paper is silent (damping form, source scaling, sparse
 * interpolation, receiver field for TTI) are listed in the design notes; the
 * damping term is "parity unpinned" beyond agreement with this oracle.
 *
 * Layout: fields are C-order [nz][ny][nx] over the padded array (physical
 * domain plus nbl layer points on every side), x contiguous.  A 2D problem is
 * ny = 1 with no y derivative.  Points outside the array read as zero
 * (homogeneous Dirichlet ghosts).  Sparse-point coordinates are in metres from
 * the physical origin, ordered (x, y, z) in 3D and (x, z) in 2D.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_BAD 1

static int g_threads = 1;

/* Thread count for the sweep loops (timing only; results do not depend on
 * it because every point is computed independently). */
int or_set_threads(int n) {
    g_threads = n < 1 ? 1 : n;
#ifdef _OPENMP
    return g_threads;
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Finite-difference weights                                                */
/* ------------------------------------------------------------------------ */

/* (r!)^2 / ((r-j)! (r+j)!) as a product of j ratios. */
static double fact_ratio(int r, int j) {
    double v = 1.0;
    for (int i = 1; i <= j; ++i) v *= (double)(r - j + i) / (double)(r + i);
    return v;
}

/* Central second-derivative weights of maximal order 2r on unit spacing:
 *   w_j = 2 (-1)^(j+1) (r!)^2 / (j^2 (r-j)! (r+j)!),  j = 1..r,
 *   w_0 = -2 sum_j w_j.
 * (Fornberg's closed form.)  Writes w[0..r]. */
int or_weights_d2(int r, double* w) {
    if (r < 1 || !w) return OR_BAD;
    double s = 0.0;
    for (int j = 1; j <= r; ++j) {
        double sgn = (j % 2 == 1) ? 1.0 : -1.0;
        w[j] = 2.0 * sgn * fact_ratio(r, j) / ((double)j * (double)j);
        s += w[j];
    }
    w[0] = -2.0 * s;
    return OR_OK;
}

/* Central first-derivative weights of maximal order 2r on unit spacing:
 *   w_j = (-1)^(j+1) (r!)^2 / (j (r-j)! (r+j)!),  w_{-j} = -w_j,  w_0 = 0.
 * Writes w[0..r] (w[0] = 0). */
int or_weights_d1(int r, double* w) {
    if (r < 1 || !w) return OR_BAD;
    w[0] = 0.0;
    for (int j = 1; j <= r; ++j) {
        double sgn = (j % 2 == 1) ? 1.0 : -1.0;
        w[j] = sgn * fact_ratio(r, j) / (double)j;
    }
    return OR_OK;
}

/* Eq. (stability), CFL condition:  v_max dt / h <= sqrt(a1 / a2), with
 * a1 = 4 (second-order time difference 1, -2, 1) and a2 the sum of the
 * absolute weights of the discrete Laplacian.  For unequal spacings the
 * Laplacian weights carry 1/h_a^2, so the bound reads
 *   dt <= sqrt(a1 / sum_a(S / h_a^2)) / v_max,  S = |w_0| + 2 sum_j |w_j|.
 * Returns the largest stable dt (seconds). */
double or_cfl_dt(int ndim, int so, const double* h, double vmax) {
    int r = so / 2;
    double w[64];
    if (r < 1 || r > 63 || vmax <= 0.0) return -1.0;
    or_weights_d2(r, w);
    double S = fabs(w[0]);
    for (int j = 1; j <= r; ++j) S += 2.0 * fabs(w[j]);
    double denom = S / (h[0] * h[0]) + S / (h[2] * h[2]);
    if (ndim == 3) denom += S / (h[1] * h[1]);
    return sqrt(4.0 / denom) / vmax;
}

/* Sum of absolute Laplacian weights a2 of Eq. (stability) on unit spacing. */
double or_a2(int ndim, int so) {
    int r = so / 2;
    double w[64];
    if (r < 1 || r > 63) return -1.0;
    or_weights_d2(r, w);
    double S = fabs(w[0]);
    for (int j = 1; j <= r; ++j) S += 2.0 * fabs(w[j]);
    return ndim * S;
}

/* ------------------------------------------------------------------------ */
/* Field access                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    long nx, ny, nz;
} dims_t;

/* A field stored as float (inputs as the user supplies them) or double
 * (the oracle's own evolving state). */
typedef struct {
    const double* d;
    const float* f;
} fld_t;

static inline double fget(fld_t a, long i) { return a.d ? a.d[i] : (double)a.f[i]; }

/* Value at (ix, iy, iz) with zero outside the array. */
static inline double at(fld_t a, dims_t n, long ix, long iy, long iz) {
    if (ix < 0 || ix >= n.nx || iy < 0 || iy >= n.ny || iz < 0 || iz >= n.nz) return 0.0;
    return fget(a, (iz * n.ny + iy) * n.nx + ix);
}

/* ------------------------------------------------------------------------ */
/* Sparse points: multilinear interpolation weights                         */
/* ------------------------------------------------------------------------ */

/* For a coordinate c (metres from the physical origin) along an axis with
 * spacing h, padded length n and layer nbl: continuous padded index
 * g = c/h + nbl, cell i = floor(g) clamped to [0, n-2], fraction f = g - i.
 * Returns 0 when the point lies outside [0, n-1]. */
static int axis_cell(double c, double h, long n, int nbl, long* i, double* f) {
    double g = c / h + (double)nbl;
    if (!(g >= 0.0) || g > (double)(n - 1)) return 0;
    if (n == 1) { *i = 0; *f = 0.0; return 1; }
    long k = (long)floor(g);
    if (k > n - 2) k = n - 2;
    if (k < 0) k = 0;
    *i = k;
    *f = g - (double)k;
    return 1;
}

/* Corner indices and weights of one point; returns the number of corners
 * (4 in 2D, 8 in 3D) or 0 if the point is outside the array. */
static int corners(int ndim, dims_t n, int nbl, const double* h, const double* c,
                   long* idx, double* w) {
    long ix, iy = 0, iz;
    double fx, fy = 0.0, fz;
    if (ndim == 2) {
        if (!axis_cell(c[0], h[0], n.nx, nbl, &ix, &fx)) return 0;
        if (!axis_cell(c[1], h[2], n.nz, nbl, &iz, &fz)) return 0;
        int m = 0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dx = 0; dx < 2; ++dx) {
                idx[m] = (iz + dz) * n.nx + (ix + dx);
                w[m] = (dx ? fx : 1.0 - fx) * (dz ? fz : 1.0 - fz);
                ++m;
            }
        return 4;
    }
    if (!axis_cell(c[0], h[0], n.nx, nbl, &ix, &fx)) return 0;
    if (!axis_cell(c[1], h[1], n.ny, nbl, &iy, &fy)) return 0;
    if (!axis_cell(c[2], h[2], n.nz, nbl, &iz, &fz)) return 0;
    int m = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                idx[m] = ((iz + dz) * n.ny + (iy + dy)) * n.nx + (ix + dx);
                w[m] = (dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy) * (dz ? fz : 1.0 - fz);
                ++m;
            }
    return 8;
}

/* Exposed for tests: corner indices (flat, padded array) and weights. */
int or_point_corners(int ndim, const long* nxyz, int nbl, const double* h, const double* c,
                     long* idx, double* w) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    return corners(ndim, n, nbl, h, c, idx, w);
}

/* ------------------------------------------------------------------------ */
/* Acoustic equation                                                        */
/* ------------------------------------------------------------------------ */

/* Discrete Laplacian of u at one point: per axis the centre weight plus the
 * symmetric neighbour pairs (u[+j] + u[-j]) weighted by w_j, j = 1..r, scaled
 * by 1/h_a^2; axes summed in the order x, y, z. */
static double laplacian_at(fld_t u, dims_t n, int ndim, const double* w, int r,
                           const double* h, long ix, long iy, long iz) {
    double c = at(u, n, ix, iy, iz);
    double sx = w[0] * c, sy = w[0] * c, sz = w[0] * c;
    for (int j = 1; j <= r; ++j) sx += w[j] * (at(u, n, ix + j, iy, iz) + at(u, n, ix - j, iy, iz));
    for (int j = 1; j <= r; ++j) sz += w[j] * (at(u, n, ix, iy, iz + j) + at(u, n, ix, iy, iz - j));
    double L = sx / (h[0] * h[0]);
    if (ndim == 3) {
        for (int j = 1; j <= r; ++j) sy += w[j] * (at(u, n, ix, iy + j, iz) + at(u, n, ix, iy - j, iz));
        L += sy / (h[1] * h[1]);
    }
    L += sz / (h[2] * h[2]);
    return L;
}

/* One damped leapfrog update at one point:
 *   u^{n+1} = [2 u^n - (1 - s) u^{n-1} + A L u^n] / (1 + s),
 * A = dt^2 v^2 (= dt^2/m), s = eta dt / 2. */
static double acoustic_point(fld_t up, fld_t uc, const float* vel, const float* eta,
                             dims_t n, int ndim, const double* w, int r, const double* h,
                             double dt, long ix, long iy, long iz) {
    long i = (iz * n.ny + iy) * n.nx + ix;
    double v = (double)vel[i];
    double A = dt * dt * v * v;
    double s = eta ? 0.5 * dt * (double)eta[i] : 0.0;
    double L = laplacian_at(uc, n, ndim, w, r, h, ix, iy, iz);
    return (2.0 * fget(uc, i) - (1.0 - s) * fget(up, i) + A * L) / (1.0 + s);
}

static double hprod(int ndim, const double* h) {
    return ndim == 3 ? h[0] * h[1] * h[2] : h[0] * h[2];
}

/* Source injection after the sweep (Algorithm 1, "Add Source"): the point
 * source q_s of Eq. (Acou) enters the discrete equation as q_s / prod(h) at
 * the grid, scaled like the stencil term by A/(1+s) and spread over the
 * multilinear corners. */
static void inject(double* un, const float* vel, const float* eta, dims_t n, int ndim, int nbl,
                   const double* h, double dt, int nsrc, const double* xyz, const float* q) {
    double hp = hprod(ndim, h);
    for (int s = 0; s < nsrc; ++s) {
        long idx[8];
        double w[8];
        int m = corners(ndim, n, nbl, h, xyz + (long)s * ndim, idx, w);
        for (int c = 0; c < m; ++c) {
            double v = (double)vel[idx[c]];
            double A = dt * dt * v * v;
            double sg = eta ? 0.5 * dt * (double)eta[idx[c]] : 0.0;
            un[idx[c]] += w[c] * A * (double)q[s] / (hp * (1.0 + sg));
        }
    }
}

/* Receiver sample: multilinear interpolation of the updated field. */
static void record(const double* un, dims_t n, int ndim, int nbl, const double* h,
                   int nrec, const double* xyz, double* d) {
    for (int j = 0; j < nrec; ++j) {
        long idx[8];
        double w[8];
        int m = corners(ndim, n, nbl, h, xyz + (long)j * ndim, idx, w);
        double acc = 0.0;
        for (int c = 0; c < m; ++c) acc += w[c] * un[idx[c]];
        d[j] = acc;
    }
}

static int check_points(int ndim, dims_t n, int nbl, const double* h, int np, const double* xyz) {
    for (int j = 0; j < np; ++j) {
        long idx[8];
        double w[8];
        if (!corners(ndim, n, nbl, h, xyz + (long)j * ndim, idx, w)) return 0;
    }
    return 1;
}

/* Acoustic forward run of nt steps (Algorithm 1 with damping, source and
 * receivers).  On entry (u_prev, u_cur) = (u^{n-1}, u^n); on return they hold
 * the last two levels.  wavelet is [nt][nsrc]; traces is [nt][nrec] and
 * sample t is taken from u^{n+1} of step t after injection. */
int or_acoustic_forward(int ndim, const long* nxyz, int nbl, const double* h, double dt, int so,
                        const float* vel, const float* eta,
                        int nsrc, const double* src_xyz, const float* wavelet,
                        int nrec, const double* rec_xyz, double* traces,
                        int nt, double* u_prev, double* u_cur) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w[64];
    if ((ndim != 2 && ndim != 3) || so < 2 || so % 2 || r > 63 || nt < 0) return OR_BAD;
    if (ndim == 2 && n.ny != 1) return OR_BAD;
    if (!check_points(ndim, n, nbl, h, nsrc, src_xyz)) return OR_BAD;
    if (!check_points(ndim, n, nbl, h, nrec, rec_xyz)) return OR_BAD;
    or_weights_d2(r, w);
    long N = n.nx * n.ny * n.nz;
    double* un = (double*)malloc(sizeof(double) * (size_t)N);
    if (!un) return OR_BAD;
    for (int t = 0; t < nt; ++t) {
        fld_t up = {u_prev, NULL}, uc = {u_cur, NULL};
#pragma omp parallel for schedule(static) num_threads(g_threads)
        for (long iz = 0; iz < n.nz; ++iz)
            for (long iy = 0; iy < n.ny; ++iy)
                for (long ix = 0; ix < n.nx; ++ix)
                    un[(iz * n.ny + iy) * n.nx + ix] =
                        acoustic_point(up, uc, vel, eta, n, ndim, w, r, h, dt, ix, iy, iz);
        inject(un, vel, eta, n, ndim, nbl, h, dt, nsrc, src_xyz, wavelet + (long)t * nsrc);
        if (nrec > 0) record(un, n, ndim, nbl, h, nrec, rec_xyz, traces + (long)t * nrec);
        /* rotate levels: prev <- cur, cur <- next */
        memcpy(u_prev, u_cur, sizeof(double) * (size_t)N);
        memcpy(u_cur, un, sizeof(double) * (size_t)N);
    }
    free(un);
    return OR_OK;
}

/* One acoustic step evaluated only at the listed points (flat indices into
 * the padded array), from an FP32 state.  No source term.  Used to check a
 * single step at full problem size point by point. */
int or_acoustic_step_points(int ndim, const long* nxyz, const double* h, double dt, int so,
                            const float* vel, const float* eta,
                            const float* u_prev, const float* u_cur,
                            long npts, const long* pts, double* out) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w[64];
    if ((ndim != 2 && ndim != 3) || so < 2 || so % 2 || r > 63) return OR_BAD;
    or_weights_d2(r, w);
    fld_t up = {NULL, u_prev}, uc = {NULL, u_cur};
    long N = n.nx * n.ny * n.nz;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long k = 0; k < npts; ++k) {
        long i = pts[k];
        if (i < 0 || i >= N) { out[k] = NAN; continue; }
        long ix = i % n.nx, iy = (i / n.nx) % n.ny, iz = i / (n.nx * n.ny);
        out[k] = acoustic_point(up, uc, vel, eta, n, ndim, w, r, h, dt, ix, iy, iz);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* TTI pseudo-acoustic system (3D)                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double dxx, dyy, dzz, dxy, dyz, dxz;
} derivs_t;

/* The six second derivatives of f at one point.  Pure second derivatives use
 * the second-derivative weights w2; the mixed ones are the product of two
 * first-derivative stencils, sum_a sum_b w1_a w1_b f(.+a, .+b). */
static derivs_t derivs_at(fld_t f, dims_t n, const double* w2, const double* w1, int r,
                          const double* h, long ix, long iy, long iz) {
    derivs_t d;
    double c = at(f, n, ix, iy, iz);
    double sx = w2[0] * c, sy = w2[0] * c, sz = w2[0] * c;
    for (int j = 1; j <= r; ++j) {
        sx += w2[j] * (at(f, n, ix + j, iy, iz) + at(f, n, ix - j, iy, iz));
        sy += w2[j] * (at(f, n, ix, iy + j, iz) + at(f, n, ix, iy - j, iz));
        sz += w2[j] * (at(f, n, ix, iy, iz + j) + at(f, n, ix, iy, iz - j));
    }
    d.dxx = sx / (h[0] * h[0]);
    d.dyy = sy / (h[1] * h[1]);
    d.dzz = sz / (h[2] * h[2]);
    double sxy = 0.0, syz = 0.0, sxz = 0.0;
    for (int a = -r; a <= r; ++a) {
        if (a == 0) continue;
        double wa = a > 0 ? w1[a] : -w1[-a];
        for (int b = -r; b <= r; ++b) {
            if (b == 0) continue;
            double wb = b > 0 ? w1[b] : -w1[-b];
            sxy += wa * wb * at(f, n, ix + a, iy + b, iz);
            syz += wa * wb * at(f, n, ix, iy + a, iz + b);
            sxz += wa * wb * at(f, n, ix + a, iy, iz + b);
        }
    }
    d.dxy = sxy / (h[0] * h[1]);
    d.dyz = syz / (h[1] * h[2]);
    d.dxz = sxz / (h[0] * h[2]);
    return d;
}

/* Rotated operators of Eq. (DiffOp), theta = tilt, phi = azimuth.  The
 * d^2/dxdy coefficient of G_ybar_ybar is taken as -sin(2 phi) (the printed
 * square is read as a typesetting slip: it is the value that makes the
 * operator (ybar . grad)^2 for ybar = (-sin phi, cos phi, 0) and makes the
 * three operators sum to the Laplacian). */
typedef struct {
    double gxx, gyy, gzz;
} rot_t;

static rot_t rotated_ops(derivs_t d, double theta, double phi) {
    double ct = cos(theta), st = sin(theta), cp = cos(phi), sp = sin(phi);
    double s2t = sin(2.0 * theta), s2p = sin(2.0 * phi);
    rot_t g;
    g.gxx = cp * cp * ct * ct * d.dxx + sp * sp * ct * ct * d.dyy + st * st * d.dzz
          + s2p * ct * ct * d.dxy - sp * s2t * d.dyz - cp * s2t * d.dxz;
    g.gyy = sp * sp * d.dxx + cp * cp * d.dyy - s2p * d.dxy;
    g.gzz = cp * cp * st * st * d.dxx + sp * sp * st * st * d.dyy + ct * ct * d.dzz
          + s2p * st * st * d.dxy + sp * s2t * d.dyz + cp * s2t * d.dxz;
    return g;
}

/* Exposed for tests: G_xbar_xbar f, G_ybar_ybar f, G_zbar_zbar f and the
 * plain Laplacian of f at every point (3D).  theta/phi are per-point FP32. */
int or_tti_operators(const long* nxyz, const double* h, int so, const double* f,
                     const float* theta, const float* phi,
                     double* gxx, double* gyy, double* gzz, double* lap) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w2[64], w1[64];
    if (so < 2 || so % 2 || r > 63) return OR_BAD;
    or_weights_d2(r, w2);
    or_weights_d1(r, w1);
    fld_t ff = {f, NULL};
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long iz = 0; iz < n.nz; ++iz)
        for (long iy = 0; iy < n.ny; ++iy)
            for (long ix = 0; ix < n.nx; ++ix) {
                long i = (iz * n.ny + iy) * n.nx + ix;
                derivs_t d = derivs_at(ff, n, w2, w1, r, h, ix, iy, iz);
                rot_t g = rotated_ops(d, (double)theta[i], (double)phi[i]);
                gxx[i] = g.gxx;
                gyy[i] = g.gyy;
                gzz[i] = g.gzz;
                lap[i] = d.dxx + d.dyy + d.dzz;
            }
    return OR_OK;
}

/* One TTI update at one point, Eq. (TTI) with m = 1/v^2 and damping:
 *   p+ = [2p - (1-s)p- + A((1+2eps)(Gxx+Gyy)p + sqrt(1+2delta) Gzz r)]/(1+s)
 *   r+ = [2r - (1-s)r- + A(sqrt(1+2delta)(Gxx+Gyy)p + Gzz r)]/(1+s)        */
static void tti_point(fld_t pp, fld_t pc, fld_t rp, fld_t rc, const float* vel, const float* eta,
                      const float* eps, const float* delta, const float* theta, const float* phi,
                      dims_t n, const double* w2, const double* w1, int r, const double* h,
                      double dt, long ix, long iy, long iz, double* pn, double* rn) {
    long i = (iz * n.ny + iy) * n.nx + ix;
    double v = (double)vel[i];
    double A = dt * dt * v * v;
    double s = eta ? 0.5 * dt * (double)eta[i] : 0.0;
    double th = (double)theta[i], ph = (double)phi[i];
    derivs_t dp = derivs_at(pc, n, w2, w1, r, h, ix, iy, iz);
    derivs_t dr = derivs_at(rc, n, w2, w1, r, h, ix, iy, iz);
    rot_t gp = rotated_ops(dp, th, ph);
    rot_t gr = rotated_ops(dr, th, ph);
    double e2 = 1.0 + 2.0 * (double)eps[i];
    double sd = sqrt(1.0 + 2.0 * (double)delta[i]);
    double hp = gp.gxx + gp.gyy;
    *pn = (2.0 * fget(pc, i) - (1.0 - s) * fget(pp, i) + A * (e2 * hp + sd * gr.gzz)) / (1.0 + s);
    *rn = (2.0 * fget(rc, i) - (1.0 - s) * fget(rp, i) + A * (sd * hp + gr.gzz)) / (1.0 + s);
}

/* TTI forward run (3D only).  The source enters both p and r (the right-hand
 * side q of both equations of Eq. (TTI)); receivers sample p. */
int or_tti_forward(const long* nxyz, int nbl, const double* h, double dt, int so,
                   const float* vel, const float* eta, const float* eps, const float* delta,
                   const float* theta, const float* phi,
                   int nsrc, const double* src_xyz, const float* wavelet,
                   int nrec, const double* rec_xyz, double* traces,
                   int nt, double* p_prev, double* p_cur, double* r_prev, double* r_cur) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w2[64], w1[64];
    if (so < 2 || so % 2 || r > 63 || nt < 0) return OR_BAD;
    if (!check_points(3, n, nbl, h, nsrc, src_xyz)) return OR_BAD;
    if (!check_points(3, n, nbl, h, nrec, rec_xyz)) return OR_BAD;
    or_weights_d2(r, w2);
    or_weights_d1(r, w1);
    long N = n.nx * n.ny * n.nz;
    double* pn = (double*)malloc(sizeof(double) * (size_t)N);
    double* rn = (double*)malloc(sizeof(double) * (size_t)N);
    if (!pn || !rn) { free(pn); free(rn); return OR_BAD; }
    for (int t = 0; t < nt; ++t) {
        fld_t pp = {p_prev, NULL}, pc = {p_cur, NULL}, rp = {r_prev, NULL}, rc = {r_cur, NULL};
#pragma omp parallel for schedule(static) num_threads(g_threads)
        for (long iz = 0; iz < n.nz; ++iz)
            for (long iy = 0; iy < n.ny; ++iy)
                for (long ix = 0; ix < n.nx; ++ix) {
                    long i = (iz * n.ny + iy) * n.nx + ix;
                    tti_point(pp, pc, rp, rc, vel, eta, eps, delta, theta, phi, n, w2, w1, r, h,
                              dt, ix, iy, iz, &pn[i], &rn[i]);
                }
        const float* q = wavelet + (long)t * nsrc;
        inject(pn, vel, eta, n, 3, nbl, h, dt, nsrc, src_xyz, q);
        inject(rn, vel, eta, n, 3, nbl, h, dt, nsrc, src_xyz, q);
        if (nrec > 0) record(pn, n, 3, nbl, h, nrec, rec_xyz, traces + (long)t * nrec);
        memcpy(p_prev, p_cur, sizeof(double) * (size_t)N);
        memcpy(p_cur, pn, sizeof(double) * (size_t)N);
        memcpy(r_prev, r_cur, sizeof(double) * (size_t)N);
        memcpy(r_cur, rn, sizeof(double) * (size_t)N);
    }
    free(pn);
    free(rn);
    return OR_OK;
}

/* One TTI step at the listed points from an FP32 state (no source).
 * out_p / out_r receive p^{n+1} and r^{n+1} at those points. */
int or_tti_step_points(const long* nxyz, const double* h, double dt, int so,
                       const float* vel, const float* eta, const float* eps, const float* delta,
                       const float* theta, const float* phi,
                       const float* p_prev, const float* p_cur, const float* r_prev,
                       const float* r_cur, long npts, const long* pts, double* out_p,
                       double* out_r) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w2[64], w1[64];
    if (so < 2 || so % 2 || r > 63) return OR_BAD;
    or_weights_d2(r, w2);
    or_weights_d1(r, w1);
    fld_t pp = {NULL, p_prev}, pc = {NULL, p_cur}, rp = {NULL, r_prev}, rc = {NULL, r_cur};
    long N = n.nx * n.ny * n.nz;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long k = 0; k < npts; ++k) {
        long i = pts[k];
        if (i < 0 || i >= N) { out_p[k] = NAN; out_r[k] = NAN; continue; }
        long ix = i % n.nx, iy = (i / n.nx) % n.ny, iz = i / (n.nx * n.ny);
        tti_point(pp, pc, rp, rc, vel, eta, eps, delta, theta, phi, n, w2, w1, r, h, dt, ix, iy,
                  iz, &out_p[k], &out_r[k]);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* VTI pseudo-acoustic system, Eq. (vVTI)                                    */
/* ------------------------------------------------------------------------ */

/* Second derivative of f along one axis (0 = x, 1 = y, 2 = z) at a point:
 * (w_0 f + sum_j w_j (f[+j] + f[-j])) / h_axis^2. */
static double d2_axis(fld_t f, dims_t n, const double* w, int r, const double* h, long ix,
                      long iy, long iz, int axis) {
    long ex = axis == 0, ey = axis == 1, ez = axis == 2;
    double acc = w[0] * at(f, n, ix, iy, iz);
    for (int j = 1; j <= r; ++j)
        acc += w[j] * (at(f, n, ix + j * ex, iy + j * ey, iz + j * ez) +
                       at(f, n, ix - j * ex, iy - j * ey, iz - j * ez));
    return acc / (h[axis] * h[axis]);
}

/* One VTI update at one point, Eq. (vVTI) with m = 1/v^2 and damping, the
 * horizontal operator D_xx in 2D and D_xx + D_yy in 3D:
 *   p+ = [2p - (1-s)p- + A((1+2eps) Dh p + sqrt(1+2delta) D_zz r)]/(1+s)
 *   r+ = [2r - (1-s)r- + A(sqrt(1+2delta) Dh p + D_zz r)]/(1+s)            */
static void vti_point(fld_t pp, fld_t pc, fld_t rp, fld_t rc, const float* vel, const float* eta,
                      const float* eps, const float* delta, dims_t n, int ndim, const double* w,
                      int r, const double* h, double dt, long ix, long iy, long iz, double* pn,
                      double* rn) {
    long i = (iz * n.ny + iy) * n.nx + ix;
    double v = (double)vel[i];
    double A = dt * dt * v * v;
    double s = eta ? 0.5 * dt * (double)eta[i] : 0.0;
    double dh = d2_axis(pc, n, w, r, h, ix, iy, iz, 0);
    if (ndim == 3) dh += d2_axis(pc, n, w, r, h, ix, iy, iz, 1);
    double dzz = d2_axis(rc, n, w, r, h, ix, iy, iz, 2);
    double e2 = 1.0 + 2.0 * (double)eps[i];
    double sd = sqrt(1.0 + 2.0 * (double)delta[i]);
    *pn = (2.0 * fget(pc, i) - (1.0 - s) * fget(pp, i) + A * (e2 * dh + sd * dzz)) / (1.0 + s);
    *rn = (2.0 * fget(rc, i) - (1.0 - s) * fget(rp, i) + A * (sd * dh + dzz)) / (1.0 + s);
}

/* VTI forward run (2D or 3D; 2D is ny = 1).  The source enters p and r;
 * receivers sample p. */
int or_vti_forward(int ndim, const long* nxyz, int nbl, const double* h, double dt, int so,
                   const float* vel, const float* eta, const float* eps, const float* delta,
                   int nsrc, const double* src_xyz, const float* wavelet,
                   int nrec, const double* rec_xyz, double* traces,
                   int nt, double* p_prev, double* p_cur, double* r_prev, double* r_cur) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w[64];
    if ((ndim != 2 && ndim != 3) || so < 2 || so % 2 || r > 63 || nt < 0) return OR_BAD;
    if (ndim == 2 && n.ny != 1) return OR_BAD;
    if (!check_points(ndim, n, nbl, h, nsrc, src_xyz)) return OR_BAD;
    if (!check_points(ndim, n, nbl, h, nrec, rec_xyz)) return OR_BAD;
    or_weights_d2(r, w);
    long N = n.nx * n.ny * n.nz;
    double* pn = (double*)malloc(sizeof(double) * (size_t)N);
    double* rn = (double*)malloc(sizeof(double) * (size_t)N);
    if (!pn || !rn) { free(pn); free(rn); return OR_BAD; }
    for (int t = 0; t < nt; ++t) {
        fld_t pp = {p_prev, NULL}, pc = {p_cur, NULL}, rp = {r_prev, NULL}, rc = {r_cur, NULL};
#pragma omp parallel for schedule(static) num_threads(g_threads)
        for (long iz = 0; iz < n.nz; ++iz)
            for (long iy = 0; iy < n.ny; ++iy)
                for (long ix = 0; ix < n.nx; ++ix) {
                    long i = (iz * n.ny + iy) * n.nx + ix;
                    vti_point(pp, pc, rp, rc, vel, eta, eps, delta, n, ndim, w, r, h, dt, ix, iy,
                              iz, &pn[i], &rn[i]);
                }
        const float* q = wavelet + (long)t * nsrc;
        inject(pn, vel, eta, n, ndim, nbl, h, dt, nsrc, src_xyz, q);
        inject(rn, vel, eta, n, ndim, nbl, h, dt, nsrc, src_xyz, q);
        if (nrec > 0) record(pn, n, ndim, nbl, h, nrec, rec_xyz, traces + (long)t * nrec);
        memcpy(p_prev, p_cur, sizeof(double) * (size_t)N);
        memcpy(p_cur, pn, sizeof(double) * (size_t)N);
        memcpy(r_prev, r_cur, sizeof(double) * (size_t)N);
        memcpy(r_cur, rn, sizeof(double) * (size_t)N);
    }
    free(pn);
    free(rn);
    return OR_OK;
}

/* One VTI step at the listed points from an FP32 state (no source). */
int or_vti_step_points(int ndim, const long* nxyz, const double* h, double dt, int so,
                       const float* vel, const float* eta, const float* eps, const float* delta,
                       const float* p_prev, const float* p_cur, const float* r_prev,
                       const float* r_cur, long npts, const long* pts, double* out_p,
                       double* out_r) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w[64];
    if ((ndim != 2 && ndim != 3) || so < 2 || so % 2 || r > 63) return OR_BAD;
    or_weights_d2(r, w);
    fld_t pp = {NULL, p_prev}, pc = {NULL, p_cur}, rp = {NULL, r_prev}, rc = {NULL, r_cur};
    long N = n.nx * n.ny * n.nz;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long k = 0; k < npts; ++k) {
        long i = pts[k];
        if (i < 0 || i >= N) { out_p[k] = NAN; out_r[k] = NAN; continue; }
        long ix = i % n.nx, iy = (i / n.nx) % n.ny, iz = i / (n.nx * n.ny);
        vti_point(pp, pc, rp, rc, vel, eta, eps, delta, n, ndim, w, r, h, dt, ix, iy, iz,
                  &out_p[k], &out_r[k]);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint and gradient of the acoustic forward map                         */
/* ------------------------------------------------------------------------ */
/*
 * The forward run is the linear recurrence, for n = 0 .. nt-1,
 *   F^{n+1} := D u^{n+1} - 2 u^n + E u^{n-1} - B (L u^n + S^T q^n / prod(h)) = 0,
 * D = diag(1 + s), E = diag(1 - s), B = diag(dt^2 v^2), with traces
 * d^n = R u^{n+1} (S, R the multilinear spreading of sources / receivers).
 * Its transpose in terms of the multipliers lambda^{n+1} of F^{n+1}:
 *   D lambda^k = 2 lambda^{k+1} + L(B lambda^{k+1}) - E lambda^{k+2} + R^T d^{k-1},
 * for k = nt .. 1 with lambda^{nt+1} = lambda^{nt+2} = 0 (L is symmetric),
 * and the wavelet-side output q'^n = S B lambda^{n+1} / prod(h).
 */

/* One level of the transposed recurrence:
 *   lambda^k = [2 lambda^{k+1} + L(B lambda^{k+1}) - E lambda^{k+2} + R^T dk] / (1 + s),
 * with L applied to the product B lambda^{k+1} (the transpose of B L is L B).
 * bl is scratch of N doubles; dk is the receiver data of index k-1 (nrec). */
static void adjoint_level(double* l0, const double* l1, const double* l2, double* bl,
                          dims_t n, int ndim, int nbl, const double* w, int r, const double* h,
                          double dt, const float* vel, const float* eta,
                          int nrec, const double* rec_xyz, const double* dk) {
    long N = n.nx * n.ny * n.nz;
    for (long i = 0; i < N; ++i) {
        double v = (double)vel[i];
        bl[i] = dt * dt * v * v * l1[i];
    }
    fld_t fb = {bl, NULL};
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long iz = 0; iz < n.nz; ++iz)
        for (long iy = 0; iy < n.ny; ++iy)
            for (long ix = 0; ix < n.nx; ++ix) {
                long i = (iz * n.ny + iy) * n.nx + ix;
                double s = eta ? 0.5 * dt * (double)eta[i] : 0.0;
                l0[i] = 2.0 * l1[i] + laplacian_at(fb, n, ndim, w, r, h, ix, iy, iz) -
                        (1.0 - s) * l2[i];
            }
    for (int j = 0; j < nrec; ++j) {
        long idx[8];
        double wc[8];
        int m = corners(ndim, n, nbl, h, rec_xyz + (long)j * ndim, idx, wc);
        for (int c = 0; c < m; ++c) l0[idx[c]] += wc[c] * dk[j];
    }
    for (long i = 0; i < N; ++i) {
        double s = eta ? 0.5 * dt * (double)eta[i] : 0.0;
        l0[i] /= (1.0 + s);
    }
}

/* F^T d: returns q'[nt][nsrc] for receiver data d[nt][nrec] (FP64), with
 * q'^{k-1} = S B lambda^k / prod(h). */
int or_acoustic_adjoint(int ndim, const long* nxyz, int nbl, const double* h, double dt, int so,
                        const float* vel, const float* eta,
                        int nsrc, const double* src_xyz, double* qout,
                        int nrec, const double* rec_xyz, const double* d, int nt) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w[64];
    if ((ndim != 2 && ndim != 3) || so < 2 || so % 2 || r > 63 || nt < 0) return OR_BAD;
    if (ndim == 2 && n.ny != 1) return OR_BAD;
    if (!check_points(ndim, n, nbl, h, nsrc, src_xyz)) return OR_BAD;
    if (!check_points(ndim, n, nbl, h, nrec, rec_xyz)) return OR_BAD;
    or_weights_d2(r, w);
    long N = n.nx * n.ny * n.nz;
    double* l0 = (double*)calloc((size_t)N, sizeof(double));
    double* l1 = (double*)calloc((size_t)N, sizeof(double));
    double* l2 = (double*)calloc((size_t)N, sizeof(double));
    double* bl = (double*)calloc((size_t)N, sizeof(double));
    if (!l0 || !l1 || !l2 || !bl) { free(l0); free(l1); free(l2); free(bl); return OR_BAD; }
    double hp = hprod(ndim, h);
    for (int k = nt; k >= 1; --k) {
        adjoint_level(l0, l1, l2, bl, n, ndim, nbl, w, r, h, dt, vel, eta, nrec, rec_xyz,
                      d + (long)(k - 1) * nrec);
        for (int s = 0; s < nsrc; ++s) {
            long idx[8];
            double wc[8];
            int m = corners(ndim, n, nbl, h, src_xyz + (long)s * ndim, idx, wc);
            double acc = 0.0;
            for (int c = 0; c < m; ++c) {
                double v = (double)vel[idx[c]];
                acc += wc[c] * dt * dt * v * v * l0[idx[c]];
            }
            qout[(long)(k - 1) * nsrc + s] = acc / hp;
        }
        double* t = l2;
        l2 = l1;
        l1 = l0;
        l0 = t;
    }
    free(l0); free(l1); free(l2); free(bl);
    return OR_OK;
}

/* Gradient of J = 1/2 sum_n |d^n - dobs^n|^2 with respect to m = 1/v^2 by the
 * adjoint state, keeping the whole forward history in memory (small grids).
 * B = dt^2 / m, so dF^k/dm = (1/m) [D u^k - 2 u^{k-1} + E u^{k-2}] (the
 * recurrence F^k = 0 turns B (L u + S^T q / prod h) into that difference) and
 *   dJ/dm = - sum_k lambda^k dF^k/dm,
 * lambda solving the transposed recurrence driven by the residual d - dobs.
 * Writes grad[N] and *misfit. */
int or_acoustic_gradient(int ndim, const long* nxyz, int nbl, const double* h, double dt, int so,
                         const float* vel, const float* eta,
                         int nsrc, const double* src_xyz, const float* wavelet,
                         int nrec, const double* rec_xyz, const double* dobs, int nt,
                         double* grad, double* misfit) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    int r = so / 2;
    double w[64];
    if ((ndim != 2 && ndim != 3) || so < 2 || so % 2 || r > 63 || nt < 1) return OR_BAD;
    or_weights_d2(r, w);
    long N = n.nx * n.ny * n.nz;
    size_t nr = (size_t)(nrec > 0 ? nrec : 1);
    /* history: slot t + 1 holds u^t for t = -1 .. nt */
    double* hist = (double*)calloc((size_t)N * (size_t)(nt + 2), sizeof(double));
    double* res = (double*)calloc((size_t)nt * nr, sizeof(double));
    double* up = (double*)calloc((size_t)N, sizeof(double));
    double* uc = (double*)calloc((size_t)N, sizeof(double));
    double* l0 = (double*)calloc((size_t)N, sizeof(double));
    double* l1 = (double*)calloc((size_t)N, sizeof(double));
    double* l2 = (double*)calloc((size_t)N, sizeof(double));
    double* bl = (double*)calloc((size_t)N, sizeof(double));
    int rc = (!hist || !res || !up || !uc || !l0 || !l1 || !l2 || !bl) ? OR_BAD : OR_OK;
    for (int t = 0; t < nt && rc == OR_OK; ++t) {
        rc = or_acoustic_forward(ndim, nxyz, nbl, h, dt, so, vel, eta, nsrc, src_xyz,
                                 wavelet + (long)t * nsrc, nrec, rec_xyz, res + (long)t * nrec, 1,
                                 up, uc);
        if (rc == OR_OK) memcpy(hist + (size_t)(t + 2) * (size_t)N, uc, sizeof(double) * (size_t)N);
    }
    if (rc == OR_OK) {
        double J = 0.0;
        for (long k = 0; k < (long)nt * nrec; ++k) {
            res[k] -= dobs[k];
            J += 0.5 * res[k] * res[k];
        }
        *misfit = J;
        for (long i = 0; i < N; ++i) grad[i] = 0.0;
        for (int k = nt; k >= 1; --k) {
            adjoint_level(l0, l1, l2, bl, n, ndim, nbl, w, r, h, dt, vel, eta, nrec, rec_xyz,
                          res + (long)(k - 1) * nrec);
            const double* uk = hist + (size_t)(k + 1) * (size_t)N;  /* u^k     */
            const double* uk1 = hist + (size_t)k * (size_t)N;      /* u^{k-1} */
            const double* uk2 = hist + (size_t)(k - 1) * (size_t)N;  /* u^{k-2} */
            for (long i = 0; i < N; ++i) {
                double s = eta ? 0.5 * dt * (double)eta[i] : 0.0;
                double v = (double)vel[i];
                double dFdm = v * v * ((1.0 + s) * uk[i] - 2.0 * uk1[i] + (1.0 - s) * uk2[i]);
                grad[i] -= l0[i] * dFdm;
            }
            double* t = l2;
            l2 = l1;
            l1 = l0;
            l0 = t;
        }
    }
    free(hist); free(res); free(up); free(uc); free(l0); free(l1); free(l2); free(bl);
    return rc;
}

/* Misfit J = 1/2 sum (d - dobs)^2 of a forward run from the zero state. */
int or_acoustic_misfit(int ndim, const long* nxyz, int nbl, const double* h, double dt, int so,
                       const float* vel, const float* eta, int nsrc, const double* src_xyz,
                       const float* wavelet, int nrec, const double* rec_xyz, const double* dobs,
                       int nt, double* misfit) {
    dims_t n = {nxyz[0], nxyz[1], nxyz[2]};
    long N = n.nx * n.ny * n.nz;
    double* tr = (double*)calloc((size_t)nt * (size_t)(nrec > 0 ? nrec : 1), sizeof(double));
    double* up = (double*)calloc((size_t)N, sizeof(double));
    double* uc = (double*)calloc((size_t)N, sizeof(double));
    if (!tr || !up || !uc) { free(tr); free(up); free(uc); return OR_BAD; }
    int rc = or_acoustic_forward(ndim, nxyz, nbl, h, dt, so, vel, eta, nsrc, src_xyz, wavelet,
                                 nrec, rec_xyz, tr, nt, up, uc);
    double J = 0.0;
    for (long k = 0; k < (long)nt * nrec; ++k) J += 0.5 * (tr[k] - dobs[k]) * (tr[k] - dobs[k]);
    *misfit = J;
    free(tr); free(up); free(uc);
    return rc;
}
