/*
 * fd.h -- C ABI of the MI355X (gfx950) explicit finite-difference wave
 * propagation library (libfd.so).
 *
 * The library implements the time-stepping scheme of Louboutin et al.,
 * "Performance prediction of finite-difference solvers for different computer
 * architectures": Algorithm 1 (section 2) -- a second-order leapfrog update of
 * the wavefield by a symmetric k-point stencil, followed by source injection --
 * for
 *   - the acoustic equation of Appendix A, Eq. (Acou): m u_tt - lap u = q with
 *     m = 1/v^2 and zero initial state, and
 *   - the TTI pseudo-acoustic system of Appendix A, Eq. (TTI), whose rotated
 *     operators are those of Eq. (DiffOp),
 * with an absorbing layer (the paper leaves boundary treatment outside its
 * model, section 2) and receivers sampled from the updated field.
 *
 * Conventions
 *   - Space order "so" is the order of the central stencils; the 1D stencil
 *     has k = so + 1 points (section 4.1) and radius r = so / 2.
 *   - Every field the caller passes or receives is float32, C-order
 *     [Nz][Ny][Nx] with x contiguous (2D: [Nz][Nx]), over the padded array
 *     N_a = n_a + 2 nbl (physical points plus the layer on both sides).
 *   - Coordinates are double, metres from the physical origin (the first
 *     physical grid point), ordered (x, y, z) in 3D and (x, z) in 2D.
 *   - Points beyond the padded array read as zero (homogeneous Dirichlet).
 *   - Sparse points are interpolated multilinearly: along each axis the cell
 *     index is i = floor(c/h + nbl) clamped to [0, N-2], weights 1-f and f.
 *
 * Ownership and threading
 *   - The caller owns every device buffer, including the workspace; the
 *     library never allocates device memory.  It owns only the small host
 *     context returned by fd_setup (freed by fd_destroy).
 *   - All device work is enqueued asynchronously on the hipStream_t passed as
 *     `stream` (NULL = default stream); calls return without waiting, except
 *     where stated.  Synchronise on that stream before reading results.
 *   - One context serves one stream at a time and is not thread-safe.  The
 *     only global state is the per-device scratch array of
 *     fd_cnn_wgrad_noalloc (and its address table, guarded by a lock).
 *
 * Errors: every entry point returns an int32 status (FD_OK = 0).  No exception
 * crosses the ABI and nothing is printed.  fd_last_error() gives a
 * per-context message for the last failure.
 */
#ifndef FD_H
#define FD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define FD_OK 0
#define FD_ERR_INVALID_ARG 1 /* bad pointer, shape, order, point or count */
#define FD_ERR_UNSTABLE_DT 2 /* dt above the CFL bound of Eq. (stability) */
#define FD_ERR_UNSUPPORTED 3 /* space order or physics not built */
#define FD_ERR_WORKSPACE 4   /* workspace too small or misaligned */
#define FD_ERR_DEVICE 5      /* a HIP runtime call failed */
#define FD_ERR_NONFINITE 6   /* non-finite or non-positive model values */
#define FD_ERR_HOST 7        /* host memory for the setup's or a point table's host-side work
                                could not be obtained (nothing is left half set up) */

/* Physics. */
#define FD_ACOUSTIC 0 /* Eq. (Acou), 2D or 3D */
#define FD_TTI 1      /* Eq. (TTI) with Eq. (DiffOp), 3D */
#define FD_VTI 2      /* Eq. (vVTI), 2D (D_xx) or 3D (D_xx + D_yy as the horizontal operator) */

/* Wavefield selectors for fd_get_field / fd_set_field.  Acoustic uses the
 * first two; VTI and TTI use all four (p and r). */
#define FD_FIELD_PREV 0   /* u^{n-1}  (VTI/TTI: p^{n-1}) */
#define FD_FIELD_CUR 1    /* u^{n}    (VTI/TTI: p^{n})   */
#define FD_FIELD_R_PREV 2 /* VTI/TTI r^{n-1} */
#define FD_FIELD_R_CUR 3  /* VTI/TTI r^{n}   */

/* fd_forward / fd_forward_shots flags. */
#define FD_ZERO_STATE 1 /* start from the zero state of Eq. (Acou)/(TTI) */
/* Use the point table of the last upload (the previous stepping call's
 * sources and receivers, in that call's order and, for fd_forward_shots, with
 * its per-shot counts) without reading coordinates: src->coords, rec->coords
 * and the count arrays may be NULL, src->n and rec->n must equal the counts of
 * that upload (FD_ERR_INVALID_ARG otherwise, or when nothing was uploaded
 * yet), and the data pointers are used as usual.  The host work of the call
 * then does not grow with the number of points. */
#define FD_KEEP_POINTS 2

/* Largest supported space order (radius 8). */
#define FD_MAX_SPACE_ORDER 16

typedef struct fd_grid {
    int32_t ndim;        /* 2 or 3 */
    int32_t space_order; /* even, 2..FD_MAX_SPACE_ORDER */
    int32_t physics;     /* FD_ACOUSTIC, FD_VTI or FD_TTI (TTI needs ndim == 3) */
    int32_t nbl;         /* absorbing-layer points added on both sides of each axis */
    int64_t shape[3];    /* physical points (nx, ny, nz); ny must be 1 in 2D */
    double spacing[3];   /* (hx, hy, hz) in metres; hy ignored in 2D */
    double dt;           /* time step in seconds */
} fd_grid;

/* Device pointers to float32 fields on the padded shape (dense
 * [Nz][Ny][Nx]).  They are read only by fd_setup and may be released once it
 * has returned. */
typedef struct fd_model {
    const float* vel;     /* P velocity v (m/s), v > 0; m = 1/v^2 */
    const float* eta;     /* damping rate (1/s) of u_tt + eta u_t = v^2 (lap u + q);
                             NULL = no damping */
    const float* epsilon; /* VTI/TTI: Thomsen epsilon (NULL for acoustic) */
    const float* delta;   /* VTI/TTI: Thomsen delta, 0 <= ... <= epsilon is required */
    const float* theta;   /* TTI: tilt from the vertical (radians; NULL for VTI) */
    const float* phi;     /* TTI: azimuth (radians; NULL for VTI) */
} fd_model;

/* A set of sparse points (sources or receivers). */
typedef struct fd_points {
    int32_t n;            /* number of points (0 allowed) */
    const double* coords; /* host [n][ndim] metres, see Conventions */
    float* data;          /* device [nt][n]: wavelet (sources, read) or traces
                             (receivers, overwritten) */
} fd_points;

typedef struct fd_ctx fd_ctx;

/* Bytes of device workspace fd_setup needs for this grid with room for up to
 * `max_points` sparse points per fd_forward call (sources + receivers,
 * 0 <= max_points <= 2^27).  Pure host computation.  Returns
 * FD_ERR_INVALID_ARG / FD_ERR_UNSUPPORTED for grids fd_setup would reject. */
int32_t fd_workspace_bytes(const fd_grid* grid, int32_t max_points, uint64_t* bytes);

/* Validates the grid, derives the per-point coefficients the time loop reads
 * (dt^2 v^2, eta dt/2 and, for VTI and TTI, the Thomsen and rotation factors
 * of Eq. (TTI) and Eq. (DiffOp)) into `workspace` (device, 256-byte aligned,
 * at least fd_workspace_bytes), checks the model (finite, v > 0, TTI:
 * delta <= epsilon) and the CFL bound of Eq. (stability) at the model's
 * fastest speed (for TTI the horizontal P speed v sqrt(1 + 2 epsilon)), and
 * sets the wavefields to zero.  The coefficients are computed in FP64 on the
 * host from the FP32 model (copied there) and rounded once to FP32; the call
 * therefore synchronises `stream` and returns when the workspace is ready.
 * On success *out receives a context; the workspace must stay allocated until
 * fd_destroy. */
int32_t fd_setup(const fd_grid* grid, const fd_model* model, void* workspace,
                 uint64_t workspace_bytes, int32_t max_points, void* stream, fd_ctx** out);

/* Runs nt time steps of Algorithm 1: for each step n, the stencil update of
 * every point (with the damping layer), then the source term q[n] added to
 * the new level (Algorithm 1, "Add Source"; for TTI into both p and r), then
 * receivers sampled from the new level into rec->data[n] (TTI: from p).
 * The sampling of step n is launched with step n + 1's work, which only
 * reads that level, and the last step's when the call's steps end: every
 * row of rec->data is written once the call's work on `stream` completes.
 * The point-source amplitude q enters as dt^2 v^2 q / (prod h) / (1 + eta dt/2)
 * spread over the multilinear corners; where several points share a corner
 * their contributions are added in point order, so runs are bitwise
 * reproducible.  flags & FD_ZERO_STATE starts from
 * zero; otherwise the run continues from the held state (fd_set_field or a
 * previous call).  src or rec may be NULL.  Asynchronous on `stream`, except
 * that new point coordinates are uploaded with one synchronisation.  A call
 * whose coordinates equal the previous call's (compared on the host, in time
 * proportional to the number of points) or that passes FD_KEEP_POINTS
 * launches kernels only, so it can be captured in a HIP graph; the index of the level holding u^n is host
 * state that advances at capture time, so replays agree with it when nt is
 * even (or every run starts from FD_ZERO_STATE and reads only traces). */
int32_t fd_forward(fd_ctx* ctx, int32_t nt, const fd_points* src, const fd_points* rec,
                   int32_t flags, void* stream);

/* Copy a wavefield level between the context and a dense device array of the
 * padded shape ([Nz][Ny][Nx] float32).  Asynchronous on `stream`. */
int32_t fd_get_field(fd_ctx* ctx, int32_t which, float* dst, void* stream);
int32_t fd_set_field(fd_ctx* ctx, int32_t which, const float* src, void* stream);

/* Host helpers (no device work).
 * fd_stencil_weights: central weights of order space_order for derivative
 *   `deriv` (1 or 2) on unit spacing, w[0..r] (w[-j] = w[j] for deriv 2,
 *   -w[j] for deriv 1), section 4.1.
 * fd_cfl_dt: largest dt allowed by Eq. (stability) with a1 = 4 for a wave
 *   speed vmax on this grid. */
int32_t fd_stencil_weights(int32_t space_order, int32_t deriv, double* w);
int32_t fd_cfl_dt(const fd_grid* grid, double vmax, double* dt_max);

/* STREAM-style triad a[i] = b[i] + s c[i] over n floats (device pointers,
 * 16-byte aligned): the measured bandwidth ceiling of section 3.1 (STREAM
 * TRIAD as the practical memory limit), and a kernel of exactly known
 * traffic (8 bytes read, 4 written per element) for calibrating hardware
 * byte counters.  Asynchronous on `stream`. */
int32_t fd_triad(float* a, const float* b, const float* c, float s, int64_t n, void* stream);

/* fd_triad with an explicit launch shape, for sweeping the ceiling: each
 * thread moves `unroll` (1, 2, 4 or 8) 16-byte vectors of each array per
 * iteration; blocks = 0 gives every 256-thread block one chunk of 256 unroll
 * vectors, blocks > 0 launches that many blocks striding over the chunks;
 * flags = FD_TRIAD_TEMPORAL uses ordinary instead of non-temporal loads and
 * stores.  Same traffic as fd_triad.  FD_ERR_INVALID_ARG for other values. */
#define FD_TRIAD_TEMPORAL 1
int32_t fd_triad_config(float* a, const float* b, const float* c, float s, int64_t n,
                        int32_t unroll, int32_t blocks, int32_t flags, void* stream);

/* ------------------------------------------------------------------------ */
/* Several shots on one model (acoustic only)                                */
/* ------------------------------------------------------------------------ */
/*
 * A survey runs many independent shots (source positions) on the same
 * model.  Section 2 notes that the operational intensity of the stencil does
 * not depend on how the work is split; sharing the model is what changes it:
 * a context of nshots wavefields advances all of them per launch, and the
 * tiled 3D kernel reads dt^2 v^2 (and the damping coefficient) once per tile
 * for a group of shots, so the bytes per shot-point fall from 16 towards 12.
 * Fields of shot k are selected with fd_get_shot_field / fd_set_shot_field;
 * such a context steps with fd_forward_shots and forms the gradient of all
 * its shots with fd_forward_checkpointed_shots / fd_gradient_shots (below);
 * fd_forward, fd_adjoint, fd_forward_checkpointed and fd_gradient accept
 * only single-shot contexts.
 */

/* Workspace bytes for a context of nshots wavefields (1 <= nshots <= 4096)
 * with room for max_points sparse points in total. */
int32_t fd_workspace_bytes_shots(const fd_grid* grid, int32_t nshots, int32_t max_points,
                                 uint64_t* bytes);

/* fd_setup for nshots wavefields on one model (FD_ERR_UNSUPPORTED for TTI
 * with nshots > 1).  fd_setup is this call with nshots = 1. */
int32_t fd_setup_shots(const fd_grid* grid, const fd_model* model, int32_t nshots,
                       void* workspace, uint64_t workspace_bytes, int32_t max_points,
                       void* stream, fd_ctx** out);

/* nt steps of Algorithm 1 for every shot of the context.  src holds the
 * sources of all shots one after another (src->n = sum of src_counts, host
 * array [nshots]), with wavelets src->data [nt][src->n]; rec likewise, with
 * traces rec->data [nt][rec->n].  Shot k's points are injected into and
 * sampled from shot k's wavefield only.  Flags and asynchrony as fd_forward. */
int32_t fd_forward_shots(fd_ctx* ctx, int32_t nt, const fd_points* src, const int32_t* src_counts,
                         const fd_points* rec, const int32_t* rec_counts, int32_t flags,
                         void* stream);

/* fd_get_field / fd_set_field for shot `shot` (0-based). */
int32_t fd_get_shot_field(fd_ctx* ctx, int32_t shot, int32_t which, float* dst, void* stream);
int32_t fd_set_shot_field(fd_ctx* ctx, int32_t shot, int32_t which, const float* src,
                          void* stream);

/* ------------------------------------------------------------------------ */
/* Adjoint and gradient (acoustic only)                                      */
/* ------------------------------------------------------------------------ */
/*
 * The zero-state forward run is a linear map F from the source wavelets q
 * (fd_points.data of the sources, [nt][nsrc]) to the traces d ([nt][nrec]) for
 * a fixed model m = 1/v^2 of Eq. (Acou).  The velocity gradient used by
 * full-waveform inversion (the application the paper's Introduction names)
 * comes from the adjoint state: with lambda the solution of the transposed
 * recurrence driven by the trace sensitivities d' = dJ/dd,
 *   dJ/dm = -sum_k lambda^k (D u^k - 2 u^{k-1} + E u^{k-2}) / m,
 * D = 1 + eta dt/2, E = 1 - eta dt/2, and dJ/dq = F^T d'.  The library runs the
 * transposed recurrence in the variable mu = dt^2 v^2 lambda, in which it has
 * exactly the form of the forward step (the same stencil kernels), with the
 * receivers as sources, backwards in time.  The forward history is rebuilt
 * from checkpoints: every `interval` steps the pair (u^{n-1}, u^n) is saved,
 * and each segment of `interval` steps is recomputed before the adjoint
 * sweeps through it, storing the acceleration A L u + source of every step
 * of the segment for the imaging condition.  Memory: 2 ceil(nt/interval)
 * dense fields plus interval + 2 padded volumes plus one dense FP64 field;
 * compute: at most two forward runs and one adjoint run.
 *
 * A context of several shots (fd_setup_shots) runs these steps for all of its
 * shots in the same launches (fd_forward_checkpointed_shots,
 * fd_gradient_shots), the tiled kernel advancing up to two shots per block on
 * shared reads of dt^2 v^2 and the damping coefficient; the store then holds
 * every shot's checkpoints, accelerations, adjoint levels and imaging sums,
 * and the gradient is the sum over the shots.
 *
 * TTI and VTI contexts return FD_ERR_UNSUPPORTED from these calls.
 */

/* fd_gradient wrt selectors. */
#define FD_WRT_M 0   /* gradient with respect to m = 1/v^2 (squared slowness) */
#define FD_WRT_VEL 1 /* gradient with respect to v */
/* ORed into wrt: add the gradient into grad instead of overwriting it (the
 * sum over the shots of a survey, one shot per fd_gradient call). */
#define FD_GRAD_ACCUMULATE 256

/* Bytes of the caller-owned checkpoint store for nt steps with a checkpoint
 * every `interval` steps (interval <= 0: the memory-minimising choice, about
 * sqrt(2 nt) scaled by the padded/dense volume ratio; *interval_out receives
 * the value used and may be NULL), for all shots of the context (nshots times
 * the single-shot store, with the same interval).  Host computation only. */
int32_t fd_checkpoint_bytes(const fd_ctx* ctx, int32_t nt, int32_t interval, uint64_t* bytes,
                            int32_t* interval_out);

/* Zero-state forward run of nt steps, exactly as fd_forward with
 * FD_ZERO_STATE (same traces), that also fills `store` (device, 256-byte
 * aligned, at least fd_checkpoint_bytes) with the checkpoints and the last
 * segment's accelerations for fd_gradient.  The context remembers the store,
 * nt and interval; fd_gradient must then be given the same store, nt,
 * interval and source wavelets.  Asynchronous on `stream`. */
int32_t fd_forward_checkpointed(fd_ctx* ctx, int32_t nt, const fd_points* src,
                                const fd_points* rec, int32_t interval, void* store,
                                uint64_t store_bytes, void* stream);

/* Gradient of J with respect to the model (wrt = FD_WRT_M or FD_WRT_VEL)
 * and the source wavelets, for the trace sensitivities adj->data ([nt][n],
 * device, read; adj->coords are the receiver positions of the forward run).
 * grad: device dense [Nz][Ny][Nx] float32 over the padded array, overwritten
 * (or added to, with FD_GRAD_ACCUMULATE in wrt).
 * wavelet_grad: device [nt][nsrc] float32 (dJ/dq), overwritten; NULL skips it.
 * Requires a preceding fd_forward_checkpointed with the same store, nt,
 * interval and sources (FD_ERR_INVALID_ARG otherwise); may be called again on
 * the same store with other sensitivities.  Leaves the held wavefields
 * undefined.  Asynchronous on `stream`, except for a point-table upload. */
int32_t fd_gradient(fd_ctx* ctx, int32_t nt, const fd_points* src, const fd_points* adj,
                    int32_t interval, void* store, uint64_t store_bytes, int32_t wrt,
                    float* grad, float* wavelet_grad, void* stream);

/* fd_forward_checkpointed and fd_gradient for a context of several shots:
 * the points of all shots one after another with per-shot counts, as in
 * fd_forward_shots (src->n = sum of src_counts; traces rec->data [nt][rec->n];
 * sensitivities adj->data [nt][adj->n] with adj_counts per shot; dJ/dq
 * wavelet_grad [nt][src->n]).  grad receives the sum over the shots of their
 * gradients, formed shot by shot in shot order (bitwise the result of one
 * fd_gradient per shot on single-shot contexts, the later ones with
 * FD_GRAD_ACCUMULATE).  On a single-shot context the counts may be NULL and
 * these are fd_forward_checkpointed and fd_gradient.  Errors as those, plus
 * FD_ERR_INVALID_ARG when counts are missing or do not sum to n. */
int32_t fd_forward_checkpointed_shots(fd_ctx* ctx, int32_t nt, const fd_points* src,
                                      const int32_t* src_counts, const fd_points* rec,
                                      const int32_t* rec_counts, int32_t interval, void* store,
                                      uint64_t store_bytes, void* stream);
int32_t fd_gradient_shots(fd_ctx* ctx, int32_t nt, const fd_points* src,
                          const int32_t* src_counts, const fd_points* adj,
                          const int32_t* adj_counts, int32_t interval, void* store,
                          uint64_t store_bytes, int32_t wrt, float* grad, float* wavelet_grad,
                          void* stream);

/* The least-squares misfit of full-waveform inversion (the objective whose
 * gradient fd_gradient returns when given res as the trace sensitivities):
 * res = d - d_obs elementwise (n FP32 values, device; res may alias d) and
 * J[0] += 1/2 sum res^2.  J is a device array of FD_MISFIT_DOUBLES doubles:
 * J[0] accumulates (the caller clears it), J[1..] receive per-block partial
 * sums, which are added to J[0] in a fixed order, so the result is the same
 * bits on every run.  The sum is taken in FP64 because finite differences of
 * J check the gradient.  Asynchronous on `stream`.  FD_ERR_INVALID_ARG for
 * n < 0 or missing pointers. */
#define FD_MISFIT_DOUBLES 1025
int32_t fd_misfit(const float* d, const float* d_obs, int64_t n, float* res, double* J,
                  void* stream);

/* The transpose of the zero-state map q -> d: reads adj->data ([nt][nrec],
 * receiver positions adj->coords) and writes out->data ([nt][nsrc], source
 * positions out->coords) = F^T d'.  Uses the context's wavefield levels as the
 * adjoint state (the held forward state is lost).  Asynchronous on `stream`,
 * except for a point-table upload. */
int32_t fd_adjoint(fd_ctx* ctx, int32_t nt, const fd_points* adj, const fd_points* out,
                   void* stream);

/* ------------------------------------------------------------------------ */
/* Learned coarse-grid correction (acoustic)                                 */
/* ------------------------------------------------------------------------ */
/*
 * Not in the paper: its cost study (section 6) trades space order against
 * grid spacing at a fixed physical problem; this is the learned end of that
 * trade.  A coarse, low-order solver is corrected every few steps by a small
 * network so that its state tracks a fine, high-order solution sampled at the
 * coarse points.  The network is three 3 x 3 x 3 convolution layers
 *   y1 = relu(conv(x, w1) + b1), y2 = relu(conv(y1, w2) + b2),
 *   d = conv(y2, w3) + b3,
 * conv(x, w)[p][co] = sum_tap sum_ci x[p + off(tap)][ci] w[tap][ci][co] (zero
 * padding, tap = 9 (dz+1) + 3 (dy+1) + (dx+1)), run on the BF16 matrix cores
 * with FP32 accumulation.  Its input x has 8 channels (s u^n, s u^{n-1},
 * s u^n nu, s u^{n-1} nu, zeros), s = 1 / max|u^n|, nu = v / vref - 1, and its
 * 2 output channels d are the corrections of u^n and u^{n-1} in the same
 * units.  Every input channel is linear in the wavefield; trained without
 * biases, the network then maps a quiet region to no correction.
 *
 * Layouts: activations are channels-last BF16 (uint16_t bit patterns)
 * [nz][ny][nx][c] with c = 8 or 16 over the padded grid, 16-byte aligned.
 * Every layer's parameters are stored padded to 16 x 16 channels as FP32
 * [27][16 ci][16 co] followed by the bias [16] (FD_CNN_LAYER_FLOATS floats;
 * unused channels are zero), which is also the layout of the weight
 * gradient.  shape[] is (nz, ny, nx).  All calls are asynchronous on
 * `stream`; the caller owns every buffer.
 */
#define FD_CNN_LAYER_FLOATS (27 * 256 + 16)
#define FD_CNN_RELU 0   /* y = bf16(relu(conv + b)), 16 channels */
#define FD_CNN_LINEAR 1 /* yf = conv + b in FP32, first cout_store channels */
#define FD_CNN_MASKED 2 /* y = bf16(conv * (mask > 0)), 16 channels, no bias (backward data) */
#define FD_CNN_IDENTITY 3 /* y = bf16(conv + b), 16 channels (a layer without activation) */
#define FD_CNN_UNMASKED 4 /* y = bf16(conv), 16 channels, no bias (its backward data) */

/* Elements (uint16_t) of a packed layer operand for cin_pad = 8 or 16. */
int32_t fd_cnn_packed_elems(int32_t cin_pad, int64_t* elems);

/* Pack one layer (layer = FD_CNN_LAYER_FLOATS FP32 values, layout above) into
 * the matrix-core operand for inputs of cin_pad channels.  transpose != 0
 * packs the backward-data operator instead (flipped taps, exchanged
 * channels). */
int32_t fd_cnn_pack(const float* layer, int32_t cin_pad, int32_t transpose, uint16_t* packed,
                    void* stream);

/* One convolution: x [shape][cin_pad] BF16 -> y (modes RELU, MASKED: BF16
 * [shape][16]) or yf (mode LINEAR: FP32 [shape][cout_store]).  bias: the 16
 * FP32 bias values (ignored by MASKED); mask: BF16 [shape][16] (MASKED
 * only). */
int32_t fd_cnn_conv(const uint16_t* x, int32_t cin_pad, const int64_t* shape,
                    const uint16_t* packed, const float* bias, int32_t mode, const uint16_t* mask,
                    int32_t cout_store, uint16_t* y, float* yf, void* stream);

/* FP32 scratch (floats) the weight gradient needs for this shape. */
int32_t fd_cnn_wgrad_scratch(const int64_t* shape, int64_t* floats);

/* Weight and bias gradient of one layer: dw[tap][ci][co] = sum_p
 * x[p + off(tap)][ci] dz[p][co], db[co] = sum_p dz[p][co], written to
 * grad (FD_CNN_LAYER_FLOATS FP32, layout above).  x: BF16 [shape][cx],
 * dz: BF16 [shape][cz]; (cx, cz) = (8, 16), (16, 16) or (16, 8). */
int32_t fd_cnn_wgrad(const uint16_t* x, int32_t cx, const uint16_t* dz, int32_t cz,
                     const int64_t* shape, float* scratch, int64_t scratch_floats, float* grad,
                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): fd_cnn_wgrad
 * without the scratch argument.  The partial sums live in a library-owned
 * device array of FD_CNN_NOALLOC_SCRATCH_FLOATS floats (48 MiB) that every
 * device the library runs on holds until the process ends; its address is
 * looked up on the first call on a device (the current device, which must
 * own `stream`).  Shapes whose fd_cnn_wgrad_scratch exceeds that size (more
 * than 1816 blocks of 32 x 4 voxels x 32 planes, e.g. beyond 168^3) return
 * FD_ERR_WORKSPACE; other arguments and results as fd_cnn_wgrad (the same
 * kernels, the same bits).  Calls that overlap on one device share the array
 * and race: serialise them (one stream, or events).  Allocates nothing. */
#define FD_CNN_NOALLOC_SCRATCH_FLOATS 12582912
int32_t fd_cnn_wgrad_noalloc(const uint16_t* x, int32_t cx, const uint16_t* dz, int32_t cz,
                             const int64_t* shape, float* grad, void* stream);

/* Masked mean-square loss L = 1/(2n) sum_mask |out - target|^2 (out, target
 * FP32 [nvox][cout]; mask uint8 [nvox]; inv_n = 1/n): dz = dL/dout as BF16
 * [nvox][cpad] and L added to loss[0]; loss is a device array of
 * FD_CNN_LOSS_FLOATS floats whose entries 1.. receive per-block partial sums
 * (added in a fixed order: the same bits on every run). */
#define FD_CNN_LOSS_FLOATS 257
int32_t fd_cnn_loss_grad(const float* out, const float* target, const uint8_t* mask,
                         int64_t nvox, int32_t cout, int32_t cpad, float inv_n, uint16_t* dz,
                         float* loss, void* stream);

/* Adam step t >= 1 on n FP32 parameters (bias-corrected). */
int32_t fd_cnn_adam(float* param, const float* grad, float* m, float* v, int64_t n, int32_t t,
                    float lr, float beta1, float beta2, float eps, void* stream);

/* Network input from a single-shot acoustic context's current state: x
 * (BF16 [padded shape][8]); *scale_bits receives max|u^n| (FP32 bits) over
 * the points where mask (uint8 [padded shape], NULL = all points) is set.
 * The mask keeps the grid-dependent near field of a point source out of the
 * scale and, in fd_cnn_correct, out of the correction. */
int32_t fd_cnn_features(fd_ctx* ctx, float vref, const uint8_t* mask, uint32_t* scale_bits,
                        uint16_t* x, void* stream);

/* Apply the network output d (FP32 [padded shape][2]) where mask is set (NULL
 * = everywhere): u^n += d0 max, u^{n-1} += d1 max with the scale of the
 * matching fd_cnn_features. */
int32_t fd_cnn_correct(fd_ctx* ctx, const float* d, const uint8_t* mask,
                       const uint32_t* scale_bits, void* stream);

/* Training target: t = (ref_cur - u^n, ref_prev - u^{n-1}) / max|u^n| (FP32
 * [padded shape][2]) for dense reference fields of the context's padded
 * shape. */
int32_t fd_cnn_residual(fd_ctx* ctx, const float* ref_cur, const float* ref_prev,
                        const uint32_t* scale_bits, float* target, void* stream);

/* Every stride-th point (all axes, from index 0) of a wavefield level into a
 * dense array of ceil(N_a / stride) points per axis: the coarse-grid samples
 * of a fine solution. */
int32_t fd_restrict(fd_ctx* ctx, int32_t which, int32_t stride, float* dst, void* stream);

/* Tuning options (kernel variant / launch shape), mainly for benchmarking.
 * FD_OPT_KERNEL: 0 = tiled (default), 1 = direct global-memory kernel.
 * FD_OPT_ZCHUNK: z-planes per thread block of the tiled 3D kernels (0 = auto).
 * FD_OPT_TILE: (x, y) tile of the tiled 3D acoustic kernel: 0 = 64x8 with 256
 *   threads, 1 = 64x16 with 256, 2 = 64x8 with 512, 3 = 64x16 with 512,
 *   4 = 64x24 with 768, -1 = the default for the space order, shot count and
 *   grid (one shot: 4 up to space order 8 when its x-y tiles number 90-100 %
 *   of the device's compute units, else 0); of the tiled TTI
 *   kernel: 0 = 64x8 with 512 threads, 1 = 64x4 with 256, 2 = 64x15 with
 *   960 (space orders up to 8, else FD_ERR_UNSUPPORTED), -1 = the default
 *   (2 up to space order 8 when its x-y tiles number 90-100 % of the
 *   device's compute units, else 0).
 *   FD_ERR_UNSUPPORTED for VTI (one tile shape).
 * FD_OPT_SHOTS_PER_BLOCK: shots a block of the tiled 3D acoustic kernel
 *   advances together (1, 2 or 4; 0 = default; 2 and 4 need tile 0 or 2).
 * FD_OPT_DAMPING_PROFILE: 1 (default) = when fd_setup found the 3D damping
 *   field to be a sum of per-axis profiles (sigma(x, y, z) = (s_x + s_y) + s_z
 *   with the profiles taken along the lines through the centre point,
 *   agreeing everywhere to within 2^-20 of the field's maximum, as for the
 *   usual absorbing layer), the tiled 3D acoustic, VTI and TTI kernels
 *   evaluate that sum instead of reading the field (4 bytes per damped point
 *   less traffic); 0 = always read the field.  Other fields, the 2D and the
 *   direct kernels always read the field. */
#define FD_OPT_KERNEL 1
#define FD_OPT_ZCHUNK 2
#define FD_OPT_TILE 3
#define FD_OPT_SHOTS_PER_BLOCK 4
#define FD_OPT_DAMPING_PROFILE 5
/* FD_OPT_FUSED_IMAGING: 1 (default) = fd_gradient adds the imaging term
 * inside the adjoint stencil launch (tiled 3D kernel with tile 0 or 4, or
 * tile 2 with two shots per block: one read of the adjoint field less per
 * point and step); 0 = a
 * separate imaging launch per step.  Both give the same bits. */
#define FD_OPT_FUSED_IMAGING 6
int32_t fd_set_option(fd_ctx* ctx, int32_t option, int64_t value);

/* The value an option has on ctx: the caller's last setting, or the default
 * the context chose for its grid, order, shot count and device (for
 * FD_OPT_TILE the configuration number; for FD_OPT_ZCHUNK 0 = automatic).
 * *value is written only on FD_OK; an unknown option is FD_ERR_INVALID_ARG.
 * Pure host. */
int32_t fd_get_option(const fd_ctx* ctx, int32_t option, int64_t* value);

/* Frees the host context (not the workspace). NULL is accepted. */
int32_t fd_destroy(fd_ctx* ctx);

/* Static description of a status code. */
const char* fd_strerror(int32_t status);

/* Message for the last failure on this context ("" if none). */
const char* fd_last_error(const fd_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FD_H */
