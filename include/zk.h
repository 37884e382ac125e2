/*
 * zk.h -- C ABI of the MI355X (gfx950) Zakharov/HOS wave-step library.
 *
 * The library evaluates the right-hand side of the canonical Zakharov system
 * for the surface elevation eta and surface potential psi (Sec. 3.1,
 * eq:zakharov_kin and eq:zakharov_dyn), whose cost is the Dirichlet-Neumann
 * operator G(eta) psi expanded in the Craig-Sulem / high-order-spectral
 * series of order M (Sec. 3.2, eq:G0, eq:G1, eq:G2, eq:dno_truncated; the
 * series is continued past G_2 by the surface-potential recursion of Sec. 4.2,
 * eq:phi0-eq:phi2).  Every product is dealiased by the 3/2 rule and tapered
 * (Sec. 6.1); the state filter of Sec. 3.4 (eq:state_filter) follows each
 * full RK4 step.
 *
 * Conventions shared by every entry point
 *   Layout     fields are device pointers to nx*ny doubles, row-major [ny][nx]
 *              (x fastest), contiguous, at least 16-byte aligned, on the
 *              device that was current when zk_bind was called.
 *   Ownership  the caller owns every field buffer and the workspace; the
 *              library never allocates device memory.  A context owns only
 *              host-side plans.
 *   Aliasing   outputs must not alias inputs (zk_step works in place).
 *   Asynchrony every call is enqueued on the bound stream and returns before
 *              the GPU finishes, except zk_hamiltonian, which synchronises
 *              the stream to return a host double.
 *   Errors     0 on success, a negative ZK_E* code otherwise, with a message
 *              in zk_last_error.  No exception crosses the ABI.
 *   Threads    a context is not thread-safe; use one context per stream.
 *   Sizes      nx and ny must each be a power of two in [4, 2048], three
 *              times one in [12, 1536] (12, 24, ..., 1536) or five times one
 *              in [20, 1280] (20, 40, ..., 1280), with nx a
 *              multiple of 16 (the mixed fields are tiled in 64-byte groups
 *              of columns: at least 16 or 48 points), and ny may be 1 (a
 *              1D grid); nx is the
 *              fast (row) axis.  The dealiased products run on the
 *              3nx/2 x 3ny/2 grid.  Spectra keep their Nyquist row and column at zero, so
 *              input fields are projected onto |m_x| < nx/2, |m_y| < ny/2.
 */
#ifndef ZK_H
#define ZK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct zk_ctx zk_ctx;

enum {
    ZK_OK = 0,
    ZK_EINVAL = -1,    /* invalid argument or state                          */
    ZK_ENOWS = -2,     /* workspace unbound or smaller than zk_workspace_bytes */
    ZK_EDEVICE = -3,   /* a HIP call failed; its text is in zk_last_error     */
    ZK_EDIVERGED = -4  /* NaN or Inf in the state after zk_step              */
};

/* Option keys for zk_set_option. */
enum {
    ZK_OPT_EPS = 1,       /* nonlinear-amplitude dial eps in [0, 1] (Sec. 3.2,
                             eq:dno_truncated, eq:dyn_truncated); default 1  */
    ZK_OPT_TAPER = 2,     /* 1: taper exp(-(|k|/kc)^8) on every product
                             (Sec. 6.1); 0: off.  Default 1                  */
    ZK_OPT_FILTER = 3,    /* 1: state filter A(k) after each RK4 step
                             (Sec. 3.4, eq:state_filter); 0: off.  Default 1 */
    ZK_OPT_PRECISION = 4, /* 64: transforms and products in FP64 (default);
                             32: transforms and products in FP32 with the
                             series sum, the state and the Hamiltonian in
                             FP64.  Changes the workspace size: set it before
                             zk_bind.                                         */
    ZK_OPT_CHECK = 5,     /* 1: zk_step checks the result for NaN/Inf, which
                             synchronises the stream (default); 0: no check,
                             zk_step stays fully asynchronous                 */
    ZK_OPT_INTEGRATOR = 7,/* ZK_INTEGRATOR_RK4 (default) or ZK_INTEGRATOR_IFAB2;
                             changes the workspace size: set it before zk_bind */
    ZK_OPT_BOUNDARY = 8,  /* ZK_BC_PERIODIC (default) or ZK_BC_REFLECT; set
                             before zk_bind                                   */
    ZK_OPT_ROW_FFT = 9,   /* form of the padded row passes' transforms:
                             ZK_ROW_FFT_STOCKHAM (default) or ZK_ROW_FFT_LANES;
                             zk_autotune times both at the chosen team shape
                             and keeps the faster.  Same results to rounding. */
    ZK_OPT_ROW_PROGRAMS = 10, /* 1 (default): padded row passes of the team
                             shapes that compile them (E = 3 teams of 64 to
                             1024 threads, E = 6 teams of 128 to 512) run each
                             row program whose operation sequence is one of
                             the compiled shapes as straight-line code; other
                             programs and shapes interpret the op list.
                             0: interpret every program.  Same results
                             bit for bit.                                     */
    ZK_OPT_PROFILE = 6    /* 1: bracket every kernel launch with HIP events on
                             the bound stream and accumulate per-kind times for
                             zk_kernel_stats (adds event records between
                             launches); 0: off (default)                      */
};

/* Row transform forms (ZK_OPT_ROW_FFT).  STOCKHAM: radix-E step in
 * registers, then radix-4/2 Stockham passes through LDS, a block barrier
 * each.  LANES (padded row passes of teams of 64 to 1024 threads whose two
 * LDS buffers fit; other shapes keep STOCKHAM): the inverse transform leaves
 * the physical row in a permuted order and the forward transform takes it
 * back, so no pass reorders; only the stages that span wavefronts go through
 * LDS behind barriers, and the 64-point stages over a wavefront's lanes
 * exchange partners by DPP lane permutes and ds_bpermute, without LDS
 * storage or barriers.  Pointwise products between the two do not see the
 * order.  (Cooley-Tukey decimation in frequency and its transpose.) */
enum {
    ZK_ROW_FFT_STOCKHAM = 0,
    ZK_ROW_FFT_LANES = 1
};

/* Integrators of zk_step (ZK_OPT_INTEGRATOR). */
enum {
    ZK_INTEGRATOR_RK4 = 0,   /* classical RK4: four right-hand sides per step  */
    ZK_INTEGRATOR_IFAB2 = 1  /* the paper's exact-linear Adams-Bashforth 2
                                (Sec. 3.4, eq:split, eq:lin_prop, eq:if_ab2_eta,
                                eq:if_ab2_psi): the linear part L = [[0, G0],
                                [-g, 0]] is integrated exactly per mode, the
                                forcing F = (G^[M] psi - G0 psi, N) enters
                                through its constant-forcing response with the
                                extrapolation F* = 3/2 F_n - 1/2 F_{n-1}; one
                                right-hand side per step.  The first step of
                                every zk_step call is the integrating-factor
                                Euler bootstrap F* = F_0 (no history is kept
                                across calls). */
};

/* Boundaries (ZK_OPT_BOUNDARY). */
enum {
    ZK_BC_PERIODIC = 0,  /* periodic rectangle                              */
    ZK_BC_REFLECT = 1    /* reflecting walls on all four sides by the even
                            extension of Sec. "Boundary conditions via even
                            extension" (eq:even_ext): the nx x ny cell-centred
                            fields are mirrored (half-sample symmetric) onto a
                            2nx x 2ny periodic grid of 2Lx x 2Ly, every
                            operator runs there, and results are cropped back;
                            normal derivatives vanish on the walls.  Needs
                            nx, ny <= 1024.  The Hamiltonian is the tank's.
                            Not for closures or batches. */
};

/* Kernel kinds reported by zk_kernel_stats. */
enum {
    ZK_KERNEL_ROW_PAD = 0,   /* row pass on the 3/2-padded grid              */
    ZK_KERNEL_ROW_BASE = 1,  /* row pass of the base-grid entry/exit transforms */
    ZK_KERNEL_COL_PAD = 2,   /* column pass on the 3/2-padded grid           */
    ZK_KERNEL_COL_BASE = 3,  /* column pass of the entry/exit transforms     */
    ZK_KERNEL_REDUCE = 4     /* FP64 Parseval reduction                     */
};

/* Create a context for an nx x ny periodic grid of size Lx x Ly, still-water
 * depth `depth` (<= 0 or +inf: deep water, tanh -> 1), gravity g and HOS order
 * M (keeps G_0 .. G_{M-1}; M = 3 is the paper's "Order 3 / HOS-3", Sec. 3.2).
 * Returns NULL on invalid arguments (sizes outside the rule above, Lx, Ly or
 * g <= 0, M outside 1..8).  Host-side only: no device call is made. */
zk_ctx *zk_create(int nx, int ny, double Lx, double Ly, double depth, double g, int M);

/* Destroy a context (host memory only; the workspace stays the caller's). */
void zk_destroy(zk_ctx *ctx);

/* Set an option (keys above).  EPS, TAPER and FILTER may change at any time
 * and apply from the next call; PRECISION must be set before zk_bind. */
int zk_set_option(zk_ctx *ctx, int key, double value);
/* Current value of an option (as set, or as zk_autotune left it; for
 * ZK_OPT_ROW_FFT the form the padded row passes run in at the current team
 * shape, which is STOCKHAM where the shape has no LANES form).  ZK_EINVAL
 * for an unknown key or a null pointer. */
int zk_get_option(const zk_ctx *ctx, int key, double *value);

/* Bytes of device workspace the context needs for its current options. */
size_t zk_workspace_bytes(const zk_ctx *ctx);

/* Bind a caller-owned device workspace (>= zk_workspace_bytes, 256-byte
 * aligned) and a HIP stream (hipStream_t passed as void*, NULL = default
 * stream).  Uploads the context's tables and schedules into the workspace
 * with copies on that stream.  May be called again to rebind. */
int zk_bind(zk_ctx *ctx, void *workspace, size_t bytes, void *stream);

/* G_psi = G^[M](eta) psi = sum_{j<M} eps^j G_j(eta) psi on the base grid:
 * the forward DNO map v = G(eta) psi (Sec. 3.5, eq:v_forward). */
int zk_dtn(zk_ctx *ctx, const double *eta, const double *psi, double *G_psi);

/* Inverse DNO map (Sec. 3.5, eq:psi_inverse): psi from the pair (eta, v),
 * v = G^[M](eta) psi, by the fixed-point iteration
 *   psi <- G0^{-1} (v - (G^[M](eta) - G0) psi),  seeded with psi = G0^{-1} v,
 * iters iterations (the paper uses eight).  G0^{-1} is 1/G0 off k = 0 and 0
 * at k = 0, so psi comes out with zero mean.  The iteration contracts when
 * |k| |eta| is small across the band. */
int zk_inverse_dtn(zk_ctx *ctx, const double *eta, const double *v, double *psi, int iters);

/* Bulk velocity at depth layers (Alg. ComputeVolumeVelFrom2D; eq:phi1,
 * eq:Ci, eq:Si, eq:CiSi_stable, eq:ui, eq:vi, eq:wi) from the surface state.
 * The first-order potential on the flat plane z = 0,
 *   Phi|0 = psi - eps P(eta, G0 psi),
 * is multiplied by the coupling taper prod_a exp(-(|k_a| / (kNyq_a / 2))^8)
 * and lifted to each depth y_i (measured downward from z = 0) with
 *   C_i = cosh(|k| (h - y_i)) / cosh(|k| h),  S_i = |k| sinh(|k| (h - y_i)) / cosh(|k| h)
 * (deep water: exp(-|k| y_i), |k| exp(-|k| y_i); C = 1, S = 0 at k = 0),
 * evaluated in exponential form without overflow.
 *   eta, psi : device, [ny][nx] row-major doubles (the context's grid)
 *   ys       : host, nlayers depths, each in [0, h] (>= 0 in deep water)
 *   uvw      : device, [nlayers][3][ny][nx]: per layer u = d_x Phi (x velocity),
 *              v = S_i Phi|0 (vertical velocity), w = d_y Phi (y velocity)
 * 1 <= nlayers <= 4096.  With reflecting walls the fields are the tank's and
 * the lift runs on the even extension.  Returns ZK_EINVAL for bad pointers,
 * counts or depths (nothing is launched then). */
int zk_depth_velocity(zk_ctx *ctx, const double *eta, const double *psi, int nlayers, const double *ys, double *uvw);

/* Zakharov right-hand side (Sec. 3.1 eq:zakharov_kin; Sec. 3.2
 * eq:dyn_truncated with eq:W):
 *   eta_t = G^[M](eta) psi,
 *   psi_t = -g eta + eps [ -1/2 |grad psi|^2 + 1/2 (1 + eps^2 |grad eta|^2) W^2 ],
 *   W = (G^[M] psi + eps grad eta . grad psi) / (1 + eps^2 |grad eta|^2). */
int zk_rhs(zk_ctx *ctx, const double *eta, const double *psi, double *eta_t, double *psi_t);

/* Advance (eta, psi) in place by nsteps steps of size dt of the selected
 * integrator (classical RK4 by default, ZK_OPT_INTEGRATOR), each followed by
 * the state filter A(k) when ZK_OPT_FILTER is on (Sec. 3.4,
 * eq:state_filter).  The state is kept spectral inside the call and
 * transformed in and out once.  Returns ZK_EDIVERGED if the result holds a
 * NaN or Inf (that check synchronises the stream). */
int zk_step(zk_ctx *ctx, double *eta, double *psi, double dt, int nsteps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): zk_step
 * with the workspace taken from a fixed device array inside the library,
 * ZK_STATIC_WS_BYTES (64 MiB) per GPU, held from its first use until the
 * process ends, instead of a bound caller workspace.  ctx needs zk_create
 * (and any zk_set_option) but no zk_bind; eta, psi, dt and nsteps are as in
 * zk_step; stream is the HIP stream to run on (NULL: the null stream).
 * Returns ZK_ENOWS, with the sizes in zk_last_error, when
 * zk_workspace_bytes(ctx) exceeds ZK_STATIC_WS_BYTES (FP64: up to about
 * 256 x 256 at M = 6).  Every call re-uploads the context's tables and
 * schedules into the array (it keeps the last call's contents, which no
 * kernel reads before writing), synchronising the stream for that upload;
 * no call allocates device memory.  All calls on one GPU share the array:
 * calls that overlap in time on one GPU (other threads, other streams) race.
 * A context bound with zk_bind keeps that binding for its other calls.
 * Kernel statistics (ZK_OPT_PROFILE) are not recorded inside this call. */
#define ZK_STATIC_WS_BYTES (64u << 20)
int zk_step_static(zk_ctx *ctx, double *eta, double *psi, double dt, int nsteps, void *stream);

/* Hamiltonian H = 1/2 int psi G^[M](eta) psi dx + 1/2 g int eta^2 dx
 * (Sec. 3.1, eq:hamiltonian), reduced in FP64 in a fixed order by Parseval on
 * the half spectrum.  Synchronises the stream; writes the value to *H_host. */
int zk_hamiltonian(zk_ctx *ctx, const double *eta, const double *psi, double *H_host);

/* Diagnostic, for measurement: totals accumulated while ZK_OPT_PROFILE is on
 * for one kernel kind -- summed event time in ms, algorithmic bytes (every
 * field a launch reads or writes counted once), FFT flops (5 N log2 N per
 * complex transform of length N) and the launch count.  Synchronises the
 * stream to read pending events.  kind = -1 resets all totals (outputs may
 * then be NULL). */
int zk_kernel_stats(zk_ctx *ctx, int kind, double *ms, double *bytes, double *flops, long long *launches);

/* Autotuner: for each pass kind (row / column, padded / base transform),
 * time every compiled team shape (T threads per transform, first-pass radix
 * E = N / T, T a power of two in [16, 1024]) on the passes of one RK4 step of this
 * context (reps timed repetitions each; the context's internal spectra are
 * overwritten, no caller field is touched) and keep the fastest for later
 * calls.  Results are identical up to FP64 (or FP32) rounding order.
 * Synchronises. */
int zk_autotune(zk_ctx *ctx, double dt, int reps);

/* Team shape in use for a pass kind (row != 0: row pass; pad != 0: padded
 * transform). */
int zk_team_shape(const zk_ctx *ctx, int row, int pad, int *T, int *E);

/* Choose the team shape of a pass kind by hand (the autotuner's setting):
 * T threads per transform, first-pass radix E = N / T for the pass's
 * transform length N (3n/2 padded, n base).  T = 0 restores the default.
 * ZK_EINVAL if T does not divide N into a compiled shape (T a power of two
 * in [16, 1024]; power-of-two axes: E in {3, 6, 12} padded or {2, 4, 8} base;
 * axes of 3 2^k points: E = 9 padded, 6 base; and the pair built for the
 * context's precision).  Host only; applies from the next call. */
int zk_set_team_shape(zk_ctx *ctx, int row, int pad, int T);

/* Text of the last error on this context ("" if none).  Valid until the next
 * call on the context. */
const char *zk_last_error(const zk_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Learned closure network.
 *
 * A reduced-order DtN (the paper's Order-2 model, Sec. 3.2, is its cheapest
 * truncation; every further order adds a comparable cost, Sec. 8) plus a
 * small convolutional network that predicts the missing part
 * r = (G^[6] - G^[2]) psi from eta, psi and G^[2] psi on the grid.  The
 * network: four 3 x 3 convolutions with circular padding, 3 -> 32 -> 32 -> 32
 * -> 1 channels, exact-erf GELU after the first three; bf16 weights and
 * activations, FP32 accumulation (layers 2 and 3 on the matrix cores);
 * FP32 master weights trained with Adam (beta1 0.9, beta2 0.999, eps 1e-8)
 * on a masked mean-squared error.
 *
 * Parameter vector (ZK_CNN_NPARAMS floats, host memory): W1 b1 W2 b2 W3 b3
 * W4 b4 with W of shape (C_out, C_in, 3, 3) in C order; convolution is
 * cross-correlation, y[o](i, j) = b[o] + sum W[o][c][u][v] x[c](i+u-1, j+v-1)
 * with indices taken modulo the tile.
 *
 * Samples (device, float): [B][4][H][W], planes 0..2 the input channels,
 * plane 3 the target (ignored by zk_cnn_forward).  Outputs y (device,
 * float): [B][H][W].  Tiles need W % 32 == 0 (W % 64 == 0 for training),
 * H >= 3 and B*H*W <= max_pixels.  The network owns no device memory: the
 * caller binds one workspace, as for zk_ctx; every call is asynchronous on
 * the bound stream unless it returns host data.
 * ------------------------------------------------------------------------- */
typedef struct zk_cnn zk_cnn;
#define ZK_CNN_NPARAMS 19681

/* Network able to run tiles of up to max_pixels pixels (B*H*W).  NULL if
 * max_pixels is outside [96, 2^28].  Host-side only. */
zk_cnn *zk_cnn_create(long long max_pixels);
void zk_cnn_destroy(zk_cnn *net);
size_t zk_cnn_workspace_bytes(const zk_cnn *net);
/* Bind a caller-owned device workspace (256-byte aligned) and a stream. */
int zk_cnn_bind(zk_cnn *net, void *workspace, size_t bytes, void *stream);
/* Load FP32 parameters from host memory and reset the Adam moments
 * (synchronises the stream). */
int zk_cnn_set_params(zk_cnn *net, const float *params_host);
/* Copy the current FP32 parameters to host memory (synchronises). */
int zk_cnn_get_params(zk_cnn *net, float *params_host);
/* y = network(samples planes 0..2). */
int zk_cnn_forward(zk_cnn *net, const float *samples, float *y, int B, int H, int W);
/* Loss (mean of (y - target)^2 over the pixels at least `halo` from every
 * tile edge) and its gradient with respect to every parameter, written to
 * host memory (ZK_CNN_NPARAMS floats).  With halo >= 4 the circular padding
 * never reaches a pixel that influences the loss, so a crop trains as a
 * valid convolution.  Synchronises. */
int zk_cnn_gradient(zk_cnn *net, const float *samples, int B, int H, int W, int halo, double *loss_host,
                    float *grad_host);
/* One Adam step on the masked loss with learning rate lr.  loss_host may be
 * NULL (then the call stays asynchronous). */
int zk_cnn_train_step(zk_cnn *net, const float *samples, int B, int H, int W, int halo, double lr,
                      double *loss_host);
const char *zk_cnn_last_error(const zk_cnn *net);

/* ---------------------------------------------------------------------------
 * Learned-closure stepper.
 *
 * Steps (eta, psi) with classical RK4 on the grid, where every stage uses
 *   G = P_B( G^[low] psi + r ),  r = out_scale * s * net(x),
 *   x = ( k0 eta / eta_scale,  k0 psi / s,  G^[low] psi / s ),  s = rms(G^[low] psi),
 * in place of G^[M] in the Zakharov RHS (Sec. 3.1 eq:zakharov_kin, Sec. 3.2
 * eq:dyn_truncated with eq:W), P_B the projection onto the band (Nyquist
 * modes removed), then the state filter A(k) (Sec. 3.4).  The residual is
 * linear in psi for fixed eta, as the DtN operator is; the psi-scale s makes
 * the network see that exactly.  The full-order context is the closure's
 * fallback and the reference for its error: an audit at the first step and every
 * audit_every steps computes e = ||G_closure - G^[full] psi||_2 /
 * ||G^[full] psi||_2 on the current state; while e > tol the next
 * audit_every steps are taken by the full-order context (zk_step), else by
 * the closure.  low, full and net must be bound to one stream and keep their
 * binding while the closure is used; full may be NULL when no audit is asked
 * for (audit_every = 0).  The grid must have nx % 32 == 0 and nx * ny <= the
 * network's max_pixels.  Workspace: caller-owned, as for zk_ctx.
 * ------------------------------------------------------------------------- */
typedef struct zk_closure zk_closure;

/* NULL if an argument is invalid (contexts of different grids, full order not
 * above low order, network too small, non-positive scales).  Host-only. */
zk_closure *zk_closure_create(zk_ctx *low, zk_ctx *full, zk_cnn *net, double k0, double eta_scale,
                              double out_scale);
void zk_closure_destroy(zk_closure *clo);
size_t zk_closure_workspace_bytes(const zk_closure *clo);
/* Bind a workspace; the stream is the one the contexts and the network share. */
int zk_closure_bind(zk_closure *clo, void *workspace, size_t bytes);
/* G = P_B(G^[low] psi + r) on the grid (the closure's DtN). */
int zk_closure_dtn(zk_closure *clo, const double *eta, const double *psi, double *G);
/* One training sample for the network from a state: samples (device float
 * [4][ny][nx]) = the three input planes x above and the target
 * (G^[full] psi - G^[low] psi) / (out_scale * s).  Needs the full context. */
int zk_closure_features(zk_closure *clo, const double *eta, const double *psi, float *samples);
/* Periodic crops of a [4][ny][nx] sample: dst[k] = planes at rows
 * offsets[2k] + (0..h-1) and columns offsets[2k+1] + (0..w-1), indices taken
 * modulo the grid; dst is device float [ncrop][4][h][w].  ncrop <= 4096;
 * offsets (host) in [0, ny) x [0, nx).  Synchronises. */
int zk_closure_crops(zk_closure *clo, const float *samples, const int *offsets_host, int ncrop, int h, int w,
                     float *dst);
/* Advance (eta, psi) in place by nsteps RK4 steps of size dt with audits and
 * fallback as described above (audit_every = 0: closure only, no audit).
 * Audits synchronise the stream. */
int zk_closure_step(zk_closure *clo, double *eta, double *psi, double dt, int nsteps, int audit_every,
                    double tol);
/* Counters since creation: steps taken by the closure and by the fallback,
 * audits, the last and the largest audited error.  Any output may be NULL. */
int zk_closure_stats(const zk_closure *clo, long long *closure_steps, long long *fallback_steps,
                     long long *audits, double *last_err, double *max_err);
const char *zk_closure_last_error(const zk_closure *clo);

/* ---------------------------------------------------------------------------
 * Batches of independent tiles.
 *
 * Many periodic tiles of different sizes, depths and orders M advanced
 * together by the same RK4 + filter step as zk_step (each tile's result is
 * that of its own context).  Each tile keeps its own spectra in a slice of
 * the batch workspace; the tiles' passes are merged into phases, one
 * batched launch per phase and tile size (blockIdx.y runs over the tiles'
 * programs or tasks), and one step's phases are replayed as a HIP graph of
 * kernel nodes.  The team shape of each pass and size (threads per
 * transform and first-pass radix) is the default one (the smallest radix,
 * as for a context) until zk_batch_autotune times the compiled alternatives on the
 * batch itself and keeps the fastest.  Tile sizes follow zk_create's rule.
 * ------------------------------------------------------------------------- */
typedef struct zk_tile {
    int nx, ny;           /* grid points (as zk_create)                     */
    double Lx, Ly, depth; /* domain size and still-water depth (<= 0: deep) */
    int M;                /* HOS order, 1..8                               */
} zk_tile;
typedef struct zk_batch zk_batch;

enum {
    ZK_BATCH_OPT_GRAPH = 1,      /* 1: replay each step as a HIP graph (default);
                                    0: launch the phases one by one           */
    ZK_BATCH_OPT_PERSISTENT = 2  /* 1: each step is one persistent launch: its
                                    workers take (tile, pass, item, block
                                    chunk) units in phase order from a device
                                    queue and wait on per-tile completion
                                    counters (bounded waits: one that runs out
                                    makes zk_batch_step return ZK_EDEVICE, and
                                    the call synchronises to read that flag).
                                    Tiles of 128 to 1024 points per axis only,
                                    transforms with the smallest first-pass
                                    radix.  0 (default): as ZK_BATCH_OPT_GRAPH */
};

/* precision: 64 (FP64 transforms) or 32 (FP32 transforms, FP64 series,
 * state and symbols), as ZK_OPT_PRECISION.  NULL on invalid tiles or
 * arguments.  Host-only. */
zk_batch *zk_batch_create(int ntiles, const zk_tile *tiles, double g, int precision);
void zk_batch_destroy(zk_batch *batch);
size_t zk_batch_workspace_bytes(const zk_batch *batch);
/* Bind a caller-owned workspace (256-byte aligned) and a stream; uploads
 * every tile's tables (synchronises). */
int zk_batch_bind(zk_batch *batch, void *workspace, size_t bytes, void *stream);
/* Register the tiles' fields: host arrays of ntiles device pointers to
 * [ny][nx] doubles, stepped in place; they must stay valid while used. */
int zk_batch_set_fields(zk_batch *batch, double *const *eta, double *const *psi);
int zk_batch_set_option(zk_batch *batch, int key, double value);
/* Advance every tile by nsteps RK4 steps of size dt (each followed by the
 * state filter).  Asynchronous on the bound stream; the first call for a dt
 * builds the merged schedule and the graphs (synchronises). */
int zk_batch_step(zk_batch *batch, double dt, int nsteps);
/* Time every compiled team shape of every pass and tile size on one step of
 * this batch (reps timed repetitions each; the tiles' internal spectra are
 * overwritten, the registered fields are not) and keep the fastest.
 * Synchronises. */
int zk_batch_autotune(zk_batch *batch, double dt, int reps);
/* Entry `index` of the autotuner's choices: pass kind (row 1 / column 0),
 * padded (1) or base (0) transform, transform length and the team shape
 * (T threads, first-pass radix E).  ZK_EINVAL past the last entry. */
int zk_batch_tuning(const zk_batch *batch, int index, int *row, int *pad, int *n_transform, int *T, int *E);
/* Phases and batched launches of one step (after the schedule is built). */
int zk_batch_stats(const zk_batch *batch, long long *phases_per_step, long long *launches_per_step);
const char *zk_batch_last_error(const zk_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* ZK_H */
