/*
 * adl.h -- C ABI of the MI355X (gfx950) Leja exponential integrator for 2D
 * anisotropic diffusion with advection and sources.
 *
 * Method: Deka, Kissmann, Einkemmer, "Efficient numerical methods for
 * anisotropic diffusion of Galactic cosmic rays" (ICRC 2023).
 *   - problem:   u_t = div(D grad u) + div(a u) + S(x, y, t)         Sec. 1, eq. 2
 *   - operator:  A = div(D grad .) + div(a .)                        Sec. 2 (below eq. 3)
 *   - rules:     exponential quadrature, midpoint and two-stage      Sec. 2, eq. 3-5
 *   - phi_l:     phi_0 = exp, phi_{l+1}(z) = (phi_l(z) - 1/l!)/z      Sec. 2
 *   - Leja:      Newton interpolation of phi_l((c + gamma xi) dt) at  Sec. 2
 *                Leja points xi in [-2, 2], c = alpha/2, gamma = -alpha/4,
 *                alpha from Gershgorin's theorem (or power iteration)
 *
 * Conventions shared by every entry point
 *   - Grids are nx * ny nodes, arrays row-major [ny][nx] (index j*nx + i, i
 *     along x, contiguous).  Every vector and field pointer is DEVICE memory
 *     (HIP, gfx950) unless a comment says host.
 *   - Spatial discretisation (the paper gives none): conservative second-order
 *     central nine-point stencil with face averages of Dxx, Dyy and the mixed
 *     terms d/dx(Dxy du/dy) + d/dy(Dxy du/dx); central differences for
 *     div(a u).  bc = ADL_BC_PERIODIC wraps; ADL_BC_DIRICHLET sets u = 0
 *     outside the interior nodes (a boundary face takes the interior node's
 *     coefficient).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     on it.  Calls that return host values (alpha, iterations, adl_stats)
 *     synchronise that stream before returning.
 *   - Vectors u, S, v, out are FP64 at the boundary in every storage mode.
 *   - The caller owns every device buffer (fields, vectors, workspace); the
 *     library owns only the opaque handles.  Fields are copied (and scaled,
 *     and in FP32 modes rounded) into the workspace by adl_op_create, so the
 *     caller may free them afterwards.
 *   - Steps are transactional: u is written only when the call returns
 *     ADL_OK.  On any error u is unchanged.
 *   - Return value: ADL_OK (0) or a negative ADL_E* code; adl_last_error()
 *     then returns a thread-local message.  No C++ exception crosses the ABI.
 *   - Calls on the same op are not thread-safe; separate ops are independent.
 */
#ifndef ADL_H
#define ADL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ADL_OK = 0,
  ADL_EINVAL = -1,       /* invalid argument (sizes, spacing, tol, dt, c1 == c2, ...) */
  ADL_ENOCONV = -2,      /* a Leja sweep hit the degree cap after all substep doublings */
  ADL_EBOUND = -3,       /* no usable spectral interval (alpha >= 0 or not finite) */
  ADL_ENAN = -4,         /* NaN / Inf met in a sweep (input or overflow) */
  ADL_EHIP = -5,         /* a HIP runtime call failed */
  ADL_ENOWORKSPACE = -6  /* workspace missing, misaligned or too small */
};

enum { ADL_BC_PERIODIC = 0, ADL_BC_DIRICHLET = 1 };

/* Storage of the operator.  Newton polynomial p, divided differences, norms
 * and all boundary vectors stay FP64 in every mode. */
enum {
  ADL_STORAGE_FP64 = 0,         /* fields and Newton vectors y_k in FP64 */
  ADL_STORAGE_FP32_FIELDS = 1,  /* fields FP32, y_k FP64 */
  ADL_STORAGE_FP32_FIELDS_Y = 2 /* fields FP32, y_k FP32 */
};

enum { ADL_BOUND_GERSHGORIN = 0, ADL_BOUND_POWER = 1 };

/* quad2 evaluation of phi_1 w1 + phi_2 w2 */
enum { ADL_QUAD2_AUGMENTED = 0, ADL_QUAD2_TWO_SWEEP = 1 };

typedef struct adl_op adl_op;
typedef struct adl_batch adl_batch;

/* Per-call statistics (host struct, filled on return when non-NULL). */
typedef struct adl_stats {
  int matvecs;      /* applications of A, the paper's cost unit (Sec. 3) */
  int sweeps;       /* Leja interpolation sweeps */
  int max_degree;   /* largest sweep degree (Newton terms) */
  int last_degree;  /* degree of the last sweep */
  int substeps;     /* substeps K of the last phi evaluation (0: zero operator) */
  int fallback;     /* 1 when a learned bound was replaced by power iteration */
  int status;       /* same value as the return code */
  int reserved_i;
  double alpha;     /* interval end used (alpha < 0) */
  double reserved[3];
} adl_stats;

/* ------------------------------------------------------------------------
 * Operator
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace an op of this size needs (256-byte aligned
 * start required).  max_degree <= 0 means the default (500). */
size_t adl_workspace_bytes(int nx, int ny, int storage, int max_degree);

/* Create the operator A of eq. 2 (Sec. 1) on an nx * ny grid.
 *   hx, hy   grid spacings (> 0); nx, ny >= 3
 *   bc       ADL_BC_PERIODIC or ADL_BC_DIRICHLET
 *   storage  ADL_STORAGE_*
 *   Dxx, Dxy, Dyy  device [ny][nx] FP64 tensor fields (Dyx = Dxy)
 *   ax, ay   device [ny][nx] FP64 advection fields, or both NULL to use the
 *            constants ax_c, ay_c
 *   workspace, ws_bytes  device buffer of >= adl_workspace_bytes(...) bytes,
 *            256-byte aligned, owned by the caller, kept alive until
 *            adl_op_destroy.
 * Returns the handle in *out. */
int adl_op_create(int nx, int ny, double hx, double hy, int bc, int storage,
                  const double* Dxx, const double* Dxy, const double* Dyy,
                  const double* ax, const double* ay, double ax_c, double ay_c,
                  void* workspace, size_t ws_bytes, void* stream, adl_op** out);

int adl_op_destroy(adl_op* op);

/* Limits of the Leja driver: max_degree = most Newton terms per sweep
 * (1 .. the value given to adl_workspace_bytes), rho_max = largest |alpha| h
 * one sweep covers (a step dt is split into K = ceil(|alpha| dt / rho_max)
 * substeps; K doubles when a sweep hits max_degree).  Defaults 500, 1600. */
int adl_op_set_limits(adl_op* op, int max_degree, double rho_max);

/* ADL_QUAD2_AUGMENTED (default) or ADL_QUAD2_TWO_SWEEP. */
int adl_op_set_quad2_mode(adl_op* op, int mode);

/* Kernel-time profiling of the Newton-Leja iteration kernel (the hot loop).
 * With enable != 0 every productive iteration launch (not the no-op launches
 * enqueued past the stopping index) is timed with HIP events attached to its
 * dispatch.  adl_op_profile_read returns the summed kernel time in ms, the
 * number of timed launches and the algorithmic bytes they moved (read y_k,
 * tensor and advection fields, p, w2 when present; write y_{k+1}, p), then
 * resets the counters.  adl_op_profile resets them too. */
int adl_op_profile(adl_op* op, int enable);
int adl_op_profile_read(adl_op* op, double* kernel_ms, long long* launches, double* bytes);

/* The same counters split by launch kind (read before adl_op_profile_read,
 * which resets them): ADL_LAUNCH_FIRST = the first term of a sweep (y_0 = v,
 * the augmented column), ADL_LAUNCH_ONE / _TWO / _THREE / _FOUR = launches of
 * one, two, three or four later terms.  terms (may be NULL) = Newton terms
 * those launches computed.  ADL_EINVAL for another kind. */
enum { ADL_LAUNCH_FIRST = 0, ADL_LAUNCH_ONE = 1, ADL_LAUNCH_TWO = 2, ADL_LAUNCH_FOUR = 3, ADL_LAUNCH_THREE = 4 };
int adl_op_profile_read_kind(const adl_op* op, int kind, double* kernel_ms, long long* launches,
                             double* bytes, long long* terms);

/* Tiling of the stencil kernels (the autotuner's knobs): rows = rows each
 * wave computes per tile (a block of four waves covers 4 * rows rows of one
 * strip; default 1), cols_per_lane = columns per lane (1, or 2 for even
 * nx >= 128); 0 selects the built-in default for each.  adl_op_get_tiling
 * reports the tiling in use and the worker block count of a launch (any
 * output pointer may be NULL). */
int adl_op_set_tiling(adl_op* op, int rows, int cols_per_lane);

/* Newton terms per launch of a sweep (Sec. 2 recurrence): mode = 1 (the
 * default) computes four terms per launch on grids below 2^20 points
 * (mode 4's form, y_{k+1} .. y_{k+3} kept on chip) and, from 2^20 points
 * on, three (mode 5's form: read y_k, the fields and p_k once, write y_{k+3}
 * and p_{k+3}; with FP64 Newton vectors and no augmented column among terms
 * 1 .. 3 the first launch takes three terms too, from y_0 = v, and in a
 * midpoint step without substeps on a grid of at least 2^24 points, or in
 * mode 5, it also forms the stage vector A u + S itself); where those
 * forms do not apply it computes terms k+1 and
 * k+2 in one launch, keeping y_{k+1} on chip, with the input rows staged in
 * LDS from 2^20 points on and one-row frames in registers below;
 * mode = 2 and mode = 3
 * force the two-term LDS-staged and register-frame forms; mode = 4 computes four
 * terms per launch (y_{k+1} .. y_{k+3} kept in LDS, three-row frames), on
 * grids swept without non-temporal hints and, on a periodic grid, ny >= 4
 * other than 5 and 9 (a block's rows wrap once; ADL_EINVAL otherwise; mode 1
 * then runs two terms per launch); mode = 5 computes three terms per launch
 * with the input rows staged in LDS (y_{k+1}, y_{k+2} kept in LDS), on grids
 * whose two-term tiling has two columns per lane (ADL_EINVAL otherwise);
 * mode = 6 computes four terms per launch with the input rows staged in LDS
 * (y_{k+1} .. y_{k+3} kept in LDS; nx even and at least 128, ADL_EINVAL
 * otherwise); mode = 0 launches one kernel per term.
 * A fused launch stores y and p of its last term only; when the sweep stops
 * at an earlier term of a launch, the launch is run again on its inputs to
 * store p of that term (the same arithmetic, so the same values).  Results
 * agree to rounding (the block partial sums of the norms are grouped
 * differently).  ADL_EINVAL for other values. */
int adl_op_set_term_fusion(adl_op* op, int mode);

/* Cache hints of the Newton-Leja launches: mode = 1 marks the vectors a
 * launch reads or writes exactly once (p_k, y and p of its terms) as
 * non-temporal, so that on grids far beyond the caches the rows re-read by
 * neighbouring tiles stay in L2; mode = 0 uses ordinary loads and stores;
 * mode = -1 (the default) chooses 1 when the sweep's working set (fields,
 * the input vector, three y and three p buffers) exceeds 512 MiB.  Results are
 * identical in every mode.  ADL_EINVAL for other values. */
int adl_op_set_streaming(adl_op* op, int mode);

/* How the host learns where a sweep stopped (the stopping rule of Sec. 2 is
 * evaluated on the GPU once per chunk of launches).  mode = 1 (the default):
 * the chunk's decision launch writes the outcome into a cache line of
 * coherent pinned host memory that the op holds, and the host spins on it;
 * mode = 0: the control block is copied back and the stream synchronised
 * (many microseconds more per chunk).  Without such memory, and while
 * adl_op_profile is on, mode 0 is used.  Results are identical in both modes;
 * a launch error ends the spin with ADL_EHIP.  adl_op_host_wait reports the
 * mode in effect (1 only if the op holds the memory).  ADL_EINVAL for other
 * values or a NULL mode. */
int adl_op_set_host_wait(adl_op* op, int mode);
int adl_op_host_wait(const adl_op* op, int* mode);
int adl_op_get_tiling(const adl_op* op, int* cols_per_lane, int* rows, int* nblocks);

/* y = A x (one stencil application).  x, y: device [ny][nx] FP64, not
 * overlapping. */
int adl_apply(adl_op* op, const double* x, double* y, void* stream);

/* Spectral interval end alpha < 0 (Sec. 2): ADL_BOUND_GERSHGORIN gives the
 * leftmost Gershgorin row-disc edge; ADL_BOUND_POWER runs power iteration
 * from a splitmix64(seed) start vector until |l_k - l_{k-1}| <= rtol l_k or
 * max_iter, and gives alpha = -min(1.1 l, |alpha_Gershgorin|).
 * The result is also installed as the op's bound.  iters_out may be NULL. */
int adl_spectral_bound(adl_op* op, int method, int max_iter, double rtol, uint64_t seed,
                       double* alpha_out, int* iters_out, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the Gershgorin interval end of
 * adl_spectral_bound(ADL_BOUND_GERSHGORIN) -- the same reduction and the
 * same value as on an FP64 op of these fields -- computed from the caller's
 * unscaled device fields (Dxx, Dxy, Dyy [ny][nx] FP64; ax, ay fields or both
 * NULL for the constants ax_c, ay_c; grid and bc as for adl_op_create) with
 * no op, no workspace and no allocation.  alpha_out: device, one double,
 * written on `stream` (the call enqueues two kernels and returns without
 * synchronising).  The reduction's scratch (block partials and a counter,
 * 8.4 KB) is a static device array of the library, one per GPU, kept until
 * the process ends; every call on a GPU shares it, so calls that overlap on
 * one GPU (different streams, no ordering) race.  At most 1024 reduction
 * blocks, i.e. grids of up to 2^31 points (ADL_EINVAL beyond). */
int adl_gershgorin_bound_noalloc(int nx, int ny, double hx, double hy, int bc, const double* Dxx,
                                 const double* Dxy, const double* Dyy, const double* ax, const double* ay,
                                 double ax_c, double ay_c, double* alpha_out, void* stream);

/* The raw estimate lambda (before the safety factor and the Gershgorin cap)
 * of the op's last power iteration; ADL_EBOUND if none has run. */
int adl_last_power_estimate(const adl_op* op, double* lambda);

/* Install an interval end directly (alpha < 0 and finite, else ADL_EBOUND),
 * e.g. from the learned predictor.  alpha == 0 is accepted only for an
 * operator whose Gershgorin bound is 0 (A = 0). */
int adl_set_bound(adl_op* op, double alpha);
int adl_get_bound(const adl_op* op, double* alpha);

/* out = phi_l(A dt) v, l in {0, 1, 2}, by Leja interpolation (Sec. 2).
 * tol in (0, 1) is the stopping threshold ||d_m y_m|| <= tol ||p_m||;
 * max_degree <= 0 uses the op's limit.  v == 0 gives out = 0 with degree 0.
 * out may not alias v.  Needs a bound (adl_spectral_bound / adl_set_bound). */
int adl_leja_phi(adl_op* op, int l, double dt, const double* v, double* out,
                 double tol, int max_degree, adl_stats* st, void* stream);

/* Exponential midpoint rule, eq. 4:
 *   u <- u + dt phi_1(A dt) (A u + S(t^n + dt/2)).
 * S_half may be NULL (no source). */
int adl_exp_midpoint_step(adl_op* op, double* u, const double* S_half, double dt,
                          double tol, adl_stats* st, void* stream);

/* Two-stage exponential quadrature, eq. 3 with s = 2 (eq. 5 for Gauss
 * nodes c = (1 -+ 1/sqrt 3)/2):
 *   u <- u + dt [phi_1(A dt) w1 + phi_2(A dt) w2],
 *   w1 = A u + (c2 S1 - c1 S2)/(c2 - c1),  w2 = (S2 - S1)/(c2 - c1),
 * S_i = S(t^n + c_i dt), either may be NULL (zero).  c1 != c2.  The phi sum is
 * one augmented-matrix sweep (Sec. 2) unless the op's quad2 mode says two. */
int adl_exp_quad2_step(adl_op* op, double* u, const double* S1, const double* S2,
                       double c1, double c2, double dt, double tol, adl_stats* st,
                       void* stream);

/* ------------------------------------------------------------------------
 * Batched momentum bins: independent operators (different grids, different
 * intervals) advanced together.  Each kernel of a step covers the tiles of
 * all bins (stage, one launch per Leja term, final decision); the step's
 * launches are captured once in a hipGraph and replayed, one graph launch
 * per step.  Bins needing substeps, a zero operator or more terms than the
 * batch allows are advanced by the single-op path inside the same call.
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace for a batch over these ops. */
size_t adl_batch_workspace_bytes(int nbins, adl_op* const* ops, int max_degree);

/* ops: host array of nbins op handles (each with a bound installed before
 * the first step); they must outlive the batch.  workspace: device,
 * 256-byte aligned, >= adl_batch_workspace_bytes.  tile_rows <= 0 picks the
 * autotuned / default tile height. */
int adl_batch_create(int nbins, adl_op* const* ops, void* workspace, size_t ws_bytes,
                     int tile_rows, adl_batch** out);
int adl_batch_destroy(adl_batch* b);

/* Tile height (rows per wave, >= 1) of the batch kernels. */
int adl_batch_set_tile_rows(adl_batch* b, int rows);
int adl_batch_get_tile_rows(const adl_batch* b, int* rows);

/* Newton terms per launch of the batched sweep (Sec. 2 recurrence): mode = 3
 * (the default when every bin has nx even and >= 128) computes terms k+1 ..
 * k+3 of every running bin in one launch, the first three included, blocks
 * of four waves marching runs of 4 * tile_rows rows of a strip of one bin
 * with the input rows staged in LDS (a launch stores y of its last two terms,
 * the second-to-last in FP32, and p of the last; a bin that stops at an
 * earlier term is advanced by p_m rebuilt from them); mode = 1 (the default
 * otherwise) computes terms k+1 and k+2 in one launch after a launch of the
 * first term alone (one wave per tile marches down its rows with y_{k+1} in
 * registers); mode = 0 launches one kernel per term.  ADL_EINVAL for other
 * values, and for mode 3 when a bin is narrower or odd. */
int adl_batch_set_term_fusion(adl_batch* batch, int mode);

/* Autotuner: times the launches of one step (stage and sweep; u is not
 * modified) for each of the ncand candidate tile heights (host array) and
 * installs the fastest; best_rows / best_ms (host, may be NULL) receive it.
 * Results are cached for the life of the process by (GPU architecture,
 * storage and advection kind, columns per lane, terms per launch, the
 * candidates, the bins' grid shapes): a later call with the same key, on
 * this batch or another, installs the cached height and its time without
 * timing again. */
int adl_batch_autotune(adl_batch* b, double* const* u, const double* const* S_half, double dt,
                       double tol, const int* candidates, int ncand, int* best_rows,
                       double* best_ms, void* stream);

/* One exponential midpoint step (eq. 4) of every bin with a shared dt:
 *   u_b <- u_b + dt phi_1(A_b dt)(A_b u_b + S_b).
 * u, S_half: host arrays of nbins device pointers (16-byte aligned; S_half or
 * its entries may be NULL).  per_bin: host array of nbins adl_stats or NULL.
 * use_graph = 1 captures the step's launches in a hipGraph on first use and
 * replays it while the pointers, dt and tol are unchanged.  Each bin's u is
 * written only when its step succeeds; the first failing bin's code is
 * returned (ADL_ENOCONV, ADL_ENAN, ...). */
int adl_batch_midpoint_step(adl_batch* b, double* const* u, const double* const* S_half,
                            double dt, double tol, int use_graph, adl_stats* per_bin,
                            void* stream);

/* ------------------------------------------------------------------------
 * Learned bound: field statistics and the 9-64-64-64-3 tanh MLP (FP32).
 * Packed parameters: for each layer W_l [in][out] row-major then b_l[out].
 * ---------------------------------------------------------------------- */

#define ADL_MLP_PARAMS 9155
#define ADL_MLP_IN 9
#define ADL_MLP_OUT 3
#define ADL_MLP_CACHE_PER_ROW 201 /* X 9 | H1 64 | H2 64 | H3 64 */

/* feats (device, 9 FP32): log10 max k_par, log10 mean k_par,
 * log10 max k_perp', log10 mean k_perp' (k_perp' = max(k_perp,0) + 1e-30),
 * max |a|, mean |a|, log10 hx, log10 hy, log10 dt, where k_par >= k_perp are
 * the eigenvalues of the op's tensor at each node (stored fields). */
int adl_field_stats(adl_op* op, double dt, float* feats, void* stream);

/* Y[B][3] = MLP(X[B][9]).  act_cache (device, B*201 floats) receives the
 * activations when non-NULL (needed by adl_mlp_backward). */
int adl_mlp_forward(const float* W, const float* X, float* Y, float* act_cache, int B,
                    void* stream);

/* dW (device, ADL_MLP_PARAMS floats) = dL/dW given dY = dL/dY [B][3] and the
 * cache of the matching forward call.  dW is overwritten. */
int adl_mlp_backward(const float* W, const float* act_cache, const float* dY, float* dW,
                     int B, void* stream);

/* Mean squared error of a batch: loss (device, 1 float, may be NULL) =
 * mean((Y - T)^2) over B x 3, dY = 2 (Y - T) / (3 B) (device [B][3]). */
int adl_mlp_mse_grad(const float* Y, const float* T, float* dY, float* loss, int B, void* stream);

/* One Adam update of W (device) with moments m1, m2 (device, zero at t = 1),
 * step t >= 1. */
int adl_mlp_adam_step(float* W, const float* dW, float* m1, float* m2, int t, float lr,
                      float beta1, float beta2, float eps, void* stream);

/* ------------------------------------------------------------------------
 * Host-side helpers (no GPU needed)
 * ---------------------------------------------------------------------- */

/* First n (<= 501) Leja points on [-2, 2] (Sec. 2) into host array out:
 * xi_0 = 2, then xi_k maximises prod_{j<k} |x - xi_j| on [-2, 2]; ties go to
 * the smaller point.  Returns ADL_EINVAL for n outside [1, 501]. */
int adl_leja_points(int n, double* out);

/* Newton coefficients d_0..d_{n-1} (host array out) of the interpolant of
 * phi_l((c + gamma xi) h) at the Leja points, c = alpha/2, gamma = -alpha/4
 * (Sec. 2: divided differences), l in {0,1,2}, alpha < 0, h > 0. */
int adl_newton_coefficients(int l, double alpha, double h, int n, double* out);

/* ------------------------------------------------------------------------
 * Learned spectral interval.  The predictor maps dimensionless inputs built
 * from the raw statistics f (adl_field_stats) and g = |alpha_Gershgorin| to
 * dimensionless targets
 *   y0 = 10 log10(rho / g), y1 = m / sqrt(rho dt / K + 1), y2 = log2 K
 * with rho the spectral radius (power iteration), m the phi_1 Leja degree and
 * K the substeps.  Host helpers (no GPU): */
int adl_learned_features(const float* raw9, double g, float* x9);
int adl_learned_targets(const float* raw9, double g, double rho, int degree, int substeps, float* y3);
int adl_learned_decode(const float* raw9, double g, const float* y3, double* rho, int* degree,
                       int* substeps);

typedef struct adl_learned_info {
  double rho_hat;     /* predicted spectral radius */
  double alpha;       /* installed interval end -min(1.2 rho_hat, |alpha_Gershgorin|) */
  double gershgorin;
  int degree_hat;     /* predicted Leja degree */
  int substeps_hat;   /* predicted substeps */
  float feats[9], x[9], y[3];
} adl_learned_info;

/* Predict and install the op's interval for step size dt with the trained
 * network W (device, ADL_MLP_PARAMS floats): field statistics, the network's
 * forward pass and the Gershgorin cap run on the GPU.  scratch: device, >= 32
 * floats.  Power iteration stays the fallback and the arbiter: while the learned
 * interval is installed, a sweep needing more than 1.5 degree_hat + 10 terms,
 * or producing a non-finite value, makes adl_exp_midpoint_step /
 * adl_exp_quad2_step replace the interval by power iteration's and redo the
 * step (adl_stats.fallback = 1).  info (host) may be NULL. */
int adl_learned_bound(adl_op* op, double dt, const float* W, float* scratch, adl_learned_info* info,
                      void* stream);

/* adl_learned_bound for n ops (momentum bins) at once, with the same result
 * per op, bit for bit: one launch reduces every op's field statistics and
 * missing Gershgorin bound (each op's blocks as its own launch would run them),
 * one readback, and one forward pass of the network over the n feature rows,
 * so the host waits twice in all instead of two or three times per op.
 * The ops' first-step Newton coefficients are built on up to 16 host threads.
 * ops: host array of n >= 1 distinct ops (EINVAL if one appears twice), all on
 * the device of stream.  scratch:
 * device, >= 72 n floats, 16-byte aligned.  infos: host array of n, or NULL.
 * On an error the ops before the failing one keep their new interval and the
 * rest their old one. */
int adl_learned_bound_many(int n, adl_op* const* ops, double dt, const float* W, float* scratch,
                           adl_learned_info* infos, void* stream);

/* Thread-local message of the last error (never NULL). */
const char* adl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ADL_H */
