/*
 * gmco.h — C-ABI of the MI355X gMCO hot path: many HDR dwell-time plans
 * optimised at once by batched L-BFGS (Belanger, Cui et al., "A GPU-based
 * multi-criteria optimization algorithm for HDR brachytherapy",
 * arXiv 1904.01567).
 *
 * Conventions (every entry point):
 *   - Return GMCO_OK (0) on success, a negative gmco_status on error.  The
 *     text of the last error of a context is available from gmco_last_error.
 *     No C++ exception crosses this boundary.
 *   - Host arrays are row-major, 0-based and are only read (or written) during
 *     the call; the library keeps no pointer to them after it returns.
 *   - Device work is issued on the context's stream (gmco_set_stream); calls
 *     that return host data synchronise that stream before returning.
 *   - One context per host thread.  Contexts on the same GPU are independent.
 *   - Per-plan numeric trouble (a failed line search, a non-finite objective)
 *     is reported in the plan's status and never fails a whole call.
 */
#ifndef GMCO_H
#define GMCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GMCO_MAX_GROUPS 8   /* structures (organs / point types) per case */
#define GMCO_MAX_HISTORY 32 /* L-BFGS pairs */
#define GMCO_MAX_DWELLS 512 /* active dwell positions per case */

typedef enum {
  GMCO_OK = 0,
  GMCO_EINVAL = -1,   /* bad argument: shape, range, NaN/Inf or negative weight */
  GMCO_ENOMEM = -2,   /* device allocation failed or bound workspace too small */
  GMCO_EHIP = -3,     /* a HIP runtime call failed; its text is in last_error */
  GMCO_ESTATE = -4,   /* wrong call order (e.g. optimise before set_weights) */
  GMCO_ENUMERIC = -5, /* every plan of the batch has a non-finite objective */
  GMCO_ENOLIB = -6    /* no usable GPU of the architecture this library is built for */
} gmco_status;

/* Arithmetic of the dose product (eq. (dose)) and of the back-projection of
 * the penalty derivative inside each evaluation.  L-BFGS vectors and history
 * are FP32 in every case; F_64 and the DVH metrics are FP64.
 *   F32        FP32 operands, FP32 accumulation in both products.
 *   BF16       BF16 operands, FP32 accumulation.
 *   FP8        OCP e4m3 operands with one scale per dwell column, FP32 accumulation.
 *   F32_ACC64  FP32 operands; the dose accumulated and the penalty evaluated
 *              in FP64 (FP32 accumulation of the dose leaves noise in the
 *              objective that stalls the line search near the optimum);
 *              FP32 back-projection.
 *   F32_CHUNK64 FP32 matrix ops sum 16 dwells at a time; these partial doses
 *              are accumulated and the penalty evaluated in FP64; FP32
 *              back-projection.  Near F32 speed, objective noise far below
 *              the FP32 mode's. */
typedef enum {
  GMCO_DTYPE_F32 = 0,
  GMCO_DTYPE_BF16 = 1,
  GMCO_DTYPE_FP8 = 2,
  GMCO_DTYPE_F32_ACC64 = 3,
  GMCO_DTYPE_F32_CHUNK64 = 4
} gmco_dtype;

/* Per-plan status. */
typedef enum {
  GMCO_PLAN_RUNNING = 0,   /* still iterating (only seen mid-run) */
  GMCO_PLAN_CONVERGED = 1, /* relative objective variation <= eps, F == 0 or g == 0 */
  GMCO_PLAN_MAXITER = 2,   /* reached max_iter accepted steps */
  GMCO_PLAN_LS_FAIL = 3,   /* max_ls trials rejected; x kept at the last accepted point */
  GMCO_PLAN_NONFINITE = 4, /* objective at the start point is NaN or Inf */
  GMCO_PLAN_INACTIVE = 5   /* slot not used by the current weight batch */
} gmco_plan_status;

typedef struct gmco_ctx gmco_ctx;

typedef struct {
  int device;    /* HIP device ordinal */
  int dtype;     /* gmco_dtype */
  int history;   /* L-BFGS pairs m, 1..GMCO_MAX_HISTORY */
  int max_plans; /* largest weight batch that set_weights will receive */
} gmco_opts;

/* One patient case (Sec. 2.1).  Points may be given in any order; group[i]
 * names the row of eq. 1 parameters of point i.  Groups belong to organs
 * (structures): eq. (obj) gives each organ one hidden weight w_j and one
 * point count N_pnt,j, shared by its groups, e.g. the surface and the volume
 * points of Table 1 (8 groups, 4 organs).  Without group_organ every group is
 * an organ of its own.  Metrics (V100, V75, D10, D90, individual objectives)
 * are per organ.  The DVH metrics use the optional DVH point set when given
 * (Sec. 2.1.1 counts separate, denser DVH points), else the optimisation
 * points; F and the individual objectives always use the optimisation points. */
typedef struct {
  int n_dwells;                  /* K, 1..GMCO_MAX_DWELLS */
  const double* dwell_xyz;       /* K x 3, cm */
  int n_points;                  /* M >= 1 */
  const double* point_xyz;       /* M x 3, cm (ignored when dose_rate != NULL) */
  const int32_t* group;          /* M, values in [0, n_groups) */
  int n_groups;                  /* 1..GMCO_MAX_GROUPS */
  const double* group_params;    /* n_groups x 4: w_min, D_min [Gy], D_max [Gy], w_max (eq. 1) */
  const double* group_volume_cc; /* n_organs structure volumes for V75 in cc; NULL -> 0 cc */
  double prescription_gy;        /* > 0; 100 % for V100 / D_x */
  int target_group;              /* organ whose mean dose sets the default start */
  const double* dose_rate;       /* optional M x K dose-rate matrix (Gy per time unit);
                                    NULL -> the point-source law
                                    (1 - 0.01 r) / max(r, 0.1 cm)^2, Sec. 2.2.1 step (i) */
  const int32_t* group_organ;    /* optional n_groups: organ of each group, in [0, n_organs);
                                    NULL -> organ j = group j */
  int n_organs;                  /* organs when group_organ != NULL (1..n_groups); the
                                    hidden weights of gmco_set_weights are per organ */
  int n_dvh_points;              /* optional DVH point set (0: none); needs point_xyz-style
                                    positions and the point-source law */
  const double* dvh_xyz;         /* n_dvh_points x 3, cm */
  const int32_t* dvh_organ;      /* n_dvh_points, organ of each DVH point */
} gmco_case;

/* Options of one optimisation run.  The paper leaves its L-BFGS details out
 * (Sec. 2.2.2); this is textbook L-BFGS (two-loop recursion, gamma scaling of
 * the newest pair) with Armijo backtracking and the relative-variation stop
 * rule of Sec. 2.2.3. */
typedef struct {
  int max_iter;       /* cap on accepted steps per plan (cumulative over calls) */
  double eps;         /* converged when F_prev - F <= eps * F_prev (0: run to max_iter) */
  double c1;          /* Armijo constant, e.g. 1e-4 */
  double beta;        /* backtracking factor in (0, 1), e.g. 0.5 */
  int max_ls;         /* trials per iteration before LS_FAIL, >= 1 */
  int check_every;    /* rounds between host checks of the active-plan count (0 -> 16) */
  int time_kernels;   /* n > 0: time the evaluation and the update launches of rounds
                         0, n, 2n, ... with HIP events on the context stream; 0: none */
  int resume_stopped; /* 1: plans stopped as CONVERGED or LS_FAIL iterate again
                         (e.g. after a change of precision); 0: they stay */
  int dtype;          /* gmco_dtype of this run's evaluations, -1: the context's.
                         F32 and F32_ACC64 are always available; BF16 and FP8 need a
                         context created with that dtype.  Successive runs with
                         rising precision form a precision ladder on one state. */
  int per_case_launches; /* gmco_optimize_many only: 0 groups the cases (per round, one
                         evaluation launch per padded dwell count and dtype, one
                         update launch per update shape, which also sums each
                         case's gradient partials);
                         1 issues every case's kernels as launches of their own */
} gmco_run;

typedef struct {
  int rounds;          /* batched evaluation rounds issued */
  int n_converged;
  int n_maxiter;
  int n_ls_fail;
  int n_nonfinite;
  int max_iters;       /* largest accepted-step count of any plan */
  float device_ms;     /* GPU time of the whole run (HIP events on the context stream) */
  float eval_ms;       /* sum of the timed evaluation-kernel durations */
  float update_ms;     /* sum of the timed split-reduction + L-BFGS update durations */
  int eval_launches;   /* evaluation launches */
  double eval_work;    /* plan evaluations done / batch size: full-batch launch
                          equivalents (stopped plans are compacted out of every
                          evaluation) */
  int timed_launches;  /* evaluation launches timed (time_kernels > 0) */
  double timed_work;   /* plan evaluations of the timed launches / batch size */
} gmco_run_info;

typedef struct {
  double F_run;                      /* objective at the final x, run arithmetic */
  double F64;                        /* eq. (obj) re-evaluated in FP64 at t = x^2 */
  double f_organ[GMCO_MAX_GROUPS];   /* (1/N_j) sum_i f_ij, FP64 */
  double V100_pct[GMCO_MAX_GROUPS];  /* % of the structure's points with d >= Rx */
  double V75_cc[GMCO_MAX_GROUPS];    /* volume_cc * share of points with d >= 0.75 Rx */
  double D10_pct[GMCO_MAX_GROUPS];   /* % Rx of the k-th hottest point, k = ceil(0.1 N) */
  double D90_pct[GMCO_MAX_GROUPS];   /* same with k = ceil(0.9 N) */
  int iterations;                    /* accepted steps */
  int evaluations;                   /* objective evaluations incl. the start point */
  int status;                        /* gmco_plan_status */
  int reserved;
} gmco_plan_metrics;

/* Create a context on opts->device.  *out is owned by the caller until
 * gmco_destroy.  Errors: EINVAL (bad opts), ENOLIB (device is not gfx950),
 * EHIP. */
int gmco_create(gmco_ctx** out, const gmco_opts* opts);

/* Free everything the library allocated.  NULL-safe.  A bound workspace is
 * not freed (its owner frees it). */
int gmco_destroy(gmco_ctx* ctx);

/* Issue all later device work on `stream` (a hipStream_t; NULL = the null
 * stream).  The library does not own the stream. */
int gmco_set_stream(gmco_ctx* ctx, void* stream);

/* Device bytes needed for a case of M points, K dwells and n_dvh_points DVH
 * points (0: none) with the context's max_plans, history and dtype. */
int gmco_workspace_bytes(const gmco_ctx* ctx, int n_points, int n_dwells, int n_dvh_points,
                         size_t* bytes);

/* Hand the library a device buffer (256-byte aligned) to carve all its device
 * arrays from, instead of allocating its own.  The caller keeps ownership and
 * must keep it alive until gmco_destroy or the next gmco_bind_workspace.
 * Must precede gmco_load_case.  A buffer smaller than gmco_workspace_bytes
 * makes gmco_load_case return ENOMEM. */
int gmco_bind_workspace(gmco_ctx* ctx, void* device_ptr, size_t bytes);

/* Copy a case to the device and build its dose-rate matrix (Sec. 2.2.1 step
 * (i)) in FP64 and in the run dtype, plus the default start time
 * t_bar = Rx / mean_{i in target} sum_l Ddot_il (uniform dwell times whose
 * mean target dose is the prescription).  Invalidates earlier weights.
 * Errors: EINVAL, ENOMEM, EHIP. */
int gmco_load_case(gmco_ctx* ctx, const gmco_case* c);

/* Set the hidden-weight batch, eq. (obj): W is P x n_organs (n_groups without
 * group_organ), finite and >= 0,
 * used as given (normalise rows to sum 1 beforehand for the paper's weighted
 * sum).  t0 is P x K start dwell times, finite and > 0 (x_l = 0 is a fixed
 * point of the x^2 substitution of Sec. 2.1.2: the gradient of eq. 2 is
 * proportional to x_l), or NULL for the uniform start t_bar.  Resets every
 * plan to its start.  Errors: EINVAL (P out of 1..max_plans, bad value),
 * ESTATE (no case loaded), EHIP. */
int gmco_set_weights(gmco_ctx* ctx, int n_plans, const double* W, const double* t0);

/* One batched evaluation of eq. (obj) and of its gradient in the dwell
 * weights (eq. 2 summed over points) at x (P x K, P = current batch size), in
 * the context's dtype with that dtype's accumulation (see gmco_dtype: FP32
 * for F32, BF16 and FP8; the dose in FP64 for F32_ACC64 and F32_CHUNK64; the
 * back-projection always in FP32).  F is P, g is P x K.  Uses the same
 * kernels as the optimiser and leaves the optimiser state untouched.
 * Errors: ESTATE, EINVAL, EHIP. */
int gmco_evaluate(gmco_ctx* ctx, const double* x, double* F, double* g);

/* gmco_evaluate for callers that cannot allocate device memory or
 * synchronise (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same evaluation kernels on device arrays,
 * enqueued on the context stream without any allocation, host copy or
 * synchronisation.  x_dev is P x K FP64 dwell weights, F_dev P and g_dev
 * P x K FP64 outputs, all device memory owned by the caller (P = current
 * batch).  The FP32 copy of x and the split partials live in a 32 MiB
 * library array, one per device, held until the process ends; the batch must
 * fit it (4 x padded plans x padded dwells bytes for x plus, per split of the
 * point range, that again and 8 bytes per padded plan: about 3,000 plans at
 * 512 dwells with one split), else EINVAL.  The split count is the context's,
 * lowered to what fits.  Every call on a device shares that device's array:
 * calls that overlap on one device (several streams or threads) race.
 * Errors: EINVAL, ESTATE, EHIP. */
int gmco_evaluate_noalloc(gmco_ctx* ctx, const double* x_dev, double* F_dev, double* g_dev);

/* Run batched L-BFGS until every plan has stopped (converged, max_iter,
 * line-search failure) or info reports the state.  Continues from the
 * current state: plans stopped by max_iter resume if run->max_iter is larger.
 * Synchronous on the context stream.  Errors: EINVAL, ESTATE, EHIP,
 * ENUMERIC (every plan non-finite at its start). */
int gmco_optimize(gmco_ctx* ctx, const gmco_run* run, gmco_run_info* info);

/* Plan evaluation and selection (Sec. 2.3.1, Sec. 2.4).  Validity after
 * RTOG 0924: target V100 >= v100_min, urethra D10 < urethra_d10_max, bladder
 * and rectum V75 below their limits; RTOG+ also needs V100 >= v100_plus. */
typedef struct {
  int target, urethra, bladder, rectum; /* structure indices */
  double v100_min;        /* 90 % */
  double v100_plus;       /* 95 % */
  double urethra_d10_max; /* 118 % of the prescription (strict) */
  double bladder_v75_max; /* 1 cc (strict) */
  double rectum_v75_max;  /* 1 cc (strict) */
} gmco_select_opts;

/* Recompute the metrics of the current plans and select one: RTOG+ over
 * RTOG over invalid; among valid plans the highest target V100; among
 * invalid plans the lowest bladder + rectum V75 among those meeting the
 * target and urethra criteria (all invalid plans if none does); ties to the
 * lowest index.  Also each plan's class (2 RTOG+, 1 RTOG, 0 invalid) and
 * whether no other plan is at least as good in every individual objective
 * and strictly better in one (Sec. 2.2.4).  opts NULL = the values above for
 * structures 0..3 = target, urethra, bladder, rectum.  plan_class and
 * nondominated (P each) and nondominated_fraction may be NULL. */
int gmco_select_plan(gmco_ctx* ctx, const gmco_select_opts* opts, int* best, int* plan_class,
                     int* nondominated, double* nondominated_fraction);

/* Batched uneven cases: run the same options on n contexts (one case and
 * weight batch each, one device) in lockstep rounds on the first context's
 * stream.  Each round evaluates every case's running plans, in one grouped
 * launch per padded dwell count (a table maps each workgroup to its case),
 * then reduces and updates them in grouped launches (run->per_case_launches
 * = 1: separate launches per case, with identical results).
 * rounds_per_graph > 0 captures that many rounds (rounded up to even) into
 * one HIP graph and replays it until every plan of every case has stopped;
 * 0 issues plain launches.  infos has n entries (NULL allowed); device_ms is
 * the whole batch's time.  Plans that stop early keep compacted out of every
 * later round on the device.  The grouped form allocates its argument tables
 * (a few hundred bytes per case) for the call.  Errors as gmco_optimize,
 * ENOMEM. */
int gmco_optimize_many(gmco_ctx* const* ctxs, int n, const gmco_run* run, gmco_run_info* infos,
                       int rounds_per_graph);

/* Autotuner: time the evaluation kernel of this case and batch for each
 * candidate launch shape and keep the fastest: the split count of the point
 * range (workgroups per plan tile of 64 plans, or per pair of tiles for the
 * BF16 and FP8 kernels up to 448 padded dwells; up to 32), the tile-to-XCD
 * mapping (all tiles of one point range on one XCD, or round-robin) and the
 * workgroup shape of dtype's kernel (gmco_tuning.lp_shape lists them).  reps timed
 * launches per candidate on the context stream.  Needs a weight batch.
 * best_split / best_us may be NULL.  The tuning belongs to the kernel family
 * of dtype (FP32 operands, or BF16 / FP8); the split is used by its rounds in
 * which every plan tile of the batch capacity is active (rounds with fewer
 * active plans, stopped plans being compacted out, choose their split on the
 * device to fill the compute units), the mapping and shape by every round.
 * No choice changes a result, except the FP64-accumulated dwell-quarter
 * shape (an FP64 rounding difference): the per-plan arithmetic and its order
 * are the same in every other shape. */
int gmco_autotune(gmco_ctx* ctx, int dtype, int reps, int* best_split, float* best_us);

/* The launch shape of a kernel family (see gmco_autotune). */
typedef struct {
  int split;     /* point-range splits of a full-batch round */
  int tuned;     /* 1: split set by the autotuner or the caller */
  int lp_shape;  /* workgroup shape.  BF16 / FP8: 0 = 8 wavefronts x 16 plans, 1 = 4 x 32
                    (Kp <= 384), 2 = 4 x 32 plans in two roles of 4 wavefronts, dose
                    product with eq. 1 and back-projection of the previous block
                    (Kp <= 384); all three give the same bits.  FP32 operands with
                    FP64-accumulated dose: 0 = 512 threads per 64-plan tile (dwell
                    halves), 1 = 256 threads per 32 plans (two workgroups per
                    compute unit), 2 = 1,024 threads per 64-plan tile (dwell
                    quarters, four waves per SIMD; Kp a multiple of 64; the dose
                    partials are added in another order, an FP64 rounding
                    difference), 3 = 512 threads per 64-plan tile in two roles
                    (dose product with eq. 1, back-projection of the previous
                    block); 0, 1 and 3 give the same bits.  Plain FP32: 0 = 256
                    threads per 64-plan tile, 3 = 512 threads in the same two roles
                    (the same bits).  FP32 with FP64-summed chunks: 0.  Defaults
                    after gmco_load_case: BF16 2 (up to 384 padded dwells), FP8 0,
                    FP32 3, FP64-accumulated 0 (3 from 448 padded dwells) */
  int xcd_map;   /* 1: tiles of one point range on one XCD when the grid allows */
} gmco_tuning;

/* Read or set the launch shape of dtype's kernel family (-1: the context's
 * dtype), e.g. to reuse an autotuned shape on cases of the same size.  Needs
 * a loaded case.  set: EINVAL for a split outside 1..the autotuner's range,
 * xcd_map not 0/1 or a shape not available for dtype at the case's dwell
 * count.  The FP32-operand kernels (plain FP32 and FP64-accumulated) share
 * split and mapping and have a workgroup shape each. */
int gmco_get_tuning(const gmco_ctx* ctx, int dtype, gmco_tuning* out);
int gmco_set_tuning(gmco_ctx* ctx, int dtype, const gmco_tuning* t);

/* Set the split count directly (e.g. from a cache of autotuned shapes) for
 * both kernel families; otherwise the autotuner's scope.  1 <= split <= the
 * autotuner's range. */
int gmco_set_split(gmco_ctx* ctx, int split);

/* Checkpoint of the optimiser (project extension; the paper has none).  The
 * state is the weight batch and, per plan, the L-BFGS state machine
 * (objective, previous objective, trial step, g'p, status, counters), x, g,
 * the search direction, the pending trial point, the history ring (s, y,
 * rho) and the context's split counts.  It does not include the case: the
 * restoring context must hold a case of the same shape (dwells, history
 * length, groups and organs; normally the same case, loaded with
 * gmco_load_case).  A gmco_optimize after gmco_set_state continues exactly as
 * the saved context would have (the same kernels on the same values, bitwise).
 *   gmco_state_bytes: size of the blob of the current batch.  ESTATE without a
 *     weight batch.
 *   gmco_get_state: write the blob to host memory owned by the caller
 *     (`bytes` >= gmco_state_bytes, else EINVAL).  ESTATE without a batch.
 *   gmco_set_state: restore a blob; it replaces the weight batch (the batch
 *     size becomes the blob's).  ESTATE without a case; EINVAL for a blob of
 *     another library version or case shape, a truncated one, or more plans
 *     than max_plans.  Layout: a 64-byte header, then plan-major arrays; it is
 *     private to this library version. */
int gmco_state_bytes(const gmco_ctx* ctx, size_t* bytes);
int gmco_get_state(gmco_ctx* ctx, void* blob, size_t bytes);
int gmco_set_state(gmco_ctx* ctx, const void* blob, size_t bytes);

/* t = x^2 of every plan, P x K, FP64 (computed on the device). */
int gmco_get_dwell_times(gmco_ctx* ctx, double* t);

/* Current dwell weights x, P x K (run state, widened to double). */
int gmco_get_weights_x(gmco_ctx* ctx, double* x);

/* Per-plan metrics at the current t (Sec. 2.3.1 DVH definitions: V_x counts
 * points with d >= x % Rx; D_x is the dose of the k-th hottest point,
 * k = max(1, ceil(x N / 100))), from an FP64 dose recomputation.  out has P
 * entries. */
int gmco_get_metrics(gmco_ctx* ctx, gmco_plan_metrics* out);

/* The dose-rate matrix as used: D64 (M x K, FP64) and/or Drun (M x K, the
 * run-dtype values widened to double, column scale applied).  Either pointer
 * may be NULL.  Rows are in the caller's point order. */
int gmco_get_dose_rate(gmco_ctx* ctx, double* D64, double* Drun);

/* Default start time t_bar of the loaded case. */
int gmco_get_start_time(gmco_ctx* ctx, double* t_bar);

/* Case features of the learned warm start: for every structure j, the
 * histogram over dwells of the distance from the dwell to the nearest point
 * of j, in 16 bins of 0.25 cm (the last bin open-ended), divided by the dwell
 * count.  out has n_organs x 16 floats (structures = organs).  Needs a case loaded with point
 * positions.  (Project extension; not in the paper.) */
int gmco_case_features(gmco_ctx* ctx, float* out);

const char* gmco_last_error(const gmco_ctx* ctx);
const char* gmco_strerror(int status);

/* ---- Learned warm start: a fully connected ReLU network (project
 * extension, not in the paper) trained on plans the method produced, mapping
 * hidden weights and case features to start dwell weights.  Products run on
 * BF16 matrix ops with FP32 accumulation; loss, gradients and Adam state are
 * FP32.  Parameter layout: for each layer W (n_out x n_in, row-major) then b
 * (n_out); hidden layers ReLU, output linear; loss = mean squared error over
 * all outputs of a batch. ---- */
typedef struct gmco_mlp gmco_mlp;

/* sizes = (n_in, hidden..., n_out), n_sizes >= 2, each 1..4096; max_batch
 * rows per forward pass.  Parameters start at zero; set them with
 * gmco_mlp_set_params.  Errors: EINVAL, ENOLIB, ENOMEM. */
int gmco_mlp_create(gmco_mlp** out, int device, const int* sizes, int n_sizes, int max_batch);
int gmco_mlp_destroy(gmco_mlp* net);
int gmco_mlp_set_stream(gmco_mlp* net, void* stream);
int gmco_mlp_param_count(const gmco_mlp* net, size_t* n);
/* Copy n parameters in (resets the Adam moments) or out. */
int gmco_mlp_set_params(gmco_mlp* net, const float* params, size_t n);
int gmco_mlp_get_params(gmco_mlp* net, float* params, size_t n);
/* Loss and gradient of one batch of B rows (host arrays X: B x n_in, Y: B x
 * n_out); grad (n parameters) may be NULL. */
int gmco_mlp_loss_grad(gmco_mlp* net, int B, const float* X, const float* Y, double* loss, float* grad);
/* Copy a training set of N rows to the device (replaces an earlier one). */
int gmco_mlp_set_data(gmco_mlp* net, int N, const float* X, const float* Y);
/* n_steps Adam steps (beta 0.9 / 0.999, eps 1e-8) on batches of B rows whose
 * indices into the training set are order[s * B .. s * B + B - 1]; the mean
 * batch loss is returned.  Errors: EINVAL, ESTATE (no data), EHIP. */
int gmco_mlp_train(gmco_mlp* net, int n_steps, int B, const int32_t* order, float lr, double* mean_loss);
/* Y (B x n_out) = network(X (B x n_in)); any B, processed in max_batch chunks. */
int gmco_mlp_predict(gmco_mlp* net, int B, const float* X, float* Y);
const char* gmco_mlp_last_error(const gmco_mlp* net);

/* Set the weight batch with the learned start: like gmco_set_weights, then
 * for each plan the network (inputs: the plan's n_organs hidden weights as
 * given, then the case's n_organs x 16 features of gmco_case_features;
 * outputs: n_dwells values x_hat, the dwell weights normalised by the
 * uniform start's sqrt(t_bar)) gives the start x0 = max(x_hat, x_floor)
 * sqrt(t_bar) (x = 0 is a fixed point of the x^2 substitution, Sec. 2.1.2).
 * Plain L-BFGS from the uniform start is the fallback: a plan keeps the
 * learned start only where eq. (obj) there (context dtype) is finite and
 * below its value at the uniform start.  Features, network and both
 * evaluations run on the device, on the context stream.  use_warm (P ints,
 * 1 = learned start kept) and n_warm may be NULL.  The network must have
 * 17 x n_organs inputs and n_dwells outputs and live on the context's device;
 * the call uses its activation buffers, so it must not overlap other work of
 * the network.  (Project extension.)  Errors: as gmco_set_weights, EINVAL
 * (network shape or device, x_floor <= 0, a case without point positions). */
int gmco_set_weights_learned(gmco_ctx* ctx, gmco_mlp* net, int n_plans, const double* W, double x_floor,
                             int* use_warm, int* n_warm);

#ifdef __cplusplus
}
#endif
#endif /* GMCO_H */
