// Internal types shared by the gMCO device kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "gmco.h"

namespace gmco {

constexpr int kGmax = GMCO_MAX_GROUPS;
constexpr int kBM = 16;   // dose points per inner block of the evaluation kernel
constexpr int kPT = 64;   // plans per tile of the evaluation (one FP32 workgroup)
// Shape of the BF16 / FP8 evaluation workgroup per padded dwell count:
// threads, and 16-plan column groups per wavefront.  Shape 0 (default): up
// to Kp = 384 eight wavefronts of 16 plans (two per SIMD) share one
// double-buffered LDS tile; at Kp = 416 four wavefronts of 32 plans; above,
// four of 16 (the registers of 32 plans no longer fit).  Shape 1 (up to
// Kp = 384, an autotuner candidate): four wavefronts of 32 plans, one per
// SIMD, each LDS operand feeding twice the matrix ops.  Shape 2 (up to
// Kp = 384, an autotuner candidate): eight wavefronts in two roles over four
// groups of 32 plans, the dose product with eq. 1 in one, the back-projection
// of the previous block in the other.  All shapes of a Kp cover the same
// plan tiles (lp_tiles), so the grid does not depend on the shape.
__host__ __device__ constexpr bool lp_shape_ok(int Kp, int shape) {
  return shape == 0 || ((shape == 1 || shape == 2) && Kp <= 384);
}
__host__ __device__ constexpr int lp_threads(int Kp, int shape = 0) {
  return (Kp <= 384 && (shape == 0 || shape == 2)) ? 512 : 256;
}
__host__ __device__ constexpr int lp_halves(int Kp, int shape = 0) {
  return (Kp == 416 || (Kp <= 384 && shape == 1)) ? 2 : 1;
}
// FP64-accumulated evaluation, workgroup shape 2: dwell quarters (1,024
// threads, four waves per SIMD), for padded dwell counts that are multiples
// of 64.
__host__ __device__ constexpr bool acc_quarters_ok(int Kp) { return Kp % 64 == 0; }
__host__ __device__ constexpr int lp_tiles(int Kp) { return lp_threads(Kp) / 64 * 16 * lp_halves(Kp) / kPT; }
constexpr int kKAlign = 32;
constexpr int kMAlign = 32;  // points: a multiple of every kernel's block
constexpr int kSplitMax = 256;  // largest split-M count the heuristic picks

// Internal plan states; 0..5 match gmco_plan_status.
enum : int {
  ST_RUNNING = 0,
  ST_CONVERGED = 1,
  ST_MAXITER = 2,
  ST_LSFAIL = 3,
  ST_NONFINITE = 4,
  ST_INACTIVE = 5,
  ST_INIT = 6  // the point in xt is to be taken as the current iterate
};

__host__ __device__ inline bool state_active(int s) { return s == ST_RUNNING || s == ST_INIT; }

// Per-plan scalars of the batched L-BFGS state machine.
struct PlanState {
  double F;      // objective at x
  double Fprev;  // objective before the last accepted step
  double alpha;  // current trial step
  double gtp;    // g' p of the current direction
  int status;
  int iter;      // accepted steps
  int ntrial;    // rejected trials of the current iteration
  int hcount;    // history pairs held
  int hhead;     // next ring slot
  int nevals;    // objective evaluations
  int pad0, pad1;
};
static_assert(sizeof(PlanState) == 64, "PlanState layout");

// Eq. 1 parameters per structure: (w_min, D_min, D_max, w_max); entry kGmax
// is the all-zero row used by padding points.
struct GroupTable {
  float4 prm[kGmax + 1];
  double prm64[kGmax + 1][4];
};

// Per-round shape of the compacted evaluation, written by the evaluation
// kernel: the running plans occupy compact columns 0..nact-1, which form
// ntiles tiles of kPT; every tile is split S ways over the points.
struct RoundTable {
  int nact;
  int ntiles;
  int S;
  int pad;
};

struct EvalArgs {
  const void* D;          // [Mp][Kp] dose-rate matrix in the run dtype
  const void* DT;         // [Kp][Mp] transposed copy (BF16 / FP8 only)
  const float* colscale;  // [Kp] FP8 column scales (NULL otherwise)
  const int* grp;         // [Mp] structure index, kGmax for padding
  const float* x;         // [Pp][Kp] points to evaluate (dwell weights)
  const float* wn;        // [Pp][kGmax] w_j / N_j
  // A workgroup covers T consecutive tiles of kPT columns (T = 1 for FP32
  // operands, lp_tiles(Kp) for BF16 / FP8); the grid of a round is S times
  // ceil(ntiles / T) workgroups.
  // Compacted rounds (flag != NULL): every workgroup counts the running
  // plans (flag[p] = 1) in plan order, takes the round's tile count
  // ntiles = ceil(nact / kPT) and split count split_tab[ntiles] (s_tuned
  // instead when every tile of the capacity is active), and maps its T kPT
  // columns to the plans of compact ranks j0 .. j0 + T kPT - 1.  Split-0
  // workgroups record each plan's rank in slot; workgroup 0 writes the
  // round's shape to rt and adds nact to work.  The partials are then
  // [S][ntiles * kPT][Kp] by rank.  flag == NULL: every plan, column = plan,
  // host S and ntiles, partials [S][Pp][Kp].
  const int* flag;
  const int* split_tab;   // [ntiles + 1] split count per active tile count
  int* slot;              // [Pp] compact rank of each running plan
  RoundTable* rt;
  unsigned long long* work;
  unsigned long long* work2;  // optional second count (the timed launches)
  int P;                  // plans of the batch
  int s_tuned;            // 0 = split_tab
  float* Gpart;           // split-M partial back-projections
  double* Fpart;          // split-M partial objectives
  int Mp, Kp, Pp;
  int nblocks;            // Mp / kBM (16-point blocks)
  int S;                  // M splits (uncompacted form)
  int ntiles;             // Pp / kPT (uncompacted form)
  int grid;               // workgroups launched; those past the round's grid exit
  int lp_shape;           // BF16 / FP8 workgroup shape (lp_threads, lp_halves)
  int xcd_map;            // 1: tiles of one point range on one XCD when the grid allows
  int last16;             // 0: dwells Kp - 16 .. Kp - 1 are all padding (FP32-operand
                          // kernels skip that 16-dwell slice: its products are zero)
  GroupTable gt;
};

struct UpdateArgs {
  const float* Gpart;     // split-M gradient partials [S][ntiles * kPT][Kp] by compact column
  const double* Fpart;
  float* x;       // [Pp][Kp] current iterate
  float* g;       // [Pp][Kp] gradient at x
  float* dir;     // [Pp][Kp] search direction
  float* xt;      // [Pp][Kp] point to evaluate next
  float* Sh;      // [Pp][m][Kp]
  float* Yh;      // [Pp][m][Kp]
  double* rho;    // [Pp][m]
  PlanState* ps;
  int* active_count;  // [2]
  int* flag;          // [Pp] 1 while the plan runs, for the next compaction
  const int* slot;    // [Pp] compact column of each active plan
  const RoundTable* rt;
  int Kp, Pp, m, K;
  int max_iter, max_ls;
  double eps, c1, beta;
  int round;
};

// Update kernel lane layout: groups of four dwells per lane, E values per
// lane (4 up to 256 padded dwells, 8 up to 512).
__host__ __device__ constexpr int update_width(int Kp) { return Kp <= 256 ? 4 : (Kp <= 512 ? 8 : 0); }
constexpr int kKpMax = 512;  // largest padded dwell count the update supports

// ---- launchers (each defined next to its kernels) ----
hipError_t launch_dose_rate(const double* dwell_xyz, const double* pt_xyz, const double* user_D,
                            const int* perm, int M, int K, int Mp, int Kp, double* D64,
                            hipStream_t st);
hipError_t launch_cast_dose(const double* D64, int Mp, int Kp, int dtype, float* D32, void* Dlp,
                            void* DTlp, float* colscale, hipStream_t st);
hipError_t launch_widen_fp8(const void* D8, const float* colscale, int Mp, int Kp, double* out,
                            hipStream_t st);
hipError_t launch_start_time(const double* D64, int Kp, int row_begin, int row_end,
                             double prescription, double* t_bar, hipStream_t st);
hipError_t launch_init_plans(int P, int Pp, int K, int Kp, const double* t0, const double* t_bar,
                             const double* W, int G, int O, const int* gorg, const int* norm,
                             float* xt, float* x, float* wn, double* W64, PlanState* ps,
                             hipStream_t st);
hipError_t launch_eval(const EvalArgs& a, int dtype, hipStream_t st);
// Several cases of one padded dwell count Kp in one launch: case c's
// workgroups are start[c] .. start[c + 1] - 1 of grid (start[c] a multiple
// of 8), its arguments args[c] (device arrays, n entries / n + 1 starts).
hipError_t launch_eval_grouped(const EvalArgs* args, const int* start, int n, int grid, int Kp, int dtype,
                               int lp_shape, hipStream_t st);
// Update of n cases in one launch (cases of one update width E); the grid is
// sized for the largest case.
hipError_t launch_update_grouped(const UpdateArgs* args, int n, int E, int Pp_max, int m, int round,
                                 hipStream_t st);
hipError_t launch_update(const UpdateArgs& a, hipStream_t st);
hipError_t launch_finish_eval(const float* Gpart, const double* Fpart, const float* x, int S,
                              int P, int Pp, int K, int Kp, double* F, double* g,
                              hipStream_t st);
hipError_t launch_resume(PlanState* ps, const float* x, float* xt, int* flag, int Pp, int Kp,
                         int max_iter, int resume_stopped, hipStream_t st);
hipError_t launch_export_t(const float* x, int P, int K, int Kp, double* t64, int Kp_out,
                           hipStream_t st);
hipError_t launch_x_to_device(const double* x_host_dev, int P, int Pp, int K, int Kp, float* xe,
                              hipStream_t st);
hipError_t launch_dose64(const double* D64, const double* t64, int Mp, int Kp, int Pp,
                         double* d64, hipStream_t st);
// One pass of the per-organ metrics over the doses d64 (P rows of stride ld)
// of a point set whose organ o is the range off[o] .. off[o] + cnt[o]:
// objective != 0 adds the individual objectives (eq. 1 with each point's
// group parameters; the optimisation points), dvh != 0 the DVH metrics.
struct MetricsArgs {
  const double* d64;
  int ld;
  const int* off;
  const int* cnt;
  const int* grp;          // group of each optimisation point
  const double* gparams;   // [kGmax][4]
  const double* volume_cc; // per organ
  const double* W64;       // [Pp][kGmax] hidden weights per organ
  const PlanState* ps;
  int P, O;
  int objective, dvh;
  double rx;
  gmco_plan_metrics* out;
};
hipError_t launch_metrics(const MetricsArgs& m, hipStream_t st);
hipError_t launch_metrics_final(const MetricsArgs& m, hipStream_t st);

hipError_t launch_select(const gmco_plan_metrics* m, int P, int G, const gmco_select_opts& o, int* cls,
                         int* meets_tu, int* nd, int* out, hipStream_t st);
// Network of the learned warm start (defined with its kernels).
int mlp_inputs(const gmco_mlp* m);
int mlp_outputs(const gmco_mlp* m);
int mlp_device(const gmco_mlp* m);
hipError_t mlp_forward_device(gmco_mlp* m, int B, const float* X, float* Y, hipStream_t st);
// Learned start: network inputs per plan (hidden weights, then the case
// features), the floored start x0 = max(y, floor) sqrt(t_bar), and the
// per-plan choice between it and the uniform start.
hipError_t launch_learned_inputs(const double* W64, const float* feat, int P, int O, float* X, hipStream_t st);
hipError_t launch_learned_start(const float* Y, int P, int Pp, int K, int Kp, const double* t_bar, double floor,
                                float* xe, hipStream_t st);
hipError_t launch_pick_start(const double* F_warm, const double* F_uniform, const float* xe, int P, int Kp,
                             float* x, float* xt, int* n_warm, int* use_warm, hipStream_t st);
hipError_t launch_features(const double* dwell, const double* pts, const int* perm, const int* goff,
                           const int* gcnt, int K, int G, unsigned* hist, float* out, hipStream_t st);

}  // namespace gmco
