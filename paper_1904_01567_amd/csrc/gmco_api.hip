// Host runtime and C-ABI of the gMCO hot path: context, device arena,
// case and batch upload, the batched optimisation loop and result export.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "gmco_internal.h"

using namespace gmco;

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
int round_up(int v, int a) { return (v + a - 1) / a * a; }

// Byte offsets of every device array inside the arena.
struct Layout {
  size_t D64, D32, Dlp, DTlp, colscale, grp, perm, stage, gparams, volume, goff, gcnt, counts, t_bar;
  size_t gorg, D64d, dstage, dperm, doff, dcnt;
  size_t Wst, t0st, xst, Fst, gst;
  size_t wn, W64, x, g, dir, xt, xe, Sh, Yh, rho, ps, Gpart, Fpart, active, work, flag, slot, rt,
      split_tab;
  size_t t64, d64, metrics, hist, feat, sel;
  size_t mlpX, mlpY, Fu, usewarm, nwarm;
  size_t total;
};

struct Dims {
  int M = 0, K = 0, Mp = 0, Kp = 0, Pp = 0, S = 1, ntiles = 1, nblocks = 0;
  int Md = 0, Mdp = 0;  // DVH points (0: none), padded
  int S_cap = 1;      // split counts up to this fit the partial buffers (autotuning range)
  int S_tuned = 0;    // split set by the caller or the autotuner, 0 = heuristic
  int S_lp = 1;       // S and S_tuned of the BF16 / FP8 kernels, whose
  int S_tuned_lp = 0; // workgroups cover lpt tiles each
  int lpt = 1;
  int lp_shape = 0;   // BF16 / FP8 workgroup shape (autotuned)
  int acc_shape = 0;  // FP64-accumulated kernel: 0 = 512 threads per plan tile,
                      // 1 = 256 threads per half tile, 2 = dwell quarters,
                      // 3 = two roles (autotuned)
  int f32_shape = 3;  // plain FP32 kernel: 0 = 256 threads per plan tile,
                      // 3 = 512 threads in two roles (the default: measured
                      // faster at the paper-scale case; autotuned)
  int xcd32 = 1;      // XCD-aware tile mapping of the FP32-operand kernels
  int xcd_lp = 1;     // and of the BF16 / FP8 kernels (autotuned)
  int grid_heur = 1;  // largest S * ntiles the per-round heuristic can choose
  int grid16 = 1;     // largest grid a compacted round launches: FP32 operands,
  int grid32 = 1;     // BF16 / FP8
  int grid_cap = 1;   // plan tiles times splits the partial buffers hold
  // split count per active tile count 0..ntiles, for 16-point (FP32 modes)
  // and 32-point (BF16, FP8) evaluation blocks
  std::vector<int> split16, split32;
};

constexpr int kSplitTuneMax = 32;

// Split count for ntiles plan tiles over nblocks point blocks on n_cu compute
// units (one evaluation workgroup per CU at a time): minimises the number of
// workgroup waves times the blocks per workgroup (plus a pipeline fill of two
// blocks), with a slight preference for multiples of 8 (the XCD-aware tile
// mapping of the evaluation kernel).
int choose_split(int ntiles, int nblocks, int n_cu, int s_max) {
  if (ntiles <= 0 || nblocks <= 0) return 1;
  const int hi = std::min(s_max, nblocks);
  int best = 1;
  double best_c = 0.0;
  for (int S = 1; S <= hi; ++S) {
    const double waves = (double)(((long long)ntiles * S + n_cu - 1) / n_cu);
    const double per = (double)((nblocks + S - 1) / S + 2);
    const double c = waves * per * ((S & 7) ? 1.02 : 1.0);
    if (S == 1 || c < best_c) {
      best_c = c;
      best = S;
    }
  }
  return best;
}

}  // namespace

struct gmco_ctx {
  int device = 0;
  int dtype = GMCO_DTYPE_F32;
  int m = 10;
  int Pmax = 1;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  std::string err;

  void* ws = nullptr;       // arena base
  size_t ws_bytes = 0;
  bool ws_owned = false;    // allocated by the library
  void* bound = nullptr;    // workspace handed in by the caller
  size_t bound_bytes = 0;

  Dims dim;
  Layout lay{};
  int G = 0;             // parameter groups (rows of eq. 1)
  int O = 0;             // organs: hidden weights, point counts, metrics
  double rx = 0.0;
  int target = 0;
  std::vector<int> counts, offsets, perm;  // host copies; offsets / counts per organ
  bool case_loaded = false;
  bool has_points = false;  // point positions were given (features need them)
  int P = 0;              // current batch, 0 = none
  int* host_count = nullptr;  // pinned copies of the running-plan count, one per block parity
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipStream_t gstream = nullptr;  // library-owned stream for graph capture
  hipEvent_t gev = nullptr;
  GroupTable gt{};

  template <class T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
  }
};

namespace {

int fail(gmco_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(gmco_ctx* c, hipError_t e, const char* what) {
  return fail(c, GMCO_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define GMCO_HIP(ctx, call)                                 \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

bool is_low_precision(int dtype) { return dtype == GMCO_DTYPE_BF16 || dtype == GMCO_DTYPE_FP8; }
size_t lp_bytes(int dtype) { return dtype == GMCO_DTYPE_BF16 ? 2 : (dtype == GMCO_DTYPE_FP8 ? 1 : 0); }
// a run may use the context's dtype and every FP32-operand mode
bool dtype_available(const int ctx_dtype, int dtype) {
  return dtype == GMCO_DTYPE_F32 || dtype == GMCO_DTYPE_F32_ACC64 ||
         dtype == GMCO_DTYPE_F32_CHUNK64 || dtype == ctx_dtype;
}

Dims make_dims(int M, int K, int Pmax, int n_cu, int Md) {
  Dims d;
  d.M = M;
  d.K = K;
  d.Md = Md;
  d.Mdp = Md > 0 ? round_up(Md, kMAlign) : 0;
  d.Kp = round_up(K, kKAlign);
  d.Mp = round_up(M, kMAlign);
  d.nblocks = d.Mp / kBM;
  d.Pp = round_up(Pmax, kPT);
  d.ntiles = d.Pp / kPT;
  d.lpt = lp_tiles(d.Kp);
  // compacted rounds choose their split on the device for 1..ntiles active
  // tiles, with the 16-point (FP32) or 32-point (BF16, FP8) block count and
  // workgroups of 1 or lpt tiles
  d.grid_heur = d.grid16 = d.grid32 = 1;
  d.split16.assign(d.ntiles + 1, 1);
  d.split32.assign(d.ntiles + 1, 1);
  for (int nt = 1; nt <= d.ntiles; ++nt) {
    const int units = (nt + d.lpt - 1) / d.lpt;
    d.split16[nt] = choose_split(nt, d.nblocks, n_cu, kSplitMax);
    d.split32[nt] = choose_split(units, d.Mp / 32, n_cu, kSplitMax);
    d.grid_heur = std::max(d.grid_heur, nt * std::max(d.split16[nt], d.split32[nt]));
    d.grid16 = std::max(d.grid16, nt * d.split16[nt]);
    d.grid32 = std::max(d.grid32, units * d.split32[nt]);
  }
  d.S = d.split16[d.ntiles];
  d.S_lp = d.split32[d.ntiles];
  d.S_cap = std::max(std::max(d.S, d.S_lp), std::min(kSplitTuneMax, d.nblocks));
  d.grid_cap = std::max(d.grid_heur, d.ntiles * d.S_cap);
  return d;
}

// Workgroup shape of the evaluation kernel of `dtype`, and its workgroups
// per split at the full plan capacity.
int eval_shape(const Dims& d, int dtype) {
  if (is_low_precision(dtype)) return d.lp_shape;
  if (dtype == GMCO_DTYPE_F32_ACC64) return d.acc_shape;
  return dtype == GMCO_DTYPE_F32 ? d.f32_shape : 0;
}
int eval_units(const Dims& d, int dtype) {
  if (is_low_precision(dtype)) return (d.ntiles + d.lpt - 1) / d.lpt;
  return (dtype == GMCO_DTYPE_F32_ACC64 && d.acc_shape == 1) ? 2 * d.ntiles : d.ntiles;
}

Layout make_layout(const Dims& d, int G, int m, int dtype, int Pmax) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t MK = (size_t)d.Mp * d.Kp;
  const size_t PK = (size_t)d.Pp * d.Kp;
  L.D64 = take(MK * 8);
  L.D32 = take(MK * 4);
  L.Dlp = take(MK * lp_bytes(dtype));
  L.DTlp = take(is_low_precision(dtype) ? MK * 2 : 0);  // BF16 for the back-projection
  L.colscale = take((size_t)d.Kp * 4);
  L.grp = take((size_t)d.Mp * 4);
  L.perm = take((size_t)d.M * 4);
  L.stage = take((size_t)d.M * d.K * 8 + ((size_t)d.M + d.K) * 3 * 8);
  L.gparams = take(kGmax * 4 * 8);
  L.volume = take(kGmax * 8);
  L.goff = take(kGmax * 4);
  L.gcnt = take(kGmax * 4);
  L.counts = take(kGmax * 4);
  L.gorg = take(kGmax * 4);
  L.D64d = take((size_t)d.Mdp * d.Kp * 8);
  L.dstage = take((size_t)d.Md * 3 * 8);
  L.dperm = take((size_t)d.Md * 4);
  L.doff = take(kGmax * 4);
  L.dcnt = take(kGmax * 4);
  L.t_bar = take(8);
  L.Wst = take((size_t)Pmax * kGmax * 8);
  L.t0st = take((size_t)Pmax * d.K * 8);
  L.xst = take((size_t)Pmax * d.K * 8);
  L.Fst = take((size_t)Pmax * 8);
  L.gst = take((size_t)Pmax * d.K * 8);
  L.wn = take((size_t)d.Pp * kGmax * 4);
  L.W64 = take((size_t)d.Pp * kGmax * 8);
  L.x = take(PK * 4);
  L.g = take(PK * 4);
  L.dir = take(PK * 4);
  L.xt = take(PK * 4);
  L.xe = take(PK * 4);
  L.Sh = take(PK * m * 4);
  L.Yh = take(PK * m * 4);
  L.rho = take((size_t)d.Pp * m * 8);
  L.ps = take((size_t)d.Pp * sizeof(PlanState));
  L.Gpart = take((size_t)d.grid_cap * kPT * d.Kp * 4);
  L.Fpart = take((size_t)d.grid_cap * kPT * 8);
  L.flag = take((size_t)d.Pp * 4);
  L.slot = take((size_t)d.Pp * 4);
  L.rt = take(sizeof(RoundTable));
  L.split_tab = take((size_t)2 * (d.ntiles + 1) * 4);
  L.active = take(2 * sizeof(int));
  L.work = take(2 * sizeof(unsigned long long));
  L.t64 = take(PK * 8);
  // final doses (Pp x Mp, then Pp x Mdp for the DVH points); an FP8 context
  // also widens its matrix (Mp x Kp) here
  L.d64 = take(std::max((size_t)d.Pp * std::max(d.Mp, d.Mdp),
                        (size_t)(dtype == GMCO_DTYPE_FP8 ? d.Kp : 0) * d.Mp) * 8);
  L.metrics = take((size_t)d.Pp * sizeof(gmco_plan_metrics));
  L.hist = take(kGmax * 16 * 4);
  L.sel = take((size_t)d.Pp * 3 * 4 + 16);
  L.feat = take(kGmax * 16 * 4);
  L.mlpX = take((size_t)Pmax * 17 * kGmax * 4);  // network inputs: weights + 16 features per organ
  L.mlpY = take((size_t)Pmax * d.K * 4);
  L.Fu = take((size_t)Pmax * 8);
  L.usewarm = take((size_t)Pmax * 4);
  L.nwarm = take(sizeof(int));
  (void)G;
  L.total = off;
  return L;
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

int copy_h2d(gmco_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return GMCO_OK;
  GMCO_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  return GMCO_OK;
}

// compacted: the evaluation ranks the running plans itself and decides the
// round's tiles and split; otherwise every plan, host split.
EvalArgs eval_args(const gmco_ctx* c, const float* x, bool compacted, int dtype) {
  EvalArgs a{};
  a.D = is_low_precision(dtype) ? c->at<void>(c->lay.Dlp) : c->at<void>(c->lay.D32);
  a.DT = c->at<void>(c->lay.DTlp);
  a.colscale = c->at<float>(c->lay.colscale);
  a.grp = c->at<int>(c->lay.grp);
  a.x = x;
  a.wn = c->at<float>(c->lay.wn);
  const Dims& d = c->dim;
  const bool lp = is_low_precision(dtype);
  const int units = eval_units(d, dtype);
  if (compacted) {
    a.flag = c->at<int>(c->lay.flag);
    a.split_tab = c->at<int>(c->lay.split_tab) + (is_low_precision(dtype) ? c->dim.ntiles + 1 : 0);
    a.slot = c->at<int>(c->lay.slot);
    a.rt = c->at<RoundTable>(c->lay.rt);
    a.work = c->at<unsigned long long>(c->lay.work);
    a.P = c->P;
    a.s_tuned = lp ? d.S_tuned_lp : d.S_tuned;
  }
  a.Gpart = c->at<float>(c->lay.Gpart);
  a.Fpart = c->at<double>(c->lay.Fpart);
  a.Mp = c->dim.Mp;
  a.Kp = c->dim.Kp;
  a.Pp = c->dim.Pp;
  a.nblocks = c->dim.nblocks;
  a.S = lp ? d.S_lp : d.S;
  a.ntiles = d.ntiles;
  // a half-tile workgroup doubles the grid of every split
  const int grid_max = lp ? d.grid32 : d.grid16 * (units / d.ntiles);
  a.grid = compacted ? std::max(grid_max, units * (lp ? d.S_tuned_lp : d.S_tuned)) : a.S * units;
  a.lp_shape = eval_shape(d, dtype);
  a.xcd_map = lp ? d.xcd_lp : d.xcd32;
  a.last16 = d.K > d.Kp - 16 ? 1 : 0;
  a.gt = c->gt;
  return a;
}

UpdateArgs update_args(gmco_ctx* c, const gmco_run* r) {
  const Layout& L = c->lay;
  const Dims& d = c->dim;
  UpdateArgs u{};
  u.Gpart = c->at<float>(L.Gpart);
  u.Fpart = c->at<double>(L.Fpart);
  u.x = c->at<float>(L.x);
  u.g = c->at<float>(L.g);
  u.dir = c->at<float>(L.dir);
  u.xt = c->at<float>(L.xt);
  u.Sh = c->at<float>(L.Sh);
  u.Yh = c->at<float>(L.Yh);
  u.rho = c->at<double>(L.rho);
  u.ps = c->at<PlanState>(L.ps);
  u.active_count = c->at<int>(L.active);
  u.slot = c->at<int>(L.slot);
  u.flag = c->at<int>(L.flag);
  u.rt = c->at<RoundTable>(L.rt);
  u.Kp = d.Kp;
  u.Pp = d.Pp;
  u.m = c->m;
  u.K = d.K;
  u.max_iter = r->max_iter;
  u.max_ls = r->max_ls;
  u.eps = r->eps;
  u.c1 = r->c1;
  u.beta = r->beta;
  return u;
}

int check_run(gmco_ctx* c, const gmco_run* r, int* dtype) {
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  if (r->max_iter < 0 || !(r->eps >= 0.0) || !(r->c1 > 0.0) || !(r->beta > 0.0 && r->beta < 1.0) ||
      r->max_ls < 1 || r->check_every < 0)
    return fail(c, GMCO_EINVAL, "bad run options");
  *dtype = r->dtype < 0 ? c->dtype : r->dtype;
  if (!dtype_available(c->dtype, *dtype))
    return fail(c, GMCO_EINVAL, "run dtype needs a context created with that dtype");
  return GMCO_OK;
}

int summarize(gmco_ctx* c, long long rounds, float ms, double eval_ms, double update_ms,
              unsigned long long work, gmco_run_info* info) {
  std::vector<PlanState> ps(c->P);
  GMCO_HIP(c, hipMemcpy(ps.data(), c->at<void>(c->lay.ps), (size_t)c->P * sizeof(PlanState), hipMemcpyDeviceToHost));
  gmco_run_info inf{};
  inf.rounds = (int)rounds;
  for (const PlanState& s : ps) {
    inf.n_converged += s.status == ST_CONVERGED;
    inf.n_maxiter += s.status == ST_MAXITER;
    inf.n_ls_fail += s.status == ST_LSFAIL;
    inf.n_nonfinite += s.status == ST_NONFINITE;
    inf.max_iters = std::max(inf.max_iters, s.iter);
  }
  inf.device_ms = ms;
  inf.eval_ms = (float)eval_ms;
  inf.update_ms = (float)update_ms;
  inf.eval_launches = (int)rounds;
  inf.eval_work = (double)work / (double)c->P;  // plan evaluations / batch size
  if (info) *info = inf;
  if (inf.n_nonfinite == c->P) return fail(c, GMCO_ENUMERIC, "every plan has a non-finite objective");
  return GMCO_OK;
}

}  // namespace

extern "C" {

const char* gmco_strerror(int s) {
  switch (s) {
    case GMCO_OK: return "ok";
    case GMCO_EINVAL: return "invalid argument";
    case GMCO_ENOMEM: return "out of device memory or workspace too small";
    case GMCO_EHIP: return "HIP runtime error";
    case GMCO_ESTATE: return "call out of order";
    case GMCO_ENUMERIC: return "every plan is non-finite";
    case GMCO_ENOLIB: return "no usable gfx950 device";
    default: return "unknown status";
  }
}

const char* gmco_last_error(const gmco_ctx* c) { return c ? c->err.c_str() : "null context"; }

int gmco_create(gmco_ctx** out, const gmco_opts* o) {
  if (!out || !o) return GMCO_EINVAL;
  *out = nullptr;
  if (o->dtype < GMCO_DTYPE_F32 || o->dtype > GMCO_DTYPE_F32_CHUNK64) return GMCO_EINVAL;
  if (o->history < 1 || o->history > GMCO_MAX_HISTORY) return GMCO_EINVAL;
  if (o->max_plans < 1 || o->max_plans > (1 << 20)) return GMCO_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GMCO_ENOLIB;
  if (o->device < 0 || o->device >= ndev) return GMCO_EINVAL;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, o->device) != hipSuccess) return GMCO_EHIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GMCO_ENOLIB;
  gmco_ctx* c = new (std::nothrow) gmco_ctx();
  if (!c) return GMCO_ENOMEM;
  c->device = o->device;
  c->dtype = o->dtype;
  c->m = o->history;
  c->Pmax = o->max_plans;
  c->n_cu = prop.multiProcessorCount;
  if (hipSetDevice(c->device) != hipSuccess ||
      hipHostMalloc((void**)&c->host_count, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    gmco_destroy(c);
    return GMCO_EHIP;
  }
  *out = c;
  return GMCO_OK;
}

int gmco_destroy(gmco_ctx* c) {
  if (!c) return GMCO_OK;
  // best-effort teardown: errors here have no caller to go to
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->ws_owned && c->ws) (void)hipFree(c->ws);
  if (c->host_count) (void)hipHostFree(c->host_count);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->gev) (void)hipEventDestroy(c->gev);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  delete c;
  return GMCO_OK;
}

int gmco_set_stream(gmco_ctx* c, void* stream) {
  if (!c) return GMCO_EINVAL;
  c->stream = static_cast<hipStream_t>(stream);
  return GMCO_OK;
}

int gmco_workspace_bytes(const gmco_ctx* c, int M, int K, int Md, size_t* bytes) {
  if (!c || !bytes || M < 1 || K < 1 || K > GMCO_MAX_DWELLS || Md < 0) return GMCO_EINVAL;
  const Dims d = make_dims(M, K, c->Pmax, c->n_cu, Md);
  *bytes = make_layout(d, kGmax, c->m, c->dtype, c->Pmax).total;
  return GMCO_OK;
}

int gmco_bind_workspace(gmco_ctx* c, void* ptr, size_t bytes) {
  if (!c) return GMCO_EINVAL;
  if (ptr && (reinterpret_cast<uintptr_t>(ptr) & 255u)) return fail(c, GMCO_EINVAL, "workspace must be 256-byte aligned");
  c->bound = ptr;
  c->bound_bytes = ptr ? bytes : 0;
  return GMCO_OK;
}

int gmco_load_case(gmco_ctx* c, const gmco_case* cs) {
  if (!c || !cs) return GMCO_EINVAL;
  const int M = cs->n_points, K = cs->n_dwells, G = cs->n_groups;
  if (M < 1 || K < 1 || K > GMCO_MAX_DWELLS) return fail(c, GMCO_EINVAL, "n_points >= 1 and 1 <= n_dwells <= 512 required");
  if (G < 1 || G > kGmax) return fail(c, GMCO_EINVAL, "n_groups must be 1..8");
  if (!cs->group || !cs->group_params || !cs->dwell_xyz || (!cs->point_xyz && !cs->dose_rate))
    return fail(c, GMCO_EINVAL, "missing case array");
  if (!(cs->prescription_gy > 0.0) || !std::isfinite(cs->prescription_gy))
    return fail(c, GMCO_EINVAL, "prescription must be > 0");
  // organs: the hidden weight and the point count of eq. (obj) are per organ
  const int O = cs->group_organ ? cs->n_organs : G;
  if (O < 1 || O > G) return fail(c, GMCO_EINVAL, "n_organs must be 1..n_groups");
  std::vector<int> gorg(kGmax, 0);
  for (int j = 0; j < G; ++j) {
    gorg[j] = cs->group_organ ? cs->group_organ[j] : j;
    if (gorg[j] < 0 || gorg[j] >= O) return fail(c, GMCO_EINVAL, "group_organ out of range");
  }
  const int Md = cs->n_dvh_points;
  if (Md < 0) return fail(c, GMCO_EINVAL, "n_dvh_points must be >= 0");
  if (Md > 0 && (!cs->dvh_xyz || !cs->dvh_organ)) return fail(c, GMCO_EINVAL, "DVH points need dvh_xyz and dvh_organ");
  if (Md > 0 && !finite_all(cs->dvh_xyz, (size_t)Md * 3)) return fail(c, GMCO_EINVAL, "non-finite DVH point position");
  std::vector<int> dcounts(kGmax, 0);
  for (int i = 0; i < Md; ++i) {
    const int o = cs->dvh_organ[i];
    if (o < 0 || o >= O) return fail(c, GMCO_EINVAL, "dvh_organ out of range");
    dcounts[o] += 1;
  }
  if (cs->target_group < 0 || cs->target_group >= O) return fail(c, GMCO_EINVAL, "target_group out of range");
  if (!finite_all(cs->group_params, (size_t)G * 4)) return fail(c, GMCO_EINVAL, "non-finite group parameter");
  for (int j = 0; j < G; ++j) {
    const double* p = cs->group_params + 4 * j;
    if (p[0] < 0 || p[3] < 0 || p[1] > p[2]) return fail(c, GMCO_EINVAL, "group parameters need w >= 0 and D_min <= D_max");
  }
  if (!finite_all(cs->dwell_xyz, (size_t)K * 3)) return fail(c, GMCO_EINVAL, "non-finite dwell position");
  if (cs->point_xyz && !finite_all(cs->point_xyz, (size_t)M * 3)) return fail(c, GMCO_EINVAL, "non-finite point position");
  if (cs->dose_rate) {
    for (size_t i = 0; i < (size_t)M * K; ++i)
      if (!std::isfinite(cs->dose_rate[i]) || cs->dose_rate[i] < 0.0) return fail(c, GMCO_EINVAL, "dose_rate must be finite and >= 0");
  }
  std::vector<int> counts(kGmax, 0);
  for (int i = 0; i < M; ++i) {
    const int g = cs->group[i];
    if (g < 0 || g >= G) return fail(c, GMCO_EINVAL, "group index out of range");
    counts[g] += 1;
  }
  std::vector<int> ocounts(kGmax, 0);
  for (int j = 0; j < G; ++j) ocounts[gorg[j]] += counts[j];
  if (ocounts[cs->target_group] == 0) return fail(c, GMCO_EINVAL, "target structure has no points");

  GMCO_HIP(c, hipSetDevice(c->device));
  const Dims d = make_dims(M, K, c->Pmax, c->n_cu, Md);
  const Layout L = make_layout(d, G, c->m, c->dtype, c->Pmax);
  // arena: bound workspace, else a library allocation (reused when big enough)
  if (c->bound) {
    if (c->bound_bytes < L.total) return fail(c, GMCO_ENOMEM, "bound workspace smaller than gmco_workspace_bytes");
    if (c->ws_owned && c->ws) (void)hipFree(c->ws);  // (the old arena; nothing to report)
    c->ws = c->bound;
    c->ws_bytes = c->bound_bytes;
    c->ws_owned = false;
  } else if (!c->ws_owned || c->ws_bytes < L.total) {
    if (c->ws_owned && c->ws) {
      GMCO_HIP(c, hipStreamSynchronize(c->stream));
      GMCO_HIP(c, hipFree(c->ws));
    }
    c->ws = nullptr;
    c->ws_owned = false;
    if (hipMalloc(&c->ws, L.total) != hipSuccess) {
      c->ws = nullptr;
      c->ws_bytes = 0;
      return fail(c, GMCO_ENOMEM, "hipMalloc of the device arena failed");
    }
    c->ws_owned = true;
    c->ws_bytes = L.total;
  }
  c->dim = d;
  // BF16: the role-split workgroup where it exists (measured faster at the
  // paper-scale case; FP8 keeps shape 0, which measured as fast)
  if (c->dtype == GMCO_DTYPE_BF16 && lp_shape_ok(d.Kp, 2)) c->dim.lp_shape = 2;
  // FP64-accumulated dose from 448 padded dwells: the role-split workgroup,
  // which needs no register spill there (shape 0 spills; 655 against 784 us
  // per full evaluation measured at 512 dwells; shape 0 stays ahead at 416)
  if (d.Kp >= 448) c->dim.acc_shape = 3;
  c->lay = L;
  c->G = G;
  c->O = O;
  c->rx = cs->prescription_gy;
  c->target = cs->target_group;
  c->case_loaded = false;
  c->P = 0;

  // points ordered by organ, then group (stable): every organ is one range
  std::vector<int> kcur(kGmax * kGmax + 1, 0);  // (organ, group) key offsets
  for (int j = 0; j < G; ++j) kcur[gorg[j] * kGmax + j + 1] += counts[j];
  for (int k = 1; k <= kGmax * kGmax; ++k) kcur[k] += kcur[k - 1];
  c->counts = ocounts;
  c->offsets.assign(kGmax, 0);
  for (int o = 0; o < kGmax; ++o) c->offsets[o] = kcur[o * kGmax];
  c->perm.assign(M, 0);
  for (int i = 0; i < M; ++i) c->perm[kcur[gorg[cs->group[i]] * kGmax + cs->group[i]]++] = i;
  std::vector<int> grp(d.Mp, kGmax);
  for (int i = 0; i < M; ++i) grp[i] = cs->group[c->perm[i]];
  std::vector<int> norm(kGmax, 0);  // N_pnt of each group's organ
  for (int j = 0; j < G; ++j) norm[j] = ocounts[gorg[j]];
  // DVH points ordered by organ
  std::vector<int> doff(kGmax, 0), dperm(Md, 0);
  for (int o = 1; o < kGmax; ++o) doff[o] = doff[o - 1] + dcounts[o - 1];
  {
    std::vector<int> cur(doff);
    for (int i = 0; i < Md; ++i) dperm[cur[cs->dvh_organ[i]]++] = i;
  }

  double* stage = c->at<double>(L.stage);
  double* st_D = stage;                         // M*K
  double* st_dw = stage + (size_t)M * K;        // K*3
  double* st_pt = st_dw + (size_t)K * 3;        // M*3
  int rc;
  if ((rc = copy_h2d(c, c->at<void>(L.perm), c->perm.data(), (size_t)M * 4))) return rc;
  if ((rc = copy_h2d(c, c->at<void>(L.grp), grp.data(), (size_t)d.Mp * 4))) return rc;
  if ((rc = copy_h2d(c, st_dw, cs->dwell_xyz, (size_t)K * 3 * 8))) return rc;
  if (cs->point_xyz && (rc = copy_h2d(c, st_pt, cs->point_xyz, (size_t)M * 3 * 8))) return rc;
  if (cs->dose_rate && (rc = copy_h2d(c, st_D, cs->dose_rate, (size_t)M * K * 8))) return rc;
  std::vector<double> gp(kGmax * 4, 0.0), vol(kGmax, 0.0);
  std::copy(cs->group_params, cs->group_params + 4 * G, gp.begin());
  if (cs->group_volume_cc) std::copy(cs->group_volume_cc, cs->group_volume_cc + O, vol.begin());
  if ((rc = copy_h2d(c, c->at<void>(L.gparams), gp.data(), gp.size() * 8))) return rc;
  if ((rc = copy_h2d(c, c->at<void>(L.volume), vol.data(), vol.size() * 8))) return rc;
  if ((rc = copy_h2d(c, c->at<void>(L.goff), c->offsets.data(), kGmax * 4))) return rc;
  if ((rc = copy_h2d(c, c->at<void>(L.gcnt), ocounts.data(), kGmax * 4))) return rc;
  if ((rc = copy_h2d(c, c->at<void>(L.counts), norm.data(), kGmax * 4))) return rc;
  if ((rc = copy_h2d(c, c->at<void>(L.gorg), gorg.data(), kGmax * 4))) return rc;
  if ((rc = copy_h2d(c, c->at<void>(L.doff), doff.data(), kGmax * 4))) return rc;
  if ((rc = copy_h2d(c, c->at<void>(L.dcnt), dcounts.data(), kGmax * 4))) return rc;
  if (Md > 0) {
    if ((rc = copy_h2d(c, c->at<void>(L.dperm), dperm.data(), (size_t)Md * 4))) return rc;
    if ((rc = copy_h2d(c, c->at<void>(L.dstage), cs->dvh_xyz, (size_t)Md * 3 * 8))) return rc;
  }
  // (host vectors of this call stay alive until the stream synchronisation below)
  std::vector<int> split_tab(d.split16);
  split_tab.insert(split_tab.end(), d.split32.begin(), d.split32.end());
  if ((rc = copy_h2d(c, c->at<void>(L.split_tab), split_tab.data(), split_tab.size() * 4))) return rc;
  for (int j = 0; j <= kGmax; ++j) {
    for (int k = 0; k < 4; ++k) c->gt.prm64[j][k] = j < G ? gp[4 * j + k] : 0.0;
    c->gt.prm[j] = make_float4((float)c->gt.prm64[j][0], (float)c->gt.prm64[j][1],
                               (float)c->gt.prm64[j][2], (float)c->gt.prm64[j][3]);
  }

  GMCO_HIP(c, launch_dose_rate(st_dw, cs->point_xyz ? st_pt : nullptr, cs->dose_rate ? st_D : nullptr,
                               c->at<int>(L.perm), M, K, d.Mp, d.Kp, c->at<double>(L.D64), c->stream));
  GMCO_HIP(c, launch_cast_dose(c->at<double>(L.D64), d.Mp, d.Kp, c->dtype, c->at<float>(L.D32),
                               c->at<void>(L.Dlp), c->at<void>(L.DTlp), c->at<float>(L.colscale),
                               c->stream));
  if (Md > 0)  // the DVH points: point-source law, organ order
    GMCO_HIP(c, launch_dose_rate(st_dw, c->at<double>(L.dstage), nullptr, c->at<int>(L.dperm), Md, K,
                                 d.Mdp, d.Kp, c->at<double>(L.D64d), c->stream));
  const int r0 = c->offsets[cs->target_group];
  GMCO_HIP(c, launch_start_time(c->at<double>(L.D64), d.Kp, r0, r0 + ocounts[cs->target_group], c->rx,
                                c->at<double>(L.t_bar), c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  c->has_points = cs->point_xyz != nullptr;
  c->case_loaded = true;
  return GMCO_OK;
}

int gmco_set_weights(gmco_ctx* c, int P, const double* W, const double* t0) {
  if (!c || !W) return GMCO_EINVAL;
  if (!c->case_loaded) return fail(c, GMCO_ESTATE, "gmco_load_case first");
  if (P < 1 || P > c->Pmax) return fail(c, GMCO_EINVAL, "n_plans out of 1..max_plans");
  const int O = c->O, K = c->dim.K;
  for (size_t i = 0; i < (size_t)P * O; ++i)
    if (!std::isfinite(W[i]) || W[i] < 0.0) return fail(c, GMCO_EINVAL, "weights must be finite and >= 0");
  if (t0) {
    for (size_t i = 0; i < (size_t)P * K; ++i)
      if (!std::isfinite(t0[i]) || !(t0[i] > 0.0)) return fail(c, GMCO_EINVAL, "t0 must be finite and > 0");
  }
  GMCO_HIP(c, hipSetDevice(c->device));
  const Layout& L = c->lay;
  int rc;
  if ((rc = copy_h2d(c, c->at<void>(L.Wst), W, (size_t)P * O * 8))) return rc;
  if (t0 && (rc = copy_h2d(c, c->at<void>(L.t0st), t0, (size_t)P * K * 8))) return rc;
  GMCO_HIP(c, launch_init_plans(P, c->dim.Pp, K, c->dim.Kp, t0 ? c->at<double>(L.t0st) : nullptr,
                                c->at<double>(L.t_bar), c->at<double>(L.Wst), c->G, O, c->at<int>(L.gorg),
                                c->at<int>(L.counts),
                                c->at<float>(L.xt), c->at<float>(L.x), c->at<float>(L.wn),
                                c->at<double>(L.W64), c->at<PlanState>(L.ps), c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  c->P = P;
  return GMCO_OK;
}

int gmco_evaluate(gmco_ctx* c, const double* x, double* F, double* g) {
  if (!c || !x || !F || !g) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  const int P = c->P, K = c->dim.K;
  if (!finite_all(x, (size_t)P * K)) return fail(c, GMCO_EINVAL, "x must be finite");
  GMCO_HIP(c, hipSetDevice(c->device));
  const Layout& L = c->lay;
  int rc;
  if ((rc = copy_h2d(c, c->at<void>(L.xst), x, (size_t)P * K * 8))) return rc;
  GMCO_HIP(c, launch_x_to_device(c->at<double>(L.xst), P, c->dim.Pp, K, c->dim.Kp, c->at<float>(L.xe), c->stream));
  EvalArgs a = eval_args(c, c->at<float>(L.xe), false, c->dtype);
  GMCO_HIP(c, launch_eval(a, c->dtype, c->stream));
  GMCO_HIP(c, launch_finish_eval(a.Gpart, a.Fpart, c->at<float>(L.xe), a.S, P, c->dim.Pp, K,
                                 c->dim.Kp, c->at<double>(L.Fst), c->at<double>(L.gst), c->stream));
  GMCO_HIP(c, hipMemcpyAsync(F, c->at<void>(L.Fst), (size_t)P * 8, hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipMemcpyAsync(g, c->at<void>(L.gst), (size_t)P * K * 8, hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  return GMCO_OK;
}

int gmco_set_weights_learned(gmco_ctx* c, gmco_mlp* net, int P, const double* W, double x_floor, int* use_warm,
                             int* n_warm) {
  if (!c || !net || !W) return GMCO_EINVAL;
  if (!c->case_loaded) return fail(c, GMCO_ESTATE, "gmco_load_case first");
  if (!c->has_points) return fail(c, GMCO_EINVAL, "the learned start needs point positions (case features)");
  if (!(x_floor > 0.0) || !std::isfinite(x_floor)) return fail(c, GMCO_EINVAL, "x_floor must be finite and > 0");
  if (mlp_device(net) != c->device) return fail(c, GMCO_EINVAL, "network and context on different devices");
  if (mlp_inputs(net) != c->O * 17 || mlp_outputs(net) != c->dim.K)
    return fail(c, GMCO_EINVAL, "network needs 17 x n_organs inputs and n_dwells outputs");
  // the uniform start first (validates P and W)
  int rc = gmco_set_weights(c, P, W, nullptr);
  if (rc) return rc;
  const Layout& L = c->lay;
  const Dims& d = c->dim;
  // objective at the uniform start
  EvalArgs a = eval_args(c, c->at<float>(L.x), false, c->dtype);
  GMCO_HIP(c, launch_eval(a, c->dtype, c->stream));
  GMCO_HIP(c, launch_finish_eval(a.Gpart, a.Fpart, a.x, a.S, P, d.Pp, d.K, d.Kp, c->at<double>(L.Fu),
                                 c->at<double>(L.gst), c->stream));
  // network inputs (weights, case features), its prediction, the floored start
  const double* dw = c->at<double>(L.stage) + (size_t)d.M * d.K;
  const double* pts = dw + (size_t)d.K * 3;
  GMCO_HIP(c, launch_features(dw, pts, c->at<int>(L.perm), c->at<int>(L.goff), c->at<int>(L.gcnt), d.K, c->O,
                              c->at<unsigned>(L.hist), c->at<float>(L.feat), c->stream));
  GMCO_HIP(c, launch_learned_inputs(c->at<double>(L.W64), c->at<float>(L.feat), P, c->O, c->at<float>(L.mlpX),
                                    c->stream));
  GMCO_HIP(c, mlp_forward_device(net, P, c->at<float>(L.mlpX), c->at<float>(L.mlpY), c->stream));
  GMCO_HIP(c, launch_learned_start(c->at<float>(L.mlpY), P, d.Pp, d.K, d.Kp, c->at<double>(L.t_bar), x_floor,
                                   c->at<float>(L.xe), c->stream));
  // objective at the learned start, and the choice per plan
  a = eval_args(c, c->at<float>(L.xe), false, c->dtype);
  GMCO_HIP(c, launch_eval(a, c->dtype, c->stream));
  GMCO_HIP(c, launch_finish_eval(a.Gpart, a.Fpart, a.x, a.S, P, d.Pp, d.K, d.Kp, c->at<double>(L.Fst),
                                 c->at<double>(L.gst), c->stream));
  int* nw = c->at<int>(L.nwarm);
  GMCO_HIP(c, hipMemsetAsync(nw, 0, sizeof(int), c->stream));
  GMCO_HIP(c, launch_pick_start(c->at<double>(L.Fst), c->at<double>(L.Fu), c->at<float>(L.xe), P, d.Kp,
                                c->at<float>(L.x), c->at<float>(L.xt), nw, c->at<int>(L.usewarm), c->stream));
  int h = 0;
  GMCO_HIP(c, hipMemcpyAsync(&h, nw, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  if (use_warm)
    GMCO_HIP(c, hipMemcpyAsync(use_warm, c->at<int>(L.usewarm), (size_t)P * 4, hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  if (n_warm) *n_warm = h;
  return GMCO_OK;
}

int gmco_optimize(gmco_ctx* c, const gmco_run* r, gmco_run_info* info) {
  if (!c || !r) return GMCO_EINVAL;
  int dtype = 0;
  int rc = check_run(c, r, &dtype);
  if (rc) return rc;
  GMCO_HIP(c, hipSetDevice(c->device));
  const Layout& L = c->lay;
  const Dims& d = c->dim;
  int* active = c->at<int>(L.active);
  unsigned long long* work = c->at<unsigned long long>(L.work);  // [0] all launches, [1] timed ones
  GMCO_HIP(c, hipMemsetAsync(active, 0, 2 * sizeof(int), c->stream));
  GMCO_HIP(c, hipMemsetAsync(work, 0, 2 * sizeof(unsigned long long), c->stream));
  GMCO_HIP(c, launch_resume(c->at<PlanState>(L.ps), c->at<float>(L.x), c->at<float>(L.xt), c->at<int>(L.flag), d.Pp, d.Kp,
                            r->max_iter, r->resume_stopped, c->stream));
  UpdateArgs u = update_args(c, r);
  EvalArgs a = eval_args(c, c->at<float>(L.xt), true, dtype);
  EvalArgs a_timed = a;  // the timed launches also count their work apart
  a_timed.work2 = work + 1;
  const int check = r->check_every > 0 ? r->check_every : 16;
  const long long max_rounds = 1 + (long long)std::max(r->max_iter, 1) * r->max_ls + 1;
  // Rounds are issued in blocks of `check`.  After each block the running-plan
  // count is copied to pinned host memory and an event recorded; the host
  // then waits for the block before last, so the device always has the next
  // block queued and never idles at a check.  When a block reports no running
  // plan, the one queued after it runs as empty rounds (every kernel exits at
  // once) and is not timed.
  // Optional sampled timing: events around the evaluation and the update of
  // every time_kernels-th round, 4 per timed round, one set per block parity.
  const int every = r->time_kernels;
  std::vector<hipEvent_t> ev;
  hipEvent_t bev[2] = {nullptr, nullptr};
  int timed = 0;
  ev.resize((every > 0 ? (size_t)8 * check : 0) + 2, nullptr);
  for (auto& e : ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& f : ev)
        if (f) (void)hipEventDestroy(f);
      return fail(c, GMCO_EHIP, "hipEventCreate failed");
    }
  }
  struct EventGuard {
    std::vector<hipEvent_t>& v;
    ~EventGuard() {
      for (auto& e : v)
        if (e) (void)hipEventDestroy(e);
    }
  } guard{ev};
  bev[0] = ev[ev.size() - 2];
  bev[1] = ev[ev.size() - 1];
  double eval_ms = 0.0, update_ms = 0.0;
  int in_block[2] = {0, 0};
  auto harvest = [&](int set) -> hipError_t {
    const int n = in_block[set];
    hipEvent_t* e = ev.data() + (size_t)set * 4 * check;
    timed += n;
    for (int i = 0; i < n; ++i) {
      float a_ms = 0.f, b_ms = 0.f;
      hipError_t er = hipEventElapsedTime(&a_ms, e[4 * i], e[4 * i + 1]);
      if (er != hipSuccess) return er;
      er = hipEventElapsedTime(&b_ms, e[4 * i + 2], e[4 * i + 3]);
      if (er != hipSuccess) return er;
      eval_ms += a_ms;
      update_ms += b_ms;
    }
    return hipSuccess;
  };
  GMCO_HIP(c, hipEventRecord(c->ev0, c->stream));
  long long round = 0;
  long long blk = 0;  // blocks issued
  bool done_flag = false;
  while (!done_flag) {
    const int set = (int)(blk & 1);
    hipEvent_t* e = every > 0 ? ev.data() + (size_t)set * 4 * check : nullptr;
    in_block[set] = 0;
    for (int k = 0; k < check && round < max_rounds; ++k, ++round) {
      u.round = (int)round;
      const bool tk = every > 0 && round % every == 0;
      const int i = in_block[set];
      if (tk) GMCO_HIP(c, hipEventRecord(e[4 * i], c->stream));
      GMCO_HIP(c, launch_eval(tk ? a_timed : a, dtype, c->stream));
      if (tk) {
        GMCO_HIP(c, hipEventRecord(e[4 * i + 1], c->stream));
        GMCO_HIP(c, hipEventRecord(e[4 * i + 2], c->stream));
      }
      GMCO_HIP(c, launch_update(u, c->stream));
      if (tk) {
        GMCO_HIP(c, hipEventRecord(e[4 * i + 3], c->stream));
        ++in_block[set];
      }
    }
    // running plans after this block's last round (the next update resets the
    // other counter, so the copy is queued before any later round)
    GMCO_HIP(c, hipMemcpyAsync(c->host_count + set, active + ((round - 1) & 1), sizeof(int),
                               hipMemcpyDeviceToHost, c->stream));
    GMCO_HIP(c, hipEventRecord(bev[set], c->stream));
    ++blk;
    if (round >= max_rounds) {  // nothing more to issue: wait for the last block
      GMCO_HIP(c, hipEventSynchronize(bev[set]));
      // the block before it is not harvested yet; the last block ran empty
      // when that one already reported no running plan
      const bool last_empty = blk >= 2 && c->host_count[set ^ 1] == 0;
      if (every > 0 && blk >= 2) GMCO_HIP(c, harvest(set ^ 1));
      if (every > 0 && !last_empty) GMCO_HIP(c, harvest(set));
      done_flag = true;
    } else if (blk >= 2) {  // wait for the block before this one
      const int prev = set ^ 1;
      GMCO_HIP(c, hipEventSynchronize(bev[prev]));
      if (every > 0) GMCO_HIP(c, harvest(prev));
      if (c->host_count[prev] == 0) {
        // the block just queued runs empty: wait for it, do not time it
        GMCO_HIP(c, hipEventSynchronize(bev[set]));
        done_flag = true;
      }
    }
  }
  GMCO_HIP(c, hipEventRecord(c->ev1, c->stream));
  GMCO_HIP(c, hipEventSynchronize(c->ev1));
  unsigned long long done[2] = {0, 0};
  GMCO_HIP(c, hipMemcpy(done, work, sizeof(done), hipMemcpyDeviceToHost));
  float ms = 0.f;
  GMCO_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  rc = summarize(c, round, ms, eval_ms, update_ms, done[0], info);
  if (info) {
    info->timed_launches = timed;
    info->timed_work = (double)done[1] / (double)c->P;
  }
  return rc;
}

int gmco_optimize_many(gmco_ctx* const* ctxs, int n, const gmco_run* r, gmco_run_info* infos,
                       int rounds_per_graph) {
  if (!ctxs || n < 1 || !r || rounds_per_graph < 0) return GMCO_EINVAL;
  gmco_ctx* c0 = ctxs[0];
  if (!c0) return GMCO_EINVAL;
  std::vector<int> dtypes(n);
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return GMCO_EINVAL;
    if (ctxs[i]->device != c0->device) return fail(ctxs[i], GMCO_EINVAL, "contexts must share one device");
    int rc = check_run(ctxs[i], r, &dtypes[i]);
    if (rc) return rc;
  }
  GMCO_HIP(c0, hipSetDevice(c0->device));
  // all work of the batch runs on a library-owned stream (graph capture needs
  // a stream of its own), ordered after and before the caller's stream
  if (!c0->gstream) {
    GMCO_HIP(c0, hipStreamCreateWithFlags(&c0->gstream, hipStreamNonBlocking));
    GMCO_HIP(c0, hipEventCreateWithFlags(&c0->gev, hipEventDisableTiming));
  }
  hipStream_t st = c0->gstream;
  GMCO_HIP(c0, hipEventRecord(c0->gev, c0->stream));
  GMCO_HIP(c0, hipStreamWaitEvent(st, c0->gev, 0));
  const int R = rounds_per_graph > 0 ? (rounds_per_graph + 1) / 2 * 2 : 0;  // even: counter parity
  std::vector<UpdateArgs> us(n);
  std::vector<EvalArgs> as(n);
  for (int i = 0; i < n; ++i) {
    gmco_ctx* c = ctxs[i];
    const Layout& L = c->lay;
    GMCO_HIP(c, hipMemsetAsync(c->at<int>(L.active), 0, 2 * sizeof(int), st));
    GMCO_HIP(c, hipMemsetAsync(c->at<unsigned long long>(L.work), 0, sizeof(unsigned long long), st));
    GMCO_HIP(c, launch_resume(c->at<PlanState>(L.ps), c->at<float>(L.x), c->at<float>(L.xt), c->at<int>(L.flag), c->dim.Pp,
                              c->dim.Kp, r->max_iter, r->resume_stopped, st));
    us[i] = update_args(c, r);
    as[i] = eval_args(c, c->at<float>(L.xt), true, dtypes[i]);
  }
  const long long max_rounds = 1 + (long long)std::max(r->max_iter, 1) * r->max_ls + 1;
  // Grouped launches: the cases' evaluations by (padded dwells, dtype), one
  // reduction for all, the updates by (update width, history capacity); the
  // argument tables live in one device buffer for the call.
  const bool grouped = r->per_case_launches == 0 && n > 1;
  struct Bucket {
    int key0, key1, key2;     // (Kp, dtype, BF16 / FP8 shape) or (E, MH, 0)
    std::vector<int> cases;
    int off = 0, soff = 0, grid = 0, pp_max = 0;
  };
  std::vector<Bucket> eb, ub;
  void* dtab = nullptr;
  struct TabGuard {
    void*& p;
    ~TabGuard() {
      if (p) (void)hipFree(p);
    }
  } tab_guard{dtab};
  EvalArgs* d_eargs = nullptr;
  int* d_start = nullptr;
  UpdateArgs* d_uargs = nullptr;
  if (grouped) {
    auto bucket_of = [](std::vector<Bucket>& v, int k0, int k1, int k2) -> Bucket& {
      for (Bucket& b : v)
        if (b.key0 == k0 && b.key1 == k1 && b.key2 == k2) return b;
      v.push_back(Bucket{k0, k1, k2, {}});
      return v.back();
    };
    auto mh = [](int m) { return m <= 4 ? 4 : (m <= 10 ? 10 : (m <= 16 ? 16 : GMCO_MAX_HISTORY)); };
    for (int i = 0; i < n; ++i) {
      bucket_of(eb, ctxs[i]->dim.Kp, dtypes[i], as[i].lp_shape).cases.push_back(i);
      bucket_of(ub, update_width(ctxs[i]->dim.Kp), mh(ctxs[i]->m), 0).cases.push_back(i);
    }
    std::vector<EvalArgs> he;
    std::vector<int> hs;
    for (Bucket& b : eb) {
      b.off = (int)he.size();
      b.soff = (int)hs.size();
      int g = 0;
      for (int i : b.cases) {
        he.push_back(as[i]);
        hs.push_back(g);
        g += (as[i].grid + 7) / 8 * 8;  // each case starts on a multiple of 8 (XCD placement)
      }
      hs.push_back(g);
      b.grid = g;
    }
    std::vector<UpdateArgs> hu;
    for (Bucket& b : ub) {
      b.off = (int)hu.size();
      for (int i : b.cases) {
        hu.push_back(us[i]);
        b.pp_max = std::max(b.pp_max, ctxs[i]->dim.Pp);
      }
    }
    const size_t be = align256(he.size() * sizeof(EvalArgs)), bs = align256(hs.size() * sizeof(int));
    const size_t bu = align256(hu.size() * sizeof(UpdateArgs));
    if (hipMalloc(&dtab, be + bs + bu) != hipSuccess) {
      dtab = nullptr;
      return fail(c0, GMCO_ENOMEM, "argument tables of the grouped launches");
    }
    char* base = static_cast<char*>(dtab);
    d_eargs = reinterpret_cast<EvalArgs*>(base);
    d_start = reinterpret_cast<int*>(base + be);
    d_uargs = reinterpret_cast<UpdateArgs*>(base + be + bs);
    GMCO_HIP(c0, hipMemcpyAsync(d_eargs, he.data(), he.size() * sizeof(EvalArgs), hipMemcpyHostToDevice, st));
    GMCO_HIP(c0, hipMemcpyAsync(d_start, hs.data(), hs.size() * sizeof(int), hipMemcpyHostToDevice, st));
    GMCO_HIP(c0, hipMemcpyAsync(d_uargs, hu.data(), hu.size() * sizeof(UpdateArgs), hipMemcpyHostToDevice, st));
    GMCO_HIP(c0, hipStreamSynchronize(st));  // the host tables above are freed on return
  }
  auto issue_round = [&](long long rd) -> int {
    if (grouped) {
      for (const Bucket& b : eb)
        GMCO_HIP(c0, launch_eval_grouped(d_eargs + b.off, d_start + b.soff, (int)b.cases.size(), b.grid, b.key0,
                                         b.key1, b.key2, st));
      for (const Bucket& b : ub)
        GMCO_HIP(c0, launch_update_grouped(d_uargs + b.off, (int)b.cases.size(), b.key0, b.pp_max, b.key1,
                                           (int)rd, st));
      return GMCO_OK;
    }
    for (int i = 0; i < n; ++i) {
      us[i].round = (int)rd;
      GMCO_HIP(ctxs[i], launch_eval(as[i], dtypes[i], st));
      GMCO_HIP(ctxs[i], launch_update(us[i], st));
    }
    return GMCO_OK;
  };
  // After each block of rounds the running-plan counts go to pinned host
  // memory (slot = block parity) with an event; the host waits for the block
  // before last, so the next block is always queued (as in gmco_optimize).
  hipEvent_t bev[2] = {nullptr, nullptr};
  struct BevGuard {
    hipEvent_t* e;
    ~BevGuard() {
      for (int k = 0; k < 2; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
    }
  } bev_guard{bev};
  for (int k = 0; k < 2; ++k)
    GMCO_HIP(c0, hipEventCreateWithFlags(&bev[k], hipEventDisableTiming));
  auto post_counts = [&](int slot, long long last_round) -> int {
    for (int i = 0; i < n; ++i)
      GMCO_HIP(ctxs[i], hipMemcpyAsync(ctxs[i]->host_count + slot,
                                       ctxs[i]->at<int>(ctxs[i]->lay.active) + (last_round & 1), sizeof(int),
                                       hipMemcpyDeviceToHost, st));
    GMCO_HIP(c0, hipEventRecord(bev[slot], st));
    return GMCO_OK;
  };
  auto all_done = [&](int slot) -> int {  // 1 done, 0 not, < 0 error
    GMCO_HIP(c0, hipEventSynchronize(bev[slot]));
    long long tot = 0;
    for (int i = 0; i < n; ++i) tot += ctxs[i]->host_count[slot];
    return tot == 0 ? 1 : 0;
  };
  // one block issued: post its counts, then decide on the block before it
  long long blk = 0;
  auto after_block = [&](long long last_round, bool at_max) -> int {  // 1 stop, 0 go on
    const int slot = (int)(blk & 1);
    int rc2 = post_counts(slot, last_round);
    if (rc2) return rc2;
    ++blk;
    if (at_max) {
      GMCO_HIP(c0, hipEventSynchronize(bev[slot]));
      return 1;
    }
    if (blk < 2) return 0;
    const int dn = all_done(slot ^ 1);
    if (dn < 0) return dn;
    if (dn) {  // the block just queued runs empty
      GMCO_HIP(c0, hipEventSynchronize(bev[slot]));
      return 1;
    }
    return 0;
  };
  GMCO_HIP(c0, hipEventRecord(c0->ev0, st));
  long long round = 0;
  if (R == 0) {
    const int check = r->check_every > 0 ? r->check_every : 16;
    while (true) {
      int rc = issue_round(round);
      if (rc) return rc;
      ++round;
      if (round % check == 0 || round >= max_rounds) {
        const int dn = after_block(round - 1, round >= max_rounds);
        if (dn < 0) return dn;
        if (dn) break;
      }
    }
  } else {
    // capture R lockstep rounds of every case into one graph and replay it;
    // each round's compaction drops the plans that have stopped
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GMCO_HIP(c0, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = GMCO_OK;
    for (int k = 0; k < R && rc == GMCO_OK; ++k) rc = issue_round(k);
    hipError_t ee = hipStreamEndCapture(st, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ee != hipSuccess) return hip_fail(c0, ee, "hipStreamEndCapture");
    ee = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ee != hipSuccess) return hip_fail(c0, ee, "hipGraphInstantiate");
    struct ExecGuard {
      hipGraphExec_t e;
      ~ExecGuard() { (void)hipGraphExecDestroy(e); }
    } eg{exec};
    while (true) {
      GMCO_HIP(c0, hipGraphLaunch(exec, st));
      round += R;
      const int dn = after_block(R - 1, round >= max_rounds);
      if (dn < 0) return dn;
      if (dn) break;
    }
  }
  GMCO_HIP(c0, hipEventRecord(c0->ev1, st));
  GMCO_HIP(c0, hipEventSynchronize(c0->ev1));
  GMCO_HIP(c0, hipEventRecord(c0->gev, st));
  GMCO_HIP(c0, hipStreamWaitEvent(c0->stream, c0->gev, 0));
  float ms = 0.f;
  GMCO_HIP(c0, hipEventElapsedTime(&ms, c0->ev0, c0->ev1));
  int status = GMCO_OK;
  for (int i = 0; i < n; ++i) {
    unsigned long long done = 0;
    GMCO_HIP(ctxs[i], hipMemcpy(&done, ctxs[i]->at<void>(ctxs[i]->lay.work), sizeof(done), hipMemcpyDeviceToHost));
    const int rc = summarize(ctxs[i], round, ms, 0.0, 0.0, done, infos ? &infos[i] : nullptr);
    if (rc && !status) status = rc;
  }
  return status;
}

}  // extern "C"

// ---- evaluation with library-held scratch (no allocation) ----
// The evaluation's split partials and its FP32 copy of x live in this array,
// one per device, held until the process ends.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// (with that device current).
hipError_t static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

extern "C" {

int gmco_evaluate_noalloc(gmco_ctx* c, const double* x_dev, double* F_dev, double* g_dev) {
  if (!c || !x_dev || !F_dev || !g_dev) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  const Dims& d = c->dim;
  const bool lp = is_low_precision(c->dtype);
  const int units = eval_units(d, c->dtype);
  const size_t PK = (size_t)d.Pp * d.Kp;
  const size_t xe_bytes = align256(PK * 4);
  const size_t per_split = align256(PK * 4) + align256((size_t)d.Pp * 8);
  if (xe_bytes + per_split > kStaticScratchBytes)
    return fail(c, GMCO_EINVAL, "batch too large for the 32 MiB evaluation scratch (plans x padded dwells)");
  // the context's split, lowered until the partials fit the scratch
  int S = lp ? d.S_lp : d.S;
  S = std::min(S, (int)((kStaticScratchBytes - xe_bytes) / per_split));
  GMCO_HIP(c, hipSetDevice(c->device));
  void* base = nullptr;
  GMCO_HIP(c, static_scratch(c->device, &base));
  char* b = static_cast<char*>(base);
  float* xe = reinterpret_cast<float*>(b);
  float* Gpart = reinterpret_cast<float*>(b + xe_bytes);
  double* Fpart = reinterpret_cast<double*>(b + xe_bytes + align256((size_t)S * PK * 4));
  GMCO_HIP(c, launch_x_to_device(x_dev, c->P, d.Pp, d.K, d.Kp, xe, c->stream));
  EvalArgs a = eval_args(c, xe, false, c->dtype);
  a.S = S;
  a.grid = S * units;
  a.Gpart = Gpart;
  a.Fpart = Fpart;
  GMCO_HIP(c, launch_eval(a, c->dtype, c->stream));
  GMCO_HIP(c, launch_finish_eval(Gpart, Fpart, xe, S, c->P, d.Pp, d.K, d.Kp, F_dev, g_dev, c->stream));
  return GMCO_OK;
}

int gmco_autotune(gmco_ctx* c, int dtype, int reps, int* best_split, float* best_us) {
  if (!c || reps < 1) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  if (dtype < 0) dtype = c->dtype;
  if (!dtype_available(c->dtype, dtype)) return fail(c, GMCO_EINVAL, "dtype not available");
  GMCO_HIP(c, hipSetDevice(c->device));
  Dims& d = c->dim;
  const bool lp = is_low_precision(dtype);
  int& S_dense = lp ? d.S_lp : d.S;  // the split this dtype's kernel uses
  int& xcd = lp ? d.xcd_lp : d.xcd32;
  std::vector<int> cand;
  for (int s : {S_dense, 4, 8, 12, 16, 20, 24, 28, 32})
    if (s >= 1 && s <= d.S_cap && s <= d.nblocks && std::find(cand.begin(), cand.end(), s) == cand.end())
      cand.push_back(s);
  std::vector<int> shapes = {0};
  if ((lp && lp_shape_ok(d.Kp, 1)) || dtype == GMCO_DTYPE_F32_ACC64) shapes.push_back(1);
  if ((lp && lp_shape_ok(d.Kp, 2)) || (dtype == GMCO_DTYPE_F32_ACC64 && acc_quarters_ok(d.Kp)))
    shapes.push_back(2);
  if (dtype == GMCO_DTYPE_F32_ACC64 || dtype == GMCO_DTYPE_F32) shapes.push_back(3);
  int chunk_shape = 0;  // the FP32 chunked mode has one shape
  int& shape_ref = lp ? d.lp_shape
                      : (dtype == GMCO_DTYPE_F32_ACC64 ? d.acc_shape
                                                       : (dtype == GMCO_DTYPE_F32 ? d.f32_shape : chunk_shape));
  const int orig_s = S_dense, orig_x = xcd, orig_shape = shape_ref;
  int best = orig_s, best_x = orig_x, best_shape = orig_shape;
  float best_t = 1e30f;
  for (int shape : shapes) {
    for (int xm : {1, 0}) {
      for (int s : cand) {
        S_dense = s;
        xcd = xm;
        shape_ref = shape;
        EvalArgs a = eval_args(c, c->at<float>(c->lay.xt), false, dtype);
        GMCO_HIP(c, launch_eval(a, dtype, c->stream));  // warm-up
        GMCO_HIP(c, hipEventRecord(c->ev0, c->stream));
        for (int k = 0; k < reps; ++k) GMCO_HIP(c, launch_eval(a, dtype, c->stream));
        GMCO_HIP(c, hipEventRecord(c->ev1, c->stream));
        GMCO_HIP(c, hipEventSynchronize(c->ev1));
        float ms = 0.f;
        GMCO_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
        const float us = 1e3f * ms / reps;
        if (us < best_t) {
          best_t = us;
          best = s;
          best_x = xm;
          best_shape = shape;
        }
      }
    }
  }
  S_dense = best;
  xcd = best_x;
  shape_ref = best_shape;
  (lp ? d.S_tuned_lp : d.S_tuned) = best;
  if (best_split) *best_split = best;
  if (best_us) *best_us = best_t;
  return GMCO_OK;
}

int gmco_get_tuning(const gmco_ctx* c, int dtype, gmco_tuning* t) {
  if (!c || !t) return GMCO_EINVAL;
  if (!c->case_loaded) return GMCO_ESTATE;
  if (dtype < 0) dtype = c->dtype;
  const bool lp = is_low_precision(dtype);
  const Dims& d = c->dim;
  t->split = lp ? d.S_lp : d.S;
  t->tuned = (lp ? d.S_tuned_lp : d.S_tuned) > 0;
  t->lp_shape = eval_shape(d, dtype);
  t->xcd_map = lp ? d.xcd_lp : d.xcd32;
  return GMCO_OK;
}

int gmco_set_tuning(gmco_ctx* c, int dtype, const gmco_tuning* t) {
  if (!c || !t) return GMCO_EINVAL;
  if (!c->case_loaded) return fail(c, GMCO_ESTATE, "gmco_load_case first");
  if (dtype < 0) dtype = c->dtype;
  if (!dtype_available(c->dtype, dtype)) return fail(c, GMCO_EINVAL, "dtype not available");
  const bool lp = is_low_precision(dtype);
  Dims& d = c->dim;
  if (t->split < 1 || t->split > d.S_cap || t->split > d.nblocks) return fail(c, GMCO_EINVAL, "split out of range");
  if (t->xcd_map != 0 && t->xcd_map != 1) return fail(c, GMCO_EINVAL, "xcd_map must be 0 or 1");
  const bool acc_ok = (dtype == GMCO_DTYPE_F32_ACC64 &&
                       (t->lp_shape == 1 || t->lp_shape == 3 || (t->lp_shape == 2 && acc_quarters_ok(d.Kp)))) ||
                      (dtype == GMCO_DTYPE_F32 && t->lp_shape == 3);
  if (lp ? !lp_shape_ok(d.Kp, t->lp_shape) : (t->lp_shape != 0 && !acc_ok))
    return fail(c, GMCO_EINVAL, "workgroup shape not available for this dtype / dwell count");
  (lp ? d.S_lp : d.S) = t->split;
  (lp ? d.S_tuned_lp : d.S_tuned) = t->split;
  (lp ? d.xcd_lp : d.xcd32) = t->xcd_map;
  if (lp) d.lp_shape = t->lp_shape;
  else if (dtype == GMCO_DTYPE_F32_ACC64) d.acc_shape = t->lp_shape;
  else if (dtype == GMCO_DTYPE_F32) d.f32_shape = t->lp_shape;
  return GMCO_OK;
}

int gmco_set_split(gmco_ctx* c, int split) {
  if (!c) return GMCO_EINVAL;
  if (!c->case_loaded) return fail(c, GMCO_ESTATE, "gmco_load_case first");
  if (split < 1 || split > c->dim.S_cap || split > c->dim.nblocks) return fail(c, GMCO_EINVAL, "split out of range");
  c->dim.S = c->dim.S_lp = split;
  c->dim.S_tuned = c->dim.S_tuned_lp = split;
  return GMCO_OK;
}

}  // extern "C"

namespace {
// Checkpoint blob: this header, then the first P rows of each plan-major
// array in the order of state_arrays().
struct StateHeader {
  uint32_t magic, version;
  int32_t P, K, Kp, m, O, G;
  int32_t S, S_lp, S_tuned, S_tuned_lp;
  uint64_t bytes;
  int32_t plan_state_bytes, pad;
};
static_assert(sizeof(StateHeader) == 64, "state header layout");
constexpr uint32_t kStateMagic = 0x53434d47u;  // "GMCS"
constexpr uint32_t kStateVersion = 1;

struct StateArray {
  size_t off;       // arena offset
  size_t row;       // bytes per plan
};

std::vector<StateArray> state_arrays(const gmco_ctx* c) {
  const Layout& L = c->lay;
  const size_t Kp = (size_t)c->dim.Kp, m = (size_t)c->m;
  return {{L.ps, sizeof(PlanState)}, {L.W64, kGmax * 8}, {L.wn, kGmax * 4},
          {L.x, Kp * 4},  {L.g, Kp * 4},  {L.dir, Kp * 4}, {L.xt, Kp * 4},
          {L.Sh, m * Kp * 4}, {L.Yh, m * Kp * 4}, {L.rho, m * 8}};
}

size_t state_size(const gmco_ctx* c, int P) {
  size_t n = sizeof(StateHeader);
  for (const StateArray& a : state_arrays(c)) n += a.row * (size_t)P;
  return n;
}
}  // namespace

extern "C" {

int gmco_state_bytes(const gmco_ctx* c, size_t* bytes) {
  if (!c || !bytes) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return GMCO_ESTATE;
  *bytes = state_size(c, c->P);
  return GMCO_OK;
}

int gmco_get_state(gmco_ctx* c, void* blob, size_t bytes) {
  if (!c || !blob) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  const size_t need = state_size(c, c->P);
  if (bytes < need) return fail(c, GMCO_EINVAL, "state buffer smaller than gmco_state_bytes");
  GMCO_HIP(c, hipSetDevice(c->device));
  StateHeader h{};
  h.magic = kStateMagic;
  h.version = kStateVersion;
  h.P = c->P;
  h.K = c->dim.K;
  h.Kp = c->dim.Kp;
  h.m = c->m;
  h.O = c->O;
  h.G = c->G;
  h.S = c->dim.S;
  h.S_lp = c->dim.S_lp;
  h.S_tuned = c->dim.S_tuned;
  h.S_tuned_lp = c->dim.S_tuned_lp;
  h.bytes = need;
  h.plan_state_bytes = (int32_t)sizeof(PlanState);
  char* out = static_cast<char*>(blob);
  std::memcpy(out, &h, sizeof(h));
  size_t pos = sizeof(h);
  for (const StateArray& a : state_arrays(c)) {
    const size_t n = a.row * (size_t)c->P;
    GMCO_HIP(c, hipMemcpyAsync(out + pos, c->at<void>(a.off), n, hipMemcpyDeviceToHost, c->stream));
    pos += n;
  }
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  return GMCO_OK;
}

int gmco_set_state(gmco_ctx* c, const void* blob, size_t bytes) {
  if (!c || !blob) return GMCO_EINVAL;
  if (!c->case_loaded) return fail(c, GMCO_ESTATE, "gmco_load_case first");
  StateHeader h{};
  if (bytes < sizeof(h)) return fail(c, GMCO_EINVAL, "state blob too small");
  std::memcpy(&h, blob, sizeof(h));
  if (h.magic != kStateMagic || h.version != kStateVersion || h.plan_state_bytes != (int32_t)sizeof(PlanState))
    return fail(c, GMCO_EINVAL, "not a state blob of this library version");
  if (h.K != c->dim.K || h.Kp != c->dim.Kp || h.m != c->m || h.O != c->O || h.G != c->G)
    return fail(c, GMCO_EINVAL, "state blob of another case shape or history length");
  if (h.P < 1 || h.P > c->Pmax) return fail(c, GMCO_EINVAL, "state blob holds more plans than max_plans");
  const size_t need = state_size(c, h.P);
  if (h.bytes != need || bytes < need) return fail(c, GMCO_EINVAL, "state blob truncated");
  if (h.S < 1 || h.S > c->dim.S_cap || h.S_lp < 1 || h.S_lp > c->dim.S_cap || h.S_tuned < 0 ||
      h.S_tuned > c->dim.S_cap || h.S_tuned_lp < 0 || h.S_tuned_lp > c->dim.S_cap)
    return fail(c, GMCO_EINVAL, "state blob split counts out of range");
  GMCO_HIP(c, hipSetDevice(c->device));
  const char* in = static_cast<const char*>(blob);
  size_t pos = sizeof(h);
  for (const StateArray& a : state_arrays(c)) {
    const size_t n = a.row * (size_t)h.P;
    GMCO_HIP(c, hipMemcpyAsync(c->at<void>(a.off), in + pos, n, hipMemcpyHostToDevice, c->stream));
    pos += n;
  }
  // slots past the restored batch are unused
  const int Pp = c->dim.Pp;
  std::vector<PlanState> pad((size_t)(Pp - h.P));
  for (PlanState& s : pad) {
    std::memset(&s, 0, sizeof(s));
    s.status = ST_INACTIVE;
  }
  if (!pad.empty())
    GMCO_HIP(c, hipMemcpyAsync(c->at<PlanState>(c->lay.ps) + h.P, pad.data(), pad.size() * sizeof(PlanState),
                               hipMemcpyHostToDevice, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  c->dim.S = h.S;
  c->dim.S_lp = h.S_lp;
  c->dim.S_tuned = h.S_tuned;
  c->dim.S_tuned_lp = h.S_tuned_lp;
  c->P = h.P;
  return GMCO_OK;
}

int gmco_get_dwell_times(gmco_ctx* c, double* t) {
  if (!c || !t) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  GMCO_HIP(c, hipSetDevice(c->device));
  const int K = c->dim.K;
  double* tst = c->at<double>(c->lay.gst);
  GMCO_HIP(c, launch_export_t(c->at<float>(c->lay.x), c->P, K, c->dim.Kp, tst, K, c->stream));
  GMCO_HIP(c, hipMemcpyAsync(t, tst, (size_t)c->P * K * 8, hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  return GMCO_OK;
}

int gmco_get_weights_x(gmco_ctx* c, double* x) {
  if (!c || !x) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  GMCO_HIP(c, hipSetDevice(c->device));
  const int K = c->dim.K, Kp = c->dim.Kp;
  std::vector<float> xs((size_t)c->P * Kp);
  GMCO_HIP(c, hipMemcpyAsync(xs.data(), c->at<void>(c->lay.x), xs.size() * 4, hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  for (int p = 0; p < c->P; ++p)
    for (int l = 0; l < K; ++l) x[(size_t)p * K + l] = xs[(size_t)p * Kp + l];
  return GMCO_OK;
}

}  // extern "C"

namespace {
// FP64 metrics at the current t: doses of the optimisation points give F and
// the individual objectives (and the DVH metrics when the case has no DVH
// point set); the DVH points, when given, then give the DVH metrics.
int compute_metrics(gmco_ctx* c) {
  const Layout& L = c->lay;
  const Dims& d = c->dim;
  const bool dvh = d.Md > 0;
  MetricsArgs m{};
  m.W64 = c->at<double>(L.W64);
  m.ps = c->at<PlanState>(L.ps);
  m.P = c->P;
  m.O = c->O;
  m.grp = c->at<int>(L.grp);
  m.gparams = c->at<double>(L.gparams);
  m.volume_cc = c->at<double>(L.volume);
  m.rx = c->rx;
  m.out = c->at<gmco_plan_metrics>(L.metrics);
  GMCO_HIP(c, launch_export_t(c->at<float>(L.x), d.Pp, d.K, d.Kp, c->at<double>(L.t64), d.Kp, c->stream));
  GMCO_HIP(c, launch_dose64(c->at<double>(L.D64), c->at<double>(L.t64), d.Mp, d.Kp, d.Pp, c->at<double>(L.d64), c->stream));
  m.d64 = c->at<double>(L.d64);
  m.ld = d.Mp;
  m.off = c->at<int>(L.goff);
  m.cnt = c->at<int>(L.gcnt);
  m.objective = 1;
  m.dvh = dvh ? 0 : 1;
  GMCO_HIP(c, launch_metrics(m, c->stream));
  if (dvh) {
    GMCO_HIP(c, launch_dose64(c->at<double>(L.D64d), c->at<double>(L.t64), d.Mdp, d.Kp, d.Pp,
                              c->at<double>(L.d64), c->stream));
    m.ld = d.Mdp;
    m.off = c->at<int>(L.doff);
    m.cnt = c->at<int>(L.dcnt);
    m.objective = 0;
    m.dvh = 1;
    GMCO_HIP(c, launch_metrics(m, c->stream));
  }
  GMCO_HIP(c, launch_metrics_final(m, c->stream));
  return GMCO_OK;
}
}  // namespace

extern "C" {

int gmco_select_plan(gmco_ctx* c, const gmco_select_opts* opts, int* best, int* plan_class, int* nondominated,
                     double* nondominated_fraction) {
  if (!c) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  gmco_select_opts o{0, 1, 2, 3, 90.0, 95.0, 118.0, 1.0, 1.0};
  if (opts) o = *opts;
  for (int j : {o.target, o.urethra, o.bladder, o.rectum})
    if (j < 0 || j >= c->O) return fail(c, GMCO_EINVAL, "structure index out of range");
  GMCO_HIP(c, hipSetDevice(c->device));
  int rc = compute_metrics(c);
  if (rc) return rc;
  const int P = c->P, Pp = c->dim.Pp;
  int* cls = c->at<int>(c->lay.sel);
  int* tu = cls + Pp;
  int* nd = tu + Pp;
  int* res = nd + Pp;
  GMCO_HIP(c, launch_select(c->at<gmco_plan_metrics>(c->lay.metrics), P, c->O, o, cls, tu, nd, res, c->stream));
  int h[2] = {0, 0};
  GMCO_HIP(c, hipMemcpyAsync(h, res, 8, hipMemcpyDeviceToHost, c->stream));
  if (plan_class) GMCO_HIP(c, hipMemcpyAsync(plan_class, cls, (size_t)P * 4, hipMemcpyDeviceToHost, c->stream));
  if (nondominated) GMCO_HIP(c, hipMemcpyAsync(nondominated, nd, (size_t)P * 4, hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  if (best) *best = h[0];
  if (nondominated_fraction) *nondominated_fraction = (double)h[1] / (double)P;
  return GMCO_OK;
}

int gmco_get_metrics(gmco_ctx* c, gmco_plan_metrics* out) {
  if (!c || !out) return GMCO_EINVAL;
  if (!c->case_loaded || c->P == 0) return fail(c, GMCO_ESTATE, "gmco_set_weights first");
  GMCO_HIP(c, hipSetDevice(c->device));
  const Layout& L = c->lay;
  const int rc = compute_metrics(c);
  if (rc) return rc;
  GMCO_HIP(c, hipMemcpyAsync(out, c->at<void>(L.metrics), (size_t)c->P * sizeof(gmco_plan_metrics),
                             hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  return GMCO_OK;
}

int gmco_get_dose_rate(gmco_ctx* c, double* D64, double* Drun) {
  if (!c) return GMCO_EINVAL;
  if (!c->case_loaded) return fail(c, GMCO_ESTATE, "gmco_load_case first");
  GMCO_HIP(c, hipSetDevice(c->device));
  const Dims& d = c->dim;
  const size_t MK = (size_t)d.Mp * d.Kp;
  std::vector<double> h64;
  std::vector<float> hr;
  if (D64) {
    h64.resize(MK);
    GMCO_HIP(c, hipMemcpyAsync(h64.data(), c->at<void>(c->lay.D64), MK * 8, hipMemcpyDeviceToHost, c->stream));
  }
  std::vector<uint16_t> hb;
  std::vector<double> h64w;
  if (Drun) {
    if (!is_low_precision(c->dtype)) {
      hr.resize(MK);
      GMCO_HIP(c, hipMemcpyAsync(hr.data(), c->at<void>(c->lay.D32), MK * 4, hipMemcpyDeviceToHost, c->stream));
    } else if (c->dtype == GMCO_DTYPE_BF16) {
      hb.resize(MK);
      GMCO_HIP(c, hipMemcpyAsync(hb.data(), c->at<void>(c->lay.Dlp), MK * 2, hipMemcpyDeviceToHost, c->stream));
    } else {
      // FP8: widen on the device (hardware encoding) into the FP64 scratch
      double* wide = c->at<double>(c->lay.d64);
      GMCO_HIP(c, launch_widen_fp8(c->at<void>(c->lay.Dlp), c->at<float>(c->lay.colscale), d.Mp, d.Kp,
                                   wide, c->stream));
      h64w.resize(MK);
      GMCO_HIP(c, hipMemcpyAsync(h64w.data(), wide, MK * 8, hipMemcpyDeviceToHost, c->stream));
    }
  }
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < d.M; ++i) {
    const size_t dst = (size_t)c->perm[i] * d.K;
    for (int l = 0; l < d.K; ++l) {
      if (D64) D64[dst + l] = h64[(size_t)i * d.Kp + l];
      if (Drun) {
        if (!hr.empty()) {
          Drun[dst + l] = hr[(size_t)i * d.Kp + l];
        } else if (!h64w.empty()) {
          Drun[dst + l] = h64w[(size_t)i * d.Kp + l];
        } else {
          // widen a BF16 bit pattern: its bits are the high half of an FP32
          const uint32_t bits = (uint32_t)hb[(size_t)i * d.Kp + l] << 16;
          float f;
          std::memcpy(&f, &bits, 4);
          Drun[dst + l] = f;
        }
      }
    }
  }
  return GMCO_OK;
}

int gmco_case_features(gmco_ctx* c, float* out) {
  if (!c || !out) return GMCO_EINVAL;
  if (!c->case_loaded) return fail(c, GMCO_ESTATE, "gmco_load_case first");
  if (!c->has_points) return fail(c, GMCO_EINVAL, "features need point positions");
  GMCO_HIP(c, hipSetDevice(c->device));
  const Layout& L = c->lay;
  const Dims& d = c->dim;
  double* stage = c->at<double>(L.stage);
  const double* dw = stage + (size_t)d.M * d.K;
  const double* pts = dw + (size_t)d.K * 3;
  GMCO_HIP(c, launch_features(dw, pts, c->at<int>(L.perm), c->at<int>(L.goff), c->at<int>(L.gcnt), d.K,
                              c->O, c->at<unsigned>(L.hist), c->at<float>(L.feat), c->stream));
  GMCO_HIP(c, hipMemcpyAsync(out, c->at<void>(L.feat), (size_t)c->O * 16 * 4, hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  return GMCO_OK;
}

int gmco_get_start_time(gmco_ctx* c, double* t_bar) {
  if (!c || !t_bar) return GMCO_EINVAL;
  if (!c->case_loaded) return fail(c, GMCO_ESTATE, "gmco_load_case first");
  GMCO_HIP(c, hipSetDevice(c->device));
  GMCO_HIP(c, hipMemcpyAsync(t_bar, c->at<void>(c->lay.t_bar), 8, hipMemcpyDeviceToHost, c->stream));
  GMCO_HIP(c, hipStreamSynchronize(c->stream));
  return GMCO_OK;
}

}  // extern "C"
