// Case and batch set-up kernels: dose-rate matrix (Sec. 2.2.1 step (i)),
// its run-dtype copy, the default start time and the per-plan state.
#include "gmco_internal.h"

namespace gmco {
namespace {

// Point-source law of the synthetic cases: (1 - 0.01 r) / max(r, 0.1 cm)^2.
// Rows follow the library's point order (grouped by structure): row i is the
// caller's point perm[i].  Padding rows and columns are zero.
__global__ void k_dose_rate(const double* __restrict__ dwell, const double* __restrict__ pts,
                            const double* __restrict__ user_D, const int* __restrict__ perm,
                            int M, int K, int Mp, int Kp, double* __restrict__ D64) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (l >= Kp || i >= Mp) return;
  double v = 0.0;
  if (i < M && l < K) {
    const int src = perm[i];
    if (user_D != nullptr) {
      v = user_D[(size_t)src * K + l];
    } else {
      const double dx = pts[3 * src + 0] - dwell[3 * l + 0];
      const double dy = pts[3 * src + 1] - dwell[3 * l + 1];
      const double dz = pts[3 * src + 2] - dwell[3 * l + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double rc = r > 0.1 ? r : 0.1;
      v = (1.0 - 0.01 * r) / (rc * rc);
    }
  }
  D64[(size_t)i * Kp + l] = v;
}

__global__ void k_cast_f32(const double* __restrict__ D64, size_t n, float* __restrict__ out) {
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x)
    out[idx] = (float)D64[idx];
}

// Round an FP32 value to BF16, nearest with ties to even (finite inputs).
__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Position of point r of a 32-point block in the BF16 / FP8 evaluation's transposed
// tile (its back-projection operand order): rows 4q .. 4q+3 and
// 16+4q .. 16+4q+3 of the block at positions 8q .. 8q+7.
__device__ inline int tpos32(int r) {
  return r < 16 ? 8 * (r >> 2) + (r & 3) : 8 * ((r - 16) >> 2) + 4 + ((r - 16) & 3);
}

// BF16 copies of the dose-rate matrix, row-major (points x dwells) for the
// dose product and dwell-major for the back-projection, the latter with the
// points of each 32-point block in the tile order above (Mp is a multiple of
// 32).
__global__ void k_cast_bf16(const double* __restrict__ D64, int Mp, int Kp,
                            uint16_t* __restrict__ D, uint16_t* __restrict__ DT) {
  const size_t n = (size_t)Mp * Kp;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / Kp, l = idx - i * Kp;
    const uint16_t v = bf16_rne((float)D64[idx]);
    D[idx] = v;
    DT[l * Mp + (i & ~(size_t)31) + tpos32((int)(i & 31))] = v;
  }
}

// Per-dwell-column scale for the FP8 copy: s_l = max_i D_il / 224 (1 for an
// all-zero column), one workgroup per column, fixed reduction order.
__global__ void k_colscale(const double* __restrict__ D64, int Mp, int Kp, float* __restrict__ cs) {
  __shared__ double red[256];
  const int l = blockIdx.x;
  double m = 0.0;
  for (int i = threadIdx.x; i < Mp; i += blockDim.x) m = fmax(m, fabs(D64[(size_t)i * Kp + l]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) cs[l] = red[0] > 0.0 ? (float)(red[0] / 224.0) : 1.f;
}

// FP8 (hardware e4m3 encoding) copy of D_il / s_l, row-major, and the BF16
// dwell-major copy for the back-projection, its points in the tile order of
// each 32-point block (Mp is a multiple of 32).
__global__ void k_cast_fp8(const double* __restrict__ D64, int Mp, int Kp,
                           const float* __restrict__ cs, unsigned char* __restrict__ D8,
                           uint16_t* __restrict__ DT) {
  const size_t n = (size_t)Mp * Kp;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / Kp, l = idx - i * Kp;
    const float v = (float)D64[idx];
    D8[idx] = (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(v / cs[l], 0.f, 0, false) & 0xff);
    DT[l * Mp + (i & ~(size_t)31) + tpos32((int)(i & 31))] = bf16_rne(v);
  }
}

// FP8 bytes widened to double with the column scale applied (for export).
__global__ void k_widen_fp8(const unsigned char* __restrict__ D8, const float* __restrict__ cs,
                            int Mp, int Kp, double* __restrict__ out) {
  const size_t n = (size_t)Mp * Kp;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t l = idx % Kp;
    out[idx] = (double)__builtin_amdgcn_cvt_f32_fp8((int)D8[idx], 0) * (double)cs[l];
  }
}

// t_bar = Rx / mean over the target rows of sum_l D_il, one workgroup, fixed
// summation order.
__global__ void k_start_time(const double* __restrict__ D64, int Kp, int r0, int r1, double rx,
                             double* __restrict__ t_bar) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    double rs = 0.0;
    for (int l = 0; l < Kp; ++l) rs += D64[(size_t)i * Kp + l];
    acc += rs;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = red[0] / (double)(r1 - r0);
    *t_bar = (r1 > r0 && mean > 0.0) ? rx / mean : 0.0;
  }
}

// Start point and weights of every plan slot.  Inactive slots (p >= P) get
// zero weights and the INACTIVE state.
// W is P x O hidden weights (one per organ); group j of organ gorg[j] gets
// w / N_pnt of its organ (eq. (obj)).
__global__ void k_init_plans(int P, int Pp, int K, int Kp, const double* __restrict__ t0,
                             const double* __restrict__ t_bar, const double* __restrict__ W,
                             int G, int O, const int* __restrict__ gorg,
                             const int* __restrict__ norm, float* __restrict__ xt,
                             float* __restrict__ x, float* __restrict__ wn,
                             double* __restrict__ W64, PlanState* __restrict__ ps) {
  const int p = blockIdx.x;
  if (p >= Pp) return;
  const bool live = p < P;
  const double tb = *t_bar;
  for (int l = threadIdx.x; l < Kp; l += blockDim.x) {
    float v = 0.f;
    if (live && l < K) {
      const double t = t0 ? t0[(size_t)p * K + l] : tb;
      v = (float)sqrt(t > 0.0 ? t : 0.0);
    }
    xt[(size_t)p * Kp + l] = v;
    x[(size_t)p * Kp + l] = v;
  }
  if (threadIdx.x < kGmax) {
    const int j = threadIdx.x;
    W64[(size_t)p * kGmax + j] = (live && j < O) ? W[(size_t)p * O + j] : 0.0;
    double w = 0.0;
    if (live && j < G) w = W[(size_t)p * O + gorg[j]];
    wn[(size_t)p * kGmax + j] = (j < G && norm[j] > 0) ? (float)(w / (double)norm[j]) : 0.f;
  }
  if (threadIdx.x == 0) {
    PlanState s;
    s.F = 0.0;
    s.Fprev = 0.0;
    s.alpha = 0.0;
    s.gtp = 0.0;
    s.status = live ? ST_INIT : ST_INACTIVE;
    s.iter = 0;
    s.ntrial = 0;
    s.hcount = 0;
    s.hhead = 0;
    s.nevals = 0;
    s.pad0 = 0;
    s.pad1 = 0;
    ps[p] = s;
  }
}

// Dwell weights given by the caller (FP64, P x K) into the padded FP32 layout.
__global__ void k_x_to_device(const double* __restrict__ xin, int P, int K, int Kp,
                              float* __restrict__ xe) {
  const int p = blockIdx.x;
  for (int l = threadIdx.x; l < Kp; l += blockDim.x)
    xe[(size_t)p * Kp + l] = (p < P && l < K) ? (float)xin[(size_t)p * K + l] : 0.f;
}

// Network inputs of the learned start: row p is the plan's hidden weights
// (one per organ, as given) followed by the case features.
__global__ void k_learned_inputs(const double* __restrict__ W64, const float* __restrict__ feat, int O,
                                 float* __restrict__ X) {
  const int p = blockIdx.x;
  const int n_in = O + 16 * O;
  for (int i = threadIdx.x; i < n_in; i += blockDim.x)
    X[(size_t)p * n_in + i] = i < O ? (float)W64[(size_t)p * kGmax + i] : feat[i - O];
}

// Start dwell weights from the network's output y (normalised by the uniform
// start): x0 = max(y, floor) sqrt(t_bar); a non-finite y stays non-finite, so
// that the plan's start objective is too and the plan falls back.
__global__ void k_learned_start(const float* __restrict__ Y, int K, int Kp, const double* __restrict__ t_bar,
                                float floor, float* __restrict__ xe) {
  const int p = blockIdx.x;
  const float sc = (float)sqrt(*t_bar);
  for (int l = threadIdx.x; l < Kp; l += blockDim.x) {
    float v = 0.f;
    if (l < K) {
      const float y = Y[(size_t)p * K + l];
      v = (isfinite(y) ? fmaxf(y, floor) : y) * sc;
    }
    xe[(size_t)p * Kp + l] = v;
  }
}

// Per plan: keep the learned start only where it is finite and its
// objective is below the uniform start's (plain L-BFGS from the uniform
// start is the fallback).  The start itself is checked, not only F: the
// penalty of eq. 1 as evaluated (min / max with the band edges) is 0 at a
// NaN dose.  The chosen point becomes the plan's start (status INIT).
__global__ void k_pick_start(const double* __restrict__ Fw, const double* __restrict__ Fu,
                             const float* __restrict__ xe, int Kp, float* __restrict__ x,
                             float* __restrict__ xt, int* __restrict__ n_warm, int* __restrict__ use_warm) {
  const int p = blockIdx.x;
  int bad = 0;
  for (int l = threadIdx.x; l < Kp; l += blockDim.x) bad |= !isfinite(xe[(size_t)p * Kp + l]);
  bad = __syncthreads_or(bad);
  const double fw = Fw[p];
  const bool warm = !bad && isfinite(fw) && fw < Fu[p];
  if (threadIdx.x == 0) {
    use_warm[p] = warm ? 1 : 0;
    if (warm) atomicAdd(n_warm, 1);
  }
  if (!warm) return;
  for (int l = threadIdx.x; l < Kp; l += blockDim.x) {
    const float v = xe[(size_t)p * Kp + l];
    x[(size_t)p * Kp + l] = v;
    xt[(size_t)p * Kp + l] = v;
  }
}

}  // namespace

hipError_t launch_learned_inputs(const double* W64, const float* feat, int P, int O, float* X, hipStream_t st) {
  hipLaunchKernelGGL(k_learned_inputs, dim3(P), dim3(128), 0, st, W64, feat, O, X);
  return hipGetLastError();
}

hipError_t launch_learned_start(const float* Y, int P, int Pp, int K, int Kp, const double* t_bar, double floor,
                                float* xe, hipStream_t st) {
  (void)Pp;
  hipLaunchKernelGGL(k_learned_start, dim3(P), dim3(128), 0, st, Y, K, Kp, t_bar, (float)floor, xe);
  return hipGetLastError();
}

hipError_t launch_pick_start(const double* F_warm, const double* F_uniform, const float* xe, int P, int Kp,
                             float* x, float* xt, int* n_warm, int* use_warm, hipStream_t st) {
  hipLaunchKernelGGL(k_pick_start, dim3(P), dim3(128), 0, st, F_warm, F_uniform, xe, Kp, x, xt, n_warm, use_warm);
  return hipGetLastError();
}

hipError_t launch_dose_rate(const double* dwell_xyz, const double* pt_xyz, const double* user_D,
                            const int* perm, int M, int K, int Mp, int Kp, double* D64,
                            hipStream_t st) {
  dim3 grid((Kp + 127) / 128, Mp);
  hipLaunchKernelGGL(k_dose_rate, grid, dim3(128), 0, st, dwell_xyz, pt_xyz, user_D, perm, M, K,
                     Mp, Kp, D64);
  return hipGetLastError();
}

hipError_t launch_cast_dose(const double* D64, int Mp, int Kp, int dtype, float* D32, void* Dlp,
                            void* DTlp, float* colscale, hipStream_t st) {
  (void)colscale;
  const size_t n = (size_t)Mp * Kp;
  hipLaunchKernelGGL(k_cast_f32, dim3(1024), dim3(256), 0, st, D64, n, D32);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == GMCO_DTYPE_BF16) {
    hipLaunchKernelGGL(k_cast_bf16, dim3(1024), dim3(256), 0, st, D64, Mp, Kp, (uint16_t*)Dlp,
                       (uint16_t*)DTlp);
    return hipGetLastError();
  }
  if (dtype == GMCO_DTYPE_FP8) {
    hipLaunchKernelGGL(k_colscale, dim3(Kp), dim3(256), 0, st, D64, Mp, Kp, colscale);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cast_fp8, dim3(1024), dim3(256), 0, st, D64, Mp, Kp, colscale,
                       (unsigned char*)Dlp, (uint16_t*)DTlp);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_widen_fp8(const void* D8, const float* colscale, int Mp, int Kp, double* out,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_widen_fp8, dim3(1024), dim3(256), 0, st, (const unsigned char*)D8,
                     colscale, Mp, Kp, out);
  return hipGetLastError();
}

hipError_t launch_start_time(const double* D64, int Kp, int row_begin, int row_end,
                             double prescription, double* t_bar, hipStream_t st) {
  hipLaunchKernelGGL(k_start_time, dim3(1), dim3(1024), 0, st, D64, Kp, row_begin, row_end,
                     prescription, t_bar);
  return hipGetLastError();
}

hipError_t launch_init_plans(int P, int Pp, int K, int Kp, const double* t0, const double* t_bar,
                             const double* W, int G, int O, const int* gorg, const int* norm,
                             float* xt, float* x, float* wn, double* W64, PlanState* ps,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_init_plans, dim3(Pp), dim3(128), 0, st, P, Pp, K, Kp, t0, t_bar, W, G, O,
                     gorg, norm, xt, x, wn, W64, ps);
  return hipGetLastError();
}

hipError_t launch_x_to_device(const double* x_host_dev, int P, int Pp, int K, int Kp, float* xe,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_x_to_device, dim3(Pp), dim3(128), 0, st, x_host_dev, P, K, Kp, xe);
  return hipGetLastError();
}

}  // namespace gmco
