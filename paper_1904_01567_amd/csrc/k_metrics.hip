// Final-plan quantities in FP64: t = x^2, the dose of every point
// (eq. (dose)), eq. (obj) re-evaluated, and the DVH metrics of Sec. 2.3.1.
#include "gmco_internal.h"

namespace gmco {
namespace {

__global__ void k_export_t(const float* __restrict__ x, int P, int K, int Kp,
                           double* __restrict__ t64, int Kp_out) {
  const int p = blockIdx.x;
  if (p >= P) return;
  for (int l = threadIdx.x; l < Kp_out; l += blockDim.x) {
    double v = 0.0;
    if (l < K) {
      const double xv = (double)x[(size_t)p * Kp + l];
      v = xv * xv;
    }
    t64[(size_t)p * Kp_out + l] = v;
  }
}

// d64[p][i] = sum_l D64[i][l] t64[p][l]; 64 points x 64 plans per workgroup,
// 4 x 4 outputs per thread, 32-dwell slices staged in LDS.
__global__ __launch_bounds__(256) void k_dose64(const double* __restrict__ D64,
                                                const double* __restrict__ t64, int Mp, int Kp,
                                                int Pp, double* __restrict__ d64) {
  __shared__ double sD[64][33];
  __shared__ double sT[64][33];
  const int i0 = blockIdx.x * 64;
  const int p0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 15;  // points i0 + tx + 16 a
  const int ty = threadIdx.x >> 4;  // plans  p0 + ty + 16 b
  double acc[4][4] = {};
  for (int k0 = 0; k0 < Kp; k0 += 32) {
    for (int idx = threadIdx.x; idx < 64 * 32; idx += 256) {
      const int r = idx >> 5, c = idx & 31;
      const int gi = i0 + r, gp = p0 + r, gk = k0 + c;
      sD[r][c] = (gi < Mp && gk < Kp) ? D64[(size_t)gi * Kp + gk] : 0.0;
      sT[r][c] = (gp < Pp && gk < Kp) ? t64[(size_t)gp * Kp + gk] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < 32; ++c) {
      double dv[4], tv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) dv[a] = sD[tx + 16 * a][c];
#pragma unroll
      for (int b = 0; b < 4; ++b) tv[b] = sT[ty + 16 * b][c];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(dv[a], tv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int gi = i0 + tx + 16 * a, gp = p0 + ty + 16 * b;
      if (gi < Mp && gp < Pp) d64[(size_t)gp * Mp + gi] = acc[a][b];
    }
}

// k-th largest of the keys (bit patterns of non-negative doubles order like
// their values), radix select over 8-bit digits from the most significant.
struct SelectState {
  unsigned long long prefix;
  unsigned long long mask;
  int k;
};

__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// One workgroup per (plan, organ): a pass over the organ's points of one
// point set (MetricsArgs).  The individual objective f_j = (1/N_j) sum f_i
// takes each point's own group parameters (surface and volume rows of one
// organ share the organ's N_j); the DVH metrics follow the definitions of
// Sec. 2.3.1 (V_x counts d >= x % Rx; D_x is the k-th hottest dose,
// k = max(1, ceil(x N / 100)), by radix select on the FP64 bit patterns).
__global__ __launch_bounds__(256) void k_metrics_group(MetricsArgs a) {
  __shared__ double red[256];
  __shared__ unsigned int h10[256], h90[256];
  __shared__ SelectState sel[2];
  const int p = blockIdx.x;
  const int j = blockIdx.y;
  if (p >= a.P) return;
  gmco_plan_metrics* m = a.out + p;
  if (j >= a.O) {
    if (threadIdx.x == 0 && j < kGmax) {
      if (a.objective) m->f_organ[j] = 0.0;
      if (a.dvh) {
        m->V100_pct[j] = 0.0;
        m->V75_cc[j] = 0.0;
        m->D10_pct[j] = 0.0;
        m->D90_pct[j] = 0.0;
      }
    }
    return;
  }
  const int N = a.cnt[j];
  const int o0 = a.off[j];
  const double* __restrict__ d = a.d64 + (size_t)p * a.ld + o0;
  const double thr100 = a.rx, thr75 = 0.75 * a.rx;

  double fs = 0.0, c100 = 0.0, c75 = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double v = d[i];
    if (a.objective) {
      const double* prm = a.gparams + 4 * a.grp[o0 + i];
      const double wmin = prm[0], dmin = prm[1], dmax = prm[2], wmax = prm[3];
      if (v < dmin) fs += wmin * ((dmin - v) * (dmin - v));
      else if (v > dmax) fs += wmax * ((v - dmax) * (v - dmax));
    }
    c100 += (v >= thr100) ? 1.0 : 0.0;
    c75 += (v >= thr75) ? 1.0 : 0.0;
  }
  fs = block_sum(fs, red);
  c100 = block_sum(c100, red);
  c75 = block_sum(c75, red);
  if (a.objective && threadIdx.x == 0) m->f_organ[j] = fs / (N > 0 ? (double)N : 1.0);
  if (!a.dvh) return;

  // D10 / D90: k = max(1, ceil(x N / 100)) in integers
  if (threadIdx.x == 0) {
    sel[0].prefix = 0ull;
    sel[0].mask = 0ull;
    sel[0].k = max(1, (10 * N + 99) / 100);
    sel[1].prefix = 0ull;
    sel[1].mask = 0ull;
    sel[1].k = max(1, (90 * N + 99) / 100);
  }
  __syncthreads();
  for (int shift = 56; shift >= 0 && N > 0; shift -= 8) {
    h10[threadIdx.x] = 0u;
    h90[threadIdx.x] = 0u;
    __syncthreads();
    const unsigned long long pf0 = sel[0].prefix, mk0 = sel[0].mask;
    const unsigned long long pf1 = sel[1].prefix, mk1 = sel[1].mask;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const unsigned long long key = (unsigned long long)__double_as_longlong(d[i]);
      const unsigned dig = (unsigned)((key >> shift) & 0xffull);
      if ((key & mk0) == pf0) atomicAdd(&h10[dig], 1u);
      if ((key & mk1) == pf1) atomicAdd(&h90[dig], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      unsigned int* h = threadIdx.x == 0 ? h10 : h90;
      SelectState& s = sel[threadIdx.x];
      int k = s.k;
      int dsel = 0;
      for (int dg = 255; dg >= 0; --dg) {
        const int c = (int)h[dg];
        if (k <= c) {
          dsel = dg;
          break;
        }
        k -= c;
      }
      s.k = k;
      s.prefix |= ((unsigned long long)dsel) << shift;
      s.mask |= 0xffull << shift;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = N > 0 ? (double)N : 1.0;
    m->V100_pct[j] = 100.0 * (c100 / n);
    m->V75_cc[j] = (a.volume_cc ? a.volume_cc[j] : 0.0) * (c75 / n);
    m->D10_pct[j] = N > 0 ? 100.0 * __longlong_as_double((long long)sel[0].prefix) / a.rx : 0.0;
    m->D90_pct[j] = N > 0 ? 100.0 * __longlong_as_double((long long)sel[1].prefix) / a.rx : 0.0;
  }
}

__global__ void k_metrics_final(const double* __restrict__ W64, const PlanState* __restrict__ ps,
                                int P, int O, gmco_plan_metrics* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  gmco_plan_metrics* m = out + p;
  double F = 0.0;
  for (int j = 0; j < O; ++j) F += W64[(size_t)p * kGmax + j] * m->f_organ[j];
  m->F64 = F;
  m->F_run = ps[p].F;
  m->iterations = ps[p].iter;
  m->evaluations = ps[p].nevals;
  m->status = ps[p].status == ST_INIT ? ST_RUNNING : ps[p].status;
  m->reserved = 0;
}

// RTOG 0924 classes (Sec. 2.3.1): 2 = RTOG+ valid, 1 = RTOG valid, 0 = invalid.
__global__ void k_classify(const gmco_plan_metrics* __restrict__ m, int P, gmco_select_opts o,
                           int* __restrict__ cls, int* __restrict__ meets_tu) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double v100 = m[p].V100_pct[o.target];
  const bool ok_t = v100 >= o.v100_min;
  const bool ok_u = m[p].D10_pct[o.urethra] < o.urethra_d10_max;
  const bool ok_b = m[p].V75_cc[o.bladder] < o.bladder_v75_max;
  const bool ok_r = m[p].V75_cc[o.rectum] < o.rectum_v75_max;
  cls[p] = (ok_t && ok_u && ok_b && ok_r) ? (v100 >= o.v100_plus ? 2 : 1) : 0;
  meets_tu[p] = (ok_t && ok_u) ? 1 : 0;
}

// Plan p is dominated when another plan is at least as good in every
// individual objective and strictly better in one (Sec. 2.2.4).
__global__ void k_pareto(const gmco_plan_metrics* __restrict__ m, int P, int G, int* __restrict__ nd) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int dominated = 0;
  for (int q = 0; q < P && !dominated; ++q) {
    if (q == p) continue;
    bool all_le = true, any_lt = false;
    for (int j = 0; j < G; ++j) {
      const double a = m[q].f_organ[j], b = m[p].f_organ[j];
      all_le = all_le && (a <= b);
      any_lt = any_lt || (a < b);
    }
    dominated = (all_le && any_lt) ? 1 : 0;
  }
  nd[p] = dominated ? 0 : 1;
}

// Selection (Sec. 2.4): RTOG+ over RTOG over invalid; among valid plans the
// highest target V100; among invalid plans the lowest bladder + rectum V75
// among those meeting the target and urethra criteria (all invalid plans if
// none does); ties to the lowest index.  One workgroup.
__global__ __launch_bounds__(1024) void k_select(const gmco_plan_metrics* __restrict__ m,
                                                 const int* __restrict__ cls,
                                                 const int* __restrict__ meets_tu, const int* __restrict__ nd,
                                                 int P, gmco_select_opts o, int* __restrict__ out) {
  __shared__ int s_i[1024];
  __shared__ double s_k[1024];
  const int t = threadIdx.x;
  // best class and whether an invalid plan meets target and urethra
  int bc = 0, tu = 0, nnd = 0;
  for (int p = t; p < P; p += blockDim.x) {
    bc = max(bc, cls[p]);
    tu |= (cls[p] == 0 && meets_tu[p]) ? 1 : 0;
    nnd += nd[p];
  }
  s_i[t] = bc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) s_i[t] = max(s_i[t], s_i[t + w]);
    __syncthreads();
  }
  const int best_class = s_i[0];
  __syncthreads();
  s_i[t] = tu;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) s_i[t] = s_i[t] | s_i[t + w];
    __syncthreads();
  }
  const int any_tu = s_i[0];
  __syncthreads();
  s_i[t] = nnd;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) s_i[t] += s_i[t + w];
    __syncthreads();
  }
  const int n_nd = s_i[0];
  __syncthreads();
  // smallest key wins, ties to the lowest index
  int bi = -1;
  double bk = 0.0;
  for (int p = t; p < P; p += blockDim.x) {
    if (cls[p] != best_class) continue;
    if (best_class == 0 && any_tu && !meets_tu[p]) continue;
    const double key = best_class > 0 ? -m[p].V100_pct[o.target]
                                       : m[p].V75_cc[o.bladder] + m[p].V75_cc[o.rectum];
    if (bi < 0 || key < bk) {
      bi = p;
      bk = key;
    }
  }
  s_i[t] = bi;
  s_k[t] = bk;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) {
      const int i2 = s_i[t + w];
      const double k2 = s_k[t + w];
      if (i2 >= 0 && (s_i[t] < 0 || k2 < s_k[t] || (k2 == s_k[t] && i2 < s_i[t]))) {
        s_i[t] = i2;
        s_k[t] = k2;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = s_i[0];
    out[1] = n_nd;
  }
}

}  // namespace

hipError_t launch_select(const gmco_plan_metrics* m, int P, int G, const gmco_select_opts& o, int* cls,
                         int* meets_tu, int* nd, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_classify, dim3((P + 255) / 256), dim3(256), 0, st, m, P, o, cls, meets_tu);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pareto, dim3((P + 255) / 256), dim3(256), 0, st, m, P, G, nd);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, st, m, cls, meets_tu, nd, P, o, out);
  return hipGetLastError();
}

hipError_t launch_export_t(const float* x, int P, int K, int Kp, double* t64, int Kp_out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_export_t, dim3(P), dim3(128), 0, st, x, P, K, Kp, t64, Kp_out);
  return hipGetLastError();
}

hipError_t launch_dose64(const double* D64, const double* t64, int Mp, int Kp, int Pp,
                         double* d64, hipStream_t st) {
  dim3 grid((Mp + 63) / 64, (Pp + 63) / 64);
  hipLaunchKernelGGL(k_dose64, grid, dim3(256), 0, st, D64, t64, Mp, Kp, Pp, d64);
  return hipGetLastError();
}

hipError_t launch_metrics(const MetricsArgs& m, hipStream_t st) {
  if (m.P < 1) return hipSuccess;
  hipLaunchKernelGGL(k_metrics_group, dim3(m.P, kGmax), dim3(256), 0, st, m);
  return hipGetLastError();
}

hipError_t launch_metrics_final(const MetricsArgs& m, hipStream_t st) {
  if (m.P < 1) return hipSuccess;
  hipLaunchKernelGGL(k_metrics_final, dim3((m.P + 127) / 128), dim3(128), 0, st, m.W64, m.ps, m.P,
                     m.O, m.out);
  return hipGetLastError();
}

}  // namespace gmco
