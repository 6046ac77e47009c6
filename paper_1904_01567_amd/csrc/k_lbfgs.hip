// Batched L-BFGS state machine: one wavefront per plan.
//
// Every round evaluates one point per active plan (k_eval); this kernel then
// advances each plan by one step of its own sequential algorithm:
//   * reduce the split-M partials into F and g = 4 x * G (eq. 2);
//   * accept or reject the trial with the Armijo test; on reject halve the
//     step (backtracking) and propose x + alpha p again;
//   * on accept push the pair (s, y) when s'y > 1e-10 |s| |y|, test the
//     relative-variation stop rule (Sec. 2.2.3) and compute the next
//     direction with the two-loop recursion (Liu & Nocedal, cited in
//     Sec. 2.2.2), gamma = s'y / y'y of the newest pair, restarting from
//     steepest descent when the direction is not a descent direction.
// Each lane owns dwells e = lane + 64 j, so every vector operation is local
// to the lane and every dot product is one wavefront reduction.
#include "gmco_internal.h"

namespace gmco {
namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int E>
__device__ inline double dot(const float (&a)[E], const float (&b)[E]) {
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < E; ++j) s = fmaf(a[j], b[j], s);
  return wave_sum((double)s);
}

// MH = register capacity for history pairs (MH >= m).  The pairs are held in
// registers in age order (0 = newest) so every loop index is a compile-time
// constant; all their loads are issued together before the recursion.
template <int E, int MH>
__global__ __launch_bounds__(256) void k_update(UpdateArgs a) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.active_count[(a.round + 1) & 1] = 0;
  if (p >= a.Pp) return;
  PlanState st = a.ps[p];
  if (!state_active(st.status)) return;

  const int Kp = a.Kp;
  const int m = a.m;
  const size_t row = (size_t)p * Kp;
  bool valid[E];
#pragma unroll
  for (int j = 0; j < E; ++j) valid[j] = (lane + 64 * j) < Kp;

  // ---- objective and gradient at the evaluated point ----
  float xt[E], gt[E], x[E], g[E], d[E];
  float G[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    G[j] = 0.f;
    const int e = lane + 64 * j;
    xt[j] = valid[j] ? a.xt[row + e] : 0.f;
    x[j] = valid[j] ? a.x[row + e] : 0.f;
    g[j] = valid[j] ? a.g[row + e] : 0.f;
    d[j] = valid[j] ? a.dir[row + e] : 0.f;
  }
  // gradient partials of this round's compact column, summed by k_reduce_g
  const RoundTable rt = *a.rt;
  const size_t stride = (size_t)rt.ntiles * kPT;
  const size_t col = (size_t)a.slot[p];
  {
    const float* src = a.Gsum + col * Kp;
#pragma unroll
    for (int j = 0; j < E; ++j)
      if (valid[j]) G[j] = src[lane + 64 * j];
  }
  // split partials of F: one load per lane, then a fixed-order wave sum
  double fpart = 0.0;
  for (int s = lane; s < rt.S; s += 64) fpart += a.Fpart[s * stride + col];
  const double Ft = wave_sum(fpart);
#pragma unroll
  for (int j = 0; j < E; ++j) gt[j] = 4.f * xt[j] * G[j];
  st.nevals += 1;

  bool need_dir = false;
  bool stop = false;
  bool pushed = false;
  float sv[E], yv[E];
  double rho_new = 0.0;
  if (st.status == ST_INIT) {
    // take the evaluated point as the current iterate (start or resume)
    const double gg = dot(gt, gt);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      x[j] = xt[j];
      g[j] = gt[j];
      if (valid[j]) {
        a.x[row + lane + 64 * j] = x[j];
        a.g[row + lane + 64 * j] = g[j];
      }
    }
    st.F = Ft;
    if (!isfinite(Ft) || !isfinite(gg)) {
      st.status = ST_NONFINITE;
      stop = true;
    } else if (Ft == 0.0) {
      st.status = ST_CONVERGED;
      stop = true;
    } else if (st.iter >= a.max_iter) {
      st.status = ST_MAXITER;
      stop = true;
    } else {
      st.status = ST_RUNNING;
      need_dir = true;
    }
  } else {
    const bool accept = isfinite(Ft) && (Ft <= st.F + a.c1 * st.alpha * st.gtp);
    if (accept) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        sv[j] = xt[j] - x[j];
        yv[j] = gt[j] - g[j];
      }
      const double sy = dot(sv, yv);
      const double ss = dot(sv, sv);
      const double yy = dot(yv, yv);
      if (sy > 1e-10 * sqrt(ss * yy)) {
        const int slot = st.hhead;
        float* Sd = a.Sh + ((size_t)p * m + slot) * Kp;
        float* Yd = a.Yh + ((size_t)p * m + slot) * Kp;
#pragma unroll
        for (int j = 0; j < E; ++j)
          if (valid[j]) {
            Sd[lane + 64 * j] = sv[j];
            Yd[lane + 64 * j] = yv[j];
          }
        rho_new = 1.0 / sy;
        if (lane == 0) a.rho[(size_t)p * m + slot] = rho_new;
        st.hhead = (slot + 1) % m;
        st.hcount = min(st.hcount + 1, m);
        pushed = true;
      }
      st.Fprev = st.F;
      st.F = Ft;
      st.iter += 1;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        x[j] = xt[j];
        g[j] = gt[j];
        if (valid[j]) {
          a.x[row + lane + 64 * j] = x[j];
          a.g[row + lane + 64 * j] = g[j];
        }
      }
      if (st.F == 0.0 || (st.Fprev - st.F) <= a.eps * st.Fprev) {
        st.status = ST_CONVERGED;
        stop = true;
      } else if (st.iter >= a.max_iter) {
        st.status = ST_MAXITER;
        stop = true;
      } else {
        need_dir = true;
      }
    } else {
      st.ntrial += 1;
      if (st.ntrial >= a.max_ls) {
        st.status = ST_LSFAIL;
        stop = true;
      } else {
        st.alpha *= a.beta;
        const float al = (float)st.alpha;
#pragma unroll
        for (int j = 0; j < E; ++j)
          if (valid[j]) a.xt[row + lane + 64 * j] = fmaf(al, d[j], x[j]);
      }
    }
  }

  if (need_dir) {
    const double gg = dot(g, g);
    if (gg == 0.0) {
      st.status = ST_CONVERGED;
      stop = true;
    } else {
      double alpha0 = 1.0;
      const int hc = st.hcount;
      if (hc == 0) {
#pragma unroll
        for (int j = 0; j < E; ++j) d[j] = -g[j];
        alpha0 = 1.0 / sqrt(gg);
      } else {
        // history in age order; the pair pushed this round comes from registers
        float hs[MH][E], hy[MH][E];
        double hr[MH];
#pragma unroll
        for (int i = 0; i < MH; ++i) {
          hr[i] = 0.0;
#pragma unroll
          for (int j = 0; j < E; ++j) {
            hs[i][j] = 0.f;
            hy[i][j] = 0.f;
          }
          if (i < hc) {
            if (i == 0 && pushed) {
              hr[0] = rho_new;
#pragma unroll
              for (int j = 0; j < E; ++j) {
                hs[0][j] = sv[j];
                hy[0][j] = yv[j];
              }
            } else {
              const int slot = (st.hhead - 1 - i + 2 * m) % m;
              const float* Sd = a.Sh + ((size_t)p * m + slot) * Kp;
              const float* Yd = a.Yh + ((size_t)p * m + slot) * Kp;
              hr[i] = a.rho[(size_t)p * m + slot];
#pragma unroll
              for (int j = 0; j < E; ++j)
                if (valid[j]) {
                  hs[i][j] = Sd[lane + 64 * j];
                  hy[i][j] = Yd[lane + 64 * j];
                }
            }
          }
        }
        // two-loop recursion: newest to oldest, scale, oldest to newest
        float qv[E];
#pragma unroll
        for (int j = 0; j < E; ++j) qv[j] = g[j];
        double al[MH];
#pragma unroll
        for (int i = 0; i < MH; ++i) {
          al[i] = 0.0;
          if (i < hc) {
            al[i] = hr[i] * dot(hs[i], qv);
            const float af = (float)al[i];
#pragma unroll
            for (int j = 0; j < E; ++j) qv[j] = fmaf(-af, hy[i][j], qv[j]);
          }
        }
        const double gamma = dot(hs[0], hy[0]) / dot(hy[0], hy[0]);
        const float gf = (float)gamma;
#pragma unroll
        for (int j = 0; j < E; ++j) qv[j] *= gf;
#pragma unroll
        for (int i = MH - 1; i >= 0; --i) {
          if (i < hc) {
            const double bi = hr[i] * dot(hy[i], qv);
            const float cf = (float)(al[i] - bi);
#pragma unroll
            for (int j = 0; j < E; ++j) qv[j] = fmaf(cf, hs[i][j], qv[j]);
          }
        }
#pragma unroll
        for (int j = 0; j < E; ++j) d[j] = -qv[j];
      }
      double gtp = dot(g, d);
      if (!(gtp < 0.0)) {  // not a descent direction: restart from -g
        st.hcount = 0;
        st.hhead = 0;
#pragma unroll
        for (int j = 0; j < E; ++j) d[j] = -g[j];
        gtp = -gg;
        alpha0 = 1.0 / sqrt(gg);
      }
      st.gtp = gtp;
      st.alpha = alpha0;
      st.ntrial = 0;
      const float af = (float)alpha0;
#pragma unroll
      for (int j = 0; j < E; ++j)
        if (valid[j]) {
          a.dir[row + lane + 64 * j] = d[j];
          a.xt[row + lane + 64 * j] = fmaf(af, d[j], x[j]);
        }
    }
  }
  if (stop) {
    // the next evaluation of this plan (if any) is at its final point
#pragma unroll
    for (int j = 0; j < E; ++j)
      if (valid[j]) a.xt[row + lane + 64 * j] = x[j];
  }
  if (lane == 0) {
    a.ps[p] = st;
    a.flag[p] = state_active(st.status) ? 1 : 0;
    if (state_active(st.status)) atomicAdd(&a.active_count[a.round & 1], 1);
  }
}

template <int E>
hipError_t launch_update_e(const UpdateArgs& a, hipStream_t st) {
  const dim3 grid((a.Pp + 3) / 4), block(256);
  if (a.m <= 4) hipLaunchKernelGGL((k_update<E, 4>), grid, block, 0, st, a);
  else if (a.m <= 10) hipLaunchKernelGGL((k_update<E, 10>), grid, block, 0, st, a);
  else if (a.m <= 16) hipLaunchKernelGGL((k_update<E, 16>), grid, block, 0, st, a);
  else hipLaunchKernelGGL((k_update<E, GMCO_MAX_HISTORY>), grid, block, 0, st, a);
  return hipGetLastError();
}

// Sum of the split-M gradient partials of every compact column, in split
// order: one thread per (column, 4 dwells), so the sum has the whole chip's
// parallelism however many splits a round uses.
__global__ __launch_bounds__(256) void k_reduce_g(const float* __restrict__ Gpart, const RoundTable* rt,
                                                  int Kp, float* __restrict__ Gsum) {
  const RoundTable r = *rt;
  const int nq = Kp / 4;
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const int j = (int)(idx / nq);
  const int c = (int)(idx - (long long)j * nq);
  if (j >= r.nact) return;
  const size_t stride = (size_t)r.ntiles * kPT * Kp;
  const float4* src = reinterpret_cast<const float4*>(Gpart + (size_t)j * Kp) + c;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  int s = 0;
  for (; s + 8 <= r.S; s += 8) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[(s + u) * stride / 4];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc.x += v[u].x;
      acc.y += v[u].y;
      acc.z += v[u].z;
      acc.w += v[u].w;
    }
  }
  for (; s < r.S; ++s) {
    const float4 v = src[s * stride / 4];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  reinterpret_cast<float4*>(Gsum + (size_t)j * Kp)[c] = acc;
}

// Partial reduction for a stand-alone evaluation: F = sum_s Fpart, g = 4 x G.
__global__ void k_finish_eval(const float* __restrict__ Gpart, const double* __restrict__ Fpart,
                              const float* __restrict__ x, int S, int P, int Pp, int K, int Kp,
                              double* __restrict__ F, double* __restrict__ g) {
  const int p = blockIdx.y;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  if (l < K) {
    float G = 0.f;
    for (int s = 0; s < S; ++s) G += Gpart[((size_t)s * Pp + p) * Kp + l];
    g[(size_t)p * K + l] = (double)(4.f * x[(size_t)p * Kp + l] * G);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double f = 0.0;
    for (int s = 0; s < S; ++s) f += Fpart[(size_t)s * Pp + p];
    F[p] = f;
  }
}

// Plans stopped by max_iter resume when the cap grows, and, on request, plans
// stopped by the stop rule or a failed line search: the current point is
// taken as the iterate again (history kept) and a new direction computed.
__global__ void k_resume(PlanState* ps, const float* __restrict__ x, float* __restrict__ xt,
                         int* __restrict__ flag, int Pp, int Kp, int max_iter, int resume_stopped) {
  const int p = blockIdx.x;
  if (p >= Pp) return;
  const int s = ps[p].status;
  const bool resume = (s == ST_MAXITER && ps[p].iter < max_iter) ||
                      (resume_stopped && (s == ST_CONVERGED || s == ST_LSFAIL) &&
                       ps[p].iter < max_iter);
  if (threadIdx.x == 0) flag[p] = (resume || state_active(s)) ? 1 : 0;
  if (!resume) return;
  for (int l = threadIdx.x; l < Kp; l += blockDim.x) xt[(size_t)p * Kp + l] = x[(size_t)p * Kp + l];
  __syncthreads();
  if (threadIdx.x == 0) {
    ps[p].status = ST_INIT;
    ps[p].nevals -= 1;  // the re-evaluation of the same point is not counted
  }
}

}  // namespace

hipError_t launch_update(const UpdateArgs& a, hipStream_t st) {
  const int E = (a.Kp + 63) / 64;
  switch (E) {
    case 1: return launch_update_e<1>(a, st);
    case 2: return launch_update_e<2>(a, st);
    case 3: return launch_update_e<3>(a, st);
    case 4: return launch_update_e<4>(a, st);
    case 5: return launch_update_e<5>(a, st);
    case 6: return launch_update_e<6>(a, st);
    case 7: return launch_update_e<7>(a, st);
    case 8: return launch_update_e<8>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce_g(const float* Gpart, const RoundTable* rt, int Pp, int Kp, float* Gsum,
                           hipStream_t st) {
  if (Kp % 4 != 0) return hipErrorInvalidValue;
  const long long threads = (long long)Pp * (Kp / 4);
  const dim3 grid((unsigned)((threads + 255) / 256));
  hipLaunchKernelGGL(k_reduce_g, grid, dim3(256), 0, st, Gpart, rt, Kp, Gsum);
  return hipGetLastError();
}

hipError_t launch_finish_eval(const float* Gpart, const double* Fpart, const float* x, int S,
                              int P, int Pp, int K, int Kp, double* F, double* g,
                              hipStream_t st) {
  dim3 grid((K + 127) / 128, P);
  hipLaunchKernelGGL(k_finish_eval, grid, dim3(128), 0, st, Gpart, Fpart, x, S, P, Pp, K, Kp, F,
                     g);
  return hipGetLastError();
}

hipError_t launch_resume(PlanState* ps, const float* x, float* xt, int* flag, int Pp, int Kp,
                         int max_iter, int resume_stopped, hipStream_t st) {
  hipLaunchKernelGGL(k_resume, dim3(Pp), dim3(128), 0, st, ps, x, xt, flag, Pp, Kp, max_iter,
                     resume_stopped);
  return hipGetLastError();
}

}  // namespace gmco
