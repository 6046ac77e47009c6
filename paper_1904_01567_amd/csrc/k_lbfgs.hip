// Batched L-BFGS state machine: one workgroup of two wavefronts per plan.
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
// Each lane owns groups of four consecutive dwells, so every vector operation
// is local to the lane and every dot product is one wavefront reduction.
#include "gmco_internal.h"

namespace gmco {
namespace {

// One lane's FP64 value moved across lanes by a DPP pattern (both halves).
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wavefront (all 64 lanes active), the same value in every lane:
// within each row of 16 lanes by DPP exchanges (pairs, quads, half-row
// mirror, row mirror; each step adds two equal-rounded operands, so every
// lane of a row ends with the same bits), then the four row sums in row
// order.  No LDS round-trips, so the chain of dependent dot products of the
// two-loop recursion stays short.
__device__ inline double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}

template <int E>
__device__ inline double dot(const float (&a)[E], const float (&b)[E]) {
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < E; ++j) s = fmaf(a[j], b[j], s);
  return wave_sum((double)s);
}

// Two-loop recursion (newest to oldest, scale gamma = s'y / y'y of the
// newest pair, oldest to newest) over hc pairs in age order; d = -H g.  With
// NEW, pair 0 is (sn, yn, rn) and pair i the stored pair i - 1; otherwise
// pair i is the stored pair i.  Every index is a compile-time constant, so
// the pairs are used where they were loaded.
template <int E, int MH, bool NEW>
__device__ inline void two_loop(const float (&g)[E], const float (&sn)[E], const float (&yn)[E],
                                double rn, const float (&os)[MH][E], const float (&oy)[MH][E],
                                const double (&orr)[MH], int hc, float (&d)[E]) {
#define GMCO_S(i) (NEW ? ((i) == 0 ? sn : os[(i) > 0 ? (i) - 1 : 0]) : os[(i)])
#define GMCO_Y(i) (NEW ? ((i) == 0 ? yn : oy[(i) > 0 ? (i) - 1 : 0]) : oy[(i)])
#define GMCO_R(i) (NEW ? ((i) == 0 ? rn : orr[(i) > 0 ? (i) - 1 : 0]) : orr[(i)])
  float qv[E];
#pragma unroll
  for (int j = 0; j < E; ++j) qv[j] = g[j];
  double al[MH];
#pragma unroll
  for (int i = 0; i < MH; ++i) {
    al[i] = 0.0;
    if (i < hc) {
      al[i] = GMCO_R(i) * dot(GMCO_S(i), qv);
      const float af = (float)al[i];
#pragma unroll
      for (int j = 0; j < E; ++j) qv[j] = fmaf(-af, GMCO_Y(i)[j], qv[j]);
    }
  }
  const double gamma = dot(GMCO_S(0), GMCO_Y(0)) / dot(GMCO_Y(0), GMCO_Y(0));
  const float gf = (float)gamma;
#pragma unroll
  for (int j = 0; j < E; ++j) qv[j] *= gf;
#pragma unroll
  for (int i = MH - 1; i >= 0; --i) {
    if (i < hc) {
      const double bi = GMCO_R(i) * dot(GMCO_Y(i), qv);
      const float cf = (float)(al[i] - bi);
#pragma unroll
      for (int j = 0; j < E; ++j) qv[j] = fmaf(cf, GMCO_S(i)[j], qv[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < E; ++j) d[j] = -qv[j];
#undef GMCO_S
#undef GMCO_Y
#undef GMCO_R
}

// Lane layout of a plan vector: element j of lane l is dwell
// 4 l + 256 (j / 4) + j % 4, so each group of four elements is one 16-byte
// access and a wavefront moves 1 KiB per instruction.  Groups at or past Kp
// read as zero (and add nothing to a dot product) and are not written.
template <int E>
__device__ inline void load_vec(const float* __restrict__ src, int lane, int Kp, float (&v)[E]) {
#pragma unroll
  for (int c = 0; c < E / 4; ++c) {
    const int e = 4 * lane + 256 * c;
    float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
    if (e < Kp) t = *reinterpret_cast<const float4*>(src + e);
    v[4 * c + 0] = t.x;
    v[4 * c + 1] = t.y;
    v[4 * c + 2] = t.z;
    v[4 * c + 3] = t.w;
  }
}

template <int E>
__device__ inline void store_vec(float* __restrict__ dst, int lane, int Kp, const float (&v)[E]) {
#pragma unroll
  for (int c = 0; c < E / 4; ++c) {
    const int e = 4 * lane + 256 * c;
    if (e < Kp)
      *reinterpret_cast<float4*>(dst + e) = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
  }
}

// Sums over the S split-M partials of up to two float4 of a gradient row
// (columns c0 and c0 + 64 of the row's float4, the second when two), each in
// split order, with the loads of both columns in flight together (16 splits
// at a time); stride4 = float4 between splits.
__device__ inline void sum_partials2(const float4* __restrict__ src, size_t stride4, int S, bool two,
                                     float4& acc0, float4& acc1) {
  acc0 = acc1 = make_float4(0.f, 0.f, 0.f, 0.f);
  auto add = [](float4& acc, const float4& v) {
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  };
  int s = 0;
  for (; s + 16 <= S; s += 16) {
    float4 v0[16], v1[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      v0[u] = src[(s + u) * stride4];
      v1[u] = two ? src[(s + u) * stride4 + 64] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      add(acc0, v0[u]);
      add(acc1, v1[u]);
    }
  }
  for (; s + 8 <= S; s += 8) {
    float4 v0[8], v1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      v0[u] = src[(s + u) * stride4];
      v1[u] = two ? src[(s + u) * stride4 + 64] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      add(acc0, v0[u]);
      add(acc1, v1[u]);
    }
  }
  for (; s < S; ++s) {
    add(acc0, src[s * stride4]);
    if (two) add(acc1, src[s * stride4 + 64]);
  }
}

template <int E>
__device__ inline void load_vec_lds(const float* src, int lane, int Kp, float (&v)[E]) {
#pragma unroll
  for (int c = 0; c < E / 4; ++c) {
    const int e = 4 * lane + 256 * c;
    float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
    if (e < Kp) t = *reinterpret_cast<const float4*>(src + e);
    v[4 * c + 0] = t.x;
    v[4 * c + 1] = t.y;
    v[4 * c + 2] = t.z;
    v[4 * c + 3] = t.w;
  }
}

// MH = register capacity for history pairs (MH >= m).  The pairs are held in
// registers in age order (0 = newest) so every loop index is a compile-time
// constant; all their loads are issued together before the recursion.
// One workgroup of two wavefronts per plan.  Wavefront 1 sums the split-M
// gradient partials of the plan's compact column, in split order, into LDS
// (so the round needs no separate reduction launch) while wavefront 0 loads
// the plan's vectors and history; wavefront 0 then advances the plan with G
// from LDS.  (Two wavefronts of up to 256 VGPRs per plan keep a 1,024-plan
// batch resident at once.)
template <int E, int MH>
__device__ inline void update_plans(const UpdateArgs& a, int p, int round) {
  __shared__ __attribute__((aligned(16))) float sGs[kKpMax];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (p == 0 && threadIdx.x == 0) a.active_count[(round + 1) & 1] = 0;
  if (p >= a.Pp) return;
  const int Kp = a.Kp;
  const int m = a.m;
  const size_t row = (size_t)p * Kp;

  // Two levels of loads: first the plan's state with the round's shape and
  // the plan's compact column (small, recently written), then, for a running
  // plan only, its vectors, history and gradient partials all at once.  A
  // stopped plan costs one 64-byte read per wavefront.
  PlanState st = a.ps[p];
  const RoundTable rt = *a.rt;
  const size_t col = (size_t)a.slot[p];
  if (!state_active(st.status)) return;  // (the same for the whole workgroup)
  const size_t stride = (size_t)rt.ntiles * kPT;
  if (wave == 1) {
    const int nq = Kp / 4;  // float4 of a row (Kp at most 512: two per lane)
    static_assert(kKpMax / 4 <= 128, "two float4 of a row per lane");
    if (lane < nq) {
      const float4* src = reinterpret_cast<const float4*>(a.Gpart + col * Kp) + lane;
      const bool two = lane + 64 < nq;
      float4 g0, g1;
      sum_partials2(src, stride * Kp / 4, rt.S, two, g0, g1);
      *reinterpret_cast<float4*>(&sGs[4 * lane]) = g0;
      if (two) *reinterpret_cast<float4*>(&sGs[4 * (lane + 64)]) = g1;
    }
  }
  // Wavefront 0 issues its loads before the barrier, so that they are in
  // flight while wavefront 1 sums the partials: the plan's vectors, the
  // stored history pairs in age order (0 = newest before this round; a pair
  // pushed this round is prepended from registers below, and a push
  // overwrites the oldest slot only after these loads) and the split
  // partials of F.
  float xt[E], gt[E], x[E], g[E], d[E];
  float G[E];
  const int hc0 = st.hcount;
  float ohs[MH][E], ohy[MH][E];
  double ohr[MH];
  double fpart = 0.0;
  if (wave == 0) {
    load_vec(a.xt + row, lane, Kp, xt);
    load_vec(a.x + row, lane, Kp, x);
    load_vec(a.g + row, lane, Kp, g);
    load_vec(a.dir + row, lane, Kp, d);
#pragma unroll
    for (int i = 0; i < MH; ++i) {
      ohr[i] = 0.0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        ohs[i][j] = 0.f;
        ohy[i][j] = 0.f;
      }
      if (i < hc0) {
        const int slot = (st.hhead - 1 - i + 2 * m) % m;
        const float* Sd = a.Sh + ((size_t)p * m + slot) * Kp;
        const float* Yd = a.Yh + ((size_t)p * m + slot) * Kp;
        ohr[i] = a.rho[(size_t)p * m + slot];
        load_vec(Sd, lane, Kp, ohs[i]);
        load_vec(Yd, lane, Kp, ohy[i]);
      }
    }
    for (int s = lane; s < rt.S; s += 64) fpart += a.Fpart[s * stride + col];
  }
  __syncthreads();
  if (wave > 0) return;

  // ---- objective and gradient at the evaluated point ----
  // gradient of this round's compact column, summed above; F from its
  // split partials in a fixed-order wave sum
  load_vec_lds(sGs, lane, Kp, G);
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
    }
    store_vec(a.x + row, lane, Kp, x);
    store_vec(a.g + row, lane, Kp, g);
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
        store_vec(Sd, lane, Kp, sv);
        store_vec(Yd, lane, Kp, yv);
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
      }
      store_vec(a.x + row, lane, Kp, x);
      store_vec(a.g + row, lane, Kp, g);
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
        float tr[E];
#pragma unroll
        for (int j = 0; j < E; ++j) tr[j] = fmaf(al, d[j], x[j]);
        store_vec(a.xt + row, lane, Kp, tr);
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
        // history in age order: the pair pushed this round (from registers),
        // then the stored pairs
        if (pushed)
          two_loop<E, MH, true>(g, sv, yv, rho_new, ohs, ohy, ohr, hc, d);
        else
          two_loop<E, MH, false>(g, sv, yv, rho_new, ohs, ohy, ohr, hc, d);
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
      float tr[E];
#pragma unroll
      for (int j = 0; j < E; ++j) tr[j] = fmaf(af, d[j], x[j]);
      store_vec(a.dir + row, lane, Kp, d);
      store_vec(a.xt + row, lane, Kp, tr);
    }
  }
  if (stop) {
    // the next evaluation of this plan (if any) is at its final point
    store_vec(a.xt + row, lane, Kp, x);
  }
  if (lane == 0) {
    a.ps[p] = st;
    a.flag[p] = state_active(st.status) ? 1 : 0;
    if (state_active(st.status)) atomicAdd(&a.active_count[round & 1], 1);
  }
}

template <int E, int MH>
__global__ __launch_bounds__(128) void k_update(UpdateArgs a) {
  update_plans<E, MH>(a, blockIdx.x, a.round);
}

// Grouped form: case blockIdx.y of n, its arguments from args (their round
// field is not used; all cases are in the same round).  Held to two waves
// per SIMD up to 10 history pairs: the case-table indirection would push it
// just past half the register file (one wave per SIMD); bounded, it spills
// a few registers and runs 16 % faster.
template <int E, int MH>
__global__ __launch_bounds__(128, (MH <= 10) ? 2 : 1) void k_update_grouped(const UpdateArgs* __restrict__ args,
                                                                           int round) {
  update_plans<E, MH>(args[blockIdx.y], blockIdx.x, round);
}

template <int E>
hipError_t launch_update_e(const UpdateArgs& a, hipStream_t st) {
  const dim3 grid(a.Pp), block(128);
  if (a.m <= 4) hipLaunchKernelGGL((k_update<E, 4>), grid, block, 0, st, a);
  else if (a.m <= 10) hipLaunchKernelGGL((k_update<E, 10>), grid, block, 0, st, a);
  else if (a.m <= 16) hipLaunchKernelGGL((k_update<E, 16>), grid, block, 0, st, a);
  else hipLaunchKernelGGL((k_update<E, GMCO_MAX_HISTORY>), grid, block, 0, st, a);
  return hipGetLastError();
}

template <int E>
hipError_t launch_update_grouped_e(const UpdateArgs* args, int n, int Pp_max, int m, int round,
                                   hipStream_t st) {
  const dim3 grid(Pp_max, n), block(128);
  if (m <= 4) hipLaunchKernelGGL((k_update_grouped<E, 4>), grid, block, 0, st, args, round);
  else if (m <= 10) hipLaunchKernelGGL((k_update_grouped<E, 10>), grid, block, 0, st, args, round);
  else if (m <= 16) hipLaunchKernelGGL((k_update_grouped<E, 16>), grid, block, 0, st, args, round);
  else hipLaunchKernelGGL((k_update_grouped<E, GMCO_MAX_HISTORY>), grid, block, 0, st, args, round);
  return hipGetLastError();
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
  // four consecutive dwells per lane and group; one or two groups
  if (a.Kp <= 256) return launch_update_e<4>(a, st);
  if (a.Kp <= 512) return launch_update_e<8>(a, st);
  return hipErrorInvalidValue;
}

hipError_t launch_update_grouped(const UpdateArgs* args, int n, int E, int Pp_max, int m, int round,
                                 hipStream_t st) {
  if (E == 4) return launch_update_grouped_e<4>(args, n, Pp_max, m, round, st);
  if (E == 8) return launch_update_grouped_e<8>(args, n, Pp_max, m, round, st);
  return hipErrorInvalidValue;
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
