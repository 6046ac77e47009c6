// Fused batched evaluation of the gMCO objective and its gradient.
//
// For a tile of 64 plans and a range of dose points, one workgroup computes
//   d   = D t                      eq. (dose), t = x^2 (Sec. 2.1.2)
//   f   = eq. 1 per point, F += (w_j / N_j) f             eq. (obj)
//   phi = (w_j / N_j) kappa(d)     kappa = the bracket of eq. 2
//   G  += D^T phi                  back-projection over the points
// and writes G and F as split-M partials; the gradient in x is 4 x * sum G
// (eq. 2).  The dose tile never leaves the chip: each 16-point block of D is
// staged once in LDS and feeds both products, the dwell times and the
// gradient accumulators of the wave's 16 plans stay in registers for the
// whole point range.
//
// Operand layout of the 16x16x4 matrix ops for lane l (q = l / 16, n = l % 16):
// A[n][q], B[q][n].  Accumulator register r holds C[4 q + r][n] for the FP32
// op and C[q + 4 r][n] for the FP64 op (measured on gfx950); the dose rows
// each lane holds therefore depend on the op, and the back-projection reads
// the matching rows of D.
#include "gmco_internal.h"

namespace gmco {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

namespace {

__device__ inline f4v mfma_f32(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// FP64 matrix op on FP32 operands: the products are exact in FP64 and the
// dose accumulates without FP32 rounding (same lane layout as the FP32 op).
__device__ inline d4v mfma_f64(float a, float b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, (double)b, c, 0, 0, 0);
}

// Maps the flat workgroup id to (split, tile).  Workgroups are dispatched to
// the 8 XCDs round-robin; when the grid allows it, all tiles of one point
// range land on the same XCD so that its L2 serves that slice of D to all of
// them.
__device__ inline void split_tile(int bid, int S, int ntiles, int& s, int& tile) {
  const int total = S * ntiles;
  if ((S & 7) == 0 && (total & 7) == 0) {
    const int xcd = bid & 7;
    const int local = bid >> 3;
    s = xcd * (S >> 3) + local / ntiles;
    tile = local % ntiles;
  } else {
    s = bid / ntiles;
    tile = bid % ntiles;
  }
}

// Resolves the evaluation's shape (split count S, tile count, row stride of
// the partial buffers), this workgroup's (split, first compact column j0) and
// the plan behind each of its kPT columns (-1: empty), and stages the
// columns' structure weights.  In a compacted round every workgroup ranks
// the running plans itself (a block-wide scan of the flags), so no separate
// launch is needed.  Returns false, for the whole workgroup, when the grid
// is larger than this round's S * ntiles.
template <int NT>
__device__ inline bool tile_setup(const EvalArgs& a, int* sPlan, int* sScan, float* sW, int& s,
                                  int& S, int& stride, int& j0) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int tile;
  if (a.flag == nullptr) {
    S = a.S;
    stride = a.Pp;
    if ((int)blockIdx.x >= S * a.ntiles) return false;
    split_tile(blockIdx.x, S, a.ntiles, s, tile);
    j0 = tile * kPT;
    if (tid < kPT) sPlan[tid] = j0 + tid;
  } else {
    if (tid < kPT) sPlan[tid] = -1;
    const int per = (a.P + NT - 1) / NT;
    const int b = tid * per;
    const int e = min(b + per, a.P);
    int cnt = 0;
    for (int p = b; p < e; ++p) cnt += a.flag[p];
    int v = cnt;  // inclusive scan over the wavefront, then over the waves
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    if (lane == 63) sScan[wave] = v;
    __syncthreads();
    int base = 0, nact = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      const int t = sScan[w];
      base += w < wave ? t : 0;
      nact += t;
    }
    const int ntiles = (nact + kPT - 1) / kPT;
    S = (a.s_tuned > 0 && ntiles == a.ntiles) ? a.s_tuned : a.split_tab[ntiles];
    stride = ntiles * kPT;
    if (blockIdx.x == 0 && tid == 0) {
      RoundTable r;
      r.nact = nact;
      r.ntiles = ntiles;
      r.S = S;
      r.pad = 0;
      *a.rt = r;
      if (a.work != nullptr) *a.work += (unsigned long long)nact;
      if (a.work2 != nullptr) *a.work2 += (unsigned long long)nact;
    }
    if ((int)blockIdx.x >= S * ntiles) return false;
    split_tile(blockIdx.x, S, ntiles, s, tile);
    j0 = tile * kPT;
    int r = base + v - cnt;
    for (int p = b; p < e; ++p) {
      if (a.flag[p]) {
        if (r >= j0 && r < j0 + kPT) {
          sPlan[r - j0] = p;
          if (s == 0) a.slot[p] = r;
        }
        ++r;
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < kPT * kGmax; i += NT) {
    const int pl = sPlan[i / kGmax];
    sW[i] = pl >= 0 ? a.wn[(size_t)pl * kGmax + (i % kGmax)] : 0.f;
  }
  return true;
}

// float4-chunk swizzle of row `row` of the FP64-accumulating kernel's LDS tile
__device__ inline int swz_row(int row) { return (row >> 1) & 3; }

// MODE_F32    : FP32 operands, FP32 accumulation (v_mfma_f32_16x16x4_f32).
// MODE_CHUNK64: FP32 matrix ops sum 16 dwells at a time from zero; those
//               partial doses are accumulated in FP64 on the vector ALU and
//               the penalty is evaluated in FP64.
// The back-projection is FP32 in both.  (FP32 operands with the dose
// accumulated in FP64 have a kernel of their own, k_eval_acc64, below.)
enum { MODE_F32 = 0, MODE_CHUNK64 = 2 };

template <int KP, int MODE>
__global__ __launch_bounds__(256, 1) void k_eval_f32(EvalArgs a) {
  // LDS row stride (floats): the dose product reads rows n = 0..15 as float4
  // at one column, the back-projection 16 consecutive columns of rows
  // 4q + r; Kp + 4 is conflict-free for both.
  constexpr int KS = KP + 4;
  constexpr int NK16 = KP / 16;    // 16-dwell slices
  constexpr int NF4 = 4 * KP;      // float4 per 16-point block
  constexpr int NPF = (NF4 + 255) / 256;

  __shared__ __attribute__((aligned(16))) float sD[2][kBM * KS];
  __shared__ float sW[kPT * kGmax];
  __shared__ int sPlan[kPT];
  __shared__ int sScan[4];
  __shared__ float4 sP[kGmax + 1];
  __shared__ double sP64[kGmax + 1][4];
  __shared__ int sG[2][kBM];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;

  int s, S, stride, j0;
  if (!tile_setup<256>(a, sPlan, sScan, sW, s, S, stride, j0)) return;
#pragma unroll
  for (int j = 0; j <= kGmax; ++j)
    if (tid == j) {
      sP[j] = a.gt.prm[j];
#pragma unroll
      for (int c = 0; c < 4; ++c) sP64[j][c] = a.gt.prm64[j][c];
    }

  const int col = wave * 16 + n;
  const int plan = sPlan[col];
  const bool pv = plan >= 0;  // an empty column evaluates t = 0 with zero weights
  const float* __restrict__ xrow = a.x + (size_t)(pv ? plan : 0) * KP;
  // B operand of the dose product: lane (q, n) holds t = x^2 of plan n at
  // dwells 16 k + 4 q + j (j = 0..3) for slice k.
  float tf[KP / 4];
#pragma unroll
  for (int k = 0; k < NK16; ++k) {
    const float4 xv = *reinterpret_cast<const float4*>(xrow + 16 * k + 4 * q);
    tf[4 * k + 0] = pv ? xv.x * xv.x : 0.f;
    tf[4 * k + 1] = pv ? xv.y * xv.y : 0.f;
    tf[4 * k + 2] = pv ? xv.z * xv.z : 0.f;
    tf[4 * k + 3] = pv ? xv.w * xv.w : 0.f;
  }
  f4v gacc[NK16];
#pragma unroll
  for (int k = 0; k < NK16; ++k) gacc[k] = f4v{0.f, 0.f, 0.f, 0.f};
  double facc = 0.0;

  const int b_begin = (int)(((long long)s * a.nblocks) / S);
  const int b_end = (int)(((long long)(s + 1) * a.nblocks) / S);
  const f4v* __restrict__ Dg = reinterpret_cast<const f4v*>(a.D);

  // Software pipeline over 16-point blocks with two LDS buffers: while the
  // dose product of block b runs on one buffer, the back-projection of block
  // b-1 runs on the other, so the matrix pipe always has independent work.
  f4v pf[NPF];
  int gpre = 0;
#define GMCO_PREFETCH(blk)                                                  \
  {                                                                         \
    const f4v* src_ = Dg + (size_t)(blk) * NF4;                             \
    _Pragma("unroll") for (int i = 0; i < NPF; ++i) {                       \
      const int idx = tid + 256 * i;                                        \
      if (NF4 % 256 == 0 || idx < NF4) pf[i] = src_[idx];                   \
    }                                                                       \
    if (tid < kBM) gpre = a.grp[(blk) * kBM + tid];                         \
  }
#define GMCO_STAGE(buf)                                                     \
  {                                                                         \
    _Pragma("unroll") for (int i = 0; i < NPF; ++i) {                       \
      const int idx = tid + 256 * i;                                        \
      if (NF4 % 256 == 0 || idx < NF4) {                                    \
        const int row = idx / (KP / 4);                                     \
        const int c4 = idx - row * (KP / 4);                                \
        *reinterpret_cast<f4v*>(&sD[(buf)][row * KS + 4 * c4]) = pf[i];     \
      }                                                                     \
    }                                                                       \
    if (tid < kBM) sG[(buf)][tid] = gpre;                                   \
  }

  float phi_prev[4] = {0.f, 0.f, 0.f, 0.f};
  for (int i = tid; i < kBM * KS; i += 256) sD[1][i] = 0.f;
  if (b_begin < b_end) GMCO_PREFETCH(b_begin);
#pragma unroll 1
  for (int b = b_begin; b <= b_end; ++b) {
    const int cur = (b - b_begin) & 1;
    const int prv = cur ^ 1;
    // The first iteration back-projects phi_prev = 0 over a zeroed buffer and
    // the last one repeats a dose product whose result is discarded: both are
    // harmless and keep the matrix loop free of branches.
    const bool have_cur = b < b_end;
    __syncthreads();
    if (have_cur) GMCO_STAGE(cur);
    __syncthreads();
    if (b + 1 < b_end) GMCO_PREFETCH(b + 1);

    float phi[4] = {0.f, 0.f, 0.f, 0.f};
    const float* __restrict__ Dc = sD[cur];
    const float* __restrict__ Dp = sD[prv];
    if constexpr (MODE == MODE_CHUNK64) {
      const f4v z = {0.f, 0.f, 0.f, 0.f};
      double ds[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < NK16; ++k) {
        const float4 av = *reinterpret_cast<const float4*>(&Dc[n * KS + 16 * k + 4 * q]);
        // one 16-dwell partial per slice, interleaved with the back-projection
        f4v c0 = mfma_f32(av.x, tf[4 * k + 0], z);
        gacc[k] = mfma_f32(Dp[(4 * q + 0) * KS + 16 * k + n], phi_prev[0], gacc[k]);
        c0 = mfma_f32(av.y, tf[4 * k + 1], c0);
        gacc[k] = mfma_f32(Dp[(4 * q + 1) * KS + 16 * k + n], phi_prev[1], gacc[k]);
        c0 = mfma_f32(av.z, tf[4 * k + 2], c0);
        gacc[k] = mfma_f32(Dp[(4 * q + 2) * KS + 16 * k + n], phi_prev[2], gacc[k]);
        c0 = mfma_f32(av.w, tf[4 * k + 3], c0);
        gacc[k] = mfma_f32(Dp[(4 * q + 3) * KS + 16 * k + n], phi_prev[3], gacc[k]);
#pragma unroll
        for (int r = 0; r < 4; ++r) ds[r] += (double)c0[r];
      }
      if (have_cur) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double d = ds[r];
          const int gi = sG[cur][4 * q + r];
          const float w = (gi < kGmax) ? sW[(wave * 16 + n) * kGmax + gi] : 0.f;
          const double lo = fmin(d - sP64[gi][1], 0.0);
          const double hi = fmax(d - sP64[gi][2], 0.0);
          const double kap = sP64[gi][0] * lo + sP64[gi][3] * hi;
          facc += (double)w * (kap * (lo + hi));
          phi[r] = (float)((double)w * kap);
        }
      }
    } else {
      f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
      for (int k = 0; k < NK16; ++k) {
        const float4 av = *reinterpret_cast<const float4*>(&Dc[n * KS + 16 * k + 4 * q]);
        acc0 = mfma_f32(av.x, tf[4 * k + 0], acc0);
        acc1 = mfma_f32(av.y, tf[4 * k + 1], acc1);
        acc0 = mfma_f32(av.z, tf[4 * k + 2], acc0);
        acc1 = mfma_f32(av.w, tf[4 * k + 3], acc1);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          gacc[k] = mfma_f32(Dp[(4 * q + r) * KS + 16 * k + n], phi_prev[r], gacc[k]);
      }
      if (have_cur) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float d = acc0[r] + acc1[r];
          const int gi = sG[cur][4 * q + r];
          const float4 pr = sP[gi];
          const float w = (gi < kGmax) ? sW[(wave * 16 + n) * kGmax + gi] : 0.f;
          const float lo = fminf(d - pr.y, 0.f);
          const float hi = fmaxf(d - pr.z, 0.f);
          const float kap = pr.x * lo + pr.w * hi;
          facc += (double)(w * (kap * (lo + hi)));
          phi[r] = w * kap;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) phi_prev[r] = phi[r];
  }
#undef GMCO_PREFETCH
#undef GMCO_STAGE

  // ---- write split partials ----
  float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP;
#pragma unroll
  for (int k = 0; k < NK16; ++k) {
    *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) =
        make_float4(gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]);
  }
  facc += __shfl_xor(facc, 16);
  facc += __shfl_xor(facc, 32);
  if (q == 0) a.Fpart[(size_t)s * stride + j0 + col] = facc;
}

// ---------------------------------------------------------------------------
// MODE_ACC64 (FP32 operands, FP64-accumulated dose, FP64 penalty, FP32
// back-projection) with 512 threads: two waves per SIMD.  The FP64 matrix op
// reaches its full rate only when two waves per SIMD issue it, and a wave
// that holds t and the gradient accumulators of 16 plans over all Kp dwells
// does not fit in half the register file.  So the 8 waves form 4 plan groups
// (16 plans each) x 2 dwell halves: each wave forms the partial dose of its
// dwell half, the two partials of a plan group are added through LDS in a
// fixed order, both waves evaluate eq. 1 on the sum, and each back-projects
// onto its own dwell half.  Same software pipeline as the 256-thread kernel
// (dose product of block b with the back-projection of block b-1, two LDS
// buffers), with two barriers per block.
// LDS tile row stride Kp + 16 with the float4 chunk index of row R XORed with
// (R >> 1) & 3: the back-projection reads 16 columns of rows q + 4r (the FP64
// op's row order), which that stride puts on opposite bank halves for
// q = 0, 1, and the swizzle keeps the dose product's float4 reads of rows
// 0..15 conflict-free.
// ---------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(512, 1) void k_eval_acc64(EvalArgs a) {
  constexpr int NT = 512;
  constexpr int KS = KP + 16;
  constexpr int NKH = KP / 32;      // 16-dwell slices per dwell half
  constexpr int NF4 = 4 * KP;       // float4 per 16-point block
  constexpr int NPF = (NF4 + NT - 1) / NT;

  __shared__ __attribute__((aligned(16))) float sD[2][kBM * KS];
  __shared__ double sX[2][4][4][64];  // partial doses [half][group][r][lane]
  __shared__ float sPhi[4][4][64];     // phi of the last block [group][r][lane]
  __shared__ double sF[4][64];         // F partial of the half-1 waves [group][lane]
  __shared__ float sW[kPT * kGmax];
  __shared__ int sPlan[kPT];
  __shared__ int sScan[NT / 64];
  __shared__ double sP64[kGmax + 1][4];
  __shared__ int sG[2][kBM];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;
  const int grp = wave & 3;   // plan group: columns 16 grp .. 16 grp + 15
  const int half = wave >> 2; // dwell half: slices half * NKH .. half * NKH + NKH - 1

  int s, S, stride, j0;
  if (!tile_setup<NT>(a, sPlan, sScan, sW, s, S, stride, j0)) return;
#pragma unroll
  for (int j = 0; j <= kGmax; ++j)
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sP64[j][c] = a.gt.prm64[j][c];
    }

  const int col = grp * 16 + n;
  const int plan = sPlan[col];
  const bool pv = plan >= 0;  // an empty column evaluates t = 0 with zero weights
  const float* __restrict__ xrow = a.x + (size_t)(pv ? plan : 0) * KP + half * (KP / 2);
  // t = x^2 of plan n at dwells 16 k + 4 q + j of this wave's half (slice k)
  float tf[KP / 8];
#pragma unroll
  for (int k = 0; k < NKH; ++k) {
    const float4 xv = *reinterpret_cast<const float4*>(xrow + 16 * k + 4 * q);
    tf[4 * k + 0] = pv ? xv.x * xv.x : 0.f;
    tf[4 * k + 1] = pv ? xv.y * xv.y : 0.f;
    tf[4 * k + 2] = pv ? xv.z * xv.z : 0.f;
    tf[4 * k + 3] = pv ? xv.w * xv.w : 0.f;
  }
  f4v gacc[NKH];
#pragma unroll
  for (int k = 0; k < NKH; ++k) gacc[k] = f4v{0.f, 0.f, 0.f, 0.f};
  double facc = 0.0;

  const int b_begin = (int)(((long long)s * a.nblocks) / S);
  const int b_end = (int)(((long long)(s + 1) * a.nblocks) / S);
  const f4v* __restrict__ Dg = reinterpret_cast<const f4v*>(a.D);

  f4v pf[NPF];
  int gpre = 0;
#define GMCO_PF64(blk)                                                      \
  {                                                                         \
    const f4v* src_ = Dg + (size_t)(blk) * NF4;                             \
    _Pragma("unroll") for (int i = 0; i < NPF; ++i) {                       \
      const int idx = tid + NT * i;                                         \
      if (NF4 % NT == 0 || idx < NF4) pf[i] = src_[idx];                    \
    }                                                                       \
    if (tid < kBM) gpre = a.grp[(blk) * kBM + tid];                         \
  }
#define GMCO_ST64(buf)                                                      \
  {                                                                         \
    _Pragma("unroll") for (int i = 0; i < NPF; ++i) {                       \
      const int idx = tid + NT * i;                                         \
      if (NF4 % NT == 0 || idx < NF4) {                                     \
        const int row = idx / (KP / 4);                                     \
        const int c4 = idx - row * (KP / 4);                                \
        *reinterpret_cast<f4v*>(&sD[(buf)][row * KS + 4 * (c4 ^ swz_row(row))]) = pf[i]; \
      }                                                                     \
    }                                                                       \
    if (tid < kBM) sG[(buf)][tid] = gpre;                                   \
  }

  for (int i = tid; i < kBM * KS; i += NT) sD[1][i] = 0.f;
  for (int i = tid; i < 4 * 4 * 64; i += NT) (&sPhi[0][0][0])[i] = 0.f;
  if (b_begin < b_end) GMCO_PF64(b_begin);
#pragma unroll 1
  for (int b = b_begin; b <= b_end; ++b) {
    const int cur = (b - b_begin) & 1;
    const int prv = cur ^ 1;
    // As in the 256-thread kernel: the first iteration back-projects
    // phi_prev = 0 over a zeroed buffer and the last repeats a dose product
    // whose result is discarded.
    const bool have_cur = b < b_end;
    // Buffer `cur` was last read by the previous iteration's matrix loop,
    // which every wave finished before that iteration's second barrier.
    if (have_cur) GMCO_ST64(cur);
    __syncthreads();
    if (b + 1 < b_end) GMCO_PF64(b + 1);

    const float* __restrict__ Dc = sD[cur];
    const float* __restrict__ Dp = sD[prv];
    // phi of block b-1 for the back-projection, written by the two waves of
    // this plan group (rows 0-1 and 2-3) before the barrier above
    float phi_prev[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) phi_prev[r] = sPhi[grp][r][lane];
    d4v acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
#pragma unroll
    for (int k = 0; k < NKH; ++k) {
      const int kg = half * NKH + k;
      const float4 av = *reinterpret_cast<const float4*>(&Dc[n * KS + 16 * kg + 4 * (q ^ swz_row(n))]);
      acc0 = mfma_f64(av.x, tf[4 * k + 0], acc0);
      acc1 = mfma_f64(av.y, tf[4 * k + 1], acc1);
      acc2 = mfma_f64(av.z, tf[4 * k + 2], acc2);
      acc3 = mfma_f64(av.w, tf[4 * k + 3], acc3);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        gacc[k] = mfma_f32(Dp[(q + 4 * r) * KS + 16 * kg + (n ^ (swz_row(q + 4 * r) << 2))],
                           phi_prev[r], gacc[k]);
    }
    // partial dose of points q + 4 r (the FP64 op's rows) for plan n
#pragma unroll
    for (int r = 0; r < 4; ++r) sX[half][grp][r][lane] = (acc0[r] + acc1[r]) + (acc2[r] + acc3[r]);
    __syncthreads();
    // eq. 1 on the summed dose: each wave of the group takes two of the four
    // rows (points q + 4r) and shares phi through LDS; the next iteration's
    // first barrier orders these writes before their reads
    if (have_cur) {
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) {
        const int r = 2 * half + rr;
        const double d = sX[0][grp][r][lane] + sX[1][grp][r][lane];
        const int gi = sG[cur][q + 4 * r];
        const float w = (gi < kGmax) ? sW[col * kGmax + gi] : 0.f;
        // without branches: at most one of the two deviations is nonzero
        const double lo = fmin(d - sP64[gi][1], 0.0);
        const double hi = fmax(d - sP64[gi][2], 0.0);
        const double kap = sP64[gi][0] * lo + sP64[gi][3] * hi;
        facc += (double)w * (kap * (lo + hi));
        sPhi[grp][r][lane] = (float)((double)w * kap);
      }
    }
  }
#undef GMCO_PF64
#undef GMCO_ST64

  // ---- split partials: each wave its dwell half; F from one wave per group ----
  float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP + half * (KP / 2);
#pragma unroll
  for (int k = 0; k < NKH; ++k) {
    *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) =
        make_float4(gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]);
  }
  // F partial: rows 0-1 (half 0) + rows 2-3 (half 1), then over q
  if (half == 1) sF[grp][lane] = facc;
  __syncthreads();
  if (half == 0) {
    facc += sF[grp][lane];
    facc += __shfl_xor(facc, 16);
    facc += __shfl_xor(facc, 32);
    if (q == 0) a.Fpart[(size_t)s * stride + j0 + col] = facc;
  }
}

// ---------------------------------------------------------------------------
// BF16 operands, FP32 accumulation: v_mfma_f32_16x16x32_bf16.  Lane l
// (q = l / 16, n = l % 16) supplies A[n][8q .. 8q+7] and B[8q .. 8q+7][n];
// accumulator register r holds C[4q + r][n].  Blocks of 32 points: the dose
// product runs two 16-point row tiles, after which each lane holds the
// penalty derivative of points {4q..4q+3} and {16+4q..16+4q+3} of its plan,
// exactly the 8 contraction slots it supplies to the back-projection; the
// back-projection's A operand (D transposed) is read in that same point
// order from a dwell-major copy of the tile.
// ---------------------------------------------------------------------------
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

__device__ inline f4v mfma_bf16(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int KP>
__global__ __launch_bounds__(256, 1) void k_eval_bf16(EvalArgs a) {
  constexpr int BMP = 32;              // points per block
  constexpr int DS = KP + 8;           // D tile row stride (elements): conflict-free b128 reads
  constexpr int TS = BMP + 4;          // transposed tile row stride: conflict-free b64 reads
  constexpr int NK32 = KP / 32;        // k-steps of the dose product
  constexpr int NK16 = KP / 16;        // 16-dwell tiles of the back-projection
  constexpr int NCH = BMP * KP / 8;    // 16-byte chunks per tile (both tiles)
  constexpr int NPF = (NCH + 255) / 256;

  __shared__ __attribute__((aligned(16))) __bf16 sD[BMP * DS];
  __shared__ __attribute__((aligned(16))) __bf16 sT[KP * TS];
  __shared__ float sW[kPT * kGmax];
  __shared__ int sPlan[kPT];
  __shared__ int sScan[4];
  __shared__ float4 sP[kGmax + 1];
  __shared__ int sG[BMP];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;
  int s, S, stride, j0;
  if (!tile_setup<256>(a, sPlan, sScan, sW, s, S, stride, j0)) return;
#pragma unroll
  for (int j = 0; j <= kGmax; ++j)
    if (tid == j) sP[j] = a.gt.prm[j];

  const int col = wave * 16 + n;
  const int plan = sPlan[col];
  const bool pv = plan >= 0;  // an empty column evaluates t = 0 with zero weights
  const float* __restrict__ xrow = a.x + (size_t)(pv ? plan : 0) * KP;
  // B operand of the dose product: t = x^2 of plan n at dwells 32 k + 8 q + e
  bf8v tb[NK32];
#pragma unroll
  for (int k = 0; k < NK32; ++k) {
    const float4 x0 = *reinterpret_cast<const float4*>(xrow + 32 * k + 8 * q);
    const float4 x1 = *reinterpret_cast<const float4*>(xrow + 32 * k + 8 * q + 4);
    tb[k][0] = (__bf16)(pv ? x0.x * x0.x : 0.f);
    tb[k][1] = (__bf16)(pv ? x0.y * x0.y : 0.f);
    tb[k][2] = (__bf16)(pv ? x0.z * x0.z : 0.f);
    tb[k][3] = (__bf16)(pv ? x0.w * x0.w : 0.f);
    tb[k][4] = (__bf16)(pv ? x1.x * x1.x : 0.f);
    tb[k][5] = (__bf16)(pv ? x1.y * x1.y : 0.f);
    tb[k][6] = (__bf16)(pv ? x1.z * x1.z : 0.f);
    tb[k][7] = (__bf16)(pv ? x1.w * x1.w : 0.f);
  }
  f4v gacc[NK16];
#pragma unroll
  for (int k = 0; k < NK16; ++k) gacc[k] = f4v{0.f, 0.f, 0.f, 0.f};
  double facc = 0.0;

  const int nb = a.Mp / BMP;
  const int b_begin = (int)(((long long)s * nb) / S);
  const int b_end = (int)(((long long)(s + 1) * nb) / S);
  const u4v* __restrict__ Dg = reinterpret_cast<const u4v*>(a.D);
  const __bf16* __restrict__ DTg = reinterpret_cast<const __bf16*>(a.DT);

  u4v pd[NPF], pt[NPF];
  int gpre = 0;
#define GMCO_PF16(blk)                                                          \
  {                                                                             \
    const u4v* srcd = Dg + (size_t)(blk) * NCH;                                 \
    _Pragma("unroll") for (int i = 0; i < NPF; ++i) {                           \
      const int c = tid + 256 * i;                                              \
      if (NCH % 256 == 0 || c < NCH) {                                          \
        pd[i] = srcd[c];                                                        \
        const int l = c >> 2, part = c & 3;                                    \
        pt[i] = *reinterpret_cast<const u4v*>(DTg + (size_t)l * a.Mp +          \
                                                (size_t)(blk) * BMP + part * 8); \
      }                                                                         \
    }                                                                           \
    if (tid < BMP) gpre = a.grp[(blk) * BMP + tid];                             \
  }
  if (b_begin < b_end) GMCO_PF16(b_begin);

  for (int b = b_begin; b < b_end; ++b) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int c = tid + 256 * i;
      if (NCH % 256 == 0 || c < NCH) {
        const int row = c / (KP / 8), c8 = c - row * (KP / 8);
        *reinterpret_cast<u4v*>(&sD[row * DS + 8 * c8]) = pd[i];
        const int l = c >> 2, part = c & 3;
        u2v* dst = reinterpret_cast<u2v*>(&sT[l * TS + part * 8]);
        dst[0] = u2v{pt[i][0], pt[i][1]};
        dst[1] = u2v{pt[i][2], pt[i][3]};
      }
    }
    if (tid < BMP) sG[tid] = gpre;
    __syncthreads();
    {
      const int bn = (b + 1 < b_end) ? b + 1 : b;
      GMCO_PF16(bn);
    }

    // ---- dose product for the two 16-point row tiles ----
    f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
    for (int k = 0; k < NK32; ++k) {
      const bf8v a0 = *reinterpret_cast<const bf8v*>(&sD[n * DS + 32 * k + 8 * q]);
      const bf8v a1 = *reinterpret_cast<const bf8v*>(&sD[(16 + n) * DS + 32 * k + 8 * q]);
      acc0 = mfma_bf16(a0, tb[k], acc0);
      acc1 = mfma_bf16(a1, tb[k], acc1);
    }
    // ---- penalty epilogue ----
    bf8v phi;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float d = e < 4 ? acc0[e] : acc1[e - 4];
      const int pt_ = e < 4 ? 4 * q + e : 16 + 4 * q + (e - 4);
      const int gi = sG[pt_];
      const float4 pr = sP[gi];
      const float w = (gi < kGmax) ? sW[(wave * 16 + n) * kGmax + gi] : 0.f;
      float kap = 0.f, dev = 0.f;
      if (d < pr.y) {
        dev = d - pr.y;
        kap = pr.x * dev;
      } else if (d > pr.z) {
        dev = d - pr.z;
        kap = pr.w * dev;
      }
      facc += (double)(w * (kap * dev));
      phi[e] = (__bf16)(w * kap);
    }
    // ---- back-projection over the 32 points ----
#pragma unroll
    for (int k = 0; k < NK16; ++k) {
      const bf4v lo = *reinterpret_cast<const bf4v*>(&sT[(16 * k + n) * TS + 4 * q]);
      const bf4v hi = *reinterpret_cast<const bf4v*>(&sT[(16 * k + n) * TS + 16 + 4 * q]);
      const bf8v av = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      gacc[k] = mfma_bf16(av, phi, gacc[k]);
    }
  }
#undef GMCO_PF16

  float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP;
#pragma unroll
  for (int k = 0; k < NK16; ++k) {
    *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) =
        make_float4(gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]);
  }
  facc += __shfl_xor(facc, 16);
  facc += __shfl_xor(facc, 32);
  if (q == 0) a.Fpart[(size_t)s * stride + j0 + col] = facc;
}

// ---------------------------------------------------------------------------
// FP8 dose product (e4m3, v_mfma_f32_16x16x32_fp8_fp8, same lane layout as the
// BF16 op with 8 one-byte elements per lane): D is stored as D_il / s_l with
// one scale per dwell column (s_l = max_i D_il / 224), the dwell times enter
// as t_l s_l / u_p with one scale per plan (u_p = max_l t_l s_l / 224), and
// d = u_p * sum.  The back-projection runs in BF16 on the BF16 transposed
// copy of D, as in the BF16 kernel.  Both conversions use the hardware's own
// FP8 encoding, so the format convention never enters the arithmetic.
// ---------------------------------------------------------------------------
__device__ inline f4v mfma_fp8(long a, long b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

__device__ inline unsigned pack_fp8x4(float a, float b, float c, float d) {
  int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, lo, true);
}

template <int KP>
__global__ __launch_bounds__(256, 1) void k_eval_fp8(EvalArgs a) {
  constexpr int BMP = 32;
  constexpr int DS = KP + 8;           // FP8 tile row stride (bytes): conflict-free b64 reads
  constexpr int TS = BMP + 4;          // BF16 transposed tile row stride (elements)
  constexpr int NK32 = KP / 32;
  constexpr int NK16 = KP / 16;
  constexpr int NCH8 = BMP * KP / 16;  // 16-byte chunks of the FP8 tile
  constexpr int NCH = BMP * KP / 8;    // 16-byte chunks of the BF16 transposed tile
  constexpr int NPF8 = (NCH8 + 255) / 256;
  constexpr int NPF = (NCH + 255) / 256;

  __shared__ __attribute__((aligned(16))) unsigned char sD[BMP * DS];
  __shared__ __attribute__((aligned(16))) __bf16 sT[KP * TS];
  __shared__ float sW[kPT * kGmax];
  __shared__ int sPlan[kPT];
  __shared__ int sScan[4];
  __shared__ float4 sP[kGmax + 1];
  __shared__ int sG[BMP];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;
  int s, S, stride, j0;
  if (!tile_setup<256>(a, sPlan, sScan, sW, s, S, stride, j0)) return;
#pragma unroll
  for (int j = 0; j <= kGmax; ++j)
    if (tid == j) sP[j] = a.gt.prm[j];

  const int col = wave * 16 + n;
  const int plan = sPlan[col];
  const bool pv = plan >= 0;  // an empty column evaluates t = 0 with zero weights
  const float* __restrict__ xrow = a.x + (size_t)(pv ? plan : 0) * KP;
  // scaled dwell times t_l s_l, their per-plan maximum, then FP8 and BF16 fragments
  float ts[NK32][8];
  float tmax = 0.f;
#pragma unroll
  for (int k = 0; k < NK32; ++k) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int l = 32 * k + 8 * q + e;
      const float xv = xrow[l];
      ts[k][e] = pv ? xv * xv * a.colscale[l] : 0.f;
      tmax = fmaxf(tmax, ts[k][e]);
    }
  }
  tmax = fmaxf(tmax, __shfl_xor(tmax, 16));
  tmax = fmaxf(tmax, __shfl_xor(tmax, 32));
  const float u = tmax > 0.f ? tmax / 224.f : 1.f;
  const float inv_u = 1.f / u;
  long tb[NK32];
#pragma unroll
  for (int k = 0; k < NK32; ++k) {
    const unsigned lo = pack_fp8x4(ts[k][0] * inv_u, ts[k][1] * inv_u, ts[k][2] * inv_u, ts[k][3] * inv_u);
    const unsigned hi = pack_fp8x4(ts[k][4] * inv_u, ts[k][5] * inv_u, ts[k][6] * inv_u, ts[k][7] * inv_u);
    tb[k] = (long)(((unsigned long)hi << 32) | lo);
  }
  f4v gacc[NK16];
#pragma unroll
  for (int k = 0; k < NK16; ++k) gacc[k] = f4v{0.f, 0.f, 0.f, 0.f};
  double facc = 0.0;

  const int nb = a.Mp / BMP;
  const int b_begin = (int)(((long long)s * nb) / S);
  const int b_end = (int)(((long long)(s + 1) * nb) / S);
  const u4v* __restrict__ Dg = reinterpret_cast<const u4v*>(a.D);
  const __bf16* __restrict__ DTg = reinterpret_cast<const __bf16*>(a.DT);

  u4v pd[NPF8], pt[NPF];
  int gpre = 0;
#define GMCO_PF8(blk)                                                           \
  {                                                                             \
    const u4v* srcd = Dg + (size_t)(blk) * NCH8;                                \
    _Pragma("unroll") for (int i = 0; i < NPF8; ++i) {                          \
      const int c = tid + 256 * i;                                              \
      if (NCH8 % 256 == 0 || c < NCH8) pd[i] = srcd[c];                         \
    }                                                                           \
    _Pragma("unroll") for (int i = 0; i < NPF; ++i) {                           \
      const int c = tid + 256 * i;                                              \
      if (NCH % 256 == 0 || c < NCH) {                                          \
        const int l = c >> 2, part = c & 3;                                     \
        pt[i] = *reinterpret_cast<const u4v*>(DTg + (size_t)l * a.Mp +          \
                                              (size_t)(blk) * BMP + part * 8);  \
      }                                                                         \
    }                                                                           \
    if (tid < BMP) gpre = a.grp[(blk) * BMP + tid];                             \
  }
  if (b_begin < b_end) GMCO_PF8(b_begin);

  for (int b = b_begin; b < b_end; ++b) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPF8; ++i) {
      const int c = tid + 256 * i;
      if (NCH8 % 256 == 0 || c < NCH8) {
        const int row = c / (KP / 16), c16 = c - row * (KP / 16);
        u2v* dst = reinterpret_cast<u2v*>(&sD[row * DS + 16 * c16]);
        dst[0] = u2v{pd[i][0], pd[i][1]};
        dst[1] = u2v{pd[i][2], pd[i][3]};
      }
    }
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int c = tid + 256 * i;
      if (NCH % 256 == 0 || c < NCH) {
        const int l = c >> 2, part = c & 3;
        u2v* dst = reinterpret_cast<u2v*>(&sT[l * TS + part * 8]);
        dst[0] = u2v{pt[i][0], pt[i][1]};
        dst[1] = u2v{pt[i][2], pt[i][3]};
      }
    }
    if (tid < BMP) sG[tid] = gpre;
    __syncthreads();
    {
      const int bn = (b + 1 < b_end) ? b + 1 : b;
      GMCO_PF8(bn);
    }

    f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
    for (int k = 0; k < NK32; ++k) {
      const long a0 = *reinterpret_cast<const long*>(&sD[n * DS + 32 * k + 8 * q]);
      const long a1 = *reinterpret_cast<const long*>(&sD[(16 + n) * DS + 32 * k + 8 * q]);
      acc0 = mfma_fp8(a0, tb[k], acc0);
      acc1 = mfma_fp8(a1, tb[k], acc1);
    }
    bf8v phi;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float d = u * (e < 4 ? acc0[e] : acc1[e - 4]);
      const int pt_ = e < 4 ? 4 * q + e : 16 + 4 * q + (e - 4);
      const int gi = sG[pt_];
      const float4 pr = sP[gi];
      const float w = (gi < kGmax) ? sW[(wave * 16 + n) * kGmax + gi] : 0.f;
      float kap = 0.f, dev = 0.f;
      if (d < pr.y) {
        dev = d - pr.y;
        kap = pr.x * dev;
      } else if (d > pr.z) {
        dev = d - pr.z;
        kap = pr.w * dev;
      }
      facc += (double)(w * (kap * dev));
      phi[e] = (__bf16)(w * kap);
    }
#pragma unroll
    for (int k = 0; k < NK16; ++k) {
      const bf4v lo = *reinterpret_cast<const bf4v*>(&sT[(16 * k + n) * TS + 4 * q]);
      const bf4v hi = *reinterpret_cast<const bf4v*>(&sT[(16 * k + n) * TS + 16 + 4 * q]);
      const bf8v av = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      gacc[k] = mfma_bf16(av, phi, gacc[k]);
    }
  }
#undef GMCO_PF8

  float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP;
#pragma unroll
  for (int k = 0; k < NK16; ++k) {
    *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) =
        make_float4(gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]);
  }
  facc += __shfl_xor(facc, 16);
  facc += __shfl_xor(facc, 32);
  if (q == 0) a.Fpart[(size_t)s * stride + j0 + col] = facc;
}

template <int KP>
hipError_t launch_kp(const EvalArgs& a, int dtype, hipStream_t st) {
  if (a.grid < 1) return hipErrorInvalidValue;
  const dim3 grid(a.grid), block(256);
  if (dtype == GMCO_DTYPE_F32_ACC64)
    hipLaunchKernelGGL((k_eval_acc64<KP>), grid, dim3(512), 0, st, a);
  else if (dtype == GMCO_DTYPE_F32_CHUNK64)
    hipLaunchKernelGGL((k_eval_f32<KP, MODE_CHUNK64>), grid, block, 0, st, a);
  else if (dtype == GMCO_DTYPE_F32)
    hipLaunchKernelGGL((k_eval_f32<KP, MODE_F32>), grid, block, 0, st, a);
  else if (dtype == GMCO_DTYPE_BF16)
    hipLaunchKernelGGL((k_eval_bf16<KP>), grid, block, 0, st, a);
  else if (dtype == GMCO_DTYPE_FP8)
    hipLaunchKernelGGL((k_eval_fp8<KP>), grid, block, 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const EvalArgs& a, int dtype, hipStream_t st) {
  switch (a.Kp) {
#define GMCO_KP_CASE(v) \
  case v:               \
    return launch_kp<v>(a, dtype, st);
    GMCO_KP_CASE(32)
    GMCO_KP_CASE(64)
    GMCO_KP_CASE(96)
    GMCO_KP_CASE(128)
    GMCO_KP_CASE(160)
    GMCO_KP_CASE(192)
    GMCO_KP_CASE(224)
    GMCO_KP_CASE(256)
    GMCO_KP_CASE(288)
    GMCO_KP_CASE(320)
    GMCO_KP_CASE(352)
    GMCO_KP_CASE(384)
    GMCO_KP_CASE(416)
    GMCO_KP_CASE(448)
    GMCO_KP_CASE(480)
    GMCO_KP_CASE(512)
#undef GMCO_KP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace gmco
