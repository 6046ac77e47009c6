// Fused batched evaluation of the gMCO objective and its gradient.
//
// For one or two tiles of 64 plans and a range of dose points, one workgroup
// computes
//   d   = D t                      eq. (dose), t = x^2 (Sec. 2.1.2)
//   f   = eq. 1 per point, F += (w_j / N_j) f             eq. (obj)
//   phi = (w_j / N_j) kappa(d)     kappa = the bracket of eq. 2
//   G  += D^T phi                  back-projection over the points
// and writes G and F as split-M partials; the gradient in x is 4 x * sum G
// (eq. 2).  The dose tile never leaves the chip: each block of D (16 points
// for FP32 operands, 32 for BF16 / FP8) is staged once in LDS and feeds both
// products, and the dwell times and gradient accumulators of each wave's
// plans stay in registers for the whole point range.  Each operand type has
// a role-split workgroup shape besides its default one: some waves run the
// dose product with eq. 1 of block b, the others back-project block b - 1
// and stage the tiles, so that one's epilogue and staging overlap the
// other's matrix ops (the default for FP32 and BF16 operands).
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

// True (the same in every lane) when any lane holds a nonzero penalty
// derivative: the back-projection of a block whose phi is zero for every
// point and plan of the wave adds only zero products, so it is skipped.
__device__ inline bool wave_any_nonzero(const float (&phi)[4]) {
  const bool nz = phi[0] != 0.f || phi[1] != 0.f || phi[2] != 0.f || phi[3] != 0.f;
  return __builtin_amdgcn_ballot_w64(nz) != 0;
}

// FP64 matrix op on FP32 operands: the products are exact in FP64 and the
// dose accumulates without FP32 rounding (same lane layout as the FP32 op).
__device__ inline d4v mfma_f64(float a, float b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, (double)b, c, 0, 0, 0);
}

// Maps the flat workgroup id to (split, tile).  Workgroups are dispatched to
// the 8 XCDs round-robin; with xcd_map, when the grid allows it, all tiles of
// one point range land on the same XCD so that its L2 serves that slice of D
// to all of them.
__device__ inline void split_tile(int bid, int S, int ntiles, int xcd_map, int& s, int& tile) {
  const int total = S * ntiles;
  if (xcd_map && (S & 7) == 0 && (total & 7) == 0) {
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
// the partial buffers), workgroup bid's (split, first compact column j0) and
// the plan behind each of its TPW * kPT columns (-1: empty), and stages the
// columns' structure weights.  In a compacted round every workgroup ranks
// the running plans itself (a block-wide scan of the flags), so no separate
// launch is needed.  Returns false, for the whole workgroup, when the grid
// is larger than this round's S * (units of NCOL columns).  A workgroup
// covers NCOL consecutive columns: TPW whole plan tiles (NCOL = TPW kPT) or
// half a tile (NCOL = kPT / 2).  Columns at or past `stride` (the second tile
// of the last workgroup when ntiles is odd) are empty and have no partials.
template <int NT, int NCOL = kPT>
__device__ inline bool tile_setup(const EvalArgs& a, int bid, int* sPlan, int* sScan, float* sW, int& s,
                                  int& S, int& stride, int& j0) {
  static_assert(NCOL % 16 == 0 && (NCOL % kPT == 0 || kPT % NCOL == 0), "whole 16-plan groups");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int unit;
  if (a.flag == nullptr) {
    S = a.S;
    stride = a.Pp;
    const int units = (a.ntiles * kPT + NCOL - 1) / NCOL;
    if (bid >= S * units) return false;
    split_tile(bid, S, units, a.xcd_map, s, unit);
    j0 = unit * NCOL;
    for (int i = tid; i < NCOL; i += NT) sPlan[i] = j0 + i < a.Pp ? j0 + i : -1;
  } else {
    for (int i = tid; i < NCOL; i += NT) sPlan[i] = -1;
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
    if (bid == 0 && tid == 0) {
      RoundTable r;
      r.nact = nact;
      r.ntiles = ntiles;
      r.S = S;
      r.pad = 0;
      *a.rt = r;
      if (a.work != nullptr) *a.work += (unsigned long long)nact;
      if (a.work2 != nullptr) *a.work2 += (unsigned long long)nact;
    }
    const int units = (ntiles * kPT + NCOL - 1) / NCOL;
    if (bid >= S * units) return false;
    split_tile(bid, S, units, a.xcd_map, s, unit);
    j0 = unit * NCOL;
    int r = base + v - cnt;
    for (int p = b; p < e; ++p) {
      if (a.flag[p]) {
        if (r >= j0 && r < j0 + NCOL) {
          sPlan[r - j0] = p;
          if (s == 0) a.slot[p] = r;
        }
        ++r;
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < NCOL * kGmax; i += NT) {
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
__device__ inline void eval_f32(const EvalArgs& a, int bid) {
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
  if (!tile_setup<256>(a, bid, sPlan, sScan, sW, s, S, stride, j0)) return;
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
    _Pragma("unroll") for (int i_ = 0; i_ < NPF; ++i_) {                    \
      const int idx = tid + 256 * i_;                                       \
      if (NF4 % 256 == 0 || idx < NF4) pf[i_] = src_[idx];                  \
    }                                                                       \
    if (tid < kBM) gpre = a.grp[(blk) * kBM + tid];                         \
  }
#define GMCO_STAGE(buf)                                                     \
  {                                                                         \
    const int buf_ = (buf);                                                 \
    _Pragma("unroll") for (int i_ = 0; i_ < NPF; ++i_) {                    \
      const int idx = tid + 256 * i_;                                       \
      if (NF4 % 256 == 0 || idx < NF4) {                                    \
        const int row = idx / (KP / 4);                                     \
        const int c4 = idx - row * (KP / 4);                                \
        *reinterpret_cast<f4v*>(&sD[buf_][row * KS + 4 * c4]) = pf[i_];     \
      }                                                                     \
    }                                                                       \
    if (tid < kBM) sG[buf_][tid] = gpre;                                    \
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
        if (k == NK16 - 1 && !a.last16) continue;  // all-padding slice: zero products
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
      // (Skipping the back-projection of a block whose phi is zero, as the
      // FP64-accumulating kernel does, measured slower here: with one wave
      // per SIMD the back-projection's independent ops fill the gaps of the
      // two dose chains, and the split loop loses that.)
#pragma unroll
      for (int k = 0; k < NK16; ++k) {
        if (k == NK16 - 1 && !a.last16) continue;  // all-padding slice: zero products
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

// Workgroup shape 3 of the FP32 kernel: the 64-plan tile as four groups of
// 16 plans in two roles of four wavefronts (512 threads, two waves per
// SIMD).  Waves 0-3 run the dose product of block b over all dwells and eq. 1
// and pass phi through LDS; waves 4-7 back-project block b - 1 onto all
// dwells (skipped when phi is zero for the group's 16 points and plans) and
// stage the D tiles.  The two products take the same matrix time, so each
// SIMD alternates between equal loads, and the epilogue and staging of one
// wave overlap the matrix ops of the other.  Three D buffers, one barrier
// per block; per column the arithmetic and its order are those of shape 0,
// so the results are bitwise the same.
template <int KP>
__device__ inline void eval_f32_ws(const EvalArgs& a, int bid) {
  constexpr int NG = 4;
  constexpr int NT = 512;
  constexpr int NTS = 256;             // threads per role
  constexpr int KS = KP + 4;           // LDS row stride (as shape 0)
  constexpr int NK16 = KP / 16;
  constexpr int NF4 = 4 * KP;          // float4 per 16-point block
  constexpr int NPF = (NF4 + NTS - 1) / NTS;

  __shared__ __attribute__((aligned(16))) float sD[3][kBM * KS];
  __shared__ float sPhi[2][NG][4][64];  // phi of a block [buffer][group][r][lane]
  __shared__ float sW[kPT * kGmax];
  __shared__ int sPlan[kPT];
  __shared__ int sScan[NT / 64];
  __shared__ float4 sP[kGmax + 1];
  __shared__ int sG[3][kBM];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wavefront
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;
  const int grp = wave & 3;
  const int nk_used = a.last16 ? NK16 : NK16 - 1;  // the all-padding slice adds zero products

  int s, S, stride, j0;
  if (!tile_setup<NT, kPT>(a, bid, sPlan, sScan, sW, s, S, stride, j0)) return;
#pragma unroll
  for (int j = 0; j <= kGmax; ++j)
    if (tid == j) sP[j] = a.gt.prm[j];
  const int col = grp * 16 + n;
  const int b_begin = (int)(((long long)s * a.nblocks) / S);
  const int b_end = (int)(((long long)(s + 1) * a.nblocks) / S);
  const int nblk = b_end - b_begin;

  // Steps i = 0 .. nblk as in the role-split FP64-accumulated kernel: the
  // dose role evaluates block b_begin + i from buffer i % 3, the
  // back-projection role block b_begin + i - 1 from buffer (i - 1) % 3 and
  // stages block b_begin + i + 1 into buffer (i + 1) % 3.
  if (wave < NG) {
    const int plan = sPlan[col];
    const bool pv = plan >= 0;  // an empty column evaluates t = 0 with zero weights
    const float* __restrict__ xrow = a.x + (size_t)(pv ? plan : 0) * KP;
    float tf[KP / 4];
#pragma unroll
    for (int k = 0; k < NK16; ++k) {
      const float4 xv = *reinterpret_cast<const float4*>(xrow + 16 * k + 4 * q);
      tf[4 * k + 0] = pv ? xv.x * xv.x : 0.f;
      tf[4 * k + 1] = pv ? xv.y * xv.y : 0.f;
      tf[4 * k + 2] = pv ? xv.z * xv.z : 0.f;
      tf[4 * k + 3] = pv ? xv.w * xv.w : 0.f;
    }
    double facc = 0.0;
    __syncthreads();
    for (int i = 0; i <= nblk; ++i) {
      if (i < nblk) {
        const int cur = i % 3;
        const float* __restrict__ Dc = sD[cur];
        f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
        for (int k = 0; k < NK16; ++k) {
          if (k == NK16 - 1 && nk_used < NK16) continue;
          const float4 av = *reinterpret_cast<const float4*>(&Dc[n * KS + 16 * k + 4 * q]);
          acc0 = mfma_f32(av.x, tf[4 * k + 0], acc0);
          acc1 = mfma_f32(av.y, tf[4 * k + 1], acc1);
          acc0 = mfma_f32(av.z, tf[4 * k + 2], acc0);
          acc1 = mfma_f32(av.w, tf[4 * k + 3], acc1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float d = acc0[r] + acc1[r];
          const int gi = sG[cur][4 * q + r];
          const float4 pr = sP[gi];
          const float w = (gi < kGmax) ? sW[col * kGmax + gi] : 0.f;
          const float lo = fminf(d - pr.y, 0.f);
          const float hi = fmaxf(d - pr.z, 0.f);
          const float kap = pr.x * lo + pr.w * hi;
          facc += (double)(w * (kap * (lo + hi)));
          sPhi[i & 1][grp][r][lane] = w * kap;
        }
      }
      __syncthreads();
    }
    facc += __shfl_xor(facc, 16);
    facc += __shfl_xor(facc, 32);
    if (q == 0) a.Fpart[(size_t)s * stride + j0 + col] = facc;
  } else {
    const int st = tid - NTS;
    const f4v* __restrict__ Dg = reinterpret_cast<const f4v*>(a.D);
    f4v pf[NPF];
    int gpre = 0;
    // threads past the last chunk load the last one again and do not store it
    auto prefetch = [&](int blk) {
      const f4v* src = Dg + (size_t)blk * NF4;
#pragma unroll
      for (int i = 0; i < NPF; ++i) pf[i] = src[min(st + NTS * i, NF4 - 1)];
      if (st < kBM) gpre = a.grp[blk * kBM + st];
    };
    auto stage = [&](int buf) {
#pragma unroll
      for (int i = 0; i < NPF; ++i) {
        const int idx = st + NTS * i;
        if (NF4 % NTS == 0 || idx < NF4) {
          const int row = idx / (KP / 4);
          const int c4 = idx - row * (KP / 4);
          *reinterpret_cast<f4v*>(&sD[buf][row * KS + 4 * c4]) = pf[i];
        }
      }
      if (st < kBM) sG[buf][st] = gpre;
    };
    f4v gacc[NK16];
#pragma unroll
    for (int k = 0; k < NK16; ++k) gacc[k] = f4v{0.f, 0.f, 0.f, 0.f};
    if (nblk > 0) {
      prefetch(b_begin);
      stage(0);
      if (nblk > 1) prefetch(b_begin + 1);
    }
    __syncthreads();
    for (int i = 0; i <= nblk; ++i) {
      if (i > 0) {
        const float* __restrict__ Dp = sD[(i - 1) % 3];
        float phi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) phi[r] = sPhi[(i - 1) & 1][grp][r][lane];
        if (wave_any_nonzero(phi)) {
#pragma unroll
          for (int k = 0; k < NK16; ++k) {
            if (k == NK16 - 1 && nk_used < NK16) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) gacc[k] = mfma_f32(Dp[(4 * q + r) * KS + 16 * k + n], phi[r], gacc[k]);
          }
        }
      }
      if (i + 1 < nblk) {
        stage((i + 1) % 3);
        if (i + 2 < nblk) prefetch(b_begin + i + 2);
      }
      __syncthreads();
    }
    float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP;
#pragma unroll
    for (int k = 0; k < NK16; ++k)
      *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) = make_float4(gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]);
  }
}

// ---------------------------------------------------------------------------
// MODE_ACC64 (FP32 operands, FP64-accumulated dose, FP64 penalty, FP32
// back-projection), by default with 512 threads: two waves per SIMD.  The
// FP64 matrix op reaches its full rate only when two waves per SIMD issue it,
// and a wave that holds t and the gradient accumulators of 16 plans over all
// Kp dwells does not fit in half the register file.  So the 8 waves form 4
// plan groups (16 plans each) x 2 dwell halves: each wave forms the partial
// dose of its dwell half, the partials of a plan group are added through LDS
// in a fixed order, the waves of the group evaluate eq. 1 on the sum (two of
// the four rows each) and each back-projects onto its own dwell half.  Per
// block: the dose product of block b, then the back-projection of block b-1
// (skipped by a wave whose phi is zero for all its points and plans), on two
// LDS buffers, with two barriers per block.
// LDS tile row stride Kp + 16 with the float4 chunk index of row R XORed with
// (R >> 1) & 3: the back-projection reads 16 columns of rows q + 4r (the FP64
// op's row order), which that stride puts on opposite bank halves for
// q = 0, 1, and the swizzle keeps the dose product's float4 reads of rows
// 0..15 conflict-free.
// ---------------------------------------------------------------------------
// NG plan groups of 16 per workgroup and NH dwell parts per group:
//   NG = 4, NH = 2: 512 threads, one workgroup of 64 plans per CU;
//   NG = 2, NH = 2: 256 threads, 32 plans (half a tile), two workgroups per
//                   CU whose barriers and eq. 1 phases are independent;
//   NG = 4, NH = 4: 1,024 threads, 64 plans, four waves per SIMD (dwell
//                   quarters, Kp a multiple of 64): a wave holds a quarter of
//                   the registers, and while some waves wait (LDS, barrier,
//                   epilogue) the others keep the FP64 matrix pipe fed.
// Per plan the arithmetic and its order are the same for a given NH; the
// NH = 4 shape adds the dose partials of four quarters instead of two
// halves (an FP64 rounding difference).
template <int KP, int NG, int NH = 2>
__device__ inline void eval_acc64(const EvalArgs& a, int bid) {
  static_assert((NH == 2 || NH == 4) && KP % (16 * NH) == 0, "dwell parts of whole 16-dwell slices");
  constexpr int NT = 64 * NG * NH;
  constexpr int NCOL = 16 * NG;
  constexpr int KS = KP + 16;
  constexpr int NKH = KP / (16 * NH);  // 16-dwell slices per dwell part
  constexpr int RPW = 4 / NH;          // epilogue rows per wave
  constexpr int NF4 = 4 * KP;          // float4 per 16-point block
  constexpr int NPF = (NF4 + NT - 1) / NT;

  __shared__ __attribute__((aligned(16))) float sD[2][kBM * KS];
  __shared__ double sX[NH][NG][4][64];  // partial doses [part][group][r][lane]
  __shared__ float sPhi[NG][4][64];      // phi of the last block [group][r][lane]
  __shared__ double sF[NH - 1][NG][64];  // F partials of the waves of parts 1.. [part-1][group][lane]
  __shared__ float sW[NCOL * kGmax];
  __shared__ int sPlan[NCOL];
  __shared__ int sScan[NT / 64];
  __shared__ double sP64[kGmax + 1][4];
  __shared__ int sG[2][kBM];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;
  const int grp = wave % NG;   // plan group: columns 16 grp .. 16 grp + 15
  const int half = wave / NG;  // dwell part: slices half * NKH .. half * NKH + NKH - 1
  // the last slice of the last part holds only padding dwells when
  // Kp - K >= 16: its products are zero, so the wave skips it (a scalar branch)
  const bool skip_last = __builtin_amdgcn_readfirstlane(half) == NH - 1 && !a.last16;

  int s, S, stride, j0;
  if (!tile_setup<NT, NCOL>(a, bid, sPlan, sScan, sW, s, S, stride, j0)) return;
#pragma unroll
  for (int j = 0; j <= kGmax; ++j)
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sP64[j][c] = a.gt.prm64[j][c];
    }

  const int col = grp * 16 + n;
  const int plan = sPlan[col];
  const bool pv = plan >= 0;  // an empty column evaluates t = 0 with zero weights
  const float* __restrict__ xrow = a.x + (size_t)(pv ? plan : 0) * KP + half * (KP / NH);
  // t = x^2 of plan n at dwells 16 k + 4 q + j of this wave's half (slice k)
  float tf[4 * NKH];
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
    _Pragma("unroll") for (int i_ = 0; i_ < NPF; ++i_) {                    \
      const int idx = tid + NT * i_;                                        \
      if (NF4 % NT == 0 || idx < NF4) pf[i_] = src_[idx];                   \
    }                                                                       \
    if (tid < kBM) gpre = a.grp[(blk) * kBM + tid];                         \
  }
#define GMCO_ST64(buf)                                                      \
  {                                                                         \
    const int buf_ = (buf);                                                 \
    _Pragma("unroll") for (int i_ = 0; i_ < NPF; ++i_) {                    \
      const int idx = tid + NT * i_;                                        \
      if (NF4 % NT == 0 || idx < NF4) {                                     \
        const int row = idx / (KP / 4);                                     \
        const int c4 = idx - row * (KP / 4);                                \
        *reinterpret_cast<f4v*>(&sD[buf_][row * KS + 4 * (c4 ^ swz_row(row))]) = pf[i_]; \
      }                                                                     \
    }                                                                       \
    if (tid < kBM) sG[buf_][tid] = gpre;                                    \
  }

  for (int i = tid; i < kBM * KS; i += NT) sD[1][i] = 0.f;
  for (int i = tid; i < NG * 4 * 64; i += NT) (&sPhi[0][0][0])[i] = 0.f;
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
    if constexpr (NH == 4) {
      // t stays FP32 in registers (a quarter-wave has 128 of them): mark it
      // as changed each block so that its FP64 conversion is redone per use
      // rather than kept live for the whole loop
#pragma unroll
      for (int i = 0; i < 4 * NKH; ++i) asm("" : "+v"(tf[i]));
    }
    // the dose product of block b, then the back-projection of block b-1,
    // skipped when phi is zero for all 16 points and 16 plans of the wave
#pragma unroll
    for (int k = 0; k < NKH; ++k) {
      if (k == NKH - 1 && skip_last) continue;
      const int kg = half * NKH + k;
      const float4 av = *reinterpret_cast<const float4*>(&Dc[n * KS + 16 * kg + 4 * (q ^ swz_row(n))]);
      if constexpr (NH == 4) {
        // two accumulator chains (four waves per SIMD interleave them)
        acc0 = mfma_f64(av.x, tf[4 * k + 0], acc0);
        acc1 = mfma_f64(av.y, tf[4 * k + 1], acc1);
        acc0 = mfma_f64(av.z, tf[4 * k + 2], acc0);
        acc1 = mfma_f64(av.w, tf[4 * k + 3], acc1);
      } else {
        acc0 = mfma_f64(av.x, tf[4 * k + 0], acc0);
        acc1 = mfma_f64(av.y, tf[4 * k + 1], acc1);
        acc2 = mfma_f64(av.z, tf[4 * k + 2], acc2);
        acc3 = mfma_f64(av.w, tf[4 * k + 3], acc3);
      }
    }
    if (wave_any_nonzero(phi_prev)) {
#pragma unroll
      for (int k = 0; k < NKH; ++k) {
        if (k == NKH - 1 && skip_last) continue;
        const int kg = half * NKH + k;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          gacc[k] = mfma_f32(Dp[(q + 4 * r) * KS + 16 * kg + (n ^ (swz_row(q + 4 * r) << 2))],
                             phi_prev[r], gacc[k]);
      }
    }
    // partial dose of points q + 4 r (the FP64 op's rows) for plan n
#pragma unroll
    for (int r = 0; r < 4; ++r) sX[half][grp][r][lane] = (acc0[r] + acc1[r]) + (acc2[r] + acc3[r]);
    __syncthreads();
    // eq. 1 on the summed dose: each wave of the group takes 4 / NH of the
    // four rows (points q + 4r) and shares phi through LDS; the next
    // iteration's first barrier orders these writes before their reads
    if (have_cur) {
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) {
        const int r = RPW * half + rr;
        double d = sX[0][grp][r][lane] + sX[1][grp][r][lane];
#pragma unroll
        for (int h = 2; h < NH; ++h) d += sX[h][grp][r][lane];
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

  // ---- split partials: each wave its dwell part; F from one wave per group ----
  float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP + half * (KP / NH);
#pragma unroll
  for (int k = 0; k < NKH; ++k) {
    *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) =
        make_float4(gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]);
  }
  // F partial: the rows of part 0, then those of parts 1.. in order, then over q
  if (half > 0) sF[half - 1][grp][lane] = facc;
  __syncthreads();
  if (half == 0) {
#pragma unroll
    for (int h = 1; h < NH; ++h) facc += sF[h - 1][grp][lane];
    facc += __shfl_xor(facc, 16);
    facc += __shfl_xor(facc, 32);
    if (q == 0) a.Fpart[(size_t)s * stride + j0 + col] = facc;
  }
}

// Workgroup shape 3: the plan tile of shape 0 (four groups of 16 plans, 512
// threads) with two roles of four wavefronts instead of dwell halves.  Waves
// 0-3 run the FP64 dose product of block b over all dwells and eq. 1 for
// their group and pass phi through LDS; waves 4-7 back-project block b - 1
// onto all dwells and stage the D tiles.  One wave of each role shares a
// SIMD, so the conversions, epilogue and staging of one overlap the matrix
// ops of the other, and no partial dose crosses waves.  Three D buffers and
// one barrier per block.  The dose keeps shape 0's accumulator chains (four
// per dwell half, the halves added last) and the objective its row order,
// so the results are bitwise those of shape 0.
template <int KP>
__device__ inline void eval_acc64_ws(const EvalArgs& a, int bid) {
  constexpr int NG = 4;
  constexpr int NT = 512;
  constexpr int NTS = 256;             // threads per role
  constexpr int NCOL = 16 * NG;
  constexpr int KS = KP + 16;
  constexpr int NK = KP / 16;          // 16-dwell slices
  constexpr int NKH = NK / 2;          // slices of a dwell half
  static_assert(KP % 32 == 0, "two dwell halves of whole slices");
  constexpr int NF4 = 4 * KP;          // float4 per 16-point block
  constexpr int NPF = (NF4 + NTS - 1) / NTS;

  __shared__ __attribute__((aligned(16))) float sD[3][kBM * KS];
  __shared__ float sPhi[2][NG][4][64];  // phi of a block [buffer][group][r][lane]
  __shared__ float sW[NCOL * kGmax];
  __shared__ int sPlan[NCOL];
  __shared__ int sScan[NT / 64];
  __shared__ double sP64[kGmax + 1][4];
  __shared__ int sG[3][kBM];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wavefront
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;
  const int grp = wave & 3;  // plan group: columns 16 grp .. 16 grp + 15
  // the last slice holds only padding dwells when Kp - K >= 16: its products
  // are zero, so both roles skip it
  const int nk_used = a.last16 ? NK : NK - 1;

  int s, S, stride, j0;
  if (!tile_setup<NT, NCOL>(a, bid, sPlan, sScan, sW, s, S, stride, j0)) return;
#pragma unroll
  for (int j = 0; j <= kGmax; ++j)
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sP64[j][c] = a.gt.prm64[j][c];
    }
  const int col = grp * 16 + n;
  const int b_begin = (int)(((long long)s * a.nblocks) / S);
  const int b_end = (int)(((long long)(s + 1) * a.nblocks) / S);
  const int nblk = b_end - b_begin;

  // Both roles pass nblk + 2 barriers: one after the first tile is staged,
  // then one per step i = 0 .. nblk, in which the dose role evaluates block
  // b_begin + i (i < nblk, from buffer i % 3) and the back-projection role
  // block b_begin + i - 1 (i > 0, buffer (i - 1) % 3) and stages block
  // b_begin + i + 1 into buffer (i + 1) % 3, last read in step i - 1; phi of
  // block b_begin + i goes to sPhi[i & 1].
  if (wave < NG) {
    const int plan = sPlan[col];
    const bool pv = plan >= 0;  // an empty column evaluates t = 0 with zero weights
    const float* __restrict__ xrow = a.x + (size_t)(pv ? plan : 0) * KP;
    // t = x^2 of plan n at dwells 16 k + 4 q + j (slice k)
    float tf[4 * NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const float4 xv = *reinterpret_cast<const float4*>(xrow + 16 * k + 4 * q);
      tf[4 * k + 0] = pv ? xv.x * xv.x : 0.f;
      tf[4 * k + 1] = pv ? xv.y * xv.y : 0.f;
      tf[4 * k + 2] = pv ? xv.z * xv.z : 0.f;
      tf[4 * k + 3] = pv ? xv.w * xv.w : 0.f;
    }
    double facc0 = 0.0, facc1 = 0.0;  // rows 0-1 and 2-3, as the two waves of shape 0
    __syncthreads();
    for (int i = 0; i <= nblk; ++i) {
      if (i < nblk) {
        const int cur = i % 3;
        const float* __restrict__ Dc = sD[cur];
        // t stays FP32 in registers: mark it as changed each block so that
        // its FP64 conversion is redone per use rather than kept live (in
        // FP64 it would take 192 registers)
#pragma unroll
        for (int j = 0; j < 4 * NK; ++j) asm("" : "+v"(tf[j]));
        d4v acc[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[h][c] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          if (k == NK - 1 && nk_used < NK) continue;
          const int h = k / NKH;
          const float4 av = *reinterpret_cast<const float4*>(&Dc[n * KS + 16 * k + 4 * (q ^ swz_row(n))]);
          acc[h][0] = mfma_f64(av.x, tf[4 * k + 0], acc[h][0]);
          acc[h][1] = mfma_f64(av.y, tf[4 * k + 1], acc[h][1]);
          acc[h][2] = mfma_f64(av.z, tf[4 * k + 2], acc[h][2]);
          acc[h][3] = mfma_f64(av.w, tf[4 * k + 3], acc[h][3]);
        }
        // eq. 1 on the dose of points q + 4 r for plan n
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double d = ((acc[0][0][r] + acc[0][1][r]) + (acc[0][2][r] + acc[0][3][r])) +
                           ((acc[1][0][r] + acc[1][1][r]) + (acc[1][2][r] + acc[1][3][r]));
          const int gi = sG[cur][q + 4 * r];
          const float w = (gi < kGmax) ? sW[col * kGmax + gi] : 0.f;
          const double lo = fmin(d - sP64[gi][1], 0.0);
          const double hi = fmax(d - sP64[gi][2], 0.0);
          const double kap = sP64[gi][0] * lo + sP64[gi][3] * hi;
          if (r < 2) facc0 += (double)w * (kap * (lo + hi));
          else facc1 += (double)w * (kap * (lo + hi));
          sPhi[i & 1][grp][r][lane] = (float)((double)w * kap);
        }
      }
      __syncthreads();
    }
    double facc = facc0 + facc1;
    facc += __shfl_xor(facc, 16);
    facc += __shfl_xor(facc, 32);
    if (q == 0) a.Fpart[(size_t)s * stride + j0 + col] = facc;
  } else {
    const int st = tid - NTS;
    const f4v* __restrict__ Dg = reinterpret_cast<const f4v*>(a.D);
    f4v pf[NPF];
    int gpre = 0;
    // threads past the last chunk load the last one again and do not store it
    auto prefetch = [&](int blk) {
      const f4v* src = Dg + (size_t)blk * NF4;
#pragma unroll
      for (int i = 0; i < NPF; ++i) pf[i] = src[min(st + NTS * i, NF4 - 1)];
      if (st < kBM) gpre = a.grp[blk * kBM + st];
    };
    auto stage = [&](int buf) {
#pragma unroll
      for (int i = 0; i < NPF; ++i) {
        const int idx = st + NTS * i;
        if (NF4 % NTS == 0 || idx < NF4) {
          const int row = idx / (KP / 4);
          const int c4 = idx - row * (KP / 4);
          *reinterpret_cast<f4v*>(&sD[buf][row * KS + 4 * (c4 ^ swz_row(row))]) = pf[i];
        }
      }
      if (st < kBM) sG[buf][st] = gpre;
    };
    f4v gacc[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) gacc[k] = f4v{0.f, 0.f, 0.f, 0.f};
    if (nblk > 0) {
      prefetch(b_begin);
      stage(0);
      if (nblk > 1) prefetch(b_begin + 1);
    }
    __syncthreads();
    for (int i = 0; i <= nblk; ++i) {
      if (i > 0) {
        const float* __restrict__ Dp = sD[(i - 1) % 3];
        float phi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) phi[r] = sPhi[(i - 1) & 1][grp][r][lane];
        // skipped when phi is zero for all 16 points and 16 plans of the group
        if (wave_any_nonzero(phi)) {
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            if (k == NK - 1 && nk_used < NK) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
              gacc[k] = mfma_f32(Dp[(q + 4 * r) * KS + 16 * k + (n ^ (swz_row(q + 4 * r) << 2))], phi[r],
                                 gacc[k]);
          }
        }
      }
      if (i + 1 < nblk) {
        stage((i + 1) % 3);
        if (i + 2 < nblk) prefetch(b_begin + i + 2);
      }
      __syncthreads();
    }
    float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP;
#pragma unroll
    for (int k = 0; k < NK; ++k)
      *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) = make_float4(gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]);
  }
}

// ---------------------------------------------------------------------------
// Low-precision operands, FP32 accumulation.
//   BF16: both products in v_mfma_f32_16x16x32_bf16.
//   FP8 : the dose product in e4m3 (v_mfma_f32_16x16x32_fp8_fp8): D is stored
//         as D_il / s_l with one scale per dwell column
//         (s_l = max_i D_il / 224), the dwell times enter as t_l s_l / u_p
//         with one scale per plan (u_p = max_l t_l s_l / 224), and
//         d = u_p * sum.  The back-projection runs in BF16 on the BF16
//         transposed copy of D.  Both conversions use the hardware's own FP8
//         encoding, so the format convention never enters the arithmetic.
// Lane l (q = l / 16, n = l % 16) supplies A[n][8q .. 8q+7] and
// B[8q .. 8q+7][n] (eight 2- or 1-byte elements); accumulator register r
// holds C[4q + r][n].
// A workgroup evaluates lp_tiles(Kp) plan tiles: 128 plans up to Kp = 448,
// where each wave holds the dwell times and gradient accumulators of 32
// plans as two 16-plan halves, so that every operand of D read from LDS
// feeds two matrix ops and every block of D staged in LDS serves 128 plans
// (64 plans, 16 per wave, above).  Blocks of 32 points: the dose
// product runs two 16-point row tiles, after which each lane holds the
// penalty derivative of points {4q..4q+3} and {16+4q..16+4q+3} of its plan,
// exactly the 8 contraction slots it supplies to the back-projection, whose
// A operand (D transposed) is read in that point order from a dwell-major
// tile.  Both kernels stage that tile from the BF16 transposed copy of D,
// which stores every 32-point block in this point order.  (Building it in
// the kernel from the row-major block with byte permutes, which reads D from
// memory once, measured 58.5-58.8 us per launch against 55.9-58.7 us.)
// ---------------------------------------------------------------------------
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

__device__ inline f4v mfma_bf16(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline f4v mfma_fp8(long a, long b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

__device__ inline unsigned pack_fp8x4(float a, float b, float c, float d) {
  int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, lo, true);
}

// Eq. 1 at dose d for the row pw = (w w_min, D_min, D_max, w w_max), the
// structure weight w = w_j / N_j folded into the slopes, without branches:
// with lo = min(d - D_min, 0) and hi = max(d - D_max, 0) (at most one is
// nonzero since D_min <= D_max) the weighted bracket of eq. 2 is
// phi = w (w_min lo + w_max hi) and the weighted penalty phi (lo + hi).  Adds
// the penalty to f (FP32, one block's points; the caller adds f to its FP64
// sum once per block) and returns phi in BF16.
__device__ inline __bf16 penalty_lp(float d, float4 pw, float& f) {
  const float lo = fminf(d - pw.y, 0.f);
  const float hi = fmaxf(d - pw.z, 0.f);
  const float phi = pw.x * lo + pw.w * hi;
  f = fmaf(phi, lo + hi, f);
  return (__bf16)phi;
}

template <bool FP8>
struct LpOp;
template <>
struct LpOp<false> {
  typedef bf8v type;
  static __device__ inline f4v mma(bf8v a, bf8v b, f4v c) { return mfma_bf16(a, b, c); }
};
template <>
struct LpOp<true> {
  typedef long type;
  static __device__ inline f4v mma(long a, long b, f4v c) { return mfma_fp8(a, b, c); }
};

// B operand of the dose product for one column of 16 plans: lane (q, n)
// holds t = x^2 of plan `plan` (-1: an empty column, t = 0) at dwells
// 32 k + 8 q + e.  FP8: the scaled times t_l s_l / u with the plan's scale u
// (the maximum over the plan's dwells / 224); BF16: u = 1.
template <int KP, bool FP8>
__device__ inline void lp_t_operand(const EvalArgs& a, int plan, int q, typename LpOp<FP8>::type (&tb)[KP / 32],
                                    float& u) {
  constexpr int NK32 = KP / 32;
  const bool pv = plan >= 0;
  const float* __restrict__ xrow = a.x + (size_t)(pv ? plan : 0) * KP;
  u = 1.f;
  if constexpr (!FP8) {
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
  } else {
    // scaled dwell times t_l s_l, their per-plan maximum, then FP8 fragments
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
    u = tmax > 0.f ? tmax / 224.f : 1.f;
    const float inv_u = 1.f / u;
#pragma unroll
    for (int k = 0; k < NK32; ++k) {
      const unsigned lo = pack_fp8x4(ts[k][0] * inv_u, ts[k][1] * inv_u, ts[k][2] * inv_u, ts[k][3] * inv_u);
      const unsigned hi = pack_fp8x4(ts[k][4] * inv_u, ts[k][5] * inv_u, ts[k][6] * inv_u, ts[k][7] * inv_u);
      tb[k] = (long)(((unsigned long)hi << 32) | lo);
    }
  }
}

// Eq. 1 epilogue of one 32-point block for NH columns of 16 plans
// (col0 + 16 h + n): from the dose accumulators (points 4 q + r and
// 16 + 4 q + r) to phi in the back-projection's operand order, adding each
// column's penalties to facc (one FP64 addition per block).
template <int NH, bool FP8>
__device__ inline void lp_epilogue(const f4v (&acc)[NH][2], const float (&u)[NH], const int* cG,
                                   const float4* sP, const float* sW, int col0, int lane, bf8v (&phi)[NH],
                                   double (&facc)[NH]) {
  constexpr int BMP = 32;
  const int q = lane >> 4, n = lane & 15;
  float fblk[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) fblk[h] = 0.f;
  // The points are stored grouped by structure, so most blocks hold a
  // single structure: then the eq. 1 row and the weight w_j / N_j are the
  // same for all points of the block and are read once.
  const int g0 = cG[0];
  if (__all(cG[lane & (BMP - 1)] == g0)) {
    const float4 pr = sP[g0];
    float4 pw[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const float w = g0 < kGmax ? sW[(col0 + 16 * h + n) * kGmax + g0] : 0.f;
      pw[h] = make_float4(w * pr.x, pr.y, pr.z, w * pr.w);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        float d = e < 4 ? acc[h][0][e] : acc[h][1][e - 4];
        if constexpr (FP8) d *= u[h];
        phi[h][e] = penalty_lp(d, pw[h], fblk[h]);
      }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gi = cG[e < 4 ? 4 * q + e : 16 + 4 * q + (e - 4)];
      const float4 pr = sP[gi];
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        float d = e < 4 ? acc[h][0][e] : acc[h][1][e - 4];
        if constexpr (FP8) d *= u[h];
        const float w = gi < kGmax ? sW[(col0 + 16 * h + n) * kGmax + gi] : 0.f;
        phi[h][e] = penalty_lp(d, make_float4(w * pr.x, pr.y, pr.z, w * pr.w), fblk[h]);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < NH; ++h) facc[h] += (double)fblk[h];
}

template <int KP, bool FP8, int SHAPE>
__device__ inline void eval_lp(const EvalArgs& a, int bid) {
  typedef typename LpOp<FP8>::type op_t;
  constexpr int BMP = 32;              // points per block
  // D tile row stride (BF16 elements or FP8 bytes), chosen by timing the
  // layouts (unpadded rows are 1.6-2.3x slower; KP + 8 for BF16 measured no
  // better than KP + 16)
  constexpr int DS = FP8 ? KP + 8 : KP + 16;
  // Transposed tile: dwell row l starts at trow(l) = l TS BF16 elements;
  // 80-byte rows keep every operand read one aligned 16-byte access.  (Rows
  // skewed by 64 bytes every 8 or 16 dwells, meant to separate the staging
  // writes' banks, measured more bank conflicts and 8 % longer launches.)
  constexpr int TS = BMP + 8;
  constexpr int TSZ = KP * TS;
  constexpr int NK32 = KP / 32;        // k-steps of the dose product
  constexpr int NK16 = KP / 16;        // 16-dwell tiles of the back-projection
  constexpr int NT = lp_threads(KP, SHAPE);  // threads
  constexpr int NW = NT / 64;
  constexpr int NH = lp_halves(KP, SHAPE);   // 16-plan column groups per wavefront
  constexpr int NCOL = NW * 16 * NH;
  constexpr int TPW = NCOL / kPT;
  static_assert(TPW == lp_tiles(KP) && TPW * kPT == NCOL, "workgroup of whole plan tiles");
  constexpr int NC8 = KP / 8;  // 16-byte chunks of a BF16 row
  // FP8 staging: 16-byte chunks of the FP8 tile and of the BF16 transposed tile
  constexpr int NCH8 = BMP * KP / 16;
  constexpr int NCH = BMP * KP / 8;
  constexpr int NPF8 = FP8 ? (NCH8 + NT - 1) / NT : 1;
  constexpr int NPF = (NCH + NT - 1) / NT;
  constexpr int SDB = BMP * DS * (FP8 ? 1 : 2);  // bytes of one D tile
  constexpr int NCHB = BMP * KP / 8;  // 16-byte chunks of the BF16 D tile
  constexpr int NPFB = FP8 ? 1 : (NCHB + NT - 1) / NT;

  // two buffers: block b is read from one while block b + 1 is staged in the other
  __shared__ __attribute__((aligned(16))) unsigned char sD[2][SDB];
  __shared__ __attribute__((aligned(16))) __bf16 sT[2][TSZ];
  auto trow = [](int l) { return l * TS; };
  __shared__ int sG[2][BMP];
  __shared__ float sW[NCOL * kGmax];
  __shared__ int sPlan[NCOL];
  __shared__ int sScan[NW];
  __shared__ float4 sP[kGmax + 1];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;
  if (tid == 0) {  // constant indices: the table is read straight from the kernel arguments
#pragma unroll
    for (int j = 0; j <= kGmax; ++j) sP[j] = a.gt.prm[j];
  }
  int s, S, stride, j0;  // (tile_setup ends with a barrier)
  if (!tile_setup<NT, NCOL>(a, bid, sPlan, sScan, sW, s, S, stride, j0)) return;

  // B operands of the dose product, t = x^2 at dwells 32 k + 8 q + e, for
  // the plans of columns 16 (NH wave + h) + n (an empty column evaluates t = 0
  // with zero weights)
  op_t tb[NH][NK32];
  float u[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) lp_t_operand<KP, FP8>(a, sPlan[16 * (NH * wave + h) + n], q, tb[h], u[h]);
  f4v gacc[NH][NK16];
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int k = 0; k < NK16; ++k) gacc[h][k] = f4v{0.f, 0.f, 0.f, 0.f};
  double facc[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) facc[h] = 0.0;

  const int nb = a.Mp / BMP;
  const int b_begin = (int)(((long long)s * nb) / S);
  const int b_end = (int)(((long long)(s + 1) * nb) / S);
  const u4v* __restrict__ Dg = reinterpret_cast<const u4v*>(a.D);
  const __bf16* __restrict__ DTg = reinterpret_cast<const __bf16*>(a.DT);

  u4v pd[NPF8], pb[NPFB];  // FP8 / BF16 D tile chunks
  u4v pt[NPF];             // transposed-tile chunks
  int gpre = 0;
  auto prefetch = [&](int blk) {
    // threads past the last chunk load the last one again (every register
    // is defined on every path) and do not store it
    if constexpr (FP8) {
      const u4v* srcd = Dg + (size_t)blk * NCH8;
#pragma unroll
      for (int i = 0; i < NPF8; ++i) pd[i] = srcd[min(tid + NT * i, NCH8 - 1)];
    } else {
      const u4v* srcd = Dg + (size_t)blk * NCHB;
#pragma unroll
      for (int i = 0; i < NPFB; ++i) pb[i] = srcd[min(tid + NT * i, NCHB - 1)];
    }
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int c = min(tid + NT * i, NCH - 1);
      const int l = c >> 2, part = c & 3;
      pt[i] = *reinterpret_cast<const u4v*>(DTg + (size_t)l * a.Mp + (size_t)blk * BMP + part * 8);
    }
    if (tid < BMP) gpre = a.grp[blk * BMP + tid];
  };
  // prefetched registers -> LDS buffer `buf`
  auto stage = [&](int buf) {
    if constexpr (!FP8) {
      __bf16* sD16 = reinterpret_cast<__bf16*>(sD[buf]);
#pragma unroll
      for (int i = 0; i < NPFB; ++i) {
        const int c = tid + NT * i;
        if (NCHB % NT == 0 || c < NCHB) {
          const int row = c / NC8, c8 = c - row * NC8;
          *reinterpret_cast<u4v*>(&sD16[row * DS + 8 * c8]) = pb[i];
        }
      }
    } else {
      // (FP8 rows of Kp + 8 bytes are 8-byte aligned)
#pragma unroll
      for (int i = 0; i < NPF8; ++i) {
        const int c = tid + NT * i;
        if (NCH8 % NT == 0 || c < NCH8) {
          const int row = c / (KP / 16), c16 = c - row * (KP / 16);
          u2v* dst = reinterpret_cast<u2v*>(&sD[buf][row * DS + 16 * c16]);
          dst[0] = u2v{pd[i][0], pd[i][1]};
          dst[1] = u2v{pd[i][2], pd[i][3]};
        }
      }
    }
    // the transposed tile: 80-byte rows, 16-byte aligned chunks
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int c = tid + NT * i;
      if (NCH % NT == 0 || c < NCH) {
        const int l = c >> 2, part = c & 3;
        *reinterpret_cast<u4v*>(&sT[buf][trow(l) + part * 8]) = pt[i];
      }
    }
    if (tid < BMP) sG[buf][tid] = gpre;
  };

  // Software pipeline with one barrier per block: block b is evaluated from
  // buffer (b - b_begin) & 1 while block b + 1, loaded into registers during
  // block b - 1, is staged into the other buffer and block b + 2 is loaded.
  // The barrier at the end of block b - 1 orders both the staging of block b
  // before its reads and the reads of block b - 1 before that buffer is
  // staged again.
  if (b_begin < b_end) {
    prefetch(b_begin);
    stage(0);
    if (b_begin + 1 < b_end) prefetch(b_begin + 1);
  }
  __syncthreads();
  for (int b = b_begin; b < b_end; ++b) {
    const int cur = (b - b_begin) & 1;
    const unsigned char* cD = sD[cur];
    const __bf16* cT = sT[cur];
    const int tbase = trow(n) + 8 * q;
    const int* cG = sG[cur];

    // ---- dose product for the two 16-point row tiles ----
    f4v acc[NH][2];
#pragma unroll
    for (int h = 0; h < NH; ++h) acc[h][0] = acc[h][1] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < NK32; ++k) {
      op_t a0, a1;
      if constexpr (!FP8) {
        const __bf16* sD16 = reinterpret_cast<const __bf16*>(cD);
        a0 = *reinterpret_cast<const bf8v*>(&sD16[n * DS + 32 * k + 8 * q]);
        a1 = *reinterpret_cast<const bf8v*>(&sD16[(16 + n) * DS + 32 * k + 8 * q]);
      } else {
        a0 = *reinterpret_cast<const long*>(&cD[n * DS + 32 * k + 8 * q]);
        a1 = *reinterpret_cast<const long*>(&cD[(16 + n) * DS + 32 * k + 8 * q]);
      }
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        acc[h][0] = LpOp<FP8>::mma(a0, tb[h][k], acc[h][0]);
        acc[h][1] = LpOp<FP8>::mma(a1, tb[h][k], acc[h][1]);
      }
    }
    // ---- penalty epilogue ----
    bf8v phi[NH];
    lp_epilogue<NH, FP8>(acc, u, cG, sP, sW, 16 * NH * wave, lane, phi, facc);
    // ---- back-projection over the 32 points ----
#pragma unroll
    for (int k = 0; k < NK16; ++k) {
      const bf8v av = *reinterpret_cast<const bf8v*>(&cT[tbase + k * 16 * TS]);
#pragma unroll
      for (int h = 0; h < NH; ++h) gacc[h][k] = mfma_bf16(av, phi[h], gacc[h][k]);
    }

    if (b + 1 < b_end) {
      stage(cur ^ 1);
      if (b + 2 < b_end) prefetch(b + 2);
    }
    __syncthreads();
  }

#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const int col = 16 * (NH * wave + h) + n;
    double f = facc[h];
    f += __shfl_xor(f, 16);
    f += __shfl_xor(f, 32);
    if (j0 + col - n < stride) {  // the same for the whole wavefront
      float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP;
#pragma unroll
      for (int k = 0; k < NK16; ++k) {
        *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) =
            make_float4(gacc[h][k][0], gacc[h][k][1], gacc[h][k][2], gacc[h][k][3]);
      }
      if (q == 0) a.Fpart[(size_t)s * stride + j0 + col] = f;
    }
  }
}

// Workgroup shape 2 (Kp <= 384): the same 128 plans as shape 0, as four
// column groups of 32 plans, with two roles of four wavefronts (one of each
// per SIMD).  Waves 0-3 run the dose product and the eq. 1 epilogue of block
// b for their group (each D operand read from LDS feeds two matrix ops), pass
// phi to the back-projection through LDS and stage the next tiles; waves 4-7
// back-project block b - 1 for the same group (each D^T operand read feeds
// two matrix ops).  So every SIMD holds one wavefront of each role, and the
// epilogue and staging of one overlap the matrix ops of the other.  Per column
// the arithmetic and its order are those of shape 0, so the results are
// bitwise the same.
template <int KP, bool FP8>
__device__ inline void eval_lp_ws(const EvalArgs& a, int bid) {
  typedef typename LpOp<FP8>::type op_t;
  constexpr int BMP = 32;                      // points per block
  constexpr int DS = FP8 ? KP + 8 : KP + 16;   // D tile row stride (as shape 0)
  constexpr int TS = BMP + 8;                  // transposed tile row stride
  constexpr int TSZ = KP * TS;
  constexpr int NK32 = KP / 32;
  constexpr int NK16 = KP / 16;
  constexpr int NT = 512, NW = 8, NG = 4;      // NG column groups of 32 plans
  constexpr int NTS = 256;                     // threads per role
  constexpr int NCOL = NG * 32;
  static_assert(KP <= 384 && NCOL == lp_tiles(KP) * kPT, "workgroup of whole plan tiles");
  constexpr int NC8 = KP / 8;                  // 16-byte chunks of a BF16 row
  constexpr int NCH = BMP * KP / 8;            // 16-byte chunks of a BF16 tile
  constexpr int NCH8 = BMP * KP / 16;          // 16-byte chunks of an FP8 tile
  constexpr int NCHD = FP8 ? NCH8 : NCH;
  constexpr int NPD = (NCHD + NTS - 1) / NTS;
  constexpr int NPT = (NCH + NTS - 1) / NTS;
  constexpr int SDB = BMP * DS * (FP8 ? 1 : 2);

  __shared__ __attribute__((aligned(16))) unsigned char sD[2][SDB];
  __shared__ __attribute__((aligned(16))) __bf16 sT[2][TSZ];
  __shared__ bf8v sPhi[2][NG][2][64];  // phi of a block, per group and 16-plan half
  __shared__ int sG[2][BMP];
  __shared__ float sW[NCOL * kGmax];
  __shared__ int sPlan[NCOL];
  __shared__ int sScan[NW];
  __shared__ float4 sP[kGmax + 1];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wavefront
  const int grp = wave & 3;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j <= kGmax; ++j) sP[j] = a.gt.prm[j];
  }
  int s, S, stride, j0;  // (tile_setup ends with a barrier)
  if (!tile_setup<NT, NCOL>(a, bid, sPlan, sScan, sW, s, S, stride, j0)) return;
  const int nb = a.Mp / BMP;
  const int b_begin = (int)(((long long)s * nb) / S);
  const int b_end = (int)(((long long)(s + 1) * nb) / S);
  const int nblk = b_end - b_begin;

  // Both roles pass nblk + 2 barriers: one after the first tiles are staged,
  // then one per step i = 0 .. nblk, in which the dose role evaluates block
  // b_begin + i (i < nblk) and the back-projection role block b_begin + i - 1
  // (i > 0).  In step i the dose role stages D of block b + 1 into D buffer
  // (i + 1) & 1 and the back-projection role D^T of block b into transposed
  // buffer i & 1, read in step i + 1; phi of block b goes to sPhi[i & 1].
  // Each buffer written in step i was last read in step i - 1.
  const u4v* __restrict__ Dg = reinterpret_cast<const u4v*>(a.D);
  const __bf16* __restrict__ DTg = reinterpret_cast<const __bf16*>(a.DT);
  if (wave < NG) {
    u4v pd[NPD];
    int gpre = 0;
    // threads past the last chunk load the last one again (every register is
    // defined on every path) and do not store it
    auto prefetch_d = [&](int blk) {
      const u4v* src = Dg + (size_t)blk * NCHD;
#pragma unroll
      for (int i = 0; i < NPD; ++i) pd[i] = src[min(tid + NTS * i, NCHD - 1)];
      if (tid < BMP) gpre = a.grp[blk * BMP + tid];
    };
    auto stage_d = [&](int buf) {
#pragma unroll
      for (int i = 0; i < NPD; ++i) {
        const int c = tid + NTS * i;
        if (NCHD % NTS == 0 || c < NCHD) {
          if constexpr (!FP8) {
            const int row = c / NC8, c8 = c - row * NC8;
            *reinterpret_cast<u4v*>(&reinterpret_cast<__bf16*>(sD[buf])[row * DS + 8 * c8]) = pd[i];
          } else {
            // (FP8 rows of Kp + 8 bytes are 8-byte aligned)
            const int row = c / (KP / 16), c16 = c - row * (KP / 16);
            u2v* dst = reinterpret_cast<u2v*>(&sD[buf][row * DS + 16 * c16]);
            dst[0] = u2v{pd[i][0], pd[i][1]};
            dst[1] = u2v{pd[i][2], pd[i][3]};
          }
        }
      }
      if (tid < BMP) sG[buf][tid] = gpre;
    };

    op_t tb[2][NK32];
    float u[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) lp_t_operand<KP, FP8>(a, sPlan[32 * grp + 16 * h + n], q, tb[h], u[h]);
    double facc[2] = {0.0, 0.0};
    if (nblk > 0) {
      prefetch_d(b_begin);
      stage_d(0);
      if (nblk > 1) prefetch_d(b_begin + 1);
    }
    __syncthreads();
    for (int i = 0; i <= nblk; ++i) {
      if (i < nblk) {
        const int cur = i & 1;
        const unsigned char* cD = sD[cur];
        f4v acc[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[h][0] = acc[h][1] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < NK32; ++k) {
          op_t a0, a1;
          if constexpr (!FP8) {
            const __bf16* sD16 = reinterpret_cast<const __bf16*>(cD);
            a0 = *reinterpret_cast<const bf8v*>(&sD16[n * DS + 32 * k + 8 * q]);
            a1 = *reinterpret_cast<const bf8v*>(&sD16[(16 + n) * DS + 32 * k + 8 * q]);
          } else {
            a0 = *reinterpret_cast<const long*>(&cD[n * DS + 32 * k + 8 * q]);
            a1 = *reinterpret_cast<const long*>(&cD[(16 + n) * DS + 32 * k + 8 * q]);
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            acc[h][0] = LpOp<FP8>::mma(a0, tb[h][k], acc[h][0]);
            acc[h][1] = LpOp<FP8>::mma(a1, tb[h][k], acc[h][1]);
          }
        }
        bf8v phi[2];
        lp_epilogue<2, FP8>(acc, u, sG[cur], sP, sW, 32 * grp, lane, phi, facc);
        sPhi[cur][grp][0][lane] = phi[0];
        sPhi[cur][grp][1][lane] = phi[1];
        if (i + 1 < nblk) {
          stage_d(cur ^ 1);
          if (i + 2 < nblk) prefetch_d(b_begin + i + 2);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = 32 * grp + 16 * h + n;
      double f = facc[h];
      f += __shfl_xor(f, 16);
      f += __shfl_xor(f, 32);
      if (j0 + col - n < stride && q == 0) a.Fpart[(size_t)s * stride + j0 + col] = f;
    }
  } else {
    const int st = tid - NTS;
    u4v pt[NPT];
    auto prefetch_t = [&](int blk) {
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int c = min(st + NTS * i, NCH - 1);
        const int l = c >> 2, part = c & 3;
        pt[i] = *reinterpret_cast<const u4v*>(DTg + (size_t)l * a.Mp + (size_t)blk * BMP + part * 8);
      }
    };
    auto stage_t = [&](int buf) {
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int c = st + NTS * i;
        if (NCH % NTS == 0 || c < NCH) {
          const int l = c >> 2, part = c & 3;
          *reinterpret_cast<u4v*>(&sT[buf][l * TS + part * 8]) = pt[i];
        }
      }
    };
    f4v gacc[2][NK16];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < NK16; ++k) gacc[h][k] = f4v{0.f, 0.f, 0.f, 0.f};
    if (nblk > 0) prefetch_t(b_begin);
    __syncthreads();
    for (int i = 0; i <= nblk; ++i) {
      if (i > 0) {
        const int prv = (i - 1) & 1;
        const bf8v phi0 = sPhi[prv][grp][0][lane];
        const bf8v phi1 = sPhi[prv][grp][1][lane];
        const __bf16* cT = sT[prv] + n * TS + 8 * q;
#pragma unroll
        for (int k = 0; k < NK16; ++k) {
          const bf8v av = *reinterpret_cast<const bf8v*>(&cT[k * 16 * TS]);
          gacc[0][k] = mfma_bf16(av, phi0, gacc[0][k]);
          gacc[1][k] = mfma_bf16(av, phi1, gacc[1][k]);
        }
      }
      if (i < nblk) {
        stage_t(i & 1);
        if (i + 1 < nblk) prefetch_t(b_begin + i + 1);
      }
      __syncthreads();
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = 32 * grp + 16 * h + n;
      if (j0 + col - n < stride) {  // the same for the whole wavefront
        float* __restrict__ gout = a.Gpart + ((size_t)s * stride + j0 + col) * KP;
#pragma unroll
        for (int k = 0; k < NK16; ++k)
          *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) =
              make_float4(gacc[h][k][0], gacc[h][k][1], gacc[h][k][2], gacc[h][k][3]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Kernels.  Each evaluation exists as a single-case kernel (workgroup id =
// blockIdx.x) and as a grouped kernel over several cases of one padded dwell
// count: grouped workgroup g belongs to the case c with start[c] <= g <
// start[c + 1] (each case's range begins at a multiple of 8, so the XCD
// placement of its tiles is as in a launch of its own) and runs as that
// case's workgroup g - start[c], with the case's arguments from args[c].
// ---------------------------------------------------------------------------
__device__ inline int group_case(const int* __restrict__ start, int n, int g) {
  int c = 0;
  while (c + 1 < n && start[c + 1] <= g) ++c;
  return c;
}

template <int KP, int MODE>
__global__ __launch_bounds__(256, 1) void k_eval_f32(EvalArgs a) {
  eval_f32<KP, MODE>(a, blockIdx.x);
}
template <int KP, int MODE>
__global__ __launch_bounds__(256, 1) void k_eval_f32_grouped(const EvalArgs* __restrict__ args,
                                                             const int* __restrict__ start, int n) {
  const int c = group_case(start, n, blockIdx.x);
  eval_f32<KP, MODE>(args[c], blockIdx.x - start[c]);
}
template <int KP>
__global__ __launch_bounds__(512, 1) void k_eval_f32_ws(EvalArgs a) {
  eval_f32_ws<KP>(a, blockIdx.x);
}
template <int KP>
__global__ __launch_bounds__(512, 1) void k_eval_f32_ws_grouped(const EvalArgs* __restrict__ args,
                                                                 const int* __restrict__ start, int n) {
  const int c = group_case(start, n, blockIdx.x);
  eval_f32_ws<KP>(args[c], blockIdx.x - start[c]);
}

template <int KP, int NG, int NH>
__global__ __launch_bounds__(64 * NG * NH, (NG * NH == 4) ? 2 : 1) void k_eval_acc64(EvalArgs a) {
  eval_acc64<KP, NG, NH>(a, blockIdx.x);
}
template <int KP, int NG, int NH>
__global__ __launch_bounds__(64 * NG * NH, (NG * NH == 4) ? 2 : 1) void k_eval_acc64_grouped(
    const EvalArgs* __restrict__ args, const int* __restrict__ start, int n) {
  const int c = group_case(start, n, blockIdx.x);
  eval_acc64<KP, NG, NH>(args[c], blockIdx.x - start[c]);
}
template <int KP>
__global__ __launch_bounds__(512, 1) void k_eval_acc64_ws(EvalArgs a) {
  eval_acc64_ws<KP>(a, blockIdx.x);
}
template <int KP>
__global__ __launch_bounds__(512, 1) void k_eval_acc64_ws_grouped(const EvalArgs* __restrict__ args,
                                                                   const int* __restrict__ start, int n) {
  const int c = group_case(start, n, blockIdx.x);
  eval_acc64_ws<KP>(args[c], blockIdx.x - start[c]);
}

template <int KP, int SHAPE>
__global__ __launch_bounds__(lp_threads(KP, SHAPE), 1) void k_eval_bf16(EvalArgs a) {
  if constexpr (SHAPE == 2) eval_lp_ws<KP, false>(a, blockIdx.x);
  else eval_lp<KP, false, SHAPE>(a, blockIdx.x);
}
template <int KP, int SHAPE>
__global__ __launch_bounds__(lp_threads(KP, SHAPE), 1) void k_eval_bf16_grouped(
    const EvalArgs* __restrict__ args, const int* __restrict__ start, int n) {
  const int c = group_case(start, n, blockIdx.x);
  if constexpr (SHAPE == 2) eval_lp_ws<KP, false>(args[c], blockIdx.x - start[c]);
  else eval_lp<KP, false, SHAPE>(args[c], blockIdx.x - start[c]);
}

template <int KP, int SHAPE>
__global__ __launch_bounds__(lp_threads(KP, SHAPE), 1) void k_eval_fp8(EvalArgs a) {
  if constexpr (SHAPE == 2) eval_lp_ws<KP, true>(a, blockIdx.x);
  else eval_lp<KP, true, SHAPE>(a, blockIdx.x);
}
template <int KP, int SHAPE>
__global__ __launch_bounds__(lp_threads(KP, SHAPE), 1) void k_eval_fp8_grouped(
    const EvalArgs* __restrict__ args, const int* __restrict__ start, int n) {
  const int c = group_case(start, n, blockIdx.x);
  if constexpr (SHAPE == 2) eval_lp_ws<KP, true>(args[c], blockIdx.x - start[c]);
  else eval_lp<KP, true, SHAPE>(args[c], blockIdx.x - start[c]);
}

// BF16 / FP8 launch in workgroup shape SHAPE (single case or grouped)
template <int KP, int SHAPE>
hipError_t launch_lp(const EvalArgs* single, const EvalArgs* args, const int* start, int n, int grid,
                     bool fp8, hipStream_t st) {
  const dim3 g(grid), b(lp_threads(KP, SHAPE));
  if (single) {
    if (fp8) hipLaunchKernelGGL((k_eval_fp8<KP, SHAPE>), g, b, 0, st, *single);
    else hipLaunchKernelGGL((k_eval_bf16<KP, SHAPE>), g, b, 0, st, *single);
  } else {
    if (fp8) hipLaunchKernelGGL((k_eval_fp8_grouped<KP, SHAPE>), g, b, 0, st, args, start, n);
    else hipLaunchKernelGGL((k_eval_bf16_grouped<KP, SHAPE>), g, b, 0, st, args, start, n);
  }
  return hipGetLastError();
}

template <int KP>
hipError_t launch_lp_shape(int shape, const EvalArgs* single, const EvalArgs* args, const int* start, int n,
                           int grid, bool fp8, hipStream_t st) {
  if constexpr (lp_shape_ok(KP, 1)) {
    if (shape == 1) return launch_lp<KP, 1>(single, args, start, n, grid, fp8, st);
  }
  if constexpr (lp_shape_ok(KP, 2)) {
    if (shape == 2) return launch_lp<KP, 2>(single, args, start, n, grid, fp8, st);
  }
  if (shape != 0) return hipErrorInvalidValue;
  return launch_lp<KP, 0>(single, args, start, n, grid, fp8, st);
}

template <int KP>
hipError_t launch_kp(const EvalArgs& a, int dtype, hipStream_t st) {
  if (a.grid < 1) return hipErrorInvalidValue;
  const dim3 grid(a.grid), block(256);
  if (dtype == GMCO_DTYPE_F32_ACC64 && a.lp_shape == 1)
    hipLaunchKernelGGL((k_eval_acc64<KP, 2, 2>), grid, dim3(256), 0, st, a);
  else if (dtype == GMCO_DTYPE_F32_ACC64 && a.lp_shape == 3)
    hipLaunchKernelGGL((k_eval_acc64_ws<KP>), grid, dim3(512), 0, st, a);
  else if (dtype == GMCO_DTYPE_F32_ACC64 && a.lp_shape == 2 && acc_quarters_ok(KP))
    hipLaunchKernelGGL((k_eval_acc64<KP, 4, (KP % 64 == 0 ? 4 : 2)>), grid, dim3(KP % 64 == 0 ? 1024 : 512), 0, st,
                       a);
  else if (dtype == GMCO_DTYPE_F32_ACC64)
    hipLaunchKernelGGL((k_eval_acc64<KP, 4, 2>), grid, dim3(512), 0, st, a);
  else if (dtype == GMCO_DTYPE_F32_CHUNK64)
    hipLaunchKernelGGL((k_eval_f32<KP, MODE_CHUNK64>), grid, block, 0, st, a);
  else if (dtype == GMCO_DTYPE_F32 && a.lp_shape == 3)
    hipLaunchKernelGGL((k_eval_f32_ws<KP>), grid, dim3(512), 0, st, a);
  else if (dtype == GMCO_DTYPE_F32)
    hipLaunchKernelGGL((k_eval_f32<KP, MODE_F32>), grid, block, 0, st, a);
  else if (dtype == GMCO_DTYPE_BF16 || dtype == GMCO_DTYPE_FP8)
    return launch_lp_shape<KP>(a.lp_shape, &a, nullptr, nullptr, 0, a.grid, dtype == GMCO_DTYPE_FP8, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int KP>
hipError_t launch_kp_grouped(const EvalArgs* args, const int* start, int n, int grid, int dtype, int lp_shape,
                             hipStream_t st) {
  if (grid < 1 || n < 1) return hipErrorInvalidValue;
  if (dtype == GMCO_DTYPE_F32_ACC64 && lp_shape == 1)
    hipLaunchKernelGGL((k_eval_acc64_grouped<KP, 2, 2>), dim3(grid), dim3(256), 0, st, args, start, n);
  else if (dtype == GMCO_DTYPE_F32_ACC64 && lp_shape == 3)
    hipLaunchKernelGGL((k_eval_acc64_ws_grouped<KP>), dim3(grid), dim3(512), 0, st, args, start, n);
  else if (dtype == GMCO_DTYPE_F32_ACC64 && lp_shape == 2 && acc_quarters_ok(KP))
    hipLaunchKernelGGL((k_eval_acc64_grouped<KP, 4, (KP % 64 == 0 ? 4 : 2)>), dim3(grid),
                       dim3(KP % 64 == 0 ? 1024 : 512), 0, st, args, start, n);
  else if (dtype == GMCO_DTYPE_F32_ACC64)
    hipLaunchKernelGGL((k_eval_acc64_grouped<KP, 4, 2>), dim3(grid), dim3(512), 0, st, args, start, n);
  else if (dtype == GMCO_DTYPE_F32_CHUNK64)
    hipLaunchKernelGGL((k_eval_f32_grouped<KP, MODE_CHUNK64>), dim3(grid), dim3(256), 0, st, args, start, n);
  else if (dtype == GMCO_DTYPE_F32 && lp_shape == 3)
    hipLaunchKernelGGL((k_eval_f32_ws_grouped<KP>), dim3(grid), dim3(512), 0, st, args, start, n);
  else if (dtype == GMCO_DTYPE_F32)
    hipLaunchKernelGGL((k_eval_f32_grouped<KP, MODE_F32>), dim3(grid), dim3(256), 0, st, args, start, n);
  else if (dtype == GMCO_DTYPE_BF16 || dtype == GMCO_DTYPE_FP8)
    return launch_lp_shape<KP>(lp_shape, nullptr, args, start, n, grid, dtype == GMCO_DTYPE_FP8, st);
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

hipError_t launch_eval_grouped(const EvalArgs* args, const int* start, int n, int grid, int Kp, int dtype,
                               int lp_shape, hipStream_t st) {
  switch (Kp) {
#define GMCO_KP_CASE(v) \
  case v:               \
    return launch_kp_grouped<v>(args, start, n, grid, dtype, lp_shape, st);
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
