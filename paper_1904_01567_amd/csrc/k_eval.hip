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

// ACC64 = false: FP32 operands, FP32 accumulation (v_mfma_f32_16x16x4_f32).
// ACC64 = true : FP32 operands, the dose accumulated in FP64
//                (v_mfma_f64_16x16x4_f64) and the penalty evaluated in FP64;
//                the back-projection stays FP32.
template <int KP, bool ACC64>
__global__ __launch_bounds__(256, 1) void k_eval_f32(EvalArgs a) {
  constexpr int KS = KP + 4;       // LDS row stride (floats): conflict-free both ways
  constexpr int NK16 = KP / 16;    // 16-dwell slices
  constexpr int NF4 = 4 * KP;      // float4 per 16-point block
  constexpr int NPF = (NF4 + 255) / 256;

  __shared__ __attribute__((aligned(16))) float sD[kBM * KS];
  __shared__ float sW[kPT * kGmax];
  __shared__ float4 sP[kGmax + 1];
  __shared__ double sP64[kGmax + 1][4];
  __shared__ int sG[kBM];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int n = lane & 15;

  int s, tile;
  split_tile(blockIdx.x, a.S, a.ntiles, s, tile);
  const int p0 = tile * kPT;

  // Skip tiles whose plans have all stopped.
  if (a.ps != nullptr) {
    int act = 0;
    if (tid < kPT) act = state_active(a.ps[p0 + tid].status) ? 1 : 0;
    if (!__syncthreads_or(act)) return;
  }
  if (a.work != nullptr && tid == 0) atomicAdd(a.work, 1ull);

  for (int i = tid; i < kPT * kGmax; i += 256) sW[i] = a.wn[(size_t)p0 * kGmax + i];
#pragma unroll
  for (int j = 0; j <= kGmax; ++j)
    if (tid == j) {
      sP[j] = a.gt.prm[j];
#pragma unroll
      for (int c = 0; c < 4; ++c) sP64[j][c] = a.gt.prm64[j][c];
    }

  const int plan = p0 + wave * 16 + n;
  const float* __restrict__ xrow = a.x + (size_t)plan * KP;
  // B operand of the dose product: lane (q, n) holds t = x^2 of plan n at
  // dwells 16 k + 4 q + j (j = 0..3) for slice k.
  float tf[KP / 4];
#pragma unroll
  for (int k = 0; k < NK16; ++k) {
    const float4 xv = *reinterpret_cast<const float4*>(xrow + 16 * k + 4 * q);
    tf[4 * k + 0] = xv.x * xv.x;
    tf[4 * k + 1] = xv.y * xv.y;
    tf[4 * k + 2] = xv.z * xv.z;
    tf[4 * k + 3] = xv.w * xv.w;
  }
  f4v gacc[NK16];
#pragma unroll
  for (int k = 0; k < NK16; ++k) gacc[k] = f4v{0.f, 0.f, 0.f, 0.f};
  double facc = 0.0;

  const int b_begin = (int)(((long long)s * a.nblocks) / a.S);
  const int b_end = (int)(((long long)(s + 1) * a.nblocks) / a.S);
  const f4v* __restrict__ Dg = reinterpret_cast<const f4v*>(a.D);

  f4v pf[NPF];
  int gpre = 0;
  if (b_begin < b_end) {
    const f4v* src = Dg + (size_t)b_begin * NF4;
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int idx = tid + 256 * i;
      if (NF4 % 256 == 0 || idx < NF4) pf[i] = src[idx];
    }
    if (tid < kBM) gpre = a.grp[b_begin * kBM + tid];
  }

  for (int b = b_begin; b < b_end; ++b) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int idx = tid + 256 * i;
      if (NF4 % 256 == 0 || idx < NF4) {
        const int row = idx / (KP / 4);
        const int c4 = idx - row * (KP / 4);
        *reinterpret_cast<f4v*>(&sD[row * KS + 4 * c4]) = pf[i];
      }
    }
    if (tid < kBM) sG[tid] = gpre;
    __syncthreads();
    {
      // next block (the last iteration reloads its own block, in bounds)
      const int bn = (b + 1 < b_end) ? b + 1 : b;
      const f4v* src = Dg + (size_t)bn * NF4;
#pragma unroll
      for (int i = 0; i < NPF; ++i) {
        const int idx = tid + 256 * i;
        if (NF4 % 256 == 0 || idx < NF4) pf[i] = src[idx];
      }
      if (tid < kBM) gpre = a.grp[bn * kBM + tid];
    }

    // ---- dose product d[16 points][16 plans] and penalty epilogue
    //      (eq. 1, the bracket of eq. 2, eq. (obj) weights) ----
    float phi[4];
    if constexpr (ACC64) {
      // four independent accumulation chains keep the FP64 pipe busy
      d4v acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
#pragma unroll
      for (int k = 0; k < NK16; ++k) {
        const float4 av = *reinterpret_cast<const float4*>(&sD[n * KS + 16 * k + 4 * q]);
        acc0 = mfma_f64(av.x, tf[4 * k + 0], acc0);
        acc1 = mfma_f64(av.y, tf[4 * k + 1], acc1);
        acc2 = mfma_f64(av.z, tf[4 * k + 2], acc2);
        acc3 = mfma_f64(av.w, tf[4 * k + 3], acc3);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double d = (acc0[r] + acc1[r]) + (acc2[r] + acc3[r]);
        const int gi = sG[q + 4 * r];
        const float w = (gi < kGmax) ? sW[(wave * 16 + n) * kGmax + gi] : 0.f;
        double kap = 0.0, dev = 0.0;
        if (d < sP64[gi][1]) {
          dev = d - sP64[gi][1];
          kap = sP64[gi][0] * dev;
        } else if (d > sP64[gi][2]) {
          dev = d - sP64[gi][2];
          kap = sP64[gi][3] * dev;
        }
        facc += (double)w * (kap * dev);
        phi[r] = (float)((double)w * kap);
      }
    } else {
      f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < NK16; ++k) {
        const float4 av = *reinterpret_cast<const float4*>(&sD[n * KS + 16 * k + 4 * q]);
        acc0 = mfma_f32(av.x, tf[4 * k + 0], acc0);
        acc1 = mfma_f32(av.y, tf[4 * k + 1], acc1);
        acc0 = mfma_f32(av.z, tf[4 * k + 2], acc0);
        acc1 = mfma_f32(av.w, tf[4 * k + 3], acc1);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float d = acc0[r] + acc1[r];
        const int gi = sG[4 * q + r];
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
        phi[r] = w * kap;
      }
    }
    // ---- back-projection: G[dwell][plan] += sum_points D[point][dwell] phi ----
#pragma unroll
    for (int k = 0; k < NK16; ++k) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ACC64 ? q + 4 * r : 4 * q + r;
        const float av = sD[row * KS + 16 * k + n];
        gacc[k] = mfma_f32(av, phi[r], gacc[k]);
      }
    }
  }

  // ---- write split partials ----
  float* __restrict__ gout = a.Gpart + ((size_t)s * a.Pp + plan) * KP;
#pragma unroll
  for (int k = 0; k < NK16; ++k) {
    *reinterpret_cast<float4*>(gout + 16 * k + 4 * q) =
        make_float4(gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]);
  }
  facc += __shfl_xor(facc, 16);
  facc += __shfl_xor(facc, 32);
  if (q == 0) a.Fpart[(size_t)s * a.Pp + plan] = facc;
}

template <int KP>
hipError_t launch_f32_kp(const EvalArgs& a, int dtype, hipStream_t st) {
  if (dtype == GMCO_DTYPE_F32_ACC64)
    hipLaunchKernelGGL((k_eval_f32<KP, true>), dim3(a.S * a.ntiles), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_eval_f32<KP, false>), dim3(a.S * a.ntiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const EvalArgs& a, int dtype, hipStream_t st) {
  if (dtype != GMCO_DTYPE_F32 && dtype != GMCO_DTYPE_F32_ACC64) return hipErrorInvalidValue;
  switch (a.Kp) {
#define GMCO_KP_CASE(v) \
  case v:               \
    return launch_f32_kp<v>(a, dtype, st);
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
