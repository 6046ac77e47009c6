// Learned warm start: a fully connected ReLU network trained on plans the
// method itself produced, and the case features it reads.
//
// Every product runs on v_mfma_f32_16x16x32_bf16 (BF16 operands rounded from
// FP32 activations and weights, FP32 accumulation); losses, gradients and the
// Adam moments are FP32.  Parameter layout: for each layer W (n_out x n_in,
// row-major) followed by b (n_out).
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gmco_internal.h"

namespace gmco {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

struct GemmArgs {
  const float* A;  // element (i, k) at A[i * sai + k * sak]
  long sai, sak;
  const float* B;  // element (k, j) at B[k * sbk + j * sbj]
  long sbk, sbj;
  float* C;        // C[i * ldc + j]
  long ldc;
  const float* bias;  // per column j, or NULL
  int M, N, K;
  int relu;
};

// 64 x 64 output tile per workgroup, 4 waves in 2 x 2, each a 32 x 32
// sub-tile of 2 x 2 matrix ops; K in slices of 32 staged in LDS as BF16.
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  constexpr int TS = 40;  // LDS row stride (elements): 80 B, conflict-free 16 B reads
  __shared__ __attribute__((aligned(16))) __bf16 sA[64 * TS];
  __shared__ __attribute__((aligned(16))) __bf16 sB[64 * TS];  // transposed: [j][k]
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, q = lane >> 4, n = lane & 15;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += 32) {
    // stage: thread t covers row t / 4, k-offset (t % 4) * 8 .. +7
    {
      const int r = tid >> 2, kk = (tid & 3) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = i0 + r, k = k0 + kk + e, j = j0 + r;
        const float av = (i < g.M && k < g.K) ? g.A[(long)i * g.sai + (long)k * g.sak] : 0.f;
        const float bv = (j < g.N && k < g.K) ? g.B[(long)k * g.sbk + (long)j * g.sbj] : 0.f;
        sA[r * TS + kk + e] = (__bf16)av;
        sB[r * TS + kk + e] = (__bf16)bv;
      }
    }
    __syncthreads();
    bf8v af[2], bfr[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      af[a] = *reinterpret_cast<const bf8v*>(&sA[(wr + 16 * a + n) * TS + 8 * q]);
      bfr[a] = *reinterpret_cast<const bf8v*>(&sB[(wc + 16 * a + n) * TS + 8 * q]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + 16 * a + 4 * q + r, j = j0 + wc + 16 * b + n;
        if (i < g.M && j < g.N) {
          float v = acc[a][b][r];
          if (g.bias) v += g.bias[j];
          if (g.relu) v = fmaxf(v, 0.f);
          g.C[(long)i * g.ldc + j] = v;
        }
      }
}

// dL/dout for L = mean((out - y)^2) over B x N entries, and the per-row
// partial sums of the squared error (summed in fixed order afterwards).
__global__ void k_mse(const float* __restrict__ out, const float* __restrict__ y, int B, int N,
                      float* __restrict__ g, double* __restrict__ row_loss) {
  const int i = blockIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  const float scale = 2.f / ((float)B * (float)N);
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const float d = out[(size_t)i * N + j] - y[(size_t)i * N + j];
    g[(size_t)i * N + j] = scale * d;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) row_loss[i] = red[0];
}

__global__ void k_sum_loss(const double* __restrict__ row_loss, int B, int N, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < B; i += blockDim.x) s += row_loss[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] / ((double)B * (double)N);
}

__global__ void k_relu_back(float* __restrict__ g, const float* __restrict__ act, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!(act[i] > 0.f)) g[i] = 0.f;
}

// db[j] = sum_i g[i][j], fixed order over rows
__global__ void k_colsum(const float* __restrict__ g, int B, int N, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int i = 0; i < B; ++i) s += g[(size_t)i * N + j];
  db[j] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_gather_rows(const float* __restrict__ src, const int* __restrict__ idx, int B, int N,
                              float* __restrict__ dst) {
  const int i = blockIdx.x;
  if (i >= B) return;
  const size_t s = (size_t)idx[i];
  for (int j = threadIdx.x; j < N; j += blockDim.x) dst[(size_t)i * N + j] = src[s * N + j];
}

// Case features: for dwell l and structure j the distance to the nearest
// point of j, binned in 16 bins of 0.25 cm (the last open-ended), divided by
// the dwell count.  (dx^2 + dy^2) + dz^2 without fused operations.
__global__ void k_features(const double* __restrict__ dwell, const double* __restrict__ pts,
                           const int* __restrict__ perm, const int* __restrict__ goff,
                           const int* __restrict__ gcnt, int K, unsigned* __restrict__ hist) {
  const int l = blockIdx.x, j = blockIdx.y;
  if (l >= K) return;  // (whole workgroup)
  __shared__ double red[256];
  double best = 1e300;
  const double qx = dwell[3 * l], qy = dwell[3 * l + 1], qz = dwell[3 * l + 2];
  for (int i = threadIdx.x; i < gcnt[j]; i += blockDim.x) {
    const int src = perm[goff[j] + i];
    const double dx = __dsub_rn(pts[3 * src], qx), dy = __dsub_rn(pts[3 * src + 1], qy);
    const double dz = __dsub_rn(pts[3 * src + 2], qz);
    const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    best = fmin(best, r2);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && gcnt[j] > 0) {
    const double r = sqrt(red[0]);
    int b = (int)floor(r / 0.25);
    b = b > 15 ? 15 : (b < 0 ? 0 : b);
    atomicAdd(&hist[j * 16 + b], 1u);
  }
}

__global__ void k_features_norm(const unsigned* __restrict__ hist, int n, int K, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)((double)hist[i] / (double)K);
}

}  // namespace
}  // namespace gmco

using namespace gmco;

struct gmco_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<int> sizes;
  int max_batch = 0;
  size_t n_params = 0;
  std::vector<size_t> woff, boff;  // parameter offsets per layer
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  std::vector<float*> act;   // act[0] = input, act[k+1] = output of layer k
  std::vector<float*> dact;  // gradient buffers, same shapes
  float* y = nullptr;        // targets of the batch
  double* row_loss = nullptr;
  double* loss = nullptr;
  int* idx = nullptr;
  float *dataX = nullptr, *dataY = nullptr;
  int n_data = 0;
  int adam_step = 0;
  std::vector<void*> owned;
  std::string err;
};

namespace {

int mfail(gmco_mlp* m, int code, const std::string& msg) {
  if (m) m->err = msg;
  return code;
}

#define MLP_HIP(mm, call)                                                             \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return mfail((mm), GMCO_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

hipError_t gemm(hipStream_t st, const float* A, long sai, long sak, const float* B, long sbk, long sbj,
                float* C, long ldc, const float* bias, int M, int N, int K, int relu) {
  GemmArgs a{A, sai, sak, B, sbk, sbj, C, ldc, bias, M, N, K, relu};
  hipLaunchKernelGGL(k_gemm_bf16, dim3((N + 63) / 64, (M + 63) / 64), dim3(256), 0, st, a);
  return hipGetLastError();
}

int layers(const gmco_mlp* m) { return (int)m->sizes.size() - 1; }

// forward over act[0] (B rows): act[k+1] = relu?(act[k] W_k^T + b_k), on
// stream st (the network's own unless a caller's)
hipError_t forward(gmco_mlp* m, int B, hipStream_t st) {
  const int L = layers(m);
  for (int k = 0; k < L; ++k) {
    const int in = m->sizes[k], out = m->sizes[k + 1];
    hipError_t e = gemm(st, m->act[k], in, 1, m->p + m->woff[k], 1, in, m->act[k + 1], out,
                        m->p + m->boff[k], B, out, in, k < L - 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t forward(gmco_mlp* m, int B) { return forward(m, B, m->stream); }

// backward from the targets in m->y; gradients into m->g, loss into *m->loss
hipError_t backward(gmco_mlp* m, int B) {
  const int L = layers(m);
  const int nout = m->sizes[L];
  hipLaunchKernelGGL(k_mse, dim3(B), dim3(256), 0, m->stream, m->act[L], m->y, B, nout, m->dact[L],
                     m->row_loss);
  hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, m->stream, m->row_loss, B, nout, m->loss);
  for (int k = L - 1; k >= 0; --k) {
    const int in = m->sizes[k], out = m->sizes[k + 1];
    float* G = m->dact[k + 1];
    if (k < L - 1) {
      hipLaunchKernelGGL(k_relu_back, dim3(256), dim3(256), 0, m->stream, G, m->act[k + 1],
                         (size_t)B * out);
    }
    // dW_k = G^T act[k]   (out x in), contraction over the batch
    hipError_t e = gemm(m->stream, G, 1, out, m->act[k], in, 1, m->g + m->woff[k], in, nullptr, out, in,
                        B, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3((out + 255) / 256), dim3(256), 0, m->stream, G, B, out,
                       m->g + m->boff[k]);
    if (k > 0) {
      // d act[k] = G W_k   (B x in)
      e = gemm(m->stream, G, out, 1, m->p + m->woff[k], in, 1, m->dact[k], in, nullptr, B, in, out, 0);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

int gmco_mlp_create(gmco_mlp** out, int device, const int* sizes, int n_sizes, int max_batch) {
  if (!out || !sizes || n_sizes < 2 || max_batch < 1) return GMCO_EINVAL;
  *out = nullptr;
  for (int k = 0; k < n_sizes; ++k)
    if (sizes[k] < 1 || sizes[k] > 4096) return GMCO_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GMCO_ENOLIB;
  if (device < 0 || device >= ndev) return GMCO_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return GMCO_EHIP;
  gmco_mlp* m = new (std::nothrow) gmco_mlp();
  if (!m) return GMCO_ENOMEM;
  m->device = device;
  m->sizes.assign(sizes, sizes + n_sizes);
  m->max_batch = max_batch;
  size_t off = 0;
  for (int k = 0; k + 1 < n_sizes; ++k) {
    m->woff.push_back(off);
    off += (size_t)sizes[k] * sizes[k + 1];
    m->boff.push_back(off);
    off += (size_t)sizes[k + 1];
  }
  m->n_params = off;
  auto alloc = [&](size_t bytes) -> void* {
    void* ptr = nullptr;
    if (hipMalloc(&ptr, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
    m->owned.push_back(ptr);
    return ptr;
  };
  bool ok = true;
  m->p = (float*)alloc(off * 4);
  m->g = (float*)alloc(off * 4);
  m->m = (float*)alloc(off * 4);
  m->v = (float*)alloc(off * 4);
  for (int k = 0; k < n_sizes; ++k) {
    m->act.push_back((float*)alloc((size_t)max_batch * sizes[k] * 4));
    m->dact.push_back((float*)alloc((size_t)max_batch * sizes[k] * 4));
  }
  m->y = (float*)alloc((size_t)max_batch * sizes[n_sizes - 1] * 4);
  m->row_loss = (double*)alloc((size_t)max_batch * 8);
  m->loss = (double*)alloc(8);
  m->idx = (int*)alloc((size_t)max_batch * 4);
  for (void* ptr : m->owned) ok = ok && ptr;
  if (!ok || hipMemset(m->p, 0, off * 4) != hipSuccess || hipMemset(m->m, 0, off * 4) != hipSuccess ||
      hipMemset(m->v, 0, off * 4) != hipSuccess) {
    gmco_mlp_destroy(m);
    return GMCO_ENOMEM;
  }
  *out = m;
  return GMCO_OK;
}

int gmco_mlp_destroy(gmco_mlp* m) {
  if (!m) return GMCO_OK;
  hipSetDevice(m->device);
  hipDeviceSynchronize();
  for (void* ptr : m->owned) hipFree(ptr);
  delete m;
  return GMCO_OK;
}

int gmco_mlp_set_stream(gmco_mlp* m, void* stream) {
  if (!m) return GMCO_EINVAL;
  m->stream = (hipStream_t)stream;
  return GMCO_OK;
}

int gmco_mlp_param_count(const gmco_mlp* m, size_t* n) {
  if (!m || !n) return GMCO_EINVAL;
  *n = m->n_params;
  return GMCO_OK;
}

const char* gmco_mlp_last_error(const gmco_mlp* m) { return m ? m->err.c_str() : "null network"; }

int gmco_mlp_set_params(gmco_mlp* m, const float* p, size_t n) {
  if (!m || !p || n != m->n_params) return GMCO_EINVAL;
  MLP_HIP(m, hipSetDevice(m->device));
  MLP_HIP(m, hipMemcpyAsync(m->p, p, n * 4, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipMemsetAsync(m->m, 0, n * 4, m->stream));
  MLP_HIP(m, hipMemsetAsync(m->v, 0, n * 4, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  m->adam_step = 0;
  return GMCO_OK;
}

int gmco_mlp_get_params(gmco_mlp* m, float* p, size_t n) {
  if (!m || !p || n != m->n_params) return GMCO_EINVAL;
  MLP_HIP(m, hipSetDevice(m->device));
  MLP_HIP(m, hipMemcpyAsync(p, m->p, n * 4, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return GMCO_OK;
}

int gmco_mlp_loss_grad(gmco_mlp* m, int B, const float* X, const float* Y, double* loss, float* grad) {
  if (!m || !X || !Y || B < 1 || B > m->max_batch) return GMCO_EINVAL;
  MLP_HIP(m, hipSetDevice(m->device));
  const int L = layers(m);
  MLP_HIP(m, hipMemcpyAsync(m->act[0], X, (size_t)B * m->sizes[0] * 4, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipMemcpyAsync(m->y, Y, (size_t)B * m->sizes[L] * 4, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, forward(m, B));
  MLP_HIP(m, backward(m, B));
  if (loss) MLP_HIP(m, hipMemcpyAsync(loss, m->loss, 8, hipMemcpyDeviceToHost, m->stream));
  if (grad) MLP_HIP(m, hipMemcpyAsync(grad, m->g, m->n_params * 4, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return GMCO_OK;
}

int gmco_mlp_set_data(gmco_mlp* m, int N, const float* X, const float* Y) {
  if (!m || N < 1 || !X || !Y) return GMCO_EINVAL;
  MLP_HIP(m, hipSetDevice(m->device));
  const int L = layers(m);
  for (float* ptr : {m->dataX, m->dataY}) {
    if (ptr) {
      m->owned.erase(std::find(m->owned.begin(), m->owned.end(), (void*)ptr));
      hipFree(ptr);
    }
  }
  m->dataX = m->dataY = nullptr;
  m->n_data = 0;
  void *dx = nullptr, *dy = nullptr;
  if (hipMalloc(&dx, (size_t)N * m->sizes[0] * 4) != hipSuccess) return mfail(m, GMCO_ENOMEM, "data X");
  m->owned.push_back(dx);
  if (hipMalloc(&dy, (size_t)N * m->sizes[L] * 4) != hipSuccess) return mfail(m, GMCO_ENOMEM, "data Y");
  m->owned.push_back(dy);
  m->dataX = (float*)dx;
  m->dataY = (float*)dy;
  MLP_HIP(m, hipMemcpyAsync(dx, X, (size_t)N * m->sizes[0] * 4, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipMemcpyAsync(dy, Y, (size_t)N * m->sizes[L] * 4, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  m->n_data = N;
  return GMCO_OK;
}

int gmco_mlp_train(gmco_mlp* m, int n_steps, int B, const int32_t* order, float lr, double* mean_loss) {
  if (!m || !order || n_steps < 1 || B < 1 || B > m->max_batch || !(lr > 0.f)) return GMCO_EINVAL;
  if (m->n_data == 0) return mfail(m, GMCO_ESTATE, "gmco_mlp_set_data first");
  for (size_t i = 0; i < (size_t)n_steps * B; ++i)
    if (order[i] < 0 || order[i] >= m->n_data) return mfail(m, GMCO_EINVAL, "sample index out of range");
  MLP_HIP(m, hipSetDevice(m->device));
  const int L = layers(m);
  int* dorder = nullptr;
  double* losses = nullptr;
  MLP_HIP(m, hipMalloc(&dorder, (size_t)n_steps * B * 4));
  if (hipMalloc(&losses, (size_t)n_steps * 8) != hipSuccess) {
    hipFree(dorder);
    return mfail(m, GMCO_ENOMEM, "loss buffer");
  }
  struct Free {
    void* a;
    void* b;
    ~Free() {
      hipFree(a);
      hipFree(b);
    }
  } guard{dorder, losses};
  MLP_HIP(m, hipMemcpyAsync(dorder, order, (size_t)n_steps * B * 4, hipMemcpyHostToDevice, m->stream));
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int s = 0; s < n_steps; ++s) {
    hipLaunchKernelGGL(k_gather_rows, dim3(B), dim3(128), 0, m->stream, m->dataX, dorder + (size_t)s * B, B,
                       m->sizes[0], m->act[0]);
    hipLaunchKernelGGL(k_gather_rows, dim3(B), dim3(128), 0, m->stream, m->dataY, dorder + (size_t)s * B, B,
                       m->sizes[L], m->y);
    MLP_HIP(m, forward(m, B));
    MLP_HIP(m, backward(m, B));
    MLP_HIP(m, hipMemcpyAsync(losses + s, m->loss, 8, hipMemcpyDeviceToDevice, m->stream));
    m->adam_step += 1;
    const float c1 = 1.f - powf(b1, (float)m->adam_step), c2 = 1.f - powf(b2, (float)m->adam_step);
    hipLaunchKernelGGL(k_adam, dim3(256), dim3(256), 0, m->stream, m->p, m->g, m->m, m->v, m->n_params, lr, b1,
                       b2, eps, c1, c2);
    MLP_HIP(m, hipGetLastError());
  }
  std::vector<double> h(n_steps);
  MLP_HIP(m, hipMemcpyAsync(h.data(), losses, (size_t)n_steps * 8, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  if (mean_loss) {
    double s = 0.0;
    for (double v : h) s += v;
    *mean_loss = s / n_steps;
  }
  return GMCO_OK;
}

int gmco_mlp_predict(gmco_mlp* m, int B, const float* X, float* Y) {
  if (!m || !X || !Y || B < 1) return GMCO_EINVAL;
  MLP_HIP(m, hipSetDevice(m->device));
  const int L = layers(m);
  for (int b0 = 0; b0 < B; b0 += m->max_batch) {
    const int nb = std::min(m->max_batch, B - b0);
    MLP_HIP(m, hipMemcpyAsync(m->act[0], X + (size_t)b0 * m->sizes[0], (size_t)nb * m->sizes[0] * 4,
                              hipMemcpyHostToDevice, m->stream));
    MLP_HIP(m, forward(m, nb));
    MLP_HIP(m, hipMemcpyAsync(Y + (size_t)b0 * m->sizes[L], m->act[L], (size_t)nb * m->sizes[L] * 4,
                              hipMemcpyDeviceToHost, m->stream));
  }
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return GMCO_OK;
}

}  // extern "C"

namespace gmco {
int mlp_inputs(const gmco_mlp* m) { return m->sizes.front(); }
int mlp_outputs(const gmco_mlp* m) { return m->sizes.back(); }
int mlp_device(const gmco_mlp* m) { return m->device; }

// The network on B rows held in device memory (X: B x n_in, Y: B x n_out),
// in chunks of max_batch rows, all on stream st.  The network's activation
// buffers are used, so st must be ordered with the network's other work.
hipError_t mlp_forward_device(gmco_mlp* m, int B, const float* X, float* Y, hipStream_t st) {
  const int L = layers(m);
  for (int b0 = 0; b0 < B; b0 += m->max_batch) {
    const int nb = std::min(m->max_batch, B - b0);
    hipError_t e = hipMemcpyAsync(m->act[0], X + (size_t)b0 * m->sizes[0], (size_t)nb * m->sizes[0] * 4,
                                  hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    e = forward(m, nb, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(Y + (size_t)b0 * m->sizes[L], m->act[L], (size_t)nb * m->sizes[L] * 4,
                       hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_features(const double* dwell, const double* pts, const int* perm, const int* goff,
                           const int* gcnt, int K, int G, unsigned* hist, float* out, hipStream_t st) {
  hipError_t e = hipMemsetAsync(hist, 0, (size_t)G * 16 * 4, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_features, dim3(K, G), dim3(256), 0, st, dwell, pts, perm, goff, gcnt, K, hist);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_features_norm, dim3(1), dim3(256), 0, st, hist, G * 16, K, out);
  return hipGetLastError();
}
}  // namespace gmco
