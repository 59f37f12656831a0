// Warm-start network kernels (a project addition, not in the paper).
//
// Network 32 -> 256 -> 256 -> 256 -> 1 with the exact GELU z Phi(z) after
// each hidden layer; inputs standardised by a fixed (mean, scale) pair; loss
// the mean squared error; Adam with bias-corrected moments (Kingma & Ba).
// Parameters are one FP32 vector: per layer W (out x in, row-major), then
// the bias. All arithmetic is FP32; every reduction runs in a fixed order,
// so results are bitwise reproducible.
//
// Training works on a batch of B samples with one tiled GEMM kernel
// (64x64 output tile per workgroup, K staged through LDS in chunks of 32,
// 4x4 outputs per thread) in three access patterns:
//   forward   Z = H W^T + c        (A = H, B = W^T)
//   data grad dH = dZ W, times GELU'(Z_prev)
//   weight    dW = dZ^T H          (reduction over the batch)
// Single-sample inference inside the solver uses one fused workgroup.
#include "common.h"
#include "kernels.h"

namespace tls {

namespace {

constexpr int MT = 64, KC = 32;

__device__ inline float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ inline float gelu_grad_f(float z) {
  const float Phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float phi = expf(-0.5f * z * z) * 0.39894228040143268f;
  return Phi + z * phi;
}

}  // namespace

// C[M x N] = sum_k A(m, k) B(k, n)
//   A(m, k) = TA ? A[k * lda + m] : A[m * lda + k]
//   B(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n]
// EPI 0: C = acc + bias[n], H = GELU(C)      (hidden layer forward)
// EPI 1: C = acc + bias[n]                   (output layer forward)
// EPI 2: C = acc * GELU'(Zp[m * ldc + n])    (gradient w.r.t. a pre-activation)
// EPI 3: C = acc                             (weight gradient)
template <int TA, int TB, int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm(int M, int N, int K, const float *A, int lda,
                                                  const float *B, int ldb, const float *bias,
                                                  const float *Zp, float *C, float *H, int ldc) {
  __shared__ float As[KC][MT + 4];
  __shared__ float Bs[KC][MT + 4];
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  const int m0 = blockIdx.x * MT, n0 = blockIdx.y * MT;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += KC) {
    float ra[8], rb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + 256 * i;
      // A chunk: 64 rows (m) x 32 k
      int mm, kk;
      if (TA) { mm = e % MT; kk = e / MT; } else { kk = e % KC; mm = e / KC; }
      const int gm = m0 + mm, gk = k0 + kk;
      ra[i] = (gm < M && gk < K) ? (TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk]) : 0.0f;
      int nn, kb;
      if (TB) { kb = e % KC; nn = e / KC; } else { nn = e % MT; kb = e / MT; }
      const int gn = n0 + nn, gkb = k0 + kb;
      rb[i] = (gn < N && gkb < K) ? (TB ? B[(size_t)gn * ldb + gkb] : B[(size_t)gkb * ldb + gn]) : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + 256 * i;
      int mm, kk;
      if (TA) { mm = e % MT; kk = e / MT; } else { kk = e % KC; mm = e / KC; }
      As[kk][mm] = ra[i];
      int nn, kb;
      if (TB) { kb = e % KC; nn = e / KC; } else { nn = e % MT; kb = e / MT; }
      Bs[kb][nn] = rb[i];
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < KC; ++k) {
      float a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) { a[x] = As[k][tr * 4 + x]; b[x] = Bs[k][tc * 4 + x]; }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(a[x], b[y], acc[x][y]);
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int gm = m0 + tr * 4 + x, gn = n0 + tc * 4 + y;
      if (gm >= M || gn >= N) continue;
      const size_t o = (size_t)gm * ldc + gn;
      float v = acc[x][y];
      if (EPI == 0 || EPI == 1) v += bias[gn];
      if (EPI == 2) v *= gelu_grad_f(Zp[o]);
      C[o] = v;
      if (EPI == 0) H[o] = gelu_f(v);
    }
}

// h0 = (x - mean) * scale
__global__ void k_mlp_standardize(int64_t B, const float *X, const float *norm, float *H0) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= B * TLS_MLP_IN) return;
  const int j = (int)(i % TLS_MLP_IN);
  H0[i] = (X[i] - norm[j]) * norm[TLS_MLP_IN + j];
}

// loss = mean (y - t)^2 and dL/dy = 2 (y - t) / B, one workgroup, fixed order
__global__ __launch_bounds__(256) void k_mlp_mse(int64_t B, const float *y, const float *t,
                                                 float *dy, float *loss) {
  __shared__ float sc[4];
  float s = 0.0f;
  const float inv = 1.0f / (float)B;
  for (int64_t i = threadIdx.x; i < B; i += 256) {
    const float d = y[i] - t[i];
    s = fmaf(d, d, s);
    dy[i] = 2.0f * d * inv;
  }
  s = block_sum(s, sc);
  if (threadIdx.x == 0) *loss = s * inv;
}

// bias gradient: column sums of dZ (M x N), each column summed in row order
__global__ void k_mlp_colsum(int64_t M, int N, const float *dZ, float *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  for (int64_t i = 0; i < M; ++i) s += dZ[i * N + j];
  out[j] = s;
}

// Adam (Kingma & Ba, Algorithm 1) with host-computed bias corrections
__global__ void k_mlp_adam(int64_t count, float *theta, float *m, float *v, const float *g, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// One sample through the network in one workgroup (solver warm start):
// y (double) = net(features). Hidden rows are split over the 4 waves; a
// lane covers 4 consecutive inputs of a row and the wave sums the row.
__global__ __launch_bounds__(256) void k_mlp_infer1(const float *theta, const float *norm,
                                                    const float *feat, double *y) {
  __shared__ float h[2][TLS_MLP_WIDTH];
  __shared__ float x0[TLS_MLP_IN];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid < TLS_MLP_IN) x0[tid] = (feat[tid] - norm[tid]) * norm[TLS_MLP_IN + tid];
  __syncthreads();
  const float *W1 = theta, *c1 = W1 + TLS_MLP_WIDTH * TLS_MLP_IN;
  {
    float z = c1[tid];
    for (int k = 0; k < TLS_MLP_IN; ++k) z = fmaf(W1[tid * TLS_MLP_IN + k], x0[k], z);
    h[0][tid] = gelu_f(z);
  }
  __syncthreads();
  const float *p = c1 + TLS_MLP_WIDTH;
  for (int layer = 0; layer < 2; ++layer) {
    const float *W = p, *c = p + TLS_MLP_WIDTH * TLS_MLP_WIDTH;
    const float *hin = h[layer & 1];
    float *hout = h[(layer + 1) & 1];
    for (int j = w; j < TLS_MLP_WIDTH; j += 4) {
      const float *row = W + (size_t)j * TLS_MLP_WIDTH + 4 * lane;
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) s = fmaf(row[q], hin[4 * lane + q], s);
      s = wave_sum(s);
      if (lane == 0) hout[j] = gelu_f(s + c[j]);
    }
    __syncthreads();
    p = c + TLS_MLP_WIDTH;
  }
  if (w == 0) {
    const float *hin = h[0];   // after two hidden layers the result is back in h[0]
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) s = fmaf(p[4 * lane + q], hin[4 * lane + q], s);
    s = wave_sum(s);
    if (lane == 0) *y = (double)(s + p[TLS_MLP_WIDTH]);
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace {

template <int TA, int TB, int EPI>
hipError_t gemm(int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                const float *bias, const float *Zp, float *C, float *H, int ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((M + MT - 1) / MT, (N + MT - 1) / MT);
  TLS_LAUNCH(PC_MLP, (k_mlp_gemm<TA, TB, EPI>), g, dim3(256), 0, st, M, N, K, A, lda, B, ldb, bias, Zp, C,
             H, ldc);
  return hipGetLastError();
}

constexpr int W_ = TLS_MLP_WIDTH, I_ = TLS_MLP_IN;
// parameter offsets
constexpr size_t OW1 = 0, OC1 = OW1 + (size_t)W_ * I_, OW2 = OC1 + W_, OC2 = OW2 + (size_t)W_ * W_,
                 OW3 = OC2 + W_, OC3 = OW3 + (size_t)W_ * W_, OW4 = OC3 + W_, OC4 = OW4 + W_;
static_assert(OC4 + 1 == TLS_MLP_PARAMS, "parameter layout");

}  // namespace

hipError_t launch_mlp_forward(const float *theta, const float *norm, const float *X, int64_t B,
                              float *y, const MlpBufs &M, hipStream_t st) {
  const int b = (int)B;
  TLS_LAUNCH(PC_MLP, k_mlp_standardize, dim3((unsigned)((B * I_ + 255) / 256)), dim3(256), 0, st, B, X,
             norm, M.h0);
  hipError_t e;
  if ((e = gemm<0, 1, 0>(b, W_, I_, M.h0, I_, theta + OW1, I_, theta + OC1, nullptr, M.z[0], M.h[0], W_, st))) return e;
  if ((e = gemm<0, 1, 0>(b, W_, W_, M.h[0], W_, theta + OW2, W_, theta + OC2, nullptr, M.z[1], M.h[1], W_, st))) return e;
  if ((e = gemm<0, 1, 0>(b, W_, W_, M.h[1], W_, theta + OW3, W_, theta + OC3, nullptr, M.z[2], M.h[2], W_, st))) return e;
  return gemm<0, 1, 1>(b, 1, W_, M.h[2], W_, theta + OW4, W_, theta + OC4, nullptr, y, nullptr, 1, st);
}

hipError_t launch_mlp_backward(const float *theta, const float *y, const float *t, int64_t B,
                               float *grad, float *loss, const MlpBufs &M, hipStream_t st) {
  const int b = (int)B;
  hipError_t e;
  TLS_LAUNCH(PC_MLP, k_mlp_mse, dim3(1), dim3(256), 0, st, B, y, t, M.dy, loss);
  // output layer: dW4 = dy^T h3, dc4 = sum dy; dz3 = (dy w4) * GELU'(z3)
  if ((e = gemm<1, 0, 3>(1, W_, b, M.dy, 1, M.h[2], W_, nullptr, nullptr, grad + OW4, nullptr, W_, st))) return e;
  TLS_LAUNCH(PC_MLP, k_mlp_colsum, dim3(1), dim3(64), 0, st, B, 1, M.dy, grad + OC4);
  if ((e = gemm<0, 0, 2>(b, W_, 1, M.dy, 1, theta + OW4, W_, nullptr, M.z[2], M.dz[0], nullptr, W_, st))) return e;
  // hidden layers 3 and 2
  const size_t OW[3] = {OW1, OW2, OW3}, OC[3] = {OC1, OC2, OC3};
  int cur = 0;
  for (int l = 2; l >= 1; --l) {
    const float *hin = M.h[l - 1];
    if ((e = gemm<1, 0, 3>(W_, W_, b, M.dz[cur], W_, hin, W_, nullptr, nullptr, grad + OW[l], nullptr, W_, st))) return e;
    TLS_LAUNCH(PC_MLP, k_mlp_colsum, dim3(W_ / 64), dim3(64), 0, st, B, W_, M.dz[cur], grad + OC[l]);
    if ((e = gemm<0, 0, 2>(b, W_, W_, M.dz[cur], W_, theta + OW[l], W_, nullptr, M.z[l - 1], M.dz[cur ^ 1], nullptr, W_, st))) return e;
    cur ^= 1;
  }
  // first layer
  if ((e = gemm<1, 0, 3>(W_, I_, b, M.dz[cur], W_, M.h0, I_, nullptr, nullptr, grad + OW1, nullptr, I_, st))) return e;
  TLS_LAUNCH(PC_MLP, k_mlp_colsum, dim3(W_ / 64), dim3(64), 0, st, B, W_, M.dz[cur], grad + OC1);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(int64_t count, float *theta, float *m, float *v, const float *g, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t st) {
  TLS_LAUNCH(PC_MLP, k_mlp_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, theta, m,
             v, g, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_infer1(const float *theta, const float *norm, const float *feat, double *y,
                             hipStream_t st) {
  TLS_LAUNCH(PC_MLP, k_mlp_infer1, dim3(1), dim3(256), 0, st, theta, norm, feat, y);
  return hipGetLastError();
}

}  // namespace tls
