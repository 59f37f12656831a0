// Explicit inverse of the triangular factor and its application.
//
// Applying R^{-1} and R^{-T} (the forward/backward substitutions of
// Table 1) is the inner operation of every PCGTLS step (Algorithm 3). A
// substitution is a chain of n/64 dependent block steps; on a GPU with
// eight L2 domains each hop costs microseconds. Since R is fixed for the
// whole solve (it is computed once, Section 2), X = R_hat^{-1} is formed
// once here (n^3/3 flops, the cost of the Cholesky factorization itself)
// and every application becomes a GEMV with the upper triangle of X: fully
// parallel, bandwidth-bound, deterministic.
//
// Inversion: recursive 2x2 block inversion of the upper triangular matrix,
//   inv([A B; 0 C]) = [inv(A), -inv(A) B inv(C); 0, inv(C)],
// bottom-up over block sizes 64, 128, 256, ...: level L combines pairs of
// inverted diagonal blocks of order h = 64*2^(L-1) with two tiled GEMM
// phases (Y = B inv(C), then X12 = -inv(A) Y), all pairs and output tiles
// of a level in one launch. Arithmetic in FP64 on the stored R_hat values.
//
// Storage of X (precision SX): two packed copies of 64x64 column-major tiles,
//   XR: tiles (I, K), K >= I, packed by block row   (for X v)
//   XC: tiles (J, I) of X^T, I <= J, packed by block row of X^T (for X^T v)
// In both products lane l owns row l of a tile and the wave reads the tile
// column by column, each load 64 consecutive elements.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tls {

// packed index helpers (N blocks)
__host__ __device__ inline size_t up_tile(int I, int J) {   // R tiles: column-packed upper
  return (size_t)J * (J + 1) / 2 + I;
}
__host__ __device__ inline size_t xr_tile(int I, int K, int N) {   // X tiles, packed by block row (upper)
  return (size_t)I * N - (size_t)I * (I - 1) / 2 + (K - I);
}
__host__ __device__ inline size_t xc_tile(int J, int I) {    // X^T tiles, packed by block row (lower)
  return (size_t)J * (J + 1) / 2 + I;
}

// ---------------------------------------------------------------------------
// inversion, working copy W in the compute precision C: FP64 for an FP64
// factor, FP32 otherwise (X is then stored in FP32, and FP32 arithmetic on
// the rounded R_hat leaves an error far below the rounding of R_hat itself).
// Full upper tiles in column-packed order (tile (I, J) at up_tile(I, J)),
// column-major inside a tile.
// ---------------------------------------------------------------------------
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_inv_init(int N, const S *Rt, const double *dinv64, C *W) {
  // diagonal tiles of W = stored diagonal inverses; off-diagonal tiles = R_hat
  const int l = blockIdx.x;
  int J = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= l) ++J;
  while (J * (J + 1) / 2 > l) --J;
  const int I = l - J * (J + 1) / 2;
  C *dst = W + (size_t)l * NB * NB;
  if (I == J) {
    const double *src = dinv64 + (size_t)I * NB * NB;
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) dst[t] = (C)src[t];
  } else {
    const S *src = Rt + (size_t)l * NB * NB;
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) dst[t] = cvt<C>(src[t]);
  }
}

// 64x64x64 tile products accumulated by 256 threads. The operand tiles
// (column-major in global memory) travel through registers: the loads of
// product k+1 are in flight while product k runs from LDS, so each product
// costs one memory latency at most once.
template <typename C>
struct TileRegs {
  C a[16], b[16];
};
template <typename C>
__device__ inline void tile_fetch(const C *A, const C *B, TileRegs<C> &R) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    R.a[i] = A[tid + 256 * i];
    R.b[i] = B[tid + 256 * i];
  }
}
template <typename C>
__device__ inline void tile_stage(const TileRegs<C> &R, C (*As)[NB + 1], C (*Bs)[NB + 1]) {
  const int tid = threadIdx.x;
  __syncthreads();   // the previous product has finished reading LDS
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int t = tid + 256 * i, r = t % NB, c = t / NB;
    As[r][c] = R.a[i];
    Bs[r][c] = R.b[i];
  }
  __syncthreads();
}
// C += A B on the matrix cores: wave w holds the 32x32 quadrant (w / 2,
// w % 2) of C. FP64: 2x2 blocks of v_mfma_f64_16x16x4 results (lane l,
// register q: row 4q + l/16, column l mod 16 of a block); FP32: one
// v_mfma_f32_32x32x2 result (register q: row 8(q/4) + 4(l/32) + q mod 4,
// column l mod 32). Each lane reads one element of A and of B per k-step.
typedef double inv_f64x4 __attribute__((ext_vector_type(4)));
typedef float inv_f32x16 __attribute__((ext_vector_type(16)));
template <typename C>
struct TileAcc;
template <>
struct TileAcc<double> {
  inv_f64x4 c[2][2];
};
template <>
struct TileAcc<float> {
  inv_f32x16 c;
};
__device__ inline void tile_zero(TileAcc<double> &T) {
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) T.c[t][u] = inv_f64x4{0.0, 0.0, 0.0, 0.0};
}
__device__ inline void tile_zero(TileAcc<float> &T) {
#pragma unroll
  for (int q = 0; q < 16; ++q) T.c[q] = 0.0f;
}
__device__ inline void tile_mma(const double (*As)[NB + 1], const double (*Bs)[NB + 1], TileAcc<double> &T) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll 4
  for (int k0 = 0; k0 < NB; k0 += 4) {
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = As[wr * 32 + t * 16 + (lane & 15)][k0 + (lane >> 4)];
      b[t] = Bs[k0 + (lane >> 4)][wc * 32 + t * 16 + (lane & 15)];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        T.c[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], T.c[t][u], 0, 0, 0);
  }
}
__device__ inline void tile_mma(const float (*As)[NB + 1], const float (*Bs)[NB + 1], TileAcc<float> &T) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll 8
  for (int k0 = 0; k0 < NB; k0 += 2) {
    const float a = As[wr * 32 + (lane & 31)][k0 + (lane >> 5)];
    const float b = Bs[k0 + (lane >> 5)][wc * 32 + (lane & 31)];
    T.c = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, T.c, 0, 0, 0);
  }
}
// dst (column-major 64x64 tile) = sign * C
__device__ inline void tile_store(const TileAcc<double> &T, double *dst, double sign) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wr * 32 + t * 16 + 4 * q + (lane >> 4);
        const int c = wc * 32 + u * 16 + (lane & 15);
        dst[c * NB + r] = sign * T.c[t][u][q];
      }
}
__device__ inline void tile_store(const TileAcc<float> &T, float *dst, float sign) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = wr * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
    const int c = wc * 32 + (lane & 31);
    dst[c * NB + r] = sign * T.c[q];
  }
}

// phase 1 of level L: Y = B inv(C) for every pair p; Y tile (a, b), a, b in [0, hb)
// B tile (a, k) = W(I0 + a, J0 + k) (still R_hat), inv(C) tile (k, b) = W(J0 + k, J0 + b), k <= b
template <typename C>
__global__ __launch_bounds__(256) void k_inv_phase1(int N, int hb, C *W, C *Y) {
  __shared__ C As[NB][NB + 1], Bs[NB][NB + 1];
  const int per = hb * hb;
  const int pair = blockIdx.x / per, rem = blockIdx.x % per;
  const int a = rem % hb, b = rem / hb;
  const int I0 = pair * 2 * hb, J0 = I0 + hb;
  if (J0 + b >= N || I0 + a >= N) return;      // partial pair at the end (uniform)
  TileAcc<C> acc;
  tile_zero(acc);
  const int kend = b;                           // J0 + b < N, so every k <= b is in range
  TileRegs<C> R;
  tile_fetch(W + up_tile(I0 + a, J0) * NB * NB, W + up_tile(J0, J0 + b) * NB * NB, R);
  for (int k = 0; k <= kend; ++k) {
    tile_stage(R, As, Bs);
    if (k < kend)
      tile_fetch(W + up_tile(I0 + a, J0 + k + 1) * NB * NB, W + up_tile(J0 + k + 1, J0 + b) * NB * NB, R);
    tile_mma(As, Bs, acc);
  }
  tile_store(acc, Y + ((size_t)pair * per + rem) * NB * NB, (C)1);
}

// phase 2: W(I0 + a, J0 + b) = - sum_{k >= a} inv(A)(a, k) Y(k, b)
template <typename C>
__global__ __launch_bounds__(256) void k_inv_phase2(int N, int hb, C *W, const C *Y) {
  __shared__ C As[NB][NB + 1], Bs[NB][NB + 1];
  const int per = hb * hb;
  const int pair = blockIdx.x / per, rem = blockIdx.x % per;
  const int a = rem % hb, b = rem / hb;
  const int I0 = pair * 2 * hb, J0 = I0 + hb;
  if (J0 + b >= N || I0 + a >= N) return;
  TileAcc<C> acc;
  tile_zero(acc);
  const int kend = hb - 1;                      // I0 + k < J0 < N for every k < hb
  TileRegs<C> R;
  auto yt = [&](int k) { return Y + ((size_t)pair * per + b * hb + k) * NB * NB; };
  tile_fetch(W + up_tile(I0 + a, I0 + a) * NB * NB, yt(a), R);
  for (int k = a; k <= kend; ++k) {
    tile_stage(R, As, Bs);
    if (k < kend) tile_fetch(W + up_tile(I0 + a, I0 + k + 1) * NB * NB, yt(k + 1), R);
    tile_mma(As, Bs, acc);
  }
  tile_store(acc, W + up_tile(I0 + a, J0 + b) * NB * NB, (C)-1);
}

// pack W (column-packed, column-major tiles) into XR and XC of precision SX
template <typename SX, typename C>
__global__ __launch_bounds__(256) void k_inv_pack(int N, const C *W, SX *XR, SX *XC) {
  const int l = blockIdx.x;
  int J = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= l) ++J;
  while (J * (J + 1) / 2 > l) --J;
  const int I = l - J * (J + 1) / 2;
  const C *src = W + (size_t)l * NB * NB;
  SX *xr = XR + xr_tile(I, J, N) * NB * NB;
  SX *xc = XC + xc_tile(J, I) * NB * NB;
  // both targets column-major within the tile (element (row, col) at
  // col * 64 + row), so that the apply kernels load one column of a tile,
  // one row per lane, as 64 consecutive elements; the transposed copy goes
  // through LDS so that both are written with consecutive addresses
  __shared__ C tl[NB][NB + 1];
  for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
    const int r = t % NB, c = t / NB;
    C v = src[c * NB + r];   // X(I*64 + r, J*64 + c)
    if (I == J && r > c) v = (C)0;
    tl[r][c] = v;
    xr[c * NB + r] = st_from<SX>((double)v);
  }
  __syncthreads();
  // X^T tile (J, I): element (row c, column r) = X(r, c), at r * 64 + c
  for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
    const int r = t / NB, c = t % NB;
    xc[t] = st_from<SX>((double)tl[r][c]);
  }
}

template <typename C>
static hipError_t invert_t(int N, int storage, const void *Rt, const double *dinv64, C *W, C *Y,
                           int xstorage, void *XR, void *XC, hipStream_t st) {
  const int T = N * (N + 1) / 2;
  switch (storage) {
    case TLS_FP64: TLS_LAUNCH(PC_PACK, (k_inv_init<double, C>), dim3(T), dim3(256), 0, st, N, (const double *)Rt, dinv64, W); break;
    case TLS_FP32: TLS_LAUNCH(PC_PACK, (k_inv_init<float, C>), dim3(T), dim3(256), 0, st, N, (const float *)Rt, dinv64, W); break;
    case TLS_FP16: TLS_LAUNCH(PC_PACK, (k_inv_init<half_t, C>), dim3(T), dim3(256), 0, st, N, (const half_t *)Rt, dinv64, W); break;
    default: TLS_LAUNCH(PC_PACK, (k_inv_init<bf16_t, C>), dim3(T), dim3(256), 0, st, N, (const bf16_t *)Rt, dinv64, W); break;
  }
  for (int hb = 1; hb < N; hb *= 2) {
    const int pairs = (N + 2 * hb - 1) / (2 * hb);
    const dim3 g(pairs * hb * hb);
    TLS_LAUNCH(PC_INVERT, k_inv_phase1<C>, g, dim3(256), 0, st, N, hb, W, Y);
    TLS_LAUNCH(PC_INVERT, k_inv_phase2<C>, g, dim3(256), 0, st, N, hb, W, (const C *)Y);
  }
  switch (xstorage) {
    case TLS_FP64: TLS_LAUNCH(PC_PACK, (k_inv_pack<double, C>), dim3(T), dim3(256), 0, st, N, W, (double *)XR, (double *)XC); break;
    case TLS_FP32: TLS_LAUNCH(PC_PACK, (k_inv_pack<float, C>), dim3(T), dim3(256), 0, st, N, W, (float *)XR, (float *)XC); break;
    case TLS_FP16: TLS_LAUNCH(PC_PACK, (k_inv_pack<half_t, C>), dim3(T), dim3(256), 0, st, N, W, (half_t *)XR, (half_t *)XC); break;
    default: TLS_LAUNCH(PC_PACK, (k_inv_pack<bf16_t, C>), dim3(T), dim3(256), 0, st, N, W, (bf16_t *)XR, (bf16_t *)XC); break;
  }
  return hipGetLastError();
}

// W and Y in FP64 when X is stored in FP64, in FP32 otherwise
hipError_t launch_invert(int N, int storage, const void *Rt, const double *dinv64, void *W, void *Y,
                         int xstorage, void *XR, void *XC, hipStream_t st) {
  if (xstorage == TLS_FP64)
    return invert_t<double>(N, storage, Rt, dinv64, (double *)W, (double *)Y, xstorage, XR, XC, st);
  return invert_t<float>(N, storage, Rt, dinv64, (float *)W, (float *)Y, xstorage, XR, XC, st);
}

size_t invert_scratch_doubles(int N) {
  // Y of the largest level: pairs * hb^2 tiles
  size_t best = 0;
  for (int hb = 1; hb < N; hb *= 2) {
    const size_t pairs = (N + 2 * hb - 1) / (2 * hb);
    best = std::max(best, pairs * hb * hb);
  }
  return std::max<size_t>(best, 1) * NB * NB;
}

// ---------------------------------------------------------------------------
// application: out = X v (TRANS = 0) or X^T v (TRANS = 1), fused PCG modes
// grid (N, CH): workgroup (I, s) covers the tiles of output block I in chunk
// s; the last workgroup to finish a block reduces the chunk partials in
// chunk order and runs the epilogue.
// ---------------------------------------------------------------------------
template <typename SX, typename C>
struct XParams {
  const SX *X;          // XR (TRANS = 0) or XC (TRANS = 1)
  const C *dscale;      // 1/d, Np
  int N, Np, n, chunk;  // chunk: tiles per workgroup
  // apply
  const double *in;
  double *out;
  int ldi, ldo;
  // PCG state, [NR][Np]
  C *s, *pb0, *pb1, *q, *w;
  C *part;              // [(L+2)][3][NR][N]
  int *done, *neg;
  double *trace;
  const double *sigma2;
  int j, L, strict;
  // chunk reduction
  C *cpart;             // [N][CH][NR][64]
  int *cnt;             // [N]
  int *status;
  int clear_flags;      // XF0: clear done, neg (0) and trace (NaN) for the run
};

template <typename C>
__device__ inline C *xpart_ptr(C *part, int j, int kind, int r, int NR, int N) {
  return part + (((size_t)j * 3 + kind) * NR + r) * N;
}

template <typename C>
__device__ inline C xsum_parts(const C *p, int N) {
  const int lane = threadIdx.x & 63;
  C v = 0;
  for (int i = lane; i < N; i += 64) v += p[i];
  return wave_sum(v);
}

enum XMode { XA = 0, XF0 = 2, XB = 3, XF = 4 };   // XA: plain apply

// ROW = 0: grid (N, CH), XS waves; workgroup (I, s) takes chunk s of the
//          tiles of block row I (chunk_of tiles, every XS-th one per wave);
//          the chunk partials are reduced by the last workgroup of each block
//          (split over the chip; the default);
// ROW = 1: grid (N), XW waves per workgroup, each wave streams every XW-th
//          tile of the block row; no cross-workgroup reduction (holds about
//          N CUs: the gate's runs use it beside a solve).
constexpr int XW = 4;
constexpr int XS = 8;   // waves per workgroup of the split variant
template <typename SX, typename C, int NR, int MODE, int TRANS, int ROW>
__global__ __launch_bounds__(ROW ? 64 * XW : 64 * XS) void k_xapply(XParams<SX, C> P) {
  constexpr int NW = ROW ? XW : XS;
  __shared__ C s_v[NW][NR][NB];      // per-wave input block
  __shared__ C s_acc[NW][NR][NB];
  __shared__ C s_scal[NR][4];
  // s_live: step j-1 ran for this right-hand side (it is still iterating);
  // s_run: step j runs (eta_j != 0 and, forward, delta_j and alpha_j finite
  // and delta_j != 0)
  __shared__ int s_live[NR], s_run[NR], s_floor[NR], s_last, s_skip;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int N = P.N, Np = P.Np;
  const int I = blockIdx.x, sidx = ROW ? 0 : blockIdx.y, CH = ROW ? 1 : gridDim.y;
  if constexpr (MODE == XF0) {
    // the run's step flags and trace start cleared (no step of this launch
    // reads them; the steps that do come after it on the stream)
    if (P.clear_flags && I == 0 && sidx == 0) {
      const int L2 = P.L + 2;
      for (int t = threadIdx.x; t < L2 * NR; t += blockDim.x) { P.done[t] = 0; P.neg[t] = 0; }
      for (int t = threadIdx.x; t < NR * 4 * L2; t += blockDim.x) P.trace[t] = __longlong_as_double(0x7ff8000000000000ll);
    }
  }
  // pbuf of the current p (step j) and of the previous one
  C *p_cur = (P.j & 1) ? P.pb1 : P.pb0;
  C *p_old = (P.j & 1) ? P.pb0 : P.pb1;

  // ---- every global read that does not depend on another is issued first,
  // so that the whole prologue costs one memory round trip ------------------
  // (a) this wave's tile: one tile per wave (chunk <= 4); lane = tile row
  const int K_lo = TRANS ? 0 : I;               // input blocks feeding output block I
  const int K_hi = TRANS ? I + 1 : N;
  const int k_end = ROW ? K_hi : min(K_hi, K_lo + sidx * P.chunk + P.chunk);
  int K = K_lo + sidx * (ROW ? 0 : P.chunk) + w;
  bool has_tile = K < k_end;
  SX t[NB];
  C in_a[NR], in_b[NR], in_ds = (C)0;
  // tile K's row for this lane and the inputs of block K (combined with the
  // step scalars later)
  auto load_tile = [&](int Kt) {
    // column c of the tile is 64 consecutive elements: lane = row
    const SX *T = P.X + (TRANS ? xc_tile(I, Kt) : xr_tile(I, Kt, N)) * NB * NB + lane;
#pragma unroll
    for (int c = 0; c < NB; ++c) t[c] = T[(size_t)c * NB];
    const int row = Kt * NB + lane;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const size_t vi = (size_t)r * Np + row;
      in_a[r] = (C)0;
      in_b[r] = (C)0;
      if constexpr (MODE == XA || MODE == XF0) {
        in_a[r] = (row < P.n) ? (C)P.in[(size_t)r * P.ldi + row] : (C)0;
      } else if constexpr (MODE == XB) {
        if (P.j > 0) { in_a[r] = P.s[vi]; in_b[r] = p_old[vi]; }
        else in_a[r] = p_cur[vi];
      } else {
        in_a[r] = P.q[vi];
      }
    }
    if constexpr (TRANS) in_ds = P.dscale[row];
  };
#pragma unroll
  for (int r = 0; r < NR; ++r) { in_a[r] = (C)0; in_b[r] = (C)0; }
  if (has_tile) load_tile(K);
  // (c) the rows of output block I that the epilogue needs (wave 0)
  const int orow = I * NB + lane;
  C e_s[NR], e_p[NR], e_po[NR], e_q[NR], e_w[NR], e_ds = (C)0;
  if (w == 0) {
    if constexpr (!TRANS) e_ds = P.dscale[orow];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const size_t vi = (size_t)r * Np + orow;
      e_s[r] = e_p[r] = e_po[r] = e_q[r] = e_w[r] = (C)0;
      if constexpr (MODE == XB) {
        e_p[r] = p_cur[vi];
        if (P.j > 0) { e_s[r] = P.s[vi]; e_po[r] = p_old[vi]; }
      } else if constexpr (MODE == XF) {
        e_s[r] = P.s[vi]; e_p[r] = p_cur[vi]; e_q[r] = P.q[vi]; e_w[r] = P.w[vi];
      }
    }
  }
  // (d) convergence flags of the previous step and the step scalars
  //     (recomputed identically by every workgroup)
  if (tid == 0) {
    int all_done = 1;
    for (int r = 0; r < NR; ++r) {
      int d = 0;
      if constexpr (MODE == XB || MODE == XF) d = (P.j > 0) ? P.done[(P.j - 1) * NR + r] : 0;
      s_live[r] = !d;
      all_done &= d;
    }
    s_skip = all_done;
    if constexpr (MODE == XF) {
      if (all_done && I == 0 && sidx == 0)
        for (int r = 0; r < NR; ++r) P.done[P.j * NR + r] = 1;
    }
  }
  if constexpr (MODE == XB || MODE == XF) {
    if (w == 1) {
      for (int r = 0; r < NR; ++r) {
        // eta_j = 0, or eta_j <= u_p^2 eta_0 for j > 0, ends the loop before
        // step j (s_j = 0 in the working precision: omega_j already solves
        // the system, and at eta_j = 0 beta_j would be 0/0); a step whose
        // delta_j or alpha_j is zero or not finite does not run either, so
        // omega never takes a NaN
        const C eta = xsum_parts(xpart_ptr(P.part, P.j, 0, r, NR, N), N);
        const C eta0 = (P.j > 0) ? xsum_parts(xpart_ptr(P.part, 0, 0, r, NR, N), N) : eta;
        const bool at_floor = P.j > 0 && eta <= pcg_eta_floor<C>() * eta0;
        if constexpr (MODE == XB) {
          C beta = 0;
          if (P.j > 0) {
            const C eta_prev = xsum_parts(xpart_ptr(P.part, P.j - 1, 0, r, NR, N), N);
            if (eta_prev != (C)0) beta = eta / eta_prev;
          }
          if (lane == 0) {
            s_scal[r][0] = eta; s_scal[r][1] = beta;
            s_run[r] = (eta != (C)0) && !at_floor;
            s_floor[r] = at_floor;
          }
        } else {
          const C pp = xsum_parts(xpart_ptr(P.part, P.j, 1, r, NR, N), N);
          const C qq = xsum_parts(xpart_ptr(P.part, P.j, 2, r, NR, N), N);
          const C sig2 = (C)(*P.sigma2);
          const C delta = pp - sig2 * qq;
          const C alpha = eta / delta;
          if (lane == 0) {
            s_scal[r][0] = eta; s_scal[r][1] = delta; s_scal[r][2] = alpha; s_scal[r][3] = sig2;
            s_run[r] = (eta != (C)0) && !at_floor && (delta != (C)0) && isfinite(delta) && isfinite(alpha);
            s_floor[r] = at_floor;
          }
        }
      }
    }
  }
  __syncthreads();
  if (s_skip) return;   // uniform for the whole grid

  // ---- the tile product ----------------------------------------------------
  C acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0;
  bool first = true;
  while (has_tile) {
    if (!first) load_tile(K);   // later tiles of the row variant
    first = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      C v;
      if constexpr (MODE == XA) v = TRANS ? in_ds * in_a[r] : in_a[r];
      else if constexpr (MODE == XF0) v = in_ds * in_a[r];
      else if constexpr (MODE == XB) v = (P.j > 0) ? in_a[r] + s_scal[r][1] * in_b[r] : in_a[r];
      else v = in_ds * in_a[r];
      s_v[w][r][lane] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // a fresh accumulator per tile: the FP32 chains stay 64 terms long
    // however many tiles a wave streams
    C tacc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) tacc[r] = 0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const C tc = cvt<C>(t[c]);
#pragma unroll
      for (int r = 0; r < NR; ++r) tacc[r] += tc * s_v[w][r][c];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += tacc[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    K += NW;
    has_tile = K < k_end;
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) s_acc[w][r][lane] = acc[r];
  __syncthreads();

  // ---- reduction over the waves (and, split, over the chunk workgroups) ----
  C res[NR];
  if (CH == 1) {
    if (w == 0) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        C v = s_acc[0][r][lane];
#pragma unroll
        for (int q = 1; q < NW; ++q) v += s_acc[q][r][lane];
        res[r] = v;
      }
    }
  } else {
    C *mine = P.cpart + (((size_t)I * CH + sidx) * NR) * NB;
    if (w == 0) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        C v = s_acc[0][r][lane];
#pragma unroll
        for (int q = 1; q < NW; ++q) v += s_acc[q][r][lane];
        mine[r * NB + lane] = v;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    if (tid == 0) s_last = (atomicAdd(&P.cnt[I], 1) == CH - 1);
    __syncthreads();
    if (!s_last) return;
    if (w == 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const C *base = P.cpart + ((size_t)I * CH * NR) * NB;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        C v = 0;
        for (int c = 0; c < CH; ++c) v += base[((size_t)c * NR + r) * NB + lane];
        res[r] = v;
      }
      if (lane == 0) P.cnt[I] = 0;
    }
  }
  if (w != 0) return;

  // ---- epilogue (wave 0, lane = row of block I) --------------------------
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const C x = res[r];
    const size_t vi = (size_t)r * Np + orow;
    if constexpr (MODE == XA) {
      if (orow < P.n) P.out[(size_t)r * P.ldo + orow] = (double)(TRANS ? x : e_ds * x);
    } else if constexpr (MODE == XF0) {
      P.s[vi] = x;
      P.pb0[vi] = x;
      P.w[vi] = 0;
      const C ss = wave_sum(x * x);
      if (lane == 0) xpart_ptr(P.part, 0, 0, r, NR, N)[I] = ss;
    } else if constexpr (MODE == XB) {
      const C qv = e_ds * x;                          // q = D^{-1} X p
      C pv = e_p[r];
      if (P.j > 0) pv = e_s[r] + s_scal[r][1] * e_po[r];
      if (s_live[r] && s_run[r]) {
        P.q[vi] = qv;
        if (P.j > 0) p_cur[vi] = pv;
      }
      const C pp = wave_sum(pv * pv), qq = wave_sum(qv * qv);
      if (lane == 0) {
        xpart_ptr(P.part, P.j, 1, r, NR, N)[I] = pp;
        xpart_ptr(P.part, P.j, 2, r, NR, N)[I] = qq;
      }
    } else {   // XF: x = t = X^T D^{-1} q
      C sv = e_s[r];
      if (s_live[r] && s_run[r]) {
        P.w[vi] = e_w[r] + s_scal[r][2] * e_q[r];                 // omega_{j+1}
        sv = sv - s_scal[r][2] * (e_p[r] - s_scal[r][3] * x);     // s_{j+1}
        P.s[vi] = sv;
      }
      const C ss = wave_sum(sv * sv);
      if (lane == 0) xpart_ptr(P.part, P.j + 1, 0, r, NR, N)[I] = ss;
    }
  }
  // step bookkeeping: block 0's finishing workgroup
  if constexpr (MODE == XB || MODE == XF) {
    if (I == 0 && lane < NR) {
      const int r = lane, L2 = P.L + 2, j = P.j;
      double *tr = P.trace + (size_t)r * 4 * L2;
      if constexpr (MODE == XB) {
        if (s_live[r]) {
          tr[0 * L2 + j] = (double)s_scal[r][0];
          if (j > 0 && s_run[r]) tr[3 * L2 + j - 1] = (double)s_scal[r][1];
        }
      } else {
        const C delta = s_scal[r][1];
        const int was = (j > 0) ? P.done[(j - 1) * NR + r] : 0;
        int now = was;
        if (!was) {
          if (s_scal[r][0] != (C)0 && !s_floor[r]) tr[1 * L2 + j] = (double)delta;
          if (s_run[r]) tr[2 * L2 + j] = (double)s_scal[r][2];
          if (!s_run[r]) now = 1;
          if (s_run[r] && delta < (C)0) {
            P.neg[j * NR + r] = 1;
            if (P.strict) {
              now = 1;
              atomicExch(P.status, (int)TLS_ERR_INDEFINITE);
            }
          }
        }
        P.done[j * NR + r] = now;
      }
    }
  }
}

template <typename SX, typename C, int NR, int MODE, int TRANS>
static hipError_t xlaunch(const XParams<SX, C> &P, int CH, hipStream_t st) {
  if (CH == 0)   // one workgroup per block row
    TLS_LAUNCH(MODE == XA ? PC_TRSV_APPLY : PC_PCG, (k_xapply<SX, C, NR, MODE, TRANS, 1>),
               dim3(P.N), dim3(64 * XW), 0, st, P);
  else
    TLS_LAUNCH(MODE == XA ? PC_TRSV_APPLY : PC_PCG, (k_xapply<SX, C, NR, MODE, TRANS, 0>),
               dim3(P.N, CH), dim3(64 * XS), 0, st, P);
  return hipGetLastError();
}

template <typename SX, typename C, int MODE, int TRANS>
static hipError_t x_nr(int nrhs, const XParams<SX, C> &P, int CH, hipStream_t st) {
  return nrhs == 1 ? xlaunch<SX, C, 1, MODE, TRANS>(P, CH, st) : xlaunch<SX, C, 2, MODE, TRANS>(P, CH, st);
}

template <typename SX, typename C>
static hipError_t x_mode(int mode, int trans, int nrhs, const XParams<SX, C> &P, int CH, hipStream_t st) {
  switch (mode) {
    case XA: return trans ? x_nr<SX, C, XA, 1>(nrhs, P, CH, st) : x_nr<SX, C, XA, 0>(nrhs, P, CH, st);
    case XF0: return x_nr<SX, C, XF0, 1>(nrhs, P, CH, st);
    case XB: return x_nr<SX, C, XB, 0>(nrhs, P, CH, st);
    default: return x_nr<SX, C, XF, 1>(nrhs, P, CH, st);
  }
}

// tiles per workgroup: one tile per wave, so that a block row of N tiles is
// spread over N/4 workgroups (the chip has 256 CUs; a single CU streams far
// below its share of the memory bandwidth)
// tiles per workgroup of the split apply (one wave takes every XS-th tile of
// the chunk): the fixed cost of a workgroup (scalars, chunk partial,
// arrival count) is spread over more tiles as N grows, while each SIMD
// keeps two waves to overlap one tile's loads with another's products
static int chunk_of(int N) {
  if (N <= XS) return N;
  if (N <= 40) return XS;
  if (N <= 96) return 2 * XS;
  return 4 * XS;
}

template <typename C>
static hipError_t x_dispatch(const FactorView &F, int mode, int trans, int nrhs, const SolveBufs &B,
                             hipStream_t st) {
  auto go = [&](auto *X) {
    using SX = std::remove_const_t<std::remove_pointer_t<decltype(X)>>;
    XParams<SX, C> P{};
    P.X = X;
    P.dscale = (const C *)(std::is_same<C, double>::value ? (const void *)F.dscale64 : (const void *)F.dscale32);
    P.N = F.N;
    P.Np = F.Np;
    P.n = F.n;
    P.chunk = chunk_of(F.N);
    P.in = B.in;
    P.out = B.out;
    P.ldi = B.ldi ? B.ldi : F.n;
    P.ldo = B.ldo ? B.ldo : F.n;
    P.s = (C *)B.s;
    P.pb0 = (C *)B.p;
    P.pb1 = (C *)B.chain;    // the substitution chain buffer doubles as the second p buffer
    P.q = (C *)B.q;
    P.w = (C *)B.w;
    P.part = (C *)B.part;
    P.done = B.done;
    P.neg = B.neg;
    P.trace = B.trace;
    P.sigma2 = B.sigma2;
    P.j = B.j;
    P.L = B.L;
    P.strict = B.strict;
    P.cpart = (C *)B.cpart;
    P.cnt = B.cnt;
    P.status = B.sync + F.N + 3;
    P.clear_flags = B.clear_flags;
    const int CH = F.xrow ? 0 : (F.N + P.chunk - 1) / P.chunk;
    return x_mode<SX, C>(mode, trans, nrhs, P, CH, st);
  };
  const void *X = trans ? F.xc : F.xr;
  switch (F.xstorage) {
    case TLS_FP64: return go((const double *)X);
    case TLS_FP32: return go((const float *)X);
    case TLS_FP16: return go((const half_t *)X);
    default: return go((const bf16_t *)X);
  }
}

// mode: 0 apply R^{-1} (X, D^{-1} after), 1 apply R^{-T} (D^{-1} before, X^T),
// 2 PCG init, 3 PCG backward, 4 PCG forward (same numbering as launch_trsv)
hipError_t launch_xapply(const FactorView &F, int compute, int mode, int nrhs, const SolveBufs &B,
                         hipStream_t st) {
  int m = XA, trans = 0;
  switch (mode) {
    case 0: m = XA; trans = 0; break;
    case 1: m = XA; trans = 1; break;
    case 2: m = XF0; trans = 1; break;
    case 3: m = XB; trans = 0; break;
    default: m = XF; trans = 1; break;
  }
  if (compute == TLS_FP64) return x_dispatch<double>(F, m, trans, nrhs, B, st);
  return x_dispatch<float>(F, m, trans, nrhs, B, st);
}

size_t xapply_chunk_count(int N) { return (N + chunk_of(N) - 1) / chunk_of(N); }

}  // namespace tls
