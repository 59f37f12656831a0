// Householder QR of the scaled, u_q-rounded A: the QR variant of the
// preconditioner (Section 3: the R-factor of A = Q [R; 0] computed in u_q;
// Section 3.1: constraint (5), u_q <~ kappa(A)^{-1}). Only R is produced;
// Q is never formed.
//
// Working matrix W: row-major, m_pad x Np (leading dimension Np), in the
// compute precision (FP64 for an FP64 factor, FP32 otherwise, every entry
// rounded to u_q when it is stored; products accumulate in FP32). m_pad = m + (Np - n): rows m..m_pad-1 hold e_j for
// the padding columns j = n..Np-1, so that R(W) = [R(A D^{-1}) 0; 0 I].
//
// Panels of NB = 64 columns are reduced one after another. Panel p works on
// rows [c0, m_pad), c0 = 64 p, cut into 64-row blocks, with a reduction tree
// of fan-in QR_FAN = 4:
//  - level 1: a slab of 4 consecutive blocks (256 rows) is factored by one
//    workgroup, four threads per row, reflector by reflector; its 64 x 64
//    triangle stays in the slab's first 64 rows and the reflectors
//    (unit lower trapezoidal Y) are stored below it in the panel columns;
//  - level l > 1: a slab stacks the triangles of 4 slabs of level l - 1
//    (their first 64 rows, read as upper triangles); the last level has one
//    slab, whose triangle lands in rows c0..c0+63.
// After the reflectors of a level are formed, they are applied to the
// panel's trailing columns in compact WY form, C <- C - Y T^T (Y^T C), with
// T the 64 x 64 upper triangular factor of H_0 ... H_63 = I - Y T Y^T. Row
// order does not change R (R^T R = A^T A), so the rows a level leaves
// behind stay in place and take part in the next panel; rows c0..c0+63
// hold rows c0..c0+63 of R when panel p is done.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tls {

namespace {

constexpr int QR_S = 256;             // rows of a slab
constexpr int QR_FAN = QR_S / NB;     // blocks (or child triangles) per slab
constexpr int LDP = NB + 1;           // padded LDS row

typedef float qr_f32x16 __attribute__((ext_vector_type(16)));
typedef double qr_f64x4 __attribute__((ext_vector_type(4)));

// global row of local row q of slab g at the level whose units are lpow
// blocks apart (lpow = QR_FAN^(level-1))
__device__ inline int64_t qr_row(int64_t c0, int64_t lpow, int g, int q) {
  const int64_t u = ((int64_t)g * QR_FAN + (q >> 6)) * lpow;
  return c0 + (int64_t)NB * u + (q & 63);
}

// round a stored value to u_q (FP16 / BF16 modes; FP32 and FP64 store as is)
__device__ inline float store_q(float x, int uq) {
  if (uq == TLS_FP16) return (float)(_Float16)x;       // IEEE RNE, overflow to Inf
  if (uq == TLS_BF16) {
    const uint32_t b = __builtin_bit_cast(uint32_t, x);
    if ((b & 0x7f800000u) == 0x7f800000u) return x;    // Inf, NaN
    const uint32_t r = (b + 0x7fffu + ((b >> 16) & 1u)) & 0xffff0000u;   // ties to even
    return __builtin_bit_cast(float, r);
  }
  return x;
}
__device__ inline double store_q(double x, int) { return x; }

// ---------------------------------------------------------------------------
// building W
// ---------------------------------------------------------------------------
template <typename C>
__global__ void k_qr_csr(int64_t m, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                         const double *d, int scaled, int uq, C *W, int64_t ld) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    const int j = col_idx[e];
    W[i * ld + j] = (C)quantize(scaled ? val[e] / d[j] : val[e], uq);
  }
}

// column-major A (ldA) to row-major W through a 64 x 64 LDS tile
template <typename C>
__global__ __launch_bounds__(256) void k_qr_dense(int64_t m, int n, int64_t ldA, const double *A,
                                                  const double *d, int scaled, int uq, C *W, int64_t ld) {
  __shared__ double t[NB][LDP];
  const int64_t i0 = (int64_t)blockIdx.x * NB;
  const int j0 = blockIdx.y * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e % NB, c = e / NB;
    const int64_t i = i0 + r;
    const int j = j0 + c;
    double v = 0.0;
    if (i < m && j < n) v = quantize(scaled ? A[i + (int64_t)j * ldA] / d[j] : A[i + (int64_t)j * ldA], uq);
    t[r][c] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int c = e % NB, r = e / NB;
    if (i0 + r < m) W[(i0 + r) * ld + j0 + c] = (C)t[r][c];
  }
}

// rows m..m_pad-1: e_{n+r}
template <typename C>
__global__ void k_qr_pad(int64_t m, int n, int Np, C *W, int64_t ld) {
  const int r = blockIdx.x;
  for (int j = threadIdx.x; j < Np; j += blockDim.x) W[(m + r) * ld + j] = (j == n + r) ? (C)1 : (C)0;
}

// ---------------------------------------------------------------------------
// local Householder QR of one slab (256 x 64 panel part)
// ---------------------------------------------------------------------------
// Four threads share a row: lane = 4 r + g of a wave holds row 16 w + r of
// the slab (w = wave) and its columns 16 g .. 16 g + 15 in registers. For
// reflector j: the norm of column j below the diagonal (block sum),
// beta_j = -sign(alpha) ||x||, v = x / (alpha - beta) with v(j) = 1,
// tau_j = (beta - alpha) / beta (no reflection when the column is already
// zero below the diagonal); the owner of column j passes v to the other
// three lanes of its row. One reduction over the slab of v_q a_q(c) for all
// 64 columns c (a transposing butterfly over the 16 rows of a wave, then the
// 16 waves through LDS) gives both w_c = v^T a(:, c) for the trailing
// columns c > j and (Y^T Y)(c, j) for the reflectors c < j (their entries
// sit below the diagonal in the same registers). Columns c > j are updated
// with a(:, c) -= tau_j v w_c. T is formed at the end from tau and Y^T Y by
// recursive doubling: T = [T1, -T1 (Y1^T Y2) T2; 0, T2].
constexpr int QR_LT = 4 * QR_S;                 // threads of the local kernel
constexpr int QR_LW = QR_LT / 64;               // its waves
template <typename C>
__global__ __launch_bounds__(QR_LT) void k_qr_local(C *W, int64_t ld, int64_t mpad, int64_t c0, int64_t lpow,
                                                    int upper_only, C *Tbuf, int uq) {
  constexpr int CG = NB / 4;                    // columns per lane
  __shared__ C red[2][QR_LW];
  __shared__ C alpha_s[2];
  __shared__ C part[2][QR_LW][NB];
  __shared__ C wsum[2][NB];
  __shared__ C Zs[NB][LDP];
  __shared__ C Ts[NB][LDP];
  __shared__ C Ms[NB][LDP];
  __shared__ C tau_s[NB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g = lane & 3, q = wv * 16 + (lane >> 2);      // column group, slab row
  const int g0 = g * CG;
  const int64_t row = qr_row(c0, lpow, blockIdx.x, q);
  const bool valid = row < mpad;
  const int t = q & 63;
  C a[CG];
  {
    const C *src = W + row * ld + c0 + g0;
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      C v = valid ? src[c] : (C)0;
      if (upper_only && t > g0 + c) v = (C)0;
      a[c] = v;
    }
  }
#pragma unroll 1
  for (int j = 0; j < NB; ++j) {
    const int buf = j & 1, gj = j / CG, cj = j % CG;
    const bool owner = (g == gj);
    C xs = (C)0;
#pragma unroll
    for (int c = 0; c < CG; ++c) xs = (c == cj) ? a[c] : xs;
    const C x = owner ? xs : (C)0;
    C s = wave_sum((q > j) ? x * x : (C)0);
    if (lane == 0) red[buf][wv] = s;
    if (owner && q == j) alpha_s[buf] = x;
    __syncthreads();
    s = red[buf][0];
#pragma unroll
    for (int w = 1; w < QR_LW; ++w) s += red[buf][w];
    const C alpha = alpha_s[buf];
    C beta = alpha, tau = (C)0, scl = (C)0;
    if (s > (C)0) {
      const C nrm = sqrt(alpha * alpha + s);
      beta = (alpha >= (C)0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scl = (C)1 / (alpha - beta);
    }
    const C vown = (q > j) ? x * scl : ((q == j) ? (C)1 : (C)0);
    const C v = __shfl(vown, (lane & ~3) | gj, 64);
    // p[c] = v_q a_q(g0 + c), summed over the wave's 16 rows by a
    // transposing butterfly: afterwards lane 4 r + g holds the sum for
    // column g0 + r
    C p[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) p[c] = v * a[c];
#define QR_BFLY(H, M)                                                \
  {                                                                  \
    const bool hi = (lane & (M)) != 0;                               \
    _Pragma("unroll") for (int i = 0; i < (H); ++i) {                \
      const C mine = hi ? p[(H) + i] : p[i];                         \
      const C other = hi ? p[i] : p[(H) + i];                        \
      p[i] = mine + __shfl_xor(other, (M), 64);                      \
    }                                                                \
  }
    QR_BFLY(8, 32) QR_BFLY(4, 16) QR_BFLY(2, 8) QR_BFLY(1, 4)
#undef QR_BFLY
    part[buf][wv][g0 + (lane >> 2)] = p[0];
    __syncthreads();
    if (tid < NB) {
      C w = part[buf][0][tid];
#pragma unroll
      for (int k = 1; k < QR_LW; ++k) w += part[buf][k][tid];
      wsum[buf][tid] = (tid > j) ? w : (C)0;    // zero where no update applies
      if (tid < j) Zs[tid][j] = w;
    }
    if (tid == 0) tau_s[j] = tau;
    __syncthreads();
    C ws[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) ws[c] = wsum[buf][g0 + c];
    const C tv = tau * v;
    const C keep = (q >= j) ? ((q == j) ? beta : v) : xs;   // new entry of column j (owner lanes)
#pragma unroll
    for (int c = 0; c < CG; ++c) a[c] -= tv * ws[c];
#pragma unroll
    for (int c = 0; c < CG; ++c) a[c] = (owner && c == cj) ? keep : a[c];
  }
  // the slab's triangle and reflectors, rounded to u_q
  if (valid) {
    C *dst = W + row * ld + c0 + g0;
#pragma unroll
    for (int c = 0; c < CG; ++c) dst[c] = store_q(a[c], uq);
  }
  // T by recursive doubling over blocks of b = 1, 2, 4, ..., 32 reflectors
  for (int e = tid; e < NB * NB; e += QR_LT) {
    const int r = e / NB, c = e % NB;
    Ts[r][c] = (r == c) ? tau_s[r] : (C)0;
  }
  for (int b = 1; b < NB; b <<= 1) {
    __syncthreads();
    const int per = b * b, total = (NB / (2 * b)) * per;
    for (int e = tid; e < total; e += QR_LT) {       // M = (Y1^T Y2) T2
      const int pr = e / per, r = (e % per) / b, cc = e % b, o = 2 * b * pr;
      C acc = (C)0;
      for (int k = 0; k <= cc; ++k) acc += Zs[o + r][o + b + k] * Ts[o + b + k][o + b + cc];
      Ms[o + r][o + b + cc] = acc;
    }
    __syncthreads();
    for (int e = tid; e < total; e += QR_LT) {       // T12 = -T1 M
      const int pr = e / per, r = (e % per) / b, cc = e % b, o = 2 * b * pr;
      C acc = (C)0;
      for (int k = r; k < b; ++k) acc += Ts[o + r][o + k] * Ms[o + k][o + b + cc];
      Ts[o + r][o + b + cc] = -acc;
    }
  }
  __syncthreads();
  C *T = Tbuf + (size_t)blockIdx.x * NB * NB;
  for (int e = tid; e < NB * NB; e += QR_LT) T[e] = Ts[e / NB][e % NB];
}

// ---------------------------------------------------------------------------
// compact-WY application to one 64-column tile of the trailing columns
// ---------------------------------------------------------------------------
// Three 64 x 64 LDS tiles: phase 1 Z = Y^T C over the slab's four 64-row
// chunks (Y chunk in B0, C chunk in B1); phase 2 Zt = T^T Z (T in B0, Z in
// B1, result into B2); phase 3 C -= Y Zt chunk by chunk (Y chunk back in
// B0). Only the updated entries of W are rounded to u_q: T and Zt are
// block intermediates and stay in the accumulation precision, as the
// column-by-column algorithm rounds only what it stores. Four waves each own a 32 x 32 quadrant of every
// 64 x 64 product; the C values stay in registers in the product layout.
template <typename C>
struct QrTile;

template <>
struct QrTile<float> {   // v_mfma_f32_32x32x2f32: one 32 x 32 block per wave
  qr_f32x16 acc;
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
  }
  // acc += sum_k A[k][i] B[k][j]   (both operands k-major)
  __device__ void kk(const float (*A)[LDP], const float (*B)[LDP], int wr, int wc, int lane) {
#pragma unroll 8
    for (int k0 = 0; k0 < NB; k0 += 2) {
      const float a = A[k0 + (lane >> 5)][wr * 32 + (lane & 31)];
      const float b = B[k0 + (lane >> 5)][wc * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
  }
  // acc += sum_k A[i][k] B[k][j]   (A row-major)
  __device__ void rk(const float (*A)[LDP], const float (*B)[LDP], int wr, int wc, int lane) {
#pragma unroll 8
    for (int k0 = 0; k0 < NB; k0 += 2) {
      const float a = A[wr * 32 + (lane & 31)][k0 + (lane >> 5)];
      const float b = B[k0 + (lane >> 5)][wc * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
  }
  static constexpr int COUNT = 16;
  __device__ static int row(int r, int wr, int lane) { return wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
  __device__ static int col(int, int wc, int lane) { return wc * 32 + (lane & 31); }
  __device__ float get(int r) const { return acc[r]; }
};

template <>
struct QrTile<double> {  // v_mfma_f64_16x16x4f64: 2 x 2 blocks of 16 x 16 per wave
  qr_f64x4 acc[2][2];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = qr_f64x4{0.0, 0.0, 0.0, 0.0};
  }
  __device__ void kk(const double (*A)[LDP], const double (*B)[LDP], int wr, int wc, int lane) {
#pragma unroll 4
    for (int k0 = 0; k0 < NB; k0 += 4) {
      double a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = A[k0 + (lane >> 4)][wr * 32 + u * 16 + (lane & 15)];
        b[u] = B[k0 + (lane >> 4)][wc * 32 + u * 16 + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
  __device__ void rk(const double (*A)[LDP], const double (*B)[LDP], int wr, int wc, int lane) {
#pragma unroll 4
    for (int k0 = 0; k0 < NB; k0 += 4) {
      double a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = A[wr * 32 + u * 16 + (lane & 15)][k0 + (lane >> 4)];
        b[u] = B[k0 + (lane >> 4)][wc * 32 + u * 16 + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
  // register r = 8 x + 4 y + q of block (x, y): row 4 q + lane/16, column lane%16
  static constexpr int COUNT = 16;
  __device__ static int row(int r, int wr, int lane) { return wr * 32 + ((r >> 3) & 1) * 16 + 4 * (r & 3) + (lane >> 4); }
  __device__ static int col(int r, int wc, int lane) { return wc * 32 + ((r >> 2) & 1) * 16 + (lane & 15); }
  __device__ double get(int r) const { return acc[(r >> 3) & 1][(r >> 2) & 1][r & 3]; }
};

template <typename C>
__global__ __launch_bounds__(256) void k_qr_apply(C *W, int64_t ld, int64_t mpad, int64_t c0, int64_t lpow,
                                                  const C *Tbuf, int uq) {
  __shared__ C B0[NB][LDP];
  __shared__ C B1[NB][LDP];
  __shared__ C B2[NB][LDP];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int g = blockIdx.x;
  const int64_t cb = c0 + NB + (int64_t)blockIdx.y * NB;   // first column of the tile
  using Tile = QrTile<C>;
  constexpr int RC = Tile::COUNT;
  C creg[QR_FAN][RC];
  auto load_y = [&](int ch) {      // Y rows 64 ch .. 64 ch + 63 into B0 (row-major)
    for (int e = tid; e < NB * NB; e += 256) {
      const int tt = e / NB, c = e % NB, ql = ch * NB + tt;
      const int64_t row = qr_row(c0, lpow, g, ql);
      C v = (C)0;
      if (row < mpad) v = (ql > c) ? W[row * ld + c0 + c] : ((ql == c) ? (C)1 : (C)0);
      B0[tt][c] = v;
    }
  };
  Tile acc;
  acc.zero();
  // phase 1: Z = Y^T C
#pragma unroll
  for (int ch = 0; ch < QR_FAN; ++ch) {
    if (ch) __syncthreads();
    load_y(ch);
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int tt = Tile::row(r, wr, lane), c = Tile::col(r, wc, lane);
      const int64_t row = qr_row(c0, lpow, g, ch * NB + tt);
      const C v = (row < mpad) ? W[row * ld + cb + c] : (C)0;
      creg[ch][r] = v;
      B1[tt][c] = v;
    }
    __syncthreads();
    acc.kk(B0, B1, wr, wc, lane);
  }
  __syncthreads();
  // phase 2: Zt = T^T Z
#pragma unroll
  for (int r = 0; r < RC; ++r) B1[Tile::row(r, wr, lane)][Tile::col(r, wc, lane)] = acc.get(r);
  {
    const C *T = Tbuf + (size_t)g * NB * NB;
    for (int e = tid; e < NB * NB; e += 256) B0[e / NB][e % NB] = T[e];
  }
  __syncthreads();
  acc.zero();
  acc.kk(B0, B1, wr, wc, lane);
#pragma unroll
  for (int r = 0; r < RC; ++r) B2[Tile::row(r, wr, lane)][Tile::col(r, wc, lane)] = acc.get(r);
  // phase 3: C -= Y Zt
#pragma unroll
  for (int ch = 0; ch < QR_FAN; ++ch) {
    __syncthreads();
    load_y(ch);
    __syncthreads();
    acc.zero();
    acc.rk(B0, B2, wr, wc, lane);
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int tt = Tile::row(r, wr, lane), c = Tile::col(r, wc, lane);
      const int64_t row = qr_row(c0, lpow, g, ch * NB + tt);
      if (row < mpad) W[row * ld + cb + c] = store_q(creg[ch][r] - acc.get(r), uq);
    }
  }
}

// ---------------------------------------------------------------------------
// R into G (column-major Np x Np, upper triangle), rows given a nonnegative
// diagonal; a zero or non-finite pivot is reported in info (column + 1)
// ---------------------------------------------------------------------------
template <typename C>
__global__ __launch_bounds__(256) void k_qr_extract(const C *W, int64_t ld, int Np, C *G, int *info) {
  __shared__ C t[NB][LDP];
  __shared__ C sgn[NB];
  const int I = blockIdx.x, J = blockIdx.y;
  if (I > J) return;
  const int tid = threadIdx.x;
  if (tid < NB) {
    const C dg = W[(int64_t)(I * NB + tid) * ld + I * NB + tid];
    sgn[tid] = (dg < (C)0) ? (C)-1 : (C)1;
    if (I == J && !(fabs((double)dg) > 0.0 && fabs((double)dg) < INFINITY)) atomicMin(info, I * NB + tid + 1);
  }
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    t[r][c] = W[(int64_t)(I * NB + r) * ld + J * NB + c];
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e % NB, c = e / NB;
    const C v = (I < J || r <= c) ? sgn[r] * t[r][c] : (C)0;
    G[(size_t)(J * NB + c) * Np + I * NB + r] = v;
  }
}

template <typename C>
hipError_t qr_t(int64_t m, int n, int Np, int format, int64_t ldA, const double *val, const int32_t *row_ptr,
                const int32_t *col_idx, const double *d, int scaled, int uq, void *work, C *G, int *info,
                hipStream_t st) {
  const int N = Np / NB;
  const int64_t mpad = m + (Np - n);
  const int64_t ld = Np;
  C *W = (C *)work;
  C *T = (C *)((char *)work + qr_matrix_bytes(m, n));
  if (format == TLS_CSR) {
    const hipError_t e = launch_fill_i32((int *)W, 0, (size_t)m * Np * (sizeof(C) / 4), st);
    if (e != hipSuccess) return e;
    TLS_LAUNCH(PC_QR, k_qr_csr<C>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, row_ptr, col_idx,
               val, d, scaled, uq, W, ld);
  } else {
    TLS_LAUNCH(PC_QR, k_qr_dense<C>, dim3((unsigned)((m + NB - 1) / NB), N), dim3(256), 0, st, m, n, ldA, val,
               d, scaled, uq, W, ld);
  }
  if (Np > n) TLS_LAUNCH(PC_QR, k_qr_pad<C>, dim3(Np - n), dim3(256), 0, st, m, n, Np, W, ld);
  for (int p = 0; p < N; ++p) {
    const int64_t c0 = (int64_t)p * NB;
    int64_t units = (mpad - c0 + NB - 1) / NB, lpow = 1;
    for (int level = 1;; ++level) {
      const int64_t slabs = (units + QR_FAN - 1) / QR_FAN;
      TLS_LAUNCH(PC_QR, k_qr_local<C>, dim3((unsigned)slabs), dim3(QR_LT), 0, st, W, ld, mpad, c0, lpow,
                 level > 1 ? 1 : 0, T, uq);
      if (p + 1 < N)
        TLS_LAUNCH(PC_QR, k_qr_apply<C>, dim3((unsigned)slabs, N - p - 1), dim3(256), 0, st, W, ld, mpad, c0,
                   lpow, (const C *)T, uq);
      if (slabs == 1) break;
      units = slabs;
      lpow *= QR_FAN;
    }
  }
  TLS_LAUNCH(PC_QR, k_qr_extract<C>, dim3(N, N), dim3(256), 0, st, (const C *)W, ld, Np, G, info);
  return hipGetLastError();
}

}  // namespace

size_t qr_matrix_bytes(int64_t m, int n) {
  const int64_t Np = (n + NB - 1) / NB * NB;
  const int64_t mpad = m + (Np - n);
  return ((size_t)mpad * Np * 8 + 255) / 256 * 256;
}

size_t qr_work_bytes(int64_t m, int n) {
  const int64_t Np = (n + NB - 1) / NB * NB;
  const int64_t mpad = m + (Np - n);
  const int64_t slabs = ((mpad + NB - 1) / NB + QR_FAN - 1) / QR_FAN;
  return qr_matrix_bytes(m, n) + (size_t)slabs * NB * NB * 8;
}

hipError_t launch_qr_factor(int64_t m, int n, int Np, int format, int64_t ldA, const double *val,
                            const int32_t *row_ptr, const int32_t *col_idx, const double *d, int scaled, int uq,
                            int compute, void *work, void *G, int *info, hipStream_t st) {
  if (compute == TLS_FP64)
    return qr_t<double>(m, n, Np, format, ldA, val, row_ptr, col_idx, d, scaled, uq, work, (double *)G, info, st);
  return qr_t<float>(m, n, Np, format, ldA, val, row_ptr, col_idx, d, scaled, uq, work, (float *)G, info, st);
}

}  // namespace tls
