// Outer loop of RQI for TLS (Algorithm 2 / 4, precision u = FP64):
//   r_k = b - A x_k,  sigma_k^2 = r^T r / (1 + x^T x),
//   f_k = -A^T r_k - sigma_k^2 x_k,  g_k = -b^T r_k + sigma_k^2,
//   psi_k = ((||f||^2 + g^2) / (||x||^2 + 1))^{1/2}          (eq. 4)
//   z = x + omega,  beta = (z^T f - g) / (z^T x + 1),  x <- z + beta u.
// The two passes over A (r = b - A x, then A^T r) stream A once each; the
// inner products are fused into them as per-block partial sums that the
// single-workgroup scalar kernels add in a fixed order.
//
// Scalar block `scal` (device, doubles):
//   0 sigma^2   1 shift mu   2 ||x||^2   3 r^T r   4 b^T r   5 g (at mu)
//   6 ||f||^2 (at mu)   7 psi   8 best psi   9 is-best flag   10 z^T f
//   11 z^T x   12 beta   13 f^T x   14 shift cap   15 iteration count
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tls {

enum { S_SIG2 = 0, S_MU, S_XX, S_RR, S_BR, S_G, S_FF, S_PSI, S_BEST, S_ISBEST, S_ZF, S_ZX,
       S_BETA, S_FX, S_CAP, S_K, S_STEPS, S_SHIFT0 };

constexpr int RES_ROWS = 256;   // rows per workgroup of the CSR residual pass
// dense row products: 64 rows per workgroup, the columns split over 16 waves
// (interleaved chunks of 8), partials joined in a fixed order through LDS
constexpr int RD_ROWS = 64, RD_WAVES = 16, RD_CHUNK = 8;

int matvec_blocks(const MatView &A) {
  const int rows = A.format == TLS_DENSE_COLMAJOR ? RD_ROWS : RES_ROWS;
  return (A.m + rows - 1) / rows;
}

// this wave's share of row i of A x: columns 8 (w + 16 t) + q, q < 8
__device__ inline double dense_row_part(int n, int64_t ld, const double *a, const double *x, int w) {
  double c[RD_CHUNK] = {0, 0, 0, 0, 0, 0, 0, 0};
  int j = RD_CHUNK * w;
  for (; j + RD_CHUNK <= n; j += RD_CHUNK * RD_WAVES) {
#pragma unroll
    for (int q = 0; q < RD_CHUNK; ++q) c[q] += __builtin_nontemporal_load(a + (size_t)(j + q) * ld) * x[j + q];
  }
#pragma unroll
  for (int q = 0; q < RD_CHUNK; ++q)
    if (j + q < n) c[q] += a[(size_t)(j + q) * ld] * x[j + q];
  return ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
}
// the 16 wave partials of the workgroup's 64 rows, summed in wave order;
// valid in wave 0 (lane = row), every thread passes the barrier
__device__ inline double dense_row_join(double v, double (*red)[RD_ROWS]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  red[w][lane] = v;
  __syncthreads();
  double s = 0;
  if (w == 0) {
    s = red[0][lane];
#pragma unroll
    for (int q = 1; q < RD_WAVES; ++q) s += red[q][lane];
  }
  return s;
}
int rmatvec_blocks(const MatView &A) { return (A.n + 3) / 4; }

// ---------------------------------------------------------------------------
// r = b - A x with partials of r.r and b.r
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_residual_dense(int m, int n, int64_t ld, const double *A,
                                                         const double *b, const double *x,
                                                         double *r, double *part) {
  __shared__ double red[RD_WAVES][RD_ROWS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * RD_ROWS + lane;
  const double p = i < m ? dense_row_part(n, ld, A + i, x, w) : 0.0;
  const double ax = dense_row_join(p, red);
  if (w != 0) return;
  double rv = 0, bv = 0;
  if (i < m) {
    bv = b[i];
    rv = bv - ax;
    r[i] = rv;
  }
  const double rr = wave_sum(rv * rv);
  const double br = wave_sum(bv * rv);
  if (lane == 0) { part[2 * blockIdx.x] = rr; part[2 * blockIdx.x + 1] = br; }
}

// CSR: RES_ROWS rows per workgroup, RES_LANES lanes per row (a row's
// entries taken RES_LANES at a time, then joined across its lanes in a
// fixed order), so that each lane's chain of dependent loads is a quarter
// of the row
constexpr int RES_LANES = 4;
__global__ __launch_bounds__(RES_ROWS * RES_LANES) void k_residual_csr(int m, const int32_t *row_ptr,
                                                                       const int32_t *col_idx, const double *val,
                                                                       const double *b, const double *x, double *r,
                                                                       double *part) {
  __shared__ double s_rr[RES_ROWS * RES_LANES / 64], s_br[RES_ROWS * RES_LANES / 64];
  const int t = threadIdx.x, sub = t % RES_LANES;
  const int i = blockIdx.x * RES_ROWS + t / RES_LANES;
  double acc = 0.0;
  if (i < m) {
    for (int e = row_ptr[i] + sub; e < row_ptr[i + 1]; e += RES_LANES) acc += val[e] * x[col_idx[e]];
  }
#pragma unroll
  for (int off = 1; off < RES_LANES; off <<= 1) acc += __shfl_xor(acc, off, 64);
  double rv = 0, bv = 0;
  if (i < m && sub == 0) {
    bv = b[i];
    rv = bv - acc;
    r[i] = rv;
  }
  const double rr = wave_sum(rv * rv), br = wave_sum(bv * rv);
  if ((t & 63) == 0) { s_rr[t >> 6] = rr; s_br[t >> 6] = br; }
  __syncthreads();
  if (t == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int q = 0; q < RES_ROWS * RES_LANES / 64; ++q) { a0 += s_rr[q]; a1 += s_br[q]; }
    part[2 * blockIdx.x] = a0;
    part[2 * blockIdx.x + 1] = a1;
  }
}

// ---------------------------------------------------------------------------
// One pass over the row-major copy of a dense A: r = b - A x and A^T r
// ---------------------------------------------------------------------------
// Algorithm 2 forms r_k = b - A x_k and then f_k = -A^T r_k - sigma_k^2 x_k.
// A^T r = sum_i a_i r_i, and r_i needs row a_i alone, so a pass that holds
// row a_i once can form r_i and add a_i r_i to a running A^T r: one read of A
// per outer step instead of two. A wave owns a row at a time (lane l holds
// columns l + 64 t, 64 t < ldr); x and the wave's share of A^T r stay in its
// registers. A workgroup of RR_WAVES waves takes `groups` consecutive 64-row
// groups (wave w: rows 8w..8w+7 of each group), joins its waves' A^T r in
// wave order through LDS and writes one partial n-vector; per 64-row group it
// writes (r^T r, b^T r) in the layout of k_residual_dense (the same number of
// partials, ceil(m / 64)). b == nullptr means b = 0 (r = -A x), x ==
// nullptr means x = 0 (r = b): the pass then gives -A^T A x or A^T b.
constexpr int RR_WAVES = 4, RR_MAXG = 64, RR_RPW = 64 / RR_WAVES;

template <typename T> struct RowLoad;
template <> struct RowLoad<double> { using type = double; static constexpr int N = 1; };
__device__ inline double vget(double v, int) { return v; }

// TT: columns per lane (the row stride ldr is 64 TT, padded with zeros).
// Lane l reads VN elements at a time: columns 64 VN s + VN l + v (v < VN) of
// load s, so that one load instruction of a wave moves 64 VN contiguous
// elements of the row. VN = 1 (8-byte loads, 512 bytes per instruction):
// on the 65536 x 4096 copy the pass takes 317 us against 334 us with
// 16-byte loads (a timing probe of the kernel alone).
// DUAL: the same pass also forms A^T A v for a second vector v (a Lanczos
// step of the factor's certificate rides on the outer step's read of A, or
// the first RQI step's u_0): t_i = a_i . v beside r_i (written to t_out when
// given), and a_i t_i summed into a second partial n-vector per workgroup
// (ppart2), joined in the same fixed order.
template <int TT, typename T, bool DUAL>
__global__ __launch_bounds__(RR_WAVES * 64) void k_resgrad_rows(int m, int n, int64_t ldr, const T *At,
                                                                const double *b, const double *x, double *r,
                                                                double *part_r, int groups, double *ppart,
                                                                const double *v2, double *ppart2,
                                                                double *t_out) {
  using V = typename RowLoad<T>::type;
  constexpr int VN = RowLoad<T>::N, NS = TT / VN;     // elements per load, loads per row
  __shared__ double sx[TT * 64], sp[TT * 64], sv[DUAL ? TT * 64 : 1];
  __shared__ double srr[RR_WAVES][RR_MAXG], sbr[RR_WAVES][RR_MAXG];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = threadIdx.x; j < TT * 64; j += RR_WAVES * 64) {
    sx[j] = (x && j < n) ? x[j] : 0.0;
    if (DUAL) sv[j] = j < n ? v2[j] : 0.0;
  }
  __syncthreads();
  double pr[TT], pq[DUAL ? TT : 1];
#pragma unroll
  for (int t = 0; t < TT; ++t) pr[t] = 0.0;
  if (DUAL) {
#pragma unroll
    for (int t = 0; t < TT; ++t) pq[t] = 0.0;
  }
  const int g0 = blockIdx.x * groups;
  for (int q = 0; q < groups; ++q) {
    double rr = 0.0, br = 0.0;
    for (int k = 0; k < RR_RPW; ++k) {
      const int i = (g0 + q) * 64 + RR_RPW * w + k;
      if (i >= m) break;
      const V *row = (const V *)(At + (size_t)i * ldr) + lane;
      V a[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) a[s] = __builtin_nontemporal_load(row + 64 * s);
      double dot = 0.0, dot2 = 0.0;
      if (x) {
        double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int v = 0; v < VN; ++v) c[(s * VN + v) & 3] += vget(a[s], v) * sx[64 * VN * s + VN * lane + v];
        dot = wave_sum((c[0] + c[1]) + (c[2] + c[3]));
      }
      if (DUAL) {
        double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int v = 0; v < VN; ++v) c[(s * VN + v) & 3] += vget(a[s], v) * sv[64 * VN * s + VN * lane + v];
        dot2 = wave_sum((c[0] + c[1]) + (c[2] + c[3]));
      }
      const double bi = b ? b[i] : 0.0;
      const double ri = bi - dot;
      if (r && lane == 0) r[i] = ri;
      if (DUAL && t_out && lane == 0) t_out[i] = dot2;
      rr += ri * ri;
      br += bi * ri;
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int v = 0; v < VN; ++v) pr[s * VN + v] += vget(a[s], v) * ri;
      if (DUAL) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int v = 0; v < VN; ++v) pq[s * VN + v] += vget(a[s], v) * dot2;
      }
    }
    if (lane == 0) { srr[w][q] = rr; sbr[w][q] = br; }
  }
  // the waves' A^T r (then A^T A v) joined in wave order
  for (int pass = 0; pass < (DUAL ? 2 : 1); ++pass) {
    for (int q = 0; q < RR_WAVES; ++q) {
      if (w == q) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int v = 0; v < VN; ++v) {
            const int c = 64 * VN * s + VN * lane + v;
            const double val = (DUAL && pass == 1) ? pq[s * VN + v] : pr[s * VN + v];
            sp[c] = (q == 0) ? val : sp[c] + val;
          }
      }
      __syncthreads();
    }
    double *dst = (pass == 0 ? ppart : ppart2) + (size_t)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += RR_WAVES * 64) dst[j] = sp[j];
    __syncthreads();   // sp is reused by the second join
  }
  if (part_r) {
    for (int q = threadIdx.x; q < groups; q += RR_WAVES * 64) {
      const int gq = g0 + q;
      if (gq * 64 >= m) break;
      double rr = 0.0, br = 0.0;
      for (int v = 0; v < RR_WAVES; ++v) { rr += srr[v][q]; br += sbr[v][q]; }
      part_r[2 * gq] = rr;
      part_r[2 * gq + 1] = br;
    }
  }
}

// The DUAL pass over a 4096-column copy. One wave per row would hold the
// row (64 values per lane) and both accumulators (A^T r and A^T A v, 64
// each): more than a wave's 256 VGPRs, so the compiler parks values in AGPRs
// and the pass runs about 20 % slower than the plain one. Here two waves
// share a row, wave h of a pair holding columns 2048 h + lane + 64 t
// (t < 32): 32 values and 2 x 32 accumulators per lane, two waves per SIMD.
// The pair's partial dot products meet in a double-buffered LDS slot, one
// barrier per row step (every wave runs the same number of steps, past the
// last row with zeros). Rows, partial layout and join order are those of
// k_resgrad_rows: pair p takes rows 16 p .. 16 p + 15 of each 64-row group.
constexpr int R2_WAVES = 8, R2_TH = 32;
__global__ __launch_bounds__(R2_WAVES * 64) void k_resgrad_rows_dual64(int m, int n, int64_t ldr, const double *At,
                                                                       const double *b, const double *x, double *r,
                                                                       double *part_r, int groups, double *ppart,
                                                                       const double *v2, double *ppart2,
                                                                       double *t_out) {
  __shared__ double sx[64 * 64], sv[64 * 64], sp[64 * 64];
  __shared__ double sd[2][RR_WAVES][2][2];   // [buffer][pair][half][x, v]
  __shared__ double srr[RR_WAVES][RR_MAXG], sbr[RR_WAVES][RR_MAXG];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, pair = w >> 1, h = w & 1;
  for (int j = threadIdx.x; j < 64 * 64; j += R2_WAVES * 64) {
    sx[j] = (x && j < n) ? x[j] : 0.0;
    sv[j] = j < n ? v2[j] : 0.0;
  }
  __syncthreads();
  const int c0 = 2048 * h + lane;          // this lane's first column
  double pr[R2_TH], pq[R2_TH];
#pragma unroll
  for (int t = 0; t < R2_TH; ++t) { pr[t] = 0.0; pq[t] = 0.0; }
  const int g0 = blockIdx.x * groups;
  int step = 0;
  for (int q = 0; q < groups; ++q) {
    double rr = 0.0, br = 0.0;
    for (int k = 0; k < RR_RPW; ++k, ++step) {
      const int i = (g0 + q) * 64 + RR_RPW * pair + k;
      const bool live = i < m;
      const double *row = At + (size_t)(live ? i : 0) * ldr + c0;
      double a[R2_TH];
#pragma unroll
      for (int t = 0; t < R2_TH; ++t) a[t] = live ? __builtin_nontemporal_load(row + 64 * t) : 0.0;
      double c[4] = {0.0, 0.0, 0.0, 0.0}, e[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < R2_TH; ++t) {
        c[t & 3] += a[t] * sx[c0 + 64 * t];
        e[t & 3] += a[t] * sv[c0 + 64 * t];
      }
      const double px = wave_sum((c[0] + c[1]) + (c[2] + c[3]));
      const double pv = wave_sum((e[0] + e[1]) + (e[2] + e[3]));
      const int buf = step & 1;
      if (lane == 0) { sd[buf][pair][h][0] = px; sd[buf][pair][h][1] = pv; }
      __syncthreads();
      // both waves of the pair add the halves in the same order
      const double dot = sd[buf][pair][0][0] + sd[buf][pair][1][0];
      const double dot2 = sd[buf][pair][0][1] + sd[buf][pair][1][1];
      if (live) {
        const double bi = b ? b[i] : 0.0;
        const double ri = bi - dot;
        if (h == 0) {
          if (lane == 0) {
            if (r) r[i] = ri;
            if (t_out) t_out[i] = dot2;
          }
          rr += ri * ri;
          br += bi * ri;
        }
#pragma unroll
        for (int t = 0; t < R2_TH; ++t) {
          pr[t] += a[t] * ri;
          pq[t] += a[t] * dot2;
        }
      }
    }
    if (h == 0 && lane == 0) { srr[pair][q] = rr; sbr[pair][q] = br; }
  }
  // the pairs' A^T r (then A^T A v) joined in pair order
  for (int pass = 0; pass < 2; ++pass) {
    for (int p = 0; p < RR_WAVES; ++p) {
      if (pair == p) {
#pragma unroll
        for (int t = 0; t < R2_TH; ++t) {
          const int col = c0 + 64 * t;
          const double val = pass ? pq[t] : pr[t];
          sp[col] = (p == 0) ? val : sp[col] + val;
        }
      }
      __syncthreads();
    }
    double *dst = (pass == 0 ? ppart : ppart2) + (size_t)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += R2_WAVES * 64) dst[j] = sp[j];
    __syncthreads();
  }
  if (part_r) {
    for (int q = threadIdx.x; q < groups; q += R2_WAVES * 64) {
      const int gq = g0 + q;
      if (gq * 64 >= m) break;
      double rr = 0.0, br = 0.0;
      for (int v = 0; v < RR_WAVES; ++v) { rr += srr[v][q]; br += sbr[v][q]; }
      part_r[2 * gq] = rr;
      part_r[2 * gq + 1] = br;
    }
  }
}

// 64-row groups per workgroup of the row pass: about one workgroup per CU
int rowpass_groups(int64_t m, int cus) {
  const int64_t ng = (m + 63) / 64;
  return (int)std::min<int64_t>(RR_MAXG, std::max<int64_t>(1, (ng + cus - 1) / cus));
}
int rowpass_blocks(int64_t m, int cus) {
  const int64_t ng = (m + 63) / 64;
  const int gpw = rowpass_groups(m, cus);
  return (int)((ng + gpw - 1) / gpw);
}
static int rowpass_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0, v = 0;
    cus = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  return cus;
}
int rowpass_partials(const MatView &A) { return rowpass_blocks(A.m, rowpass_cus()); }
int64_t rowpass_ld(int64_t n) {
  const int64_t t = (n + 63) / 64;
  return 64 * (t <= 16 ? 16 : t <= 32 ? 32 : t <= 48 ? 48 : 64);
}

template <typename T, bool DUAL>
static hipError_t rowpass_go(const MatView &A, const T *at, const double *b, const double *x, double *r,
                             double *part_r, double *ppart, const double *v2, double *ppart2, double *t_out,
                             hipStream_t st, int cls) {
  const int cus = rowpass_cus();
  const int groups = rowpass_groups(A.m, cus), blocks = rowpass_blocks(A.m, cus);
  const int nt = (int)(A.ldr >> 6);    // the copy's stride is 64 TT (rowpass_ld)
  const dim3 g(blocks), t(RR_WAVES * 64);
  switch (nt) {
    case 16:
      TLS_LAUNCH(cls, (k_resgrad_rows<16, T, DUAL>), g, t, 0, st, A.m, A.n, A.ldr, at, b, x, r, part_r, groups,
                 ppart, v2, ppart2, t_out);
      break;
    case 32:
      TLS_LAUNCH(cls, (k_resgrad_rows<32, T, DUAL>), g, t, 0, st, A.m, A.n, A.ldr, at, b, x, r, part_r, groups,
                 ppart, v2, ppart2, t_out);
      break;
    case 48:
      TLS_LAUNCH(cls, (k_resgrad_rows<48, T, DUAL>), g, t, 0, st, A.m, A.n, A.ldr, at, b, x, r, part_r, groups,
                 ppart, v2, ppart2, t_out);
      break;
    case 64:
      if constexpr (DUAL && std::is_same<T, double>::value) {
        TLS_LAUNCH(cls, k_resgrad_rows_dual64, g, dim3(R2_WAVES * 64), 0, st, A.m, A.n, A.ldr, at, b, x, r, part_r,
                   groups, ppart, v2, ppart2, t_out);
      } else {
        TLS_LAUNCH(cls, (k_resgrad_rows<64, T, DUAL>), g, t, 0, st, A.m, A.n, A.ldr, at, b, x, r, part_r, groups,
                   ppart, v2, ppart2, t_out);
      }
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_rowpass(const MatView &A, const double *b, const double *x, double *r, double *part_r,
                          double *ppart, hipStream_t st) {
  return rowpass_go<double, false>(A, A.at, b, x, r, part_r, ppart, nullptr, nullptr, nullptr, st, PC_RESIDUAL);
}
hipError_t launch_rowpass_dual(const MatView &A, const double *b, const double *x, double *r, double *part_r,
                               double *ppart, const double *v2, double *ppart2, hipStream_t st, double *t_out) {
  return rowpass_go<double, true>(A, A.at, b, x, r, part_r, ppart, v2, ppart2, t_out, st, PC_RESIDUAL);
}

// The sum of the row pass's G partial n-vectors for the 64 columns of one
// workgroup: wave w (lane = column) sums the w-th quarter of the partials
// with eight loads in flight, and the quarters are added in wave order
// (a fixed order: the result is the same on every call).
__device__ inline double partials_sum64(int n, int G, const double *ppart, int j, double *sq /* [4][64] */) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = (G + 3) / 4, g0 = w * q, g1 = min(G, g0 + q);
  double c[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (j < n) {
    int g = g0;
    for (; g + 8 <= g1; g += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) c[u] += ppart[(size_t)(g + u) * n + j];
    }
    for (; g < g1; ++g) c[0] += ppart[(size_t)g * n + j];
  }
  sq[w * 64 + lane] = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
  __syncthreads();
  return (sq[lane] + sq[64 + lane]) + (sq[128 + lane] + sq[192 + lane]);
}

// y = s * (sum of the row workgroups' partials), in a fixed order
__global__ __launch_bounds__(256) void k_rowpass_sum(int n, int G, const double *ppart, double s, double *y) {
  __shared__ double sq[256];
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const double v = partials_sum64(n, G, ppart, j, sq);
  if (threadIdx.x < 64 && j < n) y[j] = s * v;
}
hipError_t launch_rowpass_sum(const MatView &A, const double *ppart, double s, double *y, hipStream_t st) {
  TLS_LAUNCH(PC_GRADIENT, k_rowpass_sum, dim3((A.n + 63) / 64), dim3(256), 0, st, A.n, rowpass_partials(A),
             ppart, s, y);
  return hipGetLastError();
}

hipError_t launch_residual(const MatView &A, const double *b, const double *x, double *r,
                           double *part, hipStream_t st) {
  const dim3 g(matvec_blocks(A));
  if (A.format == TLS_DENSE_COLMAJOR)
    TLS_LAUNCH(PC_RESIDUAL, k_residual_dense, g, dim3(RD_ROWS * RD_WAVES), 0, st, A.m, A.n, A.ld, A.val, b,
               x, r, part);
  else
    TLS_LAUNCH(PC_RESIDUAL, k_residual_csr, g, dim3(RES_ROWS * RES_LANES), 0, st, A.m, A.row_ptr, A.col_idx, A.val, b, x,
                       r, part);
  return hipGetLastError();
}

// plain products (tests and x_LS): y = A x, y = A^T x
__global__ __launch_bounds__(1024) void k_matvec_dense(int m, int n, int64_t ld, const double *A,
                                                       const double *x, double *y) {
  __shared__ double red[RD_WAVES][RD_ROWS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * RD_ROWS + lane;
  const double p = i < m ? dense_row_part(n, ld, A + i, x, w) : 0.0;
  const double ax = dense_row_join(p, red);
  if (w == 0 && i < m) y[i] = ax;
}
// CSR: RES_LANES lanes per row, as in k_residual_csr
__global__ __launch_bounds__(RES_ROWS * RES_LANES) void k_matvec_csr(int m, const int32_t *row_ptr,
                                                                     const int32_t *col_idx, const double *val,
                                                                     const double *x, double *y) {
  const int t = threadIdx.x, sub = t % RES_LANES;
  const int i = blockIdx.x * RES_ROWS + t / RES_LANES;
  double acc = 0.0;
  if (i < m) {
    for (int e = row_ptr[i] + sub; e < row_ptr[i + 1]; e += RES_LANES) acc += val[e] * x[col_idx[e]];
  }
#pragma unroll
  for (int off = 1; off < RES_LANES; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (i < m && sub == 0) y[i] = acc;
}
// A^T x: one wave per column (dense) / per CSC column
__global__ void k_rmatvec_dense(int m, int n, int64_t ld, const double *A, const double *x, double *y) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= n) return;
  // as in k_gradient: eight 512-byte loads in flight, A streamed once
  const double *col = A + (size_t)j * ld;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = lane;
  for (; i + 448 < m; i += 512) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += __builtin_nontemporal_load(col + i + 64 * u) * x[i + 64 * u];
  }
  for (; i < m; i += 64) s[0] += col[i] * x[i];
  const double acc = wave_sum(((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
  if (lane == 0) y[j] = acc;
}
__global__ void k_rmatvec_csc(int n, const int32_t *col_ptr, const int32_t *row_idx,
                              const double *cval, const double *x, double *y) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= n) return;
  double acc = 0;
  for (int e = col_ptr[j] + lane; e < col_ptr[j + 1]; e += 64) acc += cval[e] * x[row_idx[e]];
  acc = wave_sum(acc);
  if (lane == 0) y[j] = acc;
}

hipError_t launch_matvec(const MatView &A, const double *x, double *y, hipStream_t st) {
  const dim3 g(matvec_blocks(A));
  if (A.format == TLS_DENSE_COLMAJOR)
    TLS_LAUNCH(PC_RESIDUAL, k_matvec_dense, g, dim3(RD_ROWS * RD_WAVES), 0, st, A.m, A.n, A.ld, A.val, x, y);
  else
    TLS_LAUNCH(PC_RESIDUAL, k_matvec_csr, g, dim3(RES_ROWS * RES_LANES), 0, st, A.m, A.row_ptr, A.col_idx, A.val,
               x, y);
  return hipGetLastError();
}
hipError_t launch_rmatvec(const MatView &A, const double *x, double *y, hipStream_t st) {
  const dim3 g((A.n + 3) / 4);
  if (A.format == TLS_DENSE_COLMAJOR)
    TLS_LAUNCH(PC_GRADIENT, k_rmatvec_dense, g, dim3(256), 0, st, A.m, A.n, A.ld, A.val, x, y);
  else
    TLS_LAUNCH(PC_GRADIENT, k_rmatvec_csc, g, dim3(256), 0, st, A.n, A.col_ptr, A.row_idx, A.cval, x, y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// f = -A^T r - mu x with partials of f.f and f.x (one wave per column)
// ---------------------------------------------------------------------------
__device__ inline double sum_pairs(const double *part, int nb, int which, double *sc);

// sigma^2 = rr / (1 + x^T x), the clamped shift mu and g = -b^T r + mu from the
// residual partials (every workgroup of the gradient computes the same values
// in the same order; workgroup 0 records them)
struct RqScalars { double sig2, mu, xx, br; };
__device__ inline RqScalars rq_scalars(int n, const double *x, const double *part_r, int nb_r,
                                       double *scal, double cap, double *sc) {
  double xx = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) xx += x[i] * x[i];
  xx = block_sum(xx, sc);
  const double rr = sum_pairs(part_r, nb_r, 0, sc + 4);
  const double br = sum_pairs(part_r, nb_r, 1, sc);
  const double sig2 = rr / (1.0 + xx);
  const double mu = (cap > 0 && sig2 > cap) ? cap : sig2;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[S_SIG2] = sig2;
    scal[S_MU] = mu;
    scal[S_XX] = xx;
    scal[S_RR] = rr;
    scal[S_BR] = br;
    scal[S_G] = -br + mu;
    scal[S_CAP] = cap;
  }
  return RqScalars{sig2, mu, xx, br};
}

template <bool CSC>
__global__ __launch_bounds__(256) void k_gradient(int m, int n, int64_t ld, const double *A,
                                                  const int32_t *col_ptr, const int32_t *row_idx,
                                                  const double *cval, const double *r,
                                                  const double *x, double *scal, double *f,
                                                  double *part, const double *part_r, int nb_r,
                                                  double cap) {
  __shared__ double sff[4], sfx[4];
  __shared__ double sc[8];
  const double mu = rq_scalars(n, x, part_r, nb_r, scal, cap, sc).mu;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + w;
  double fv = 0, xv = 0;
  if (j < n) {
    double acc = 0;
    if (CSC) {
      for (int e = col_ptr[j] + lane; e < col_ptr[j + 1]; e += 64) acc += cval[e] * r[row_idx[e]];
    } else {
      // eight independent 512-byte loads of the column in flight per wave;
      // A is streamed once (non-temporal), r is reused by every column
      const double *col = A + (size_t)j * ld;
      int i = lane;
      double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (; i + 448 < m; i += 512) {
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += __builtin_nontemporal_load(col + i + 64 * u) * r[i + 64 * u];
      }
      for (; i < m; i += 64) s[0] += col[i] * r[i];
      acc = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    }
    acc = wave_sum(acc);
    xv = x[j];
    fv = -acc - mu * xv;
    if (lane == 0) f[j] = fv;
  }
  if (lane == 0) { sff[w] = fv * fv; sfx[w] = fv * xv; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = (sff[0] + sff[1]) + (sff[2] + sff[3]);
    part[2 * blockIdx.x + 1] = (sfx[0] + sfx[1]) + (sfx[2] + sfx[3]);
  }
}

hipError_t launch_gradient(const MatView &A, const double *r, const double *x, double *scal,
                           double *f, double *part, const double *part_r, int nb_r, double cap,
                           hipStream_t st) {
  const dim3 g(rmatvec_blocks(A));
  if (A.format == TLS_DENSE_COLMAJOR)
    TLS_LAUNCH(PC_GRADIENT, k_gradient<false>, g, dim3(256), 0, st, A.m, A.n, A.ld, A.val, nullptr,
                       nullptr, nullptr, r, x, scal, f, part, part_r, nb_r, cap);
  else
    TLS_LAUNCH(PC_GRADIENT, k_gradient<true>, g, dim3(256), 0, st, A.m, A.n, (int64_t)0, nullptr,
                       A.col_ptr, A.row_idx, A.cval, r, x, scal, f, part, part_r, nb_r, cap);
  return hipGetLastError();
}

__device__ inline void psi_step(int n, const double *part_f, int nb_f, double *scal, int k, double *rec,
                                const double *x, const double *f, double *rhs, double *xbest, double tie,
                                RqScalars q, double *sc, int *s_best);

// f = -A^T r - mu x from the row pass's partial A^T r (fixed order over its
// workgroups), with per-block partials of f.f and f.x as k_gradient writes them
// With ppart2 (the first step after a merged pass): A^T r = (sum of ppart)
// - scal[S_SHIFT0] (sum of ppart2), i.e. A^T r_0 - sigma_0^2 A^T A u_0.
__device__ inline RqScalars gradient_rows_body(int n, int G, const double *ppart, const double *x,
                                               double *scal, double *f, double *part,
                                               const double *part_r, int nb_r, double cap,
                                               const double *ppart2, double *sc, double *sff, double *sq) {
  const RqScalars q = rq_scalars(n, x, part_r, nb_r, scal, cap, sc);
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  double atr = partials_sum64(n, G, ppart, j, sq);
  if (ppart2) {
    __syncthreads();   // sq is reused
    atr -= scal[S_SHIFT0] * partials_sum64(n, G, ppart2, j, sq);
  }
  double fv = 0.0, xv = 0.0;
  if (threadIdx.x < 64 && j < n) {
    xv = x[j];
    fv = -atr - q.mu * xv;
    f[j] = fv;
  }
  const double ff = block_sum(fv * fv, sff);
  const double fx = block_sum(fv * xv, sff + 4);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ff;
    part[2 * blockIdx.x + 1] = fx;
  }
  return q;
}
// The gradient with psi_k formed by the last workgroup to finish (the work of
// k_outer_psi, without a launch of its own): every workgroup publishes its f
// and partials with a release fence before it counts itself in *cnt; the
// last one acquires them, resets the count and takes the step. Every
// workgroup forms the Rayleigh-quotient scalars identically, so the last one
// uses its own.
__global__ __launch_bounds__(256) void k_gradient_rows_psi(int n, int G, const double *ppart, const double *x,
                                                           double *scal, double *f, double *part,
                                                           const double *part_r, int nb_r, double cap,
                                                           const double *ppart2, int *cnt, int k, double *rec,
                                                           double *rhs, double *xbest, double tie) {
  __shared__ double sc[8], sff[8], sq[256];
  __shared__ int s_last, s_best;
  const RqScalars q = gradient_rows_body(n, G, ppart, x, scal, f, part, part_r, nb_r, cap, ppart2, sc, sff, sq);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) s_last = (atomicAdd(cnt, 1) == (int)gridDim.x - 1);
  __syncthreads();
  if (!s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (threadIdx.x == 0) *cnt = 0;
  psi_step(n, part, (int)gridDim.x, scal, k, rec, x, f, rhs, xbest, tie, q, sc, &s_best);
}
int gradient_rows_blocks(int n) { return (n + 63) / 64; }
hipError_t launch_gradient_rows_psi(const MatView &A, const double *ppart, const double *x, double *scal,
                                    double *f, double *part, const double *part_r, int nb_r, double cap,
                                    const double *ppart2, int *cnt, int k, double *rec, double *rhs,
                                    double *xbest, double tie, hipStream_t st) {
  TLS_LAUNCH(PC_GRADIENT, k_gradient_rows_psi, dim3(gradient_rows_blocks(A.n)), dim3(256), 0, st, A.n,
             rowpass_partials(A), ppart, x, scal, f, part, part_r, nb_r, cap, ppart2, cnt, k, rec, rhs, xbest,
             tie);
  return hipGetLastError();
}

// r_1 = r_0 - sigma_0^2 t with t = A u_0 (x_1 = x_0 + sigma_0^2 u_0, so this
// is b - A x_1), in place, with the per-64-row partials of r.r and b.r in
// the row pass's layout; sigma_0^2 (scal[S_SIG2]) is kept in scal[S_SHIFT0]
// for the gradient's A^T r_1
__global__ __launch_bounds__(64) void k_shift_residual(int m, const double *b, double *r, const double *t,
                                                       double *scal, double *part_r) {
  const double c = scal[S_SIG2];
  const int i = blockIdx.x * 64 + threadIdx.x;
  double ri = 0.0, bi = 0.0;
  if (i < m) {
    bi = b[i];
    ri = r[i] - c * t[i];
    r[i] = ri;
  }
  const double rr = wave_sum(ri * ri), br = wave_sum(bi * ri);
  if (threadIdx.x == 0) {
    part_r[2 * blockIdx.x] = rr;
    part_r[2 * blockIdx.x + 1] = br;
    if (blockIdx.x == 0) scal[S_SHIFT0] = c;
  }
}
hipError_t launch_shift_residual(int m, const double *b, double *r, const double *t, double *scal,
                                 double *part_r, hipStream_t st) {
  TLS_LAUNCH(PC_GRADIENT, k_shift_residual, dim3((m + 63) / 64), dim3(64), 0, st, m, b, r, t, scal, part_r);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scalar kernels (one workgroup of 256 threads)
// ---------------------------------------------------------------------------
__device__ inline double sum_pairs(const double *part, int nb, int which, double *sc) {
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[2 * i + which];
  return block_sum(v, sc);
}

// sigma^2, the clamped shift and g from the residual partials
__global__ __launch_bounds__(256) void k_outer_rq(int n, const double *x, const double *part_r,
                                                  int nb_r, double *scal, double cap) {
  __shared__ double sc[8];
  double xx = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) xx += x[i] * x[i];
  xx = block_sum(xx, sc);
  const double rr = sum_pairs(part_r, nb_r, 0, sc + 4);
  const double br = sum_pairs(part_r, nb_r, 1, sc);
  if (threadIdx.x == 0) {
    const double sig2 = rr / (1.0 + xx);
    const double mu = (cap > 0 && sig2 > cap) ? cap : sig2;
    scal[S_CAP] = cap;
    scal[S_SIG2] = sig2;
    scal[S_MU] = mu;
    scal[S_XX] = xx;
    scal[S_RR] = rr;
    scal[S_BR] = br;
    scal[S_G] = -br + mu;
  }
}
hipError_t launch_outer_rq(int n, const double *x, const double *part_r, int nb_r, double *scal,
                           double clamp_max, hipStream_t st) {
  TLS_LAUNCH(PC_SCALARS, k_outer_rq, dim3(1), dim3(256), 0, st, n, x, part_r, nb_r, scal, clamp_max);
  return hipGetLastError();
}

// psi_k from the gradient partials; record (sigma, psi, mu); the returned
// iterate: x_k is kept (copied to xbest) when psi_k is within the factor tie
// of the smallest psi before it (k = 1 always); slot S_BEST holds that minimum
__device__ inline void psi_step(int n, const double *part_f, int nb_f, double *scal, int k, double *rec,
                                const double *x, const double *f, double *rhs, double *xbest, double tie,
                                RqScalars q, double *sc, int *s_best) {
  const double ff = sum_pairs(part_f, nb_f, 0, sc);
  const double fx = sum_pairs(part_f, nb_f, 1, sc + 4);
  if (threadIdx.x == 0) {
    const double sig2 = q.sig2, mu = q.mu, xx = q.xx, br = q.br;
    const double dm = sig2 - mu;   // f at sigma^2 = f_mu - (sigma^2 - mu) x
    const double ffs = (dm == 0.0) ? ff : fmax(0.0, ff - 2.0 * dm * fx + dm * dm * xx);
    const double gs = -br + sig2;
    const double psi = sqrt((ffs + gs * gs) / (xx + 1.0));
    const double best = scal[S_BEST];
    const int isbest = (k == 1) || (psi <= tie * best);
    scal[S_FF] = ff;
    scal[S_FX] = fx;
    scal[S_PSI] = psi;
    scal[S_ISBEST] = isbest ? 1.0 : 0.0;
    if (k == 1 || psi < best) scal[S_BEST] = psi;
    scal[S_K] = (double)k;
    rec[4 * (k - 1) + 0] = sig2;
    rec[4 * (k - 1) + 1] = psi;
    rec[4 * (k - 1) + 2] = mu;
    rec[4 * (k - 1) + 3] = isbest;
    *s_best = isbest;
  }
  __syncthreads();
  // the next PCGTLS right-hand sides [-f, x], and the best iterate so far
  const bool keep = *s_best && xbest;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double xi = x[i];
    if (rhs) { rhs[i] = -f[i]; rhs[n + i] = xi; }
    if (keep) xbest[i] = xi;
  }
}
__global__ __launch_bounds__(256) void k_outer_psi(int n, const double *part_f, int nb_f,
                                                   double *scal, int k, double *rec,
                                                   const double *x, const double *f, double *rhs,
                                                   double *xbest, double tie) {
  __shared__ double sc[8];
  __shared__ int s_best;
  const RqScalars q{scal[S_SIG2], scal[S_MU], scal[S_XX], scal[S_BR]};
  psi_step(n, part_f, nb_f, scal, k, rec, x, f, rhs, xbest, tie, q, sc, &s_best);
}
hipError_t launch_outer_psi(int n, const double *x, const double *f, const double *part_f, int nb_f,
                            double *scal, int k, double *rec, double *rhs, double *xbest, double tie,
                            hipStream_t st) {
  TLS_LAUNCH(PC_SCALARS, k_outer_psi, dim3(1), dim3(256), 0, st, n, part_f, nb_f, scal, k, rec, x, f,
             rhs, xbest, tie);
  return hipGetLastError();
}

// right-hand sides of the two PCGTLS solves: [-f, x]
__global__ void k_make_rhs(int n, const double *f, const double *x, double *rhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  rhs[i] = -f[i];
  rhs[n + i] = x[i];
}
hipError_t launch_make_rhs(int n, const double *f, const double *x, double *rhs, hipStream_t st) {
  TLS_LAUNCH(PC_SCALARS, k_make_rhs, dim3((n + 255) / 256), dim3(256), 0, st, n, f, x, rhs);
  return hipGetLastError();
}

// z = x + omega, beta = (z^T f - g)/(z^T x + 1), x <- z + beta u; keeps the
// best iterate and an optional snapshot of x_k first. With done != NULL (the
// step flags of the two PCGTLS runs just finished, nsteps of them launched)
// it also records how many steps the longer run executed: a run's first
// step flagged done is the one its exits skipped. omega and u are read in
// the precision PCGTLS kept them (rows 0 and ldw of wu), so no conversion
// launch precedes the update.
template <typename WT>
__global__ __launch_bounds__(1024) void k_rqi_update(int n, double *x, const WT *wu, int ldw,
                                                     const double *f, double *scal, double *xbest,
                                                     double *xsnap, const int *done, int nsteps) {
  __shared__ double sc[32];
  const bool isbest = scal[S_ISBEST] != 0.0;
  double zf = 0, zx = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double xv = x[i];
    if (xbest && isbest) xbest[i] = xv;
    if (xsnap) xsnap[i] = xv;
    const double z = xv + (double)wu[i];
    zf += z * f[i];
    zx += z * xv;
  }
  // block reduction over 16 waves
  zf = wave_sum(zf);
  zx = wave_sum(zx);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sc[w] = zf; sc[16 + w] = zx; }
  __syncthreads();
  double tzf = 0, tzx = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) { tzf += sc[i]; tzx += sc[16 + i]; }
  const double beta = (tzf - scal[S_G]) / (tzx + 1.0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double z = x[i] + (double)wu[i];
    x[i] = z + beta * (double)wu[ldw + i];
  }
  if (threadIdx.x == 0) {
    scal[S_ZF] = tzf; scal[S_ZX] = tzx; scal[S_BETA] = beta;
    if (done) {
      int used = 0;
      for (int r = 0; r < 2; ++r) {
        int e = 0;
        while (e < nsteps && !done[2 * e + r]) ++e;
        used = e > used ? e : used;
      }
      scal[S_STEPS] = (double)used;
    }
  }
}
hipError_t launch_rqi_update(int n, double *x, const double *omega_u, const double *f,
                             const double *scal, double *xbest, double *xsnap, const int *done,
                             int nsteps, hipStream_t st) {
  TLS_LAUNCH(PC_SCALARS, k_rqi_update<double>, dim3(1), dim3(1024), 0, st, n, x, omega_u, n, f, (double *)scal,
                     xbest, xsnap, done, nsteps);
  return hipGetLastError();
}
hipError_t launch_rqi_update_pcg(int n, double *x, int compute, const void *w, int Np, const double *f,
                                 const double *scal, const int *done, int nsteps, hipStream_t st) {
  if (compute == TLS_FP64)
    TLS_LAUNCH(PC_SCALARS, k_rqi_update<double>, dim3(1), dim3(1024), 0, st, n, x, (const double *)w, Np, f,
               (double *)scal, (double *)nullptr, (double *)nullptr, done, nsteps);
  else
    TLS_LAUNCH(PC_SCALARS, k_rqi_update<float>, dim3(1), dim3(1024), 0, st, n, x, (const float *)w, Np, f,
               (double *)scal, (double *)nullptr, (double *)nullptr, done, nsteps);
  return hipGetLastError();
}

// x += scal[which] * u  (initial step x_1 = x_0 + sigma_0^2 u_0), or x += u when which < 0
__global__ void k_axpy_scal(int n, double *x, const double *u, const double *scal, int which) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = which >= 0 ? scal[which] : 1.0;
  x[i] += a * u[i];
}
hipError_t launch_axpy_init(int n, double *x, const double *u, const double *scal, int which,
                            hipStream_t st) {
  TLS_LAUNCH(PC_SCALARS, k_axpy_scal, dim3((n + 255) / 256), dim3(256), 0, st, n, x, u, scal, which);
  return hipGetLastError();
}

__global__ void k_copy(double *dst, const double *src, size_t count) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i < count; i += (size_t)gridDim.x * blockDim.x) dst[i] = src[i];
}
hipError_t launch_copy_f64(double *dst, const double *src, size_t count, hipStream_t st) {
  if (!count) return hipSuccess;
  size_t g = (count + 255) / 256;
  if (g > 4096) g = 4096;
  TLS_LAUNCH(PC_SCALARS, k_copy, dim3((unsigned)g), dim3(256), 0, st, dst, src, count);
  return hipGetLastError();
}
__global__ void k_add(double *x, const double *dx, size_t count) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i < count; i += (size_t)gridDim.x * blockDim.x) x[i] += dx[i];
}
hipError_t launch_add_f64(double *x, const double *dx, size_t count, hipStream_t st) {
  if (!count) return hipSuccess;
  size_t g = (count + 255) / 256;
  if (g > 4096) g = 4096;
  TLS_LAUNCH(PC_SCALARS, k_add, dim3((unsigned)g), dim3(256), 0, st, x, dx, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compensated residual (double-double): r_i = b_i - sum_j a_ij x_j with
// TwoProd (fma) and TwoSum error terms (Ogita, Rump and Oishi, "Accurate
// sum and dot product", 2005), then r.r accumulated the same way.
// ---------------------------------------------------------------------------
struct dd { double hi, lo; };
__device__ inline dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ inline dd two_prod(double a, double b) {
  const double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return two_sum(s.hi, s.lo);
}

// s - a x, exactly split: s + c stays the compensated running value
__device__ inline void comp_sub(double &s, double &c, double a, double x) {
  const dd p = two_prod(a, x);
  const dd t = two_sum(s, -p.hi);
  s = t.hi;
  c += t.lo - p.lo;
}
// r_i^2 in double-double from the compensated pair (s, c) of r_i
__device__ inline dd dd_square(double s, double c) {
  const dd r = two_sum(s, c);
  // (hi + lo)^2 ~ hi^2 + 2 hi lo
  const dd sq = two_prod(r.hi, r.hi);
  return two_sum(sq.hi, sq.lo + 2.0 * r.hi * r.lo);
}

// dense: 64 rows per workgroup, columns split over 16 waves as in the plain
// product; each wave keeps two compensated sums (even and odd columns of a
// chunk), the wave sums are joined to b_i in wave order with TwoSum
__global__ __launch_bounds__(1024) void k_residual_dd_dense(int m, int n, int64_t ld,
                                                            const double *A, const double *b,
                                                            const double *x, double *part) {
  __shared__ double rhi[RD_WAVES][RD_ROWS], rlo[RD_WAVES][RD_ROWS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * RD_ROWS + lane;
  double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
  if (i < m) {
    const double *a = A + i;
    int j = RD_CHUNK * w;
    for (; j + RD_CHUNK <= n; j += RD_CHUNK * RD_WAVES) {
#pragma unroll
      for (int q = 0; q < RD_CHUNK; q += 2) {
        comp_sub(s0, c0, a[(size_t)(j + q) * ld], x[j + q]);
        comp_sub(s1, c1, a[(size_t)(j + q + 1) * ld], x[j + q + 1]);
      }
    }
#pragma unroll
    for (int q = 0; q < RD_CHUNK; ++q)
      if (j + q < n) comp_sub(s0, c0, a[(size_t)(j + q) * ld], x[j + q]);
    const dd t = two_sum(s0, s1);
    s0 = t.hi;
    c0 += t.lo + c1;
  }
  rhi[w][lane] = s0;
  rlo[w][lane] = c0;
  __syncthreads();
  if (w != 0) return;
  dd rsq{0.0, 0.0};
  if (i < m) {
    double s = b[i], c = 0.0;
#pragma unroll
    for (int q = 0; q < RD_WAVES; ++q) {
      const dd t = two_sum(s, rhi[q][lane]);
      s = t.hi;
      c += t.lo + rlo[q][lane];
    }
    rsq = dd_square(s, c);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const dd o{__shfl_xor(rsq.hi, off, 64), __shfl_xor(rsq.lo, off, 64)};
    rsq = dd_add(rsq, o);
  }
  if (lane == 0) { part[2 * blockIdx.x] = rsq.hi; part[2 * blockIdx.x + 1] = rsq.lo; }
}

// CSR: one row per thread, 256 rows per workgroup
__global__ __launch_bounds__(256) void k_residual_dd_csr(int m, const double *val,
                                                         const int32_t *row_ptr,
                                                         const int32_t *col_idx, const double *b,
                                                         const double *x, double *part) {
  __shared__ double shi[256], slo[256];
  const int i = blockIdx.x * RES_ROWS + threadIdx.x;
  dd rsq{0.0, 0.0};
  if (i < m) {
    double s = b[i], c = 0.0;
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) comp_sub(s, c, val[e], x[col_idx[e]]);
    rsq = dd_square(s, c);
  }
  shi[threadIdx.x] = rsq.hi;
  slo[threadIdx.x] = rsq.lo;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      const dd a{shi[threadIdx.x], slo[threadIdx.x]};
      const dd bq{shi[threadIdx.x + off], slo[threadIdx.x + off]};
      const dd s = dd_add(a, bq);
      shi[threadIdx.x] = s.hi;
      slo[threadIdx.x] = s.lo;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = shi[0]; part[2 * blockIdx.x + 1] = slo[0]; }
}
hipError_t launch_residual_dd(const MatView &A, const double *b, const double *x, double *part,
                              hipStream_t st) {
  if (A.format == TLS_DENSE_COLMAJOR)
    TLS_LAUNCH(PC_RESID_DD, k_residual_dd_dense, dim3(matvec_blocks(A)), dim3(RD_ROWS * RD_WAVES), 0, st,
               A.m, A.n, A.ld, A.val, b, x, part);
  else
    TLS_LAUNCH(PC_RESID_DD, k_residual_dd_csr, dim3(matvec_blocks(A)), dim3(256), 0, st, A.m, A.val,
               A.row_ptr, A.col_idx, b, x, part);
  return hipGetLastError();
}

// sigma^2 = (sum r^2) / (1 + ||x||^2) with both sums in double-double; result in scal[0]
__global__ __launch_bounds__(256) void k_sigma_dd(int n, const double *x, const double *part, int nb,
                                                  double *scal) {
  __shared__ double shi[256], slo[256];
  dd acc{0.0, 0.0};
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc = dd_add(acc, dd{part[2 * i], part[2 * i + 1]});
  dd xx{0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const dd p = two_prod(x[i], x[i]);
    xx = dd_add(xx, p);
  }
  // reduce acc then xx
  for (int pass = 0; pass < 2; ++pass) {
    const dd v = pass == 0 ? acc : xx;
    shi[threadIdx.x] = v.hi;
    slo[threadIdx.x] = v.lo;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
      if (threadIdx.x < off) {
        const dd s = dd_add(dd{shi[threadIdx.x], slo[threadIdx.x]},
                            dd{shi[threadIdx.x + off], slo[threadIdx.x + off]});
        shi[threadIdx.x] = s.hi;
        slo[threadIdx.x] = s.lo;
      }
      __syncthreads();
    }
    if (pass == 0) acc = dd{shi[0], slo[0]};
    else xx = dd{shi[0], slo[0]};
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // sigma^2 = acc / (1 + xx), one Newton correction of the double quotient
    const dd den = dd_add(dd{1.0, 0.0}, xx);
    const double q = acc.hi / den.hi;
    const dd qd = two_prod(q, den.hi);
    const double rem = ((acc.hi - qd.hi) - qd.lo + acc.lo - q * den.lo);
    const double q2 = q + rem / den.hi;
    scal[0] = q2;
    scal[1] = sqrt(q2);
  }
}
hipError_t launch_sigma_dd(int n, const double *x, const double *part, int nb, double *scal,
                           hipStream_t st) {
  TLS_LAUNCH(PC_RESID_DD, k_sigma_dd, dim3(1), dim3(256), 0, st, n, x, part, nb, scal);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lanczos step bookkeeping (gate estimates), up to two recurrences at once
// (one workgroup each): run 0 on M_s = R_hat^{-1} R_hat^{-T}, run 1 on
// M = D^{-1} M_s D^{-1} = (R^T R)^{-1}. The device applies M_s to the pair
// [v0_k, D^{-1} v1_k]; here w1 = D^{-1} (M_s D^{-1} v1_k). The three-term
// recurrence orthogonalises w against v_k and v_{k-1} by classical
// Gram-Schmidt applied twice (enough for the extreme Ritz values after the
// dozen steps the gate takes); alpha_k from the first pass,
// beta_k = ||w||, v_{k+1} = w / beta_k, and the next operator input
// (D^{-1} v1_{k+1} for run 1) is written to `nxt`.
// Layout: V[run][K+1][Np]; ab[run][2K+2]: alpha, beta, active, steps.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_lanczos_orth(int n, int Np, int k, int K, double *V,
                                                       const double *Wout, double *nxt,
                                                       const double *dsc, double *ab) {
  __shared__ double red[16][2];
  __shared__ double h[2];
  const int run = blockIdx.x;
  double *Vr = V + (size_t)run * (K + 1) * Np;
  double *abr = ab + (size_t)run * (2 * K + 2);
  if (abr[2 * K] == 0.0) return;        // this run stopped earlier (uniform per block)
  double *w = Vr + (size_t)(k + 1) * Np;
  const double *vk = Vr + (size_t)k * Np;
  const double *vp = (k > 0) ? Vr + (size_t)(k - 1) * Np : nullptr;
  const double *src = Wout + (size_t)run * Np;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nw = blockDim.x >> 6;
  for (int j = tid; j < n; j += blockDim.x) w[j] = run ? dsc[j] * src[j] : src[j];
  __syncthreads();
  double alpha = 0;
  for (int pass = 0; pass < 2; ++pass) {
    double a0 = 0, a1 = 0;
    for (int j = tid; j < n; j += blockDim.x) {
      const double wj = w[j];
      a0 += vk[j] * wj;
      if (vp) a1 += vp[j] * wj;
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) { red[wv][0] = a0; red[wv][1] = a1; }
    __syncthreads();
    if (tid < 2) {
      double t = 0;
      for (int q = 0; q < nw; ++q) t += red[q][tid];
      h[tid] = t;
    }
    __syncthreads();
    const double hk = h[0], hp = h[1];
    if (pass == 0) alpha = hk;
    for (int j = tid; j < n; j += blockDim.x) w[j] -= hk * vk[j] + (vp ? hp * vp[j] : 0.0);
    __syncthreads();   // w complete; red and h are rewritten next
  }
  double nn = 0;
  for (int j = tid; j < n; j += blockDim.x) nn += w[j] * w[j];
  nn = wave_sum(nn);
  if (lane == 0) red[wv][0] = nn;
  __syncthreads();
  double tot = 0;
  for (int q = 0; q < nw; ++q) tot += red[q][0];
  const double beta = sqrt(tot);
  const bool stop = !(beta > 1e-13 * fabs(alpha)) || (k + 1 >= K);
  if (!stop) {
    const double ib = 1.0 / beta;
    for (int j = tid; j < n; j += blockDim.x) {
      const double v = w[j] * ib;
      w[j] = v;
      nxt[(size_t)run * Np + j] = run ? dsc[j] * v : v;
    }
  }
  __syncthreads();
  if (tid == 0) {
    abr[k] = alpha;
    abr[K + k] = beta;
    abr[2 * K + 1] = (double)(k + 1);
    if (stop) abr[2 * K] = 0.0;
  }
}
hipError_t launch_lanczos_orth(int n, int Np, int k, int K, double *V, const double *Wout,
                               double *nxt, const double *dsc, double *ab, hipStream_t st, int runs) {
  TLS_LAUNCH(PC_LANCZOS, k_lanczos_orth, dim3(runs), dim3(1024), 0, st, n, Np, k, K, V, Wout, nxt, dsc, ab);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Refinement sweep: PCG on the explicit operator K = A^T A - mu I (two
// right-hand sides), preconditioned by M = (R^T R)^{-1}. Scalar and vector
// steps in one workgroup per right-hand side (n <= 65536).
//   rs layout per rhs (doubles): 0 r.z (current), 1 alpha, 2 beta, 3 p.q
// ---------------------------------------------------------------------------
// q_r = A^T t_r - mu p_r; alpha = rz / (p.q); x += alpha p; r -= alpha q
__global__ __launch_bounds__(1024) void k_ref_step1(int n, const double *scal, double *x, double *r,
                                                    const double *p, double *q, double *rs) {
  __shared__ double sc[16];
  const int rhs = blockIdx.x;
  const size_t o = (size_t)rhs * n;
  const double mu = scal[1];
  double pq = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double qi = q[o + i] - mu * p[o + i];
    q[o + i] = qi;
    pq += p[o + i] * qi;
  }
  pq = wave_sum(pq);
  if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = pq;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sc[w];
  const double rz = rs[4 * rhs + 0];
  const double alpha = (t != 0.0) ? rz / t : 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    x[o + i] += alpha * p[o + i];
    r[o + i] -= alpha * q[o + i];
  }
  if (threadIdx.x == 0) { rs[4 * rhs + 1] = alpha; rs[4 * rhs + 3] = t; }
}
// beta = r.z_new / r.z_old; p = z + beta p (first: p = z)
__global__ __launch_bounds__(1024) void k_ref_step2(int n, const double *r, const double *z, double *p,
                                                    double *rs, int first) {
  __shared__ double sc[16];
  const int rhs = blockIdx.x;
  const size_t o = (size_t)rhs * n;
  double rz = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) rz += r[o + i] * z[o + i];
  rz = wave_sum(rz);
  if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = rz;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sc[w];
  const double beta = first ? 0.0 : ((rs[4 * rhs] != 0.0) ? t / rs[4 * rhs] : 0.0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[o + i] = z[o + i] + beta * p[o + i];
  __syncthreads();
  if (threadIdx.x == 0) { rs[4 * rhs + 0] = t; rs[4 * rhs + 2] = beta; }
}
hipError_t launch_ref_step1(int n, int nrhs, const double *scal, double *x, double *r,
                            const double *p, double *q, double *rs, hipStream_t st) {
  TLS_LAUNCH(PC_SCALARS, k_ref_step1, dim3(nrhs), dim3(1024), 0, st, n, scal, x, r, p, q, rs);
  return hipGetLastError();
}
hipError_t launch_ref_step2(int n, int nrhs, const double *r, const double *z, double *p, double *rs,
                            int first, hipStream_t st) {
  TLS_LAUNCH(PC_SCALARS, k_ref_step2, dim3(nrhs), dim3(1024), 0, st, n, r, z, p, rs, first);
  return hipGetLastError();
}

}  // namespace tls

namespace tls {

// ---------------------------------------------------------------------------
// warm start: dot products (one workgroup per pair, fixed order) and
// x_w = x_0 + c1 u_0 + c2 u_1
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dots(DotPairs D, double *out) {
  __shared__ double sc[4];
  const int p = blockIdx.x;
  const double *a = D.a[p], *b = D.b[p];
  const int64_t len = D.len[p];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += 256) s = fma(a[i], b[i], s);
  s = block_sum(s, sc);
  if (threadIdx.x == 0) out[p] = s;
}
hipError_t launch_dots(const DotPairs &D, int count, double *out, hipStream_t st) {
  if (count <= 0 || count > DotPairs::MAX) return hipErrorInvalidValue;
  TLS_LAUNCH(PC_SCALARS, k_dots, dim3(count), dim3(256), 0, st, D, out);
  return hipGetLastError();
}

__global__ void k_axpy2(int n, const double *x0, const double *u0, const double *u1, double c1,
                        double c2, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x0[i] + (c1 * u0[i] + c2 * u1[i]);
}
__global__ void k_scale_copy(int n, const double *src, double alpha, double *dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = alpha * src[i];
}
hipError_t launch_scale_copy(int n, const double *src, double alpha, double *dst, hipStream_t st) {
  TLS_LAUNCH(PC_SETUP, k_scale_copy, dim3((n + 255) / 256), dim3(256), 0, st, n, src, alpha, dst);
  return hipGetLastError();
}
hipError_t launch_axpy2(int n, const double *x0, const double *u0, const double *u1, double c1,
                        double c2, double *out, hipStream_t st) {
  TLS_LAUNCH(PC_SCALARS, k_axpy2, dim3((n + 255) / 256), dim3(256), 0, st, n, x0, u0, u1, c1, c2, out);
  return hipGetLastError();
}

}  // namespace tls
