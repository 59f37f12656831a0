// Preconditioner construction: CSC copy of a CSR matrix, column scaling and
// rounding to u_q (two-sided diagonal scaling, Section 3.1), the Gram
// matrix A^T A (sparse and dense), its blocked Cholesky factorization
// (Section 2: the factor R of A^T A, computed once), and the packing of R
// into the tiled storage the triangular solves read.
//
// Dense matrices are column-major. The Gram matrix G is Np x Np
// column-major with only its upper triangle meaningful; Cholesky overwrites
// it with R (G = R^T R). Padding rows/columns n..Np-1 hold the identity.
#include <algorithm>
#include <climits>

#include "common.h"
#include "kernels.h"

namespace tls {

// --------------------------------------------------------------------------
// small utilities
// --------------------------------------------------------------------------
__global__ void k_fill_i32(int *p, int v, size_t count) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, size_t count) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
static int grid_for(size_t count) {
  size_t g = (count + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}
hipError_t launch_fill_i32(int *p, int v, size_t count, hipStream_t st) {
  if (!count) return hipSuccess;
  TLS_LAUNCH(PC_SETUP, k_fill_i32, dim3(grid_for(count)), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, double v, size_t count, hipStream_t st) {
  if (!count) return hipSuccess;
  TLS_LAUNCH(PC_SETUP, k_fill_f64, dim3(grid_for(count)), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

// several fills in one launch (regions of 4- or 8-byte words)
__global__ void k_fill_multi(FillSet F) {
  for (int r = 0; r < F.count; ++r) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (F.wide[r]) {
      uint64_t *p = (uint64_t *)F.ptr[r];
      for (; i < F.n[r]; i += (size_t)gridDim.x * blockDim.x) p[i] = F.bits[r];
    } else {
      uint32_t *p = (uint32_t *)F.ptr[r];
      for (; i < F.n[r]; i += (size_t)gridDim.x * blockDim.x) p[i] = (uint32_t)F.bits[r];
    }
  }
}
hipError_t launch_fill_multi(const FillSet &F, hipStream_t st) {
  size_t most = 1;
  for (int r = 0; r < F.count; ++r) most = std::max(most, F.n[r]);
  TLS_LAUNCH(PC_SETUP, k_fill_multi, dim3(grid_for(most)), dim3(256), 0, st, F);
  return hipGetLastError();
}
void FillSet::add_i32(int *p, int v, size_t cnt) {
  if (!cnt || count >= MAX) return;
  ptr[count] = p; n[count] = cnt; bits[count] = (uint32_t)v; wide[count] = 0; ++count;
}
void FillSet::add_f64(double *p, double v, size_t cnt) {
  if (!cnt || count >= MAX) return;
  ptr[count] = p; n[count] = cnt; bits[count] = __builtin_bit_cast(uint64_t, v); wide[count] = 1; ++count;
}

__global__ void k_check_finite(const double *v, size_t count, int *flag) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  int bad = 0;
  for (; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v[i]);
    bad |= ((u & 0x7ff0000000000000ull) == 0x7ff0000000000000ull);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}
// structure of a CSR matrix as the device code relies on it: row_ptr[0] = 0,
// row_ptr[m] = nnz, row_ptr nondecreasing, 0 <= col_idx < n and strictly
// increasing inside each row. Any violation sets *bad (read by the host
// before any kernel uses the indices).
__global__ void k_validate_csr(int m, int n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                               int *bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int b = 0;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t == 0) b |= (row_ptr[0] != 0) | (row_ptr[m] != nnz);
  for (int64_t i = t; i < m; i += stride) {
    const int32_t a = row_ptr[i], c = row_ptr[i + 1];
    if (a > c || a < 0 || c > nnz) { b = 1; continue; }
    for (int32_t e = a; e < c; ++e) {
      const int32_t j = col_idx[e];
      b |= (j < 0) | (j >= n);
      if (e > a) b |= (col_idx[e - 1] >= j);
    }
  }
  if (__any(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}
hipError_t launch_validate_csr(int m, int n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                               int *bad, hipStream_t st) {
  TLS_LAUNCH(PC_SETUP, k_validate_csr, dim3(grid_for((size_t)m)), dim3(256), 0, st, m, n, nnz, row_ptr, col_idx,
             bad);
  return hipGetLastError();
}
hipError_t launch_check_finite(const double *v, size_t count, int *flag, hipStream_t st) {
  if (!count) return hipSuccess;
  TLS_LAUNCH(PC_SETUP, k_check_finite, dim3(grid_for(count)), dim3(256), 0, st, v, count, flag);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// CSC copy of a CSR matrix, rows ascending inside each column
// --------------------------------------------------------------------------
__global__ void k_csc_count(int64_t nnz, const int32_t *col_idx, int32_t *cnt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[col_idx[e]], 1);
}
// the same count through a per-workgroup histogram in LDS (n <= CSC_HIST):
// a workgroup takes a range of rows, counts its columns in LDS and adds each
// nonzero bin to the global count once, instead of one global atomic per
// entry on a few thousand addresses
constexpr int CSC_HIST = 12288, CSC_HIST_ROWS = 1024;
constexpr int CSC_BATCH = 8;   // independent loads in flight per thread in the entry loops
__global__ __launch_bounds__(256) void k_csc_count_lds(int m, int n, const int32_t *row_ptr,
                                                       const int32_t *col_idx, int32_t *cnt) {
  __shared__ int32_t h[CSC_HIST];
  for (int c = threadIdx.x; c < n; c += 256) h[c] = 0;
  __syncthreads();
  const int r0 = blockIdx.x * CSC_HIST_ROWS, r1 = min(m, r0 + CSC_HIST_ROWS);
  const int e0 = row_ptr[r0], e1 = row_ptr[r1];
  for (int e = e0 + threadIdx.x; e < e1; e += 256 * CSC_BATCH) {
    int ci[CSC_BATCH];
#pragma unroll
    for (int u = 0; u < CSC_BATCH; ++u) ci[u] = (e + 256 * u < e1) ? col_idx[e + 256 * u] : -1;
#pragma unroll
    for (int u = 0; u < CSC_BATCH; ++u)
      if (ci[u] >= 0) atomicAdd(&h[ci[u]], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += 256)
    if (h[c]) atomicAdd(&cnt[c], h[c]);
}

// exclusive scan of cnt[0..n) into col_ptr[0..n], one workgroup
__global__ void k_scan(int n, const int32_t *cnt, int32_t *col_ptr) {
  __shared__ int32_t s_tot[256];
  const int tid = threadIdx.x;
  const int per = (n + 255) / 256;
  const int a = tid * per, b = min(n, a + per);
  int32_t sum = 0;
  for (int i = a; i < b; ++i) sum += cnt[i];
  s_tot[tid] = sum;
  __syncthreads();
  if (tid == 0) {
    int32_t run = 0;
    for (int t = 0; t < 256; ++t) { const int32_t v = s_tot[t]; s_tot[t] = run; run += v; }
    col_ptr[n] = run;
  }
  __syncthreads();
  int32_t run = s_tot[tid];
  for (int i = a; i < b; ++i) { col_ptr[i] = run; run += cnt[i]; }
}

// Global-atomic build (used past the segmented build's size limit): one
// thread per entry (its row by binary search in row_ptr, which stays in L2)
// takes the next free slot of its column in arbitrary order; k_csc_rank
// orders the rows of each column after. With global counters, one thread
// per row chains a row's returning atomics and was slower (50 us against
// 30 us at 20000 x 2000, 0.5%).
__global__ void k_csc_scatter(int m, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                              const double *val, const int32_t *col_ptr, int32_t *fill,
                              int32_t *tmp_row, double *tmp_val) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int lo = 0, hi = m;            // row_ptr[lo] <= e < row_ptr[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (row_ptr[mid] <= e) lo = mid; else hi = mid;
  }
  const int c = col_idx[e];
  const int pos = col_ptr[c] + atomicAdd(&fill[c], 1);
  tmp_row[pos] = lo;
  tmp_val[pos] = val[e];
}

// one thread per CSC slot: its final position is the number of entries of
// the same column with a smaller row (rows are distinct inside a column)
__global__ void k_csc_rank(int64_t nnz, int n, const int32_t *col_ptr, const int32_t *tmp_row,
                           const double *tmp_val, int32_t *row_idx, double *cval) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  // column of slot e by binary search in col_ptr
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (col_ptr[mid] <= e) lo = mid; else hi = mid;
  }
  const int a = col_ptr[lo], b = col_ptr[lo + 1];
  const int r = tmp_row[e];
  int rank = 0;
  for (int t = a; t < b; ++t) rank += (tmp_row[t] < r);
  row_idx[a + rank] = r;
  cval[a + rank] = tmp_val[e];
}

// Block-segmented build (n <= CSC_HIST and nb * n <= CSC_BLK_MAX, nb row
// blocks of CSC_HIST_ROWS rows): bc[b * n + c] holds the count of column c in
// row block b, bo[b * n + c] the offset of that block's segment inside
// column c. The segments of a column follow each other in row order, so an
// entry's rank is found among the few entries of its own segment, and the
// slots are claimed with LDS atomics instead of global ones. Every loop over
// entries keeps CSC_BATCH independent loads in flight per thread.
constexpr int64_t CSC_BLK_MAX = 1 << 20;
static bool csc_blocked(int64_t m, int64_t n) {
  const int64_t nb = (m + CSC_HIST_ROWS - 1) / CSC_HIST_ROWS;
  return n <= CSC_HIST && nb * n <= CSC_BLK_MAX;
}
size_t csc_fill_ints(int64_t m, int64_t n) {
  const int64_t nb = std::max<int64_t>(1, (m + CSC_HIST_ROWS - 1) / CSC_HIST_ROWS);
  return (size_t)std::max<int64_t>(1, csc_blocked(m, n) ? 2 * nb * n : n);
}

__global__ __launch_bounds__(1024) void k_csc_count_blk(int m, int n, const int32_t *row_ptr,
                                                        const int32_t *col_idx, int32_t *bc) {
  __shared__ int32_t h[CSC_HIST];
  for (int c = threadIdx.x; c < n; c += 1024) h[c] = 0;
  __syncthreads();
  const int r0 = blockIdx.x * CSC_HIST_ROWS, r1 = min(m, r0 + CSC_HIST_ROWS);
  const int e0 = row_ptr[r0], e1 = row_ptr[r1];
  for (int e = e0 + threadIdx.x; e < e1; e += 1024 * CSC_BATCH) {
    int ci[CSC_BATCH];
#pragma unroll
    for (int u = 0; u < CSC_BATCH; ++u) ci[u] = (e + 1024 * u < e1) ? col_idx[e + 1024 * u] : -1;
#pragma unroll
    for (int u = 0; u < CSC_BATCH; ++u)
      if (ci[u] >= 0) atomicAdd(&h[ci[u]], 1);
  }
  __syncthreads();
  int32_t *dst = bc + (size_t)blockIdx.x * n;
  for (int c = threadIdx.x; c < n; c += 1024) dst[c] = h[c];
}

// one workgroup: per column the exclusive prefix of its block counts (into
// bo) and its total, then col_ptr as the exclusive scan of the totals
// (thread t owns a contiguous range of columns)
__global__ __launch_bounds__(1024) void k_csc_scan_blk(int n, int nb, const int32_t *__restrict__ bc,
                                                       int32_t *__restrict__ bo, int32_t *__restrict__ col_ptr) {
  __shared__ int32_t s_tot[1024];
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int a = min(n, tid * per), z = min(n, a + per);
  int32_t sum = 0;
  for (int c = a; c < z; ++c) {
    int32_t run = 0;
    for (int b0 = 0; b0 < nb; b0 += CSC_BATCH) {
      int32_t v[CSC_BATCH];
#pragma unroll
      for (int u = 0; u < CSC_BATCH; ++u) v[u] = (b0 + u < nb) ? bc[(size_t)(b0 + u) * n + c] : 0;
#pragma unroll
      for (int u = 0; u < CSC_BATCH; ++u) {
        if (b0 + u < nb) bo[(size_t)(b0 + u) * n + c] = run;
        run += v[u];
      }
    }
    col_ptr[c] = run;   // the column total until the scan below
    sum += run;
  }
  s_tot[tid] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan of the thread sums
    const int32_t v = tid >= off ? s_tot[tid - off] : 0;
    __syncthreads();
    s_tot[tid] += v;
    __syncthreads();
  }
  int32_t run = s_tot[tid] - sum;
  for (int c = a; c < z; ++c) {
    const int32_t t = col_ptr[c];
    col_ptr[c] = run;
    run += t;
  }
  if (tid == 1023) col_ptr[n] = s_tot[1023];
}

// one workgroup per row block, one thread per row: each entry takes the next
// free slot of its column's segment for this block (LDS counter)
static_assert(CSC_HIST_ROWS == 1024, "k_csc_scatter_blk runs one thread per row of a block");
__global__ __launch_bounds__(1024) void k_csc_scatter_blk(int m, int n, const int32_t *row_ptr,
                                                          const int32_t *col_idx, const double *val,
                                                          const int32_t *col_ptr, const int32_t *bo,
                                                          int32_t *tmp_row, double *tmp_val) {
  __shared__ int32_t base[CSC_HIST], used[CSC_HIST];
  const int32_t *off = bo + (size_t)blockIdx.x * n;
  for (int c = threadIdx.x; c < n; c += 1024) {
    base[c] = col_ptr[c] + off[c];
    used[c] = 0;
  }
  __syncthreads();
  const int r = blockIdx.x * CSC_HIST_ROWS + threadIdx.x;   // CSC_HIST_ROWS == blockDim.x
  if (r >= m) return;
  const int e1 = row_ptr[r + 1];
  for (int e = row_ptr[r]; e < e1; e += CSC_BATCH) {
    int ci[CSC_BATCH];
    double v[CSC_BATCH];
#pragma unroll
    for (int u = 0; u < CSC_BATCH; ++u) {
      ci[u] = (e + u < e1) ? col_idx[e + u] : -1;
      v[u] = (e + u < e1) ? val[e + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CSC_BATCH; ++u) {
      if (ci[u] < 0) continue;
      const int pos = base[ci[u]] + atomicAdd(&used[ci[u]], 1);
      tmp_row[pos] = r;
      tmp_val[pos] = v[u];
    }
  }
}

// one thread per CSC slot: its final position inside its block segment is
// the number of entries of the segment with a smaller row
__global__ void k_csc_rank_blk(int64_t nnz, int n, int nb, const int32_t *col_ptr, const int32_t *bo,
                               const int32_t *tmp_row, const double *tmp_val, int32_t *row_idx,
                               double *cval) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int lo = 0, hi = n;   // column of slot e: col_ptr[lo] <= e < col_ptr[lo + 1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (col_ptr[mid] <= e) lo = mid; else hi = mid;
  }
  const int r = tmp_row[e];
  const int b = r / CSC_HIST_ROWS;
  const int s0 = col_ptr[lo] + bo[(size_t)b * n + lo];
  const int s1 = (b + 1 < nb) ? col_ptr[lo] + bo[(size_t)(b + 1) * n + lo] : col_ptr[lo + 1];
  int rank = 0;
  for (int t = s0; t < s1; ++t) rank += (tmp_row[t] < r);
  row_idx[s0 + rank] = r;
  cval[s0 + rank] = tmp_val[e];
}

hipError_t launch_csc_build(int m, int n, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col_idx, const double *val, int32_t *col_ptr,
                            int32_t *row_idx, double *cval, int32_t *tmp_row, double *tmp_val,
                            int32_t *fill, hipStream_t st) {
  hipError_t e;
  if (nnz == 0) return launch_fill_i32(col_ptr, 0, (size_t)n + 1, st);
  if (csc_blocked(m, n)) {
    const int nb = (m + CSC_HIST_ROWS - 1) / CSC_HIST_ROWS;
    int32_t *bo = fill + (size_t)nb * n;
    TLS_LAUNCH(PC_SETUP, k_csc_count_blk, dim3(nb), dim3(1024), 0, st, m, n, row_ptr, col_idx, fill);
    TLS_LAUNCH(PC_SETUP, k_csc_scan_blk, dim3(1), dim3(1024), 0, st, n, nb, (const int32_t *)fill, bo, col_ptr);
    TLS_LAUNCH(PC_SETUP, k_csc_scatter_blk, dim3(nb), dim3(CSC_HIST_ROWS), 0, st, m, n, row_ptr, col_idx, val,
               col_ptr, (const int32_t *)bo, tmp_row, tmp_val);
    TLS_LAUNCH(PC_SETUP, k_csc_rank_blk, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, nnz, n, nb,
               col_ptr, (const int32_t *)bo, tmp_row, tmp_val, row_idx, cval);
    return hipGetLastError();
  }
  if ((e = launch_fill_i32(fill, 0, n, st)) != hipSuccess) return e;
  const unsigned ge = (unsigned)((nnz + 255) / 256);
  if (nnz > 0) {
    if (n <= CSC_HIST)
      TLS_LAUNCH(PC_SETUP, k_csc_count_lds, dim3((unsigned)((m + CSC_HIST_ROWS - 1) / CSC_HIST_ROWS)), dim3(256),
                 0, st, m, n, row_ptr, col_idx, fill);
    else
      TLS_LAUNCH(PC_SETUP, k_csc_count, dim3(ge), dim3(256), 0, st, nnz, col_idx, fill);
  }
  TLS_LAUNCH(PC_SETUP, k_scan, dim3(1), dim3(256), 0, st, n, fill, col_ptr);
  if ((e = launch_fill_i32(fill, 0, n, st)) != hipSuccess) return e;
  if (nnz > 0)
    TLS_LAUNCH(PC_SETUP, k_csc_scatter, dim3(ge), dim3(256), 0, st, m, nnz, row_ptr, col_idx, val,
               col_ptr, fill, tmp_row, tmp_val);
  if (nnz > 0)
    TLS_LAUNCH(PC_SETUP, k_csc_rank, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, nnz, n,
                       col_ptr, tmp_row, tmp_val, row_idx, cval);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// statistics of the column norms for the solve (one workgroup, fixed order):
// out = {sum d_j^2, min, max, mean, std of ln max(d_j, 1e-300)}
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dstats(int n, const double *d, double *out) {
  __shared__ double sc[8];
  __shared__ double ext[2][4];
  double s2 = 0, sl = 0, sq = 0, lo = INFINITY, hi = -INFINITY;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double v = d[j], l = log(fmax(v, 1e-300));
    s2 += v * v;
    sl += l;
    sq += l * l;
    lo = fmin(lo, l);
    hi = fmax(hi, l);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { ext[0][w] = lo; ext[1][w] = hi; }
  s2 = block_sum(s2, sc);
  sl = block_sum(sl, sc + 4);
  sq = block_sum(sq, sc);
  if (threadIdx.x == 0) {
    lo = fmin(fmin(ext[0][0], ext[0][1]), fmin(ext[0][2], ext[0][3]));
    hi = fmax(fmax(ext[1][0], ext[1][1]), fmax(ext[1][2], ext[1][3]));
    const double mean = sl / n;
    out[0] = s2;
    out[1] = lo;
    out[2] = hi;
    out[3] = mean;
    out[4] = sqrt(fmax(0.0, sq / n - mean * mean));
  }
}
hipError_t launch_dstats(int n, const double *d, double *out, hipStream_t st) {
  TLS_LAUNCH(PC_SETUP, k_dstats, dim3(1), dim3(256), 0, st, n, d, out);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// column norms d_j = ||A e_j|| (one wave per column, fixed order)
// --------------------------------------------------------------------------
__global__ void k_colnorms_csc(int n, const int32_t *col_ptr, const double *cval, double *d) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n) return;
  double s = 0;
  for (int e = col_ptr[j] + lane; e < col_ptr[j + 1]; e += 64) s += cval[e] * cval[e];
  s = wave_sum(s);
  if (lane == 0) d[j] = sqrt(s);
}
__global__ void k_colnorms_dense(int m, int n, int64_t ld, const double *A, double *d) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n) return;
  const double *col = A + (size_t)j * ld;
  double s = 0;
  for (int i = lane; i < m; i += 64) s += col[i] * col[i];
  s = wave_sum(s);
  if (lane == 0) d[j] = sqrt(s);
}
// Row-major working copy of a dense column-major A (row stride ldr >= n, a
// multiple of 64, padding columns zero): 64 x 64 tiles, each read column by
// column (512-byte loads), transposed through LDS and written row by row.
// A bounded grid walks the tiles (row-block major, so neighbouring
// workgroups write neighbouring pieces of the same rows): the copy runs
// beside the factorization's narrow launches and must leave them CUs and
// LDS, which a grid of one workgroup per tile, queued behind each other,
// would not.
constexpr int ROWCOPY_WGS = 256;
__global__ __launch_bounds__(256) void k_rowcopy_dense(int m, int n, int64_t ld, const double *A, int64_t ldr,
                                                       double *At) {
  __shared__ double tile[64][65];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nJ = (int)(ldr / 64);
  const int64_t ntiles = (int64_t)((m + 63) / 64) * nJ;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int I = (int)(t / nJ), J = (int)(t % nJ);
    const int i = I * 64 + lane;
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {        // the thread's 16 loads in flight together
      const int j = J * 64 + 4 * q + w;
      v[q] = (i < m && j < n) ? __builtin_nontemporal_load(A + (size_t)j * ld + i) : 0.0;
    }
    __syncthreads();                      // the previous tile's reads of LDS are done
#pragma unroll
    for (int q = 0; q < 16; ++q) tile[4 * q + w][lane] = v[q];
    __syncthreads();
    const int j = J * 64 + lane;          // < ldr
#pragma unroll 4
    for (int rr = 0; rr < 64; rr += 4) {
      const int r = I * 64 + rr + w;
      if (r < m) At[(size_t)r * ldr + j] = (j < n) ? tile[lane][rr + w] : 0.0;
    }
  }
}
// d_j = sqrt(sum over the row blocks of colsq), in block order
__global__ void k_colnorms_parts(int n, int nblk, const double *colsq, double *d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  int b = 0;
  for (; b + 4 <= nblk; b += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] += colsq[(size_t)(b + u) * n + j];
  }
  for (; b < nblk; ++b) c[0] += colsq[(size_t)b * n + j];
  d[j] = sqrt((c[0] + c[1]) + (c[2] + c[3]));
}
// the sums of colsq over slices of COLSQ_SLICE row blocks (slice s into
// out[s][j]), so that the final sum reads few partials per column and the
// long reduction is spread over the chip
constexpr int COLSQ_SLICE = 64;
__global__ void k_colnorms_slices(int n, int nblk, const double *colsq, double *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, sl = blockIdx.y;
  if (j >= n) return;
  const int b0 = sl * COLSQ_SLICE, b1 = min(nblk, b0 + COLSQ_SLICE);
  double c[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int b = b0;
  for (; b + 8 <= b1; b += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] += colsq[(size_t)(b + u) * n + j];
  }
  for (; b < b1; ++b) c[0] += colsq[(size_t)b * n + j];
  out[(size_t)sl * n + j] = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
}
// Column sums of squares of a dense column-major A over slabs of CS_ROWS
// rows (part[s][j]) and the finite-input flag, in one read of A's m rows:
// each wave streams CS_ROWS consecutive entries of one column (32 loads of
// 512 bytes in flight per wave)
constexpr int CS_ROWS = 2048;
__global__ __launch_bounds__(256) void k_colsq_dense(int m, int n, int64_t ld, const double *A, double *part,
                                                     int *flag) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + w;
  if (j >= n) return;   // uniform per wave; no barrier below
  const int nslab = (m + CS_ROWS - 1) / CS_ROWS;
  int bad = 0;
  for (int S = blockIdx.y; S < nslab; S += gridDim.y) {
    const int64_t r0 = (int64_t)S * CS_ROWS;
    const double *col = A + (size_t)j * ld + r0;
    const int rows = (int)min((int64_t)CS_ROWS, (int64_t)m - r0);
    double v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int i = lane + 64 * q;
      v[q] = i < rows ? __builtin_nontemporal_load(col + i) : 0.0;
    }
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const uint64_t u = __builtin_bit_cast(uint64_t, v[q]);
      bad |= ((u & 0x7ff0000000000000ull) == 0x7ff0000000000000ull);
      s[q & 3] += v[q] * v[q];
    }
    const double t = wave_sum((s[0] + s[1]) + (s[2] + s[3]));
    if (lane == 0) part[(size_t)S * n + j] = t;
  }
  if (__any(bad) && lane == 0) atomicOr(flag, 1);
}
size_t colsq_dense_doubles(int64_t m, int64_t n) {
  const int64_t ns = std::max<int64_t>(1, (m + CS_ROWS - 1) / CS_ROWS);
  return (size_t)(ns + (ns + COLSQ_SLICE - 1) / COLSQ_SLICE) * (size_t)n;
}
hipError_t launch_colsq_dense(int m, int n, int64_t ld, const double *A, double *part, double *d, int *flag,
                              hipStream_t st) {
  const int ns = std::max(1, (m + CS_ROWS - 1) / CS_ROWS);
  TLS_LAUNCH(PC_SETUP, k_colsq_dense, dim3((n + 3) / 4, std::min(ns, 65535)), dim3(256), 0, st, m, n, ld, A,
             part, flag);
  if (ns <= COLSQ_SLICE) {
    TLS_LAUNCH(PC_SETUP, k_colnorms_parts, dim3((n + 255) / 256), dim3(256), 0, st, n, ns, part, d);
  } else {
    // the slice sums go after the ns rows of slab sums (colsq_dense_doubles)
    const int nsl = (ns + COLSQ_SLICE - 1) / COLSQ_SLICE;
    double *sl = part + (size_t)ns * n;
    TLS_LAUNCH(PC_SETUP, k_colnorms_slices, dim3((n + 255) / 256, nsl), dim3(256), 0, st, n, ns, part, sl);
    TLS_LAUNCH(PC_SETUP, k_colnorms_parts, dim3((n + 255) / 256), dim3(256), 0, st, n, nsl, sl, d);
  }
  return hipGetLastError();
}
hipError_t launch_rowcopy_dense(int m, int n, int64_t ld, const double *A, int64_t ldr, double *At,
                                hipStream_t st) {
  const int64_t ntiles = (int64_t)((m + 63) / 64) * (ldr / 64);
  const int grid = (int)std::min<int64_t>(ntiles, ROWCOPY_WGS);
  if (grid == 0) return hipSuccess;
  TLS_LAUNCH(PC_SETUP, k_rowcopy_dense, dim3(grid), dim3(256), 0, st, m, n, ld, A, ldr, At);
  return hipGetLastError();
}

hipError_t launch_colnorms_csc(int n, const int32_t *col_ptr, const double *cval, double *d,
                               hipStream_t st) {
  TLS_LAUNCH(PC_SETUP, k_colnorms_csc, dim3((n + 3) / 4), dim3(256), 0, st, n, col_ptr, cval, d);
  return hipGetLastError();
}
hipError_t launch_colnorms_dense(int m, int n, int64_t ld, const double *A, double *d,
                                 hipStream_t st) {
  TLS_LAUNCH(PC_SETUP, k_colnorms_dense, dim3((n + 3) / 4), dim3(256), 0, st, m, n, ld, A, d);
  return hipGetLastError();
}

__global__ void k_scale_vectors(int n, int Np, const double *d, int scaled, double *dsc64,
                                float *dsc32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Np) return;
  const double v = (i < n && scaled) ? 1.0 / d[i] : 1.0;
  dsc64[i] = v;
  dsc32[i] = (float)v;
}
hipError_t launch_scale_vectors(int n, int Np, const double *d, int scaled, double *dsc64,
                                float *dsc32, hipStream_t st) {
  TLS_LAUNCH(PC_SETUP, k_scale_vectors, dim3((Np + 255) / 256), dim3(256), 0, st, n, Np, d, scaled,
                     dsc64, dsc32);
  return hipGetLastError();
}

__global__ void k_round(const double *in, int64_t count, int q, double *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) out[i] = quantize(in[i], q);
}
hipError_t launch_round(const double *in, int64_t count, int q, double *out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  TLS_LAUNCH(PC_SETUP, k_round, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, in, count, q, out);
  return hipGetLastError();
}

template <typename C>
__global__ void k_quantize_sparse(int64_t nnz, const int32_t *cols, const double *val,
                                  const double *d, int scaled, int q, C *out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const double v = scaled ? val[e] / d[cols[e]] : val[e];
  out[e] = (C)quantize(v, q);
}
hipError_t launch_quantize_sparse(int64_t nnz, const int32_t *cols, const double *val,
                                  const double *d, int scaled, int q, int compute, void *out,
                                  hipStream_t st) {
  if (nnz <= 0) return hipSuccess;
  const dim3 g((unsigned)((nnz + 255) / 256));
  if (compute == TLS_FP64)
    TLS_LAUNCH(PC_SETUP, k_quantize_sparse<double>, g, dim3(256), 0, st, nnz, cols, val, d, scaled, q,
                       (double *)out);
  else
    TLS_LAUNCH(PC_SETUP, k_quantize_sparse<float>, g, dim3(256), 0, st, nnz, cols, val, d, scaled, q,
                       (float *)out);
  return hipGetLastError();
}

template <typename C>
__global__ void k_quantize_csc(int n, const int32_t *col_ptr, const double *cval, const double *d,
                               int scaled, int q, C *out) {
  const int j = blockIdx.x;
  const double dj = d[j];
  for (int e = col_ptr[j] + threadIdx.x; e < col_ptr[j + 1]; e += blockDim.x) {
    const double v = scaled ? cval[e] / dj : cval[e];
    out[e] = (C)quantize(v, q);
  }
}
hipError_t launch_quantize_csc(int n, const int32_t *col_ptr, const double *cval, const double *d,
                               int scaled, int q, int compute, void *out, hipStream_t st) {
  if (compute == TLS_FP64)
    TLS_LAUNCH(PC_SETUP, k_quantize_csc<double>, dim3(n), dim3(64), 0, st, n, col_ptr, cval, d, scaled,
                       q, (double *)out);
  else
    TLS_LAUNCH(PC_SETUP, k_quantize_csc<float>, dim3(n), dim3(64), 0, st, n, col_ptr, cval, d, scaled,
                       q, (float *)out);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// sparse Gram: column j of the upper triangle, G(k, j) = sum_i A(i,k) A(i,j)
// for k <= j. One wave per column; rows of column j are visited in
// ascending order and the lanes of the wave split the entries of each row
// (distinct columns k), so every G(k, j) is accumulated in row order.
// --------------------------------------------------------------------------
constexpr int GRAM_KC = 2048;   // k-chunk held in LDS per wave

template <typename C>
__global__ __launch_bounds__(256) void k_gram_sparse(int n, int Np, const int32_t *row_ptr,
                                                     const int32_t *col_idx, const C *valq,
                                                     const int32_t *col_ptr,
                                                     const int32_t *row_idx, const C *cvalq, C *G) {
  __shared__ C acc[4][GRAM_KC];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + w;
  if (j >= n) return;   // whole wave leaves together; no block barriers below
  C *a = acc[w];
  const int ca = col_ptr[j], cb = col_ptr[j + 1];
  for (int k0 = 0; k0 <= j; k0 += GRAM_KC) {
    const int k1 = min(j + 1, k0 + GRAM_KC);
    for (int k = k0 + lane; k < k1; k += 64) a[k - k0] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the nonzeros of column j four at a time, one 16-lane group per row:
    // the four rows' loads are in flight together, and the groups add into
    // the accumulator in row order (entries of one row have distinct
    // columns, so the lanes of a group never collide)
    const int grp = lane >> 4, gl = lane & 15;
    for (int t0 = ca; t0 < cb; t0 += 4) {
      const int t = t0 + grp;
      const bool live = t < cb;
      int ra = 0, rb = 0;
      C aij = 0;
      if (live) {
        const int i = row_idx[t];
        aij = cvalq[t];
        ra = row_ptr[i];
        rb = row_ptr[i + 1];
      }
      for (int eb = 0;; eb += 16) {   // 16 entries of each group's row per pass
        const int e = ra + eb + gl;
        const bool have = live && e < rb;
        int k = -1;
        C v = 0;
        if (have) {
          k = col_idx[e];
          v = aij * valq[e];
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          if (grp == g && have && k >= k0 && k < k1) a[k - k0] += v;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (__ballot(live && ra + eb + 16 < rb) == 0) break;   // uniform over the wave
      }
    }
    C *colj = G + (size_t)j * Np;
    for (int k = k0 + lane; k < k1; k += 64) colj[k] = a[k - k0];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}
hipError_t launch_gram_sparse(int m, int n, int Np, const int32_t *row_ptr, const int32_t *col_idx,
                              const void *valq, const int32_t *col_ptr, const int32_t *row_idx,
                              const void *cvalq, int compute, void *G, hipStream_t st) {
  const dim3 g((n + 3) / 4);
  if (compute == TLS_FP64)
    TLS_LAUNCH(PC_GRAM, k_gram_sparse<double>, g, dim3(256), 0, st, n, Np, row_ptr, col_idx,
                       (const double *)valq, col_ptr, row_idx, (const double *)cvalq, (double *)G);
  else
    TLS_LAUNCH(PC_GRAM, k_gram_sparse<float>, g, dim3(256), 0, st, n, Np, row_ptr, col_idx,
                       (const float *)valq, col_ptr, row_idx, (const float *)cvalq, (float *)G);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// dense Gram (VALU): tile (I, J), I <= J, of G = Ahat^T Ahat with
// Ahat = round_q(A D^{-1}) formed on load; 16x16 threads, 4x4 outputs each
// --------------------------------------------------------------------------
template <typename C>
__global__ __launch_bounds__(256) void k_gram_dense(int m, int n, int Np, int64_t ld,
                                                    const double *A, const double *d, int scaled,
                                                    int q, C *G) {
  constexpr int KT = 16;
  __shared__ C As[KT][NB + 1];
  __shared__ C Bs[KT][NB + 1];
  // decode the upper-triangle tile index
  const int l = blockIdx.x;
  int J = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= l) ++J;
  while (J * (J + 1) / 2 > l) --J;
  const int I = l - J * (J + 1) / 2;
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  C acc[4][4] = {};
  // loader mapping: 1024 elements per operand per chunk, 4 per thread
  const int lcol = tid >> 2, lrow = (tid & 3) * 4;
  const int colI = I * NB + lcol, colJ = J * NB + lcol;
  const double sI = (colI < n && scaled) ? 1.0 / d[colI] : 1.0;
  const double sJ = (colJ < n && scaled) ? 1.0 / d[colJ] : 1.0;
  for (int k0 = 0; k0 < m; k0 += KT) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + lrow + u;
      double va = 0, vb = 0;
      if (k < m && colI < n) va = quantize(A[(size_t)colI * ld + k] * sI, q);
      if (k < m && colJ < n) vb = quantize(A[(size_t)colJ * ld + k] * sJ, q);
      As[lrow + u][lcol] = (C)va;
      Bs[lrow + u][lcol] = (C)vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      C a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) { a[x] = As[kk][tr * 4 + x]; b[x] = Bs[kk][tc * 4 + x]; }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int r = I * NB + tr * 4 + x, c = J * NB + tc * 4 + y;
      if (r <= c && c < n) G[(size_t)c * Np + r] = acc[x][y];
    }
}
hipError_t launch_gram_dense(int m, int n, int Np, int64_t ld, const double *A, const double *d,
                             int scaled, int q, int compute, void *G, hipStream_t st) {
  const int N = Np / NB;
  const dim3 g(N * (N + 1) / 2);
  if (compute == TLS_FP64)
    TLS_LAUNCH(PC_GRAM, k_gram_dense<double>, g, dim3(256), 0, st, m, n, Np, ld, A, d, scaled, q,
                       (double *)G);
  else
    TLS_LAUNCH(PC_GRAM, k_gram_dense<float>, g, dim3(256), 0, st, m, n, Np, ld, A, d, scaled, q,
                       (float *)G);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// dense Gram on the matrix cores
//
// G = Ahat^T Ahat (upper tiles) with 128 x 128 output tiles per workgroup
// of four waves (64 x 64 each). FP64 and FP32 inputs (k_gram_mfma): a
// K-chunk of 32 rows of the two column panels is staged in LDS (row = one
// column of Ahat, 32 consecutive entries); the next chunk's global loads
// are in flight while the current one feeds the MFMAs
// (v_mfma_f64_16x16x4_f64, v_mfma_f32_32x32x2_f32). FP16 / BF16 inputs
// (k_gram_mfma16, below): v_mfma_f32_32x32x16 with FP32 accumulation, an
// operand being 8 consecutive k of one column.
// The MFMA's A operand takes the output-column panel and its B operand the
// output-row panel, so that a lane's results lie along a column of the
// column-major G and the stores coalesce.
// Low-precision inputs come from a cast buffer (zero padded to whole
// chunks and tiles, 16-byte vector loads); FP64 reads A itself with
// bounds checks.
// --------------------------------------------------------------------------
typedef __bf16 g_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 g_f16x8 __attribute__((ext_vector_type(8)));
typedef float g_f32x16 __attribute__((ext_vector_type(16)));
typedef double g_f64x4 __attribute__((ext_vector_type(4)));

constexpr int GT = 128, GKC = 32;

template <typename T> __device__ inline T cast_bits(double v);
template <> __device__ inline float cast_bits<float>(double v) {
  return __builtin_bit_cast(float, f64_to_f32_bits(v));
}
template <> __device__ inline half_t cast_bits<half_t>(double v) { return half_t{f64_to_f16_bits(v)}; }
template <> __device__ inline bf16_t cast_bits<bf16_t>(double v) { return bf16_t{f64_to_bf16_bits(v)}; }

// out (mp x n128, column-major) = round(A D^{-1}) (or round(A)), zero padding
template <typename T>
__global__ __launch_bounds__(256) void k_cast_dense(int m, int n, int64_t ld, const double *A,
                                                    const double *d, int scaled, int mp, T *out) {
  const int c = blockIdx.y;
  const double sc = (c < n && scaled) ? 1.0 / d[c] : 1.0;
  const double *col = A + (size_t)c * ld;
  T *o = out + (size_t)c * mp;
  for (int r = blockIdx.x * 1024 + threadIdx.x; r < min(mp, (int)(blockIdx.x + 1) * 1024); r += 256) {
    const double v = (r < m && c < n) ? col[r] * sc : 0.0;
    o[r] = cast_bits<T>(v);
  }
}


// Grid: (segment, tile) jobs, tile l = J (J + 1) / 2 + I of the upper 128 x
// 128 tiles, rows [seg seglen, (seg + 1) seglen) of A. One segment: the
// tile goes to G. Several: the workgroup writes its unscaled FP64 sums to
// part (tile-major, 128 x 128 per job, column c - c0 at stride 128) and
// k_gram_reduce64 adds the segments in order.
template <typename T, typename C>
__global__ __launch_bounds__(256) void k_gram_mfma(int m, int n, int64_t ld, const T *A, int Np, C *G,
                                                   const double *d, int scaled, int seglen, int nseg,
                                                   double *part) {
  constexpr bool F64 = std::is_same<T, double>::value;
  constexpr int PADE = 16 / (int)sizeof(T);
  constexpr int RL = GKC + PADE;                     // LDS row length (elements)
  __shared__ __attribute__((aligned(16))) T Ps[GT][RL];   // output-column panel (J)
  __shared__ __attribute__((aligned(16))) T Qs[GT][RL];   // output-row panel (I)
  const int ntl = (int)gridDim.x / nseg;
  const int l = (int)blockIdx.x % ntl, seg = (int)blockIdx.x / ntl;
  int J = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= l) ++J;
  while (J * (J + 1) / 2 > l) --J;
  const int I = l - J * (J + 1) / 2;
  const bool diag = (I == J);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;                 // wave's 64 x 64 block (rows, cols)
  const int r0 = I * GT, c0 = J * GT;

  // ---- global -> register staging --------------------------------------
  constexpr int VPC = GKC * (int)sizeof(T) / 16;     // 16-byte vectors per column chunk
  constexpr int NV = GT * VPC / 256;                 // per thread per panel (cast buffer)
  uint4 pv[F64 ? 1 : NV], qv[F64 ? 1 : NV];
  double pe[F64 ? 16 : 1], qe[F64 ? 16 : 1];
  auto fetch = [&](int k0) {
    if constexpr (F64) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e = tid + 256 * i, c = e / GKC, r = k0 + e % GKC;
        pe[i] = (r < m && c0 + c < n) ? ((const double *)A)[(size_t)(c0 + c) * ld + r] : 0.0;
        qe[i] = (!diag && r < m && r0 + c < n) ? ((const double *)A)[(size_t)(r0 + c) * ld + r] : 0.0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int v = tid + 256 * i, c = v / VPC, o = (v % VPC) * (16 / (int)sizeof(T));
        pv[i] = *(const uint4 *)(A + (size_t)(c0 + c) * ld + k0 + o);
        if (!diag) qv[i] = *(const uint4 *)(A + (size_t)(r0 + c) * ld + k0 + o);
      }
    }
  };
  auto stage = [&]() {
    if constexpr (F64) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e = tid + 256 * i, c = e / GKC, r = e % GKC;
        Ps[c][r] = pe[i];
        if (!diag) Qs[c][r] = qe[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int v = tid + 256 * i, c = v / VPC, o = (v % VPC) * (16 / (int)sizeof(T));
        *(uint4 *)&Ps[c][o] = pv[i];
        if (!diag) *(uint4 *)&Qs[c][o] = qv[i];
      }
    }
  };
  const T (*Qp)[RL] = diag ? Ps : Qs;

  // ---- accumulators ------------------------------------------------------
  g_f32x16 acc32[2][2];
  g_f64x4 acc64[4][4];
  if constexpr (F64) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc64[t][u] = g_f64x4{0, 0, 0, 0};
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc32[t][u][q] = 0.0f;
  }

  // FP32 accumulators are folded into FP64 sums after every chunk, so that
  // the accumulation error over the m rows stays near that of one chunk
  // (about sqrt(32) u_32 relative) instead of growing like sqrt(m) u_32
  constexpr int FLUSH = 1;
  double sum64[F64 ? 1 : 2][F64 ? 1 : 2][F64 ? 1 : 16];
  if constexpr (!F64) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 16; ++q) sum64[t][u][q] = 0.0;
  }
  auto flush = [&]() {
    if constexpr (!F64) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            sum64[t][u][q] += (double)acc32[t][u][q];
            acc32[t][u][q] = 0.0f;
          }
    }
  };
  // segments are whole GKC-row chunks, so only the last one can be ragged
  const int kall = F64 ? m : ((m + GKC - 1) / GKC) * GKC;
  const int kbeg = seg * seglen, kend = min(kall, kbeg + seglen);
  int chunk = 0;
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += GKC) {
    if (++chunk == FLUSH) { flush(); chunk = 0; }
    __syncthreads();                 // previous chunk fully consumed
    stage();
    __syncthreads();
    if (k0 + GKC < kend) fetch(k0 + GKC);
    if constexpr (F64) {
#pragma unroll
      for (int s = 0; s < GKC / 4; ++s) {
        double a[4], b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          a[t] = Ps[wc * 64 + t * 16 + (lane & 15)][s * 4 + (lane >> 4)];
          b[t] = Qp[wr * 64 + t * 16 + (lane & 15)][s * 4 + (lane >> 4)];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc64[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc64[t][u], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < GKC / 2; ++s) {
        float a[2], b[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          a[t] = Ps[wc * 64 + t * 32 + (lane & 31)][s * 2 + (lane >> 5)];
          b[t] = Qp[wr * 64 + t * 32 + (lane & 31)][s * 2 + (lane >> 5)];
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int u = 0; u < 2; ++u)
            acc32[t][u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], b[u], acc32[t][u], 0, 0, 0);
      }
    }
  }

  // ---- epilogue: D(i, j) = G(c0 + .. i, r0 + .. j), stored at G[c * Np + r], r <= c
  if constexpr (F64) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = c0 + wc * 64 + t * 16 + 4 * q + (lane >> 4);
          const int r = r0 + wr * 64 + u * 16 + (lane & 15);
          if (nseg > 1) {
            part[(size_t)blockIdx.x * GT * GT + (size_t)(c - c0) * GT + (r - r0)] = acc64[t][u][q];
          } else if (r <= c && c < Np) {
            // FP64 reads A unscaled: H = D^{-1} (A^T A) D^{-1} on output
            double v = acc64[t][u][q];
            if (scaled && c < n) v *= (1.0 / d[r]) * (1.0 / d[c]);
            G[(size_t)c * Np + r] = (C)v;
          }
        }
  } else {
    flush();
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int c = c0 + wc * 64 + t * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
          const int r = r0 + wr * 64 + u * 32 + (lane & 31);
          if (nseg > 1) part[(size_t)blockIdx.x * GT * GT + (size_t)(c - c0) * GT + (r - r0)] = sum64[t][u][q];
          else if (r <= c && c < Np) G[(size_t)c * Np + r] = (C)sum64[t][u][q];
        }
  }
}

// ---- 16-bit inputs: K-split Gram on paired tiles --------------------------
// FP16 / BF16 inputs (and the two planes of the split BF16 input) go through
// their own kernel. A workgroup of eight waves computes two upper 128 x 128
// tiles of one tile column J, (I0, J) and (I0 + 1, J) with I0 even, over one
// segment of the K range: three 128-column panels (J, I0, I0 + 1) per 64-row
// chunk, so a chunk's 48 KB feed 4.2 MFLOP (twice the flops per byte of a
// single tile). Each wave owns a 64 x 64 quarter of one tile (2 x 2
// v_mfma_f32_32x32x16 blocks). Chunks are prefetched two ahead into
// registers and double buffered in LDS, one barrier per chunk; with about
// 110 KB of LDS and 200 VGPRs the kernel runs one workgroup (two waves per
// SIMD) per CU, and the host picks the segment length so that the
// (pair, segment) jobs fill whole rounds of the chip.
//
// Accumulation: the MFMA accumulates 128 rows (G16FOLD chunks) from zero,
// and that partial is added into an FP32 sum with round-to-nearest. The
// matrix cores' own running sum drifts with the number of accumulations
// (over 8192 rows it moved the diagonal of the scaled 65536 x 4096 planted
// Gram matrix, whose smallest eigenvalue is near 7e-5, by about 1% of that
// eigenvalue and cost the BF16 path 10 RQIs); restarting it every 128 rows
// bounds that drift, and the second level adds only rounding errors of
// random sign. A segment's sum goes to a scratch tile; k_gram_reduce adds
// the segments in FP64 in a fixed order.
//
// Work order: dispatch id L runs on XCD L mod 8; each XCD takes a contiguous
// range of the (segment, pair) order, so the workgroups resident on one XCD
// work on neighbouring pairs of one segment and share its panels in their L2.
constexpr int G16K = 64, G16RL = G16K + 8, G16FOLD = 2, G16LANES = 512;
constexpr int G16NV = 3 * GT * G16K * 2 / 16 / G16LANES;   // 16-byte loads per thread per chunk (6)

// upper tile (I, J), I <= J, of linear index l = J (J + 1) / 2 + I
__device__ inline void gram_tile_of(int l, int &I, int &J) {
  J = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= l) ++J;
  while (J * (J + 1) / 2 > l) --J;
  I = l - J * (J + 1) / 2;
}

// pairs in tile columns < J: ceil((j + 1) / 2) per column j
__host__ __device__ inline int gram_pairs_before(int J) {
  const int a = J >> 1;
  return (J & 1) ? (a + 1) * (a + 1) : a * (a + 1);
}
__device__ inline void gram_pair_of(int p, int &I0, int &J) {
  int j = (int)(2.0 * sqrt((double)p));
  if (j > 0) --j;
  while (gram_pairs_before(j + 1) <= p) ++j;
  while (j > 0 && gram_pairs_before(j) > p) --j;
  J = j;
  I0 = 2 * (p - gram_pairs_before(j));
}

inline int64_t gram_rows_padded(int64_t m) { return ((m + G16K - 1) / G16K) * G16K; }

struct GramPlan { int nseg, seglen, npairs; };
// segment length (a multiple of 64 rows, at least 1024 unless m is smaller)
// that minimises rounds x rows per round for one workgroup per CU
static GramPlan gram_plan(int64_t m, int64_t n, int cus) {
  const int64_t mp = gram_rows_padded(m);
  const int NT = (int)((n + GT - 1) / GT);
  GramPlan best{1, (int)mp, gram_pairs_before(NT)};
  int64_t best_cost = LLONG_MAX;
  for (int ns = 1; ns <= 64; ++ns) {
    const int64_t len = ((mp + ns - 1) / ns + G16K - 1) / G16K * G16K;
    if (ns > 1 && len < 1024) break;
    const int used = (int)((mp + len - 1) / len);
    if (used != ns) continue;
    const int64_t jobs = (int64_t)best.npairs * ns;
    const int64_t cost = (jobs + cus - 1) / cus * len;
    if (cost < best_cost) { best_cost = cost; best.nseg = ns; best.seglen = (int)len; }
  }
  return best;
}
static int device_cus() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  return cus;
}
// the partial tiles are sized for the largest plan any device could pick
static int gram_max_segments(int64_t m) { return std::max(1, (int)((gram_rows_padded(m) + 1023) / 1024)); }
inline size_t gram_cast_only_bytes(int64_t m, int64_t n) {
  const int64_t n128 = ((n + GT - 1) / GT) * GT;
  return ((size_t)gram_rows_padded(m) * n128 * 4 + 255) / 256 * 256;   // FP32-sized
}

// A D^{-1} rounded to 16 bits in the chunk-major layout the Gram kernels
// read: element (r, c) at ((r / 64) n128 + c) 64 + r % 64, zero padding (so
// a 64-row chunk of all columns is contiguous, and a panel's chunk is 16 KB
// in one piece for the Gram kernel). A wave takes CAST_ROWS consecutive rows
// of one column: 32 loads of 512 contiguous bytes in flight per wave (the
// access that streams A at close to the HBM rate), the rounded values
// through LDS, then 16-byte stores of 8 consecutive rows (each 64-row chunk
// of the column is 128 contiguous bytes of the output).
// SPLIT: the pair hi = bf16(v), lo = bf16(v - hi) into out and lo.
template <typename T> __device__ inline uint16_t bits16(double v);
template <> __device__ inline uint16_t bits16<half_t>(double v) { return f64_to_f16_bits(v); }
template <> __device__ inline uint16_t bits16<bf16_t>(double v) { return f64_to_bf16_bits(v); }
constexpr int CAST_ROWS = 2048;
template <typename T, bool SPLIT>
__global__ __launch_bounds__(256) void k_cast16(int m, int n, int64_t ld, const double *A, const double *d,
                                                int scaled, int mp, int n128, T *out, T *lo) {
  __shared__ __align__(16) uint16_t sh[4][CAST_ROWS];
  __shared__ __align__(16) uint16_t sl[SPLIT ? 4 : 1][SPLIT ? CAST_ROWS : 8];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.y * 4 + w;                 // < n128
  const int rb = blockIdx.x * CAST_ROWS;            // < mp
  double v[32];
  if (c < n) {
    const double sc = scaled ? 1.0 / d[c] : 1.0;
    const double *src = A + (size_t)c * ld + rb;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int i = lane + 64 * q;
      v[q] = (rb + i < m) ? __builtin_nontemporal_load(src + i) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] *= sc;
  } else {
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] = 0.0;
  }
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const uint16_t h = bits16<T>(v[q]);
    sh[w][lane + 64 * q] = h;
    if constexpr (SPLIT) sl[w][lane + 64 * q] = f64_to_bf16_bits(v[q] - (double)bf16_bits_to_float(h));
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < CAST_ROWS / 512; ++t) {
    const int p = lane + 64 * t;                    // 8 rows: rb + 8p ..
    const int r = rb + 8 * p;
    if (r < mp) {                                   // mp is a multiple of 64
      const size_t o = ((size_t)(r / G16K) * n128 + c) * G16K + (r % G16K);
      *reinterpret_cast<uint4 *>(out + o) = *reinterpret_cast<const uint4 *>(&sh[w][8 * p]);
      if constexpr (SPLIT) *reinterpret_cast<uint4 *>(lo + o) = *reinterpret_cast<const uint4 *>(&sl[w][8 * p]);
    }
  }
}

template <typename T>
__device__ inline g_f32x16 mfma16(uint4 a, uint4 b, g_f32x16 c) {
  if constexpr (std::is_same<T, bf16_t>::value)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(g_bf16x8, a),
                                                    __builtin_bit_cast(g_bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(g_f16x8, a),
                                                   __builtin_bit_cast(g_f16x8, b), c, 0, 0, 0);
}

template <typename T>
__global__ __launch_bounds__(G16LANES) void k_gram_mfma16(int mp, const T *A, float *part, int NT,
                                                          int seglen, int npairs, int nseg) {
  // stage b holds panel J in rows 0..127, I0 in 128..255, I0 + 1 in 256..383
  __shared__ __attribute__((aligned(16))) T S[2][3 * GT][G16RL];
  const int ntiles = NT * (NT + 1) / 2;
  // XCD-contiguous work order
  const int total = npairs * nseg, L = blockIdx.x;
  const int xcd = L & 7, k = L >> 3, q8 = total >> 3, r8 = total & 7;
  const int Wl = xcd * q8 + min(xcd, r8) + k;
  const int seg = Wl / npairs, p = Wl - seg * npairs;
  int I0, J;
  gram_pair_of(p, I0, J);
  const int I1 = I0 + 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int h = w >> 2, wr = (w >> 1) & 1, wc = w & 1;
  const bool live = (h == 0) || (I1 <= J);          // tile (I0 + h, J) is an upper tile
  const int kbeg = seg * seglen;
  const int nch = (min(mp, kbeg + seglen) - kbeg) / G16K;
  const size_t cstride = (size_t)NT * GT * G16K;     // elements per 64-row chunk
  // thread tid moves 16 bytes of column (tid >> 3) + 64 (i & 1) of panel
  // i >> 1 (J, I0, I0 + 1) at offset 8 (tid & 7) in load slot i = 0..5
  const int colJ = J * GT, colI0 = I0 * GT, colI1 = min(I1, NT - 1) * GT;
  const int crow = tid >> 3, coff = (tid & 7) * 8;
  const T *gbase[G16NV];
#pragma unroll
  for (int i = 0; i < G16NV; ++i) {
    const int pn = i >> 1, c = crow + 64 * (i & 1);
    gbase[i] = A + (size_t)kbeg * NT * GT + (size_t)((pn == 0 ? colJ : pn == 1 ? colI0 : colI1) + c) * G16K + coff;
  }

  g_f32x16 acc[2][2];
  float sum[2][2][16];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        acc[t][u][q] = 0.0f;
        sum[t][u][q] = 0.0f;
      }
  // register prefetch buffers (named, so that they stay in VGPRs)
  uint4 a0, a1, a2, a3, a4, a5, b0, b1, b2, b3, b4, b5;
#define G16_FETCH(X, ch)                                                          \
  do {                                                                            \
    const size_t off_ = (size_t)(ch) * cstride;                                   \
    X##0 = *(const uint4 *)(gbase[0] + off_); X##1 = *(const uint4 *)(gbase[1] + off_); \
    X##2 = *(const uint4 *)(gbase[2] + off_); X##3 = *(const uint4 *)(gbase[3] + off_); \
    X##4 = *(const uint4 *)(gbase[4] + off_); X##5 = *(const uint4 *)(gbase[5] + off_); \
  } while (0)
#define G16_STAGE(X, b)                                                           \
  do {                                                                            \
    *(uint4 *)&S[b][0 * GT + crow][coff] = X##0;                                  \
    *(uint4 *)&S[b][0 * GT + crow + 64][coff] = X##1;                             \
    *(uint4 *)&S[b][1 * GT + crow][coff] = X##2;                                  \
    *(uint4 *)&S[b][1 * GT + crow + 64][coff] = X##3;                             \
    *(uint4 *)&S[b][2 * GT + crow][coff] = X##4;                                  \
    *(uint4 *)&S[b][2 * GT + crow + 64][coff] = X##5;                             \
  } while (0)
  auto fold = [&]() {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          sum[t][u][q] += acc[t][u][q];
          acc[t][u][q] = 0.0f;
        }
  };
  const int arow = wc * 64 + (lane & 31), brow = (1 + h) * GT + wr * 64 + (lane & 31);
  const int koff = 8 * (lane >> 5);
  auto compute = [&](int b) {
    if (!live) return;
#pragma unroll
    for (int s = 0; s < G16K / 16; ++s) {
      uint4 a[2], bb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = *(const uint4 *)&S[b][arow + t * 32][s * 16 + koff];
        bb[t] = *(const uint4 *)&S[b][brow + t * 32][s * 16 + koff];
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[t][u] = mfma16<T>(a[t], bb[u], acc[t][u]);
    }
  };

  // chunk c is prefetched into a* (c even) or b* (c odd). Iteration it
  // computes chunk it from LDS buffer it & 1, stages chunk it + 1 into the
  // other buffer (last read in iteration it - 1) and refills the registers
  // it came from with chunk it + 3
  if (nch > 0) G16_FETCH(a, 0);
  if (nch > 1) G16_FETCH(b, 1);
  if (nch > 0) G16_STAGE(a, 0);
  if (nch > 2) G16_FETCH(a, 2);
  __syncthreads();
  for (int it = 0; it < nch; it += 2) {
    compute(0);
    if (it + 1 < nch) {
      G16_STAGE(b, 1);
      if (it + 3 < nch) G16_FETCH(b, it + 3);
    }
    if ((it + 1) % G16FOLD == 0) fold();
    __syncthreads();
    if (it + 1 >= nch) break;
    compute(1);
    if (it + 2 < nch) {
      G16_STAGE(a, 0);
      if (it + 4 < nch) G16_FETCH(a, it + 4);
    }
    if ((it + 2) % G16FOLD == 0) fold();
    __syncthreads();
  }
#undef G16_FETCH
#undef G16_STAGE
  fold();
  if (!live) return;
  // partial tile, column-major inside the tile: part[seg][l][c_local][r_local]
  const int l = J * (J + 1) / 2 + I0 + h;
  float *dst = part + ((size_t)seg * ntiles + l) * GT * GT;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int cl = wc * 64 + t * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        const int rl = wr * 64 + u * 32 + (lane & 31);
        dst[cl * GT + rl] = sum[t][u][q];
      }
}

// ---- split BF16 inputs: a = hi + lo ------------------------------------------
// Each entry a of A D^{-1} is carried as hi = bf16(a) and lo = bf16(a - hi)
// (a - hi is exact in FP64), two planes in the chunk-major layout of the
// 16-bit cast (k_cast16 with SPLIT). The Gram matrix is
// hi^T hi + hi^T lo + lo^T hi: three BF16 MFMAs into one FP32 accumulator per
// block step, so the factor sees the entries to 2^-16 relative (hi + lo) at
// the BF16 matrix-core rate. The kernel is the paired-tile kernel above with
// 32-row half chunks (the two planes of three panels fill 123 KB of LDS
// double buffered) and the same two-level accumulation (the MFMA partial
// restarted every 128 rows).
constexpr int G3K = 32, G3RL = G3K + 8, G3FOLD = 4;   // half chunks; fold every 128 rows

__global__ __launch_bounds__(G16LANES) void k_gram_mfma16x3(int mp, const bf16_t *Ahi, const bf16_t *Alo,
                                                            float *part, int NT, int seglen, int npairs,
                                                            int nseg) {
  // stage b: rows 0..127 panel J hi, 128..255 J lo, 256.. I0 hi, I0 lo, I0+1 hi, I0+1 lo
  __shared__ __attribute__((aligned(16))) bf16_t S[2][6 * GT][G3RL];
  const int ntiles = NT * (NT + 1) / 2;
  const int total = npairs * nseg, L = blockIdx.x;
  const int xcd = L & 7, k = L >> 3, q8 = total >> 3, r8 = total & 7;
  const int Wl = xcd * q8 + min(xcd, r8) + k;
  const int seg = Wl / npairs, p = Wl - seg * npairs;
  int I0, J;
  gram_pair_of(p, I0, J);
  const int I1 = I0 + 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int h = w >> 2, wr = (w >> 1) & 1, wc = w & 1;
  const bool live = (h == 0) || (I1 <= J);
  const int kbeg = seg * seglen;
  const int nhc = 2 * ((min(mp, kbeg + seglen) - kbeg) / G16K);    // 32-row half chunks
  const size_t cstride = (size_t)NT * GT * G16K;                    // elements per 64-row chunk
  // load slot i (0..5): panel i >> 1, plane i & 1; thread tid moves 16 bytes
  // (part tid & 3 of the 32-row segment) of column tid >> 2
  const int colJ = J * GT, colI0 = I0 * GT, colI1 = min(I1, NT - 1) * GT;
  const int ccol = tid >> 2, cpart = (tid & 3) * 8;
  const bf16_t *gbase[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int pn = i >> 1;
    const bf16_t *plane = (i & 1) ? Alo : Ahi;
    gbase[i] = plane + (size_t)kbeg * NT * GT + (size_t)((pn == 0 ? colJ : pn == 1 ? colI0 : colI1) + ccol) * G16K +
               cpart;
  }
  g_f32x16 acc[2][2];
  float sum[2][2][16];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        acc[t][u][q] = 0.0f;
        sum[t][u][q] = 0.0f;
      }
  uint4 a0, a1, a2, a3, a4, a5, b0, b1, b2, b3, b4, b5;
  // half chunk hc: 64-row chunk hc >> 1, rows 32 (hc & 1) onwards
#define G3_FETCH(X, hc)                                                                       \
  do {                                                                                        \
    const size_t off_ = (size_t)((hc) >> 1) * cstride + (size_t)((hc) & 1) * G3K;             \
    X##0 = *(const uint4 *)(gbase[0] + off_); X##1 = *(const uint4 *)(gbase[1] + off_);       \
    X##2 = *(const uint4 *)(gbase[2] + off_); X##3 = *(const uint4 *)(gbase[3] + off_);       \
    X##4 = *(const uint4 *)(gbase[4] + off_); X##5 = *(const uint4 *)(gbase[5] + off_);       \
  } while (0)
#define G3_STAGE(X, b)                                                                        \
  do {                                                                                        \
    *(uint4 *)&S[b][0 * GT + ccol][cpart] = X##0; *(uint4 *)&S[b][1 * GT + ccol][cpart] = X##1; \
    *(uint4 *)&S[b][2 * GT + ccol][cpart] = X##2; *(uint4 *)&S[b][3 * GT + ccol][cpart] = X##3; \
    *(uint4 *)&S[b][4 * GT + ccol][cpart] = X##4; *(uint4 *)&S[b][5 * GT + ccol][cpart] = X##5; \
  } while (0)
  auto fold = [&]() {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          sum[t][u][q] += acc[t][u][q];
          acc[t][u][q] = 0.0f;
        }
  };
  // A operand: panel J (hi rows 0.., lo rows 128..); B operand: panel I0 + h
  const int arow = wc * 64 + (lane & 31), brow = (2 + 2 * h) * GT + wr * 64 + (lane & 31);
  const int koff = 8 * (lane >> 5);
  auto compute = [&](int b) {
    if (!live) return;
#pragma unroll
    for (int s = 0; s < G3K / 16; ++s) {
      uint4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ah[t] = *(const uint4 *)&S[b][arow + t * 32][s * 16 + koff];
        al[t] = *(const uint4 *)&S[b][GT + arow + t * 32][s * 16 + koff];
        bh[t] = *(const uint4 *)&S[b][brow + t * 32][s * 16 + koff];
        bl[t] = *(const uint4 *)&S[b][GT + brow + t * 32][s * 16 + koff];
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          acc[t][u] = mfma16<bf16_t>(ah[t], bh[u], acc[t][u]);
          acc[t][u] = mfma16<bf16_t>(ah[t], bl[u], acc[t][u]);
          acc[t][u] = mfma16<bf16_t>(al[t], bh[u], acc[t][u]);
        }
    }
  };
  if (nhc > 0) G3_FETCH(a, 0);
  if (nhc > 1) G3_FETCH(b, 1);
  if (nhc > 0) G3_STAGE(a, 0);
  if (nhc > 2) G3_FETCH(a, 2);
  __syncthreads();
  for (int it = 0; it < nhc; it += 2) {
    compute(0);
    if (it + 1 < nhc) {
      G3_STAGE(b, 1);
      if (it + 3 < nhc) G3_FETCH(b, it + 3);
    }
    if ((it + 1) % G3FOLD == 0) fold();
    __syncthreads();
    if (it + 1 >= nhc) break;
    compute(1);
    if (it + 2 < nhc) {
      G3_STAGE(a, 0);
      if (it + 4 < nhc) G3_FETCH(a, it + 4);
    }
    if ((it + 2) % G3FOLD == 0) fold();
    __syncthreads();
  }
#undef G3_FETCH
#undef G3_STAGE
  fold();
  if (!live) return;
  const int l = J * (J + 1) / 2 + I0 + h;
  float *dst = part + ((size_t)seg * ntiles + l) * GT * GT;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int cl = wc * 64 + t * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        const int rl = wr * 64 + u * 32 + (lane & 31);
        dst[cl * GT + rl] = sum[t][u][q];
      }
}

// G (upper, column-major, FP32) = sum over segments of the partial tiles,
// added in FP64 in segment order. Grid (tiles, 4): a workgroup takes a
// quarter of a tile, a thread four consecutive entries (16-byte loads) in
// four places, with the segment loads of each group issued before the adds.
__global__ __launch_bounds__(256) void k_gram_reduce(const float *part, int nseg, int NT, int Np, float *G) {
  const int l = blockIdx.x, ntiles = NT * (NT + 1) / 2;
  int I, J;
  gram_tile_of(l, I, J);
  const size_t sstride = (size_t)ntiles * GT * GT;      // floats between segments
  const float *base = part + (size_t)l * GT * GT;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = blockIdx.y * (GT * GT / 4) + i * 1024 + threadIdx.x * 4;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = 0;
    for (; k + 4 <= nseg; k += 4) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = *(const float4 *)(base + (size_t)(k + u) * sstride + e);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s0 += (double)v[u].x; s1 += (double)v[u].y; s2 += (double)v[u].z; s3 += (double)v[u].w;
      }
    }
    for (; k < nseg; ++k) {
      const float4 v = *(const float4 *)(base + (size_t)k * sstride + e);
      s0 += (double)v.x; s1 += (double)v.y; s2 += (double)v.z; s3 += (double)v.w;
    }
    const int c = J * GT + e / GT, r = I * GT + e % GT;
    if (c < Np) {
      float *g = G + (size_t)c * Np + r;
      if (r + 0 <= c) g[0] = (float)s0;
      if (r + 1 <= c) g[1] = (float)s1;
      if (r + 2 <= c) g[2] = (float)s2;
      if (r + 3 <= c) g[3] = (float)s3;
    }
  }
}

// the FP64 / FP32 Gram's segments: FP64 partial tiles, added in segment
// order; the FP64 input's scaling H = D^{-1} (A^T A) D^{-1} is applied here
template <typename C>
__global__ __launch_bounds__(256) void k_gram_reduce64(const double *part, int nseg, int NT, int n, int Np, C *G,
                                                       const double *d, int scaled) {
  const int l = blockIdx.x, ntiles = NT * (NT + 1) / 2;
  int I, J;
  gram_tile_of(l, I, J);
  const size_t sstride = (size_t)ntiles * GT * GT;
  const double *base = part + (size_t)l * GT * GT;
  const int e0 = blockIdx.y * (GT * GT / 4);
  for (int e = e0 + threadIdx.x; e < e0 + GT * GT / 4; e += 256) {
    double v = 0.0;
    for (int k = 0; k < nseg; ++k) v += base[(size_t)k * sstride + e];
    const int c = J * GT + e / GT, r = I * GT + e % GT;
    if (r <= c && c < Np) {
      if (scaled && c < n) v *= (1.0 / d[r]) * (1.0 / d[c]);
      G[(size_t)c * Np + r] = (C)v;
    }
  }
}

// The FP64 / FP32 kernel holds two workgroups per CU (about 200 VGPRs per
// wave, 70 KB of LDS): with one workgroup per 128 x 128 tile over all m rows,
// 528 tiles (n = 4096) fill 512 slots once and then 16 of them, and 36 tiles
// (n = 1024) hold a seventh of the chip. The rows are cut into segments
// (whole 64-row multiples, at least 1024 rows) so that the jobs fill whole
// rounds of the slots, within a budget for the partial tiles.
constexpr size_t GRAM64_PART_BYTES = 640ull << 20;
static int gram64_seg_cap(int64_t m, int64_t n) {
  const int64_t NT = (n + GT - 1) / GT;
  const size_t per = (size_t)(NT * (NT + 1) / 2) * GT * GT * 8;
  return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)(GRAM64_PART_BYTES / per), gram_max_segments(m)));
}
size_t gram_part64_bytes(int64_t m, int64_t n) {
  const int cap = gram64_seg_cap(m, n);
  const int64_t NT = (n + GT - 1) / GT;
  return cap > 1 ? (size_t)cap * (NT * (NT + 1) / 2) * GT * GT * 8 : 0;
}
struct Gram64Plan { int nseg, seglen; };
static Gram64Plan gram64_plan(int64_t m, int64_t n, int cus, bool have_part) {
  const int64_t kall = ((m + GKC - 1) / GKC) * GKC;
  const int64_t NT = (n + GT - 1) / GT, ntiles = NT * (NT + 1) / 2, slots = 2 * (int64_t)cus;
  Gram64Plan best{1, (int)kall};
  if (!have_part) return best;
  int64_t best_cost = LLONG_MAX;
  const int cap = gram64_seg_cap(m, n);
  for (int ns = 1; ns <= cap; ++ns) {
    const int64_t len = ((kall + ns - 1) / ns + 63) / 64 * 64;
    if (ns > 1 && len < 1024) break;
    if ((kall + len - 1) / len != ns) continue;
    const int64_t cost = (ntiles * ns + slots - 1) / slots * len;
    if (cost < best_cost) { best_cost = cost; best.nseg = ns; best.seglen = (int)len; }
  }
  return best;
}

size_t gram_cast_bytes(int64_t m, int64_t n) {
  const int64_t NT = (n + GT - 1) / GT;
  // the cast (room for the widest low-precision input, FP32) and the
  // segment partials of the 16-bit kernel
  return gram_cast_only_bytes(m, n) + (size_t)gram_max_segments(m) * (NT * (NT + 1) / 2) * GT * GT * 4;
}

hipError_t launch_gram_mfma(int m, int n, int Np, int64_t ld, const double *A, const double *d,
                            int scaled, int q, void *cast, void *G, void *gpart, hipStream_t st) {
  const int NT = (n + GT - 1) / GT;
  const Gram64Plan g64 = gram64_plan(m, n, device_cus(), gpart != nullptr);
  const dim3 g((unsigned)(NT * (NT + 1) / 2 * g64.nseg));
  const dim3 gr((unsigned)(NT * (NT + 1) / 2), 4);
  double *p64 = (double *)gpart;
  if (q == TLS_FP64) {
    TLS_LAUNCH(PC_GRAM, (k_gram_mfma<double, double>), g, dim3(256), 0, st, m, n, ld, A, Np, (double *)G,
               d, scaled, g64.seglen, g64.nseg, p64);
    if (g64.nseg > 1)
      TLS_LAUNCH(PC_GRAM, k_gram_reduce64<double>, gr, dim3(256), 0, st, p64, g64.nseg, NT, n, Np, (double *)G,
                 d, scaled);
    return hipGetLastError();
  }
  const int mp = (int)gram_rows_padded(m);
  const int n128 = NT * GT;
  const int ntiles = NT * (NT + 1) / 2;
  const GramPlan gp = gram_plan(m, n, device_cus());
  const int nseg = gp.nseg;
  float *part = (float *)((char *)cast + gram_cast_only_bytes(m, n));
  const dim3 gc((unsigned)((mp + 1023) / 1024), (unsigned)n128);
  const dim3 g8((unsigned)((mp + CAST_ROWS - 1) / CAST_ROWS), (unsigned)(n128 / 4));
  const dim3 g16((unsigned)(gp.npairs * nseg));
  switch (q) {
    case TLS_FP32:
      TLS_LAUNCH(PC_GRAM, k_cast_dense<float>, gc, dim3(256), 0, st, m, n, ld, A, d, scaled, mp, (float *)cast);
      TLS_LAUNCH(PC_GRAM, (k_gram_mfma<float, float>), g, dim3(256), 0, st, m, n, (int64_t)mp,
                 (const float *)cast, Np, (float *)G, d, 0, g64.seglen, g64.nseg, p64);
      if (g64.nseg > 1)
        TLS_LAUNCH(PC_GRAM, k_gram_reduce64<float>, gr, dim3(256), 0, st, p64, g64.nseg, NT, n, Np, (float *)G,
                   d, 0);
      break;
    case TLS_FP16:
      TLS_LAUNCH(PC_GRAM, (k_cast16<half_t, false>), g8, dim3(256), 0, st, m, n, ld, A, d, scaled, mp, n128,
                 (half_t *)cast, (half_t *)nullptr);
      TLS_LAUNCH(PC_GRAM, k_gram_mfma16<half_t>, g16, dim3(G16LANES), 0, st, mp, (const half_t *)cast, part, NT,
                 gp.seglen, gp.npairs, nseg);
      TLS_LAUNCH(PC_GRAM, k_gram_reduce, dim3(ntiles, 4), dim3(256), 0, st, (const float *)part, nseg, NT, Np,
                 (float *)G);
      break;
    case TLS_BF16X3: {
      bf16_t *hi = (bf16_t *)cast, *lo = hi + (size_t)mp * n128;
      TLS_LAUNCH(PC_GRAM, (k_cast16<bf16_t, true>), g8, dim3(256), 0, st, m, n, ld, A, d, scaled, mp, n128,
                 hi, lo);
      TLS_LAUNCH(PC_GRAM, k_gram_mfma16x3, g16, dim3(G16LANES), 0, st, mp, (const bf16_t *)hi, (const bf16_t *)lo,
                 part, NT, gp.seglen, gp.npairs, nseg);
      TLS_LAUNCH(PC_GRAM, k_gram_reduce, dim3(ntiles, 4), dim3(256), 0, st, (const float *)part, nseg, NT, Np,
                 (float *)G);
      break;
    }
    default:
      TLS_LAUNCH(PC_GRAM, (k_cast16<bf16_t, false>), g8, dim3(256), 0, st, m, n, ld, A, d, scaled, mp, n128,
                 (bf16_t *)cast, (bf16_t *)nullptr);
      TLS_LAUNCH(PC_GRAM, k_gram_mfma16<bf16_t>, g16, dim3(G16LANES), 0, st, mp, (const bf16_t *)cast, part, NT,
                 gp.seglen, gp.npairs, nseg);
      TLS_LAUNCH(PC_GRAM, k_gram_reduce, dim3(ntiles, 4), dim3(256), 0, st, (const float *)part, nseg, NT, Np,
                 (float *)G);
      break;
  }
  return hipGetLastError();
}

// the upper triangle of G (Np x Np, compute precision) into out (n x n FP64)
template <typename C>
__global__ void k_gram_export(int n, int Np, const C *G, double *out) {
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) out[(size_t)j * n + i] = (double)G[(size_t)j * Np + i];
}
hipError_t launch_gram_export(int n, int Np, int compute, const void *G, double *out, hipStream_t st) {
  if (compute == TLS_FP64)
    TLS_LAUNCH(PC_GRAM, k_gram_export<double>, dim3(n), dim3(256), 0, st, n, Np, (const double *)G, out);
  else
    TLS_LAUNCH(PC_GRAM, k_gram_export<float>, dim3(n), dim3(256), 0, st, n, Np, (const float *)G, out);
  return hipGetLastError();
}

// identity in the padding columns n..Np-1 (upper triangle)
template <typename C>
__global__ void k_gram_pad(int n, int Np, C *G) {
  const int j = n + blockIdx.x;
  for (int k = threadIdx.x; k <= j; k += blockDim.x) G[(size_t)j * Np + k] = (k == j) ? (C)1 : (C)0;
}
hipError_t launch_gram_pad(int n, int Np, int compute, void *G, hipStream_t st) {
  if (Np == n) return hipSuccess;
  if (compute == TLS_FP64)
    TLS_LAUNCH(PC_GRAM, k_gram_pad<double>, dim3(Np - n), dim3(256), 0, st, n, Np, (double *)G);
  else
    TLS_LAUNCH(PC_GRAM, k_gram_pad<float>, dim3(Np - n), dim3(256), 0, st, n, Np, (float *)G);
  return hipGetLastError();
}

template <typename C>
__global__ void k_gram_shift(int n, int Np, C *G, double shift) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) G[(size_t)i * Np + i] += (C)shift;
}
hipError_t launch_gram_shift(int n, int Np, int compute, void *G, double shift, hipStream_t st) {
  const dim3 g((n + 255) / 256);
  if (compute == TLS_FP64)
    TLS_LAUNCH(PC_GRAM, k_gram_shift<double>, g, dim3(256), 0, st, n, Np, (double *)G, shift);
  else
    TLS_LAUNCH(PC_GRAM, k_gram_shift<float>, g, dim3(256), 0, st, n, Np, (float *)G, shift);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// blocked right-looking Cholesky, upper: G = R^T R, 64x64 tiles
// --------------------------------------------------------------------------

// U = Ri^T Rj for two 64x64 tiles in LDS (Ri[t][r] = entry (t, r) of the
// tile of R whose columns index U's rows) on the matrix cores, by a group of
// four waves: wave w takes the 32x32 quadrant (rows 32 (w % 2).., columns
// 32 ((w / 2) % 2)..), so waves 4-7 of a larger workgroup form a second group. The operands
// are passed transposed (A from Rj, B from Ri) so that consecutive lanes
// hold consecutive rows r of U: the callback emit(r, c, value) then touches
// contiguous column-major addresses.
template <typename C, typename Emit>
__device__ inline void tile_product_t(const C (*Ri)[NB + 1], const C (*Rj)[NB + 1], Emit emit) {
  const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) & 3, wr = w >> 1, wc = w & 1;
  if constexpr (std::is_same<C, double>::value) {
    g_f64x4 acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) acc[t][u] = g_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < NB; k0 += 4) {
      double a[2], bb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = Rj[k0 + (lane >> 4)][wr * 32 + t * 16 + (lane & 15)];
        bb[t] = Ri[k0 + (lane >> 4)][wc * 32 + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], bb[u], acc[t][u], 0, 0, 0);
    }
    // D(row, col) = sum Rj(t, c) Ri(t, r): col -> r, row -> c
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          emit(wc * 32 + u * 16 + (lane & 15), wr * 32 + t * 16 + 4 * q + (lane >> 4), acc[t][u][q]);
  } else {
    g_f32x16 acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
#pragma unroll 8
    for (int k0 = 0; k0 < NB; k0 += 2) {
      const float a = Rj[k0 + (lane >> 5)][wr * 32 + (lane & 31)];
      const float bb = Ri[k0 + (lane >> 5)][wc * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q)
      emit(wc * 32 + (lane & 31), wr * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3), acc[q]);
  }
}

// the (r, c) positions tile_product_t gives this lane, in the same order
template <typename C, typename At>
__device__ inline void tile_product_t_index(At at) {
  const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) & 3, wr = w >> 1, wc = w & 1;
  if constexpr (std::is_same<C, double>::value) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) at(wc * 32 + u * 16 + (lane & 15), wr * 32 + t * 16 + 4 * q + (lane >> 4));
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) at(wc * 32 + (lane & 31), wr * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3));
  }
}

// a 64x64 tile at (row block I, column block J) of G into registers
// (NB * NB / THR values per thread), and from there into LDS. The two halves
// are separate so that a workgroup can put all of its global loads in flight
// before the first wait.
template <int THR, typename C>
__device__ inline void tile_fetch(const C *G, int Np, int I, int J, C (&tmp)[NB * NB / THR]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NB * NB / THR; ++q) {
    const int t = tid + THR * q;
    tmp[q] = G[((size_t)J * NB + t / NB) * Np + (size_t)I * NB + t % NB];
  }
}
template <int THR, typename C>
__device__ inline void tile_put(const C (&tmp)[NB * NB / THR], C (*dst)[NB + 1]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NB * NB / THR; ++q) {
    const int t = tid + THR * q;
    dst[t % NB][t / NB] = tmp[q];
  }
}
template <int THR, typename C>
__device__ inline void tile_to_lds(const C *G, int Np, int I, int J, C (*dst)[NB + 1]) {
  C tmp[NB * NB / THR];
  tile_fetch<THR>(G, Np, I, J, tmp);
  tile_put<THR>(tmp, dst);
}

// four consecutive entries of a column (16-byte aligned for float, 32 for double)
__device__ inline void store_col4(float *p, float a, float b, float c, float d) {
  *reinterpret_cast<float4 *>(p) = make_float4(a, b, c, d);
}
__device__ inline void store_col4(double *p, double a, double b, double c, double d) {
  reinterpret_cast<double2 *>(p)[0] = make_double2(a, b);
  reinterpret_cast<double2 *>(p)[1] = make_double2(c, d);
}

// the value v holds in lane src of the wave (src the same for all active lanes)
__device__ inline float read_lane(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double read_lane(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src), hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// One step of the blocked right-looking Cholesky (upper, G = R^T R, 64x64
// tiles), for block row p. Launch k (FUSED) carries two kinds of workgroups
// that touch disjoint tiles:
//  - panel workgroups 0 .. N-p-1 factor block row p = k + 1. Workgroup j
//    takes step k's update of its two tiles itself,
//      G(p,p) - R(k,p)^T R(k,p),  G(p,p+j) - R(k,p)^T R(k,p+j)
//    (two MFMA products from the R tiles of row k), then eliminates the
//    augmented block [G(p,p) | G(p,p+j)] (j = 0: the diagonal tile alone):
//    the elimination that turns G(p,p) into R(p,p) turns the appended
//    columns into R(p,p+j) = R(p,p)^{-T} G(p,p+j);
//  - update workgroups take step k's update G(i,j) -= R(k,i)^T R(k,j) of the
//    tiles in block rows i >= k + 2 (k + 2 <= i <= j < N), one pair each.
// So the trailing update of step k runs beside the panel of step k + 1,
// and the chain of dependent launches is one per block row. The first
// launch (not FUSED) is the panel of block row 0 alone.
// Panel elimination: thread (tr, tc) holds the 4x4 register blocks of rows
// 4tr.. and columns 4tc.. of both tiles; the 32 threads of one row group (16
// per tile) are half a wave. The 64 columns are taken four at a time. For
// group g the owning half wave reads the 4x4 diagonal block from the
// registers of the lane that holds it, factors it (redundantly in each lane,
// so all lanes agree bit for bit), turns its four rows into rows of R and
// publishes them in a double-buffered LDS slab; after one barrier the rows
// below take the rank-4 update. One barrier per four columns. A row group's
// registers are final once its own group is done (no later group updates
// them), so every lane writes its rows to memory after the loop, as pieces of
// four column entries, and no store or flag sits on the elimination's chain.
// A failed pivot (not positive, or NaN) leaves a NaN on its diagonal entry of
// R (the reciprocal square root of a value <= 0 is NaN or Inf, times the
// value is NaN) and the NaN runs on through every later pivot, so the first
// diagonal entry of R that is not positive names the first failed pivot; the
// diagonal lanes check theirs after the loop (the rows written are then of no
// use: the factorization is reported as failed).
// R(p,p) goes to rdiag (tile p, column-major), not to G: the other panel
// workgroups of the launch still read G(p,p). The packing kernel takes the
// diagonal tiles from rdiag.
constexpr int CHOL_THREADS = 512;
template <typename C, bool FUSED>
__global__ __launch_bounds__(CHOL_THREADS) void k_chol_step(int k, int N, int Np, C *G, C *rdiag, int *info) {
  constexpr int THR = CHOL_THREADS;
  __shared__ C ta[NB][NB + 1];     // R(k, .) operand / staged G(p,p)
  __shared__ C tb[NB][NB + 1];     // R(k, .) operand / staged G(p,p+j)
  __shared__ C slab[2][4][2 * NB];
  const int tid = threadIdx.x;
  const int p = FUSED ? k + 1 : k;
  if (FUSED && (int)blockIdx.x >= N - p) {
    // ---- update role: pair (i, j), k + 2 <= i <= j < N -------------------
    const int l = blockIdx.x - (N - p);
    int bq = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
    while ((bq + 1) * (bq + 2) / 2 <= l) ++bq;
    while (bq * (bq + 1) / 2 > l) --bq;
    const int i = k + 2 + (l - bq * (bq + 1) / 2), j = k + 2 + bq;
    // the two R tiles and this thread's entries of G(i,j) in flight together
    C ri[NB * NB / THR], rj[NB * NB / THR], gv[16];
    tile_fetch<THR>(G, Np, k, i, ri);
    tile_fetch<THR>(G, Np, k, j, rj);
    C *Gij = G + (size_t)j * NB * Np + (size_t)i * NB;
    int nn = 0;
    if (tid < 256) tile_product_t_index<C>([&](int r, int c) { gv[nn++] = Gij[(size_t)c * Np + r]; });
    tile_put<THR>(ri, ta);
    tile_put<THR>(rj, tb);
    __syncthreads();
    if (tid >= 256) return;   // one group of four waves takes the product
    nn = 0;
    tile_product_t<C>(ta, tb, [&](int r, int c, C v) {
      if (i < j || r <= c) Gij[(size_t)c * Np + r] = gv[nn] - v;
      ++nn;
    });
    return;
  }
  // ---- panel role: workgroup jb of block row p ---------------------------
  // thread (tr, tq): row group tr = rows 4tr..; tq < 16 holds the 4x4 block
  // of columns 4tq.. of G(p,p) (a v-lane), tq >= 16 the block of columns
  // 4(tq - 16).. of the appended tile G(p,p+jb) (a w-lane). A row group is
  // half a wave, so its v-lanes and w-lanes take the solves side by side.
  const int jb = blockIdx.x;
  const int tr = tid >> 5, tq = tid & 31, tc = tq & 15;
  const bool isw = tq >= 16;
  const size_t base = (size_t)p * NB;
  const bool has_b = jb > 0;
  const size_t cb = (size_t)(p + jb) * NB;
  if (FUSED) {
    // step k's update of the two tiles: ta <- R(k,p), tb <- R(k,p+jb);
    // waves 0-3 form G(p,p) - R(k,p)^T R(k,p), waves 4-7 G(p,p+jb) - R(k,p)^T R(k,p+jb)
    // the R tiles and this thread's entries of G(p,p) or G(p,p+jb), all in flight together
    const bool second = tid >= 256;
    C rp[NB * NB / THR], rq[NB * NB / THR], u[16], gv[16];
    tile_fetch<THR>(G, Np, k, p, rp);
    if (has_b) tile_fetch<THR>(G, Np, k, p + jb, rq);
    int nn = 0;
    if (!second) tile_product_t_index<C>([&](int r, int c) { gv[nn++] = G[(base + c) * Np + base + r]; });
    else if (has_b) tile_product_t_index<C>([&](int r, int c) { gv[nn++] = G[(cb + c) * Np + base + r]; });
    tile_put<THR>(rp, ta);
    if (has_b) tile_put<THR>(rq, tb);
    __syncthreads();
    nn = 0;
    if (!second) tile_product_t<C>(ta, ta, [&](int, int, C v) { u[nn++] = v; });
    else if (has_b) tile_product_t<C>(ta, tb, [&](int, int, C v) { u[nn++] = v; });
    __syncthreads();   // every wave is done reading the R tiles
    nn = 0;
    if (!second) {
      tile_product_t_index<C>([&](int r, int c) {
        ta[r][c] = (r <= c) ? gv[nn] - u[nn] : (C)0;
        ++nn;
      });
    } else if (has_b) {
      tile_product_t_index<C>([&](int r, int c) {
        tb[r][c] = gv[nn] - u[nn];
        ++nn;
      });
    }
  } else {
    constexpr int Q = NB * NB / THR;
    C tmp[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int t = tid + THR * q;
      tmp[q] = G[(base + t / NB) * Np + base + t % NB];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int t = tid + THR * q, r = t % NB, c = t / NB;
      ta[r][c] = (r <= c) ? tmp[q] : (C)0;
    }
    if (has_b) tile_to_lds<THR>(G, Np, p, p + jb, tb);
  }
  __syncthreads();
  C blk[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
      blk[x][y] = isw ? (has_b ? tb[4 * tr + x][4 * tc + y] : (C)0) : ta[4 * tr + x][4 * tc + y];
  const int col0 = (isw ? NB : 0) + 4 * tc;   // this block's columns in the slab
  for (int g = 0; g < NB / 4; ++g) {
    const int buf = g & 1;
    if (tr == g) {
      // the v-lane holding the diagonal block: lane g of this half wave, the
      // same for every active lane, so a register read of that lane suffices
      const int src = ((g & 1) << 5) + g;
      C d[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) d[x][y] = read_lane(blk[x][y], src);
      C rd[4][4], inv[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const C pv = d[s][s];
        inv[s] = chol_rsqrt(pv);
        const C rs = pv * inv[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) rd[s][t] = (t == s) ? rs : (t > s ? d[s][t] * inv[s] : (C)0);
#pragma unroll
        for (int s2 = s + 1; s2 < 4; ++s2)
#pragma unroll
          for (int t = s2; t < 4; ++t) d[s2][t] -= rd[s][s2] * rd[s][t];
      }
      if (!isw && tc == g) {
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) blk[x][y] = rd[x][y];
      } else if (isw ? has_b : tc > g) {
        // rows 4g.. of R in this block's columns: rd^{-T} applied to the block
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
          for (int y = 0; y < 4; ++y) blk[s][y] *= inv[s];
#pragma unroll
          for (int s2 = s + 1; s2 < 4; ++s2)
#pragma unroll
            for (int y = 0; y < 4; ++y) blk[s2][y] -= rd[s][s2] * blk[s][y];
        }
      } else {
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) blk[x][y] = (C)0;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int y = 0; y < 4; ++y) slab[buf][s][col0 + y] = blk[s][y];
    }
    __syncthreads();
    if (tr > g) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        C rr[4], rc[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          rr[x] = slab[buf][s][4 * tr + x];
          rc[x] = slab[buf][s][col0 + x];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) blk[x][y] -= rr[x] * rc[y];
      }
    }
  }
  // rows 4tr.. of R in this block's four columns: G(p,p+jb) from the w-lanes,
  // the upper part of R(p,p) into rdiag from the v-lanes (jb = 0)
  if (isw == has_b && (isw || tc >= tr)) {
    C *dst = isw ? G + (cb + 4 * tc) * Np + base + 4 * tr
                 : rdiag + (size_t)p * NB * NB + (size_t)(4 * tc) * NB + 4 * tr;
    const size_t ld = isw ? (size_t)Np : (size_t)NB;
#pragma unroll
    for (int y = 0; y < 4; ++y) store_col4(dst + y * ld, blk[0][y], blk[1][y], blk[2][y], blk[3][y]);
  }
  if (blockIdx.x == 0 && !isw && tc == tr) {
    int s = 0;
    while (s < 4 && blk[s][s] > (C)0) ++s;
    if (s < 4) atomicMin(info, p * NB + 4 * tr + s + 1);
  }
}

// the row copy starts beside the first Cholesky launch of at most this many
// workgroups: on 4096 columns that is the last 32 of 64 block rows, whose
// launches are bound by the panel's latency, not by the update's tiles;
// starting it beside wider launches slows their updates, later leaves the
// copy running when the factor is done
constexpr int CHOL_NARROW_GRID = 528;
template <typename C>
static hipError_t cholesky_t(int N, int Np, C *G, C *rdiag, int *info, hipStream_t st, hipEvent_t narrow) {
  TLS_LAUNCH(PC_CHOL_PANEL, (k_chol_step<C, false>), dim3(N), dim3(CHOL_THREADS), 0, st, 0, N, Np, G, rdiag,
             info);
  for (int k = 0; k + 1 < N; ++k) {
    const int M = N - k - 2;   // trailing block rows of the update role
    const int grid = (N - k - 1) + M * (M + 1) / 2;
    if (narrow && grid <= CHOL_NARROW_GRID) {
      const hipError_t e = hipEventRecord(narrow, st);
      if (e != hipSuccess) return e;
      narrow = nullptr;
    }
    TLS_LAUNCH(PC_CHOL_PANEL, (k_chol_step<C, true>), dim3(grid), dim3(CHOL_THREADS), 0, st, k, N, Np, G,
               rdiag, info);
  }
  if (narrow) return hipEventRecord(narrow, st);
  return hipGetLastError();
}
hipError_t launch_cholesky(int N, int Np, int compute, void *G, void *rdiag, int *info, hipStream_t st,
                           hipEvent_t narrow) {
  if (compute == TLS_FP64) return cholesky_t<double>(N, Np, (double *)G, (double *)rdiag, info, st, narrow);
  return cholesky_t<float>(N, Np, (float *)G, (float *)rdiag, info, st, narrow);
}

// --------------------------------------------------------------------------
// packing into tiles of the storage precision, diagonal-tile inverses
// --------------------------------------------------------------------------
// upper tiles of R from G, the diagonal ones from rdiag when given (the
// Cholesky steps leave them there; NULL: G holds them, as after the QR)
template <typename C, typename S>
__global__ void k_pack(int N, int Np, const C *G, const C *rdiag, S *tiles) {
  const int l = blockIdx.x;
  int J = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= l) ++J;
  while (J * (J + 1) / 2 > l) --J;
  const int I = l - J * (J + 1) / 2;
  S *T = tiles + (size_t)l * NB * NB;
  for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
    const int r = t % NB, c = t / NB;
    double v = 0;
    if (I < J) v = (double)G[((size_t)J * NB + c) * Np + (size_t)I * NB + r];
    else if (r <= c) v = rdiag ? (double)rdiag[(size_t)I * NB * NB + t] : (double)G[((size_t)J * NB + c) * Np + (size_t)I * NB + r];
    T[t] = st_from<S>(v);
  }
}
template <typename C>
static hipError_t pack_c(int N, int Np, const C *G, const C *rdiag, int storage, void *tiles, hipStream_t st) {
  const dim3 g(N * (N + 1) / 2);
  switch (storage) {
    case TLS_FP64: TLS_LAUNCH(PC_PACK, (k_pack<C, double>), g, dim3(256), 0, st, N, Np, G, rdiag, (double *)tiles); break;
    case TLS_FP32: TLS_LAUNCH(PC_PACK, (k_pack<C, float>), g, dim3(256), 0, st, N, Np, G, rdiag, (float *)tiles); break;
    case TLS_FP16: TLS_LAUNCH(PC_PACK, (k_pack<C, half_t>), g, dim3(256), 0, st, N, Np, G, rdiag, (half_t *)tiles); break;
    default: TLS_LAUNCH(PC_PACK, (k_pack<C, bf16_t>), g, dim3(256), 0, st, N, Np, G, rdiag, (bf16_t *)tiles); break;
  }
  return hipGetLastError();
}
hipError_t launch_pack_tiles(int N, int Np, int compute, const void *G, const void *rdiag, int storage,
                             void *tiles, hipStream_t st) {
  if (compute == TLS_FP64)
    return pack_c<double>(N, Np, (const double *)G, (const double *)rdiag, storage, tiles, st);
  return pack_c<float>(N, Np, (const float *)G, (const float *)rdiag, storage, tiles, st);
}

// inverse of each stored diagonal tile, computed in FP64 from the stored values
template <typename S>
__global__ __launch_bounds__(1024) void k_diag_inverse(const S *tiles, double *dinv64, float *dinv32) {
  // X = T^{-1} for the upper triangular 64x64 tile T, by 16x16 blocks:
  //  1. the four diagonal blocks at once by backward substitution (T_qq
  //     X_qq = I, 16 steps with one barrier each; thread (q, i, t) holds
  //     entry (i, t) of the right-hand side of block q), with the 64
  //     reciprocal pivots computed once beforehand;
  //  2. the blocks above the diagonal by block back-substitution, in order
  //     of their distance d = J - I from the diagonal (all blocks of one
  //     distance together): S = sum_{K = I+1..J} T_IK X_KJ, then
  //     X_IJ = -X_II S (two barriers per distance).
  __shared__ double T[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  __shared__ double Sb[3][16][17];
  __shared__ double rpiv[NB];
  const int I = blockIdx.x, tid = threadIdx.x;
  const S *src = tiles + ((size_t)I * (I + 1) / 2 + I) * NB * NB;
  for (int e = tid; e < NB * NB; e += 1024) {
    const int r = e % NB, c = e / NB;
    T[r][c] = cvt<double>(src[e]);
    X[r][c] = 0.0;
  }
  __syncthreads();
  if (tid < NB) rpiv[tid] = 1.0 / T[tid][tid];
  __syncthreads();
  {
    const int q = tid >> 8, i = (tid >> 4) & 15, t = tid & 15, o = 16 * q;
    double b = (i == t) ? 1.0 : 0.0;
    for (int l = 15; l >= 0; --l) {
      if (i == l) X[o + l][o + t] = b * rpiv[o + l];
      __syncthreads();
      const double xl = X[o + l][o + t];
      if (i < l) b -= T[o + i][o + l] * xl;
    }
  }
  for (int d = 1; d <= 3; ++d) {
    const int active = (4 - d) * 256;   // blocks (Ib, Ib + d), 256 entries each
    const int pr = tid >> 8, r = (tid >> 4) & 15, c = tid & 15;
    const int ib = pr, jb = pr + d;
    if (tid < active) {
      double sacc = 0.0;
      for (int k = 0; k < 16 * d; ++k) sacc += T[16 * ib + r][16 * (ib + 1) + k] * X[16 * (ib + 1) + k][16 * jb + c];
      Sb[pr][r][c] = sacc;
    }
    __syncthreads();
    if (tid < active) {
      double xacc = 0.0;
      for (int k = r; k < 16; ++k) xacc += X[16 * ib + r][16 * ib + k] * Sb[pr][k][c];
      X[16 * ib + r][16 * jb + c] = -xacc;
    }
    __syncthreads();
  }
  double *o64 = dinv64 + (size_t)I * NB * NB;
  float *o32 = dinv32 + (size_t)I * NB * NB;
  for (int e = tid; e < NB * NB; e += 1024) {
    const int r = e % NB, c = e / NB;
    o64[e] = X[r][c];
    o32[e] = (float)X[r][c];
  }
}
hipError_t launch_diag_inverse(int N, int storage, const void *tiles, double *dinv64, float *dinv32,
                               hipStream_t st) {
  switch (storage) {
    case TLS_FP64: TLS_LAUNCH(PC_PACK, k_diag_inverse<double>, dim3(N), dim3(1024), 0, st, (const double *)tiles, dinv64, dinv32); break;
    case TLS_FP32: TLS_LAUNCH(PC_PACK, k_diag_inverse<float>, dim3(N), dim3(1024), 0, st, (const float *)tiles, dinv64, dinv32); break;
    case TLS_FP16: TLS_LAUNCH(PC_PACK, k_diag_inverse<half_t>, dim3(N), dim3(1024), 0, st, (const half_t *)tiles, dinv64, dinv32); break;
    default: TLS_LAUNCH(PC_PACK, k_diag_inverse<bf16_t>, dim3(N), dim3(1024), 0, st, (const bf16_t *)tiles, dinv64, dinv32); break;
  }
  return hipGetLastError();
}

// import a caller factor (column-major n x n upper, FP64) into tiles
template <typename S>
__global__ void k_import(int n, const double *R, S *tiles) {
  const int l = blockIdx.x;
  int J = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= l) ++J;
  while (J * (J + 1) / 2 > l) --J;
  const int I = l - J * (J + 1) / 2;
  S *T = tiles + (size_t)l * NB * NB;
  for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
    const int r = t % NB, c = t / NB;
    const int gr = I * NB + r, gc = J * NB + c;
    double v;
    if (gr >= n || gc >= n) v = (gr == gc) ? 1.0 : 0.0;
    else v = (gr <= gc) ? R[(size_t)gc * n + gr] : 0.0;
    T[t] = st_from<S>(v);
  }
}
hipError_t launch_import_tiles(int n, int N, int Np, const double *R, int storage, void *tiles,
                               hipStream_t st) {
  (void)Np;
  const dim3 g(N * (N + 1) / 2);
  switch (storage) {
    case TLS_FP64: hipLaunchKernelGGL(k_import<double>, g, dim3(256), 0, st, n, R, (double *)tiles); break;
    case TLS_FP32: hipLaunchKernelGGL(k_import<float>, g, dim3(256), 0, st, n, R, (float *)tiles); break;
    case TLS_FP16: hipLaunchKernelGGL(k_import<half_t>, g, dim3(256), 0, st, n, R, (half_t *)tiles); break;
    default: hipLaunchKernelGGL(k_import<bf16_t>, g, dim3(256), 0, st, n, R, (bf16_t *)tiles); break;
  }
  return hipGetLastError();
}

template <typename S>
__global__ void k_export(int n, const S *tiles, double *R) {
  const int l = blockIdx.x;
  int J = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= l) ++J;
  while (J * (J + 1) / 2 > l) --J;
  const int I = l - J * (J + 1) / 2;
  const S *T = tiles + (size_t)l * NB * NB;
  for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
    const int r = t % NB, c = t / NB;
    const int gr = I * NB + r, gc = J * NB + c;
    if (gr < n && gc < n) {
      R[(size_t)gc * n + gr] = (gr <= gc) ? cvt<double>(T[t]) : 0.0;
      if (I < J) R[(size_t)gr * n + gc] = 0.0;    // the mirrored lower entry
    }
  }
}
hipError_t launch_export_tiles(int n, int N, int Np, int storage, const void *tiles, double *R,
                               hipStream_t st) {
  (void)Np;
  const dim3 g(N * (N + 1) / 2);
  switch (storage) {
    case TLS_FP64: hipLaunchKernelGGL(k_export<double>, g, dim3(256), 0, st, n, (const double *)tiles, R); break;
    case TLS_FP32: hipLaunchKernelGGL(k_export<float>, g, dim3(256), 0, st, n, (const float *)tiles, R); break;
    case TLS_FP16: hipLaunchKernelGGL(k_export<half_t>, g, dim3(256), 0, st, n, (const half_t *)tiles, R); break;
    default: hipLaunchKernelGGL(k_export<bf16_t>, g, dim3(256), 0, st, n, (const bf16_t *)tiles, R); break;
  }
  return hipGetLastError();
}

}  // namespace tls
