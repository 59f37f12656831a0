// Internal launch interface between the host driver and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "tls.h"

namespace tls {

// kernel classes of the profiling hooks (order as in tls.h)
enum ProfClass { PC_TRSV_APPLY = 0, PC_PCG, PC_GRAM, PC_CHOL_PANEL, PC_CHOL_UPDATE, PC_RESIDUAL,
                 PC_GRADIENT, PC_SCALARS, PC_SETUP, PC_LANCZOS, PC_PACK, PC_RESID_DD, PC_INVERT,
                 PC_MLP, PC_GATE, PC_QR };
// no-ops unless profiling is on (see tls_profile_start)
void prof_begin(int cls, hipStream_t st);
// launches on a stream noted here are counted as PC_GATE whatever their kernel
void prof_note_side_stream(hipStream_t st);
void prof_end(hipStream_t st);

// a kernel launch on stream `st`, bracketed by the profiling hooks; one statement
#define TLS_LAUNCH(cls, ...)          \
  do {                                \
    ::tls::prof_begin((cls), st);     \
    hipLaunchKernelGGL(__VA_ARGS__);  \
    ::tls::prof_end(st);              \
  } while (0)

// view of a packed factor (device pointers)
struct FactorView {
  int n, N, Np, storage;
  const void *tiles;
  const double *dinv64;
  const float *dinv32;
  const double *dscale64;   // 1/d, length Np (ones beyond n)
  const float *dscale32;
  // explicit inverse X = R_hat^{-1} (row-packed tiles of X and of X^T)
  const void *xr, *xc;
  int xstorage;
  int xrow;                 // 1: one workgroup per block row; 0: split over the chip
};

// buffers of one triangular-solve / PCGTLS launch
struct SolveBufs {
  int *sync;
  void *chain;
  const double *in;
  double *out;
  void *s, *p, *q, *w, *part;
  int *done, *neg;
  double *trace;
  const double *sigma2;
  int j, L, strict;
  int ldi = 0, ldo = 0;   // stride between right-hand sides of in/out (0: n)
  void *cpart;   // chunk partials of the inverse-apply kernels
  int *cnt;      // per-block arrival counters (zero between launches)
  int clear_flags = 0;   // the PCG init launch of the X application also clears done, neg and trace
};

// ---- kernels_trsv.hip ------------------------------------------------------
hipError_t launch_trsv(const FactorView &F, int compute, int mode, int nrhs, const SolveBufs &B,
                       hipStream_t st);
// ---- kernels_inv.hip --------------------------------------------------------
hipError_t launch_invert(int N, int storage, const void *Rt, const double *dinv64, void *W, void *Y,
                         int xstorage, void *XR, void *XC, hipStream_t st);
size_t invert_scratch_doubles(int N);
hipError_t launch_xapply(const FactorView &F, int compute, int mode, int nrhs, const SolveBufs &B,
                         hipStream_t st);
size_t xapply_chunk_count(int N);

hipError_t launch_pcg_finish(int compute, const void *w, double *out, int n, int Np, int nrhs,
                             hipStream_t st);

// ---- kernels_factor.hip ----------------------------------------------------
hipError_t launch_fill_i32(int *p, int v, size_t count, hipStream_t st);
// up to MAX fills in one launch
struct FillSet {
  static constexpr int MAX = 8;
  void *ptr[MAX];
  size_t n[MAX];
  uint64_t bits[MAX];
  int wide[MAX];
  int count = 0;
  void add_i32(int *p, int v, size_t cnt);
  void add_f64(double *p, double v, size_t cnt);
};
hipError_t launch_fill_multi(const FillSet &F, hipStream_t st);
hipError_t launch_fill_f64(double *p, double v, size_t count, hipStream_t st);
hipError_t launch_round(const double *in, int64_t count, int q, double *out, hipStream_t st);
hipError_t launch_check_finite(const double *v, size_t count, int *flag, hipStream_t st);
// int32 entries the CSC build needs in its `fill` buffer for an m x n matrix
size_t csc_fill_ints(int64_t m, int64_t n);
hipError_t launch_csc_build(int m, int n, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col_idx, const double *val, int32_t *col_ptr,
                            int32_t *row_idx, double *cval, int32_t *tmp_row, double *tmp_val,
                            int32_t *fill, hipStream_t st);
hipError_t launch_colnorms_csc(int n, const int32_t *col_ptr, const double *cval, double *d,
                               hipStream_t st);
// column norms d of a dense column-major A and the finite-input flag (any
// NaN or Inf among its m x n entries) in one read of A; part holds
// colsq_dense_doubles(m, n) doubles of scratch
size_t colsq_dense_doubles(int64_t m, int64_t n);
hipError_t launch_colsq_dense(int m, int n, int64_t ld, const double *A, double *part, double *d, int *flag,
                              hipStream_t st);
// row-major copy At (stride ldr, a multiple of 64, padding columns zero) of a
// dense column-major A
hipError_t launch_rowcopy_dense(int m, int n, int64_t ld, const double *A, int64_t ldr, double *At,
                                hipStream_t st);
// CSR structure check (row pointers, column range, sorted rows): *bad |= 1
hipError_t launch_validate_csr(int m, int n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                               int *bad, hipStream_t st);
hipError_t launch_colnorms_dense(int m, int n, int64_t ld, const double *A, double *d,
                                 hipStream_t st);
// scaling vectors: dinv = 1/d (or ones when unscaled), both precisions, padded to Np
hipError_t launch_dstats(int n, const double *d, double *out, hipStream_t st);
hipError_t launch_scale_vectors(int n, int Np, const double *d, int scaled, double *dsc64,
                                float *dsc32, hipStream_t st);
// quantised scaled values (CSR and CSC arrays): out = round_q(val / d[col]) as compute type
hipError_t launch_quantize_sparse(int64_t nnz, const int32_t *cols, const double *val,
                                  const double *d, int scaled, int q, int compute, void *out,
                                  hipStream_t st);
hipError_t launch_quantize_csc(int n, const int32_t *col_ptr, const double *cval, const double *d,
                               int scaled, int q, int compute, void *out, hipStream_t st);
hipError_t launch_gram_sparse(int m, int n, int Np, const int32_t *row_ptr, const int32_t *col_idx,
                              const void *valq, const int32_t *col_ptr, const int32_t *row_idx,
                              const void *cvalq, int compute, void *G, hipStream_t st);
size_t gram_cast_bytes(int64_t m, int64_t n);
// FP64 partial tiles of the FP64 / FP32 Gram's row segments (0: one segment)
size_t gram_part64_bytes(int64_t m, int64_t n);
hipError_t launch_gram_mfma(int m, int n, int Np, int64_t ld, const double *A, const double *d,
                            int scaled, int q, void *cast, void *G, void *gpart, hipStream_t st);
hipError_t launch_gram_dense(int m, int n, int Np, int64_t ld, const double *A, const double *d,
                             int scaled, int q, int compute, void *G, hipStream_t st);
hipError_t launch_gram_pad(int n, int Np, int compute, void *G, hipStream_t st);
hipError_t launch_gram_export(int n, int Np, int compute, const void *G, double *out, hipStream_t st);
hipError_t launch_gram_shift(int n, int Np, int compute, void *G, double shift, hipStream_t st);
// blocked Cholesky of G in place (upper); rdiag: N 64x64 tiles of scratch
// in the compute precision (the diagonal tiles while the steps run)
// narrow (optional) is recorded on st before the first launch of the chain
// whose grid leaves most of the chip free (at the end if none does)
hipError_t launch_cholesky(int N, int Np, int compute, void *G, void *rdiag, int *info, hipStream_t st,
                           hipEvent_t narrow = nullptr);
// Householder QR (kernels_qr.hip): bytes of the working matrix (FP64-sized,
// m_pad x Np, m_pad = m + Np - n) and of all QR scratch; R goes to G
// (column-major Np x Np, compute precision) with a nonnegative diagonal,
// info receives the first zero or non-finite pivot (column + 1) by atomicMin
size_t qr_matrix_bytes(int64_t m, int n);
size_t qr_work_bytes(int64_t m, int n);
hipError_t launch_qr_factor(int64_t m, int n, int Np, int format, int64_t ldA, const double *val,
                            const int32_t *row_ptr, const int32_t *col_idx, const double *d, int scaled, int uq,
                            int compute, void *work, void *G, int *info, hipStream_t st);
// upper tiles of R into tiles of the storage precision; the diagonal tiles
// from rdiag (as the Cholesky steps leave them) or, when rdiag is NULL, from G
hipError_t launch_pack_tiles(int N, int Np, int compute, const void *G, const void *rdiag, int storage,
                             void *tiles, hipStream_t st);
hipError_t launch_diag_inverse(int N, int storage, const void *tiles, double *dinv64,
                               float *dinv32, hipStream_t st);
hipError_t launch_import_tiles(int n, int N, int Np, const double *R, int storage, void *tiles,
                               hipStream_t st);
hipError_t launch_export_tiles(int n, int N, int Np, int storage, const void *tiles, double *R,
                               hipStream_t st);

// ---- kernels_rqi.hip -------------------------------------------------------
struct MatView {
  int format;
  int m, n;
  int64_t ld, nnz;
  const double *val;
  const int32_t *row_ptr, *col_idx;
  // CSC copy (CSR only)
  const int32_t *col_ptr, *row_idx;
  const double *cval;
  // row-major copy of a dense A (row stride ldr, a multiple of 64, zero
  // padded), made by the factorization; nullptr when absent
  const double *at;
  int64_t ldr;
};

// r = b - A x; per-block partial sums of r.r and b.r written to part[2*blocks]
int matvec_blocks(const MatView &A);
hipError_t launch_residual(const MatView &A, const double *b, const double *x, double *r,
                           double *part, hipStream_t st);
// y = A x (plain), y = A^T x (plain)
hipError_t launch_matvec(const MatView &A, const double *x, double *y, hipStream_t st);
hipError_t launch_rmatvec(const MatView &A, const double *x, double *y, hipStream_t st);
// f = -A^T r - shift x with shift read from scal; partial f.f per block
int rmatvec_blocks(const MatView &A);
// one pass over the row-major copy (A.at): r = b - A x (b or x may be NULL
// for 0), residual partials in the k_residual_dense layout (part_r, may be
// NULL) and rowpass_partials(A) partial n-vectors of A^T r in ppart
int rowpass_groups(int64_t m, int cus);
int rowpass_blocks(int64_t m, int cus);
int rowpass_partials(const MatView &A);
// row stride of the copy the row pass reads (1024, 2048, 3072 or 4096 columns)
int64_t rowpass_ld(int64_t n);
hipError_t launch_rowpass(const MatView &A, const double *b, const double *x, double *r, double *part_r,
                          double *ppart, hipStream_t st);
// the same pass with the products of a second vector v2: ppart2 receives
// the partials of +A^T A v2 (summed by launch_rowpass_sum with s = 1), and
// t_out (optional, m) the products A v2
hipError_t launch_rowpass_dual(const MatView &A, const double *b, const double *x, double *r, double *part_r,
                               double *ppart, const double *v2, double *ppart2, hipStream_t st,
                               double *t_out = nullptr);
// y = s * sum of the partial n-vectors
hipError_t launch_rowpass_sum(const MatView &A, const double *ppart, double s, double *y, hipStream_t st);
// f = -A^T r - mu x from the partials (gradient_rows_blocks(n) partial pairs)
int gradient_rows_blocks(int n);
// f = -A^T r - mu x from the row pass's partials with psi_k (launch_outer_psi's
// work) taken by the last of its workgroups to finish; ppart2 (optional):
// A^T r = sum(ppart) - sigma_0^2 sum(ppart2), sigma_0^2 as
// launch_shift_residual kept it; *cnt counts arrivals (zero before the first
// launch, left at zero)
hipError_t launch_gradient_rows_psi(const MatView &A, const double *ppart, const double *x, double *scal,
                                    double *f, double *part, const double *part_r, int nb_r, double cap,
                                    const double *ppart2, int *cnt, int k, double *rec, double *rhs,
                                    double *xbest, double tie, hipStream_t st);
// r <- r - sigma_0^2 t (t = A u_0, sigma_0^2 = scal[0]) with the residual partials
hipError_t launch_shift_residual(int m, const double *b, double *r, const double *t, double *scal,
                                 double *part_r, hipStream_t st);
hipError_t launch_gradient(const MatView &A, const double *r, const double *x, double *scal,
                           double *f, double *part, const double *part_r, int nb_r, double cap,
                           hipStream_t st);
// compensated residual r = b - A x in double-double, partial sums (hi/lo) of r.r
hipError_t launch_residual_dd(const MatView &A, const double *b, const double *x, double *part,
                              hipStream_t st);

// scalar kernels of the outer loop, all single-workgroup, deterministic
struct OuterScalars;   // device struct, see kernels_rqi.hip
hipError_t launch_outer_rq(int n, const double *x, const double *part_r, int nb_r, double *scal,
                           double clamp_max, hipStream_t st);
hipError_t launch_outer_psi(int n, const double *x, const double *f, const double *part_f, int nb_f,
                            double *scal, int k, double *rec, double *rhs, double *xbest, double tie,
                            hipStream_t st);
hipError_t launch_make_rhs(int n, const double *f, const double *x, double *rhs, hipStream_t st);
hipError_t launch_rqi_update(int n, double *x, const double *omega_u, const double *f,
                             const double *scal, double *xbest, double *xsnap, const int *done,
                             int nsteps, hipStream_t st);
// the same on the PCGTLS state itself: omega and u are rows 0 and Np of w,
// in the compute precision of the runs (no FP64 copy first)
hipError_t launch_rqi_update_pcg(int n, double *x, int compute, const void *w, int Np, const double *f,
                                 const double *scal, const int *done, int nsteps, hipStream_t st);
hipError_t launch_axpy_init(int n, double *x, const double *u, const double *scal, int which,
                            hipStream_t st);
hipError_t launch_copy_f64(double *dst, const double *src, size_t count, hipStream_t st);
hipError_t launch_add_f64(double *x, const double *dx, size_t count, hipStream_t st);
hipError_t launch_lanczos_orth(int n, int Np, int k, int K, double *V, const double *Wout,
                               double *nxt, const double *dsc, double *ab, hipStream_t st, int runs = 2);
hipError_t launch_ref_step1(int n, int nrhs, const double *scal, double *x, double *r,
                            const double *p, double *q, double *rs, hipStream_t st);
hipError_t launch_ref_step2(int n, int nrhs, const double *r, const double *z, double *p, double *rs,
                            int first, hipStream_t st);
hipError_t launch_sigma_dd(int n, const double *x, const double *part, int nb, double *scal,
                           hipStream_t st);

// ---- warm start (kernels_rqi.hip) ---------------------------------------------
struct DotPairs {
  static constexpr int MAX = 8;
  const double *a[MAX], *b[MAX];
  int64_t len[MAX];
};
hipError_t launch_dots(const DotPairs &D, int count, double *out, hipStream_t st);
hipError_t launch_axpy2(int n, const double *x0, const double *u0, const double *u1, double c1,
                        double c2, double *out, hipStream_t st);
hipError_t launch_scale_copy(int n, const double *src, double alpha, double *dst, hipStream_t st);
// ---- kernels_mlp.hip --------------------------------------------------------
// activations of a training batch of B samples (row-major, B x width)
struct MlpBufs {
  float *h0;              // standardised inputs, B x 32
  float *z[3], *h[3];     // hidden pre-activations and GELU outputs, B x 256
  float *dz[2];           // gradients w.r.t. pre-activations (ping-pong), B x 256
  float *dy;              // dL/dy, B
};
hipError_t launch_mlp_forward(const float *theta, const float *norm, const float *X, int64_t B,
                              float *y, const MlpBufs &M, hipStream_t st);
hipError_t launch_mlp_backward(const float *theta, const float *y, const float *t, int64_t B,
                               float *grad, float *loss, const MlpBufs &M, hipStream_t st);
hipError_t launch_mlp_adam(int64_t count, float *theta, float *m, float *v, const float *g, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t st);
hipError_t launch_mlp_infer1(const float *theta, const float *norm, const float *feat, double *y,
                             hipStream_t st);

}  // namespace tls
