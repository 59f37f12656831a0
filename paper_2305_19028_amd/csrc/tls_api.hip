// Host driver and C ABI of libtls (declarations and contracts in tls.h).
//
// Every entry point validates its arguments, carves its workspace with a
// fixed layout (the *_workspace_size functions run the same carving on a
// null base), enqueues kernels on the caller's stream and maps failures to
// tls_status with a thread-local message. Nothing here computes on the
// host except scalar control decisions (the psi stopping rule, the gate
// verdict, the Lanczos tridiagonal eigenvalues).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "tls.h"

using namespace tls;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err = "no error";

static tls_status fail(tls_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess)                                                             \
      return fail(TLS_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                  __FILE__, __LINE__);                                                \
  } while (0)

#define TRY(expr)                      \
  do {                                 \
    tls_status _s = (expr);            \
    if (_s != TLS_OK) return _s;       \
  } while (0)

// ---------------------------------------------------------------------------
// workspace carving
// ---------------------------------------------------------------------------
namespace {

struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base((char *)b) {}
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t size() const { return (off + 255) & ~(size_t)255; }
};

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

MatView make_view(const tls_matrix *A, const tls_precond_s *P);

}  // namespace

// ---------------------------------------------------------------------------
// the preconditioner object
// ---------------------------------------------------------------------------
struct FactorWsRef;
struct tls_precond_s {
  int64_t n = 0;
  int N = 0, Np = 0;
  int storage = TLS_FP64, requested = TLS_FP64, scaled = 0, format = TLS_DENSE_COLMAJOR;
  int uq = TLS_FP64;               // factor precision (storage_of(uq) == storage)
  int64_t m = 0, nnz = 0;
  void *tiles = nullptr;
  double *dinv64 = nullptr;
  float *dinv32 = nullptr;
  double *dsc64 = nullptr;
  float *dsc32 = nullptr;
  double *d = nullptr;
  int32_t *col_ptr = nullptr, *row_idx = nullptr;
  double *cval = nullptr;
  const int32_t *csr_row_ptr = nullptr, *csr_col_idx = nullptr;   // the validated structure
  double *at = nullptr;            // row-major copy of a dense A (stride ldr), or NULL
  int64_t ldr = 0;
  tls_gate_report rep{};
  void *xr = nullptr, *xc = nullptr;   // explicit inverse tiles
  int xstorage = TLS_FP64;
  int apply_mode = 0;             // 0 explicit inverse (split GEMV), 1 substitution, 2 row GEMV
  void *fws_base = nullptr;       // the factor workspace (re-carved on demand)
  int64_t fws_m = 0;
  int fws_cast = 0;               // the factor workspace holds a cast buffer
  int fws_rows = 0;               // ... and the row-major copy of a dense A
  int method = 0;                 // 0 Cholesky of the Gram matrix, 1 Householder QR of A
  int have_sigma_n = 0, have_kappa = 0;
  double smin_s = 0, smax_s = 0;   // Lanczos extremes of sigma(A D^{-1})
  double normA_F2 = 0;             // ||A||_F^2 = sum_j d_j^2
  double lnd[4] = {0, 0, 0, 0};    // min, max, mean, std of ln d_j (warm-start features)
  // the gate's two Lanczos runs (estimates, certificate) on the library's
  // side streams: fork point, completion of each run, pending until collected
  hipEvent_t ev_fork = nullptr, ev_pair = nullptr, ev_cert = nullptr, ev_ride = nullptr;
  // a dense A's row-major copy is made on side2 beside the Cholesky: its
  // source until it is enqueued (rc_todo), and ev_rows marks its end while
  // the caller's stream has not yet been made to wait for it (rc_inflight)
  const double *rc_src = nullptr;
  int64_t rc_ld = 0;
  int rc_todo = 0, rc_inflight = 0;
  hipEvent_t ev_rows = nullptr;
  hipStream_t side = nullptr;
  hipStream_t side2 = nullptr;     // a dense A's certificate work between passes
  double *hgate = nullptr;         // pinned host block: the runs' tridiagonal scalars
  int hgate_dev = -1;
  int gate_pending = 0, have_quality = 0;
  // a dense A's certificate rides on the solve's passes over the row copy:
  // steps still to take (cert_todo) and the next step's index; its work
  // between passes runs on side2 and ev_cert marks the last of it
  int cert_todo = 0, cert_k = 0;
  ~tls_precond_s();
  FactorView view() const {
    FactorView F;
    F.n = (int)n;
    F.N = N;
    F.Np = Np;
    F.storage = storage;
    F.tiles = tiles;
    F.dinv64 = dinv64;
    F.dinv32 = dinv32;
    F.dscale64 = dsc64;
    F.dscale32 = dsc32;
    F.xr = xr;
    F.xc = xc;
    F.xstorage = xstorage;
    F.xrow = (apply_mode == 2);
    return F;
  }
};

namespace {

tls_status gate_finish(tls_precond_s *P);

MatView make_view(const tls_matrix *A, const tls_precond_s *P) {
  MatView V{};
  V.format = A->format;
  V.m = (int)A->m;
  V.n = (int)A->n;
  V.ld = A->ld;
  V.nnz = A->nnz;
  V.val = A->val;
  V.row_ptr = A->row_ptr;
  V.col_idx = A->col_idx;
  if (P) {
    V.col_ptr = P->col_ptr;
    V.row_idx = P->row_idx;
    V.cval = P->cval;
    V.at = P->at;
    V.ldr = P->ldr;
  }
  return V;
}

tls_status check_matrix(const tls_matrix *A) {
  if (!A) return fail(TLS_ERR_ARG, "A is NULL");
  if (A->m <= 0 || A->n <= 0) return fail(TLS_ERR_ARG, "A has m = %lld, n = %lld", (long long)A->m, (long long)A->n);
  if (A->m < A->n + 1) return fail(TLS_ERR_ARG, "need m >= n + 1 (m = %lld, n = %lld)", (long long)A->m, (long long)A->n);
  if (A->m > (int64_t)INT32_MAX || A->n > 65536) return fail(TLS_ERR_ARG, "A too large for this build (m < 2^31, n <= 65536)");
  if (!A->val) return fail(TLS_ERR_ARG, "A->val is NULL");
  if (A->format == TLS_DENSE_COLMAJOR) {
    if (A->ld < A->m) return fail(TLS_ERR_ARG, "ld (%lld) < m (%lld)", (long long)A->ld, (long long)A->m);
  } else if (A->format == TLS_CSR) {
    if (!A->row_ptr || !A->col_idx) return fail(TLS_ERR_ARG, "CSR index arrays are NULL");
    if (A->nnz < 0 || A->nnz > (int64_t)INT32_MAX) return fail(TLS_ERR_ARG, "nnz out of range");
  } else {
    return fail(TLS_ERR_ARG, "unknown format %d", A->format);
  }
  return TLS_OK;
}

tls_status check_prec(int p, const char *what) {
  if (p < TLS_FP64 || p > TLS_BF16X3) return fail(TLS_ERR_ARG, "invalid precision %d for %s", p, what);
  return TLS_OK;
}

// ---- factor workspace layout -----------------------------------------------
struct FactorWs {
  void *tiles;
  double *dinv64;
  float *dinv32;
  double *dsc64;
  float *dsc32;
  double *d;
  void *G;
  int32_t *col_ptr, *row_idx, *tmp_row, *fill;
  double *cval, *tmp_val;
  void *valq, *cvalq;
  int *info;
  int *sync;
  void *rdiag;     // diagonal tiles of R during the Cholesky steps
  double *lz;      // Lanczos vectors
  double *lzs;     // Lanczos scalars
  int *flag;
  double *dstats;  // column-norm statistics for the solve (k_dstats)
  void *xr, *xc;   // explicit inverse tiles (FP64-sized)
  double *yinv;    // inversion scratch
  int *cnt;        // per-block arrival counters of internal applies
  double *tm;      // m-vector (products with A in the certificate)
  void *cast;      // dense A rounded to u_q (matrix-core Gram input), or NULL
  void *gpart;     // FP64 partial tiles of the FP64 / FP32 Gram's row segments, or NULL
  void *qrw;       // Householder QR working matrix and reflector scratch, or NULL
  // the certificate's own buffers (it runs concurrently with the estimates)
  int *qsync, *qcnt;
  double *qpart, *qlz, *qlzs;
  // row-major copy of a dense A (rows of stride ldr), its column-norm scratch
  // and the certificate's row-pass partials; NULL unless made
  double *at, *colsq, *qppart;
  int64_t ldr;
};

// dense A whose rows fit the row pass's registers (n <= 4096) get a
// row-major working copy: every product with A in the outer iteration, the
// certificate and the refinement is then one pass over it
inline bool use_rowcopy(int format, int64_t n) { return format == TLS_DENSE_COLMAJOR && n <= 4096; }
inline int64_t rowcopy_ld(int64_t n) { return rowpass_ld(n); }
constexpr int LANCZOS_STEPS = 8;
constexpr int QUALITY_STEPS = 6;
constexpr double CERT_RITZ_MARGIN = 0.05;

FactorWs carve_factor(Carver &c, int64_t m, int64_t n, int64_t nnz, int format, int cast, int qr = 0,
                      int rows = 0) {
  const int Np = ceil_div(n, NB) * NB, N = Np / NB;
  FactorWs W{};
  W.tiles = c.take<char>((size_t)N * (N + 1) / 2 * NB * NB * 8);
  W.dinv64 = c.take<double>((size_t)N * NB * NB);
  W.dinv32 = c.take<float>((size_t)N * NB * NB);
  W.dsc64 = c.take<double>(Np);
  W.dsc32 = c.take<float>(Np);
  W.d = c.take<double>(Np);
  W.G = c.take<char>((size_t)Np * Np * 8);
  if (format == TLS_CSR) {
    W.col_ptr = c.take<int32_t>(n + 1);
    W.row_idx = c.take<int32_t>(nnz);
    W.cval = c.take<double>(nnz);
    W.tmp_row = c.take<int32_t>(nnz);
    W.tmp_val = c.take<double>(nnz);
    W.fill = c.take<int32_t>(csc_fill_ints(m, n));
    W.valq = c.take<char>(nnz * 8);
    W.cvalq = c.take<char>(nnz * 8);
  }
  {
    // one status block, read back in one copy: breakdown info, the
    // finite-input flag and the column statistics
    char *stat = c.take<char>(128);
    W.info = (int *)stat;
    W.flag = (int *)(stat + 16);
    W.dstats = (double *)(stat + 32);
  }
  W.sync = c.take<int>(N + 8);
  W.rdiag = c.take<double>((size_t)N * NB * NB);
  W.lz = c.take<double>((size_t)(2 * (LANCZOS_STEPS + 1) + 9) * Np);
  W.lzs = c.take<double>(4 * LANCZOS_STEPS + 8);
  W.xr = c.take<char>((size_t)N * (N + 1) / 2 * NB * NB * 8);
  W.xc = c.take<char>((size_t)N * (N + 1) / 2 * NB * NB * 8);
  W.yinv = c.take<double>(std::max(invert_scratch_doubles(N),
                                    (size_t)N * xapply_chunk_count(N) * 2 * NB));
  W.cnt = c.take<int>(N);
  W.tm = c.take<double>((size_t)std::max<int64_t>(m, 1));
  W.qsync = c.take<int>(N + 8);
  W.qcnt = c.take<int>(N);
  W.qpart = c.take<double>((size_t)N * xapply_chunk_count(N) * 2 * NB);
  W.qlz = c.take<double>((size_t)(QUALITY_STEPS + 1 + 9) * Np);
  W.qlzs = c.take<double>(2 * QUALITY_STEPS + 8);
  // low-precision copy of a dense A for the matrix-core Gram
  W.cast = (cast && format == TLS_DENSE_COLMAJOR) ? c.take<char>(gram_cast_bytes(m, n)) : nullptr;
  {
    const size_t gp = format == TLS_DENSE_COLMAJOR ? gram_part64_bytes(m, n) : 0;
    W.gpart = gp ? c.take<char>(gp) : nullptr;
  }
  W.qrw = qr ? c.take<char>(qr_work_bytes(m, (int)n)) : nullptr;
  W.at = W.colsq = W.qppart = nullptr;
  W.ldr = 0;
  if (rows && format == TLS_DENSE_COLMAJOR) W.colsq = c.take<double>(colsq_dense_doubles(m, n));
  if (rows && use_rowcopy(format, n)) {
    MatView V{};
    V.format = format;
    V.m = (int)m;
    V.n = (int)n;
    W.ldr = rowcopy_ld(n);
    W.at = c.take<double>((size_t)m * W.ldr);
    W.qppart = c.take<double>((size_t)rowpass_partials(V) * n);
  }
  return W;
}

// ---- solve workspace (one triangular solve / PCGTLS run) --------------------
struct PcgWs {
  int *sync;
  double *chain, *s, *p, *q, *w;   // sized for FP64 compute
  double *part;
  int *done, *neg;
  double *trace;
  double *sigma2;
  void *cpart;
  int *cnt;
  int L;
};

PcgWs carve_pcg(Carver &c, int Np, int N, int nrhs, int L) {
  PcgWs W{};
  W.L = L;
  W.sync = c.take<int>(N + 8);
  W.chain = c.take<double>((size_t)nrhs * Np);
  W.s = c.take<double>((size_t)nrhs * Np);
  W.p = c.take<double>((size_t)nrhs * Np);
  W.q = c.take<double>((size_t)nrhs * Np);
  W.w = c.take<double>((size_t)nrhs * Np);
  W.part = c.take<double>((size_t)(L + 2) * 3 * nrhs * N);
  W.done = c.take<int>((size_t)(L + 2) * nrhs);
  W.neg = c.take<int>((size_t)(L + 2) * nrhs);
  W.trace = c.take<double>((size_t)nrhs * 4 * (L + 2));
  W.sigma2 = c.take<double>(2);
  W.cpart = c.take<double>((size_t)N * xapply_chunk_count(N) * nrhs * NB);
  W.cnt = c.take<int>(N);
  return W;
}

SolveBufs bufs_of(const PcgWs &W) {
  SolveBufs B{};
  B.sync = W.sync;
  B.chain = W.chain;
  B.s = W.s;
  B.p = W.p;
  B.q = W.q;
  B.w = W.w;
  B.part = W.part;
  B.done = W.done;
  B.neg = W.neg;
  B.trace = W.trace;
  B.sigma2 = W.sigma2;
  B.L = W.L;
  B.cpart = W.cpart;
  B.cnt = W.cnt;
  return B;
}

// read the status word of a sync area (blocking)
tls_status sync_status(const int *sync, int N, hipStream_t st) {
  int v[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(v, sync + N + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (v[1] == TLS_ERR_SYNC_TIMEOUT) return fail(TLS_ERR_SYNC_TIMEOUT, "inter-workgroup wait timed out");
  if (v[1] == TLS_ERR_INDEFINITE) return fail(TLS_ERR_INDEFINITE, "delta_j <= 0 in PCGTLS (shifted system not positive definite)");
  if (v[0]) return fail(TLS_ERR_SYNC_TIMEOUT, "solve aborted");
  return TLS_OK;
}

hipError_t launch_precond(const tls_precond_s *P, int compute, int mode, int nrhs,
                          const SolveBufs &B, hipStream_t st) {
  if (P->apply_mode != 1 && P->xr) return launch_xapply(P->view(), compute, mode, nrhs, B, st);
  return launch_trsv(P->view(), compute, mode, nrhs, B, st);
}

// zero the synchronisation state of a solve workspace
tls_status reset_solve_ws(const tls_precond_s *P, PcgWs &W, hipStream_t st) {
  FillSet F;
  F.add_i32(W.sync, 0, P->N + 8);
  F.add_i32(W.cnt, 0, P->N);
  HIPCHK(launch_fill_multi(F, st));
  return TLS_OK;
}

// R^{-1} (trans = 0) or R^{-T} (trans = 1) on nrhs FP64 vectors
tls_status apply_R(const tls_precond_s *P, int trans, int nrhs, const double *in, double *out,
                   int compute, PcgWs &W, hipStream_t st, int ld = 0) {
  SolveBufs B = bufs_of(W);
  B.in = in;
  B.out = out;
  B.ldi = B.ldo = ld;
  HIPCHK(launch_precond(P, compute, trans ? 1 : 0, nrhs, B, st));
  return TLS_OK;
}

// PCGTLS (Algorithm 3), l+1 steps, sigma2 read from device memory
tls_status pcg_run(const tls_precond_s *P, const double *sig2_dev, int nrhs, const double *rhs,
                   double *omega, int l, int compute, int strict, PcgWs &W, hipStream_t st) {
  if (l + 1 > W.L + 1) return fail(TLS_ERR_WORKSPACE, "PCG workspace sized for l <= %d", W.L);
  const int N = P->N;
  // the X application's init launch clears the run's flags itself; the
  // triangular-solve route takes a fill launch first
  const bool xclear = P->apply_mode != 1 && P->xr;
  if (!xclear) {
    FillSet F;
    F.add_i32(W.done, 0, (size_t)(W.L + 2) * nrhs);
    F.add_i32(W.neg, 0, (size_t)(W.L + 2) * nrhs);
    F.add_f64(W.trace, std::numeric_limits<double>::quiet_NaN(), (size_t)nrhs * 4 * (W.L + 2));
    HIPCHK(launch_fill_multi(F, st));
  }
  SolveBufs B = bufs_of(W);
  B.sigma2 = sig2_dev;
  B.strict = strict;
  B.in = rhs;
  B.j = 0;
  B.clear_flags = xclear ? 1 : 0;
  HIPCHK(launch_precond(P, compute, 2 /* init: s_0 = R^{-T} f */, nrhs, B, st));
  B.clear_flags = 0;
  for (int j = 0; j <= l; ++j) {
    B.j = j;
    HIPCHK(launch_precond(P, compute, 3 /* q = R^{-1} p */, nrhs, B, st));
    HIPCHK(launch_precond(P, compute, 4 /* R^{-T} q, s update */, nrhs, B, st));
  }
  if (omega) HIPCHK(launch_pcg_finish(compute, W.w, omega, (int)P->n, P->Np, nrhs, st));
  (void)N;
  return TLS_OK;
}

// ---------------------------------------------------------------------------
// Lanczos on M = R^{-T}... estimates for the precision gate (K11)
// ---------------------------------------------------------------------------
// eigenvalues of a symmetric tridiagonal matrix by bisection (Sturm counts)
void tridiag_extremes(const std::vector<double> &a, const std::vector<double> &b, double *lo,
                      double *hi) {
  const int k = (int)a.size();
  double gl = a[0], gu = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0) + (i + 1 < k ? std::fabs(b[i]) : 0);
    gl = std::min(gl, a[i] - r);
    gu = std::max(gu, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < k; ++i) {
      const double qq = (q == 0) ? 1e-300 : q;
      q = a[i] - x - b[i - 1] * b[i - 1] / qq;
      if (q < 0) ++c;
    }
    return c;
  };
  auto kth = [&](int idx) {
    double l = gl, u = gu;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (l + u);
      if (mid <= l || mid >= u) break;
      if (count_below(mid) > idx) u = mid; else l = mid;
    }
    return 0.5 * (l + u);
  };
  *lo = kth(0);
  *hi = kth(k - 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// kernel-class profiling (HIP events on the launch stream)
// ---------------------------------------------------------------------------
namespace tls {
namespace {
struct ProfRec { int cls; hipEvent_t a, b; };
struct ProfState {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<ProfRec> recs;
  int open_cls = -1;
  hipEvent_t open_ev = nullptr;
  std::vector<hipStream_t> side;   // launches on these count as PC_GATE
};
ProfState g_prof;
hipEvent_t prof_event() {
  if (g_prof.next == g_prof.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof.pool.push_back(e);
  }
  return g_prof.pool[g_prof.next++];
}
}  // namespace
void prof_note_side_stream(hipStream_t st) { g_prof.side.push_back(st); }
void prof_begin(int cls, hipStream_t st) {
  if (!g_prof.on) return;
  if (std::find(g_prof.side.begin(), g_prof.side.end(), st) != g_prof.side.end()) cls = PC_GATE;
  hipEvent_t e = prof_event();
  if (!e || hipEventRecord(e, st) != hipSuccess) return;   // this launch goes unrecorded
  g_prof.open_cls = cls;
  g_prof.open_ev = e;
}
void prof_end(hipStream_t st) {
  if (!g_prof.on || g_prof.open_cls < 0) return;
  hipEvent_t e = prof_event();
  if (e && hipEventRecord(e, st) == hipSuccess) g_prof.recs.push_back({g_prof.open_cls, g_prof.open_ev, e});
  g_prof.open_cls = -1;
}
}  // namespace tls

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *tls_last_error(void) { return g_err.c_str(); }

tls_status tls_profile_start(void) {
  g_prof.on = true;
  g_prof.next = 0;
  g_prof.recs.clear();
  g_prof.open_cls = -1;
  return TLS_OK;
}

tls_status tls_profile_stop(tls_kernel_times *out) {
  g_prof.on = false;
  tls_kernel_times t{};
  for (const ProfRec &r : g_prof.recs) {
    HIPCHK(hipEventSynchronize(r.b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    if (r.cls >= 0 && r.cls < TLS_PROF_CLASSES) {
      t.launches[r.cls]++;
      t.total_ms[r.cls] += ms;
    }
  }
  g_prof.recs.clear();
  g_prof.next = 0;
  if (out) *out = t;
  return TLS_OK;
}
const char *tls_version(void) { return "libtls 0.1 (gfx950)"; }

void tls_default_opts(tls_rqi_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->u_p = TLS_FP64;
  o->kmax = 60;
  o->stop_patience = 1;
  o->stop_ge = 0;
  o->ls_corrections = 1;
  o->strict_pd = 0;
  o->shift_clamp = 0;
  o->refine_sweeps = 0;
  o->refine_pcg_steps = 8;
  o->allow_escalate = 0;
  o->gate_enforce = 0;
  o->shift_clamp_tau = 0.9;
  o->sigma0_hint = -1.0;
  o->psi_tie = 4.0;
  o->step_margin = 1;
  o->x_snapshots = nullptr;
  o->features = 0;
  o->mlp_theta = nullptr;
  o->mlp_norm = nullptr;
}

size_t tls_factor_workspace_size(const tls_matrix *A, int32_t u_q) {
  (void)u_q;
  if (check_matrix(A) != TLS_OK) return 0;
  Carver c(nullptr);
  carve_factor(c, A->m, A->n, A->nnz, A->format, u_q != TLS_FP64, 0, 1);
  return c.size();
}

size_t tls_factor_qr_workspace_size(const tls_matrix *A, int32_t u_q) {
  (void)u_q;
  if (check_matrix(A) != TLS_OK) return 0;
  Carver c(nullptr);
  carve_factor(c, A->m, A->n, A->nnz, A->format, 0, 1, 1);
  return c.size();
}

size_t tls_precond_import_workspace_size(int64_t n) {
  if (n <= 0) return 0;
  Carver c(nullptr);
  carve_factor(c, n + 1, n, 0, TLS_DENSE_COLMAJOR, 0);
  return c.size();
}

void tls_precond_destroy(tls_precond P) { delete P; }

tls_status tls_precond_set_apply(tls_precond P, int32_t mode) {
  if (!P) return fail(TLS_ERR_ARG, "P is NULL");
  if (mode < 0 || mode > 2) return fail(TLS_ERR_ARG, "apply mode must be 0, 1 or 2");
  P->apply_mode = mode;
  return TLS_OK;
}

tls_status tls_precond_info(const tls_precond P, int64_t *n, int32_t *storage, tls_gate_report *rep) {
  if (!P) return fail(TLS_ERR_ARG, "P is NULL");
  if (n) *n = P->n;
  if (storage) *storage = P->storage;
  if (rep) {
    TRY(gate_finish(P));   // the report is complete once the gate's runs are
    *rep = P->rep;
  }
  return TLS_OK;
}

}  // extern "C"

namespace {

// form the Gram matrix of the scaled, u_q-rounded A in G (compute precision)
tls_status form_gram(const tls_matrix *A, tls_precond_s *P, FactorWs &W, int uq, int compute,
                     hipStream_t st) {
  const int n = (int)A->n, Np = P->Np;
  if (A->format == TLS_CSR) {
    HIPCHK(launch_quantize_sparse(A->nnz, A->col_idx, A->val, W.d, P->scaled, uq, compute, W.valq, st));
    HIPCHK(launch_quantize_csc(n, W.col_ptr, W.cval, W.d, P->scaled, uq, compute, W.cvalq, st));
    HIPCHK(launch_gram_sparse((int)A->m, n, Np, A->row_ptr, A->col_idx, W.valq, W.col_ptr,
                              W.row_idx, W.cvalq, compute, W.G, st));
  } else {
    if (uq != TLS_FP64 && !W.cast)
      return fail(TLS_ERR_WORKSPACE, "factor workspace sized for FP64 cannot hold a u_q = %d cast of A", uq);
    HIPCHK(launch_gram_mfma((int)A->m, n, Np, A->ld, A->val, W.d, P->scaled, uq, W.cast, W.G, W.gpart, st));
  }
  HIPCHK(launch_gram_pad(n, Np, compute, W.G, st));
  return TLS_OK;
}

// the factor as the gate's runs apply it: a view that owns no events, with
// the row GEMV of the explicit inverse (one workgroup per 64-row block) so
// that a run on the side stream, overlapping a solve, holds about N CUs
// instead of the whole chip
tls_precond_s gate_view(const tls_precond_s *P) {
  tls_precond_s Q = *P;
  // the copy owns nothing: its destructor must release none of P's handles
  Q.ev_fork = Q.ev_pair = Q.ev_cert = Q.ev_ride = Q.ev_rows = nullptr;
  Q.rc_todo = Q.rc_inflight = 0;
  Q.hgate = nullptr;
  Q.gate_pending = 0;
  if (Q.xr && Q.xc) Q.apply_mode = 2;
  return Q;
}

// Lanczos for the gate estimates (eigenvalues 1/sigma_i^2): run 0 on
// R_hat^{-1} R_hat^{-T} (the scaled A D^{-1}), run 1 on R^{-1} R^{-T} with
// R = R_hat D (A itself). Both recurrences share each 2-RHS application of
// the preconditioner; all of it stays on the device and the two
// tridiagonal matrices are read back once (collect_pair). Extremal
// eigenvalues of each tridiagonal matrix come from bisection on the host.
tls_status enqueue_pair(tls_precond_s *P, FactorWs &W, hipStream_t st) {
  const int n = (int)P->n, Np = P->Np;
  const int K = std::min(LANCZOS_STEPS, n);
  double *V = W.lz;                                   // [2][K+1][Np]
  double *inb = W.lz + (size_t)2 * (LANCZOS_STEPS + 1) * Np;     // [2][Np] operator input
  double *tmp = inb + (size_t)2 * Np;                            // [2][Np] R^{-T} output
  double *outb = tmp + (size_t)2 * Np;                           // [2][Np]
  double *ones = outb + (size_t)2 * Np;                          // [Np]
  PcgWs S{};
  S.sync = W.sync;
  S.chain = ones + Np;                                           // [2][Np]
  S.L = 0;
  S.cpart = W.yinv;     // free after the inversion
  S.cnt = W.cnt;
  double *ab = W.lzs;                                 // [2][2K+2]
  tls_precond_s Q = gate_view(P);
  // a sparse A's solve is latency-bound launches too: there the estimates
  // take the split GEMV (the whole chip, 7 instead of 17 us per apply at
  // n = 2000) and the verdict comes earlier; beside a dense solve's
  // bandwidth-bound passes they keep the row GEMV (about N CUs)
  if (P->format == TLS_CSR) Q.apply_mode = P->apply_mode;
  Q.dsc64 = ones;                                     // apply R_hat alone
  // v_0 = ones/sqrt(n) for both runs; operator input [v0, D^{-1} v0]
  const double v0 = 1.0 / std::sqrt((double)n);
  {
    FillSet F;
    F.add_i32(W.sync, 0, P->N + 8);
    F.add_i32(W.cnt, 0, P->N);
    F.add_f64(ones, 1.0, (size_t)Np);
    F.add_f64(V, v0, (size_t)n);
    F.add_f64(V + (size_t)(K + 1) * Np, v0, (size_t)n);
    F.add_f64(inb, v0, (size_t)n);
    HIPCHK(launch_fill_multi(F, st));
  }
  HIPCHK(launch_scale_copy(n, P->dsc64, v0, inb + Np, st));           // v0 D^{-1} 1
  {
    // per run: alpha, beta = 0, active = 1, steps = 0 (disjoint regions)
    FillSet F;
    for (int run = 0; run < 2; ++run) {
      double *abr = ab + (size_t)run * (2 * K + 2);
      F.add_f64(abr, 0.0, 2 * (size_t)K);
      F.add_f64(abr + 2 * K, 1.0, 1);
      F.add_f64(abr + 2 * K + 1, 0.0, 1);
    }
    HIPCHK(launch_fill_multi(F, st));
  }
  // the apply kernels read [nrhs][n]-packed inputs: pack with stride n
  tls_status s = TLS_OK;
  for (int k = 0; k < K && s == TLS_OK; ++k) {
    s = apply_R(&Q, 1, 2, inb, tmp, TLS_FP64, S, st, Np);
    if (s == TLS_OK) s = apply_R(&Q, 0, 2, tmp, outb, TLS_FP64, S, st, Np);
    if (s == TLS_OK && launch_lanczos_orth(n, Np, k, K, V, outb, inb, P->dsc64, ab, st) != hipSuccess)
      s = fail(TLS_ERR_HIP, "Lanczos orthogonalization launch failed");
  }
  if (s == TLS_OK)   // the two tridiagonal matrices into the pinned block
    HIPCHK(hipMemcpyAsync(P->hgate, ab, 2 * (2 * K + 2) * sizeof(double), hipMemcpyDeviceToHost, st));
  return s;
}

// the two tridiagonal matrices (in the pinned block once ev_pair has
// completed) and the estimates: kappa(A D^{-1}) and sigma'_n(A), sigma'_1(A)
tls_status collect_pair(tls_precond_s *P) {
  const int K = std::min(LANCZOS_STEPS, (int)P->n);
  const double *h = P->hgate;
  double lam[2][2];
  int steps[2];
  for (int run = 0; run < 2; ++run) {
    const double *hr = h + run * (2 * K + 2);
    const int done = (int)hr[2 * K + 1];
    std::vector<double> a(hr, hr + done), b(hr + K, hr + K + std::max(done - 1, 0));
    tridiag_extremes(a, b, &lam[run][0], &lam[run][1]);
    steps[run] = done;
  }
  tls_gate_report &R = P->rep;
  P->smin_s = 1.0 / std::sqrt(lam[0][1]);
  P->smax_s = 1.0 / std::sqrt(std::max(lam[0][0], 1e-300));
  R.sigma_n_est = 1.0 / std::sqrt(lam[1][1]);
  R.sigma_1_est = 1.0 / std::sqrt(std::max(lam[1][0], 1e-300));
  R.lanczos_steps = steps[1];
  P->have_sigma_n = 1;
  // the A-only constraints of Section 3.1 from the estimates
  const double n = (double)P->n;
  const double smin_s = P->smin_s, smax_s = P->smax_s;
  const double kap = P->scaled ? smax_s / smin_s : R.sigma_1_est / R.sigma_n_est;
  R.kappa_est = kap;
  // ||A D^{-1}||_F = sqrt(n) exactly when scaled
  R.kappaF_est = P->scaled ? std::sqrt(n) / smin_s : std::numeric_limits<double>::quiet_NaN();
  R.lam_min_H = smin_s * smin_s;
  R.bound5 = 1.0 / kap;
  R.bound_chol = 1.0 / (kap * kap);
  R.bound_wilkinson = 1.0 / (20.0 * std::pow(n, 1.5) * kap * kap);
  R.bound_hp = R.lam_min_H / ((2.0 * R.lam_min_H + n) * (n + 1.0));
  R.u_q = unit_roundoff(P->uq);
  int v = R.verdict & ~(1 | 2 | 4);
  if (R.u_q < R.bound5) v |= 1;
  if (R.u_q < R.bound_chol) v |= 2;
  if (R.u_q < R.bound_hp) v |= 4;
  R.verdict = v;
  P->have_kappa = 1;
  return TLS_OK;
}

// A-posteriori certificate of the factor: extreme Ritz values of
// M = R^{-T} A^T A R^{-1} after QUALITY_STEPS Lanczos steps (products with A
// and the applications of R in FP64). M = I for the exact factor. Its
// buffers are its own, so it may run beside enqueue_pair. A step k takes
// A^T A R^{-1} v_k into tn (cert_product or a solve's fused pass), then
// cert_after_product: R^{-T} of it, the Lanczos recurrence, and R^{-1} v_{k+1}
// into tmp for the next product (after the last step: the read-back).
struct CertRun {
  int K;
  double *Vb, *inb, *tmp, *outb, *tn, *ab;
  PcgWs S;
  tls_precond_s Q;
};
CertRun cert_run(tls_precond_s *P, FactorWs &W, int on_main) {
  const int Np = P->Np;
  CertRun C{};
  C.K = std::min(QUALITY_STEPS, (int)P->n);
  C.Vb = W.qlz;                                             // [K+1][Np]
  C.inb = W.qlz + (size_t)(QUALITY_STEPS + 1) * Np;          // operator input
  C.tmp = C.inb + (size_t)2 * Np;
  C.outb = C.tmp + (size_t)2 * Np;
  C.tn = C.outb + (size_t)2 * Np;
  C.S.sync = W.qsync;
  C.S.chain = C.tn + Np;                                    // [2][Np]
  C.S.L = 0;
  C.S.cpart = W.qpart;
  C.S.cnt = W.qcnt;
  C.ab = W.qlzs;
  C.Q = gate_view(P);
  if (on_main) C.Q.apply_mode = P->apply_mode;   // the whole chip is the run's
  return C;
}
// v_0 = ones / sqrt(n), the recurrence's scalars, and R^{-1} v_0
tls_status cert_begin(tls_precond_s *P, FactorWs &W, hipStream_t st, int on_main) {
  CertRun C = cert_run(P, W, on_main);
  const int n = (int)P->n;
  const double v0 = 1.0 / std::sqrt((double)n);
  {
    FillSet F;
    F.add_i32(W.qsync, 0, P->N + 8);
    F.add_i32(W.qcnt, 0, P->N);
    F.add_f64(C.Vb, v0, (size_t)n);
    F.add_f64(C.inb, v0, (size_t)n);
    F.add_f64(C.ab, 0.0, 2 * (size_t)C.K);
    F.add_f64(C.ab + 2 * C.K, 1.0, 1);
    F.add_f64(C.ab + 2 * C.K + 1, 0.0, 1);
    HIPCHK(launch_fill_multi(F, st));
  }
  TRY(apply_R(&C.Q, 0, 1, C.inb, C.tmp, TLS_FP64, C.S, st));    // R^{-1} v_0
  return TLS_OK;
}
tls_status cert_after_product(tls_precond_s *P, FactorWs &W, hipStream_t st, int on_main, int k) {
  CertRun C = cert_run(P, W, on_main);
  const int n = (int)P->n, Np = P->Np;
  TRY(apply_R(&C.Q, 1, 1, C.tn, C.outb, TLS_FP64, C.S, st));    // R^{-T} A^T A R^{-1} v_k
  HIPCHK(launch_lanczos_orth(n, Np, k, C.K, C.Vb, C.outb, C.inb, P->dsc64, C.ab, st, 1));
  if (k + 1 < C.K) {
    TRY(apply_R(&C.Q, 0, 1, C.inb, C.tmp, TLS_FP64, C.S, st));  // R^{-1} v_{k+1}
  } else {
    HIPCHK(hipMemcpyAsync(P->hgate + 2 * (2 * LANCZOS_STEPS + 2), C.ab, (2 * C.K + 2) * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  }
  return TLS_OK;
}
// the product of step k on its own: A^T A R^{-1} v_k into tn
tls_status cert_product(tls_precond_s *P, FactorWs &W, const MatView &V, hipStream_t st) {
  CertRun C = cert_run(P, W, 0);
  if (V.at) {                                              // one pass over the row copy
    HIPCHK(launch_rowpass(V, nullptr, C.tmp, nullptr, nullptr, W.qppart, st));
    HIPCHK(launch_rowpass_sum(V, W.qppart, -1.0, C.tn, st));
  } else {
    HIPCHK(launch_matvec(V, C.tmp, W.tm, st));               // A R^{-1} v
    HIPCHK(launch_rmatvec(V, W.tm, C.tn, st));               // A^T A R^{-1} v
  }
  return TLS_OK;
}
// the whole run on st
tls_status enqueue_cert(tls_precond_s *P, FactorWs &W, const MatView &V, hipStream_t st, int on_main) {
  TRY(cert_begin(P, W, st, on_main));
  for (int k = 0; k < std::min(QUALITY_STEPS, (int)P->n); ++k) {
    TRY(cert_product(P, W, V, st));
    TRY(cert_after_product(P, W, st, on_main, k));
  }
  return TLS_OK;
}
// the dense row copy as the certificate's passes see it (no caller matrix
// needed: the copy is the factor workspace's)
MatView rowcopy_view(const tls_precond_s *P) {
  MatView V{};
  V.format = TLS_DENSE_COLMAJOR;
  V.m = (int)P->m;
  V.n = (int)P->n;
  V.at = P->at;
  V.ldr = P->ldr;
  return V;
}

// the certificate's tridiagonal matrix (pinned block, after ev_cert)
tls_status collect_cert(tls_precond_s *P) {
  const int K = std::min(QUALITY_STEPS, (int)P->n);
  const double *h = P->hgate + 2 * (2 * LANCZOS_STEPS + 2);
  const int done = std::max(1, (int)h[2 * K + 1]);
  std::vector<double> a(h, h + done), b(h + K, h + K + done - 1);
  double lo = 0, hi = 0;
  tridiag_extremes(a, b, &lo, &hi);
  P->rep.quality_lo = lo;
  P->rep.quality_hi = hi;
  P->have_quality = 1;
  return TLS_OK;
}

// one side stream per device, created once (default priority, non-blocking
// so that work on the legacy default stream does not serialize with it);
// it lives until the process ends. Pinned host blocks for the gate's
// read-back come from a per-device free list (allocated once, reused).
constexpr size_t GATE_HOST_DOUBLES = 2 * (2 * LANCZOS_STEPS + 2) + (2 * QUALITY_STEPS + 2);
// every block of the pool: the gate's read-back, or the solve's scalar
// read-back (64 doubles and a flag)
constexpr size_t PINNED_DOUBLES = GATE_HOST_DOUBLES > 72 ? GATE_HOST_DOUBLES : 72;
std::mutex g_side_mu;
std::map<std::pair<int, int>, hipStream_t> g_side_pool;
std::map<int, std::vector<double *>> g_pinned_free;

// side stream `which` (0: the gate's estimates and a sparse certificate,
// 1: a dense certificate's work between the solve's passes)
hipError_t side_stream(hipStream_t *out, int which = 0) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_side_mu);
  auto it = g_side_pool.find({dev, which});
  if (it == g_side_pool.end()) {
    hipStream_t a = nullptr;
    e = hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    it = g_side_pool.emplace(std::make_pair(dev, which), a).first;
    prof_note_side_stream(a);
  }
  *out = it->second;
  return hipSuccess;
}
hipError_t pinned_take(double **out, int *dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_side_mu);
  auto &fl = g_pinned_free[dev];
  if (!fl.empty()) {
    *out = fl.back();
    fl.pop_back();
  } else {
    e = hipHostMalloc((void **)out, PINNED_DOUBLES * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return e;
  }
  *dev_out = dev;
  return hipSuccess;
}
void pinned_give(double *p, int dev) {
  std::lock_guard<std::mutex> lk(g_side_mu);
  g_pinned_free[dev].push_back(p);
}

// a pinned block for the length of a solve; returned to the pool on every
// exit (declare it before the event that guards copies into it, so that the
// event is waited for first)
struct PinnedBlock {
  double *p = nullptr;
  int dev = 0;
  PinnedBlock() = default;
  PinnedBlock(const PinnedBlock &) = delete;
  PinnedBlock &operator=(const PinnedBlock &) = delete;
  ~PinnedBlock() {
    if (p) pinned_give(p, dev);
  }
};
// an event recorded after copies into host memory; destruction waits for it,
// so no copy is still in flight when its target is reused
struct CopyEvent {
  hipEvent_t e = nullptr;
  CopyEvent() = default;
  CopyEvent(const CopyEvent &) = delete;
  CopyEvent &operator=(const CopyEvent &) = delete;
  ~CopyEvent() {
    if (e) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  }
};

}  // namespace

tls_precond_s::~tls_precond_s() {
  if (gate_pending) {
    (void)hipStreamSynchronize(side);
    if (side2) (void)hipStreamSynchronize(side2);
  }
  if (rc_inflight && side2) (void)hipStreamSynchronize(side2);   // a factorization that failed midway
  for (hipEvent_t e : {ev_fork, ev_pair, ev_cert, ev_ride, ev_rows})
    if (e) (void)hipEventDestroy(e);
  if (hgate) pinned_give(hgate, hgate_dev);
}

namespace {

// the gate's Lanczos runs after everything enqueued on st so far: the
// estimates on the side stream, the certificate beside them on side2 (a
// sparse A) or riding on the solve's passes (a dense A with a row copy)
tls_status gate_start(tls_precond_s *P, FactorWs &W, const MatView &V, hipStream_t st) {
  HIPCHK(side_stream(&P->side, 0));
  HIPCHK(side_stream(&P->side2, 1));
  if (!P->hgate) HIPCHK(pinned_take(&P->hgate, &P->hgate_dev));
  for (hipEvent_t *e : {&P->ev_fork, &P->ev_pair, &P->ev_cert, &P->ev_ride})
    if (!*e) HIPCHK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  P->have_kappa = P->have_sigma_n = P->have_quality = 0;
  HIPCHK(hipEventRecord(P->ev_fork, st));
  HIPCHK(hipStreamWaitEvent(P->side, P->ev_fork, 0));
  // from here on the runs may be in flight: mark them before any early return
  P->gate_pending = 1;
  P->cert_todo = 0;
  // the certificate of a dense A is started on the caller's stream, and its
  // six products ride on the solve's passes over the row copy (each pass
  // reads A once for both; a pass of its own would cost as much as the
  // solve's, on the same HBM). Steps that no pass took are finished on the
  // side stream when the verdict is needed (cert_finish). A sparse A's
  // certificate (latency-bound launches, like the solve's) runs whole on
  // the side stream.
  const bool ride = V.at != nullptr;
  tls_status s1 = TLS_OK;
  hipError_t e1 = hipSuccess;
  if (ride) {
    s1 = cert_begin(P, W, st, 0);
    e1 = hipEventRecord(P->ev_cert, st);
    P->cert_todo = 1;
    P->cert_k = 0;
  }
  // the estimates on the side stream (after the caller's stream work above,
  // so that the factor's stream never waits for these launches); a sparse
  // certificate beside them on side2, so that the verdict waits for the
  // longer of the two runs rather than their sum
  tls_status s0 = enqueue_pair(P, W, P->side);
  hipError_t e0 = hipEventRecord(P->ev_pair, P->side);
  if (!ride) {
    hipError_t ew = hipStreamWaitEvent(P->side2, P->ev_fork, 0);
    s1 = (ew == hipSuccess) ? enqueue_cert(P, W, V, P->side2, 1) : fail(TLS_ERR_HIP, "hipStreamWaitEvent failed");
    e1 = hipEventRecord(P->ev_cert, P->side2);
  }
  if (e0 != hipSuccess || e1 != hipSuccess || s0 != TLS_OK || s1 != TLS_OK) {
    (void)hipStreamSynchronize(P->side);
    (void)hipStreamSynchronize(P->side2);
    (void)hipStreamSynchronize(st);
    P->gate_pending = 0;
    P->cert_todo = 0;
    if (s0 != TLS_OK) return s0;
    if (s1 != TLS_OK) return s1;
    return fail(TLS_ERR_HIP, "hipEventRecord failed on the side stream");
  }
  return TLS_OK;
}

FactorWs factor_ws_of(const tls_precond_s *P);

// both runs finished (without waiting)
bool gate_ready(const tls_precond_s *P) {
  return !P->gate_pending || (!P->cert_todo && hipEventQuery(P->ev_pair) == hipSuccess &&
                              hipEventQuery(P->ev_cert) == hipSuccess);
}

// the solve's pass at x also takes certificate step cert_k (when one is due):
// r = b - A x with A^T r, and A^T A R^{-1} v_k, in one read of the row copy.
// The step's other work (R^{-T}, the recurrence, R^{-1} v_{k+1}) runs on
// side2 beside the solve's own kernels; the next riding pass waits for it.
bool cert_rides(const tls_precond_s *P, const MatView &V) {
  return P->gate_pending && P->cert_todo && V.at && V.at == P->at;
}
tls_status cert_ride_pass(tls_precond_s *P, const MatView &V, const double *b, const double *x, double *r,
                          double *part_r, double *ppart, hipStream_t st) {
  FactorWs W = factor_ws_of(P);
  CertRun C = cert_run(P, W, 0);
  HIPCHK(hipStreamWaitEvent(st, P->ev_cert, 0));       // R^{-1} v_k and the partials' buffer
  HIPCHK(launch_rowpass_dual(V, b, x, r, part_r, ppart, C.tmp, W.qppart, st));
  HIPCHK(hipEventRecord(P->ev_ride, st));
  HIPCHK(hipStreamWaitEvent(P->side2, P->ev_ride, 0));
  HIPCHK(launch_rowpass_sum(V, W.qppart, 1.0, C.tn, P->side2));
  TRY(cert_after_product(P, W, P->side2, 0, P->cert_k));
  HIPCHK(hipEventRecord(P->ev_cert, P->side2));
  if (++P->cert_k == C.K) P->cert_todo = 0;
  return TLS_OK;
}

// the certificate's remaining steps on side2, after the work enqueued for it
// so far (ev_cert)
tls_status cert_finish(tls_precond_s *P) {
  if (!P->cert_todo) return TLS_OK;
  FactorWs W = factor_ws_of(P);
  const MatView V = rowcopy_view(P);
  HIPCHK(hipStreamWaitEvent(P->side2, P->ev_cert, 0));
  const int K = std::min(QUALITY_STEPS, (int)P->n);
  for (; P->cert_k < K; ++P->cert_k) {
    TRY(cert_product(P, W, V, P->side2));
    TRY(cert_after_product(P, W, P->side2, 0, P->cert_k));
  }
  HIPCHK(hipEventRecord(P->ev_cert, P->side2));
  P->cert_todo = 0;
  return TLS_OK;
}

// wait for both runs and evaluate them on the host
tls_status gate_finish(tls_precond_s *P) {
  if (!P->gate_pending) return TLS_OK;
  TRY(cert_finish(P));
  P->gate_pending = 0;
  HIPCHK(hipEventSynchronize(P->ev_pair));
  HIPCHK(hipEventSynchronize(P->ev_cert));
  TRY(collect_pair(P));
  TRY(collect_cert(P));
  return TLS_OK;
}

// the estimates alone, synchronously on st (the shift clamp of a
// preconditioner whose gate never ran, e.g. an imported FP64 factor)
tls_status estimate_sigma_n(tls_precond_s *P, FactorWs &W, hipStream_t st) {
  TRY(gate_finish(P));
  if (!P->hgate) HIPCHK(pinned_take(&P->hgate, &P->hgate_dev));
  TRY(enqueue_pair(P, W, st));
  HIPCHK(hipStreamSynchronize(st));
  return collect_pair(P);
}

// the b-dependent part of the gate: constraint (6) with sigma_{n+1} <=
// sigma_0 and the estimates, and the certificate's verdict
void gate_decide(tls_precond_s *P, double sigma_ls) {
  tls_gate_report &R = P->rep;
  const double ratio = (sigma_ls / R.sigma_n_est) * (sigma_ls / R.sigma_n_est);
  R.ctilde_min = 1.0 - ratio;
  R.bound6 = (1.0 - ratio) / R.kappaF_est;
  R.verdict &= ~(8 | 16);
  if (R.u_q < R.bound6) R.verdict |= 8;
  // Ritz values lie inside the spectrum, so the window gives up
  // CERT_RITZ_MARGIN on each side: the six-step Ritz values of the
  // benchmark workloads' FP16, BF16 and split-BF16 factors came within 0.0032
  // of the exact extreme eigenvalues (dense eigenvalues on the host). The
  // products are FP64 throughout, so their rounding adds nothing visible.
  R.cert_margin = CERT_RITZ_MARGIN;
  if (R.quality_lo - R.cert_margin >= 0.5 && R.quality_hi + R.cert_margin <= 1.5) R.verdict |= 16;
}

FactorWs factor_ws_of(const tls_precond_s *P) {
  Carver c(P->fws_base);
  return carve_factor(c, P->fws_m, P->n, P->nnz, P->format, P->fws_cast, P->method, P->fws_rows);
}

// tiles of the storage precision, diagonal-tile inverses and the explicit
// inverse from the factor R_hat in G (the Cholesky steps leave its diagonal
// tiles in W.rdiag: chol = 1)
tls_status finish_factor(tls_precond_s *P, FactorWs &W, int uq, int compute, int chol, hipStream_t st) {
  const int sq = storage_of(uq);   // the split BF16 factor is stored in FP32
  HIPCHK(launch_pack_tiles(P->N, P->Np, compute, W.G, chol ? W.rdiag : nullptr, sq, W.tiles, st));
  HIPCHK(launch_diag_inverse(P->N, sq, W.tiles, W.dinv64, W.dinv32, st));
  P->storage = sq;
  P->uq = uq;
  P->xstorage = (sq == TLS_FP64) ? TLS_FP64 : TLS_FP32;
  HIPCHK(launch_invert(P->N, sq, W.tiles, W.dinv64, (double *)W.G, W.yinv, P->xstorage, W.xr, W.xc, st));
  P->xr = W.xr;
  P->xc = W.xc;
  return TLS_OK;
}

// wait for gate runs started on a factor that turned out broken
void gate_drain(tls_precond_s *P) {
  if (P->gate_pending) {
    (void)hipStreamSynchronize(P->side);
    (void)hipStreamSynchronize(P->side2);
    P->gate_pending = 0;
    P->cert_todo = 0;
  }
}

// the one read-back of a factorization (synchronizes the stream): breakdown
// info, then the finite-input flag (NaN or Inf in A takes precedence) and the
// column statistics
tls_status read_factor_status(tls_precond_s *P, const FactorWs &W, hipStream_t st, int *info) {
  alignas(8) char stat[72];
  HIPCHK(hipMemcpyAsync(stat, W.info, sizeof(stat), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int flag = 0;
  double ds[5];
  std::memcpy(info, stat, sizeof(int));
  std::memcpy(&flag, stat + 16, sizeof(int));
  std::memcpy(ds, stat + 32, sizeof(ds));
  if (flag) return fail(TLS_ERR_NONFINITE, "A contains NaN or Inf");
  P->normA_F2 = ds[0];
  for (int i = 0; i < 4; ++i) P->lnd[i] = ds[1 + i];
  return TLS_OK;
}

// R_hat from the Householder QR of the scaled, u_q-rounded A (Section 3)
tls_status factor_qr_once(const tls_matrix *A, tls_precond_s *P, FactorWs &W, int uq, hipStream_t st,
                          int *breakdown, const MatView *gate) {
  const int compute = (uq == TLS_FP64) ? TLS_FP64 : TLS_FP32;
  *breakdown = 0;
  if (!W.qrw) return fail(TLS_ERR_WORKSPACE, "factor workspace was not sized for QR");
  HIPCHK(launch_fill_i32(W.info, INT32_MAX, 1, st));
  HIPCHK(launch_qr_factor(A->m, (int)A->n, P->Np, A->format, A->ld, A->val, A->row_ptr, A->col_idx, W.d,
                          P->scaled, uq, compute, W.qrw, W.G, W.info, st));
  TRY(finish_factor(P, W, uq, compute, 0, st));   // enqueued before the pivot check
  if (gate) TRY(gate_start(P, W, *gate, st));
  int info = 0;
  const tls_status rs = read_factor_status(P, W, st, &info);
  if (rs != TLS_OK || info != INT32_MAX) gate_drain(P);
  if (rs != TLS_OK) return rs;
  if (info != INT32_MAX) {
    *breakdown = info;
    return fail(TLS_ERR_NOT_SPD, "QR: zero or non-finite pivot at column %d", info - 1);
  }
  return TLS_OK;
}

// gate != NULL: the gate's runs on the new factor are started before the
// breakdown flag is read, so that their enqueueing overlaps the factor's last
// kernels; after a breakdown they are drained and started again with the
// next attempt
// The row-major copy of a dense A (read by every pass of the solve, not by
// the factorization) is made once, on side2, beside the second half of the
// Cholesky chain and the inverse: launches bound by the panel's latency,
// which leave HBM and most CUs idle (beside the wide early launches it would
// slow the chain's trailing updates). The caller's stream waits for it before the
// factorization's status is read, so the call returns with the copy made.
// The fork event was recorded on st by launch_cholesky.
tls_status start_rowcopy(tls_precond_s *P) {
  P->rc_todo = 0;
  HIPCHK(side_stream(&P->side2, 1));
  HIPCHK(hipStreamWaitEvent(P->side2, P->ev_rows, 0));
  P->rc_inflight = 1;
  HIPCHK(launch_rowcopy_dense((int)P->m, (int)P->n, P->rc_ld, P->rc_src, P->ldr, P->at, P->side2));
  HIPCHK(hipEventRecord(P->ev_rows, P->side2));
  return TLS_OK;
}
tls_status join_rowcopy(tls_precond_s *P, hipStream_t st) {
  if (!P->rc_inflight) return TLS_OK;
  HIPCHK(hipStreamWaitEvent(st, P->ev_rows, 0));
  P->rc_inflight = 0;
  return TLS_OK;
}

tls_status factor_once(const tls_matrix *A, tls_precond_s *P, FactorWs &W, int uq,
                       hipStream_t st, int *breakdown, const MatView *gate) {
  if (P->method == 1) {
    if (P->rc_todo) {
      P->rc_todo = 0;
      HIPCHK(launch_rowcopy_dense((int)P->m, (int)P->n, P->rc_ld, P->rc_src, P->ldr, P->at, st));
    }
    return factor_qr_once(A, P, W, uq, st, breakdown, gate);
  }
  const int compute = (uq == TLS_FP64) ? TLS_FP64 : TLS_FP32;
  const int n = (int)A->n;
  *breakdown = 0;
  for (int attempt = 0; attempt < 4; ++attempt) {
    TRY(form_gram(A, P, W, uq, compute, st));
    if (attempt > 0) {
      // diagonal perturbation 2^(attempt-1) n u_q (scaled H has unit diagonal)
      const double shift = std::ldexp(1.0, attempt - 1) * n * unit_roundoff(uq) *
                           (P->scaled ? 1.0 : 1.0);
      HIPCHK(launch_gram_shift(n, P->Np, compute, W.G, shift, st));
      P->rep.chol_retries = attempt;
    }
    HIPCHK(launch_fill_i32(W.info, INT32_MAX, 1, st));
    const bool fork = P->rc_todo;
    if (fork && !P->ev_rows) HIPCHK(hipEventCreateWithFlags(&P->ev_rows, hipEventDisableTiming));
    HIPCHK(launch_cholesky(P->N, P->Np, compute, W.G, W.rdiag, W.info, st, fork ? P->ev_rows : nullptr));
    if (fork) TRY(start_rowcopy(P));
    // packing, diagonal inverses and the explicit inverse are enqueued before
    // the breakdown flag is read (one synchronization); after a breakdown the
    // next attempt redoes them
    TRY(finish_factor(P, W, uq, compute, 1, st));
    TRY(join_rowcopy(P, st));
    if (gate) TRY(gate_start(P, W, *gate, st));
    int info = 0;
    const tls_status rs = read_factor_status(P, W, st, &info);
    if (rs != TLS_OK || info != INT32_MAX) gate_drain(P);
    if (rs != TLS_OK) return rs;
    if (info == INT32_MAX) return TLS_OK;
    *breakdown = info;
    if (!P->scaled) break;   // the shift ladder is defined for the scaled matrix
  }
  return fail(TLS_ERR_NOT_SPD, "Cholesky breakdown at column %d", *breakdown - 1);
}

}  // namespace

namespace {

tls_status factor_precond(const tls_matrix *A, int32_t u_q, int32_t scaling, int32_t allow_escalate, void *ws,
                          size_t ws_bytes, hipStream_t stream, tls_precond *out, tls_gate_report *rep,
                          int method) {
  try {
    TRY(check_matrix(A));
    TRY(check_prec(u_q, "u_q"));
    if (!out) return fail(TLS_ERR_ARG, "out is NULL");
    if (!ws || ((uintptr_t)ws & 255)) return fail(TLS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (!scaling && u_q != TLS_FP64) return fail(TLS_ERR_ARG, "unscaled factorization is FP64 only");
    if (method && u_q == TLS_BF16X3) return fail(TLS_ERR_ARG, "the split BF16 precision is a Gram (Cholesky) route only");
    const size_t need = method ? tls_factor_qr_workspace_size(A, u_q) : tls_factor_workspace_size(A, u_q);
    if (ws_bytes < need) return fail(TLS_ERR_WORKSPACE, "factor workspace %zu < %zu bytes", ws_bytes, need);
    const int cast = (u_q != TLS_FP64) && !method;
    Carver c(ws);
    FactorWs W = carve_factor(c, A->m, A->n, A->nnz, A->format, cast, method, 1);
    auto *P = new (std::nothrow) tls_precond_s();
    if (!P) return fail(TLS_ERR_ARG, "out of host memory");
    std::unique_ptr<tls_precond_s> guard(P);
    const int n = (int)A->n;
    P->n = n;
    P->Np = ceil_div(n, NB) * NB;
    P->N = P->Np / NB;
    P->m = A->m;
    P->nnz = A->nnz;
    P->format = A->format;
    P->scaled = scaling ? 1 : 0;
    P->requested = u_q;
    P->tiles = W.tiles;
    P->dinv64 = W.dinv64;
    P->dinv32 = W.dinv32;
    P->dsc64 = W.dsc64;
    P->dsc32 = W.dsc32;
    P->d = W.d;
    P->fws_base = ws;
    P->fws_m = A->m;
    P->fws_cast = cast;
    P->fws_rows = 1;
    P->method = method;
    P->rep = tls_gate_report{};
    P->rep.requested = u_q;
    P->rep.method = method;
    P->rep.sigma_n_est = P->rep.sigma_1_est = std::numeric_limits<double>::quiet_NaN();
    {
      // the solve-sync counters and the finite-input flag, in one launch
      FillSet F;
      F.add_i32(W.sync, 0, P->N + 8);
      F.add_i32(W.flag, 0, 1);
      HIPCHK(launch_fill_multi(F, stream));
    }
    // column norms: dense, with the finite-input flag in one read of A (the
    // row-major copy for the solve follows the Gram matrix: start_rowcopy);
    // CSR, from the CSC copy
    if (A->format == TLS_DENSE_COLMAJOR) {
      HIPCHK(launch_colsq_dense((int)A->m, n, A->ld, A->val, W.colsq, W.d, W.flag, stream));
      if (W.at) {
        P->at = W.at;
        P->ldr = W.ldr;
        P->rc_src = A->val;
        P->rc_ld = A->ld;
        P->rc_todo = 1;
      }
    } else {
      HIPCHK(launch_check_finite(A->val, (size_t)A->nnz, W.flag, stream));
      // the structure is checked before any kernel uses the indices (one
      // synchronization, CSR only): a malformed matrix is an argument error,
      // never an out-of-bounds access
      int *badp = W.info + 1;
      HIPCHK(launch_fill_i32(badp, 0, 1, stream));
      HIPCHK(launch_validate_csr((int)A->m, n, A->nnz, A->row_ptr, A->col_idx, badp, stream));
      int bad = 0;
      HIPCHK(hipMemcpyAsync(&bad, badp, sizeof(int), hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));
      if (bad)
        return fail(TLS_ERR_ARG, "CSR structure invalid: row_ptr must start at 0, end at nnz and not "
                    "decrease; column indices must lie in [0, n) and increase within each row");
      HIPCHK(launch_csc_build((int)A->m, n, A->nnz, A->row_ptr, A->col_idx, A->val, W.col_ptr,
                              W.row_idx, W.cval, W.tmp_row, W.tmp_val, W.fill, stream));
      HIPCHK(launch_colnorms_csc(n, W.col_ptr, W.cval, W.d, stream));
      P->col_ptr = W.col_ptr;
      P->row_idx = W.row_idx;
      P->cval = W.cval;
      P->csr_row_ptr = A->row_ptr;
      P->csr_col_idx = A->col_idx;
    }
    HIPCHK(launch_scale_vectors(n, P->Np, W.d, P->scaled, W.dsc64, W.dsc32, stream));
    // ||A||_F^2 and the statistics of ln d_j for the solve; they and the
    // finite-input flag come back with the factorization's breakdown flag
    // (read_factor_status), so no synchronization precedes the factorization
    HIPCHK(launch_dstats(n, W.d, W.dstats, stream));
    int uq = u_q;
    for (;;) {
      int bd = 0;
      const MatView gv = make_view(A, P);
      tls_status s = factor_once(A, P, W, uq, stream, &bd, uq != TLS_FP64 ? &gv : nullptr);
      if (s == TLS_OK) {
        P->rep.u_q = unit_roundoff(uq);
        // a low-precision factor is kept here even where the A-only
        // constraints fail: the decision belongs to the certificate, read in
        // the solve (which escalates if asked to); with rep == NULL the two
        // Lanczos runs finish in the background
        if (uq != TLS_FP64 && rep) TRY(gate_finish(P));   // started by factor_once
        break;
      }
      if (s != TLS_ERR_NOT_SPD || !allow_escalate || uq == TLS_FP64) return s;
      // escalate: BF16 -> FP16 -> FP32 -> FP64
      uq = (uq == TLS_BF16) ? TLS_FP16 : (uq == TLS_FP16 || uq == TLS_BF16X3) ? TLS_FP32 : TLS_FP64;
      P->rep.escalations++;
    }
    P->rep.used = P->uq;
    if (rep) *rep = P->rep;
    *out = guard.release();
    return TLS_OK;
  } catch (...) {
    return fail(TLS_ERR_ARG, "unexpected C++ exception");
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// static PCGTLS scratch for tls_pcg_step_noalloc (callers that cannot
// allocate): one array per device, resolved once per device to its device
// address. The host-side name `scratch` is only a stand-in for the symbol;
// kernels and fills always get the resolved address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[TLS_PCG_NOALLOC_MAX_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// address of the current device's copy of `scratch`, looked up with that
// device current on its first use and kept for the life of the process
tls_status pcg_scratch_of_current_device(void **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return fail(TLS_ERR_ARG, "device ordinal %d beyond the %d the static scratch table holds", dev,
                SCRATCH_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255)) return fail(TLS_ERR_HIP, "static scratch address not 256-byte aligned");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TLS_OK;
}

}  // namespace

extern "C" {

tls_status tls_gram(const tls_matrix *A, int32_t u_q, int32_t scaling, double *G, double *d, void *ws,
                    size_t ws_bytes, hipStream_t stream) {
  try {
    TRY(check_matrix(A));
    TRY(check_prec(u_q, "u_q"));
    if (A->format == TLS_CSR) return fail(TLS_ERR_ARG, "tls_gram takes a dense A");
    if (!G) return fail(TLS_ERR_ARG, "G is NULL");
    if (!scaling && u_q != TLS_FP64) return fail(TLS_ERR_ARG, "unscaled Gram matrices are FP64 only");
    if (!ws || ((uintptr_t)ws & 255)) return fail(TLS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    const size_t need = tls_factor_workspace_size(A, u_q);
    if (ws_bytes < need) return fail(TLS_ERR_WORKSPACE, "Gram workspace %zu < %zu bytes", ws_bytes, need);
    Carver c(ws);
    FactorWs W = carve_factor(c, A->m, A->n, A->nnz, A->format, u_q != TLS_FP64, 0);
    tls_precond_s P{};
    const int n = (int)A->n;
    P.n = n;
    P.Np = ceil_div(n, NB) * NB;
    P.N = P.Np / NB;
    P.scaled = scaling ? 1 : 0;
    HIPCHK(launch_colnorms_dense((int)A->m, n, A->ld, A->val, W.d, stream));
    const int compute = (u_q == TLS_FP64) ? TLS_FP64 : TLS_FP32;
    TRY(form_gram(A, &P, W, u_q, compute, stream));
    HIPCHK(launch_gram_export(n, P.Np, compute, W.G, G, stream));
    if (d) HIPCHK(hipMemcpyAsync(d, W.d, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, stream));
    return TLS_OK;
  } catch (...) {
    return fail(TLS_ERR_ARG, "unexpected C++ exception");
  }
}

tls_status tls_factor_precond(const tls_matrix *A, int32_t u_q, int32_t scaling,
                              int32_t allow_escalate, void *ws, size_t ws_bytes,
                              hipStream_t stream, tls_precond *out, tls_gate_report *rep) {
  return factor_precond(A, u_q, scaling, allow_escalate, ws, ws_bytes, stream, out, rep, 0);
}

tls_status tls_factor_precond_qr(const tls_matrix *A, int32_t u_q, int32_t scaling,
                                 int32_t allow_escalate, void *ws, size_t ws_bytes,
                                 hipStream_t stream, tls_precond *out, tls_gate_report *rep) {
  return factor_precond(A, u_q, scaling, allow_escalate, ws, ws_bytes, stream, out, rep, 1);
}

tls_status tls_precond_import(int64_t n, const double *R_host, const double *d_host, int32_t storage,
                              void *ws, size_t ws_bytes, hipStream_t stream, tls_precond *out) {
  try {
    if (n <= 0 || !R_host || !out) return fail(TLS_ERR_ARG, "bad arguments to tls_precond_import");
    TRY(check_prec(storage, "storage"));
    if (storage == TLS_BF16X3) return fail(TLS_ERR_ARG, "TLS_BF16X3 is a factor precision, not a storage format");
    if (!ws || ((uintptr_t)ws & 255)) return fail(TLS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    const size_t need = tls_precond_import_workspace_size(n);
    if (ws_bytes < need) return fail(TLS_ERR_WORKSPACE, "import workspace %zu < %zu bytes", ws_bytes, need);
    Carver c(ws);
    FactorWs W = carve_factor(c, n + 1, n, 0, TLS_DENSE_COLMAJOR, 0);
    auto P = std::make_unique<tls_precond_s>();
    P->n = n;
    P->Np = ceil_div(n, NB) * NB;
    P->N = P->Np / NB;
    P->storage = storage;
    P->uq = storage;
    P->requested = storage;
    P->scaled = d_host ? 1 : 0;
    P->tiles = W.tiles;
    P->dinv64 = W.dinv64;
    P->dinv32 = W.dinv32;
    P->dsc64 = W.dsc64;
    P->dsc32 = W.dsc32;
    P->d = W.d;
    P->fws_base = ws;
    P->fws_m = n + 1;
    P->format = TLS_DENSE_COLMAJOR;
    P->nnz = 0;
    // stage R (host) through the G region of the workspace
    HIPCHK(hipMemcpyAsync(W.G, R_host, (size_t)n * n * sizeof(double), hipMemcpyHostToDevice, stream));
    std::vector<double> dh(P->Np, 1.0);
    if (d_host) for (int64_t i = 0; i < n; ++i) dh[i] = d_host[i];
    HIPCHK(hipMemcpyAsync(W.d, dh.data(), P->Np * sizeof(double), hipMemcpyHostToDevice, stream));
    HIPCHK(launch_scale_vectors((int)n, P->Np, W.d, 1, W.dsc64, W.dsc32, stream));
    HIPCHK(launch_import_tiles((int)n, P->N, P->Np, (const double *)W.G, storage, W.tiles, stream));
    HIPCHK(launch_diag_inverse(P->N, storage, W.tiles, W.dinv64, W.dinv32, stream));
    P->xstorage = (storage == TLS_FP64) ? TLS_FP64 : TLS_FP32;
    HIPCHK(launch_invert(P->N, storage, W.tiles, W.dinv64, (double *)W.G, W.yinv, P->xstorage, W.xr,
                         W.xc, stream));
    P->xr = W.xr;
    P->xc = W.xc;
    HIPCHK(hipStreamSynchronize(stream));
    P->rep.requested = P->rep.used = storage;
    P->rep.u_q = unit_roundoff(storage);
    *out = P.release();
    return TLS_OK;
  } catch (...) {
    return fail(TLS_ERR_ARG, "unexpected C++ exception");
  }
}

tls_status tls_precond_export(const tls_precond P, double *R_host, double *d_host, hipStream_t stream) {
  if (!P || !R_host) return fail(TLS_ERR_ARG, "bad arguments to tls_precond_export");
  // tiles -> dense column-major staged in device memory right after the tiles is not
  // available here; use a temporary device buffer owned by the runtime is not allowed,
  // so the export reuses the Gram region of the factor workspace, which is free after
  // the factorization.
  const size_t bytes = (size_t)P->n * P->n * sizeof(double);
  char *tiles_end = (char *)P->tiles + (size_t)P->N * (P->N + 1) / 2 * NB * NB * 8;
  // G follows dinv64, dinv32, dsc64, dsc32, d in the carve order
  (void)tiles_end;
  Carver c((char *)P->tiles);
  c.take<char>((size_t)P->N * (P->N + 1) / 2 * NB * NB * 8);
  c.take<double>((size_t)P->N * NB * NB);
  c.take<float>((size_t)P->N * NB * NB);
  c.take<double>(P->Np);
  c.take<float>(P->Np);
  c.take<double>(P->Np);
  double *G = c.take<double>((size_t)P->Np * P->Np);
  HIPCHK(launch_export_tiles((int)P->n, P->N, P->Np, P->storage, P->tiles, G, stream));
  HIPCHK(hipMemcpyAsync(R_host, G, bytes, hipMemcpyDeviceToHost, stream));
  if (d_host) HIPCHK(hipMemcpyAsync(d_host, P->d, P->n * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return TLS_OK;
}

size_t tls_pcg_workspace_size(const tls_precond P, int32_t nrhs, int32_t l) {
  if (!P || nrhs < 1 || nrhs > 2 || l < 0) return 0;
  Carver c(nullptr);
  carve_pcg(c, P->Np, P->N, nrhs, l);
  return c.size();
}

tls_status tls_pcg_step(const tls_precond P, double sigma2, int32_t nrhs, const double *rhs,
                        double *omega, int32_t l, int32_t u_p, int32_t strict_pd, void *ws,
                        size_t ws_bytes, hipStream_t stream, double *trace) {
  try {
    if (!P) return fail(TLS_ERR_ARG, "P is NULL");
    if (nrhs < 1 || nrhs > 2) return fail(TLS_ERR_ARG, "nrhs must be 1 or 2");
    if (l < 0 || l > 4096) return fail(TLS_ERR_ARG, "l out of range");
    if (u_p != TLS_FP64 && u_p != TLS_FP32) return fail(TLS_ERR_ARG, "u_p must be FP64 or FP32");
    if (!rhs || !omega) return fail(TLS_ERR_ARG, "rhs/omega NULL");
    if (!std::isfinite(sigma2) || sigma2 < 0) return fail(TLS_ERR_ARG, "sigma2 must be finite and >= 0");
    if (!ws || ((uintptr_t)ws & 255)) return fail(TLS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    const size_t need = tls_pcg_workspace_size(P, nrhs, l);
    if (ws_bytes < need) return fail(TLS_ERR_WORKSPACE, "PCG workspace %zu < %zu bytes", ws_bytes, need);
    Carver c(ws);
    PcgWs W = carve_pcg(c, P->Np, P->N, nrhs, l);
    TRY(reset_solve_ws(P, W, stream));
    HIPCHK(launch_fill_f64(W.sigma2, sigma2, 1, stream));
    TRY(pcg_run(P, W.sigma2, nrhs, rhs, omega, l, u_p, strict_pd, W, stream));
    if (trace || strict_pd) {
      TRY(sync_status(W.sync, P->N, stream));
      if (trace) {
        HIPCHK(hipMemcpyAsync(trace, W.trace, (size_t)nrhs * 4 * (l + 2) * sizeof(double),
                              hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
      }
    }
    return TLS_OK;
  } catch (...) {
    return fail(TLS_ERR_ARG, "unexpected C++ exception");
  }
}

tls_status tls_pcg_step_noalloc(const tls_precond P, double sigma2, int32_t nrhs, const double *rhs,
                                double *omega, int32_t l, int32_t u_p, int32_t strict_pd,
                                hipStream_t stream, double *trace) {
  try {
    if (!P) return fail(TLS_ERR_ARG, "P is NULL");
    if (nrhs < 1 || nrhs > 2) return fail(TLS_ERR_ARG, "nrhs must be 1 or 2");
    if (l < 0 || l > 4096) return fail(TLS_ERR_ARG, "l out of range");
    const size_t need = tls_pcg_workspace_size(P, nrhs, l);
    if (need > TLS_PCG_NOALLOC_MAX_BYTES)
      return fail(TLS_ERR_WORKSPACE,
                  "PCGTLS for n = %lld, nrhs = %d, l = %d needs %zu bytes of scratch; the static "
                  "scratch holds %zu (use tls_pcg_step with a workspace)",
                  (long long)P->n, (int)nrhs, (int)l, need, (size_t)TLS_PCG_NOALLOC_MAX_BYTES);
    void *ws = nullptr;
    TRY(pcg_scratch_of_current_device(&ws));
    return tls_pcg_step(P, sigma2, nrhs, rhs, omega, l, u_p, strict_pd, ws,
                        (size_t)TLS_PCG_NOALLOC_MAX_BYTES, stream, trace);
  } catch (...) {
    return fail(TLS_ERR_ARG, "unexpected C++ exception");
  }
}

tls_status tls_apply_precond(const tls_precond P, int32_t trans, int32_t nrhs, const double *in,
                             double *out, int32_t u_p, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!P || !in || !out) return fail(TLS_ERR_ARG, "bad arguments to tls_apply_precond");
  if (nrhs < 1 || nrhs > 2) return fail(TLS_ERR_ARG, "nrhs must be 1 or 2");
  if (u_p != TLS_FP64 && u_p != TLS_FP32) return fail(TLS_ERR_ARG, "u_p must be FP64 or FP32");
  const size_t need = tls_pcg_workspace_size(P, nrhs, 0);
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need) return fail(TLS_ERR_WORKSPACE, "apply workspace too small (%zu < %zu)", ws_bytes, need);
  Carver c(ws);
  PcgWs W = carve_pcg(c, P->Np, P->N, nrhs, 0);
  TRY(reset_solve_ws(P, W, stream));
  TRY(apply_R(P, trans, nrhs, in, out, u_p, W, stream));
  return TLS_OK;
}

tls_status tls_round(const double *in, int64_t count, int32_t prec, double *out, hipStream_t stream) {
  TRY(check_prec(prec, "prec"));
  if (count < 0 || (count > 0 && (!in || !out))) return fail(TLS_ERR_ARG, "bad arguments to tls_round");
  HIPCHK(launch_round(in, count, prec, out, stream));
  return TLS_OK;
}

tls_status tls_matvec(const tls_matrix *A, const tls_precond P, int32_t trans, const double *x,
                      double *y, hipStream_t stream) {
  TRY(check_matrix(A));
  if (!x || !y) return fail(TLS_ERR_ARG, "x/y NULL");
  if (trans && A->format == TLS_CSR && !P) return fail(TLS_ERR_ARG, "CSR A^T x needs the CSC copy in P");
  MatView V = make_view(A, P);
  if (trans) HIPCHK(launch_rmatvec(V, x, y, stream));
  else HIPCHK(launch_matvec(V, x, y, stream));
  return TLS_OK;
}

}  // extern "C"

// ===========================================================================
// RQI driver
// ===========================================================================
namespace {

struct RqiWs {
  double *r, *f, *xbest, *rhs, *wu, *t1, *t2, *part, *scal, *rec;
  double *ppart;                         // row-pass partials (dense A with a row-major copy)
  double *ppart2, *tu;                   // the merged first step: A^T A u_0 partials, A u_0
  int *gcnt;                             // arrival count of the gradient's workgroups (psi in the last)
  double *rr, *rz, *rp, *rq, *rt, *rs;   // refinement PCG: residual, M r, direction, K p, A p, scalars
  PcgWs pcg;
};

RqiWs carve_rqi(Carver &c, int format, int64_t m, int64_t n, const tls_precond_s *P, int kmax, int L) {
  RqiWs W{};
  MatView V{};
  V.format = format;   // the block counts of the row passes depend on it
  V.m = (int)m;
  V.n = (int)n;
  const int nb = std::max({matvec_blocks(V), rmatvec_blocks(V), gradient_rows_blocks((int)n)}) + 1;
  W.r = c.take<double>(m);
  W.f = c.take<double>(n);
  W.xbest = c.take<double>(n);
  W.rhs = c.take<double>(2 * n);
  W.wu = c.take<double>(2 * n);
  W.t1 = c.take<double>(n);
  W.t2 = c.take<double>(n);
  W.part = c.take<double>(4 * (size_t)nb);   // residual and gradient partials
  W.scal = c.take<double>(64);
  W.rec = c.take<double>(4 * (size_t)(kmax + 8));
  W.rr = c.take<double>(2 * n);
  W.rz = c.take<double>(2 * n);
  W.rp = c.take<double>(2 * n);
  W.rq = c.take<double>(2 * n);
  W.rt = c.take<double>(2 * m);
  W.rs = c.take<double>(16);
  W.pcg = carve_pcg(c, P->Np, P->N, 2, L);
  W.ppart = P->at ? c.take<double>((size_t)rowpass_partials(V) * n) : nullptr;
  W.ppart2 = P->at ? c.take<double>((size_t)rowpass_partials(V) * n) : nullptr;
  W.tu = P->at ? c.take<double>((size_t)m) : nullptr;
  W.gcnt = c.take<int>(64);
  return W;
}

// x = R^{-1} R^{-T} v (FP64 arithmetic on the stored factor)
tls_status solve_normal(const tls_precond_s *P, const double *v, double *x, double *tmp, PcgWs &W,
                        hipStream_t st) {
  TRY(apply_R(P, 1, 1, v, tmp, TLS_FP64, W, st));
  TRY(apply_R(P, 0, 1, tmp, x, TLS_FP64, W, st));
  return TLS_OK;
}

struct WarmScalars {
  double m, n, nA2, bb, atb2, s0, xx, rr, xu, uu, uv, vv;
  double lnd[4];
};

// Relative gap 1 - lam / sigma_0^2 from the secular equation of f = 0, g = 0
// (eq. 2) in its form lam (1 + x_0^T (I - lam M)^{-1} x_0) = ||r_0||^2,
// M = (A^T A)^{-1}, with the quadratic form replaced by its two-point Gauss
// rule from the Lanczos process on M started at x_0 (moments xx, xu, uu, uv).
// Floored at 1e-13 (relative gaps below are rounding).
double gauss_gap(const WarmScalars &w) {
  const double floor_gap = 1e-13;
  if (!(w.xx > 0) || !(w.xu > 0) || !(w.rr > 0)) return floor_gap;
  const double a1 = w.xu / w.xx;
  const double b2 = w.uu / w.xx - a1 * a1;
  double th[2] = {a1, a1}, om[2] = {w.xx, 0.0};
  if (b2 > 1e-12 * a1 * a1) {
    const double a2 = (w.uv - 2.0 * a1 * w.uu + a1 * a1 * w.xu) / (w.xx * b2);
    // eigenpairs of [a1 b; b a2], b = sqrt(b2)
    const double mean = 0.5 * (a1 + a2), half = 0.5 * (a1 - a2);
    const double rad = std::sqrt(half * half + b2);
    th[0] = mean + rad;
    th[1] = mean - rad;
    for (int j = 0; j < 2; ++j) {
      // eigenvector (b, th - a1) normalised; weight xx * (first component)^2
      const double z0 = std::sqrt(b2), z1 = th[j] - a1;
      om[j] = w.xx * z0 * z0 / (z0 * z0 + z1 * z1);
    }
  }
  const double thmax = std::max(th[0], th[1]);
  auto h = [&](double lam) {
    double y = 0.0;
    for (int j = 0; j < 2; ++j) y += om[j] / (1.0 - lam * th[j]);
    return lam * (1.0 + y) - w.rr;
  };
  double lo = 0.0, hi = std::min(w.rr, thmax > 0 ? 1.0 / thmax : w.rr);
  for (int it = 0; it < 200 && hi > lo; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (h(mid) > 0) hi = mid; else lo = mid;
  }
  const double s02 = w.rr / (1.0 + w.xx);
  const double gap = 1.0 - 0.5 * (lo + hi) / s02;
  return std::max(gap, floor_gap);
}

// the 32 warm-start features (definitions in the tls_rqi_solve comment of tls.h)
void warm_features(const WarmScalars &w, float *f) {
  auto L = [](double v) { return std::log(std::max(v, 1e-300)); };
  const double s02 = w.s0 * w.s0;
  const double t = s02 * w.xu / (1.0 + w.xx);
  // Ritz values of (R^T R)^{-1} on span{x_0, u_0}: det(K - th G) = 0 with
  // G = [xx xu; xu uu], K = [xu uu; uu uv]
  const double a2 = w.xx * w.uu - w.xu * w.xu;
  const double a1 = w.xx * w.uv - w.xu * w.uu;
  const double a0 = w.xu * w.uv - w.uu * w.uu;
  double thmax = w.xu / std::max(w.xx, 1e-300), thmin = thmax;
  if (a2 > 1e-12 * w.xx * w.uu) {
    const double disc = std::sqrt(std::max(0.0, a1 * a1 - 4.0 * a2 * a0));
    thmax = (a1 + disc) / (2.0 * a2);
    thmin = (a1 - disc) / (2.0 * a2);
    if (!(thmin > 0)) thmin = std::min(thmax, w.xu / std::max(w.xx, 1e-300));
  }
  double v[TLS_MLP_IN];
  v[0] = L(w.m);
  v[1] = L(w.n);
  v[2] = 0.5 * L(w.nA2);
  v[3] = 0.5 * L(w.bb);
  v[4] = 0.5 * L(w.atb2);
  v[5] = L(w.s0);
  v[6] = 0.5 * L(w.xx);
  v[7] = 0.5 * L(w.rr);
  v[8] = v[7] - v[3];
  v[9] = L(t);
  v[10] = 0.5 * L(w.uu / std::max(w.xx, 1e-300));
  v[11] = -0.5 * L(thmax);
  v[12] = -0.5 * L(thmin);
  v[13] = v[5] - v[11];
  v[14] = s02 * thmax;
  v[15] = t / (1.0 + t);
  for (int i = 0; i < 4; ++i) v[16 + i] = w.lnd[i];
  v[20] = v[4] - v[2] - v[3];
  v[21] = std::log1p(w.xx);
  v[22] = L(w.uv * w.xx / std::max(w.xu * w.uu, 1e-300));
  v[23] = L(w.uu * w.xx / std::max(w.xu * w.xu, 1e-300));
  v[24] = v[2] - 0.5 * v[1] - v[5];
  v[25] = v[3] - 0.5 * v[0];
  v[26] = 0.5 * L(thmax / std::max(thmin, 1e-300));
  v[27] = L(s02 * w.uv / std::max(w.uu, 1e-300));
  v[28] = L(s02 * std::sqrt(w.vv / std::max(w.uu, 1e-300)));
  v[29] = 0.5 * L(s02 * s02 * w.vv / std::max(w.xx, 1e-300));
  v[30] = 1.0;
  v[31] = std::log(gauss_gap(w));
  for (int i = 0; i < TLS_MLP_IN; ++i) f[i] = (float)v[i];
}

}  // namespace

extern "C" {

size_t tls_rqi_workspace_size(const tls_matrix *A, const tls_precond P, const tls_rqi_opts *o) {
  if (check_matrix(A) != TLS_OK || !P || !o) return 0;
  const int kmax = std::max(1, std::min(o->kmax, TLS_MAX_ITERS));
  const int L = std::max({kmax, o->refine_pcg_steps, std::min(std::max(o->min_inner_steps, 0), 4096)}) + 1;
  Carver c(nullptr);
  carve_rqi(c, A->format, A->m, A->n, P, kmax, L);
  return c.size();
}

}  // extern "C"

namespace {

using solve_clock = std::chrono::steady_clock;

// the solve from a given start time (an escalation re-enters with the
// caller's start, so t_ms keeps counting from the original call)
tls_status rqi_solve_from(const tls_matrix *A, const double *b, tls_precond P, const tls_rqi_opts *o,
                          double *x, double *sigma, tls_rqi_stats *stats, void *ws, size_t ws_bytes,
                          hipStream_t st, solve_clock::time_point t0, double t_factor_prior,
                          int accurate_ls) {
  try {
    using clk = solve_clock;
    auto ms_since = [&](clk::time_point a) {
      return std::chrono::duration<double, std::milli>(clk::now() - a).count();
    };
    TRY(check_matrix(A));
    if (!P || !o || !b || !x) return fail(TLS_ERR_ARG, "NULL argument to tls_rqi_solve");
    if (P->n != A->n) return fail(TLS_ERR_ARG, "preconditioner order %lld != n %lld", (long long)P->n, (long long)A->n);
    if (A->format == TLS_CSR && !P->col_ptr) return fail(TLS_ERR_ARG, "CSR A needs a preconditioner built from it (CSC copy)");
    if (A->format == TLS_CSR && (A->row_ptr != P->csr_row_ptr || A->col_idx != P->csr_col_idx ||
                                 A->nnz != P->nnz || A->m != P->m))
      return fail(TLS_ERR_ARG, "CSR A must be the matrix the preconditioner was built from (its "
                  "structure was validated there)");
    if (o->u_p != TLS_FP64 && o->u_p != TLS_FP32) return fail(TLS_ERR_ARG, "u_p must be FP64 or FP32");
    if (o->kmax < 1 || o->kmax > TLS_MAX_ITERS) return fail(TLS_ERR_ARG, "kmax must be in [1, %d]", TLS_MAX_ITERS);
    if (o->stop_patience < 1) return fail(TLS_ERR_ARG, "stop_patience must be >= 1");
    if (!(o->psi_tie >= 1.0) || !std::isfinite(o->psi_tie)) return fail(TLS_ERR_ARG, "psi_tie must be a finite value >= 1");
    if (o->refine_sweeps < 0 || o->refine_sweeps > 4) return fail(TLS_ERR_ARG, "refine_sweeps must be in [0, 4]");
    if (o->refine_sweeps > 0 && o->refine_pcg_steps < 1) return fail(TLS_ERR_ARG, "refine_pcg_steps must be >= 1");
    if (o->mlp_theta && !o->mlp_norm) return fail(TLS_ERR_ARG, "mlp_theta needs mlp_norm");
    if (o->min_inner_steps < 0 || o->min_inner_steps > 4096)
      return fail(TLS_ERR_ARG, "min_inner_steps must be in [0, 4096]");
    if (o->step_margin < 0 || o->step_margin > 4096)
      return fail(TLS_ERR_ARG, "step_margin must be in [0, 4096]");
    if (!ws || ((uintptr_t)ws & 255)) return fail(TLS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    const size_t need = tls_rqi_workspace_size(A, P, o);
    if (ws_bytes < need) return fail(TLS_ERR_WORKSPACE, "RQI workspace %zu < %zu bytes", ws_bytes, need);
    const int kmax = o->kmax;
    const int L = std::max({kmax, o->refine_pcg_steps, o->min_inner_steps}) + 1;
    Carver c(ws);
    RqiWs W = carve_rqi(c, A->format, A->m, A->n, P, kmax, L);
    const int n = (int)A->n;
    const int m = (int)A->m;
    const MatView V = make_view(A, P);
    const int nb_r = matvec_blocks(V), nb_f = V.at ? gradient_rows_blocks(n) : rmatvec_blocks(V);
    tls_rqi_stats local{};
    tls_rqi_stats &S = stats ? *stats : local;
    std::memset(&S, 0, sizeof S);
    S.t_factor_ms = t_factor_prior;

    {
      FillSet F;
      F.add_i32(W.pcg.sync, 0, P->N + 8);
      F.add_i32(W.pcg.cnt, 0, P->N);
      F.add_f64(W.scal, 0.0, 48);
      F.add_i32(W.pcg.done, 0, 1);
      F.add_i32(W.gcnt, 0, 1);
      HIPCHK(launch_fill_multi(F, st));
    }
    // finite b: the flag is read back with sigma_0 below (NaN or Inf on the
    // way produce no fault, only values that are then discarded)
    HIPCHK(launch_check_finite(b, (size_t)A->m, W.pcg.done, st));
    int bad_b = 0;

    // one Rayleigh-quotient evaluation at x (residual pass, scalars, gradient pass, psi)
    // residual partials -> (gradient with the Rayleigh-quotient scalars) ->
    // (psi, the next right-hand sides [-f, x], and x into xbest when psi is
    // the smallest so far): three launches
    double *part_f = W.part + 2 * (size_t)nb_r;
    // one pass over the row-major copy: r = b - A xv (b or xv may be
    // NULL) and A^T r; a step of the factor's certificate rides along when
    // one is due
    auto rowpass = [&](const double *bv, const double *xv, double *r, double *part_r) -> tls_status {
      if (cert_rides(P, V)) return cert_ride_pass(P, V, bv, xv, r, part_r, W.ppart, st);
      HIPCHK(launch_rowpass(V, bv, xv, r, part_r, W.ppart, st));
      return TLS_OK;
    };
    auto evaluate_at = [&](const double *xv, int k, double cap) -> tls_status {
      if (V.at) {   // r and A^T r in one pass over the row-major copy; psi in the gradient's last workgroup
        TRY(rowpass(b, xv, W.r, W.part));
        HIPCHK(launch_gradient_rows_psi(V, W.ppart, xv, W.scal, W.f, part_f, W.part, nb_r, cap, nullptr,
                                        W.gcnt, k, W.rec, W.rhs, W.xbest, o->psi_tie, st));
        return TLS_OK;
      }
      HIPCHK(launch_residual(V, b, xv, W.r, W.part, st));
      HIPCHK(launch_gradient(V, W.r, xv, W.scal, W.f, part_f, W.part, nb_r, cap, st));
      HIPCHK(launch_outer_psi(n, xv, W.f, part_f, nb_f, W.scal, k, W.rec, W.rhs, W.xbest, o->psi_tie, st));
      return TLS_OK;
    };
    // out = A^T (b - A xv) (xv NULL: A^T b), with r = b - A xv and its
    // partials in W.r, W.part when xv is given
    auto atr_pass = [&](const double *xv, double *out) -> tls_status {
      if (V.at) {
        TRY(rowpass(b, xv, xv ? W.r : nullptr, xv ? W.part : nullptr));
        HIPCHK(launch_rowpass_sum(V, W.ppart, 1.0, out, st));
      } else {
        if (xv) {
          HIPCHK(launch_residual(V, b, xv, W.r, W.part, st));
          HIPCHK(launch_rmatvec(V, W.r, out, st));
        } else {
          HIPCHK(launch_rmatvec(V, b, out, st));
        }
      }
      return TLS_OK;
    };
    auto evaluate = [&](int k, double cap) -> tls_status { return evaluate_at(x, k, cap); };
    // Algorithm 2's first step at x_1 = x_0 + sigma_0^2 u_0 from the merged
    // pass at x_0: r_1 = r_0 - sigma_0^2 A u_0 and A^T r_1 = A^T r_0 -
    // sigma_0^2 A^T A u_0 (the same quantities, formed from products of A
    // already taken), then the gradient and psi as in evaluate_at
    auto evaluate_merged = [&](double cap) -> tls_status {
      HIPCHK(launch_shift_residual(m, b, W.r, W.tu, W.scal, W.part, st));
      HIPCHK(launch_gradient_rows_psi(V, W.ppart, x, W.scal, W.f, part_f, W.part, nb_r, cap, W.ppart2, W.gcnt,
                                      1, W.rec, W.rhs, W.xbest, o->psi_tie, st));
      return TLS_OK;
    };

    // ---- lines 1-5: x_0 = x_LS, sigma_0, u_0, x_1; the b-dependent gate ---
    // dense A with the row copy and the plain start: the pass at x_0 also
    // takes u_0, so that the first step needs no pass of its own
    const bool merged = V.at != nullptr && !o->mlp_theta && !(o->sigma0_hint > 0);
    double rr0 = 0.0;
    bool spec = false, ls_deferred = false;
    for (;;) {
      TRY(atr_pass(nullptr, W.t1));                                 // A^T b
      if (o->mlp_theta || o->sigma0_hint > 0 || o->features) {
        DotPairs D{};
        D.a[0] = D.b[0] = b; D.len[0] = m;
        D.a[1] = D.b[1] = W.t1; D.len[1] = n;
        HIPCHK(launch_dots(D, 2, W.scal + 24, st));                  // ||b||^2, ||A^T b||^2
      }
      TRY(solve_normal(P, W.t1, x, W.t2, W.pcg, st));               // x = R^{-1} R^{-T} A^T b
      for (int c2 = 0; c2 < o->ls_corrections; ++c2) {               // corrected semi-normal equations
        TRY(atr_pass(x, W.t1));
        TRY(solve_normal(P, W.t1, W.rhs, W.t2, W.pcg, st));
        HIPCHK(launch_add_f64(x, W.rhs, (size_t)n, st));
      }
      if (accurate_ls) {
        // more corrections until the last one is below 1e-8 ||x|| (the
        // error contracts by about max |1 - theta| over the factor's
        // certificate per correction)
        S.ls_refined = 1;
        for (int c2 = 0; c2 < 64; ++c2) {
          TRY(atr_pass(x, W.t1));
          TRY(solve_normal(P, W.t1, W.rhs, W.t2, W.pcg, st));
          HIPCHK(launch_add_f64(x, W.rhs, (size_t)n, st));
          DotPairs D{};
          D.a[0] = D.b[0] = W.rhs; D.len[0] = n;
          D.a[1] = D.b[1] = x; D.len[1] = n;
          HIPCHK(launch_dots(D, 2, W.scal + 40, st));
          double dd[2];
          HIPCHK(hipMemcpyAsync(dd, W.scal + 40, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          ++S.ls_refined;
          if (!(dd[0] > 1e-16 * dd[1])) break;
        }
      }
      if (merged) {
        // u_0 first, then one pass for r_0 = b - A x_0, A^T r_0, A u_0 and
        // A^T A u_0: r_1 and A^T r_1 at x_1 = x_0 + sigma_0^2 u_0 follow
        // from them without a pass of their own (evaluate_merged)
        TRY(solve_normal(P, x, W.t1, W.t2, W.pcg, st));             // A^T A u_0 = x_0
        HIPCHK(launch_rowpass_dual(V, b, x, W.r, W.part, W.ppart, W.t1, W.ppart2, st, W.tu));
      } else if (V.at) {
        TRY(rowpass(b, x, W.r, W.part));   // r_0
      } else {
        HIPCHK(launch_residual(V, b, x, W.r, W.part, st));
      }
      HIPCHK(launch_outer_rq(n, x, W.part, nb_r, W.scal, 0.0, st));  // sigma_0^2
      // nothing before the first psi read-back needs sigma_0 on the host
      // unless a warm start, the shift clamp or a waiting gate does: then
      // sigma_0 and the finite-b flag come back with that read-back (the
      // scalars saved at scal[48..52]) instead of in a synchronization of
      // their own
      const bool gated = o->gate_enforce && P->storage != TLS_FP64;
      ls_deferred = !o->mlp_theta && !(o->sigma0_hint > 0) && !o->features && !o->shift_clamp &&
                    !accurate_ls && (!gated || P->gate_pending);
      if (ls_deferred) {
        HIPCHK(launch_copy_f64(W.scal + 48, W.scal, 5, st));
        spec = gated;
        break;
      }
      double h2[5];
      HIPCHK(hipMemcpyAsync(h2, W.scal, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(&bad_b, W.pcg.done, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (bad_b) return fail(TLS_ERR_NONFINITE, "b contains NaN or Inf");
      S.sigma_ls = std::sqrt(h2[0]);
      rr0 = h2[3];
      if (!gated) break;
      // constraint (6) with sigma_{n+1} <= sigma_0 and the Lanczos estimates,
      // and the a-posteriori certificate of the factor itself (the estimates
      // come from the factor and cannot reveal that it is poor)
      if (!P->gate_pending && !P->have_quality) {
        FactorWs FW = factor_ws_of(P);
        TRY(gate_start(P, FW, V, st));
      }
      // runs still in flight: iterate speculatively and decide at a later
      // host synchronisation (the shift clamp needs the estimates first)
      spec = P->gate_pending && !o->shift_clamp;
      if (!spec) {
        TRY(gate_finish(P));
        gate_decide(P, S.sigma_ls);
        S.t_verdict_ms = ms_since(t0);
      }
      break;
    }
    const bool gate_failed = !spec && o->gate_enforce && P->storage != TLS_FP64 &&
                             !(P->rep.verdict & 16);
    auto escalate = [&]() -> tls_status {
      tls_gate_report &R = P->rep;
      if (!o->allow_escalate)
        return fail(TLS_ERR_PRECISION, "the u_q = %g factor fails the a-posteriori certificate "
                    "(Ritz values of R^-T A^T A R^-1 in [%.3g, %.3g]; (6) bound %.3g)", R.u_q,
                    R.quality_lo, R.quality_hi, R.bound6);
      const auto tf = clk::now();
      const int next = (P->uq == TLS_BF16) ? TLS_FP16
                       : (P->uq == TLS_FP16 || P->uq == TLS_BF16X3) ? TLS_FP32 : TLS_FP64;
      FactorWs FW = factor_ws_of(P);
      int bd = 0;
      TRY(gate_finish(P));   // its runs read the factor that is replaced now
      TRY(factor_once(A, P, FW, next, st, &bd, next != TLS_FP64 ? &V : nullptr));
      if (next == TLS_FP64) P->have_kappa = P->have_sigma_n = P->have_quality = 0;
      R.escalations++;
      R.used = P->uq;
      S.t_factor_ms += ms_since(tf);
      return TLS_OK;
    };
    auto resolve = [&]() -> tls_status {
      TRY(escalate());
      return rqi_solve_from(A, b, P, o, x, sigma, stats, ws, ws_bytes, st, t0, S.t_factor_ms, 0);
    };
    // the start violates the positive-definiteness assumption (sigma_0 at or
    // above the estimate of sigma'_n, c~ <= 0 in (6)) with a low-precision
    // factor: x_LS may be short of convergence (a weak factor); a second
    // solve recomputes it to convergence on the same factor (once)
    auto start_suspect = [&]() {
      return !accurate_ls && P->storage != TLS_FP64 && std::isfinite(P->rep.ctilde_min) &&
             P->rep.ctilde_min <= 0.0;
    };
    auto restart_ls = [&]() -> tls_status {
      return rqi_solve_from(A, b, P, o, x, sigma, stats, ws, ws_bytes, st, t0, S.t_factor_ms, 1);
    };
    if (gate_failed) return resolve();
    // shift cap for the clamp (a deviation for starts above sigma'_n)
    double cap = 0.0;
    if (o->shift_clamp && !P->have_sigma_n) {
      TRY(gate_finish(P));
      if (!P->have_sigma_n) {
        FactorWs FW = factor_ws_of(P);
        TRY(estimate_sigma_n(P, FW, st));
      }
    }
    if (o->shift_clamp && std::isfinite(P->rep.sigma_n_est) && P->rep.sigma_n_est > 0)
      cap = o->shift_clamp_tau * P->rep.sigma_n_est * P->rep.sigma_n_est;

    S.gate_async = spec ? 1 : 0;
    // everything from here on uses the factor; under speculation the gate's
    // verdict is read when its runs are done (polled at each psi read-back,
    // awaited at the end) and a failed certificate discards the result
    auto body = [&]() -> tls_status {
      if (!merged) TRY(solve_normal(P, x, W.t1, W.t2, W.pcg, st));  // A^T A u_0 = x_0
      const bool warm = o->mlp_theta != nullptr || o->sigma0_hint > 0;
      bool plain_step = true;
      if (warm || o->features) {
        // u_1 = (R^T R)^{-1} u_0 and the dot products of the features
        double *u1 = W.rp, *xw = W.rq;
        TRY(solve_normal(P, W.t1, u1, W.t2, W.pcg, st));
        DotPairs D{};
        const double *pa[5] = {x, x, W.t1, W.t1, u1}, *pb[5] = {x, W.t1, W.t1, u1, u1};
        for (int i = 0; i < 5; ++i) { D.a[i] = pa[i]; D.b[i] = pb[i]; D.len[i] = n; }
        HIPCHK(launch_dots(D, 5, W.scal + 26, st));
        double hd[7];
        HIPCHK(hipMemcpyAsync(hd, W.scal + 24, 7 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        WarmScalars ws_{};
        ws_.m = (double)m; ws_.n = (double)n; ws_.nA2 = P->normA_F2; ws_.bb = hd[0]; ws_.atb2 = hd[1];
        ws_.s0 = S.sigma_ls; ws_.xx = hd[2]; ws_.xu = hd[3]; ws_.uu = hd[4]; ws_.uv = hd[5];
        ws_.vv = hd[6]; ws_.rr = rr0;
        for (int i = 0; i < 4; ++i) ws_.lnd[i] = P->lnd[i];
        warm_features(ws_, S.features);
        double sig_hat = -1.0;
        if (o->mlp_theta) {
          HIPCHK(hipMemcpyAsync(W.rs, S.features, TLS_MLP_IN * sizeof(float), hipMemcpyHostToDevice, st));
          HIPCHK(launch_mlp_infer1(o->mlp_theta, o->mlp_norm, (const float *)W.rs, W.scal + 22, st));
          double yh = 0.0;
          HIPCHK(hipMemcpyAsync(&yh, W.scal + 22, sizeof(double), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          // y = ln(1 - sigma^2 / sigma_0^2) = two-point Gauss estimate + learned correction
          const double y = (double)S.features[31] + yh;
          if (std::isfinite(y)) sig_hat = S.sigma_ls * std::sqrt(std::max(0.0, -std::expm1(std::min(y, 0.0))));
        } else if (o->sigma0_hint > 0) {
          sig_hat = o->sigma0_hint;
        }
        if (warm && sig_hat >= 0.0) {
          sig_hat = std::min(sig_hat, S.sigma_ls);
          if (cap > 0) sig_hat = std::min(sig_hat, std::sqrt(cap));
          const double lam = sig_hat * sig_hat;
          HIPCHK(launch_axpy2(n, x, W.t1, u1, lam, lam * lam, xw, st));      // warm candidate
          HIPCHK(launch_axpy_init(n, x, W.t1, W.scal, 0, st));              // plain x_1
          plain_step = false;
          double pw = 0.0, pp = 0.0;
          TRY(evaluate_at(xw, 1, cap));
          HIPCHK(hipMemcpyAsync(&pw, W.scal + 7, sizeof(double), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          TRY(evaluate_at(x, 1, cap));
          HIPCHK(hipMemcpyAsync(&pp, W.scal + 7, sizeof(double), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          S.sigma_hat = sig_hat;
          S.psi_warm = pw;
          S.psi_plain = pp;
          if (pw < pp) {
            HIPCHK(launch_copy_f64(x, xw, (size_t)n, st));
            S.warm_used = 1;
          }
        }
      }
      if (plain_step) HIPCHK(launch_axpy_init(n, x, W.t1, W.scal, 0, st));   // x_1 = x_0 + sigma_0^2 u_0

      // ---- main loop -----------------------------------------------------------
      // Lookahead: iteration k's two PCGTLS solves and its update are
      // enqueued before the host waits for psi_k (read back into pinned
      // memory behind an event), so the GPU works through the host's
      // turnaround. They never touch the best iterate, which only the psi
      // kernel writes, and x is reset to it after the loop, so a stop at k
      // leaves the result unchanged. Off with strict_pd: a run past the stop
      // must not turn delta_j <= 0 into an error of a finished solve.
      PinnedBlock hb;
      HIPCHK(pinned_take(&hb.p, &hb.dev));
      CopyEvent hev;
      HIPCHK(hipEventCreateWithFlags(&hev.e, hipEventDisableTiming));
      double *const h = hb.p;                                  // 64 scalars
      int *const bad_h = reinterpret_cast<int *>(hb.p + 64);   // finite-b flag
      const bool ahead = !o->strict_pd;
      // two PCGTLS solves with l = k (at most k+1 steps; at least
      // min_inner_steps when asked), sharing the shift; the right-hand sides
      // [-f, x] were written by the psi kernel; then the RQI update of x,
      // which also records the steps the runs executed (scalar S_STEPS)
      auto inner = [&](int steps) -> tls_status {
        TRY(pcg_run(P, W.scal + 1, 2, W.rhs, nullptr, steps - 1, o->u_p, o->strict_pd, W.pcg, st));
        HIPCHK(launch_rqi_update_pcg(n, x, o->u_p, W.pcg.w, P->Np, W.f, W.scal, W.pcg.done, steps, st));
        return TLS_OK;
      };
      // Steps launched per run. A run that ends at its exits (Algorithm 3:
      // eta = 0, the precision floor, delta = 0) leaves the steps after its
      // last one with nothing to do, but each still costs a launch that
      // reads the done flags. Once the host has read that a run ended after
      // e of the steps it was given, later runs are given e + step_margin
      // (never more than k + 1): a run that ends within them is unchanged,
      // and one that does not stops after them, which Algorithm 2's bound of
      // at most k + 1 steps allows; a run that used every step it was given
      // lifts the cap again.
      std::vector<int> launched((size_t)kmax + 2, 0);
      int step_cap = std::numeric_limits<int>::max();
      double best = std::numeric_limits<double>::infinity();
      int no_improve = 0, k = 0;
      S.stopped = 1;
      for (k = 1; k <= kmax; ++k) {
        if (k == 1 && merged) TRY(evaluate_merged(cap));
        else TRY(evaluate(k, cap));
        if (o->x_snapshots) HIPCHK(launch_copy_f64(o->x_snapshots + (size_t)(k - 1) * n, x, (size_t)n, st));
        const bool first = ls_deferred && k == 1;
        HIPCHK(hipMemcpyAsync(h, W.scal, (first ? 64 : 17) * sizeof(double), hipMemcpyDeviceToHost, st));
        if (first) HIPCHK(hipMemcpyAsync(bad_h, W.pcg.done, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(hev.e, st));
        const int l = std::max(k, o->min_inner_steps);
        const bool enq = ahead && k < kmax;
        auto steps_k = [&]() {
          return (int)std::min<long long>((long long)l + 1, step_cap);
        };
        int steps = 0;
        if (enq) TRY(inner(steps = steps_k()));
        HIPCHK(hipEventSynchronize(hev.e));
        if (k >= 2 && launched[k - 1] > 0 && o->step_margin > 0) {
          // the runs of iteration k - 1 finished before psi_k was formed
          const int used = (int)h[16];
          step_cap = used < launched[k - 1] ? used + o->step_margin : std::numeric_limits<int>::max();
        }
        if (first) {
          bad_b = *bad_h;
          if (bad_b) return fail(TLS_ERR_NONFINITE, "b contains NaN or Inf");
          S.sigma_ls = std::sqrt(h[48]);
          rr0 = h[51];
        }
        const double psi = h[7], sig2 = h[0];
        S.iters = k;
        S.psi[k - 1] = psi;
        S.sigma[k - 1] = std::sqrt(sig2);
        S.t_ms[k - 1] = ms_since(t0);
        // the verdict is read as soon as its runs are done; once a dense A's
        // certificate has taken its last pass, the host waits for that
        // step's remaining work on side2 here (the GPU meanwhile runs the
        // PCGTLS solves already enqueued) instead of polling again an
        // iteration later
        const bool cert_enqueued = V.at && V.at == P->at && !P->cert_todo;
        if (spec && P->gate_pending && (cert_enqueued || gate_ready(P))) {
          TRY(gate_finish(P));
          gate_decide(P, S.sigma_ls);
          S.t_verdict_ms = ms_since(t0);
          if (!(P->rep.verdict & 16)) return TLS_OK;   // discarded below: escalation
        }
        if (h[1] != h[0]) S.clamped++;
        if (!std::isfinite(psi)) return fail(TLS_ERR_NO_CONVERGENCE, "psi became non-finite at k = %d", k);
        // the psi kernel has copied x to xbest when psi is within psi_tie of
        // the smallest psi before it (best): the latest such iterate is returned
        if (k == 1 || psi <= o->psi_tie * best) S.k_best = k;
        if (psi < best) {
          best = psi;
          no_improve = 0;
        } else if (o->stop_ge ? (psi >= best) : (psi > best)) {
          ++no_improve;
        }
        // psi == 0, or exactly the previous psi: the iterate no longer moves
        if (psi == 0.0 || (k > 1 && psi == S.psi[k - 2])) { S.stopped = 2; break; }
        if (no_improve >= o->stop_patience) { S.stopped = 0; break; }
        if (k == kmax) break;
        if (!enq) TRY(inner(steps = steps_k()));
        launched[k] = steps;
        S.pcg_steps += steps;
      }
      // the returned iterate needs the gate's verdict: wait for runs still
      // in flight now rather than after the refinement
      if (spec && P->gate_pending) {
        TRY(gate_finish(P));
        gate_decide(P, S.sigma_ls);
        S.t_verdict_ms = ms_since(t0);
        if (!(P->rep.verdict & 16)) return TLS_OK;     // discarded below: escalation
      }
      HIPCHK(launch_copy_f64(x, W.xbest, (size_t)n, st));

      // ---- final FP64 refinement: RQI steps with explicit-operator PCG --------
      // (skipped when psi already sits at the float64 rounding floor u ||A||_F^2)
      const bool at_floor = P->normA_F2 > 0 && best <= 32.0 * unit_roundoff(TLS_FP64) * P->normA_F2;
      for (int sw = 0; sw < (at_floor ? 0 : o->refine_sweeps); ++sw) {
        TRY(evaluate(kmax + 1 + sw, cap));                   // f, g and the (clamped) shift at x
        {
          // a Newton step is only meaningful at the Rayleigh-quotient shift: if the
          // clamp is active the iterate is not yet near sigma_{n+1}; stop refining
          double hs[2];
          HIPCHK(hipMemcpyAsync(hs, W.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          if (hs[1] != hs[0]) break;
        }
        HIPCHK(launch_make_rhs(n, W.f, x, W.rr, st));          // r = [-f, x], omega = u = 0
        HIPCHK(launch_fill_f64(W.wu, 0.0, 2 * (size_t)n, st));
        // z = M r with M = (R^T R)^{-1} applied in FP64 arithmetic to the stored
        // factor: a fixed symmetric preconditioner, so CG reaches FP64 accuracy
        TRY(apply_R(P, 1, 2, W.rr, W.rq, TLS_FP64, W.pcg, st));
        TRY(apply_R(P, 0, 2, W.rq, W.rz, TLS_FP64, W.pcg, st));
        HIPCHK(launch_ref_step2(n, 2, W.rr, W.rz, W.rp, W.rs, 1, st));
        double rz0[8];
        HIPCHK(hipMemcpyAsync(rz0, W.rs, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int j = 0; j < o->refine_pcg_steps; ++j) {
          if (j > 0 && j % 8 == 0) {
            // stop when both preconditioned residuals r^T M r fell by 1e-26
            double rzj[8];
            HIPCHK(hipMemcpyAsync(rzj, W.rs, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (rzj[0] <= 1e-26 * rz0[0] && rzj[4] <= 1e-26 * rz0[4]) break;
          }
          for (int q = 0; q < 2; ++q) {                         // K p = A^T (A p) - mu p
            if (V.at) {                                         // A^T A p in one pass
              HIPCHK(launch_rowpass(V, nullptr, W.rp + (size_t)q * n, nullptr, nullptr, W.ppart, st));
              HIPCHK(launch_rowpass_sum(V, W.ppart, -1.0, W.rq + (size_t)q * n, st));
            } else {
              HIPCHK(launch_matvec(V, W.rp + (size_t)q * n, W.rt + (size_t)q * m, st));
              HIPCHK(launch_rmatvec(V, W.rt + (size_t)q * m, W.rq + (size_t)q * n, st));
            }
          }
          HIPCHK(launch_ref_step1(n, 2, W.scal, W.wu, W.rr, W.rp, W.rq, W.rs, st));
          TRY(apply_R(P, 1, 2, W.rr, W.rq, TLS_FP64, W.pcg, st));
          TRY(apply_R(P, 0, 2, W.rq, W.rz, TLS_FP64, W.pcg, st));
          HIPCHK(launch_ref_step2(n, 2, W.rr, W.rz, W.rp, W.rs, 0, st));
        }
        HIPCHK(launch_rqi_update(n, x, W.wu, W.f, W.scal, nullptr, nullptr, nullptr, 0, st));
        S.refine_steps++;
        // keep the refined iterate under the same rule as the loop's (the psi
        // kernel has already copied it to xbest when it qualifies)
        TRY(evaluate(kmax + 1 + sw, cap));
        HIPCHK(hipMemcpyAsync(h, W.scal, 16 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (h[7] <= o->psi_tie * best) {
          best = std::min(best, h[7]);
        } else {
          HIPCHK(launch_copy_f64(x, W.xbest, (size_t)n, st));
          break;
        }
      }
      // final sigma from a compensated residual at x
      HIPCHK(launch_residual_dd(V, b, x, W.part, st));
      HIPCHK(launch_sigma_dd(n, x, W.part, nb_r, W.scal + 20, st));
      double sg[2];
      HIPCHK(hipMemcpyAsync(sg, W.scal + 20, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      TRY(sync_status(W.pcg.sync, P->N, st));
      {
        // PCGTLS steps that met delta_j < 0 (the last run's flags)
        std::vector<int> neg((size_t)(W.pcg.L + 2) * 2);
        HIPCHK(hipMemcpyAsync(neg.data(), W.pcg.neg, neg.size() * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int v : neg) S.negative_delta += v;
      }
      S.sigma_final = sg[1];
      if (sigma) *sigma = sg[1];
      S.t_total_ms = ms_since(t0);
      if (S.stopped == 1)
        return fail(TLS_ERR_NO_CONVERGENCE, "kmax = %d reached before the psi rule fired", kmax);
      return TLS_OK;
    };
    // a solve on a low-precision factor that ends without convergence (kmax
    // before the psi rule) under the gate: the factor could not separate
    // sigma_{n+1} from its neighbours (the operator R^T R - sigma^2 I is off
    // by about u_q in every direction, more than a narrow gap), so with
    // allow_escalate the next precision solves again
    auto settle = [&](tls_status s) -> tls_status {
      if (s == TLS_ERR_NO_CONVERGENCE && o->gate_enforce && o->allow_escalate && P->storage != TLS_FP64)
        return resolve();
      return s;
    };
    const tls_status bs = body();
    if (spec) {
      if (P->gate_pending) {
        TRY(gate_finish(P));
        gate_decide(P, S.sigma_ls);
        S.t_verdict_ms = ms_since(t0);
      }
      if (!(P->rep.verdict & 16)) return resolve();
    }
    if (o->gate_enforce && start_suspect() && (bs == TLS_OK || bs == TLS_ERR_NO_CONVERGENCE)) {
      // second solve from the converged x_LS; any Rayleigh quotient bounds
      // sigma_{n+1} from above, so the smaller converged sigma is kept
      std::vector<double> x_first((size_t)n);
      HIPCHK(hipMemcpyAsync(x_first.data(), x, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      const tls_rqi_stats S_first = S;
      const tls_status b1 = restart_ls();
      if (b1 != TLS_OK && b1 != TLS_ERR_NO_CONVERGENCE) return b1;
      if (!(S.sigma_final < S_first.sigma_final)) {
        const int refined = S.ls_refined;
        HIPCHK(hipMemcpyAsync(x, x_first.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        S = S_first;
        S.ls_refined = -refined;
        if (sigma) *sigma = S.sigma_final;
        return settle(bs);
      }
      return settle(b1);
    }
    return settle(bs);
  } catch (...) {
    return fail(TLS_ERR_ARG, "unexpected C++ exception");
  }
}

}  // namespace

extern "C" {

tls_status tls_rqi_solve(const tls_matrix *A, const double *b, tls_precond P, const tls_rqi_opts *o,
                         double *x, double *sigma, tls_rqi_stats *stats, void *ws, size_t ws_bytes,
                         hipStream_t st) {
  return rqi_solve_from(A, b, P, o, x, sigma, stats, ws, ws_bytes, st, solve_clock::now(), 0.0, 0);
}

}  // extern "C"

// ===========================================================================
// warm-start network
// ===========================================================================
namespace {

MlpBufs carve_mlp(Carver &c, int64_t B, float **y) {
  MlpBufs M{};
  M.h0 = c.take<float>((size_t)B * TLS_MLP_IN);
  for (int i = 0; i < 3; ++i) {
    M.z[i] = c.take<float>((size_t)B * TLS_MLP_WIDTH);
    M.h[i] = c.take<float>((size_t)B * TLS_MLP_WIDTH);
  }
  for (int i = 0; i < 2; ++i) M.dz[i] = c.take<float>((size_t)B * TLS_MLP_WIDTH);
  M.dy = c.take<float>((size_t)B);
  *y = c.take<float>((size_t)B);
  return M;
}

tls_status check_mlp_ws(int64_t batch, void *ws, size_t ws_bytes) {
  if (batch < 1 || batch > (int64_t)1 << 24) return fail(TLS_ERR_ARG, "batch must be in [1, 2^24]");
  if (!ws || ((uintptr_t)ws & 255)) return fail(TLS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  const size_t need = tls_mlp_workspace_size(batch);
  if (ws_bytes < need) return fail(TLS_ERR_WORKSPACE, "MLP workspace %zu < %zu bytes", ws_bytes, need);
  return TLS_OK;
}

}  // namespace

extern "C" {

size_t tls_mlp_workspace_size(int64_t batch) {
  if (batch < 1) return 0;
  Carver c(nullptr);
  float *y = nullptr;
  carve_mlp(c, batch, &y);
  return c.size();
}

tls_status tls_mlp_forward(const float *theta, const float *norm, const float *X, int64_t batch,
                           float *y, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!theta || !norm || !X || !y) return fail(TLS_ERR_ARG, "NULL argument to tls_mlp_forward");
  TRY(check_mlp_ws(batch, ws, ws_bytes));
  Carver c(ws);
  float *yw = nullptr;
  MlpBufs M = carve_mlp(c, batch, &yw);
  HIPCHK(launch_mlp_forward(theta, norm, X, batch, y, M, stream));
  return TLS_OK;
}

tls_status tls_mlp_loss_grad(const float *theta, const float *norm, const float *X, const float *t,
                             int64_t batch, float *grad, float *loss, void *ws, size_t ws_bytes,
                             hipStream_t stream) {
  if (!theta || !norm || !X || !t || !grad || !loss)
    return fail(TLS_ERR_ARG, "NULL argument to tls_mlp_loss_grad");
  TRY(check_mlp_ws(batch, ws, ws_bytes));
  Carver c(ws);
  float *y = nullptr;
  MlpBufs M = carve_mlp(c, batch, &y);
  HIPCHK(launch_mlp_forward(theta, norm, X, batch, y, M, stream));
  HIPCHK(launch_mlp_backward(theta, y, t, batch, grad, loss, M, stream));
  return TLS_OK;
}

tls_status tls_mlp_adam(float *theta, float *m, float *v, const float *grad, int64_t count,
                        int64_t step, float lr, float beta1, float beta2, float eps,
                        hipStream_t stream) {
  if (!theta || !m || !v || !grad || count < 1) return fail(TLS_ERR_ARG, "bad arguments to tls_mlp_adam");
  if (step < 1) return fail(TLS_ERR_ARG, "Adam step numbers start at 1");
  if (!(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 && lr > 0))
    return fail(TLS_ERR_ARG, "Adam needs 0 <= beta < 1, eps > 0, lr > 0");
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)step));
  const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)step));
  HIPCHK(launch_mlp_adam(count, theta, m, v, grad, lr, beta1, beta2, eps, (float)c1, (float)c2, stream));
  return TLS_OK;
}

}  // extern "C"
