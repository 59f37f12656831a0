// Blocked triangular solves with the preconditioner R = R_hat D and the
// PCGTLS iteration (Algorithm 3) built on them.
//
// Storage: R_hat (upper triangular, order Np = N*64, zero padded with an
// identity diagonal beyond n) is kept as 64x64 tiles (I, J), I <= J, packed
// by block column (tile index J(J+1)/2 + I), column-major inside a tile, in
// the storage precision S. The inverses of the diagonal tiles are kept in
// the compute precision C. D^{-1} is a length-Np vector.
//
// One launch solves one triangular system for NR (1 or 2) right-hand sides.
// Each workgroup owns one block row; workgroups take block rows in
// dependency order from a ticket counter, so a workgroup only waits on
// blocks owned by workgroups that started before it (no deadlock for any
// grid). A finished block is published through a per-block flag with
// release/acquire ordering at agent scope. Each wave accumulates its
// 16-column slice of every off-diagonal tile as soon as the block it needs
// is published, without workgroup barriers; the diagonal block is applied
// as a small GEMV with the stored inverse. The last workgroup to finish
// resets the flags and counters for the next launch.
//
// The PCGTLS modes fuse the vector work of Algorithm 3 into the two solves
// of each step: the backward solve q = R^{-1} p carries the p update and
// the partial sums of ||p||^2 and ||q||^2; the forward solve R^{-T} q
// carries delta, alpha, the omega update, the s update and ||s||^2. All
// scalars are recomputed by every workgroup from the per-block partial
// sums of the previous launch in a fixed order, so no workgroup reads a
// value another workgroup of the same launch writes.
#include "common.h"
#include "kernels.h"

namespace tls {

enum TrsvMode { APPLY_B = 0, APPLY_F = 1, PCG_F0 = 2, PCG_B = 3, PCG_F = 4 };

// sync area layout (ints): flags[0..N), ticket, done counter, abort, status
struct SyncIdx {
  int N;
  __device__ int ticket() const { return N; }
  __device__ int done() const { return N + 1; }
  __device__ int abort() const { return N + 2; }
  __device__ int status() const { return N + 3; }
};

template <typename S, typename C>
struct TrsvParams {
  const S *tiles;
  const C *dinv;       // N x 64 x 64 inverse diagonal tiles (column-major)
  const C *dscale;     // Np, 1/d (ones when unscaled)
  int N, Np, n;
  int *sync;
  C *chain;            // [NR][Np] published block solutions
  // apply modes
  const double *in;    // [NR][ldi]
  double *out;         // [NR][ldo]
  int ldi, ldo;
  // PCG modes
  C *s, *p, *q, *w;    // [NR][Np]
  C *part;             // [(L+2)][3][NR][N]: ss, pp, qq
  int *done;           // [(L+2)][NR]: done after step j
  int *neg;            // [(L+2)][NR]
  double *trace;       // [NR][4][L+2]: eta, delta, alpha, beta
  const double *sigma2;
  int j, L, strict;
};

template <typename C>
__device__ inline C *part_ptr(C *part, int j, int kind, int r, int NR, int N) {
  return part + (((size_t)j * 3 + kind) * NR + r) * N;
}

// fixed-order sum of N per-block partials, evaluated by one wave
template <typename C>
__device__ inline C sum_parts(const C *p, int N) {
  const int lane = threadIdx.x & 63;
  C v = 0;
  for (int i = lane; i < N; i += 64) v += p[i];
  return wave_sum(v);
}

template <typename S, typename C, int NR, int MODE>
__global__ __launch_bounds__(WG) void k_trsv(TrsvParams<S, C> P) {
  constexpr bool BWD = (MODE == APPLY_B || MODE == PCG_B);
  __shared__ int s_blk, s_skip, s_abort;
  __shared__ C s_part[4][NR][NB];
  __shared__ C s_rhs[NR][NB];
  __shared__ C s_scal[NR][4];
  // s_live: step j-1 ran for this right-hand side; s_run: step j runs
  // (eta_j != 0 and, forward, delta_j and alpha_j finite and delta_j != 0)
  __shared__ int s_live[NR], s_run[NR], s_floor[NR];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int N = P.N, Np = P.Np;
  const SyncIdx SI{N};
  int *sync = P.sync;

  if (tid == 0) {
    const int t = atomicAdd(&sync[SI.ticket()], 1);
    s_blk = BWD ? (N - 1 - t) : t;
    s_abort = flag_load_relaxed(&sync[SI.abort()]);
    int skip = s_abort;
    if constexpr (MODE == PCG_B || MODE == PCG_F) {
      int all_done = 1;
      for (int r = 0; r < NR; ++r) {
        const int d = (P.j > 0) ? P.done[(P.j - 1) * NR + r] : 0;
        s_live[r] = !d;
        all_done &= d;
      }
      skip |= all_done;
      // a skipped forward step still carries the done flags to step j
      if constexpr (MODE == PCG_F) {
        if (all_done && t == 0)
          for (int r = 0; r < NR; ++r) P.done[P.j * NR + r] = 1;
      }
    } else {
      for (int r = 0; r < NR; ++r) s_live[r] = 1;
    }
    s_skip = skip;
  }
  __syncthreads();
  const int I = s_blk;

  if (!s_skip) {
    // ---- step-level scalars (identical in every workgroup) --------------
    if constexpr (MODE == PCG_B || MODE == PCG_F) {
      if (w == 0) {
        // eta_j = 0, or eta_j <= u_p^2 eta_0 for j > 0, ends the loop before
        // step j (at eta_j = 0 beta_j would be 0/0); a step whose delta_j or
        // alpha_j is zero or not finite does not run
        for (int r = 0; r < NR; ++r) {
          const C eta = sum_parts(part_ptr(P.part, P.j, 0, r, NR, N), N);
          const C eta0 = (P.j > 0) ? sum_parts(part_ptr(P.part, 0, 0, r, NR, N), N) : eta;
          const bool at_floor = P.j > 0 && eta <= pcg_eta_floor<C>() * eta0;
          if constexpr (MODE == PCG_B) {
            C beta = 0;
            if (P.j > 0) {
              const C eta_prev = sum_parts(part_ptr(P.part, P.j - 1, 0, r, NR, N), N);
              if (eta_prev != (C)0) beta = eta / eta_prev;
            }
            if (lane == 0) {
              s_scal[r][0] = eta; s_scal[r][1] = beta;
              s_run[r] = (eta != (C)0) && !at_floor;
              s_floor[r] = at_floor;
            }
          } else {
            const C pp = sum_parts(part_ptr(P.part, P.j, 1, r, NR, N), N);
            const C qq = sum_parts(part_ptr(P.part, P.j, 2, r, NR, N), N);
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
      __syncthreads();
    }

    // ---- off-diagonal tiles: each wave owns 16 columns (BWD) / rows (FWD)
    C acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0;
    bool aborted = false;
    const int K0 = BWD ? N - 1 : 0;
    const int K1 = BWD ? I : I;       // exclusive bound
    for (int K = K0; BWD ? (K > K1) : (K < K1); K += BWD ? -1 : 1) {
      // tile (I, K) for the backward solve, (K, I) for the forward one
      const size_t tidx = BWD ? ((size_t)K * (K + 1) / 2 + I) : ((size_t)I * (I + 1) / 2 + K);
      const S *T = P.tiles + tidx * (NB * NB);
      C tv[16];
      if (BWD) {
#pragma unroll
        for (int c = 0; c < 16; ++c) tv[c] = cvt<C>(T[(16 * w + c) * NB + lane]);
      } else {
#pragma unroll
        for (int c = 0; c < 16; ++c) tv[c] = cvt<C>(T[lane * NB + 16 * w + c]);
      }
      int spins = 0;
      while (flag_load_acquire(&sync[K]) == 0) {
        if (flag_load_relaxed(&sync[SI.abort()])) { aborted = true; break; }
        if (++spins > SPIN_LIMIT) {
          __hip_atomic_store(&sync[SI.abort()], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&sync[SI.status()], (int)TLS_ERR_SYNC_TIMEOUT, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          aborted = true;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (aborted) break;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const C *xk = P.chain + (size_t)r * Np + (size_t)K * NB + 16 * w;
        C a = acc[r];
#pragma unroll
        for (int c = 0; c < 16; ++c) a += tv[c] * xk[c];
        acc[r] = a;
      }
    }
    if (aborted) s_abort = 1;
#pragma unroll
    for (int r = 0; r < NR; ++r) s_part[w][r][lane] = acc[r];
    __syncthreads();

    if (!s_abort) {
      // ---- right-hand side of the diagonal block (prologue) ---------------
      if (w == 0) {
        const int row = I * NB + lane;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          C y = 0;
          const size_t vi = (size_t)r * Np + row;
          if constexpr (MODE == APPLY_B) {
            y = (row < P.n) ? (C)P.in[(size_t)r * P.ldi + row] : (C)0;
          } else if constexpr (MODE == APPLY_F || MODE == PCG_F0) {
            y = (row < P.n) ? P.dscale[row] * (C)P.in[(size_t)r * P.ldi + row] : (C)0;
          } else if constexpr (MODE == PCG_B) {
            C pv = P.p[vi];
            if (P.j > 0 && s_live[r] && s_run[r]) {
              pv = P.s[vi] + s_scal[r][1] * pv;        // p_{j} = s_j + beta_{j-1} p_{j-1}
              P.p[vi] = pv;
            }
            y = pv;
          } else {  // PCG_F
            const C qv = P.q[vi];
            if (s_live[r] && s_run[r]) P.w[vi] += s_scal[r][2] * qv;       // omega_{j+1}
            y = P.dscale[row] * qv;                                       // R^{-T} q = R_hat^{-T} D^{-1} q
          }
          s_rhs[r][lane] = y - (s_part[0][r][lane] + s_part[1][r][lane] + s_part[2][r][lane] +
                                s_part[3][r][lane]);
        }
      }
      __syncthreads();

      // ---- diagonal block: x_I = Dinv_I * rhs (BWD) or Dinv_I^T * rhs -----
      const C *D = P.dinv + (size_t)I * NB * NB;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        C a = 0;
        if (BWD) {
#pragma unroll
          for (int c = 0; c < 16; ++c) a += D[(16 * w + c) * NB + lane] * s_rhs[r][16 * w + c];
        } else {
#pragma unroll
          for (int c = 0; c < 16; ++c) a += D[lane * NB + 16 * w + c] * s_rhs[r][16 * w + c];
        }
        s_part[w][r][lane] = a;
      }
      __syncthreads();

      // ---- publish and epilogue ------------------------------------------
      if (w == 0) {
        const int row = I * NB + lane;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const C x = s_part[0][r][lane] + s_part[1][r][lane] + s_part[2][r][lane] + s_part[3][r][lane];
          const size_t vi = (size_t)r * Np + row;
          P.chain[vi] = x;
          if constexpr (MODE == APPLY_B) {
            if (row < P.n) P.out[(size_t)r * P.ldo + row] = (double)(P.dscale[row] * x);
          } else if constexpr (MODE == APPLY_F) {
            if (row < P.n) P.out[(size_t)r * P.ldo + row] = (double)x;
          } else if constexpr (MODE == PCG_F0) {
            P.s[vi] = x;
            P.p[vi] = x;
            P.w[vi] = 0;
            const C ss = wave_sum(x * x);
            if (lane == 0) part_ptr(P.part, 0, 0, r, NR, N)[I] = ss;
          } else if constexpr (MODE == PCG_B) {
            const C qv = P.dscale[row] * x;        // q = R^{-1} p = D^{-1} R_hat^{-1} p
            const C pv = P.p[vi];
            if (s_live[r] && s_run[r]) P.q[vi] = qv;
            const C pp = wave_sum(pv * pv);
            const C qq = wave_sum(qv * qv);
            if (lane == 0) {
              part_ptr(P.part, P.j, 1, r, NR, N)[I] = pp;
              part_ptr(P.part, P.j, 2, r, NR, N)[I] = qq;
            }
          } else {  // PCG_F: x = t = R^{-T} q
            C sv = P.s[vi];
            if (s_live[r] && s_run[r]) {
              sv = sv - s_scal[r][2] * (P.p[vi] - s_scal[r][3] * x);   // s_{j+1}
              P.s[vi] = sv;
            }
            const C ss = wave_sum(sv * sv);
            if (lane == 0) part_ptr(P.part, P.j + 1, 0, r, NR, N)[I] = ss;
          }
        }
      }
      // step scalars for the trace and the done flags: block 0 writes them
      if constexpr (MODE == PCG_B || MODE == PCG_F) {
        if (I == 0 && tid < NR) {
          const int r = tid, L2 = P.L + 2, j = P.j;
          double *tr = P.trace + (size_t)r * 4 * L2;
          if constexpr (MODE == PCG_B) {
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
                  __hip_atomic_store(&sync[SI.status()], (int)TLS_ERR_INDEFINITE, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
                }
              }
            }
            P.done[j * NR + r] = now;
          }
        }
      }
      __threadfence();
      __syncthreads();
      if (tid == 0) flag_store_release(&sync[I], 1);
    }
  }

  // ---- completion: the last workgroup resets the sync area ---------------
  __syncthreads();
  if (tid == 0) {
    const int old = atomicAdd(&sync[SI.done()], 1);
    if (old == (int)gridDim.x - 1) {
      for (int i = 0; i < N; ++i) sync[i] = 0;
      sync[SI.ticket()] = 0;
      sync[SI.done()] = 0;
      __threadfence();
    }
  }
}

// omega (compute precision, padded) -> FP64 output, trace/done bookkeeping
template <typename C>
__global__ void k_pcg_finish(const C *w, double *out, int n, int Np, int NR) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int r = 0; r < NR; ++r) out[(size_t)r * n + i] = (double)w[(size_t)r * Np + i];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename S, typename C, int NR, int MODE>
static hipError_t launch_one(const TrsvParams<S, C> &P, hipStream_t st) {
  prof_begin(MODE <= APPLY_F ? PC_TRSV_APPLY : PC_PCG, st);
  hipLaunchKernelGGL((k_trsv<S, C, NR, MODE>), dim3(P.N), dim3(WG), 0, st, P);
  prof_end(st);
  return hipGetLastError();
}

template <typename S, typename C, int MODE>
static hipError_t launch_nr(int nrhs, const TrsvParams<S, C> &P, hipStream_t st) {
  return nrhs == 1 ? launch_one<S, C, 1, MODE>(P, st) : launch_one<S, C, 2, MODE>(P, st);
}

template <typename S, typename C>
static hipError_t dispatch_mode(int mode, int nrhs, const TrsvParams<S, C> &P, hipStream_t st) {
  switch (mode) {
    case APPLY_B: return launch_nr<S, C, APPLY_B>(nrhs, P, st);
    case APPLY_F: return launch_nr<S, C, APPLY_F>(nrhs, P, st);
    case PCG_F0: return launch_nr<S, C, PCG_F0>(nrhs, P, st);
    case PCG_B: return launch_nr<S, C, PCG_B>(nrhs, P, st);
    default: return launch_nr<S, C, PCG_F>(nrhs, P, st);
  }
}

template <typename C>
static hipError_t dispatch_storage(const FactorView &F, int mode, int nrhs, const SolveBufs &B,
                                   hipStream_t st) {
  auto fill = [&](auto *tiles) {
    using S = std::remove_const_t<std::remove_pointer_t<decltype(tiles)>>;
    TrsvParams<S, C> P{};
    P.tiles = tiles;
    P.dinv = (const C *)(std::is_same<C, double>::value ? (const void *)F.dinv64 : (const void *)F.dinv32);
    P.dscale = (const C *)(std::is_same<C, double>::value ? (const void *)F.dscale64 : (const void *)F.dscale32);
    P.N = F.N;
    P.Np = F.Np;
    P.n = F.n;
    P.sync = B.sync;
    P.chain = (C *)B.chain;
    P.in = B.in;
    P.out = B.out;
    P.ldi = B.ldi ? B.ldi : F.n;
    P.ldo = B.ldo ? B.ldo : F.n;
    P.s = (C *)B.s; P.p = (C *)B.p; P.q = (C *)B.q; P.w = (C *)B.w;
    P.part = (C *)B.part;
    P.done = B.done;
    P.neg = B.neg;
    P.trace = B.trace;
    P.sigma2 = B.sigma2;
    P.j = B.j;
    P.L = B.L;
    P.strict = B.strict;
    return dispatch_mode<S, C>(mode, nrhs, P, st);
  };
  switch (F.storage) {
    case TLS_FP64: return fill((const double *)F.tiles);
    case TLS_FP32: return fill((const float *)F.tiles);
    case TLS_FP16: return fill((const half_t *)F.tiles);
    default: return fill((const bf16_t *)F.tiles);
  }
}

hipError_t launch_trsv(const FactorView &F, int compute, int mode, int nrhs, const SolveBufs &B,
                       hipStream_t st) {
  if (compute == TLS_FP64) return dispatch_storage<double>(F, mode, nrhs, B, st);
  return dispatch_storage<float>(F, mode, nrhs, B, st);
}

hipError_t launch_pcg_finish(int compute, const void *w, double *out, int n, int Np, int nrhs,
                             hipStream_t st) {
  const int g = (n + 255) / 256;
  prof_begin(PC_SCALARS, st);
  if (compute == TLS_FP64)
    hipLaunchKernelGGL(k_pcg_finish<double>, dim3(g), dim3(256), 0, st, (const double *)w, out, n, Np, nrhs);
  else
    hipLaunchKernelGGL(k_pcg_finish<float>, dim3(g), dim3(256), 0, st, (const float *)w, out, n, Np, nrhs);
  prof_end(st);
  return hipGetLastError();
}

}  // namespace tls
