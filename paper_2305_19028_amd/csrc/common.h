// Shared device/host helpers of libtls: storage types, IEEE round-to-nearest-
// even conversions, fixed-order reductions, inter-workgroup flags.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tls.h"

namespace tls {

constexpr int NB = 64;          // tile order of the blocked factor and solves
constexpr int WG = 256;         // threads per workgroup (4 waves of 64)
constexpr int SPIN_LIMIT = 1 << 22;

// 16-bit storage words (raw IEEE bits)
struct half_t { uint16_t bits; };
struct bf16_t { uint16_t bits; };

// --------------------------------------------------------------------------
// Round-to-nearest-even from binary64 to a narrower binary format with
// MB stored significand bits, minimum normal exponent EMIN and exponent
// bias BIAS (IEEE 754: keep MB+1 significant bits, quantum floored at the
// subnormal quantum 2^(EMIN-MB), overflow to infinity).
// --------------------------------------------------------------------------
template <int MB, int EMIN, int BIAS, int EBITS>
__host__ __device__ inline uint32_t rne_from_double(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t sign = (uint32_t)(u >> 63) << (MB + EBITS);
  const uint64_t a = u & 0x7fffffffffffffffull;
  const uint32_t inf = ((1u << EBITS) - 1u) << MB;
  if (a >= 0x7ff0000000000000ull)  // Inf or NaN
    return sign | inf | (a > 0x7ff0000000000000ull ? (1u << (MB - 1)) : 0u);
  if (a == 0) return sign;
  const int e = (int)(a >> 52) - 1023;  // exponent of the leading bit
  if (e > BIAS) return sign | inf;      // >= 2^(emax+1): overflow
  const uint64_t mant = (a & 0xfffffffffffffull) | 0x10000000000000ull;
  int shift = 52 - MB;
  if (e < EMIN) shift += EMIN - e;      // subnormal result
  if (shift >= 64) return sign;         // far below half the smallest subnormal
  uint64_t kept = mant >> shift;
  const uint64_t rem = mant & ((1ull << shift) - 1ull);
  const uint64_t halfway = 1ull << (shift - 1);
  if (rem > halfway || (rem == halfway && (kept & 1ull))) ++kept;
  if (e < EMIN) return sign | (uint32_t)kept;  // kept <= 2^MB: 2^MB encodes the min normal
  int E = e + BIAS;
  if (kept == (1ull << (MB + 1))) { kept >>= 1; ++E; }
  if (E >= (1 << EBITS) - 1) return sign | inf;
  return sign | ((uint32_t)E << MB) | ((uint32_t)kept & ((1u << MB) - 1u));
}

__host__ __device__ inline uint16_t f64_to_f16_bits(double x) {
  return (uint16_t)rne_from_double<10, -14, 15, 5>(x);
}
__host__ __device__ inline uint16_t f64_to_bf16_bits(double x) {
  return (uint16_t)rne_from_double<7, -126, 127, 8>(x);
}
__host__ __device__ inline uint32_t f64_to_f32_bits(double x) {
  return rne_from_double<23, -126, 127, 8>(x);
}

__device__ inline float f16_bits_to_float(uint16_t h) {
  return (float)__builtin_bit_cast(_Float16, h);
}
__device__ inline float bf16_bits_to_float(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// load a storage element as compute type C
template <typename C> __device__ inline C ld_as(const double *p) { return (C)(*p); }
template <typename C> __device__ inline C ld_as(const float *p) { return (C)(*p); }
template <typename C> __device__ inline C ld_as(const half_t *p) { return (C)f16_bits_to_float(p->bits); }
template <typename C> __device__ inline C ld_as(const bf16_t *p) { return (C)bf16_bits_to_float(p->bits); }

template <typename C> __device__ inline C cvt(const double &v) { return (C)v; }
template <typename C> __device__ inline C cvt(const float &v) { return (C)v; }
template <typename C> __device__ inline C cvt(const half_t &v) { return (C)f16_bits_to_float(v.bits); }
template <typename C> __device__ inline C cvt(const bf16_t &v) { return (C)bf16_bits_to_float(v.bits); }

// store a double as storage type S with a single rounding
template <typename S> __device__ inline S st_from(double v);
template <> __device__ inline double st_from<double>(double v) { return v; }
template <> __device__ inline float st_from<float>(double v) {
  return __builtin_bit_cast(float, f64_to_f32_bits(v));
}
template <> __device__ inline half_t st_from<half_t>(double v) { return half_t{f64_to_f16_bits(v)}; }
template <> __device__ inline bf16_t st_from<bf16_t>(double v) { return bf16_t{f64_to_bf16_bits(v)}; }

// round one value to u_q, returned as double (exactly representable)
__device__ inline double quantize(double v, int q) {
  switch (q) {
    case TLS_FP64: return v;
    case TLS_FP32: return (double)__builtin_bit_cast(float, f64_to_f32_bits(v));
    case TLS_FP16: return (double)f16_bits_to_float(f64_to_f16_bits(v));
    case TLS_BF16X3: {                 // hi + lo, each rounded to BF16 (exact in FP32)
      const double hi = (double)bf16_bits_to_float(f64_to_bf16_bits(v));
      return hi + (double)bf16_bits_to_float(f64_to_bf16_bits(v - hi));
    }
    default: return (double)bf16_bits_to_float(f64_to_bf16_bits(v));
  }
}
// storage precision of the factor computed at factor precision q
inline int storage_of(int q) { return q == TLS_BF16X3 ? TLS_FP32 : q; }

template <typename S> constexpr int prec_of();
template <> constexpr int prec_of<double>() { return TLS_FP64; }
template <> constexpr int prec_of<float>() { return TLS_FP32; }
template <> constexpr int prec_of<half_t>() { return TLS_FP16; }
template <> constexpr int prec_of<bf16_t>() { return TLS_BF16; }

inline size_t prec_bytes(int p) { return p == TLS_FP64 ? 8 : p == TLS_FP32 ? 4 : 2; }

inline double unit_roundoff(int p) {
  switch (p) {
    case TLS_FP64: return 1.1102230246251565e-16;   // 2^-53
    case TLS_FP32: return 5.9604644775390625e-08;   // 2^-24
    case TLS_FP16: return 4.8828125e-04;            // 2^-11
    case TLS_BF16X3: return 1.52587890625e-05;      // split BF16 pair: 2^-16
    default: return 3.90625e-03;                    // bf16: 2^-8
  }
}

// --------------------------------------------------------------------------
// fixed-order reductions
// --------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_sum(T v) {
  // butterfly over 64 lanes; every lane ends with the same value, combined
  // in the same order on every call
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// PCGTLS (Algorithm 3) does not run step j > 0 once eta_j <= u_p^2 eta_0:
// the preconditioned residual s_j is then zero in the working precision
// relative to s_0, and further steps only add rounding to omega
template <typename C> __host__ __device__ constexpr C pcg_eta_floor();
template <> __host__ __device__ constexpr float pcg_eta_floor<float>() { return 0x1p-48f; }
template <> __host__ __device__ constexpr double pcg_eta_floor<double>() { return 0x1p-106; }

// 1/sqrt(p) for the Cholesky pivots. FP32: the hardware reciprocal square
// root alone (within about one unit in the last place, the size of the
// factorization's own rounding). FP64: the hardware estimate refined by one
// Newton step y <- y (3 - p y^2) / 2 (relative error about the square of the
// estimate's). For p <= 0 or NaN both give NaN or Inf, and p times the
// result is NaN.
__device__ inline float chol_rsqrt(float p) { return __builtin_amdgcn_rsqf(p); }
__device__ inline double chol_rsqrt(double p) {
  const double y = __builtin_amdgcn_rsq(p);
  return y * (1.5 - 0.5 * p * y * y);
}

// sum over a 256-thread block; result valid in every thread
template <typename T>
__device__ inline T block_sum(T v, T *scratch /* >= 4 */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[w] = v;
  __syncthreads();
  T r = scratch[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r += scratch[i];
  return r;
}

// --------------------------------------------------------------------------
// inter-workgroup flags (agent scope: visible across XCDs)
// --------------------------------------------------------------------------
__device__ inline int flag_load_acquire(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void flag_store_release(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int flag_load_relaxed(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace tls
