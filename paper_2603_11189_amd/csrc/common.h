// Shared device helpers of the DysonNet HIP library (gfx950 / CDNA4, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dn {

constexpr int WAVE = 64;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core tiles. Operand A (16 x 4): lane l holds A[l % 16][l / 16].
// Operand B (4 x 16): lane l holds B[l / 16][l % 16]. The accumulator of 4 values per
// lane holds column l % 16; its row for register r differs by element type (measured on
// gfx950): float: 4*(l/16) + r, double: 4*r + l/16.
template <typename T> struct Mma;
template <> struct Mma<float> {
  using acc = f4;
  __device__ static inline acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  // row = lane_row(lane) + r_row(r): the first part per lane, the second the same for all
  __device__ static inline int lane_row(int lane) { return 4 * (lane >> 4); }
  __device__ static inline int r_row(int r) { return r; }
};
template <> struct Mma<double> {
  using acc = d4;
  __device__ static inline acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
  __device__ static inline int lane_row(int lane) { return lane >> 4; }
  __device__ static inline int r_row(int r) { return 4 * r; }
};

// 16x16x32 bf16 matrix-core tile (gfx950) with float accumulation. Operand A (16 x 32): lane l
// holds A[l % 16][8 (l / 16) + e], e = 0..7; operand B (32 x 16): lane l holds
// B[8 (l / 16) + e][l % 16]; the accumulator is laid out as Mma<float> (row 4 (l / 16) + r,
// column l % 16). float -> bf16 conversion rounds to nearest even.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
__device__ inline f4 mma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Green's-function tap tables: per channel TS = 2 Np + 128 entries, offset r = i - i' stored
// at r + TOFF. Offsets |r| < N hold the taps (periodic chains: the aliased g(r mod N) for every
// stored r); the 64-entry margins let slice windows run past the chain ends without bounds
// checks (open chains: zeros there).
__host__ __device__ inline int tap_stride(int Np) { return 2 * Np + 128; }
__host__ __device__ inline int tap_off(int Np) { return Np - 1 + 64; }

template <typename T> __device__ inline T act_fn(int act, T x) {
  if (act == 0) return x / (T(1) + exp(-x));          // SiLU
  if (act == 1) return tanh(x);                      // tanh
  return x;                                          // identity
}

// log cosh(x), relative-accurate everywhere (double).
__device__ inline double logcosh_d(double x) {
  double ax = fabs(x);
  if (ax <= 1.0) {
    double sh = sinh(0.5 * x);
    return log1p(2.0 * sh * sh);
  }
  return ax + log1p(exp(-2.0 * ax)) - 0.69314718055994530942;
}

// log cosh(a + d) - log cosh(a) without cancellation: cosh(a+d)/cosh(a) =
// 1 + 2 sinh^2(d/2) + tanh(a) sinh(d) for |d| <= 1, plain difference otherwise.
__device__ inline double lcd_d(double a, double d) {
  if (fabs(d) <= 1.0) {
    double sh = sinh(0.5 * d);
    return log1p(2.0 * sh * sh + tanh(a) * sinh(d));
  }
  return logcosh_d(a + d) - logcosh_d(a);
}

// Wave-level sum (all 64 lanes get the total).
template <typename T> __device__ inline T wave_sum(T v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

}  // namespace dn
