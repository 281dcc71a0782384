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

// ---- complex read-out (a complex output matrix A: Omega_0 + i Omega_1 is one complex unit) ----

// x - 2 pi k with k the nearest integer: the phase representative in [-pi, pi].
__device__ inline double wrap_phase_d(double y) {
  const double two_pi = 6.28318530717958647692;
  return y - two_pi * rint(y / two_pi);
}

// tanh(x + iy) = (sinh 2x + i sin 2y) / (cosh 2x + cos 2y), and +-1 once |x| > 20 (the
// remainder is below e^-40).
__device__ inline void ctanh_d(double x, double y, double* tr, double* ti) {
  if (fabs(x) > 20.0) {
    *tr = copysign(1.0, x);
    *ti = 0.0;
    return;
  }
  const double den = cosh(2.0 * x) + cos(2.0 * y);
  *tr = sinh(2.0 * x) / den;
  *ti = sin(2.0 * y) / den;
}

// log cosh(x + iy). |cosh z|^2 / cosh^2 x is both 1 - (sin y / cosh x)^2 and
// tanh^2 x + (cos y / cosh x)^2: log1p of the first while (sin y / cosh x)^2 <= 1/2, the log
// of the second (no cancellation next to a zero of cosh) beyond. arg = atan2(tanh x sin y, cos y).
__device__ inline void logcosh_cd(double x, double y, double* re, double* im) {
  const double ch = cosh(x), sy = sin(y), cy = cos(y), th = tanh(x);
  const double q = sy / ch, c = cy / ch;
  const double r = q * q > 0.5 ? log(th * th + c * c) : log1p(-q * q);
  *re = logcosh_d(x) + 0.5 * r;
  *im = atan2(th * sy, cy);
}

// log cosh(a + d) - log cosh(a) for complex a, d, phase in [-pi, pi]. For |d| <= 1:
// cosh(a + d)/cosh(a) = 1 + w with w = 2 sinh^2(d/2) + tanh(a) sinh(d), and
// log|1 + w| = 1/2 log1p(u), u = 2 Re w + |w|^2, while |u| <= 1/2 (else the log of
// (1 + Re w)^2 + (Im w)^2); otherwise the difference of two log cosh values.
__device__ inline void lcd_cd(double ar, double ai, double dr, double di, double* re, double* im) {
  if (hypot(dr, di) <= 1.0) {
    const double p = 0.5 * dr, q = 0.5 * di;
    const double hr = sinh(p) * cos(q), hi = cosh(p) * sin(q);  // sinh(d/2)
    double wr = 2.0 * (hr * hr - hi * hi), wi = 4.0 * hr * hi;
    const double sr = sinh(dr) * cos(di), si = cosh(dr) * sin(di);  // sinh(d)
    double tr, ti;
    ctanh_d(ar, ai, &tr, &ti);
    wr += tr * sr - ti * si;
    wi += tr * si + ti * sr;
    const double u = 2.0 * wr + wr * wr + wi * wi;
    const double lm = fabs(u) <= 0.5 ? log1p(u) : log((1.0 + wr) * (1.0 + wr) + wi * wi);
    *re = 0.5 * lm;
    *im = atan2(wi, 1.0 + wr);
    return;
  }
  double r1, i1, r0, i0;
  logcosh_cd(ar + dr, ai + di, &r1, &i1);
  logcosh_cd(ar, ai, &r0, &i0);
  *re = r1 - r0;
  *im = wrap_phase_d(i1 - i0);
}

// The read-out of the two output pre-activations (a0, a1): two real log-cosh units (cplx = 0,
// one double at lp[b]) or one complex unit a0 + i a1 (cplx = 1, (re, im) at lp[2b], lp[2b+1]).
__device__ inline void put_logpsi(double* lp, long b, double a0, double a1, int cplx) {
  if (cplx) {
    logcosh_cd(a0, a1, &lp[2 * b], &lp[2 * b + 1]);
  } else {
    lp[b] = logcosh_d(a0) + logcosh_d(a1);
  }
}

// log psi(s')/psi(s) from Omega(s) = (a0, a1) and dOmega = (d0, d1), stored like put_logpsi.
__device__ inline void put_ratio(double* lr, long o, double a0, double a1, double d0, double d1, int cplx) {
  if (cplx) {
    lcd_cd(a0, a1, d0, d1, &lr[2 * o], &lr[2 * o + 1]);
  } else {
    lr[o] = lcd_d(a0, d0) + lcd_d(a1, d1);
  }
}

// log |psi(s')/psi(s)|: the real part of put_ratio's value.
__device__ inline double ratio_re(double a0, double a1, double d0, double d1, int cplx) {
  if (cplx) {
    double re, im;
    lcd_cd(a0, a1, d0, d1, &re, &im);
    return re;
  }
  return lcd_d(a0, d0) + lcd_d(a1, d1);
}

// Workgroup barrier that orders LDS only: global requests stay in flight across it (for
// kernels whose waves share no global data within the launch).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// fourth word of a raw buffer resource on gfx9-family devices (32-bit data format)
constexpr int BUF_DW3 = 0x00020000;

// Cross-lane exchanges without the LDS crossbar, word by word (T of 4 or 8 bytes).
// dpp_get<CTRL>: the value of the lane the data-parallel-primitive control CTRL names.
constexpr int DPP_XOR1 = 0xB1;         // quad permutation [1, 0, 3, 2]: lane l ^ 1
constexpr int DPP_XOR2 = 0x4E;         // quad permutation [2, 3, 0, 1]: lane l ^ 2
constexpr int DPP_HALF_MIRROR = 0x141;  // lane 7 - l within each group of 8
constexpr int DPP_MIRROR = 0x140;       // lane 15 - l within each group of 16
template <int CTRL, typename T> __device__ inline T dpp_get(T v) {
  static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
  int w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_update_dpp(0, w[i], CTRL, 0xF, 0xF, false);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}
// v(l) + v(l ^ H) for H = 16 or 32 with the gfx950 row swaps: swapping the odd 16-lane rows
// of one copy of v with the even rows of another (H = 16), or the upper half of one with
// the lower half of the other (H = 32), leaves every lane holding v(l) in one copy and
// v(l ^ H) in the other.
template <int H, typename T> __device__ inline T swap_sum(T v) {
  static_assert(H == 16 || H == 32, "row swaps pair lanes 16 or 32 apart");
  constexpr int NW = sizeof(T) / 4;
  unsigned w[NW], a[NW], b[NW];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if constexpr (H == 16) {
      const auto r = __builtin_amdgcn_permlane16_swap(w[i], w[i], false, false);
      a[i] = r[0];
      b[i] = r[1];
    } else {
      const auto r = __builtin_amdgcn_permlane32_swap(w[i], w[i], false, false);
      a[i] = r[0];
      b[i] = r[1];
    }
  }
  T x, y;
  __builtin_memcpy(&x, a, sizeof(T));
  __builtin_memcpy(&y, b, sizeof(T));
  return x + y;
}

// Wave-level sum (all 64 lanes get the total; call with the whole wave active). Pairs of
// lanes 1, 2, 4, 8, 16, 32 apart are added in turn; for 4 and 8 the mirrored lane holds the
// same partial sum as lane l ^ 4 or l ^ 8, since the earlier steps made it uniform over
// each group of 4 or 8.
template <typename T> __device__ inline T wave_sum(T v) {
  v += dpp_get<DPP_XOR1>(v);
  v += dpp_get<DPP_XOR2>(v);
  v += dpp_get<DPP_HALF_MIRROR>(v);
  v += dpp_get<DPP_MIRROR>(v);
  v = swap_sum<16>(v);
  return swap_sum<32>(v);
}

}  // namespace dn
