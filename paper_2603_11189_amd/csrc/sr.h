// Stochastic reconfiguration (natural-gradient) update of VMC (Sec. II and VI; App. "Network
// parameters": standard SR with a diagonal shift). With samples of weight w_b (sum 1),
// log-derivatives O [B][P] and local energies E_b:
//   Ebar = sum_b w_b E_b,  F = O^T (w * (E - Ebar)),  Obar = O^T w,
//   S v = O^T (w * t),  t_b = (O v)_b - Obar . v          (= Oc^T W Oc v, Oc = O - 1 Obar^T)
//   (S + shift I) x = F by conjugate gradients,  delta = -eta x.
// O is read in the model's field type and every sum is float64. The passes over O are
// bandwidth bound: one thread per parameter for the column sums (coalesced rows), one
// workgroup per sample for the row products.
// A complex wavefunction with real parameters (complex read-out) has O = Or + i Oi and complex
// E_b; its force and SR matrix are the real parts of the conjugated moments, which split into
// the real problem of the rows Or (energies Re E) plus that of the rows Oi (energies Im E), each
// centred by its own mean: O is then [2][B][P] (2B rows) and every row pass covers both halves.
#pragma once
#include "common.h"

namespace dn {

// Ebar and the weighted centred energies we_b = w_b (E_b - Ebar) of the energies E[b * stride];
// w = 1/B when not given.
__global__ __launch_bounds__(1024) void sr_energy_kernel(const double* __restrict__ E, int stride,
                                                         const double* __restrict__ w, int B,
                                                         double* __restrict__ wout, double* __restrict__ we,
                                                         double* __restrict__ ebar) {
  __shared__ double part[1024];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) s += (w ? w[b] : 1.0 / B) * E[(long)b * stride];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  const double eb = part[0];
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    const double wb = w ? w[b] : 1.0 / B;
    wout[b] = wb;
    we[b] = wb * (E[(long)b * stride] - eb);
  }
  if (threadIdx.x == 0) *ebar = eb;
}

// out_k = sum_b coef_b O_bk (+ shift v_k when v is given), one thread per parameter.
template <typename T>
__global__ __launch_bounds__(256) void sr_colsum_kernel(const T* __restrict__ O, long P, int B,
                                                        const double* __restrict__ coef, const double* __restrict__ v,
                                                        double shift, double* __restrict__ out) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  // four partial sums, sixteen rows requested together (the loads, not the adds, set the pace)
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int b = 0;
  for (; b + 16 <= B; b += 16) {
    T o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) o[i] = O[(long)(b + i) * P + k];
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i & 3] += coef[b + i] * (double)o[i];
  }
  for (; b < B; ++b) s[0] += coef[b] * (double)O[(long)b * P + k];
  double r = (s[0] + s[1]) + (s[2] + s[3]);
  if (v) r += shift * v[k];
  out[k] = r;
}

// t_b = sum_k O_bk v_k - *sub (one workgroup per sample), scaled by w_b.
template <typename T>
__global__ __launch_bounds__(256) void sr_rowdot_kernel(const T* __restrict__ O, long P, const double* __restrict__ v,
                                                        const double* __restrict__ sub, const double* __restrict__ w,
                                                        double* __restrict__ t) {
  __shared__ double part[4];
  const int b = blockIdx.x;
  const T* row = O + (long)b * P;
  // eight elements of the row requested together, four partial sums
  double sp[4] = {0.0, 0.0, 0.0, 0.0};
  const long st = blockDim.x;
  long k = threadIdx.x;
  for (; k + 7 * st < P; k += 8 * st) {
    T o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = row[k + i * st];
#pragma unroll
    for (int i = 0; i < 8; ++i) sp[i & 3] += (double)o[i] * v[k + i * st];
  }
  for (; k < P; k += st) sp[0] += (double)row[k] * v[k];
  double s = wave_sum((sp[0] + sp[1]) + (sp[2] + sp[3]));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) t[b] = w[b] * (part[0] + part[1] + part[2] + part[3] - *sub);
}

// a . b in a fixed order, in two steps: SR_DOT_WG workgroups of 256 threads form partial sums
// (sr_dot_kernel), one workgroup adds them (sr_dot_sum_kernel).
constexpr int SR_DOT_WG = 256;
__global__ __launch_bounds__(256) void sr_dot_kernel(const double* __restrict__ a, const double* __restrict__ b, long n,
                                                     double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)SR_DOT_WG * 256) s += a[i] * b[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ __launch_bounds__(256) void sr_dot_sum_kernel(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[4];
  double s = wave_sum(part[threadIdx.x]);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// CG scalars in one small array: [0] r.r, [1] p.Ap, [2] new r.r, [3] Obar.p, [4] F.F, [5] Ebar
// (real part), [6] Ebar (imaginary part), [7] Obar.p of the imaginary rows
// x += alpha p, r -= alpha Ap with alpha = r.r / p.Ap.
__global__ void sr_step_kernel(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                               const double* __restrict__ Ap, long n, const double* __restrict__ sc) {
  const double alpha = sc[1] > 0.0 ? sc[0] / sc[1] : 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    r[i] -= alpha * Ap[i];
  }
}

// p = r + beta p with beta = new r.r / r.r (a last workgroup-independent read of sc[0]).
__global__ void sr_dir_kernel(double* __restrict__ p, const double* __restrict__ r, long n,
                              const double* __restrict__ sc) {
  const double beta = sc[0] > 0.0 ? sc[2] / sc[0] : 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = r[i] + beta * p[i];
}

// sc[0] = sc[2] (after the direction update), and the initial copies x = 0, r = p = F.
__global__ void sr_roll_kernel(double* sc) { sc[0] = sc[2]; }
__global__ void sr_init_kernel(double* __restrict__ x, double* __restrict__ r, double* __restrict__ p,
                               const double* __restrict__ F, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    x[i] = 0.0;
    r[i] = F[i];
    p[i] = F[i];
  }
}
__global__ void sr_scale_kernel(const double* __restrict__ x, double eta, long n, double* __restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = -eta * x[i];
}

}  // namespace dn
