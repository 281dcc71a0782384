// Stochastic reconfiguration (natural-gradient) update of VMC (Sec. II and VI; App. "Network
// parameters": standard SR with a diagonal shift). With samples of weight w_b (sum 1),
// log-derivatives O [B][P] and local energies E_b:
//   Ebar = sum_b w_b E_b,  F = O^T (w * (E - Ebar)),  Obar = O^T w,
//   S v = O^T (w * t),  t_b = (O v)_b - Obar . v          (= Oc^T W Oc v, Oc = O - 1 Obar^T)
//   (S + shift I) x = F by conjugate gradients,  delta = -eta x.
// O is read in the model's field type and every sum is float64. The passes over O are
// bandwidth bound: one thread per parameter for the column sums (coalesced rows), workgroups
// over segments of each sample's row for the row products.
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

// The passes over O split their reduction so that enough waves are in flight to keep HBM
// busy: the column sums over SR_ROW_SLICES slices of the rows (partials [slice][P], added
// in slice order by sr_colsum_fin_kernel), the row products over SR_ROW_SEGS segments of
// each row, SR_ROW_BLK rows per workgroup (partials [row][segment], added in order by
// sr_rowdot_fin_kernel).
constexpr int SR_ROW_SLICES = 8;
constexpr int SR_ROW_SEGS = 16;
constexpr int SR_ROW_BLK = 4;  // rows per workgroup of the row products

// part[y][k] = sum over rows b of slice y of coef_b O_bk, one thread per parameter.
template <typename T>
__global__ __launch_bounds__(256) void sr_colsum_part_kernel(const T* __restrict__ O, long P, int B,
                                                             const double* __restrict__ coef, double* __restrict__ part) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const int per = (B + SR_ROW_SLICES - 1) / SR_ROW_SLICES;
  const int b0 = blockIdx.y * per, b1 = min(B, b0 + per);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int b = b0;
  for (; b + 16 <= b1; b += 16) {
    T o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) o[i] = O[(long)(b + i) * P + k];
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i & 3] += coef[b + i] * (double)o[i];
  }
  for (; b < b1; ++b) s[0] += coef[b] * (double)O[(long)b * P + k];
  part[(long)blockIdx.y * P + k] = (s[0] + s[1]) + (s[2] + s[3]);
}

// out_k = sum_y part[y][k] in slice order (+ shift v_k when v is given).
__global__ __launch_bounds__(256) void sr_colsum_fin_kernel(const double* __restrict__ part, long P,
                                                            const double* __restrict__ v, double shift,
                                                            double* __restrict__ out) {
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (long)gridDim.x * blockDim.x) {
    double r = 0.0;
#pragma unroll
    for (int y = 0; y < SR_ROW_SLICES; ++y) r += part[(long)y * P + k];
    if (v) r += shift * v[k];
    out[k] = r;
  }
}

// part[b][y] = sum over the y-th segment of row b of O_bk v_k. Workgroup (g, y) takes rows
// SR_ROW_BLK g .. SR_ROW_BLK g + SR_ROW_BLK - 1, so every element of v read serves that many
// rows (v, float64, would otherwise move twice the bytes of O through the caches).
template <typename T>
__global__ __launch_bounds__(256) void sr_rowdot_part_kernel(const T* __restrict__ O, long P, int B,
                                                             const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double red[SR_ROW_BLK][4];
  const int b0 = blockIdx.x * SR_ROW_BLK, y = blockIdx.y;
  const long seg = (P + SR_ROW_SEGS - 1) / SR_ROW_SEGS;
  const long k0 = (long)y * seg, k1 = min(P, k0 + seg);
  const T* rows[SR_ROW_BLK];
#pragma unroll
  for (int r = 0; r < SR_ROW_BLK; ++r) rows[r] = O + (long)min(b0 + r, B - 1) * P;  // a row past B repeats the last
  double sp[SR_ROW_BLK][2] = {};
  const long st = blockDim.x;
  long k = k0 + threadIdx.x;
  constexpr int U = 8;  // columns in flight per thread
  for (; k + (U - 1) * st < k1; k += U * st) {
    double vv[U];
    T o[SR_ROW_BLK][U];
#pragma unroll
    for (int i = 0; i < U; ++i) vv[i] = v[k + i * st];
#pragma unroll
    for (int r = 0; r < SR_ROW_BLK; ++r)
#pragma unroll
      for (int i = 0; i < U; ++i) o[r][i] = rows[r][k + i * st];
#pragma unroll
    for (int r = 0; r < SR_ROW_BLK; ++r)
#pragma unroll
      for (int i = 0; i < U; ++i) sp[r][i & 1] += (double)o[r][i] * vv[i];
  }
  for (; k < k1; k += st) {
    const double vk = v[k];
#pragma unroll
    for (int r = 0; r < SR_ROW_BLK; ++r) sp[r][0] += (double)rows[r][k] * vk;
  }
#pragma unroll
  for (int r = 0; r < SR_ROW_BLK; ++r) {
    const double s = wave_sum(sp[r][0] + sp[r][1]);
    if ((threadIdx.x & 63) == 0) red[r][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < SR_ROW_BLK && b0 + (int)threadIdx.x < B) {
    const int r = threadIdx.x;
    part[(long)(b0 + r) * SR_ROW_SEGS + y] = (red[r][0] + red[r][1]) + (red[r][2] + red[r][3]);
  }
}

// t_b = w_b (sum_y part[b][y] - *sub), the segments added in order.
__global__ __launch_bounds__(256) void sr_rowdot_fin_kernel(const double* __restrict__ part, int B,
                                                            const double* __restrict__ sub,
                                                            const double* __restrict__ w, double* __restrict__ t) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
#pragma unroll
  for (int y = 0; y < SR_ROW_SEGS; ++y) s += part[(long)b * SR_ROW_SEGS + y];
  t[b] = w[b] * (s - *sub);
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
