// ABACUS for networks of one or two blocks with per-flip cost independent of the chain
// length (Sec. III, Theorem 1; App. "Efficient construction of link tensors").
//
// With two blocks the only link whose source is the input change itself and whose path
// crosses a background vertex is the pivot-0 link of block 2 (the paper's two-layer link,
// built there from a composite Green's function by FFT):
//   Lam_b(z, delta) = [G^(2) D0^(1) G^(1) E delta_z]_(z + delta),     D0^(1)_i = U diag(chi0_i) V,
// the response at site z + delta of block 2's mixer to a unit input change at site z, seen
// through sample b's frozen block-1 vertices. Written out per channel c,
//   Lam_b(z, delta)_c = sum_c' U_(c,c') sum_u g^(2)_c(delta - u) Pq_c'(u) chi0_(z+u, c'),
// Pq(u) = V^(1) (E * g^(1)(u)): for every (delta, c, c') a correlation over u of the sample's
// block-1 gate with the parameter-only kernel K(u) = g^(2)_c(delta - u) Pq_c'(u). It is
// formed in the frequency domain: the kernels' spectra (times U) are parameter-only and built
// once per parameter update (lam_param_kernel); per sample the gate's channels are
// transformed (lam_fwd_kernel), contracted over c' at every frequency on the matrix cores
// (lam_gemm_kernel, a complex [d x d] x [d x samples] product per offset and frequency) and
// transformed back (lam_inv_kernel). Transform length n: a power of two >= 2N - 1, so the
// circular correlation equals the linear one (open chains: u in [-(N-1), N-1]; periodic
// chains: u in [0, N) over the gate extended periodically to 2N - 1 sites).
//
// Per flip (shallow_kernel) only slice-sized work remains:
//   e1_i = U^(1) (dchi1_i * (p0^(1)_i + sum_z c_z Pq(i - z))),                i in S_1
//   x2_a = v0^(2)_a + sum_(i in S_1) g^(2)(a - i) e1_i + sum_z c_z Lam(z, a - z), a in S_2
//   e2_a = U^(2) (dchi2_a * V^(2) x2_a)
//   dOmega = sum_z c_z T^(0)_z . E + sum_(i in S_1) T^(1)_i . e1_i + sum_(a in S_2) Wk_a . e2_a
// with c_z = -2 s_z at the cluster sites z and the output links T^(l) = dOmega/dh^(l)
// (per-sample adjoint fields: T^(1) = Wk + G^(2)T D0^(2)T Wk, T^(0) = Wk + G^(1)T D0^(1)T T^(1)).
// One block: e1 is read out with Wk and e^(0) with T^(0) = Wk + G^(1)T D0^(1)T Wk.
#pragma once
#include "common.h"
#include "kernels.h"

namespace dn {

__device__ inline int bitrev(int q, int logn) { return (int)(__brev((unsigned)q) >> (32 - logn)); }

// Twiddles w_k = exp(-2 pi i k / n), k < n / 2, from a float64 sincos.
template <typename T> __device__ inline void fft_twiddles(T* twr, T* twi, int logn) {
  const int n = 1 << logn;
  for (int k = threadIdx.x; k < n / 2; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    twr[k] = (T)c;
    twi[k] = (T)(-s);
  }
}

// In-place decimation-in-time transforms of nseq complex sequences of length n = 2^logn held
// in LDS at row stride ld, already in bit-reversed order. Forward: sum_k x_k w^(jk); inverse:
// the conjugate twiddles (unscaled). Two radix-2 stages at a time (spans h and 2h) as one
// radix-4 step per thread, after a first radix-2 stage when logn is odd: half the LDS passes
// and barriers of stage-by-stage butterflies. Ends with a workgroup barrier.
template <typename T>
__device__ void fft_stages(T* xr, T* xi, const T* twr, const T* twi, int logn, int ld, int nseq, bool inverse) {
  int ls = 1;
  if (logn & 1) {  // span-1 stage (twiddle 1)
    const int hn = 1 << (logn - 1);
    for (int idx = threadIdx.x; idx < nseq * hn; idx += blockDim.x) {
      const int s = idx >> (logn - 1), b = idx & (hn - 1);
      const int i = s * ld + 2 * b;
      const T ur = xr[i], ui = xi[i], vr = xr[i + 1], vi = xi[i + 1];
      xr[i] = ur + vr;
      xi[i] = ui + vi;
      xr[i + 1] = ur - vr;
      xi[i + 1] = ui - vi;
    }
    __syncthreads();
    ls = 2;
  }
  const int qn = logn >= 2 ? 1 << (logn - 2) : 0;
  for (; ls < logn; ls += 2) {
    const int h = 1 << (ls - 1);
    for (int idx = threadIdx.x; idx < nseq * qn; idx += blockDim.x) {
      const int s = idx >> (logn - 2), b = idx & (qn - 1);
      const int k = b & (h - 1), grp = b >> (ls - 1);
      const int i0 = s * ld + (grp << (ls + 1)) + k, i1 = i0 + h, i2 = i1 + h, i3 = i2 + h;
      // w1 = W_(2h)^k for the span-h stage, w2 = W_(4h)^k and w3 = W_(4h)^(k+h) = w2 (-+ i)
      const T w1r = twr[k << (logn - ls)], w1i = inverse ? -twi[k << (logn - ls)] : twi[k << (logn - ls)];
      const T w2r = twr[k << (logn - ls - 1)], w2i = inverse ? -twi[k << (logn - ls - 1)] : twi[k << (logn - ls - 1)];
      const T w3r = inverse ? -w2i : w2i, w3i = inverse ? w2r : -w2r;
      const T a0r = xr[i0], a0i = xi[i0], a1r = xr[i1], a1i = xi[i1];
      const T a2r = xr[i2], a2i = xi[i2], a3r = xr[i3], a3i = xi[i3];
      const T t1r = w1r * a1r - w1i * a1i, t1i = w1r * a1i + w1i * a1r;
      const T t3r = w1r * a3r - w1i * a3i, t3i = w1r * a3i + w1i * a3r;
      const T b0r = a0r + t1r, b0i = a0i + t1i, b1r = a0r - t1r, b1i = a0i - t1i;
      const T b2r = a2r + t3r, b2i = a2i + t3i, b3r = a2r - t3r, b3i = a2i - t3i;
      const T u2r = w2r * b2r - w2i * b2i, u2i = w2r * b2i + w2i * b2r;
      const T u3r = w3r * b3r - w3i * b3i, u3i = w3r * b3i + w3i * b3r;
      xr[i0] = b0r + u2r;
      xi[i0] = b0i + u2i;
      xr[i2] = b0r - u2r;
      xi[i2] = b0i - u2i;
      xr[i1] = b1r + u3r;
      xi[i1] = b1i + u3i;
      xr[i3] = b1r - u3r;
      xi[i3] = b1i - u3i;
    }
    __syncthreads();
  }
}

// Offsets delta of the pivot-0 link: [dlo, dlo + ND). S_2 of a cluster with sites z and
// z + ext reaches 2 w_c sites beyond it, so delta in [-(2 w_c + ext), 2 w_c + ext].
__host__ __device__ inline int lam_nd(int w_c, int ext_max) { return 2 * (2 * w_c + ext_max) + 1; }

// ---- parameter-only spectra (float64): M[delta][omega][c'][c] = U^(1)_(c,c') Kc(omega),
// Kc(omega) = sum_u K(u) exp(+2 pi i omega u / n) = conj(DFT of K), omega = 0 .. n/2.
struct LamParamArgs {
  const double* taps;  // float64 tap table [L][DP][TS] (block 2 = row block 1)
  const double* Pq;    // float64 unit-flip table, unshifted copy [DP][TS]
  const double* Ut;    // float64 operand table of U^(1): Ut[c'][c] = U_(c,c')
  int N, Np, d, DP, logn, ND, dlo, periodic;
  double *Mr, *Mi;     // [ND][n/2 + 1][DP][DP]
};

// grid (ND, DP): one workgroup per (delta, c) transforms the kernels of every c'.
__global__ __launch_bounds__(256) void lam_param_kernel(LamParamArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = 1 << a.logn, nh = n / 2 + 1, ld = n + 1;
  const int nseq = max(1, min(a.DP, 4096 >> a.logn));
  double* xr = reinterpret_cast<double*>(smem_raw);
  double* xi = xr + nseq * ld;
  double* twr = xi + nseq * ld;
  double* twi = twr + n / 2;
  const int di = blockIdx.x, c = blockIdx.y, delta = a.dlo + di;
  const int TS = tap_stride(a.Np), TO = tap_off(a.Np);
  const double* g2 = a.taps + ((long)a.DP + c) * TS + TO;
  fft_twiddles(twr, twi, a.logn);
  for (int cp0 = 0; cp0 < a.DP; cp0 += nseq) {
    const int ns = min(nseq, a.DP - cp0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < ns * n; idx += blockDim.x) {
      const int s = idx >> a.logn, q = idx & (n - 1), cp = cp0 + s;
      int u;
      bool ok;
      if (a.periodic) {
        u = q;
        ok = q < a.N;
      } else {  // u in [-(N-1), N-1] stored at u mod n
        u = q < a.N ? q : q - n;
        ok = q < a.N || q > n - a.N;
      }
      double v = 0.0;
      if (ok && c < a.d && cp < a.d) v = g2[delta - u] * a.Pq[(long)cp * TS + TO + u];
      const int p = s * ld + bitrev(q, a.logn);
      xr[p] = v;
      xi[p] = 0.0;
    }
    __syncthreads();
    fft_stages(xr, xi, twr, twi, a.logn, ld, ns, false);
    for (int idx = threadIdx.x; idx < ns * nh; idx += blockDim.x) {
      const int w = idx / ns, s = idx % ns, cp = cp0 + s;
      const double u1 = a.Ut[(long)cp * a.DP + c];
      const long o = (((long)di * nh + w) * a.DP + cp) * a.DP + c;
      a.Mr[o] = u1 * xr[s * ld + w];
      a.Mi[o] = -u1 * xi[s * ld + w];
    }
  }
}

// ---- per-sample construction
template <typename T> struct LamArgs {
  int N, Np, DP, logn, ND, periodic;
  int di0;            // first offset of this pass inside the parameter-only table
  int Bc;             // samples in this pass
  int chf;            // channels per transform workgroup (even)
  const T* chi1;      // block-1 gate of the pass's first sample [Bc][DP][Np]
  T *Xr, *Xi;         // [n/2 + 1][Bc][DP]
  const T *Mr, *Mi;   // [ND_table][n/2 + 1][DP][DP]
  T *Zr, *Zi;         // [ND][n/2 + 1][Bc][DP]
  T* lam;             // [Bc][N][ND][DP] (the pass's first sample)
};

// grid (Bc, DP / chf): the gate's channels of one sample, two real sequences per complex
// transform, X(omega) for omega = 0 .. n/2.
template <typename T> __global__ __launch_bounds__(256) void lam_fwd_kernel(LamArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int logn = a.logn, n = 1 << logn, nh = n / 2 + 1, ld = n + 1, np = a.chf / 2;
  T* xr = reinterpret_cast<T*>(smem_raw);
  T* xi = xr + np * ld;
  T* twr = xi + np * ld;
  T* twi = twr + n / 2;
  const int b = blockIdx.x, c0 = blockIdx.y * a.chf;
  const T* x = a.chi1 + (long)b * a.DP * a.Np;
  fft_twiddles(twr, twi, logn);
#pragma unroll 8
  for (int idx = threadIdx.x; idx < np * n; idx += blockDim.x) {
    const int p = idx >> logn, k = idx & (n - 1);
    int src;
    bool ok;
    if (a.periodic) {  // the gate extended periodically to 2N - 1 sites
      ok = k < 2 * a.N - 1;
      src = k < a.N ? k : k - a.N;
    } else {
      ok = k < a.N;
      src = k;
    }
    const int ca = c0 + 2 * p;
    const int q = p * ld + bitrev(k, logn);
    xr[q] = ok ? x[(long)ca * a.Np + src] : T(0);
    xi[q] = ok ? x[(long)(ca + 1) * a.Np + src] : T(0);
  }
  __syncthreads();
  fft_stages(xr, xi, twr, twi, logn, ld, np, false);
  // Z = X_a + i X_b: X_a(w) = (Z(w) + conj Z(n - w)) / 2, X_b(w) = (Z(w) - conj Z(n - w)) / (2i)
  for (int idx = threadIdx.x; idx < np * nh; idx += blockDim.x) {
    const int w = idx / np, p = idx % np, wm = (n - w) & (n - 1);
    const T ar = xr[p * ld + w], ai = xi[p * ld + w], br = xr[p * ld + wm], bi = xi[p * ld + wm];
    const long o = ((long)w * a.Bc + b) * a.DP + c0 + 2 * p;
    a.Xr[o] = (ar + br) * T(0.5);
    a.Xi[o] = (ai - bi) * T(0.5);
    a.Xr[o + 1] = (ai + bi) * T(0.5);
    a.Xi[o + 1] = (br - ar) * T(0.5);
  }
}

// grid (n/2 + 1, ceil(Bc / 64)): at one frequency, 64 samples x all output channels, for every
// offset: Z[delta][w][b][c] = sum_c' M[delta][w][c][c'] X[w][b][c'] (complex, four real
// matrix-core products per step). Operand B (the samples' spectra) stays in registers across
// the offsets; operand A is staged in LDS per offset.
template <typename T, int DP> __global__ __launch_bounds__(256) void lam_gemm_kernel(LamArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MT = DP / 16, KS = DP / 4, LDX = 64 + 1;
  T* xsr = reinterpret_cast<T*>(smem_raw);  // [DP][LDX]
  T* xsi = xsr + DP * LDX;
  T* msr = xsi + DP * LDX;                   // [DP][DP]
  T* msi = msr + DP * DP;
  const int nh = (1 << a.logn) / 2 + 1;
  const int w = blockIdx.x, b0 = blockIdx.y * 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 15, kq = lane >> 4;
  // every thread's share of the samples' spectra requested at once (64 DP / 256 per part)
  constexpr int XPT = 64 * DP / 256, MPT = DP * DP / 256;
  {
    T vr[XPT], vi[XPT];
#pragma unroll
    for (int k = 0; k < XPT; ++k) {
      const int idx = threadIdx.x + 256 * k;
      const int bl = idx / DP, cp = idx % DP, b = b0 + bl;
      const long o = ((long)w * a.Bc + (b < a.Bc ? b : 0)) * DP + cp;
      vr[k] = a.Xr[o];
      vi[k] = a.Xi[o];
    }
#pragma unroll
    for (int k = 0; k < XPT; ++k) {
      const int idx = threadIdx.x + 256 * k;
      const int bl = idx / DP, cp = idx % DP;
      const bool ok = b0 + bl < a.Bc;
      xsr[cp * LDX + bl] = ok ? vr[k] : T(0);
      xsi[cp * LDX + bl] = ok ? vi[k] : T(0);
    }
  }
  // the parameter-only operand of the next offset is requested while the current one is used
  T mr[MPT], mi[MPT];
  auto fetch_m = [&](int di) {
    const long mo = ((long)(a.di0 + di) * nh + w) * DP * DP;
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
      mr[k] = a.Mr[mo + threadIdx.x + 256 * k];
      mi[k] = a.Mi[mo + threadIdx.x + 256 * k];
    }
  };
  fetch_m(0);
  __syncthreads();
  T br[KS], bi[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    br[ks] = xsr[(4 * ks + kq) * LDX + 16 * wave + j];
    bi[ks] = xsi[(4 * ks + kq) * LDX + 16 * wave + j];
  }
  const int b = b0 + 16 * wave + j;
  for (int di = 0; di < a.ND; ++di) {
    __syncthreads();  // the previous offset's operand is consumed
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
      msr[threadIdx.x + 256 * k] = mr[k];
      msi[threadIdx.x + 256 * k] = mi[k];
    }
    __syncthreads();
    if (di + 1 < a.ND) fetch_m(di + 1);
    acc_t cr[MT], ci[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) cr[mt] = ci[mt] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const T ar = msr[(4 * ks + kq) * DP + 16 * mt + j], ai = msi[(4 * ks + kq) * DP + 16 * mt + j];
        cr[mt] = M::mma(ar, br[ks], cr[mt]);
        cr[mt] = M::mma(-ai, bi[ks], cr[mt]);
        ci[mt] = M::mma(ar, bi[ks], ci[mt]);
        ci[mt] = M::mma(ai, br[ks], ci[mt]);
      }
    if (b < a.Bc) {
      const long zo = (((long)di * nh + w) * a.Bc + b) * DP;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = 16 * mt + M::row(lane, r);
          a.Zr[zo + c] = cr[mt][r];
          a.Zi[zo + c] = ci[mt][r];
        }
    }
  }
}

// grid (Bc, ND, DP / chf): the inverse transforms of one sample and offset, two channels per
// complex transform (each spectrum extended by Hermitian symmetry), scaled by 1/n; sites
// z < N are written to lam[b][z][delta][c].
template <typename T> __global__ __launch_bounds__(256) void lam_inv_kernel(LamArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int logn = a.logn, n = 1 << logn, nh = n / 2 + 1, ld = n + 1, np = a.chf / 2;
  T* xr = reinterpret_cast<T*>(smem_raw);
  T* xi = xr + np * ld;
  T* twr = xi + np * ld;
  T* twi = twr + n / 2;
  const int b = blockIdx.x, di = blockIdx.y, c0 = blockIdx.z * a.chf;
  fft_twiddles(twr, twi, logn);
#pragma unroll 8
  for (int idx = threadIdx.x; idx < np * n; idx += blockDim.x) {
    const int w = idx / np, p = idx % np;
    const bool lo = w <= n / 2;
    const int ws = lo ? w : n - w;
    const long o = (((long)di * nh + ws) * a.Bc + b) * a.DP + c0 + 2 * p;
    const T z0r = a.Zr[o], z0i = a.Zi[o], z1r = a.Zr[o + 1], z1i = a.Zi[o + 1];
    // W = Z_a + i Z_b, with Z(w) = conj Z(n - w) above n/2
    const int q = p * ld + bitrev(w, logn);
    xr[q] = lo ? z0r - z1i : z0r + z1i;
    xi[q] = lo ? z0i + z1r : z1r - z0i;
  }
  __syncthreads();
  fft_stages(xr, xi, twr, twi, logn, ld, np, true);
  const T inv = T(1) / T(n);
  for (int idx = threadIdx.x; idx < np * a.N; idx += blockDim.x) {
    const int z = idx / np, p = idx % np;
    const long o = (((long)b * a.N + z) * a.ND + di) * a.DP + c0 + 2 * p;
    a.lam[o] = xr[p * ld + z] * inv;
    a.lam[o + 1] = xi[p * ld + z] * inv;
  }
}

// ---- per-flip update (one or two blocks): the per-sample operands beside the slice's
template <typename T> struct Flip12Args {
  const T* p0;          // [L][Bf][DP][Np]: V v0 of every block
  long fldB;            // Bf DP Np
  const T* T0;          // [Bf][2][DP][Np]: output link of the input change (h^(0))
  const T* T1;          // [Bf][2][DP][Np]: output link of block 1 (two blocks; one block: Wk)
  const T* lam;         // [tok][Bf][N][ND][DP]: pivot-0 link of block 2, per position in a token
  long lamk;            // elements between the positions' links
  int ND, dlo;
  const double* Om0;    // [B][2]
  double* logratio;     // [B][M_max] ([B][M_max][2] with a complex read-out)
  double* dom;          // nullable: [B][M_max][2] the output changes dOmega themselves
  int cplx;             // 1: complex read-out unit Omega_0 + i Omega_1
};

// One or two blocks in one kernel per group of flips: the slice recompute (slm_layers) keeps
// each flip's vertex changes in registers, and the per-flip update below follows on the same
// matrix-core columns (flip p, slice position t), so neither the vertex changes nor
// the cluster geometry go through HBM. Wave w owns channels 16 w .. 16 w + 15 of every
// product (U^(1); V^(2) and U^(2) for two blocks) with those weight rows in registers; the
// read-outs are summed per column over the wave's channels, then over waves and a flip's
// columns in LDS.
template <typename T, int DP, bool TWO, bool TOK = false>
__global__ __launch_bounds__(4 * DP) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1)))
void shallow_kernel(SliceArgs<T> A, Flip12Args<T> F) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int LF = TWO ? 2 : 1, NW = DP / 16;
  using M = Mma<T>;
  using acc_t = typename M::acc;
  const int N = A.N, Np = A.Np, wc = A.w_c;
  const int Wc = A.ext_max + 2 * LF * wc + 1;  // widest S_L of the launch
  const int P = slm_flips(Wc);
  const int lda = slm_lda(P, Wc, wc);
  T* ph = reinterpret_cast<T*>(smem_raw);      // [DP][SLM_LDC]
  T* ab = ph + DP * SLM_LDC;                   // [DP][lda]
  int* gs = reinterpret_cast<int*>(ab + DP * lda);
  // two blocks: block 2's mixer taps at the offsets S_2 - S_1 takes, [DP][TW] from offset g_lo
  const int W1m = A.ext_max + 2 * wc + 1, W2m = W1m + 2 * wc;  // column strides of S_1, S_2
  const int TW = W1m + W2m - 1, g_lo = -wc - (W1m - 1);
  T* g2s = reinterpret_cast<T*>(gs + SLM_GS * P);
  const int nfl = A.dyn.count(A.F);
  const int fg = slm_group() * P;
  if (fg >= nfl) return;
  const int f0 = A.dyn.first(A.f0);
  const int TS = tap_stride(Np), TO = tap_off(Np);
  if constexpr (TWO)
    for (int idx = threadIdx.x; idx < DP * TW; idx += blockDim.x)
      g2s[idx] = A.tb.taps[((long)DP + idx / TW) * TS + TO + g_lo + idx % TW];
  slm_geometry<TOK>(A, gs, P, fg, nfl, f0, false);
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, q = lane >> 4;
  T dch[LF][SLM_NT][4];
  slm_layers<T, DP, LF, TOK>(A, ph, ab, gs, P, lda, [&](int l, int n, int r, T v) { dch[l - 1][n][r] = v; });
  const bool per = A.periodic != 0;
  auto wrap = [&](int i) { if (per) { i %= N; if (i < 0) i += N; } return i; };
  auto inside = [&](int i) { return per || (i >= 0 && i < N); };
  const long fld = (long)DP * Np;
  T u1[DP / 4], v2[DP / 4], u2[DP / 4];
  slm_rows<T, DP>(A.tb.Ut, wave, lane, u1);
  if constexpr (TWO) {
    slm_rows<T, DP>(A.tb.Vt + (long)DP * DP, wave, lane, v2);
    slm_rows<T, DP>(A.tb.Ut + (long)DP * DP, wave, lane, u2);
  }
  // the lane's S_1 columns: x1 = dchi1 (p0^(1) + c_a Pq(i - z_a) + c_b Pq(i - z_b)) to LDS;
  // operands of all columns are requested first (addresses clamped to valid ones for columns
  // that hold no slice site; the Pq offsets t - w_c and t - w_c - ext stay in its margins)
  {
    T pv[SLM_NT][4], qa[SLM_NT][4], qb[SLM_NT][4];
    bool v1q[SLM_NT];
#pragma unroll
    for (int n = 0; n < SLM_NT; ++n) {
      const int j = 16 * n + col, p = j / W1m, t = j - p * W1m;
      const int* g = gs + SLM_GS * (p < P ? p : 0);
      const int s1u = g[1] - wc + t;
      v1q[n] = p < P && g[0] >= 0 && t < g[2] + 2 * wc + 1 && inside(s1u);
      const int s1 = v1q[n] ? wrap(s1u) : g[1];
      const T* p01 = F.p0 + (long)(g[0] >= 0 ? g[0] - A.b0 : 0) * fld + s1;
      // the unit-flip tables of the flipped spins' positions inside their tokens
      const int ka = TOK && g[3] >= 0 ? g[3] % A.tok : 0, kb = TOK && g[4] >= 0 ? g[4] % A.tok : ka;
      const T* pqa = A.tb.Pq + (long)ka * 4 * DP * TS;
      const T* pqb = A.tb.Pq + (long)kb * 4 * DP * TS;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long ch = 16 * wave + M::row(lane, r);
        pv[n][r] = p01[ch * Np];
        qa[n][r] = pqa[ch * TS + TO + t - wc];
        qb[n][r] = pqb[ch * TS + TO + t - wc - g[2]];
      }
    }
#pragma unroll
    for (int n = 0; n < SLM_NT; ++n) {
      const int j = 16 * n + col, p = j / W1m;
      const int* g = gs + SLM_GS * (p < P ? p : 0);
      const T ca = (T)g[6], cb = (T)g[7];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        ph[(16 * wave + M::row(lane, r)) * SLM_LDC + j] =
            v1q[n] ? dch[0][n][r] * (pv[n][r] + ca * qa[n][r] + cb * qb[n][r]) : T(0);
    }
  }
  __syncthreads();
  // e1 = U^(1) x1; its read-out with T^(1) (one block: Wk), and e^(0) = c_z E at the cluster
  // sites with T^(0), per column
  double oa0[SLM_NT], oa1[SLM_NT];
  {
    acc_t e1[SLM_NT];
    slm_prod_n<T, DP>((P * W1m + 15) / 16, u1, ph, SLM_LDC, q, col, e1);
    // the read-out weights of all columns requested together (clamped addresses)
    T r0v[SLM_NT][4], r1v[SLM_NT][4];
    bool v1q[SLM_NT];
#pragma unroll
    for (int n = 0; n < SLM_NT; ++n) {
      const int j = 16 * n + col, p = j / W1m, t = j - p * W1m;
      const int* g = gs + SLM_GS * (p < P ? p : 0);
      const int s1u = g[1] - wc + t;
      v1q[n] = p < P && g[0] >= 0 && t < g[2] + 2 * wc + 1 && inside(s1u);
      const long bl = g[0] >= 0 ? g[0] - A.b0 : 0;
      const T* r0 = (TWO ? F.T1 + 2 * bl * fld : A.tb.Wk) + (v1q[n] ? wrap(s1u) : g[1]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long o = (long)(16 * wave + M::row(lane, r)) * Np;
        r0v[n][r] = r0[o];
        r1v[n][r] = r0[fld + o];
      }
    }
#pragma unroll
    for (int n = 0; n < SLM_NT; ++n) {
      oa0[n] = 0.0;
      oa1[n] = 0.0;
      const int j = 16 * n + col, p = j / W1m, t = j - p * W1m;
      const int* g = gs + SLM_GS * (p < P ? p : 0);
      if (v1q[n]) {
        T q0 = 0, q1 = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          q0 += r0v[n][r] * e1[n][r];
          q1 += r1v[n][r] * e1[n][r];
        }
        oa0[n] = (double)q0;
        oa1[n] = (double)q1;
        const int s1u = g[1] - wc + t;
        // e^(0) at the cluster's tokens: both flips may sit in one token
        const bool at_a = s1u == g[1], at_b = g[4] >= 0 && s1u == g[1] + g[2];
        if (at_a || at_b) {
          const T* t0 = F.T0 + 2 * (long)(g[0] - A.b0) * fld + wrap(s1u);
          const T* Ea = A.tb.E + (TOK ? g[3] % A.tok : 0) * DP;
          const T* Eb = A.tb.E + (TOK && g[4] >= 0 ? g[4] % A.tok : 0) * DP;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ch = 16 * wave + M::row(lane, r);
            double e = 0.0;
            if (at_a) e += (double)g[6] * (double)Ea[ch];
            if (at_b) e += (double)g[7] * (double)Eb[ch];
            oa0[n] += e * (double)t0[(long)ch * Np];
            oa1[n] += e * (double)t0[fld + (long)ch * Np];
          }
        }
      }
      if constexpr (TWO) {
#pragma unroll
        for (int r = 0; r < 4; ++r) ab[(16 * wave + M::row(lane, r)) * lda + j] = e1[n][r];
      }
    }
  }
  double ob0[SLM_NT], ob1[SLM_NT];
#pragma unroll
  for (int n = 0; n < SLM_NT; ++n) { ob0[n] = 0.0; ob1[n] = 0.0; }
  if constexpr (TWO) {
    __syncthreads();
    // x2 = G^(2) e1 + Lam on S_2: thread (channel c, part k) takes columns k, k + 4, ...
    // The mixer taps g2(s2 - s1) = g2(t2 - w_c - u) depend on the slice positions only; the
    // link rows of four columns are requested together (offsets t2 + ext_max - ext from dlo
    // lie inside [0, ND) for every column of the widest slice).
    {
      const int c = tid % DP, part = tid / DP;
      const T* g2c = g2s + c * TW - g_lo;  // g2c[r] = tap r of channel c
      const int ncol = P * W2m;
      for (int j0 = part; j0 < ncol; j0 += 16) {
        T la[4], lb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j2 = j0 + 4 * i;
          const int p = j2 / W2m, t2 = j2 - p * W2m;
          const int* g = gs + SLM_GS * (j2 < ncol ? p : 0);
          const long bl = g[0] >= 0 ? g[0] - A.b0 : 0;
          const int ka = TOK && g[3] >= 0 ? g[3] % A.tok : 0, kb = TOK && g[4] >= 0 ? g[4] % A.tok : ka;
          const T* lamb = F.lam + bl * N * F.ND * DP + c;
          la[i] = lamb[ka * F.lamk + ((long)g[1] * F.ND + (t2 - 2 * wc - F.dlo)) * DP];
          lb[i] = lamb[kb * F.lamk + ((long)wrap(g[1] + g[2]) * F.ND + (t2 - 2 * wc - g[2] - F.dlo)) * DP];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j2 = j0 + 4 * i;
          if (j2 >= ncol) break;
          const int p = j2 / W2m, t2 = j2 - p * W2m;
          const int* g = gs + SLM_GS * p;
          const int s2u = g[1] - 2 * wc + t2;
          T x = 0;
          if (g[0] >= 0 && t2 < g[2] + 4 * wc + 1 && inside(s2u)) {
            const int W1 = g[2] + 2 * wc + 1;
            const T* g2 = g2c + t2 - wc;
            const T* e1c = ab + c * lda + p * W1m;
            for (int u = 0; u < W1; ++u) x += g2[-u] * e1c[u];
            x += (T)g[6] * la[i];
            if (g[4] >= 0) x += (T)g[7] * lb[i];
          }
          ph[c * SLM_LDC + j2] = x;
        }
      }
    }
    __syncthreads();
    // q2 = V^(2) x2; x = dchi2 (p0^(2) + q2) to LDS (over e1, whose readers are done). The
    // operands of all columns are requested before the products (clamped addresses).
    {
      bool v2q[SLM_NT];
      int s2q[SLM_NT];
      T p2v[SLM_NT][4];
#pragma unroll
      for (int n = 0; n < SLM_NT; ++n) {
        const int j = 16 * n + col, p = j / W2m, t = j - p * W2m;
        const int* g = gs + SLM_GS * (p < P ? p : 0);
        const int s2u = g[1] - 2 * wc + t;
        v2q[n] = p < P && g[0] >= 0 && t < g[2] + 4 * wc + 1 && inside(s2u);
        s2q[n] = v2q[n] ? wrap(s2u) : g[1];
        const T* p02 = F.p0 + F.fldB + (long)(g[0] >= 0 ? g[0] - A.b0 : 0) * fld + s2q[n];
#pragma unroll
        for (int r = 0; r < 4; ++r) p2v[n][r] = p02[(long)(16 * wave + M::row(lane, r)) * Np];
      }
      acc_t q2[SLM_NT];
      slm_prod_n<T, DP>((P * W2m + 15) / 16, v2, ph, SLM_LDC, q, col, q2);
#pragma unroll
      for (int n = 0; n < SLM_NT; ++n) {
        const int j = 16 * n + col;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ab[(16 * wave + M::row(lane, r)) * lda + j] = v2q[n] ? dch[LF - 1][n][r] * (p2v[n][r] + q2[n][r]) : T(0);
      }
      T w0v[SLM_NT][4], w1v[SLM_NT][4];
#pragma unroll
      for (int n = 0; n < SLM_NT; ++n) {
        const T* w0 = A.tb.Wk + s2q[n];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long o = (long)(16 * wave + M::row(lane, r)) * Np;
          w0v[n][r] = w0[o];
          w1v[n][r] = w0[fld + o];
        }
      }
      __syncthreads();
      // e2 = U^(2) x, read out with Wk on S_2
      acc_t e2[SLM_NT];
      slm_prod_n<T, DP>((P * W2m + 15) / 16, u2, ab, lda, q, col, e2);
#pragma unroll
      for (int n = 0; n < SLM_NT; ++n) {
        if (v2q[n]) {
          T q0 = 0, q1 = 0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            q0 += w0v[n][r] * e2[n][r];
            q1 += w1v[n][r] * e2[n][r];
          }
          ob0[n] = (double)q0;
          ob1[n] = (double)q1;
        }
      }
    }
  }
  // column sums over the wave's channels (lanes 16 and 32 apart share a column), then over the
  // waves and each flip's columns; red[layout][output][wave][column]
  __syncthreads();
  double* red = reinterpret_cast<double*>(ph);
#pragma unroll
  for (int n = 0; n < SLM_NT; ++n) {
    const double a0 = swap_sum<32>(swap_sum<16>(oa0[n])), a1 = swap_sum<32>(swap_sum<16>(oa1[n]));
    const double b0 = swap_sum<32>(swap_sum<16>(ob0[n])), b1 = swap_sum<32>(swap_sum<16>(ob1[n]));
    if (lane < 16) {
      const int j = 16 * n + lane;
      red[(0 * NW + wave) * SLM_CAP + j] = a0;
      red[(1 * NW + wave) * SLM_CAP + j] = a1;
      red[(2 * NW + wave) * SLM_CAP + j] = b0;
      red[(3 * NW + wave) * SLM_CAP + j] = b1;
    }
  }
  __syncthreads();
  if (tid < P) {
    const int* g = gs + SLM_GS * tid;
    if (g[0] >= 0) {
      double s0 = 0.0, s1 = 0.0;
      for (int w = 0; w < NW; ++w) {
        for (int t = 0; t < W1m; ++t) {
          s0 += red[(0 * NW + w) * SLM_CAP + tid * W1m + t];
          s1 += red[(1 * NW + w) * SLM_CAP + tid * W1m + t];
        }
        if (TWO)
          for (int t = 0; t < W2m; ++t) {
            s0 += red[(2 * NW + w) * SLM_CAP + tid * W2m + t];
            s1 += red[(3 * NW + w) * SLM_CAP + tid * W2m + t];
          }
      }
      const int gg = f0 + g[5];
      const int bg = A.map.cb[gg], mm = A.map.cm[gg];
      const long o = (long)bg * A.map.M_max + mm;
      put_ratio(F.logratio, o, F.Om0[2 * bg], F.Om0[2 * bg + 1], s0, s1, F.cplx);
      if (F.dom) { F.dom[2 * o] = s0; F.dom[2 * o + 1] = s1; }
    }
  }
}

}  // namespace dn
