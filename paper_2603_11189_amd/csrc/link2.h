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
// Per flip (flip12_kernel) only slice-sized work remains:
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

// In-place radix-2 decimation-in-time transforms of nseq complex sequences of length n = 2^logn
// held in LDS at row stride ld, already in bit-reversed order. Forward: sum_k x_k w^(jk);
// inverse: the conjugate twiddles (unscaled). Ends with a workgroup barrier.
template <typename T>
__device__ void fft_stages(T* xr, T* xi, const T* twr, const T* twi, int logn, int ld, int nseq, bool inverse) {
  const int hn = 1 << (logn - 1);
  for (int ls = 1; ls <= logn; ++ls) {
    const int half = 1 << (ls - 1), sh = logn - ls;
    for (int idx = threadIdx.x; idx < nseq * hn; idx += blockDim.x) {
      const int s = idx >> (logn - 1), b = idx & (hn - 1);
      const int k = b & (half - 1), grp = b >> (ls - 1);
      const int i = s * ld + (grp << ls) + k, jj = i + half;
      const T wr = twr[k << sh];
      const T wi = inverse ? -twi[k << sh] : twi[k << sh];
      const T xjr = xr[jj], xji = xi[jj];
      const T tr = wr * xjr - wi * xji, ti = wr * xji + wi * xjr;
      const T ur = xr[i], ui = xi[i];
      xr[i] = ur + tr;
      xi[i] = ui + ti;
      xr[jj] = ur - tr;
      xi[jj] = ui - ti;
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
  for (int idx = threadIdx.x; idx < 64 * DP; idx += blockDim.x) {
    const int bl = idx / DP, cp = idx % DP, b = b0 + bl;
    const long o = ((long)w * a.Bc + b) * DP + cp;
    xsr[cp * LDX + bl] = b < a.Bc ? a.Xr[o] : T(0);
    xsi[cp * LDX + bl] = b < a.Bc ? a.Xi[o] : T(0);
  }
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
    const long mo = ((long)(a.di0 + di) * nh + w) * DP * DP;
    for (int idx = threadIdx.x; idx < DP * DP; idx += blockDim.x) {
      msr[idx] = a.Mr[mo + idx];
      msi[idx] = a.Mi[mo + idx];
    }
    __syncthreads();
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

// ---- per-flip update (one or two blocks)
template <typename T> struct Flip12Args {
  Tables<T> tb;
  int N, Np, L, w_c, periodic;
  int F, f0, b0;        // flips [f0, f0 + F) of the work list; b0: first sample of the background chunk
  CfgMap map;
  const int8_t* spins;
  const int4* geom;     // [F] (clo, ext, j0, j1) from slice_kernel
  const T* dchi;        // [F][L][Wmax][DP]
  int Wmax;
  int colw;             // matrix-core columns per flip (the widest last slice); 16 / colw flips per step
  const T* p0;          // [L][Bf][DP][Np]: V v0 of every block
  long fldB;            // Bf DP Np
  const T* T0;          // [Bf][2][DP][Np]: output link of the input change (h^(0))
  const T* T1;          // [Bf][2][DP][Np]: output link of block 1 (two blocks; one block: Wk)
  const T* lam;         // [Bf][N][ND][DP]: pivot-0 link of block 2
  int ND, dlo;
  const double* Om0;    // [B][2]
  double* logratio;     // [B][M_max]
  double* dom;          // nullable: [B][M_max][2] the output changes dOmega themselves
  DynRange dyn;
};

// waves per workgroup (they share one copy of the weight operands in LDS)
template <typename T> constexpr int flip12_waves() { return sizeof(T) == 4 ? 8 : 4; }
template <typename T, int DP> constexpr size_t flip12_lds_bytes(bool two) {
  return ((two ? 3 : 1) * DP * DP + (two ? flip12_waves<T>() * DP * 17 : 0)) * sizeof(T) +
         (size_t)flip12_waves<T>() * 32 * sizeof(double);
}

// Persistent workgroups; the weight operands live in LDS in fragment order. A wave takes
// 16 / colw flips at a time: flip p of the step owns matrix-core columns p colw .. p colw +
// colw - 1, column t of them being slice position t, so one product serves several flips.
template <typename T, int DP, bool TWO>
__global__ __launch_bounds__(64 * flip12_waves<T>()) void flip12_kernel(Flip12Args<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MT = DP / 16, KS = DP / 4, NW = flip12_waves<T>();
  T* FU1 = reinterpret_cast<T*>(smem_raw);  // [KS][64][MT]: operand A of U^(1)
  T* FV2 = FU1 + DP * DP;                   // [KS][64][MT]: operand A of V^(2)
  T* FU2 = FV2 + DP * DP;                   // [MT][MT][64][4]: U^(2) in accumulator channel order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 15, kq = lane >> 4;
  T* E1s = FU1 + (TWO ? 3 : 1) * DP * DP + wave * DP * 17;  // [DP][17]: this wave's e1 (TWO)
  double* red = reinterpret_cast<double*>(FU1 + (TWO ? 3 * DP * DP + NW * DP * 17 : DP * DP)) + wave * 32;
  for (int idx = threadIdx.x; idx < DP * DP; idx += blockDim.x) {
    const int mt = idx % MT, ln = (idx / MT) % 64, ks = idx / (MT * 64);
    FU1[idx] = A.tb.Ut[(4 * ks + (ln >> 4)) * DP + 16 * mt + (ln & 15)];
    if constexpr (TWO) {
      FV2[idx] = A.tb.Vt[(long)DP * DP + (4 * ks + (ln >> 4)) * DP + 16 * mt + (ln & 15)];
      const int r = idx & 3, l2 = (idx >> 2) & 63, mi = (idx >> 8) % MT, mo = (idx >> 8) / MT;
      FU2[idx] = A.tb.Ut[(long)DP * DP + (16 * mi + M::row(l2, r)) * DP + 16 * mo + (l2 & 15)];
    }
  }
  __syncthreads();
  const int N = A.N, Np = A.Np, wc = A.w_c;
  const int TS = tap_stride(Np), TO = tap_off(Np);
  const int F = A.dyn.count(A.F);
  const int cfg0 = A.dyn.first(A.f0);
  const int W = A.colw, P = 16 / W;
  const int p = j / W, t = j - p * W;  // this lane's flip slot and slice position
  auto wrap = [&](int i) { if (A.periodic) { i %= N; if (i < 0) i += N; } return i; };
  for (int gb = (blockIdx.x * NW + wave) * P; gb < F; gb += gridDim.x * NW * P) {
    const int g = gb + p;
    const bool have = p < P && g < F;
    int4 sg = make_int4(0, 0, 0, -1);
    int bglob = 0, bl = 0;
    if (have) {
      sg = A.geom[g];
      bglob = A.map.cb[cfg0 + g];
      bl = bglob - A.b0;
    }
    const int8_t* sp = A.spins + (long)bglob * N;
    // cluster sites (unwrapped): za = clo, zb = clo + ext for a pair
    const int za = sg.x, zb = sg.x + sg.y;
    const bool pair = sg.w >= 0;
    const T ca = have ? (T)(-2 * sp[za]) : T(0);
    const T cb = have && pair ? (T)(-2 * sp[wrap(zb)]) : T(0);
    // ---- block 1 on S_1
    const int lo1 = sg.x - wc, W1 = sg.y + 2 * wc + 1;
    const int s1u = lo1 + t;
    const bool v1 = have && t < W1 && (A.periodic || (s1u >= 0 && s1u < N));
    const int s1 = v1 ? wrap(s1u) : 0;
    const T* dchi1 = A.dchi + (long)(have ? g : 0) * A.L * A.Wmax * DP;
    const T* p01 = A.p0 + (long)bl * DP * Np;
    acc_t e1[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) e1[mt] = acc_t{0, 0, 0, 0};
#pragma unroll 4
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + kq;
      T x = 0;
      if (v1) {
        const T* pq = A.tb.Pq + (long)c * TS + TO + s1u;
        x = dchi1[t * DP + c] * (p01[(long)c * Np + s1] + ca * pq[-za] + cb * pq[-zb]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) e1[mt] = M::mma(FU1[(ks * 64 + lane) * MT + mt], x, e1[mt]);
      // keep the scheduler from hoisting every later operand load (register pressure)
      if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    // read-outs: a lane's partial over its channels in the field precision, float64 across
    // lanes and stages
    double o0 = 0.0, o1 = 0.0;
    if (v1) {
      const T* r0 = TWO ? A.T1 + (long)2 * bl * DP * Np : A.tb.Wk;
      const T* r1 = r0 + (long)DP * Np;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        T q0 = 0, q1 = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = (16 * mt + M::row(lane, r)) * Np + s1;
          q0 += r0[o] * e1[mt][r];
          q1 += r1[o] * e1[mt][r];
        }
        o0 += (double)q0;
        o1 += (double)q1;
      }
    }
    if constexpr (TWO) {
      // e1 to LDS, then x2 = G^(2) e1 + pivot-0 link on S_2 in operand-B layout
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) E1s[(16 * mt + M::row(lane, r)) * 17 + j] = e1[mt][r];
      wave_sync();
      const int lo2 = sg.x - 2 * wc, W2 = sg.y + 4 * wc + 1;
      const int s2u = lo2 + t;
      const bool v2 = have && t < W2 && (A.periodic || (s2u >= 0 && s2u < N));
      const int s2 = v2 ? wrap(s2u) : 0;
      const T* lamb = A.lam + (long)bl * N * A.ND * DP;
      const T* la = lamb + ((long)za * A.ND + (s2u - za - A.dlo)) * DP;
      const T* lb = lamb + ((long)wrap(zb) * A.ND + (s2u - zb - A.dlo)) * DP;
      const T* e1c = E1s + p * W;  // this flip's columns of e1
      acc_t q2[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) q2[mt] = acc_t{0, 0, 0, 0};
#pragma unroll 4
      for (int ks = 0; ks < KS; ++ks) {
        const int c = 4 * ks + kq;
        T x = 0;
        if (v2) {
          const T* g2 = A.tb.taps + ((long)DP + c) * TS + TO + s2u - lo1;
          for (int u = 0; u < W1; ++u) x += g2[-u] * e1c[c * 17 + u];
          x += ca * la[c];
          if (pair) x += cb * lb[c];
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) q2[mt] = M::mma(FV2[(ks * 64 + lane) * MT + mt], x, q2[mt]);
        if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
      // x = dchi2 * (p0^(2) + V x2), in accumulator order
      const T* dchi2 = dchi1 + (long)A.Wmax * DP;
      const T* p02 = A.p0 + A.fldB + (long)bl * DP * Np;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = 16 * mt + M::row(lane, r);
          q2[mt][r] = v2 ? dchi2[t * DP + c] * (p02[(long)c * Np + s2] + q2[mt][r]) : T(0);
        }
      const T* w0 = A.tb.Wk;
      const T* w1 = w0 + (long)DP * Np;
#pragma unroll 1
      for (int mo = 0; mo < MT; ++mo) {
        acc_t e2 = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int mi = 0; mi < MT; ++mi)
#pragma unroll
          for (int r = 0; r < 4; ++r) e2 = M::mma(FU2[((mo * MT + mi) * 64 + lane) * 4 + r], q2[mi][r], e2);
        if (v2) {
          T q0 = 0, q1 = 0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int o = (16 * mo + M::row(lane, r)) * Np + s2;
            q0 += w0[o] * e2[r];
            q1 += w1[o] * e2[r];
          }
          o0 += (double)q0;
          o1 += (double)q1;
        }
      }
    }
    // the input change e^(0) = c_z E at the cluster sites, read out with T^(0): the lanes of
    // a flip's first column take the channels 4 ks + kq
    if (have && t == 0) {
      const T* t0 = A.T0 + (long)2 * bl * DP * Np;
      const int zbw = wrap(zb);
#pragma unroll 4
      for (int ks = 0; ks < KS; ++ks) {
        const int c = 4 * ks + kq;
        const double e = (double)A.tb.E[c];
        const long oa = (long)c * Np + za, ob = (long)c * Np + zbw;
        o0 += e * ((double)ca * (double)t0[oa] + (double)cb * (double)t0[ob]);
        o1 += e * ((double)ca * (double)t0[(long)DP * Np + oa] + (double)cb * (double)t0[(long)DP * Np + ob]);
      }
    }
    // column sums (lanes 16 and 32 apart share a column), then each flip's columns
    o0 = swap_sum<32>(swap_sum<16>(o0));
    o1 = swap_sum<32>(swap_sum<16>(o1));
    if (lane < 16) { red[lane] = o0; red[16 + lane] = o1; }
    wave_sync();
    if (lane < P && gb + lane < F) {
      double s0 = 0.0, s1v = 0.0;
      for (int u = 0; u < W; ++u) { s0 += red[lane * W + u]; s1v += red[16 + lane * W + u]; }
      const int gg = gb + lane;
      const int bg = A.map.cb[cfg0 + gg], mm = A.map.cm[cfg0 + gg];
      const long o = (long)bg * A.map.M_max + mm;
      A.logratio[o] = lcd_d(A.Om0[2 * bg], s0) + lcd_d(A.Om0[2 * bg + 1], s1v);
      if (A.dom) { A.dom[2 * o] = s0; A.dom[2 * o + 1] = s1v; }
    }
    wave_sync();  // red and E1s are rewritten by the wave's next step
  }
}

}  // namespace dn
