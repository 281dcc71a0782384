// Per-sample log-derivatives O_theta(s) = d log psi(s) / d theta (reverse mode, hand written).
//
// The forward stores layer-boundary checkpoints (phi^(l), h^(l)) and the residual sum R; the
// backward walks the blocks from L down to 1, recomputing each block from its checkpoint and
// propagating adjoints through the vertex/mixing products (mixbwd_kernel), the Green's-function
// mixer (conv with reversed taps) and the phi stream (phibwd_kernel). Weight gradients of one
// sample are contractions over sites of two of its fields (outer_kernel, rowdot_kernel); the
// Green's-function taps get per-sample correlations (tapgrad_kernel), and the S4 parameters
// follow through the tap Jacobian dg/dtheta_S4, which is shared by all samples (s4jac_*).
#pragma once
#include "common.h"
#include "kernels.h"
#include "s4gen.h"

namespace dn {

// ------------------------------------------------------------------------------------------
// Backward of the vertex + channel mixing of block l, per configuration (one workgroup,
// one wave per 64-site block as in mix_kernel):
//   dh = du_next + dOmega_0 Wk_0 + dOmega_1 Wk_1       (read-out adjoint enters every block)
//   dx = U^T dh;  dq = chi * dx;  dchi = q * dx;  dv = V^T dq
template <typename T> struct MixBwdArgs {
  const T *Um, *Vm;       // operand tables of U^T and V^T for this block
  const T* Wk;            // [2][DP][Np]
  int N, Np;
  const T* du_next;       // nullable (last block)
  const double* dOm;      // [C][2]
  const T *chi, *q;       // recomputed block fields
  T *dh, *dq, *dchi, *dv; // outputs
};

template <typename T, int DP>
__global__ __launch_bounds__(512) void mixbwd_kernel(MixBwdArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MT = DP / 16, KS = DP / 4;
  const int g = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int N = A.N, Np = A.Np;
  const int j = lane & 15, kq = lane >> 4;
  T* xs = reinterpret_cast<T*>(smem_raw) + wave * DP * MIX_XS;
  const long fo = (long)g * DP * Np;
  const int s0 = 64 * wave + 4 * j;
  const T d0 = (T)A.dOm[2 * g], d1 = (T)A.dOm[2 * g + 1];
  acc_t acc[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[mt][n] = acc_t{0, 0, 0, 0};
#pragma unroll 4
  for (int ks = 0; ks < KS; ++ks) {
    const int kc = 4 * ks + kq;
    const long o = (long)kc * Np + s0;
    V4<T> w0 = ld4(A.Wk + o), w1 = ld4(A.Wk + (long)DP * Np + o);
    T bv[4];
    if (A.du_next) {
      V4<T> u = ld4(A.du_next + fo + o);
#pragma unroll
      for (int n = 0; n < 4; ++n) bv[n] = u.v[n] + d0 * w0.v[n] + d1 * w1.v[n];
    } else {
#pragma unroll
      for (int n = 0; n < 4; ++n) bv[n] = d0 * w0.v[n] + d1 * w1.v[n];
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) if (s0 + n >= N) bv[n] = T(0);
    st4(A.dh + fo + o, bv);
    T af[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) af[mt] = A.Um[kc * DP + 16 * mt + j];
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt][n] = M::mma(af[mt], bv[n], acc[mt][n]);
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ch = 16 * mt + M::row(lane, r);
      const long o = fo + (long)ch * Np + s0;
      V4<T> c = ld4(A.chi + o), q = ld4(A.q + o);
      T dqv[4], dcv[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const T dx = (s0 + n < N) ? acc[mt][n][r] : T(0);
        dqv[n] = c.v[n] * dx;
        dcv[n] = q.v[n] * dx;
      }
      st4(A.dq + o, dqv);
      st4(A.dchi + o, dcv);
      st4(xs + ch * MIX_XS + 4 * j, dqv);
    }
  wave_sync();
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[mt][n] = acc_t{0, 0, 0, 0};
#pragma unroll 4
  for (int ks = 0; ks < KS; ++ks) {
    const int kc = 4 * ks + kq;
    V4<T> v = ld4(xs + kc * MIX_XS + 4 * j);
    T af[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) af[mt] = A.Vm[kc * DP + 16 * mt + j];
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt][n] = M::mma(af[mt], v.v[n], acc[mt][n]);
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ch = 16 * mt + M::row(lane, r);
      T y[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) y[n] = (s0 + n < N) ? acc[mt][n][r] : T(0);
      st4(A.dv + fo + (long)ch * Np + s0, y);
    }
}

// ------------------------------------------------------------------------------------------
// Backward of the phi stream of block l, per configuration (one workgroup, 4 waves):
//   dzeta = dchi * g'(zeta);  dphi = A_D^T dzeta + dphi_next (+ du^(l) with phi injected into
//   the mixer input u^(l) = h^(l-1) + phi^(l), Fig. 1c);  dz = dphi * g'(z)
//   da_i = sum_r K_r * dz_{i-r};  dphi_prev = W_D^T da
template <typename T> struct PhiBwdArgs {
  const T *ADm, *WDm;      // operand tables of A_D^T, W_D^T for this block
  const T* Kc;             // [2w_c+1][DP]
  int N, Np, w_c, periodic, act;
  const T *dchi, *zeta, *z, *dphi_next;  // dphi_next nullable
  T *dzeta, *dz, *da, *dphi_prev;        // dphi_prev nullable
  const T* dphi_inj;                     // nullable: phi injected, the gradient of the mixer input u^(l)
};

template <typename T> __device__ inline T act_grad(int act, T x) {
  if (act == 0) {  // SiLU: s (1 + x (1 - s))
    const T s = T(1) / (T(1) + exp(-x));
    return s * (T(1) + x * (T(1) - s));
  }
  if (act == 1) { const T t = tanh(x); return T(1) - t * t; }
  return T(1);
}

template <typename T, int DP, int NT>
__global__ __launch_bounds__(256) void phibwd_kernel(PhiBwdArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* zs = reinterpret_cast<T*>(smem_raw);  // dz with halo [DP][Np + 2w_c + 1]
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MT = DP / 16;
  const int g = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int N = A.N, Np = A.Np, wc = A.w_c;
  const int ld = Np + 2 * wc + 1;
  const long fo = (long)g * DP * Np;
  const int span = 16 * NT;
  {
    WFrag<T, DP> ad;
    ad.load(A.ADm, lane);
    for (int i0 = wave * span; i0 < Np; i0 += 4 * span) {
      acc_t acc[MT][NT];
      mix_tile<T, DP, NT>(ad, [&](int kc, int n) -> T {
        const int i = i0 + 16 * n + (lane & 15);
        const long o = fo + (long)kc * Np + i;
        const T dzt = (i < N) ? A.dchi[o] * act_grad<T>(A.act, A.zeta[o]) : T(0);
        A.dzeta[o] = dzt;
        return dzt;
      }, acc);
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int i = i0 + 16 * n + (lane & 15);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ch = 16 * mt + M::row(lane, r);
            const long o = fo + (long)ch * Np + i;
            T dphi = acc[mt][n][r] + (A.dphi_next ? A.dphi_next[o] : T(0)) + (A.dphi_inj ? A.dphi_inj[o] : T(0));
            T dzv = (i < N) ? dphi * act_grad<T>(A.act, A.z[o]) : T(0);
            A.dz[o] = dzv;
            zs[ch * ld + i + wc] = dzv;
          }
      }
    }
  }
  __syncthreads();
  if (wc > 0) {
    for (int idx = threadIdx.x; idx < DP * 2 * wc; idx += 256) {
      int c = idx / (2 * wc), h = idx % (2 * wc);
      int col, src;
      if (h < wc) { col = h; src = N - wc + h; }
      else { col = N + wc + (h - wc); src = h - wc; }
      zs[c * ld + col] = A.periodic ? zs[c * ld + src + wc] : T(0);
    }
  }
  __syncthreads();
  WFrag<T, DP> wd;
  wd.load(A.WDm, lane);
  for (int i0 = wave * span; i0 < Np; i0 += 4 * span) {
    acc_t acc[MT][NT];
    mix_tile<T, DP, NT>(wd, [&](int kc, int n) -> T {
      const int i = i0 + 16 * n + (lane & 15);
      T s = 0;
      if (i < N)
        for (int r = -wc; r <= wc; ++r) s += A.Kc[(r + wc) * DP + kc] * zs[kc * ld + i - r + wc];
      A.da[fo + (long)kc * Np + i] = s;
      return s;
    }, acc);
    if (A.dphi_prev) {
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int i = i0 + 16 * n + (lane & 15);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ch = 16 * mt + M::row(lane, r);
            A.dphi_prev[fo + (long)ch * Np + i] = (i < N) ? acc[mt][n][r] : T(0);
          }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Per-sample contraction over sites of two fields:
//   out[b][c][c'] = sum_i P[b][c][i] * Q[b][c'][i]   (c, c' < d), Q = Q1 * Q2 when Q2 is set,
// or Q[c'][i] = emb[c'] * s_i (spin embedding of block 1). The d x d result goes to
// grads[b*P + off + c*d + c'] (row-major, output index first, as the parameter vector).
template <typename T> struct OuterArgs {
  const T *P, *Q1, *Q2;
  const T* emb;           // spin-embedding mode when non-null
  const int8_t* spins;
  int b0;                 // first global sample of the chunk (spins)
  int N, Np, d, DP;
  T* grads;
  long Pn, off;
  int tok;                // spins per token: the embedding is sum_k emb[k][c] s(tok i + k)
};

template <typename T, int DP>
__global__ __launch_bounds__(256) void outer_kernel(OuterArgs<T> A) {
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MT = DP / 16;
  const int g = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int N = A.N, Np = A.Np, j = lane & 15, kq = lane >> 4;
  const long fo = (long)g * DP * Np;
  const int8_t* sp = A.spins ? A.spins + (long)(A.b0 + g) * N * A.tok : nullptr;
  // wave w owns output column tile nt = w % MT and row tiles mt; waves split the sites when MT < 4
  const int nt = wave % MT;
  const int sgrp = wave / MT, nsg = 4 / MT;  // site groups (1 for DP=64, 2 for 32, 4 for 16)
  acc_t acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = acc_t{0, 0, 0, 0};
  for (int k0 = 4 * sgrp; k0 < N; k0 += 4 * nsg) {
    const int i = k0 + kq;
    const int cq = 16 * nt + j;
    T bq = 0;
    if (i < N) {
      if (A.emb) {
        bq = A.emb[cq] * (T)sp[i * A.tok];
        for (int k = 1; k < A.tok; ++k) bq += A.emb[k * DP + cq] * (T)sp[i * A.tok + k];
      }
      else {
        bq = A.Q1[fo + (long)cq * Np + i];
        if (A.Q2) bq *= A.Q2[fo + (long)cq * Np + i];
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const T ap = (i < N) ? A.P[fo + (long)(16 * mt + j) * Np + i] : T(0);
      acc[mt] = M::mma(ap, bq, acc[mt]);
    }
  }
  __shared__ T red[4][DP / 16][4][64];
  if (nsg > 1) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][mt][r][lane] = acc[mt][r];
    __syncthreads();
    if (sgrp != 0) return;
    for (int s = 1; s < nsg; ++s)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mt][r] += red[wave + s * MT][mt][r][lane];
  }
  T* out = A.grads + (long)(g + 0) * A.Pn + A.off;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 16 * mt + M::row(lane, r), cp = 16 * nt + j;
      if (c < A.d && cp < A.d) out[(long)c * A.d + cp] = acc[mt][r];
    }
}

// ------------------------------------------------------------------------------------------
// Per-sample, per-channel sums over sites: out[c] = sum_i P[c][i] * Q(c, i + shift) with
// Q = 1 (plain sum), a field (open: zero outside the chain; periodic: wrap), or the spins.
// One wave per (sample, channel block); writes grads[b*P + off + shift_index*d + c].
template <typename T> struct RowdotArgs {
  const T* P;
  const T* Q;             // nullable: Q = 1
  const int8_t* spins;    // used when use_spins
  int use_spins, b0;
  int N, Np, d, DP, periodic;
  int shift0, nshift;     // shifts shift0 .. shift0+nshift-1
  T* grads;
  long Pn, off;
  int accumulate;
  const T* Wk;            // with dOm: P_eff = P + dOm_0 Wk_0 + dOm_1 Wk_1 (read-out adjoint)
  const double* dOm;
  int tok, kpos;          // use_spins: the spin at position kpos of each token (spins per token tok)
};

template <typename T>
__global__ __launch_bounds__(64) void rowdot_kernel(RowdotArgs<T> A) {
  const int g = blockIdx.x, c = blockIdx.y;
  const int lane = threadIdx.x;
  const int N = A.N, Np = A.Np;
  const long ro = ((long)g * A.DP + c) * Np;
  const int8_t* sp = A.use_spins ? A.spins + (long)(A.b0 + g) * N * A.tok + A.kpos : nullptr;
  const T d0 = A.dOm ? (T)A.dOm[2 * g] : T(0), d1 = A.dOm ? (T)A.dOm[2 * g + 1] : T(0);
  for (int si = 0; si < A.nshift; ++si) {
    const int sh = A.shift0 + si;
    T acc = 0;
    for (int i = lane; i < N; i += 64) {
      T q = 1;
      if (A.use_spins) q = (T)sp[i * A.tok];
      else if (A.Q) {
        int k = i + sh;
        if (A.periodic) { k %= N; if (k < 0) k += N; q = A.Q[ro + k]; }
        else q = (k >= 0 && k < N) ? A.Q[ro + k] : T(0);
      }
      T pv = A.P[ro + i];
      if (A.dOm) pv += d0 * A.Wk[(long)c * Np + i] + d1 * A.Wk[((long)A.DP + c) * Np + i];
      acc += pv * q;
    }
    acc = wave_sum(acc);
    if (lane == 0 && c < A.d) {
      T* o = A.grads + (long)g * A.Pn + A.off + (long)si * A.d + c;
      *o = A.accumulate ? *o + acc : acc;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Tap gradients of one block mixer, per (sample, channel): dg(r) = sum_i dv[i] u[i - r] for
// r in [-(N-1), N-1] (open chain). One workgroup per (sample, channel); the rows are staged in LDS.
template <typename T> struct TapGradArgs {
  const T *dv, *u;
  int N, Np, d, DP;
  T* dg;                  // [C][mixers][d][2N-1]
  int mixer, nmix;
};

template <typename T>
__global__ __launch_bounds__(256) void tapgrad_kernel(TapGradArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* a = reinterpret_cast<T*>(smem_raw);  // dv row
  T* u = a + A.Np;                         // u row
  const int g = blockIdx.x, c = blockIdx.y;
  const int N = A.N, Np = A.Np;
  const long ro = ((long)g * A.DP + c) * Np;
  for (int i = threadIdx.x; i < Np; i += 256) { a[i] = A.dv[ro + i]; u[i] = A.u[ro + i]; }
  __syncthreads();
  const int TG = 2 * N - 1;
  T* out = A.dg + (((long)g * A.nmix + A.mixer) * A.d + c) * TG;
  for (int q = threadIdx.x; q < TG; q += 256) {
    const int r = q - (N - 1);
    const int i0 = r > 0 ? r : 0, i1 = r > 0 ? N : N + r;  // i - r in [0, N)
    T s = 0;
    for (int i = i0; i < i1; ++i) s += a[i] * u[i - r];
    out[q] = s;
  }
}

// The off-block entries of U and V of a block-diagonal vertex are not parameters: their
// gradients (U then V, d x d each, from offU) are set to zero.
template <typename T>
__global__ void block_grad_mask_kernel(T* __restrict__ grads, int B, long Pn, long offU, int d, int dblk) {
  const long per = 2L * d * d, n = (long)B * per;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long b = i / per, e = i - b * per;
    const int mo = (int)(e % ((long)d * d)), r = mo / d, c = mo - r * d;
    if (r / dblk != c / dblk) grads[b * Pn + offU + e] = T(0);
  }
}

// ------------------------------------------------------------------------------------------
// Read-out gradients per sample: dOmega_k = tanh(Omega_k); rho_c = (1/N) sum_i omega_{i,c} R_{i,c};
// a complex read-out (one unit z = Omega_0 + i Omega_1, t = tanh z) has d log psi = t (dOmega_0 +
// i dOmega_1), so part 0 (the real part) seeds (Re t, -Im t) and part 1 (the imaginary part)
// (Im t, Re t); everything below is linear in the seed;
// dA[c][k] = rho_c dOmega_k; the final mixer enters only through omega_{i,c} = sum_j g^f_c(j - i),
// so dg^f_c(r) = sum_{i : 0 <= i + r < N} R_{i,c} drho_c / N with drho_c = sum_k A[c][k] dOmega_k.
template <typename T> struct ReadoutGradArgs {
  const T* R;             // [C][DP][Np]
  const double* Om;       // [C][2]
  const double* omega;    // [DP][Np]
  const double* A;        // [DP][2]
  int N, Np, d, DP, nmix;
  T* grads;
  long Pn, offA;
  T* dg;                  // [C][nmix][d][2N-1], final mixer = nmix-1
  double* dOm;            // [C][2] out
  int cplx, part;         // complex read-out; which part of log psi is differentiated
};

template <typename T>
__global__ __launch_bounds__(256) void readout_grad_kernel(ReadoutGradArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* pre = reinterpret_cast<double*>(smem_raw);  // prefix sums of R_{.,c}, [Np+1]
  const int g = blockIdx.x, c = blockIdx.y;
  const int N = A.N, Np = A.Np;
  double t0, t1;
  if (A.cplx) {
    double tr, ti;
    ctanh_d(A.Om[2 * g], A.Om[2 * g + 1], &tr, &ti);
    t0 = A.part ? ti : tr;
    t1 = A.part ? tr : -ti;
  } else {
    t0 = tanh(A.Om[2 * g]);
    t1 = tanh(A.Om[2 * g + 1]);
  }
  if (c == 0 && threadIdx.x == 0) { A.dOm[2 * g] = t0; A.dOm[2 * g + 1] = t1; }
  if (c >= A.d) return;
  const long ro = ((long)g * A.DP + c) * Np;
  // rho_c and the prefix sums of R over sites
  __shared__ double wsum[4];
  double part = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) part += A.omega[(long)c * Np + i] * (double)A.R[ro + i];
  part = wave_sum(part);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = part;
  if (threadIdx.x == 0) {
    double s = 0.0;
    pre[0] = 0.0;
    for (int i = 0; i < N; ++i) { s += (double)A.R[ro + i]; pre[i + 1] = s; }
  }
  __syncthreads();
  const double rho = (wsum[0] + wsum[1] + wsum[2] + wsum[3]) / N;
  const double drho = A.A[2 * c] * t0 + A.A[2 * c + 1] * t1;
  if (threadIdx.x == 0) {
    A.grads[(long)g * A.Pn + A.offA + 2 * c] = (T)(rho * t0);
    A.grads[(long)g * A.Pn + A.offA + 2 * c + 1] = (T)(rho * t1);
  }
  T* out = A.dg + (((long)g * A.nmix + (A.nmix - 1)) * A.d + c) * (2 * N - 1);
  for (int q = threadIdx.x; q < 2 * N - 1; q += 256) {
    const int r = q - (N - 1);
    const int i0 = r < 0 ? -r : 0, i1 = r < 0 ? N : N - r;  // 0 <= i + r < N
    out[q] = (T)((pre[i1] - pre[i0]) * drho / N);
  }
}

// ------------------------------------------------------------------------------------------
// S4 tap Jacobian (open chains), float64. For one mixer channel with A_d = M^-1 R, B_d = M^-1 Delta Bbar,
// M = I - Delta/2 Abar, R = I + Delta/2 Abar, X_r = A_d^r B_d, w+-_r = C+-^T A_d^r:
//  * C+- directions:  d g+-_r = Re(e_n . X_r) (x i for the imaginary part);
//  * Bbar directions: d X_r = A_d^r M^-1 Delta e_n, so d g+-_r = Re(Delta (w+-_r M^-1)_n) (x i);
//  * Lambda, p, q directions change Abar by a rank-one a b^T, so dA_d = alpha beta^T with
//    alpha = Delta/2 M^-1 a, beta^T = b^T (I + A_d), and dB_d = alpha (b^T B_d); then
//    d g+-_r = Re( sum_{k<r} (w+-_k . alpha)(beta^T X_{r-1-k}) + (w+-_r . alpha)(b^T B_d) );
//  * the step offset changes Delta (dDelta = Delta): dA_d = dDelta/2 M^-1 Abar (I + A_d),
//    dB_d = M^-1 (dDelta Bbar + dDelta/2 Abar B_d), propagated by dX_r = dA X_{r-1} + A dX_{r-1}.
// Layout: J[(mixer*d + c)][2N-1][12s+1] (tap offset r stored at r + N - 1), parameter order of
// the channel block: Lambda re/im, p re/im, q re/im, B re/im, C+ re/im, C- re/im, step.
struct S4Prep {
  double *Minv, *Ad, *Bd, *X, *Wp, *Wm, *Up, *Um;  // per channel: s*s, s*s, s, N*s, N*s, N*s, N*s, N*s (complex: x2)
};

__device__ inline long s4p_stride(int N, int s) { return 2L * (2 * s * s + s + 5 * (long)N * s); }

// One wave per (mixer, channel): M^-1, A_d, B_d, X_r, w+-_r, w+-_r M^-1 and the step direction.
__global__ __launch_bounds__(S4_THREADS) void s4jac_prep_kernel(const double* __restrict__ params, long s4_off,
                                                                int N, int d, int s, double* __restrict__ ws,
                                                                double* __restrict__ J) {
  __shared__ cx G[S4_SMAX * (2 * S4_SMAX + 1)];
  __shared__ cx Abar[S4_SMAX * S4_SMAX];
  __shared__ cx xa[S4_SMAX], xb[S4_SMAX], ya[S4_SMAX], yb[S4_SMAX], Cp[S4_SMAX], Cm[S4_SMAX], fac[S4_SMAX];
  __shared__ int piv_s;
  const int t = threadIdx.x;
  const int ch = blockIdx.x, c = ch % d;
  const int NP = 12 * s + 1;
  const double* p = params + s4_off + (long)ch * NP;
  const double delta = exp(log(1e-2) + log(10.0) * (double)c / (double)(d > 1 ? d - 1 : 1) + p[12 * s]);
  cx* base = reinterpret_cast<cx*>(ws + (long)ch * s4p_stride(N, s));
  cx* Minv = base;
  cx* Ad = Minv + s * s;
  cx* Bd = Ad + s * s;
  cx* X = Bd + s;
  cx* Wp = X + (long)N * s;
  cx* Wm = Wp + (long)N * s;
  cx* Up = Wm + (long)N * s;
  cx* Umm = Up + (long)N * s;
  const int ld = 2 * s + 1;
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx a = cmul(cx{p[2 * s + i], p[3 * s + i]}, cx{p[4 * s + jj], p[5 * s + jj]});
    if (i == jj) a = cadd(a, cx{-exp(p[i]), p[s + i]});
    Abar[i * S4_SMAX + jj] = a;
    cx h{0.5 * delta * a.re, 0.5 * delta * a.im};
    G[i * ld + jj] = cx{(i == jj ? 1.0 : 0.0) - h.re, -h.im};
    G[i * ld + s + jj] = cx{i == jj ? 1.0 : 0.0, 0.0};  // [M | I]
  }
  for (int i = t; i < s; i += S4_THREADS) {
    G[i * ld + 2 * s] = cx{0.0, 0.0};
    Cp[i] = cx{p[8 * s + i], p[9 * s + i]};
    Cm[i] = cx{p[10 * s + i], p[11 * s + i]};
  }
  __syncthreads();
  gauss_jordan(G, s, 2 * s, ld, fac, &piv_s);
  for (int idx = t; idx < s * s; idx += S4_THREADS) Minv[idx] = G[(idx / s) * ld + s + idx % s];
  __syncthreads();
  // A_d = M^-1 (I + Delta/2 Abar), B_d = M^-1 Delta Bbar
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) {
      cx r = Abar[k * S4_SMAX + jj];
      r = cx{0.5 * delta * r.re + (k == jj ? 1.0 : 0.0), 0.5 * delta * r.im};
      acc = cadd(acc, cmul(Minv[i * s + k], r));
    }
    Ad[idx] = acc;
  }
  for (int i = t; i < s; i += S4_THREADS) {
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(Minv[i * s + k], cx{delta * p[6 * s + k], delta * p[7 * s + k]}));
    Bd[i] = acc;
  }
  __threadfence_block();
  __syncthreads();
  // X_r (columns) and w+-_r (rows) by repeated products; u+-_r = w+-_r M^-1
  for (int i = t; i < s; i += S4_THREADS) { xa[i] = Bd[i]; ya[i] = Cp[i]; yb[i] = Cm[i]; }
  __syncthreads();
  for (int r = 0; r < N; ++r) {
    if (t < s) {
      X[(long)r * s + t] = xa[t];
      Wp[(long)r * s + t] = ya[t];
      Wm[(long)r * s + t] = yb[t];
      cx up{0.0, 0.0}, um{0.0, 0.0};
      for (int k = 0; k < s; ++k) { up = cadd(up, cmul(ya[k], Minv[k * s + t])); um = cadd(um, cmul(yb[k], Minv[k * s + t])); }
      Up[(long)r * s + t] = up;
      Umm[(long)r * s + t] = um;
    }
    __syncthreads();
    cx nx{0.0, 0.0}, np{0.0, 0.0}, nm{0.0, 0.0};
    if (t < s) {
      for (int k = 0; k < s; ++k) {
        nx = cadd(nx, cmul(Ad[t * s + k], xa[k]));
        np = cadd(np, cmul(ya[k], Ad[k * s + t]));
        nm = cadd(nm, cmul(yb[k], Ad[k * s + t]));
      }
    }
    __syncthreads();
    if (t < s) { xa[t] = nx; ya[t] = np; yb[t] = nm; }
    __syncthreads();
  }
  // step direction: dA = 1/2 M^-1 Abar (I + A_d) dDelta, dB = M^-1 (Bbar + 1/2 Abar B_d) dDelta, dDelta = Delta
  // G (free now) holds dA in its first s columns
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx acc{0.0, 0.0};  // (Abar (I + A_d))[i][jj]
    for (int k = 0; k < s; ++k) {
      cx ia = Ad[k * s + jj];
      if (k == jj) ia.re += 1.0;
      acc = cadd(acc, cmul(Abar[i * S4_SMAX + k], ia));
    }
    G[i * ld + s + jj] = acc;
  }
  __syncthreads();
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(Minv[i * s + k], G[k * ld + s + jj]));
    G[i * ld + jj] = cx{0.5 * delta * acc.re, 0.5 * delta * acc.im};
  }
  for (int i = t; i < s; i += S4_THREADS) {
    cx ab{0.0, 0.0};
    for (int k = 0; k < s; ++k) ab = cadd(ab, cmul(Abar[i * S4_SMAX + k], Bd[k]));
    fac[i] = cx{p[6 * s + i] + 0.5 * ab.re, p[7 * s + i] + 0.5 * ab.im};
  }
  __syncthreads();
  for (int i = t; i < s; i += S4_THREADS) {
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(Minv[i * s + k], fac[k]));
    xb[i] = cx{delta * acc.re, delta * acc.im};  // dX_0 = dB_d
  }
  __syncthreads();
  double* Jc = J + (long)ch * (2 * N - 1) * NP;
  for (int r = 0; r < N; ++r) {
    double gp = cdot_re(Cp, xb, s), gm = cdot_re(Cm, xb, s);
    if (t == 0) {
      Jc[(long)(N - 1 + r) * NP + 12 * s] = gp;
      if (r > 0) Jc[(long)(N - 1 - r) * NP + 12 * s] = gm;
    }
    cx nx{0.0, 0.0};
    if (t < s && r + 1 < N) {
      // dX_{r+1} = dA X_r + A_d dX_r
      for (int k = 0; k < s; ++k) nx = cadd(nx, cadd(cmul(G[t * ld + k], X[(long)r * s + k]), cmul(Ad[t * s + k], xb[k])));
    }
    __syncthreads();
    if (t < s) xb[t] = nx;
    __syncthreads();
  }
}

// One block per (mixer, channel, direction group): the C, Bbar and rank-one directions.
__global__ __launch_bounds__(256) void s4jac_dir_kernel(const double* __restrict__ params, long s4_off, int N, int d,
                                                        int s, const double* __restrict__ ws, double* __restrict__ J) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx* ap = reinterpret_cast<cx*>(smem_raw);  // [N] w+_k . alpha
  cx* am = ap + N;                            // [N] w-_k . alpha
  cx* cc = am + N;                            // [N] beta^T X_m
  __shared__ cx alpha[S4_SMAX], beta[S4_SMAX], avec[S4_SMAX], bvec[S4_SMAX];
  __shared__ cx beta0;
  const int t = threadIdx.x;
  const int ch = blockIdx.x, dir = blockIdx.y;  // dir in [0, 12s): param index within the channel block
  const int c = ch % d;
  const int NP = 12 * s + 1;
  const double* p = params + s4_off + (long)ch * NP;
  const double delta = exp(log(1e-2) + log(10.0) * (double)c / (double)(d > 1 ? d - 1 : 1) + p[12 * s]);
  const cx* base = reinterpret_cast<const cx*>(ws + (long)ch * s4p_stride(N, s));
  const cx* Minv = base;
  const cx* Ad = Minv + s * s;
  const cx* Bd = Ad + s * s;
  const cx* X = Bd + s;
  const cx* Wp = X + (long)N * s;
  const cx* Wm = Wp + (long)N * s;
  const cx* Up = Wm + (long)N * s;
  const cx* Umm = Up + (long)N * s;
  double* Jc = J + (long)ch * (2 * N - 1) * NP;
  const int grp = dir / s, n = dir % s;
  const bool imag = grp & 1;
  const int TG = 2 * N - 1;
  if (grp >= 8) {  // C+ (8,9) and C- (10,11): d g_r = Re(e_n X_r) or Re(i X_r[n]) = -Im
    const bool plus = grp < 10;
    for (int q = t; q < TG; q += 256) {
      const int r = q - (N - 1);
      double v = 0.0;
      if (plus && r >= 0) v = imag ? -X[(long)r * s + n].im : X[(long)r * s + n].re;
      if (!plus && r < 0) v = imag ? -X[(long)(-r) * s + n].im : X[(long)(-r) * s + n].re;
      Jc[(long)q * NP + dir] = v;
    }
    return;
  }
  if (grp >= 6) {  // Bbar (6,7): Re(Delta u_r[n]) or Re(i Delta u_r[n])
    for (int q = t; q < TG; q += 256) {
      const int r = q - (N - 1);
      const cx u = r >= 0 ? Up[(long)r * s + n] : Umm[(long)(-r) * s + n];
      Jc[(long)q * NP + dir] = imag ? -delta * u.im : delta * u.re;
    }
    return;
  }
  // rank-one directions: a b^T
  for (int i = t; i < s; i += 256) {
    cx a{0.0, 0.0}, b{0.0, 0.0};
    if (grp < 2) {          // Lambda_n: a = e_n dlambda, b = e_n
      if (i == n) { a = imag ? cx{0.0, 1.0} : cx{-exp(p[n]), 0.0}; b = cx{1.0, 0.0}; }
    } else if (grp < 4) {   // p_n: a = e_n (x i), b = q
      if (i == n) a = imag ? cx{0.0, 1.0} : cx{1.0, 0.0};
      b = cx{p[4 * s + i], p[5 * s + i]};
    } else {                // q_n: a = p, b = e_n (x i)
      a = cx{p[2 * s + i], p[3 * s + i]};
      if (i == n) b = imag ? cx{0.0, 1.0} : cx{1.0, 0.0};
    }
    avec[i] = a;
    bvec[i] = b;
  }
  __syncthreads();
  for (int i = t; i < s; i += 256) {
    cx al{0.0, 0.0}, be{0.0, 0.0};
    for (int k = 0; k < s; ++k) {
      al = cadd(al, cmul(Minv[i * s + k], avec[k]));
      cx ia = Ad[k * s + i];
      if (k == i) ia.re += 1.0;
      be = cadd(be, cmul(bvec[k], ia));  // (b^T (I + A_d))_i
    }
    alpha[i] = cx{0.5 * delta * al.re, 0.5 * delta * al.im};
    beta[i] = be;
  }
  if (t == 0) {
    cx b0{0.0, 0.0};
    for (int k = 0; k < s; ++k) b0 = cadd(b0, cmul(bvec[k], Bd[k]));
    beta0 = b0;
  }
  __syncthreads();
  for (int k = t; k < N; k += 256) {
    cx sp{0.0, 0.0}, sm{0.0, 0.0}, sc{0.0, 0.0};
    for (int i = 0; i < s; ++i) {
      sp = cadd(sp, cmul(Wp[(long)k * s + i], alpha[i]));
      sm = cadd(sm, cmul(Wm[(long)k * s + i], alpha[i]));
      sc = cadd(sc, cmul(beta[i], X[(long)k * s + i]));
    }
    ap[k] = sp; am[k] = sm; cc[k] = sc;
  }
  __syncthreads();
  for (int q = t; q < TG; q += 256) {
    const int r = q - (N - 1);
    const int rr = r >= 0 ? r : -r;
    const cx* a = r >= 0 ? ap : am;
    cx acc = cmul(a[rr], beta0);
    for (int k = 0; k < rr; ++k) acc = cadd(acc, cmul(a[k], cc[rr - 1 - k]));
    Jc[(long)q * NP + dir] = acc.re;
  }
}

// ------------------------------------------------------------------------------------------
// S4 tap Jacobian of periodic chains (the aliased kernel), float64:
//   g_p = Re(C+^T A_d^p Q B_d) + Re(C-^T A_d^(N-p) Q B_d),  Q = (I - A_d^N)^-1,  p = 0..N-1,
// stored at the Toeplitz rows r = p and r = p - N of the open layout (the kernel tables hold
// the circulant as a Toeplitz matrix with g_(r mod N) at offset r). Q is a function of A_d and
// commutes with it, so with Xt_m = A_d^m Q B_d, w+-_m = C+-^T A_d^m, wt+-_m = C+-^T Q A_d^m:
//  * C+- directions: Re(e_n . Xt_p), Re(e_n . Xt_(N-p));
//  * Bbar directions: d(Q B_d) = Q M^-1 Delta e_n, so d g_p = Re(Delta (wt+_p M^-1)_n) +
//    Re(Delta (wt-_(N-p) M^-1)_n);
//  * rank-one directions dA_d = alpha beta^T, dB_d = alpha b0 (b0 = b^T B_d): with
//    dQ = Q d(A_d^N) Q and c_m = beta^T Xt_m,
//      C^T d(A_d^j Q B_d) = sum_(k<j) (w_k.alpha) c_(j-1-k) + sum_(k<N) (wt_(j+k).alpha) c_(N-1-k)
//                           + (wt_j.alpha) b0,  j = p (C+) or N - p (C-);
//  * the step offset: the tangent of A_d^N Q B_d by the recurrence T_(j+1) = dA Xt_j + A_d T_j,
//    d(Q B_d) = Q (T_N + dB_d), dXt_(p+1) = dA Xt_p + A_d dXt_p.
__device__ inline long s4pp_stride(int N, int s) { return 2L * (4L * s * s + s + (long)s * (9L * N + 3)); }

struct S4PerPtr {
  cx *Minv, *Ad, *Q, *dA, *Bd, *Xt, *Wp, *Wm, *Wtp, *Wtm, *Utp, *Utm;
};
__device__ inline S4PerPtr s4pp_ptrs(double* ws, int ch, int N, int s) {
  S4PerPtr q;
  cx* b = reinterpret_cast<cx*>(ws + (long)ch * s4pp_stride(N, s));
  q.Minv = b; q.Ad = q.Minv + s * s; q.Q = q.Ad + s * s; q.dA = q.Q + s * s; q.Bd = q.dA + s * s;
  q.Xt = q.Bd + s;                      // [N+1][s]
  q.Wp = q.Xt + (long)(N + 1) * s;      // [N][s]
  q.Wm = q.Wp + (long)N * s;            // [N][s]
  q.Wtp = q.Wm + (long)N * s;           // [2N][s]
  q.Wtm = q.Wtp + 2L * N * s;           // [2N][s]
  q.Utp = q.Wtm + 2L * N * s;           // [N+1][s]
  q.Utm = q.Utp + (long)(N + 1) * s;    // [N+1][s]
  return q;
}

// Value v of direction k at circulant offset p, written to both Toeplitz rows.
__device__ inline void s4pp_put(double* Jc, int N, int NP, int p, int k, double v) {
  Jc[(long)(p + N - 1) * NP + k] = v;
  if (p >= 1) Jc[(long)(p - 1) * NP + k] = v;
}

// Static LDS of s4jacp_prep_kernel (its dynamic part is 2(N+1) doubles) and of the direction
// kernels s4jac_dir_kernel / s4jacp_dir_kernel (their dynamic part is 3N / 7N complex values).
constexpr size_t S4JACP_STATIC_LDS =
    sizeof(cx) * (S4_SMAX * (2 * S4_SMAX + 1) + 4 * S4_SMAX * S4_SMAX + 7 * S4_SMAX) + sizeof(int);
constexpr size_t S4JAC_DIR_STATIC_LDS = sizeof(cx) * (4 * S4_SMAX + 1);

// One wave per (mixer, channel): M^-1, A_d, Q, B_d, Xt, w+-, wt+-, wt+- M^-1 and the step direction.
__global__ __launch_bounds__(S4_THREADS) void s4jacp_prep_kernel(const double* __restrict__ params, long s4_off,
                                                                 int N, int d, int s, double* __restrict__ ws,
                                                                 double* __restrict__ J) {
  __shared__ cx G[S4_SMAX * (2 * S4_SMAX + 1)];
  __shared__ cx Abar[S4_SMAX * S4_SMAX];
  __shared__ cx W1[S4_SMAX * S4_SMAX], W2[S4_SMAX * S4_SMAX], W3[S4_SMAX * S4_SMAX];
  __shared__ cx xa[S4_SMAX], xb[S4_SMAX], ya[S4_SMAX], yb[S4_SMAX], Cp[S4_SMAX], Cm[S4_SMAX], fac[S4_SMAX];
  __shared__ int piv_s;
  extern __shared__ double resp[];  // [2][N+1]: Re(C+ . dXt_p), Re(C- . dXt_p)
  const int t = threadIdx.x;
  const int ch = blockIdx.x, c = ch % d;
  const int NP = 12 * s + 1;
  const double* p = params + s4_off + (long)ch * NP;
  const double delta = exp(log(1e-2) + log(10.0) * (double)c / (double)(d > 1 ? d - 1 : 1) + p[12 * s]);
  const S4PerPtr w = s4pp_ptrs(ws, ch, N, s);
  const int ld = 2 * s + 1;
  // M^-1 from [M | I], M = I - Delta/2 Abar
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx a = cmul(cx{p[2 * s + i], p[3 * s + i]}, cx{p[4 * s + jj], p[5 * s + jj]});
    if (i == jj) a = cadd(a, cx{-exp(p[i]), p[s + i]});
    Abar[i * S4_SMAX + jj] = a;
    G[i * ld + jj] = cx{(i == jj ? 1.0 : 0.0) - 0.5 * delta * a.re, -0.5 * delta * a.im};
    G[i * ld + s + jj] = cx{i == jj ? 1.0 : 0.0, 0.0};
  }
  for (int i = t; i < s; i += S4_THREADS) {
    G[i * ld + 2 * s] = cx{0.0, 0.0};
    Cp[i] = cx{p[8 * s + i], p[9 * s + i]};
    Cm[i] = cx{p[10 * s + i], p[11 * s + i]};
  }
  __syncthreads();
  gauss_jordan(G, s, 2 * s, ld, fac, &piv_s);
  for (int idx = t; idx < s * s; idx += S4_THREADS) w.Minv[idx] = G[(idx / s) * ld + s + idx % s];
  __threadfence_block();
  __syncthreads();
  // A_d = M^-1 (I + Delta/2 Abar), B_d = M^-1 Delta Bbar; A_d also into W2 for the powering
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) {
      cx r = Abar[k * S4_SMAX + jj];
      r = cx{0.5 * delta * r.re + (k == jj ? 1.0 : 0.0), 0.5 * delta * r.im};
      acc = cadd(acc, cmul(w.Minv[i * s + k], r));
    }
    w.Ad[idx] = acc;
    W2[i * S4_SMAX + jj] = acc;
    W1[i * S4_SMAX + jj] = cx{i == jj ? 1.0 : 0.0, 0.0};
  }
  for (int i = t; i < s; i += S4_THREADS) {
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(w.Minv[i * s + k], cx{delta * p[6 * s + k], delta * p[7 * s + k]}));
    w.Bd[i] = acc;
  }
  __threadfence_block();
  __syncthreads();
  // A_d^N by binary powering (W1), then Q = (I - A_d^N)^-1 from [I - A_d^N | I]
  for (int e = N; e > 0; e >>= 1) {
    if (e & 1) {
      cmatmul(W1, W2, W3, s, S4_SMAX);
      for (int idx = t; idx < s * s; idx += S4_THREADS) W1[(idx / s) * S4_SMAX + idx % s] = W3[(idx / s) * S4_SMAX + idx % s];
      __syncthreads();
    }
    if (e > 1) {
      cmatmul(W2, W2, W3, s, S4_SMAX);
      for (int idx = t; idx < s * s; idx += S4_THREADS) W2[(idx / s) * S4_SMAX + idx % s] = W3[(idx / s) * S4_SMAX + idx % s];
      __syncthreads();
    }
  }
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx a = W1[i * S4_SMAX + jj];
    G[i * ld + jj] = cx{(i == jj ? 1.0 : 0.0) - a.re, -a.im};
    G[i * ld + s + jj] = cx{i == jj ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  gauss_jordan(G, s, 2 * s, ld, fac, &piv_s);
  for (int idx = t; idx < s * s; idx += S4_THREADS) w.Q[idx] = G[(idx / s) * ld + s + idx % s];
  __threadfence_block();
  __syncthreads();
  // Xt_m = A_d^m Q B_d, m = 0..N
  if (t < s) {
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(w.Q[t * s + k], w.Bd[k]));
    xa[t] = acc;
  }
  __syncthreads();
  for (int m = 0; m <= N; ++m) {
    if (t < s) w.Xt[(long)m * s + t] = xa[t];
    cx nx{0.0, 0.0};
    if (t < s) for (int k = 0; k < s; ++k) nx = cadd(nx, cmul(w.Ad[t * s + k], xa[k]));
    __syncthreads();
    if (t < s) xa[t] = nx;
    __syncthreads();
  }
  // w+-_m = C+-^T A_d^m (m < N)
  for (int i = t; i < s; i += S4_THREADS) { ya[i] = Cp[i]; yb[i] = Cm[i]; }
  __syncthreads();
  for (int m = 0; m < N; ++m) {
    cx np{0.0, 0.0}, nm{0.0, 0.0};
    if (t < s) {
      w.Wp[(long)m * s + t] = ya[t];
      w.Wm[(long)m * s + t] = yb[t];
      for (int k = 0; k < s; ++k) { np = cadd(np, cmul(ya[k], w.Ad[k * s + t])); nm = cadd(nm, cmul(yb[k], w.Ad[k * s + t])); }
    }
    __syncthreads();
    if (t < s) { ya[t] = np; yb[t] = nm; }
    __syncthreads();
  }
  // wt+-_m = C+-^T Q A_d^m (m < 2N) and wt+-_m M^-1 (m <= N)
  if (t < s) {
    cx np{0.0, 0.0}, nm{0.0, 0.0};
    for (int k = 0; k < s; ++k) { np = cadd(np, cmul(Cp[k], w.Q[k * s + t])); nm = cadd(nm, cmul(Cm[k], w.Q[k * s + t])); }
    ya[t] = np;
    yb[t] = nm;
  }
  __syncthreads();
  for (int m = 0; m < 2 * N; ++m) {
    cx np{0.0, 0.0}, nm{0.0, 0.0};
    if (t < s) {
      w.Wtp[(long)m * s + t] = ya[t];
      w.Wtm[(long)m * s + t] = yb[t];
      if (m <= N) {
        cx up{0.0, 0.0}, um{0.0, 0.0};
        for (int k = 0; k < s; ++k) { up = cadd(up, cmul(ya[k], w.Minv[k * s + t])); um = cadd(um, cmul(yb[k], w.Minv[k * s + t])); }
        w.Utp[(long)m * s + t] = up;
        w.Utm[(long)m * s + t] = um;
      }
      for (int k = 0; k < s; ++k) { np = cadd(np, cmul(ya[k], w.Ad[k * s + t])); nm = cadd(nm, cmul(yb[k], w.Ad[k * s + t])); }
    }
    __syncthreads();
    if (t < s) { ya[t] = np; yb[t] = nm; }
    __syncthreads();
  }
  // step direction: dA = Delta/2 M^-1 Abar (I + A_d), dB_d = Delta M^-1 (Bbar + Abar B_d / 2)
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) {
      cx ia = w.Ad[k * s + jj];
      if (k == jj) ia.re += 1.0;
      acc = cadd(acc, cmul(Abar[i * S4_SMAX + k], ia));
    }
    W3[i * S4_SMAX + jj] = acc;
  }
  __syncthreads();
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, jj = idx % s;
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(w.Minv[i * s + k], W3[k * S4_SMAX + jj]));
    w.dA[idx] = cx{0.5 * delta * acc.re, 0.5 * delta * acc.im};
  }
  for (int i = t; i < s; i += S4_THREADS) {
    cx ab{0.0, 0.0};
    for (int k = 0; k < s; ++k) ab = cadd(ab, cmul(Abar[i * S4_SMAX + k], w.Bd[k]));
    fac[i] = cx{p[6 * s + i] + 0.5 * ab.re, p[7 * s + i] + 0.5 * ab.im};
  }
  __threadfence_block();
  __syncthreads();
  if (t < s) {
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(w.Minv[t * s + k], fac[k]));
    ya[t] = cx{delta * acc.re, delta * acc.im};  // dB_d
    xb[t] = cx{0.0, 0.0};                          // T_0
  }
  __syncthreads();
  for (int jj = 0; jj < N; ++jj) {  // T_(j+1) = dA Xt_j + A_d T_j
    cx nx{0.0, 0.0};
    if (t < s)
      for (int k = 0; k < s; ++k)
        nx = cadd(nx, cadd(cmul(w.dA[t * s + k], w.Xt[(long)jj * s + k]), cmul(w.Ad[t * s + k], xb[k])));
    __syncthreads();
    if (t < s) xb[t] = nx;
    __syncthreads();
  }
  if (t < s) {  // d(Q B_d) = Q (T_N + dB_d)
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(w.Q[t * s + k], cadd(xb[k], ya[k])));
    xa[t] = acc;
  }
  __syncthreads();
  double* rp = resp;
  double* rm = resp + N + 1;
  for (int m = 0; m <= N; ++m) {
    const double gp = cdot_re(Cp, xa, s), gm = cdot_re(Cm, xa, s);
    if (t == 0) { rp[m] = gp; rm[m] = gm; }
    cx nx{0.0, 0.0};
    if (t < s && m < N)
      for (int k = 0; k < s; ++k)
        nx = cadd(nx, cadd(cmul(w.dA[t * s + k], w.Xt[(long)m * s + k]), cmul(w.Ad[t * s + k], xa[k])));
    __syncthreads();
    if (t < s) xa[t] = nx;
    __syncthreads();
  }
  double* Jc = J + (long)ch * (2 * N - 1) * NP;
  for (int pp = t; pp < N; pp += S4_THREADS) s4pp_put(Jc, N, NP, pp, 12 * s, rp[pp] + rm[N - pp]);
}

// One block per (mixer, channel, direction): the C, Bbar and rank-one directions (periodic).
__global__ __launch_bounds__(256) void s4jacp_dir_kernel(const double* __restrict__ params, long s4_off, int N, int d,
                                                         int s, double* __restrict__ ws, double* __restrict__ J) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx* ap = reinterpret_cast<cx*>(smem_raw);  // [N] w+_k . alpha
  cx* am = ap + N;                            // [N] w-_k . alpha
  cx* tp = am + N;                            // [2N] wt+_m . alpha
  cx* tm = tp + 2 * N;                        // [2N] wt-_m . alpha
  cx* cc = tm + 2 * N;                        // [N] beta^T Xt_m
  __shared__ cx alpha[S4_SMAX], beta[S4_SMAX], avec[S4_SMAX], bvec[S4_SMAX];
  __shared__ cx beta0;
  const int t = threadIdx.x;
  const int ch = blockIdx.x, dir = blockIdx.y;
  const int c = ch % d;
  const int NP = 12 * s + 1;
  const double* p = params + s4_off + (long)ch * NP;
  const double delta = exp(log(1e-2) + log(10.0) * (double)c / (double)(d > 1 ? d - 1 : 1) + p[12 * s]);
  const S4PerPtr w = s4pp_ptrs(ws, ch, N, s);
  double* Jc = J + (long)ch * (2 * N - 1) * NP;
  const int grp = dir / s, n = dir % s;
  const bool imag = grp & 1;
  if (grp >= 8) {  // C+ (8,9) and C- (10,11)
    const bool plus = grp < 10;
    for (int pp = t; pp < N; pp += 256) {
      const cx x = w.Xt[(long)(plus ? pp : N - pp) * s + n];
      s4pp_put(Jc, N, NP, pp, dir, imag ? -x.im : x.re);
    }
    return;
  }
  if (grp >= 6) {  // Bbar (6,7)
    for (int pp = t; pp < N; pp += 256) {
      const cx u = cadd(w.Utp[(long)pp * s + n], w.Utm[(long)(N - pp) * s + n]);
      s4pp_put(Jc, N, NP, pp, dir, imag ? -delta * u.im : delta * u.re);
    }
    return;
  }
  for (int i = t; i < s; i += 256) {
    cx a{0.0, 0.0}, b{0.0, 0.0};
    if (grp < 2) {
      if (i == n) { a = imag ? cx{0.0, 1.0} : cx{-exp(p[n]), 0.0}; b = cx{1.0, 0.0}; }
    } else if (grp < 4) {
      if (i == n) a = imag ? cx{0.0, 1.0} : cx{1.0, 0.0};
      b = cx{p[4 * s + i], p[5 * s + i]};
    } else {
      a = cx{p[2 * s + i], p[3 * s + i]};
      if (i == n) b = imag ? cx{0.0, 1.0} : cx{1.0, 0.0};
    }
    avec[i] = a;
    bvec[i] = b;
  }
  __syncthreads();
  for (int i = t; i < s; i += 256) {
    cx al{0.0, 0.0}, be{0.0, 0.0};
    for (int k = 0; k < s; ++k) {
      al = cadd(al, cmul(w.Minv[i * s + k], avec[k]));
      cx ia = w.Ad[k * s + i];
      if (k == i) ia.re += 1.0;
      be = cadd(be, cmul(bvec[k], ia));
    }
    alpha[i] = cx{0.5 * delta * al.re, 0.5 * delta * al.im};
    beta[i] = be;
  }
  if (t == 0) {
    cx b0{0.0, 0.0};
    for (int k = 0; k < s; ++k) b0 = cadd(b0, cmul(bvec[k], w.Bd[k]));
    beta0 = b0;
  }
  __syncthreads();
  for (int k = t; k < 2 * N; k += 256) {
    cx sp{0.0, 0.0}, sm{0.0, 0.0}, ep{0.0, 0.0}, em{0.0, 0.0}, sc{0.0, 0.0};
    for (int i = 0; i < s; ++i) {
      ep = cadd(ep, cmul(w.Wtp[(long)k * s + i], alpha[i]));
      em = cadd(em, cmul(w.Wtm[(long)k * s + i], alpha[i]));
      if (k < N) {
        sp = cadd(sp, cmul(w.Wp[(long)k * s + i], alpha[i]));
        sm = cadd(sm, cmul(w.Wm[(long)k * s + i], alpha[i]));
        sc = cadd(sc, cmul(beta[i], w.Xt[(long)k * s + i]));
      }
    }
    tp[k] = ep;
    tm[k] = em;
    if (k < N) { ap[k] = sp; am[k] = sm; cc[k] = sc; }
  }
  __syncthreads();
  auto f = [&](int j, const cx* a, const cx* at) {
    cx acc = cmul(at[j], beta0);
    for (int k = 0; k < j; ++k) acc = cadd(acc, cmul(a[k], cc[j - 1 - k]));
    for (int k = 0; k < N; ++k) acc = cadd(acc, cmul(at[j + k], cc[N - 1 - k]));
    return acc.re;
  };
  for (int pp = t; pp < N; pp += 256) s4pp_put(Jc, N, NP, pp, dir, f(pp, ap, tp) + f(N - pp, am, tm));
}

// ------------------------------------------------------------------------------------------
// Per-sample S4 parameter gradients: for every mixer channel, grads[b][off(ch) + k] =
// sum_r dg[b][ch][r] J[ch][r][k] (a [B x (2N-1)] x [(2N-1) x (12s+1)] product on the matrix cores).
template <typename T> struct S4GradArgs {
  const T* dg;            // [C][nch][TG]
  const T* J;             // [nch][TG][NP]
  int C, nch, TG, NP;
  T* grads;
  long Pn, off;           // offset of the first mixer channel's block
};

template <typename T>
__global__ __launch_bounds__(256) void s4grad_kernel(S4GradArgs<T> A) {
  using M = Mma<T>;
  using acc_t = typename M::acc;
  const int ch = blockIdx.x;
  const int b0 = blockIdx.y * 64, k0 = blockIdx.z * 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kq = lane >> 4;
  // wave w: rows b0 + 16 w .. +15, columns k0 .. k0+63 (4 tiles)
  acc_t acc[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) acc[n] = acc_t{0, 0, 0, 0};
  const int brow = b0 + 16 * wave + j;
  const T* Jc = A.J + (long)ch * A.TG * A.NP;
  for (int r0 = 0; r0 < A.TG; r0 += 4) {
    const int r = r0 + kq;
    const T av = (brow < A.C && r < A.TG) ? A.dg[((long)brow * A.nch + ch) * A.TG + r] : T(0);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int k = k0 + 16 * n + j;
      const T bv = (r < A.TG && k < A.NP) ? Jc[(long)r * A.NP + k] : T(0);
      acc[n] = M::mma(av, bv, acc[n]);
    }
  }
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int b = b0 + 16 * wave + M::row(lane, rr), k = k0 + 16 * n + j;
      if (b < A.C && k < A.NP) A.grads[(long)b * A.Pn + A.off + (long)ch * A.NP + k] = acc[n][rr];
    }
}

// wsum[p] = sum_b w[b] grads[b][p] (float64 accumulation).
template <typename T>
__global__ void wsum_kernel(const T* __restrict__ grads, const double* __restrict__ w, int B, long Pn,
                            double* __restrict__ out) {
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < Pn; p += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += w[b] * (double)grads[(long)b * Pn + p];
    out[p] = s;
  }
}

}  // namespace dn
