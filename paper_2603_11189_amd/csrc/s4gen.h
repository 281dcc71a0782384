// Parameter-only work, float64: S4 Green's-function taps and the kernel-layout tables.
//
// Kernel generation follows Sec. V (bidirectional SSM, Eq. (resolvent) as the transform of
// the impulse response) and App. "Details on the implementation of the DysonNet block",
// Eq. (discretization): per mixer and channel, Abar = diag(Lambda) + p q^T,
// A_d = (I - Delta/2 Abar)^-1 (I + Delta/2 Abar), B_d = (I - Delta/2 Abar)^-1 Delta Bbar
// (Gauss-Jordan elimination with partial pivoting in LDS), then the impulse response
// K+-_r = Re(C+-^T A_d^r B_d) by repeated state-matrix products. Open chains use g_r = K+_r
// (r >= 0) and g_-r = K-_r (r >= 1); periodic chains the aliased kernel
// g_p = Re(C+^T A_d^p Q B_d) + Re(C-^T A_d^(N-p) Q B_d) with Q = (I - A_d^N)^-1.
#pragma once
#include "common.h"

namespace dn {

struct cx {
  double re, im;
};
__device__ inline cx cmul(cx a, cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cx cadd(cx a, cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cx csub(cx a, cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cx cdiv(cx a, cx b) {
  double den = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ inline double cabs2(cx a) { return a.re * a.re + a.im * a.im; }

constexpr int S4_SMAX = 32;     // state size limit of the on-chip solver
constexpr int S4_THREADS = 64;  // one wave per (mixer, channel)

// Gauss-Jordan on the s x ncol augmented matrix G (row stride ld) held in LDS:
// reduces the leading s x s block to the identity with partial pivoting.
__device__ inline void gauss_jordan(cx* G, int s, int ncol, int ld, cx* fac, int* piv_s) {
  const int t = threadIdx.x;
  for (int k = 0; k < s; ++k) {
    if (t == 0) {
      int piv = k;
      double best = cabs2(G[k * ld + k]);
      for (int i = k + 1; i < s; ++i) {
        double v = cabs2(G[i * ld + k]);
        if (v > best) { best = v; piv = i; }
      }
      *piv_s = piv;
    }
    __syncthreads();
    const int piv = *piv_s;
    if (piv != k)
      for (int j = t; j < ncol; j += S4_THREADS) {
        cx a = G[k * ld + j];
        G[k * ld + j] = G[piv * ld + j];
        G[piv * ld + j] = a;
      }
    __syncthreads();
    const cx inv = cdiv(cx{1.0, 0.0}, G[k * ld + k]);
    __syncthreads();
    for (int j = t; j < ncol; j += S4_THREADS) G[k * ld + j] = cmul(G[k * ld + j], inv);
    __syncthreads();
    for (int i = t; i < s; i += S4_THREADS) fac[i] = G[i * ld + k];
    __syncthreads();
    for (int idx = t; idx < s * ncol; idx += S4_THREADS) {
      int i = idx / ncol, j = idx % ncol;
      if (i != k) G[i * ld + j] = csub(G[i * ld + j], cmul(fac[i], G[k * ld + j]));
    }
    __syncthreads();
  }
}

// y = A x for an s x s matrix (row stride ld) and vectors in LDS; thread i < s owns row i.
__device__ inline void cmatvec(const cx* A, int ld, const cx* x, cx* y, int s) {
  const int i = threadIdx.x;
  if (i < s) {
    cx acc{0.0, 0.0};
    for (int j = 0; j < s; ++j) acc = cadd(acc, cmul(A[i * ld + j], x[j]));
    y[i] = acc;
  }
  __syncthreads();
}

// Re(sum_i C_i x_i) over the state (thread i < s contributes), broadcast to all threads.
__device__ inline double cdot_re(const cx* C, const cx* x, int s) {
  const int i = threadIdx.x;
  double v = 0.0;
  if (i < s) v = C[i].re * x[i].re - C[i].im * x[i].im;
  return wave_sum(v);
}

// C = A * B for s x s complex matrices (row stride ld) in LDS.
__device__ inline void cmatmul(const cx* A, const cx* B, cx* C, int s, int ld) {
  for (int idx = threadIdx.x; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, j = idx % s;
    cx acc{0.0, 0.0};
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(A[i * ld + k], B[k * ld + j]));
    C[i * ld + j] = acc;
  }
  __syncthreads();
}

// One block per (mixer, channel); writes taps64[(mixer*d + c)*(2N-1) + r + N - 1].
// params: the flat float64 vector; s4_off: offset of the first mixer's first channel.
__global__ __launch_bounds__(S4_THREADS) void s4_taps_kernel(const double* __restrict__ params,
                                                             long s4_off, int N, int d, int s,
                                                             int periodic, double* __restrict__ taps64) {
  __shared__ cx G[S4_SMAX * (2 * S4_SMAX + 1)];
  __shared__ cx Ad[S4_SMAX * S4_SMAX];
  __shared__ cx W1[S4_SMAX * S4_SMAX];
  __shared__ cx W2[S4_SMAX * S4_SMAX];
  __shared__ cx W3[S4_SMAX * S4_SMAX];
  __shared__ cx xa[S4_SMAX], xb[S4_SMAX], Cp[S4_SMAX], Cm[S4_SMAX], fac[S4_SMAX];
  __shared__ int piv_s;
  extern __shared__ double resp[];  // periodic: [2][N+1]
  const int t = threadIdx.x;
  const int mixer = blockIdx.x / d, c = blockIdx.x % d;
  const double* p = params + s4_off + (long)(mixer * d + c) * (12 * s + 1);
  const double delta = exp(log(1e-2) + log(10.0) * (double)c / (double)(d > 1 ? d - 1 : 1) + p[12 * s]);
  const int ld = 2 * s + 1;
  // augmented [I - Delta/2 Abar | I + Delta/2 Abar | Delta Bbar], Abar = diag(Lambda) + p q^T
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, j = idx % s;
    cx pi{p[2 * s + i], p[3 * s + i]}, qj{p[4 * s + j], p[5 * s + j]};
    cx a = cmul(pi, qj);
    if (i == j) a = cadd(a, cx{-exp(p[i]), p[s + i]});
    cx h{0.5 * delta * a.re, 0.5 * delta * a.im};
    G[i * ld + j] = cx{(i == j ? 1.0 : 0.0) - h.re, -h.im};
    G[i * ld + s + j] = cx{(i == j ? 1.0 : 0.0) + h.re, h.im};
  }
  for (int i = t; i < s; i += S4_THREADS) {
    G[i * ld + 2 * s] = cx{delta * p[6 * s + i], delta * p[7 * s + i]};
    Cp[i] = cx{p[8 * s + i], p[9 * s + i]};
    Cm[i] = cx{p[10 * s + i], p[11 * s + i]};
  }
  __syncthreads();
  gauss_jordan(G, s, 2 * s + 1, ld, fac, &piv_s);
  for (int idx = t; idx < s * s; idx += S4_THREADS) Ad[(idx / s) * S4_SMAX + idx % s] = G[(idx / s) * ld + s + idx % s];
  for (int i = t; i < s; i += S4_THREADS) xa[i] = G[i * ld + 2 * s];  // B_d
  __syncthreads();
  double* out = taps64 + (long)(mixer * d + c) * (2 * N - 1);
  if (!periodic) {
    for (int r = 0; r < N; ++r) {
      cx* x = (r & 1) ? xb : xa;
      cx* y = (r & 1) ? xa : xb;
      double kp = cdot_re(Cp, x, s), km = cdot_re(Cm, x, s);
      if (t == 0) {
        out[N - 1 + r] = kp;
        if (r > 0) out[N - 1 - r] = km;
      }
      cmatvec(Ad, S4_SMAX, x, y, s);
    }
    return;
  }
  // A_d^N by binary powering: W1 = result, W2 = running square.
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, j = idx % s;
    W1[i * S4_SMAX + j] = cx{i == j ? 1.0 : 0.0, 0.0};
    W2[i * S4_SMAX + j] = Ad[i * S4_SMAX + j];
  }
  __syncthreads();
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
  // solve (I - A_d^N) y = B_d
  const int ld2 = s + 1;
  for (int idx = t; idx < s * s; idx += S4_THREADS) {
    int i = idx / s, j = idx % s;
    cx a = W1[i * S4_SMAX + j];
    G[i * ld2 + j] = cx{(i == j ? 1.0 : 0.0) - a.re, -a.im};
  }
  for (int i = t; i < s; i += S4_THREADS) G[i * ld2 + s] = xa[i];
  __syncthreads();
  gauss_jordan(G, s, s + 1, ld2, fac, &piv_s);
  for (int i = t; i < s; i += S4_THREADS) xa[i] = G[i * ld2 + s];
  __syncthreads();
  double* rp = resp;          // Re(C+ A^p Q B), p = 0..N
  double* rm = resp + N + 1;  // Re(C- A^p Q B), p = 0..N
  for (int r = 0; r <= N; ++r) {
    cx* x = (r & 1) ? xb : xa;
    cx* y = (r & 1) ? xa : xb;
    double kp = cdot_re(Cp, x, s), km = cdot_re(Cm, x, s);
    if (t == 0) { rp[r] = kp; rm[r] = km; }
    cmatvec(Ad, S4_SMAX, x, y, s);
  }
  __syncthreads();
  for (int q = t; q < 2 * N - 1; q += S4_THREADS) {
    int r = q - (N - 1);
    int pidx = ((r % N) + N) % N;
    out[q] = rp[pidx] + rm[N - pidx];
  }
}

// Kernel-layout tables from the float64 parameters and taps (all float64 here).
struct PrepArgs {
  const double* params;
  const double* taps64;  // [L+1][d][2N-1]
  int N, Np, L, d, DP, s, w_c, d_out, periodic, tok;
  int dblk;                                // > 0: U and V block-diagonal in channel blocks of dblk
  long off_layers, off_A;
  // outputs (double tables)
  double *E, *Ephi, *wE1;                  // [tok][DP]: per position inside a token
  double *WDt, *ADt, *Ut, *Vt, *Um, *Vm;  // [L][DP][DP]; *t transposed (t[k][m] = M[m][k])
  double *wv, *Kc, *kv, *bv;               // [L][DP], K: [L][2w_c+1][DP]
  double *taps, *tapsR;                    // [L][DP][TS] mixers and their transposes
  double *omega, *Wk, *A;                  // [DP][Np], [2][DP][Np], [DP][2]
  double *omN, *Ac;                        // omega / N [DP][Np]; A transposed [2][DP]
  double *ADm, *WDm;                       // operand tables of A_D^T, W_D^T
};

__global__ void prep_kernel(PrepArgs a) {
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  const int d = a.d, DP = a.DP, L = a.L, Wc = 2 * a.w_c + 1;
  const long lay_sz = 4L * d * d + 6L * d + (long)(Wc - 3) * d;  // W_D,w,K,k,A_D,b,U,V
  for (long i = tid; i < DP; i += nth)
    for (int k = 0; k < 2; ++k) a.A[i * 2 + k] = i < d ? a.params[a.off_A + i * a.d_out + k] : 0.0;
  for (long ik = tid; ik < (long)a.tok * DP; ik += nth) {
    const int k = (int)(ik / DP), i = (int)(ik % DP);  // position inside the token, channel
    const double* Ek = a.params + (long)k * d;
    const double* Fk = a.params + (long)(a.tok + k) * d;
    a.E[ik] = i < d ? Ek[i] : 0.0;
    a.Ephi[ik] = i < d ? Fk[i] : 0.0;
    double acc = 0.0;
    if (i < d) {
      const double* WD = a.params + a.off_layers;  // block 1
      for (int j = 0; j < d; ++j) acc += WD[i * d + j] * Fk[j];
    }
    a.wE1[ik] = acc;
  }
  // Operand tables of out = M in: table[kin][mout] = M[mout][kin] (row = input channel).
  // WDt, ADt, Ut, Vt hold W_D, A_D, U, V; Um, Vm hold U^T, V^T (table[kin][mout] = U[kin][mout]).
  for (long idx = tid; idx < (long)L * DP * DP; idx += nth) {
    int l = idx / (DP * DP), row = (idx / DP) % DP, col = idx % DP;
    const double* base = a.params + a.off_layers + l * lay_sz;
    const double* WD = base;
    const double* AD = base + d * d + d + Wc * d + d;
    const double* U = AD + d * d + d;
    const double* V = U + d * d;
    bool in = (row < d && col < d);
    // the block-diagonal vertex: U and V vanish off the channel blocks
    const bool uv = in && (a.dblk <= 0 || row / a.dblk == col / a.dblk);
    a.WDt[idx] = in ? WD[col * d + row] : 0.0;
    a.ADt[idx] = in ? AD[col * d + row] : 0.0;
    a.Ut[idx] = uv ? U[col * d + row] : 0.0;
    a.Vt[idx] = uv ? V[col * d + row] : 0.0;
    a.Um[idx] = uv ? U[row * d + col] : 0.0;
    a.Vm[idx] = uv ? V[row * d + col] : 0.0;
    a.ADm[idx] = in ? AD[row * d + col] : 0.0;
    a.WDm[idx] = in ? WD[row * d + col] : 0.0;
  }
  for (long idx = tid; idx < (long)L * DP; idx += nth) {
    int l = idx / DP, c = idx % DP;
    const double* base = a.params + a.off_layers + l * lay_sz;
    bool in = c < d;
    a.wv[idx] = in ? base[d * d + c] : 0.0;
    a.kv[idx] = in ? base[d * d + d + Wc * d + c] : 0.0;
    a.bv[idx] = in ? base[d * d + d + Wc * d + d + d * d + c] : 0.0;
    for (int r = 0; r < Wc; ++r) a.Kc[(l * Wc + r) * DP + c] = in ? base[d * d + d + r * d + c] : 0.0;
  }
  const int N = a.N, Np = a.Np, TS = tap_stride(Np), TO = tap_off(Np);
  const int periodic = a.periodic;
  auto tap = [&](int l, int c, int r) -> double {  // g of mixer l, channel c at offset r
    if (periodic) { int p = ((r % N) + N) % N; return a.taps64[((long)l * d + c) * (2 * N - 1) + p + N - 1]; }
    if (r <= -N || r >= N) return 0.0;
    return a.taps64[((long)l * d + c) * (2 * N - 1) + r + N - 1];
  };
  for (long idx = tid; idx < (long)L * DP * TS; idx += nth) {
    int l = idx / ((long)DP * TS), c = (idx / TS) % DP, q = idx % TS;
    int r = q - TO;
    a.taps[idx] = (c < d) ? tap(l, c, r) : 0.0;
    a.tapsR[idx] = (c < d) ? tap(l, c, -r) : 0.0;  // transposed mixer
  }
  for (long idx = tid; idx < (long)DP * Np; idx += nth) {
    int c = idx / Np, i = idx % Np;
    double om = 0.0;
    if (c < d && i < N) {
      const double* g = a.taps64 + ((long)L * d + c) * (2 * N - 1);
      for (int j = 0; j < N; ++j) om += g[(j - i) + N - 1];  // column sum of the final mixer
    }
    a.omega[idx] = om;
    a.omN[idx] = om / (double)N;
    for (int k = 0; k < 2; ++k) {
      double A = (c < d) ? a.params[a.off_A + c * a.d_out + k] : 0.0;
      a.Wk[(long)k * DP * Np + idx] = om * A / (double)N;
      if (i == 0) a.Ac[k * DP + c] = A;
    }
  }
}

__global__ void convert_kernel(const double* __restrict__ src, float* __restrict__ dst, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void finite_check_kernel(const double* __restrict__ x, long n, int* __restrict__ bad) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) atomicOr(bad, 1);
}

// First deep block of ABACUS for a unit flip: a flip at site z injects e^(0) = -2 s_z E there,
// so the block's first channel-mixing product is q(i) = -2 s_z Pq(i - z) with the
// parameter-only table Pq[k][r] = sum_c V^(1)[k][c] E_c g^(1)_c(r), formed here for every
// stored offset r of the tap table (margins included). It is stored four times, copy sh
// shifted by sh entries (Pq4[sh][k][r] = Pq[k][r + sh]), so that four consecutive sites can
// be read as one aligned vector whatever z is. Vt is the operand table of V^(1)
// (Vt[c][k] = V[k][c]).
__global__ void ptab_kernel(const double* __restrict__ taps1, const double* __restrict__ Vt,
                            const double* __restrict__ E, int DP, int TS, double* __restrict__ Pq4) {
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < 4L * DP * TS;
       idx += (long)gridDim.x * blockDim.x) {
    const int sh = (int)(idx / ((long)DP * TS));
    const int k = (int)((idx / TS) % DP), rr = (int)(idx % TS) + sh;
    double acc = 0.0;
    if (rr < TS)
      for (int c = 0; c < DP; ++c) acc += Vt[(long)c * DP + k] * E[c] * taps1[(long)c * TS + rr];
    Pq4[idx] = acc;
  }
}

}  // namespace dn
