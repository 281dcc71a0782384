// Network kernels: phi stream, Green's-function mixer (Toeplitz products on the matrix
// cores), vertex + channel mixing with the read-out, and the ABACUS update.
//
// Field layout in HBM: [configuration][channel DP][site Np], sites fastest, DP = d padded
// to a multiple of 16, Np = N padded to a multiple of 64. Padded channels hold exact
// zeros (their weights are zero); padded sites are written as zeros and never read as
// inputs of real sites.
#pragma once
#include "common.h"

namespace dn {

template <typename T> struct Tables {
  const T *E, *Ephi, *wE1;                 // [token][DP]: one vector per position inside a token
  const T *WDt, *ADt, *Ut, *Vt, *Um, *Vm;  // [L][DP][DP] operand tables (row = input channel)
  const T *wv, *Kc, *kv, *bv;              // [L][DP], K [L][2w_c+1][DP]
  const T *taps, *tapsR;                   // [L][DP][tap_stride]: mixers and their transposes
  const T *Wk;                             // [2][DP][Np]
  const T *ADm, *WDm;                      // operand tables of A_D^T and W_D^T
  const T *Pq;                             // [token][4][DP][tap_stride]: V^(1) (E_k * g^(1)(r)), see ptab_kernel
  const T *omN, *Ac;                       // omega / N [DP][Np] and A^T [2][DP]: Wk = Ac omN
};

// Which configuration a block works on. Plain path: cfg g -> sample b, element m (m = -1
// is the unflipped sample). ABACUS: flip f -> (b, m).
struct CfgMap {
  const int32_t* cb;  // [count]
  const int32_t* cm;  // [count]
  const int32_t* sites;  // [B][M_max][2]
  int M_max;
};

// Element i of an array at a workgroup-uniform base with a 32-bit offset: the address is a
// scalar base plus one vector register, instead of a 64-bit vector address per array and
// index (the phi stream touches up to seven [DP][Np] arrays per channel).
template <typename T> __device__ inline T& elem(T* base, unsigned i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T));
}
template <typename T> __device__ inline const T& elem(const T* base, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}

// ---------------------------------------------------------------------------------------
// Channel-mixing tile on the matrix cores: acc[mt][n] += W x for the DP x DP weight W whose
// operand table Wt (row = input channel) is given, over NT 16-site tiles starting at site i0.
// B operands come from a caller-supplied loader bload(kc, n) = x[kc][i0 + 16 n + lane % 16].
// float: the weight fragments are held in registers across tiles (wreg); double: read per step.
template <typename T, int DP> struct WFrag {
  static constexpr int MT = DP / 16, KS = DP / 4;
  T f[MT][KS];
  __device__ void load(const T* __restrict__ Wt, int lane) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) f[mt][ks] = Wt[(4 * ks + (lane >> 4)) * DP + 16 * mt + (lane & 15)];
  }
};

template <typename T, int DP, int NT, typename BL>
__device__ inline void mix_tile(const WFrag<T, DP>& w, BL bload, typename Mma<T>::acc (&acc)[DP / 16][NT]) {
  constexpr int MT = DP / 16, KS = DP / 4;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[mt][n] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {  // fully unrolled: the weight fragments stay in registers
    T bv[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) bv[n] = bload(4 * ks + (threadIdx.x & 63) / 16, n);
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt][n] = Mma<T>::mma(w.f[mt][ks], bv[n], acc[mt][n]);
  }
}

// mix_tile with the weight operands read from the table at each step instead of held in
// registers (kernels whose register budget has no room for a whole fragment set).
template <typename T, int DP, int NT, typename BL>
__device__ inline void mix_tile_ptr(const T* __restrict__ Wt, BL bload, typename Mma<T>::acc (&acc)[DP / 16][NT]) {
  constexpr int MT = DP / 16, KS = DP / 4;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[mt][n] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    T bv[NT], af[MT];
#pragma unroll
    for (int n = 0; n < NT; ++n) bv[n] = bload(4 * ks + (lane >> 4), n);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) af[mt] = elem(Wt, (4 * ks + (lane >> 4)) * DP + 16 * mt + (lane & 15));
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt][n] = Mma<T>::mma(af[mt], bv[n], acc[mt][n]);
    if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
}

// Site tiles per wave for a padded chain of Np sites and 4 waves per workgroup.
__host__ __device__ inline int tiles_per_wave(int Np) { return Np >= 256 ? 4 : Np / 64; }

// ---------------------------------------------------------------------------------------
// phi stream of block l (App. "Details on the implementation of the DysonNet block"):
//   a = W_D phi^(l-1) + w;  phi^(l) = g(sum_r K_r * a_{i+r} + k);  chi^(l) = g(A_D phi^(l) + b)
// Block 1 uses phi^(0) = E_phi s', so a = s'_i (W_D E_phi) + w (rank one). Block 1 also
// writes u^(1) = E s' (+ phi^(1) when injected) and starts the read-out sum with h^(0).
// One workgroup (4 waves) per configuration; a is staged in LDS with a halo of w_c.
template <typename T> struct PhiArgs {
  Tables<T> tb;
  int N, Np, l, w_c, periodic, act, inject;
  int first;
  int tok;              // spins per token
  const int8_t* spins;  // [B][N * tok]
  CfgMap map;
  int cfg0, C;          // configurations [cfg0, cfg0 + C)
  const T* phi_in;      // [C][DP][Np]
  T* phi_out;           // nullable
  T* chi_out;
  T* a_out;             // cache, nullable
  T* u_out;             // first block only
  double* rho;          // first block only: [C][2]
  T* z_out;             // pre-activation of phi (nullable)
  T* zeta_out;          // pre-activation of chi (nullable)
  T* R_out;             // first block: residual sum initialised with h^(0) (nullable)
};

// TOK: tokens of more than one spin (A.tok); without it the embedding is the per-site one.
template <typename T, int DP, int NT, bool TOK = false>
__global__ __launch_bounds__(256) void phi_kernel(PhiArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* as = reinterpret_cast<T*>(smem_raw);
  const int g = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, col = lane & 15;
  const int N = A.N, Np = A.Np, wc = A.w_c;
  const int ld = Np + 2 * wc + 1;  // odd row stride
  T* sp_s = as + DP * ld;          // s' (first block), [tok][Np]: spin k of every token
  __shared__ double red[2][4];
  constexpr int MT = DP / 16;
  using M = Mma<T>;
  using acc_t = typename M::acc;
  const int l = A.l;
  const int span = 16 * NT;  // sites per wave per pass
  // this configuration's [DP][Np] slices (workgroup-uniform bases)
  const long fo = (long)g * DP * Np;
  T* a_out = A.a_out ? A.a_out + fo : nullptr;
  T* phi_out = A.phi_out ? A.phi_out + fo : nullptr;
  T* z_out = A.z_out ? A.z_out + fo : nullptr;
  T* zeta_out = A.zeta_out ? A.zeta_out + fo : nullptr;
  T* chi_out = A.chi_out + fo;
  if (A.first) {
    const int gg = A.cfg0 + g;
    const int b = A.map.cb[gg], m = A.map.cm[gg];
    int f0 = -1, f1 = -1;
    if (m >= 0) {
      f0 = A.map.sites[((long)b * A.map.M_max + m) * 2];
      f1 = A.map.sites[((long)b * A.map.M_max + m) * 2 + 1];
    }
    const int tk = TOK ? A.tok : 1;
    const int8_t* sp = A.spins + (long)b * N * tk;
    for (int i = threadIdx.x; i < tk * Np; i += 256) {
      const int k = i / Np, ti = i - k * Np;  // position inside the token, token
      T v = 0;
      if (ti < N) {
        const int si = ti * tk + k;
        v = (T)sp[si];
        if (si == f0 || si == f1) v = -v;
      }
      sp_s[i] = v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < DP * Np; idx += 256) {
      int c = idx / Np, i = idx % Np;
      T v = 0;
      if (i < N) {
        v = sp_s[i] * A.tb.wE1[c] + A.tb.wv[c];
        for (int k = 1; k < tk; ++k) v += sp_s[k * Np + i] * A.tb.wE1[k * DP + c];
      }
      as[c * ld + i + wc] = v;
      if (a_out) elem(a_out, idx) = v;
    }
  } else {
    const T* Wd = A.tb.WDt + (long)l * DP * DP;
    const T* x = A.phi_in + fo;
    for (int i0 = wave * span; i0 < Np; i0 += 4 * span) {
      acc_t acc[MT][NT];
      mix_tile_ptr<T, DP, NT>(Wd, [&](int kc, int n) { return elem(x, kc * Np + i0 + 16 * n + col); }, acc);
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int i = i0 + 16 * n + col;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ch = 16 * mt + M::row(lane, r);
            T v = (i < N) ? acc[mt][n][r] + A.tb.wv[l * DP + ch] : T(0);
            as[ch * ld + i + wc] = v;
            if (a_out) elem(a_out, ch * Np + i) = v;
          }
      }
    }
  }
  __syncthreads();
  // halos of width w_c (open: zero; periodic: wrap-around)
  if (wc > 0) {
    for (int idx = threadIdx.x; idx < DP * 2 * wc; idx += 256) {
      int c = idx / (2 * wc), h = idx % (2 * wc);
      int cl, src;
      if (h < wc) { cl = h; src = N - wc + h; }           // sites -wc..-1
      else { cl = N + wc + (h - wc); src = h - wc; }      // sites N..N+wc-1
      as[c * ld + cl] = A.periodic ? as[c * ld + src + wc] : T(0);
    }
  }
  // the block's per-channel vectors in LDS: k [DP], then K_r [2 w_c + 1][DP]
  T* kvs = sp_s + (TOK ? A.tok : 1) * Np;
  for (int idx = threadIdx.x; idx < (2 * wc + 2) * DP; idx += 256)
    kvs[idx] = idx < DP ? A.tb.kv[l * DP + idx] : A.tb.Kc[(long)l * (2 * wc + 1) * DP + idx - DP];
  __syncthreads();
  const T* Ad = A.tb.ADt + (long)l * DP * DP;
  double part0 = 0.0, part1 = 0.0;
  for (int i0 = wave * span; i0 < Np; i0 += 4 * span) {
    // phi of the tile in operand-B layout (channel 4 ks + lane / 16, site i0 + 16 n + lane % 16):
    // the taps run outermost so that the lane's DP / 4 channels accumulate side by side
    T xb[DP / 4][NT];
#pragma unroll
    for (int ks = 0; ks < DP / 4; ++ks)
#pragma unroll
      for (int n = 0; n < NT; ++n) xb[ks][n] = kvs[4 * ks + q];
    for (int r = 0; r <= 2 * wc; ++r) {
      const T* kr = kvs + (r + 1) * DP + q;
      const T* ar = as + q * ld + i0 + col + r;
#pragma unroll
      for (int ks = 0; ks < DP / 4; ++ks) {
        const T kk = kr[4 * ks];
#pragma unroll
        for (int n = 0; n < NT; ++n) xb[ks][n] += kk * ar[4 * ks * ld + 16 * n];
      }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int i = i0 + 16 * n + col;
      const bool in = i < N;
      const T h0s = (A.first && in) ? sp_s[i] : T(0);
#pragma unroll
      for (int ks = 0; ks < DP / 4; ++ks) {
        const int kc = 4 * ks + q;
        const unsigned o = kc * Np + i;
        const T s = xb[ks][n];
        const T ph = in ? act_fn<T>(A.act, s) : T(0);
        if (z_out) elem(z_out, o) = in ? s : T(0);
        if (phi_out) elem(phi_out, o) = ph;
        if (A.first) {
          T h0 = A.tb.E[kc] * h0s;
          if constexpr (TOK)
            for (int k = 1; k < A.tok; ++k) h0 += A.tb.E[k * DP + kc] * (in ? sp_s[k * Np + i] : T(0));
          if (A.R_out) elem(A.R_out + fo, o) = h0;
          elem(A.u_out + fo, o) = h0 + (A.inject ? ph : T(0));
          part0 += (double)elem(A.tb.Wk, o) * (double)h0;
          part1 += (double)elem(A.tb.Wk, DP * Np + o) * (double)h0;
        }
        xb[ks][n] = ph;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    acc_t acc[MT][NT];
    mix_tile_ptr<T, DP, NT>(Ad, [&](int kc, int n) { return xb[kc >> 2][n]; }, acc);
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int i = i0 + 16 * n + col;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ch = 16 * mt + M::row(lane, r);
          const unsigned o = ch * Np + i;
          const T zt = acc[mt][n][r] + A.tb.bv[l * DP + ch];
          elem(chi_out, o) = (i < N) ? act_fn<T>(A.act, zt) : T(0);
          if (zeta_out) elem(zeta_out, o) = (i < N) ? zt : T(0);
        }
    }
  }
  if (A.first) {
    part0 = wave_sum(part0);
    part1 = wave_sum(part1);
    if (lane == 0) { red[0][wave] = part0; red[1][wave] = part1; }
    __syncthreads();
    if (threadIdx.x == 0) {
      A.rho[2 * g] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
      A.rho[2 * g + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
  }
}

// ---------------------------------------------------------------------------------------
// Green's-function mixer for a batch of fields, per channel c: Y[cfg, c, :] = X[cfg, c, :] G_c^T,
// i.e. Y_i = sum_i' g_c(i - i') X_i'. The Toeplitz operand is generated on the fly from the
// taps staged in LDS; the field operand is staged in LDS in 64-site chunks (row stride 66
// floats: conflict-free fragment reads). One workgroup: 64 configurations x 256 output
// sites of one channel; each wave owns 64 (or fewer) output sites.
// Launch-time work count. With offs == nullptr the host value holds; otherwise the launch
// covers flips offs[b0] .. offs[b0 + Bc] of the device work list (a grid sized for the
// upper bound Bc * M_max whose surplus workgroups return at once), so a launch sequence
// needs no host round trip and can be captured once and replayed for any spins.
struct DynRange {
  const int32_t* offs;
  int b0, Bc;
  __device__ inline int first(int f0) const { return offs ? offs[b0] : f0; }
  __device__ inline int count(int n) const { return offs ? offs[b0 + Bc] - offs[b0] : n; }
};

template <typename T> struct ConvArgs {
  const T* X;
  T* Y;
  const T* taps;  // [DP][tap_stride(Np)] for this mixer
  int N, Np, C, DP;
  DynRange dyn;   // configurations counted on the device (nullable)
  const T* add;   // nullable: Y[cfg] += add[cfg mod 2] (field [2][DP][Np])
};

constexpr int CONV_MC = 64;   // configurations per workgroup
constexpr int CONV_KC = 64;   // input sites per LDS chunk
constexpr int CONV_LD = 66;   // LDS row stride of the field chunk

template <typename T, int NT>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);   // [CONV_MC][CONV_LD]
  T* ts = xs + CONV_MC * CONV_LD;           // [2Np]
  using M = Mma<T>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.y;
  const int cfg0 = blockIdx.x * CONV_MC;
  const int C = A.dyn.count(A.C);
  if (cfg0 >= C) return;
  const int Np = A.Np;
  // output block of 4 waves x 16*NT sites; the host picks NT with Np a multiple of 16*NT
  const int site0 = blockIdx.z * 64 * NT;
  const int wsite0 = site0 + wave * 16 * NT;              // this wave's first output site
  const T* tp = A.taps + (long)c * tap_stride(Np) + 64;  // offsets -(Np-1).. at ts[0..]
  for (int q = threadIdx.x; q < 2 * Np; q += 256) ts[q] = tp[q];
  typename M::acc acc[4][NT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[a][n] = typename M::acc{0, 0, 0, 0};
  const long cstride = (long)A.DP * Np;
  // The field chunk is staged through registers one chunk ahead: thread (wave, lane) moves
  // element lane of configuration rows wave + 4u, so the loads of the next chunk are in
  // flight while the matrix cores work on the current one.
  constexpr int SU = CONV_MC * CONV_KC / 256;
  const T* xrow = A.X + (long)c * Np + lane;
  T pre[SU];
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int cfg = cfg0 + wave + 4 * u;
    pre[u] = (cfg < C) ? xrow[(long)cfg * cstride] : T(0);
  }
  for (int k0 = 0; k0 < Np; k0 += CONV_KC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SU; ++u) xs[(wave + 4 * u) * CONV_LD + lane] = pre[u];
    __syncthreads();
    if (k0 + CONV_KC < Np) {
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int cfg = cfg0 + wave + 4 * u;
        pre[u] = (cfg < C) ? xrow[(long)cfg * cstride + k0 + CONV_KC] : T(0);
      }
    }
    if (wsite0 < Np) {
#pragma unroll 2
      for (int ks = 0; ks < CONV_KC / 4; ++ks) {
        const int kk = 4 * ks + (lane >> 4);
        T av[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = xs[(16 * a + (lane & 15)) * CONV_LD + kk];
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          // B[k][n] = g(i - i') with i = output site, i' = input site
          const int off = (wsite0 + 16 * n + (lane & 15)) - (k0 + kk) + Np - 1;
          const T bv = ts[off];
#pragma unroll
          for (int a = 0; a < 4; ++a) acc[a][n] = M::mma(av[a], bv, acc[a][n]);
        }
      }
    }
  }
  if (wsite0 >= Np) return;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int cfg = cfg0 + 16 * a + M::row(lane, r);
        const int i = wsite0 + 16 * n + (lane & 15);
        if (cfg < C && i < Np) {
          T y = (i < A.N) ? acc[a][n][r] : T(0);
          if (A.add) y += A.add[(long)(cfg & 1) * cstride + (long)c * Np + i];
          A.Y[(long)cfg * cstride + (long)c * Np + i] = y;
        }
      }
}

// Toeplitz product of float fields on the bf16 matrix cores. Both operands are split into
// three bf16 terms, x = x0 + x1 + x2 (exactly: each term carries the next 8 significant
// bits of what the previous ones left), and the six partial products x_a g_b with
// a + b <= 2 are accumulated in float; the three dropped ones are below 2^-24 of |x g|, the
// rounding unit of a float product, so the result has the error of a float dot product.
// Workgroup: 64 configurations x 64 NT output sites of one channel (4 waves x 16 NT sites).
// The field chunk (64 configurations x 64 input sites) is split into LDS as [3][64][CS_LD];
// the Toeplitz operand uses the reversed taps R[p] = g(Np - 1 - p), split likewise and held
// as eight shifted copies tsh[b][s][q] = R_b[q + s], so that the eight consecutive taps a
// lane needs are one aligned 16-byte read.
constexpr int CS_KC = 64;  // input sites per chunk
constexpr int CS_LD = 72;  // bf16 row stride of the split field chunk (64 + 8: conflict-free rows)

__device__ inline void split3(float v, __bf16& b0, __bf16& b1, __bf16& b2) {
  b0 = (__bf16)v;
  const float r1 = v - (float)b0;
  b1 = (__bf16)r1;
  b2 = (__bf16)(r1 - (float)b1);
}
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
// the same for two values, each bf16 pair formed by one packed conversion
__device__ inline void split3x2(f2v v, bf2& b0, bf2& b1, bf2& b2) {
  b0 = __builtin_convertvector(v, bf2);
  const f2v r1 = v - __builtin_convertvector(b0, f2v);
  b1 = __builtin_convertvector(r1, bf2);
  b2 = __builtin_convertvector(r1 - __builtin_convertvector(b1, f2v), bf2);
}
// NS-term splits (NS = 1: the value rounded to bf16; 2: hi + lo, 16 significant bits; 3: exact)
template <int NS> __device__ inline void splitn(float v, __bf16* b) {
  if constexpr (NS == 3) {
    split3(v, b[0], b[1], b[2]);
  } else {
    b[0] = (__bf16)v;
    if constexpr (NS == 2) b[1] = (__bf16)(v - (float)b[0]);
  }
}
template <int NS> __device__ inline void splitnx2(f2v v, bf2* b) {
  if constexpr (NS == 3) {
    split3x2(v, b[0], b[1], b[2]);
  } else {
    b[0] = __builtin_convertvector(v, bf2);
    if constexpr (NS == 2) b[1] = __builtin_convertvector(v - __builtin_convertvector(b[0], f2v), bf2);
  }
}

// NS: bf16 terms per operand: 3 (exact split, float32 error bound, six partial products) or
// 2 (hi + lo, 16 significant bits, three partial products: the BF16-mixed mode).
template <int NT, int NS = 3>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv_split_kernel(ConvArgs<float> A) {
  static_assert(NS == 2 || NS == 3, "two or three bf16 terms");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* xs = reinterpret_cast<__bf16*>(smem_raw);  // [NS][CONV_MC][CS_LD]
  __bf16* tsh = xs + NS * CONV_MC * CS_LD;           // [NS][8][TL]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.y;
  const int C = A.dyn.count(A.C);
  const int nblk = (C + CONV_MC - 1) / CONV_MC;  // blocks of 64 configurations
  if ((int)blockIdx.x >= nblk) return;
  // copy length: 2 Np - 1 taps and room for the last 8-wide read; 16 mod 64 (Np a multiple
  // of 64) puts the eight shifted copies on different banks for the reads of 8 lanes
  const int Np = A.Np, TL = 2 * Np + 16;
  const int wsite0 = blockIdx.z * 64 * NT + wave * 16 * NT;  // this wave's first output site
  {
    // tp[-p] = g(Np - 1 - p) = R[p], p = 0 .. 2 Np - 2 (zero beyond); every thread requests
    // its entries before splitting any
    const float* tp = A.taps + (long)c * tap_stride(Np) + tap_off(Np) + Np - 1;
    constexpr int PER = 8;  // entries per thread and pass
    for (int base = 0; base < 8 * TL; base += 256 * PER) {
      float v[PER];
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int idx = base + e * 256 + threadIdx.x;
        const int s = idx / TL, p = idx - s * TL + s;
        v[e] = (idx < 8 * TL && p <= 2 * Np - 2) ? tp[-p] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int idx = base + e * 256 + threadIdx.x;
        if (idx < 8 * TL) {
          __bf16 b[NS];
          splitn<NS>(v[e], b);
#pragma unroll
          for (int q = 0; q < NS; ++q) tsh[q * 8 * TL + idx] = b[q];  // idx = s TL + q
        }
      }
    }
  }
  const long cstride = (long)A.DP * Np;
  // staging: thread t moves sites 4 (t mod 16) .. + 3 of configuration rows t / 16 + 16 u.
  // The workgroup runs over configuration blocks blockIdx.x, blockIdx.x + gridDim.x, ...
  // (the split taps are built once), each in chunks of CS_KC input sites; the chunks are
  // numbered in that order and each is requested two chunks ahead, alternating between two
  // register buffers
  const int srow = threadIdx.x >> 4, scol = 4 * (threadIdx.x & 15);
  const int nk = Np / CS_KC;
  const int nmine = (nblk - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x;
  const int nchunk = nmine * nk;
  // buffer resource over the configuration rows cfg0 .. min(cfg0 + 64, C) - 1 of channel c
  // (the last row's channel segment ends the byte range); on = false: an empty range.
  // Requests outside the range read zeros, so every chunk issues the same four requests and
  // the wait for a chunk's data is a fixed count (its barriers order LDS only)
  auto rows_rsrc = [&](const float* base, int cfg0, bool on) __attribute__((always_inline)) {
    const int nrow = min(C - cfg0, CONV_MC);
    const int nbytes = on ? (int)(((long)(nrow - 1) * cstride + Np) * 4) : 0;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base + (long)cfg0 * cstride + (long)c * Np), 0, nbytes, BUF_DW3);
  };
  auto fetch = [&](float4 (&p)[4], int ci) __attribute__((always_inline)) {
    const bool on = ci < nchunk;
    const int blk = on ? blockIdx.x + (ci / nk) * gridDim.x : blockIdx.x, k0 = (ci % nk) * CS_KC;
    const auto rx = rows_rsrc(A.X, blk * CONV_MC, on);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      p[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rx, (int)(((long)(srow + 16 * u) * cstride + k0 + scol) * 4), 0, 0));
  };
  // matrix-core column j of output tile n is site wsite0 + NT j + n, so that a lane's NT
  // tiles hold NT consecutive sites and 16 lanes a contiguous row segment of one
  // configuration (full-line stores). B operand of tile n: R[p + e] with p = p0 + k0 + 32 ks;
  // k0 and 32 ks are multiples of 8, so the shifted copy (p0 mod 8) and a per-lane base are
  // fixed
  int tbase[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int p0 = Np - 1 - (wsite0 + NT * (lane & 15) + n) + 8 * (lane >> 4);
    const int sh = p0 & 7;
    tbase[n] = sh * TL + p0 - sh;
  }
  float4 preA[4], preB[4];
  fetch(preA, 0);
  fetch(preB, 1);
  f4 acc[4][NT];
  auto chunk = [&](float4 (&p)[4], int ci) __attribute__((always_inline)) {
    const int blk = blockIdx.x + (ci / nk) * gridDim.x, k0 = (ci % nk) * CS_KC;
    const int cfg0 = blk * CONV_MC;
    if (k0 == 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[a][n] = f4{0, 0, 0, 0};
    }
    lds_barrier();  // the previous chunk is consumed (and the taps are in place)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      bf2 a[NS], b[NS];
      splitnx2<NS>(f2v{p[u].x, p[u].y}, a);
      splitnx2<NS>(f2v{p[u].z, p[u].w}, b);
      typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
      __bf16* d = xs + (srow + 16 * u) * CS_LD + scol;
#pragma unroll
      for (int q = 0; q < NS; ++q) *reinterpret_cast<bf4*>(d + q * CONV_MC * CS_LD) = bf4{a[q][0], a[q][1], b[q][0], b[q][1]};
    }
    lds_barrier();
    fetch(p, ci + 2);
    if (wsite0 < Np) {
      // A: configuration rows 16 mt + (lane mod 16), sites 32 ks + 8 (lane / 16) + e
      auto lda = [&](int b, int ks, int mt) {
        return *reinterpret_cast<const bf8*>(xs + (b * CONV_MC + 16 * mt + (lane & 15)) * CS_LD + 32 * ks + 8 * (lane >> 4));
      };
      // B: g(i - k) for output site i = wsite0 + NT (lane mod 16) + n and the lane's 8
      // input sites k = k0 + 32 ks + 8 (lane / 16) + e, i.e. R[p + e]
      auto ldb = [&](int b, int ks, int n) {
        return *reinterpret_cast<const bf8*>(tsh + b * 8 * TL + tbase[n] + k0 + 32 * ks);
      };
      bf8 xa[NS][4], tb[NS][NT];
#pragma unroll
      for (int b = 0; b < NS; ++b) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) xa[b][mt] = lda(b, 0, mt);
#pragma unroll
        for (int n = 0; n < NT; ++n) tb[b][n] = ldb(b, 0, n);
      }
      // the products of a step (six or three), smallest first; an operand term is replaced by
      // the next step's as soon as its last product of this step is issued
#pragma unroll
      for (int ks = 0; ks < CS_KC / 32 && NS == 2; ++ks) {
        const bool more = ks + 1 < CS_KC / 32;
#pragma unroll
        for (int term = 0; term < 3; ++term) {
          const int ta = term == 0 ? 1 : 0, tg = term == 1 ? 1 : 0;
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[mt][n] = mma_bf16(xa[ta][mt], tb[tg][n], acc[mt][n]);
          if (more) {
            if (term == 0) {
#pragma unroll
              for (int mt = 0; mt < 4; ++mt) xa[1 % NS][mt] = lda(1, ks + 1, mt);
            } else if (term == 1) {
#pragma unroll
              for (int n = 0; n < NT; ++n) tb[1 % NS][n] = ldb(1, ks + 1, n);
            } else {
#pragma unroll
              for (int mt = 0; mt < 4; ++mt) xa[0][mt] = lda(0, ks + 1, mt);
#pragma unroll
              for (int n = 0; n < NT; ++n) tb[0][n] = ldb(0, ks + 1, n);
            }
          }
        }
      }
#pragma unroll
      for (int ks = 0; ks < CS_KC / 32 && NS == 3; ++ks) {
        const bool more = ks + 1 < CS_KC / 32;
#pragma unroll
        for (int term = 0; term < 6; ++term) {
          const int ta = (term == 0 ? 2 : term == 1 ? 1 : term == 2 ? 0 : term == 3 ? 1 : 0) % NS;
          const int tg = (term == 0 ? 0 : term == 1 ? 1 : term == 2 ? 2 : term == 3 ? 0 : term == 4 ? 1 : 0) % NS;
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[mt][n] = mma_bf16(xa[ta][mt], tb[tg][n], acc[mt][n]);
          if (more) {
            if (term == 0) {
#pragma unroll
              for (int mt = 0; mt < 4; ++mt) xa[2 % NS][mt] = lda(2, ks + 1, mt);
            } else if (term == 2) {
#pragma unroll
              for (int n = 0; n < NT; ++n) tb[2 % NS][n] = ldb(2, ks + 1, n);
            } else if (term == 3) {
#pragma unroll
              for (int mt = 0; mt < 4; ++mt) xa[1][mt] = lda(1, ks + 1, mt);
            } else if (term == 4) {
#pragma unroll
              for (int n = 0; n < NT; ++n) tb[1][n] = ldb(1, ks + 1, n);
            } else if (term == 5) {
#pragma unroll
              for (int mt = 0; mt < 4; ++mt) xa[0][mt] = lda(0, ks + 1, mt);
#pragma unroll
              for (int n = 0; n < NT; ++n) tb[0][n] = ldb(0, ks + 1, n);
            }
          }
        }
      }
    }
    if (k0 + CS_KC >= Np && wsite0 < Np) {
      // accumulator (mt, n) entry r: configuration 16 mt + 4 (lane / 16) + r, site
      // wsite0 + NT (lane mod 16) + n (the wave's sites all lie below Np)
      const int i0 = wsite0 + NT * (lane & 15);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int cfg = cfg0 + 16 * a + 4 * (lane >> 4) + r;
          if (cfg >= C) continue;
          float y[NT];
#pragma unroll
          for (int n = 0; n < NT; ++n) y[n] = (i0 + n < A.N) ? acc[a][n][r] : 0.f;
          const long o = (long)cfg * cstride + (long)c * Np + i0;
          if (A.add) {
#pragma unroll
            for (int n = 0; n < NT; ++n) y[n] += A.add[(long)(cfg & 1) * cstride + (long)c * Np + i0 + n];
          }
          if constexpr (NT == 4) {
            *reinterpret_cast<float4*>(A.Y + o) = make_float4(y[0], y[1], y[2], y[3]);
          } else {
#pragma unroll
            for (int n = 0; n < NT; ++n) A.Y[o + n] = y[n];
          }
        }
    }
  };
  for (int ci = 0; ci < nchunk; ci += 2) {
    chunk(preA, ci);
    if (ci + 1 < nchunk) chunk(preB, ci + 1);
  }
}

// ---------------------------------------------------------------------------------------
// Vertex and channel mixing, fused with the read-out. One workgroup per configuration,
// one wave per 64-site block; a wave's 16 matrix-core columns j and 4 tiles n cover sites
// 64 w + 4 j + n, so every lane moves 4 consecutive sites as one vector.
//   phase 1: q = M1 X (matrix cores), x = elementwise(q, ...) in place in the accumulators;
//   phase 2: y = M2 x, one 16-channel output tile at a time, written out and contracted
//            with the read-out weights.
// The contraction of phase 2 runs over the channels in accumulator order: at step (mi, r)
// the lanes of group kq hold channel 16 mi + row(lane, r) of their sites, which is a valid
// operand B for the matrix cores when operand A (M2) is gathered with the same channel per
// lane group, so x never leaves the registers.
// Modes:
//   FWD:  X = v, x = chi * q (q = V v cached as p0 when requested), y = h = U x;
//         out = h (+ phi^(l+1) when injected) as the next mixer input; rho += Wk . h.
//   TAU:  X = Wk[k] (cfg = 2b + k), or the field X[2b + k] when given, x = chi0[b] * (U^T X),
//         y = V^T x  (the adjoint D0^T of a block applied to the read-out weights or to the
//         next block's output link; a conv with reversed taps then gives G^T D0^T X).
// The per-flip blocks of ABACUS run in deep_kernel.
enum { MIX_FWD = 0, MIX_TAU = 1 };

template <typename T> struct MixArgs {
  Tables<T> tb;
  int N, Np, l, L, w_c, periodic, inject;
  int C;                 // configurations (flips) in this launch
  int cfg0;              // global index of the first (flips: offset in the flip map)
  const T* X;            // [C][DP][Np] (FWD; deep blocks after the first)
  const T* chi;          // FWD: [C][DP][Np]; TAU/deep: chi0 of the block [Bc][DP][Np]
  const T* p0;           // deep: V v0 of the block [Bc][DP][Np]
  T* p0_out;             // FWD cache of q (nullable)
  const T* phi_next;     // FWD inject: phi^(l+1) [C][DP][Np]
  T* out;                // [C][DP][Np] (unused by the last deep block)
  double* rho;           // FWD: [C][2] accumulated; deep: [L-1][Fa][Np/64][2] per block and tile
  long rho_blk;          // deep: doubles between the blocks' parts of rho (Fa Np/64 2)
  T* R_acc;              // FWD: residual sum R += h (nullable)
  // deep blocks (per flip)
  CfgMap map;            // flip -> (b, m)
  int b0;                // first sample of the chunk (caches are chunk-local)
  const int8_t* spins;
  const int4* geom;      // [F] (clo, ext, j0, j1)
  const T* dchi;         // [F][L][Wmax][DP]
  int Wmax;
  const T* tau;          // [Bc][2][DP][Np]
  const T* tapsL;        // taps of block L [DP][tap_stride] (last block)
  const T* taps1;        // taps of block 1 [DP][tap_stride] (first block)
  const T* p0L;          // last block: V v0 of block L [Bc][DP][Np]
  const double* Om0;     // last block: [B][2]
  double* logratio;      // last block: [B][M_max] ([B][M_max][2] with a complex read-out)
  double* dom;           // last block, nullable: [B][M_max][2] the output changes dOmega
  DynRange dyn;          // flips counted on the device (nullable)
  T* slice_part;         // last block: [F][Np/64][SLICE_WIN][DP] partial slices
  int cplx;              // 1: complex read-out unit Omega_0 + i Omega_1
  int tok;               // spins per token (spins: [B][N * tok]; geom's flip sites index spins)
  const T* dphi;         // phi injected: dphi^(l) on S_l [F][L][Wmax][DP] (slice recompute)
};

constexpr int MIX_XS = 68;      // LDS row stride of a wave tile (64 sites + 4; gradient kernels)
constexpr int SLICE_WIN = 16;   // slice positions handled by the last block's window

template <typename T> struct V4 { T v[4]; };
template <typename T> __device__ inline V4<T> ld4(const T* p) {
  V4<T> r;
  if constexpr (sizeof(T) == 4) {
    float4 f = *reinterpret_cast<const float4*>(p);
    r.v[0] = f.x; r.v[1] = f.y; r.v[2] = f.z; r.v[3] = f.w;
  } else {
#pragma unroll
    for (int n = 0; n < 4; ++n) r.v[n] = p[n];
  }
  return r;
}
// ld4 as a streaming (non-temporal) load, for fields read once
template <typename T> __device__ inline V4<T> ld4_stream(const T* p) {
  V4<T> r;
  if constexpr (sizeof(T) == 4) {
    const f4 f = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
#pragma unroll
    for (int n = 0; n < 4; ++n) r.v[n] = f[n];
  } else {
#pragma unroll
    for (int n = 0; n < 4; ++n) r.v[n] = __builtin_nontemporal_load(p + n);
  }
  return r;
}
template <typename T> __device__ inline void st4(T* p, const T* v) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int n = 0; n < 4; ++n) p[n] = v[n];
  }
}
// the same into global memory as a streaming (non-temporal) store, for fields that are not
// read again before they leave L2
template <typename T> __device__ inline void st4_stream(T* p, const T* v) {
  if constexpr (sizeof(T) == 4) {
    __builtin_nontemporal_store(f4{v[0], v[1], v[2], v[3]}, reinterpret_cast<f4*>(p));
  } else {
#pragma unroll
    for (int n = 0; n < 4; ++n) __builtin_nontemporal_store(v[n], p + n);
  }
}

// Wave-scope ordering of LDS traffic between lanes of one wave.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// BF (float fields only): both channel-mixing products on the bf16 matrix cores with float
// accumulation; each operand is split into hi + lo bf16 terms as it is formed (16 significant
// bits) and the three partial products hi*hi, hi*lo, lo*hi are accumulated (fields stay float).
template <typename T, int DP, int MODE, bool BF>
__global__ __launch_bounds__(512) void mix_kernel(MixArgs<T> A) {
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MT = DP / 16, KS = DP / 4;
  __shared__ double red[2][8];
  const int g = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int N = A.N, Np = A.Np, l = A.l;
  const int j = lane & 15, kq = lane >> 4;
  const long fo = (long)g * DP * Np;
  int b = 0, kk_tau = 0;
  if (MODE == MIX_TAU) { b = g >> 1; kk_tau = g & 1; }
  const long bo = (long)b * DP * Np;
  const T* M1 = (MODE == MIX_TAU) ? A.tb.Um + (long)l * DP * DP : A.tb.Vt + (long)l * DP * DP;
  const T* M2 = (MODE == MIX_TAU) ? A.tb.Vm + (long)l * DP * DP : A.tb.Ut + (long)l * DP * DP;
  const int s0 = 64 * wave + 4 * j;  // first of this lane's 4 sites
  const T* X = (MODE == MIX_TAU) ? (A.X ? A.X + fo : A.tb.Wk + (long)kk_tau * DP * Np) : A.X + fo;
  // ---- phase 1
  acc_t acc[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[mt][n] = acc_t{0, 0, 0, 0};
  if constexpr (BF) {
    // k-step s covers channels 32 s + 8 kq + e on lane group kq
#pragma unroll
    for (int s = 0; s < DP / 32; ++s) {
      V4<T> xv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xv[e] = ld4(X + (long)(32 * s + 8 * kq + e) * Np + s0);
      bf8 bb[2][4];
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 h[2];
          splitn<2>(xv[e].v[n], h);
          bb[0][n][e] = h[0];
          bb[1][n][e] = h[1];
        }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        bf8 af[2];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 h[2];
          splitn<2>(M1[(32 * s + 8 * kq + e) * DP + 16 * mt + j], h);
          af[0][e] = h[0];
          af[1][e] = h[1];
        }
        // hi * lo and lo * hi first, then hi * hi
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          acc[mt][n] = mma_bf16(af[1], bb[0][n], acc[mt][n]);
          acc[mt][n] = mma_bf16(af[0], bb[1][n], acc[mt][n]);
          acc[mt][n] = mma_bf16(af[0], bb[0][n], acc[mt][n]);
        }
      }
    }
  } else {
#pragma unroll 4
    for (int ks = 0; ks < KS; ++ks) {
      const int kc = 4 * ks + kq;
      const V4<T> v = ld4(X + (long)kc * Np + s0);
      T af[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) af[mt] = M1[kc * DP + 16 * mt + j];
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt][n] = M::mma(af[mt], v.v[n], acc[mt][n]);
    }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ch = 16 * mt + M::row(lane, r);
      const long o = (long)ch * Np + s0;
      T q[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) q[n] = acc[mt][n][r];
      const V4<T> c = ld4(A.chi + (MODE == MIX_FWD ? fo : bo) + o);
      if (MODE == MIX_FWD && A.p0_out) st4(A.p0_out + fo + o, q);
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[mt][n][r] = (s0 + n < N) ? c.v[n] * q[n] : T(0);
    }
  // BF: x as hi + lo bf16 operands of phase 2, in accumulator channel order (step s:
  // channels 16 (2 s + e / 4) + row(lane, e mod 4))
  bf8 xh[BF ? 2 : 1][BF ? DP / 32 : 1][4];
  if constexpr (BF) {
#pragma unroll
    for (int s = 0; s < DP / 32; ++s)
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 h[2];
          splitn<2>(acc[2 * s + (e >> 2)][n][e & 3], h);
          xh[0][s][n][e] = h[0];
          xh[1][s][n][e] = h[1];
        }
  }
  // ---- phase 2, one 16-channel output tile at a time
  double part0 = 0.0, part1 = 0.0;
#pragma unroll 1
  for (int mo = 0; mo < MT; ++mo) {
    acc_t a2[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) a2[n] = acc_t{0, 0, 0, 0};
    if constexpr (BF) {
#pragma unroll
      for (int s = 0; s < DP / 32; ++s) {
        bf8 af[2];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 h[2];
          splitn<2>(M2[(16 * (2 * s + (e >> 2)) + M::row(lane, e & 3)) * DP + 16 * mo + j], h);
          af[0][e] = h[0];
          af[1][e] = h[1];
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          a2[n] = mma_bf16(af[1], xh[0][s][n], a2[n]);
          a2[n] = mma_bf16(af[0], xh[1][s][n], a2[n]);
          a2[n] = mma_bf16(af[0], xh[0][s][n], a2[n]);
        }
      }
    } else {
#pragma unroll
      for (int mi = 0; mi < MT; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T af = M2[(16 * mi + M::row(lane, r)) * DP + 16 * mo + j];
#pragma unroll
          for (int n = 0; n < 4; ++n) a2[n] = M::mma(af, acc[mi][n][r], a2[n]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ch = 16 * mo + M::row(lane, r);
      const long o = (long)ch * Np + s0;
      T y[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) y[n] = (s0 + n < N) ? a2[n][r] : T(0);
      if (MODE == MIX_TAU) {
        st4(A.out + fo + o, y);
      } else {
        const V4<T> w0 = ld4(A.tb.Wk + o), w1 = ld4(A.tb.Wk + (long)DP * Np + o);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          part0 += (double)w0.v[n] * (double)y[n];
          part1 += (double)w1.v[n] * (double)y[n];
        }
        if (A.R_acc) {
          V4<T> rr = ld4(A.R_acc + fo + o);
#pragma unroll
          for (int n = 0; n < 4; ++n) rr.v[n] += y[n];
          st4(A.R_acc + fo + o, rr.v);
        }
        if (A.out) {
          if (A.inject) {
            const V4<T> ph = ld4(A.phi_next + fo + o);
#pragma unroll
            for (int n = 0; n < 4; ++n) y[n] += ph.v[n];
          }
          st4(A.out + fo + o, y);
        }
      }
    }
  }
  if (MODE == MIX_TAU) return;
  part0 = wave_sum(part0);
  part1 = wave_sum(part1);
  if (lane == 0) { red[0][wave] = part0; red[1][wave] = part1; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r0 = 0.0, r1 = 0.0;
    for (int w = 0; w < nw; ++w) { r0 += red[0][w]; r1 += red[1][w]; }
    A.rho[2 * g] += r0;
    A.rho[2 * g + 1] += r1;
  }
}

// ---------------------------------------------------------------------------------------
// Deep blocks of the ABACUS background propagation: du^(l+1) = D0^(l) G^(l) du^(l) + z^(l)
// on the full chain, x = chi0 q + [i in S_l] dchi (p0 + q) with q = V w, w = G^(l) du (the
// perturbation through the frozen vertex plus the vertex change on the slice), one 64-site
// tile per wave step. Block 1 builds q from the unit-flip table Pq instead of reading w.
// Each wave walks its tiles with the next tile's input already in flight while the current
// one is mixed. Flips are dealt out per XCD in contiguous ranges (workgroup w runs on XCD
// w mod 8), so the flips of one sample, which share their background caches, meet in the
// same L2; within an XCD every workgroup keeps one tile position t and runs over flips.
// Each tile's read-out is stored (not accumulated) in the block's part of rho[l][f][t].
// Every workgroup keeps both channel-mixing matrices in LDS in fragment order (every
// operand read is one contiguous 64-lane access), and, before the last block, the read-out
// weights omega / N of its tile position and A. Blocks before the last store du. The
// last block (LAST) instead reads out dh with Wk + tau and forms, per tile, the partial
// slice of the last mixer's output, part[f][t][s][c] = sum_{i' in tile} g^(L)_c(site_s - i')
// dh[c][i'], 32 channels at a time from a channel-major copy in LDS (row stride DH_LD, odd,
// so the per-channel reads hit distinct banks): lane (c, h) runs channel c over the h-th
// part of the tile's sites with a register window over the taps, and the parts are added
// across lanes. last_finish_kernel completes the flip.
constexpr int DEEP_WAVES = 4;
constexpr int NXCD = 8;
// waves per SIMD each variant's register budget is sized for (the last block's LDS holds it
// to two workgroups per CU in any case; three-term bf16 operands need the room of two)
constexpr int deep_occ(int elem_bytes, bool prefetch, bool last, int bf) {
  return elem_bytes == 4 && !prefetch && !last && bf < 2 ? 3 : 2;
}
// bytes of LDS the weight fragments of a deep block take: F1 (not in the first block), F2
constexpr int deep_wbytes(int DP, int elem_bytes, bool first, int bf) {
  return (first ? 1 : 2) * DP * DP * (bf ? 2 * bf : elem_bytes);
}

constexpr bool DEEP_PF = true;  // register prefetch of the next tile in the blocks between first and last
constexpr int DH_LD = 65;
constexpr int DH_CH = 32;  // channels of the last block's LDS copy per group
// LAST: channels of the LDS copy of dh per slice group (16 with three-term operands, whose
// weight fragments take half as much LDS again)
constexpr int deep_cpg(int DP, int bf) { return DP < (bf == 3 ? 16 : DH_CH) ? DP : (bf == 3 ? 16 : DH_CH); }

// BF (float fields only; the number of bf16 terms per operand, 0 = float matrix cores):
// both channel-mixing products on the bf16 matrix cores with float accumulation, the weight
// fragments held in LDS as bf16 terms; the partial products x_a v_b with a + b <= BF - 1 are
// accumulated, smallest first. BF = 1: operands rounded to bf16. BF = 2 (the BF16-mixed
// mode): hi + lo terms (16 significant bits), three partial products, relative error of a
// product below 2^-15. BF = 3: x = x0 + x1 + x2 exactly and six partial products, which keeps
// the error bound of a float product (the dropped ones are below 2^-24 |x v|).
// NU (last block, float): slice positions the partial slices cover, at least the widest
// slice S_L of the launch (the others keep SLICE_WIN).
template <typename T, int DP, bool FIRST, bool LAST, int BF, int NU = SLICE_WIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(deep_occ(sizeof(T), DEEP_PF && !FIRST && !LAST, LAST, BF)))) void deep_kernel(MixArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MT = DP / 16, KS = DP / 4, KB = DP / 32;
  // the next tile's input is prefetched into registers unless that would not fit
  constexpr bool PF = DEEP_PF && !FIRST && !LAST && KS * 4 * sizeof(T) <= 256;
  constexpr bool BFM = BF != 0;     // bf16 matrix cores
  constexpr int NS = BFM ? BF : 1;  // bf16 terms per operand
  static_assert(BF >= 0 && BF <= 3, "one to three bf16 terms");
  static_assert(NU == SLICE_WIN || (LAST && sizeof(T) == 4 && NU >= 1 && NU < SLICE_WIN), "narrow partial slices: last block, float");
  // LDS: F1 (not in the first block), F2, then the last block's per-wave copies of dh or
  // the other blocks' read-out weights (sized by the host in launch_deep)
  constexpr int WB1 = deep_wbytes(DP, sizeof(T), true, BF);  // bytes of one weight matrix
  T* F1 = reinterpret_cast<T*>(smem_raw);                                  // [KS][64][MT]: operand A of V, phase 1
  T* F2 = reinterpret_cast<T*>(smem_raw + (FIRST ? 0 : WB1));              // [MT][MT][64][4]: operand A of U, phase 2
  T* tail_s = reinterpret_cast<T*>(smem_raw + (FIRST ? 1 : 2) * WB1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kq = lane >> 4;
  constexpr int CPG = deep_cpg(DP, BF);            // LAST: channels per slice group
  T* dh = tail_s + wave * CPG * DH_LD;             // LAST: this wave's [CPG][DH_LD] copy
  T* om_s = tail_s;                                // not LAST: omega / N [DP][64] of tile t
  double* ac_s = reinterpret_cast<double*>(om_s + DP * 64);  // not LAST: A^T [2][DP], float64
  const int N = A.N, Np = A.Np, l = A.l;
  const int nt = Np / 64;
  const int xcd = blockIdx.x % NXCD, bx = blockIdx.x / NXCD, nbx = gridDim.x / NXCD;
  const int t = bx % nt;  // this workgroup's tile position (the host makes nbx a multiple of nt)
  const bool full = 64 * t + 64 <= N;  // no site of the tile lies past the chain end
  constexpr bool MXI = !FIRST && !LAST;
  const T* Vt = A.tb.Vt + (long)(l - 1) * DP * DP;
  const T* Ut = A.tb.Ut + (long)(l - 1) * DP * DP;
  __bf16* F1h = reinterpret_cast<__bf16*>(F1);  // BF: [NS][KB][MT][64][8]
  __bf16* F2h = reinterpret_cast<__bf16*>(F2);  // BF: [NS][MT][KB][64][8]
  if constexpr (BFM)
  for (int idx = threadIdx.x; idx < DP * DP; idx += blockDim.x) {
    const int e = idx & 7, ln = (idx >> 3) & 63, hi = idx >> 9;
    __bf16 b[3];
    if (!FIRST) {
      const int mt = hi % MT, sk = hi / MT;
      const float v = Vt[(32 * sk + 8 * (ln >> 4) + e) * DP + 16 * mt + (ln & 15)];
      splitn<NS>(v, b);
#pragma unroll
      for (int q = 0; q < NS; ++q) F1h[q * DP * DP + idx] = b[q];
    }
    const int sk = hi % KB, mo = hi / KB;
    const float v = Ut[(16 * (2 * sk + (e >> 2)) + M::row(ln, e & 3)) * DP + 16 * mo + (ln & 15)];
    splitn<NS>(v, b);
#pragma unroll
    for (int q = 0; q < NS; ++q) F2h[q * DP * DP + idx] = b[q];
  }
  else
  for (int idx = threadIdx.x; idx < DP * DP; idx += blockDim.x) {
    if (!FIRST) {  // the first block reads its phase-1 product from a table
      const int mt = idx % MT, ln = (idx / MT) % 64, ks = idx / (MT * 64);
      F1[idx] = Vt[(4 * ks + (ln >> 4)) * DP + 16 * mt + (ln & 15)];
    }
    {
      // phase 2 contracts over the channels in accumulator order (see mix_kernel)
      // lanes 16 bytes apart: the four r entries of a lane are one conflict-free vector read
      const int r = idx & 3, ln = (idx >> 2) & 63, mi = (idx >> 8) % MT, mo = (idx >> 8) / MT;
      F2[idx] = Ut[(16 * mi + M::row(ln, r)) * DP + 16 * mo + (ln & 15)];
    }
  }
  if constexpr (!LAST) {
    for (int idx = threadIdx.x; idx < DP * 64; idx += blockDim.x)
      om_s[idx] = A.tb.omN[(long)(idx >> 6) * Np + 64 * t + (idx & 63)];
    for (int idx = threadIdx.x; idx < 2 * DP; idx += blockDim.x) ac_s[idx] = (double)A.tb.Ac[idx];
  }
  __syncthreads();  // the only workgroup barrier: the waves run independently from here
  const int F = A.dyn.count(A.C);
  const int cfg0 = A.dyn.first(A.cfg0);
  // flips of this XCD: [g_lo, g_hi); the nbx / nt workgroups of tile position t share them
  const int perF = (F + NXCD - 1) / NXCD;
  const int g_hi = min(F, xcd * perF + perF);
  const int gstride = (nbx / nt) * DEEP_WAVES;
  int g = xcd * perF + (bx / nt) * DEEP_WAVES + wave;
  const int TO = tap_off(Np), TS = tap_stride(Np);
  // Addresses are a per-lane base plus an offset that is the same for every lane (kept in
  // scalar registers), so that no per-lane 64-bit offsets stay live across the tile loop.
  const int lrow = M::lane_row(lane);
  // input row of slot ks on this lane: kq_row + urow(ks) (bf16 steps take 8 rows per lane group)
  const int kq_row = BFM ? 8 * kq : kq;
  auto urow = [](int ks) { return BFM ? 32 * (ks >> 3) + (ks & 7) : 4 * ks; };
  V4<T> xb[PF ? KS : 1];
  // with the input also the tile's background gate chi0 is fetched one tile ahead (float
  // operands only: it does not fit the register budget of the other variants)
  constexpr bool PFC = PF && !BFM && sizeof(T) == 4;
  // split variants: the gate is requested while phase 1 runs (after the first block
  // half of it when the tile starts and half once the first half of the input is consumed;
  // in the first block all of it, ahead of the table reads)
  constexpr bool EC = BF >= 2 && sizeof(T) == 4;
  V4<T> cb[PFC || EC ? MT * 4 : 1];
  // without that prefetch (the last block, float) the whole input tile is requested at once
  // when the tile starts, so its latency is met once rather than at every step
  constexpr bool XL = !PF && !FIRST && sizeof(T) == 4;
  V4<T> xl[XL ? KS : 1];
  auto prefetch = [&](int gq) {
    const T* src = A.X + (long)gq * DP * Np + 64 * t + kq_row * Np + 4 * j;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) xb[ks] = ld4_stream(src + urow(ks) * Np);
    if constexpr (PFC) {
      const T* cs = A.chi + (long)(A.map.cb[cfg0 + gq] - A.b0) * DP * Np + (long)lrow * Np + 64 * t + 4 * j;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) cb[mt * 4 + r] = ld4(cs + (16 * mt + M::r_row(r)) * Np);
    }
  };
  if (PF && g < g_hi) prefetch(g);
  for (; g < g_hi; g += gstride) {
    // compiler-only barrier: the weight operands are reloaded per tile rather than hoisted
    // out of the loop into registers (which would halve the occupancy)
    asm volatile("" ::: "memory");
    const int4 sg = A.geom[g];
    const int bglob = A.map.cb[cfg0 + g];
    const long fo = (long)g * DP * Np, bo = (long)(bglob - A.b0) * DP * Np;
    const int s0 = 64 * t + 4 * j;
    const long lo_off = (long)lrow * Np + s0;  // this lane's part of a field offset
    // ---- phase 1: q = V w
    acc_t acc[MT][4];
    if constexpr (FIRST) {
      // w = G^(1) e^(0) with e^(0)_c = -2 s_z E_c at the cluster sites z, so
      // q(i) = -2 s_z Pq(i - z) summed over the cluster (Pq: parameter-only table)
      // (with tokens: the flipped spin's token z and its position's table Pq_k)
      const int8_t* sp = A.spins + (long)bglob * N * A.tok;
      const T c0 = (T)(-2 * sp[sg.z]);
      const bool pair = sg.w >= 0;
      const T c1 = pair ? (T)(-2 * sp[sg.w]) : T(0);
      const int za = sg.z / A.tok, ka = sg.z - za * A.tok;
      const int jw = pair ? sg.w : sg.z, z1 = jw / A.tok, kb = jw - z1 * A.tok;
      // the copy shifted by (TO - z) mod 4 makes the four sites one aligned vector
      const int shz = (TO - za) & 3, shw = (TO - z1) & 3;
      const long PK = 4L * DP * TS;
      const T* pz = A.tb.Pq + ka * PK + ((long)shz * DP + lrow) * TS + TO + s0 - za - shz;
      const T* pw = A.tb.Pq + kb * PK + ((long)shw * DP + lrow) * TS + TO + s0 - z1 - shw;
      if constexpr (EC) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) cb[mt * 4 + r] = ld4(A.chi + bo + lo_off + (16 * mt + M::r_row(r)) * Np);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int uo = (16 * mt + M::r_row(r)) * TS;
          const V4<T> vz = ld4(pz + uo);
          V4<T> vw{};
          if (pair) vw = ld4(pw + uo);
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[mt][n][r] = c0 * vz.v[n] + c1 * vw.v[n];
          if (r == 3) __builtin_amdgcn_sched_barrier(0);
        }
    } else if constexpr (BFM) {
      if constexpr (XL) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) xl[ks] = ld4_stream(A.X + fo + kq_row * Np + urow(ks) * Np + s0);
      }
      auto fetch_chi = [&](int m0, int m1) {
#pragma unroll
        for (int mt = m0; mt < m1; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) cb[mt * 4 + r] = ld4(A.chi + bo + lo_off + (16 * mt + M::r_row(r)) * Np);
      };
      if constexpr (EC) fetch_chi(0, MT / 2);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[mt][n] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int sk = 0; sk < KB; ++sk) {
        bf8 bb[NS][4];
        // slots e and e + 1 of a lane's operand are one 32-bit word: converted together
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          V4<T> v[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int ks = 8 * sk + e + h;
            if constexpr (PF) v[h] = xb[ks];
            else if constexpr (XL) v[h] = xl[ks];
            else v[h] = ld4_stream(A.X + fo + kq_row * Np + urow(ks) * Np + s0);
          }
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            const f2v pr{v[0].v[n], v[1].v[n]};
            bf2 bq[NS];
            splitnx2<NS>(pr, bq);
#pragma unroll
            for (int q = 0; q < NS; ++q) { bb[q][n][e] = bq[q][0]; bb[q][n][e + 1] = bq[q][1]; }
          }
        }
        if constexpr (EC) {
          if (sk == (KB == 1 ? 0 : KB / 2 - 1)) fetch_chi(MT / 2, MT);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          bf8 af[NS];
#pragma unroll
          for (int q = 0; q < NS; ++q) af[q] = reinterpret_cast<const bf8*>(F1h + q * DP * DP)[(sk * MT + mt) * 64 + lane];
          // partial products a + b <= NS - 1, smallest first
#pragma unroll
          for (int sum = NS - 1; sum >= 0; --sum)
#pragma unroll
            for (int a = 0; a <= sum; ++a)
#pragma unroll
              for (int n = 0; n < 4; ++n) acc[mt][n] = mma_bf16(af[a], bb[sum - a][n], acc[mt][n]);
        }
      }
    } else {
      if constexpr (XL) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) xl[ks] = ld4_stream(A.X + fo + kq * Np + 4 * ks * Np + s0);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[mt][n] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kc = 4 * ks + kq;
        T bv[4];
        if constexpr (PF) {
#pragma unroll
          for (int n = 0; n < 4; ++n) bv[n] = xb[ks].v[n];
        } else if constexpr (XL) {
#pragma unroll
          for (int n = 0; n < 4; ++n) bv[n] = xl[ks].v[n];
        } else {
          const V4<T> v = ld4_stream(A.X + fo + kq * Np + 4 * ks * Np + s0);
#pragma unroll
          for (int n = 0; n < 4; ++n) bv[n] = v.v[n];
        }
        T af[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) af[mt] = F1[(ks * 64 + lane) * MT + mt];
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][n] = M::mma(af[mt], bv[n], acc[mt][n]);
        // keep the scheduler from hoisting every later operand load (register pressure)
        if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    // ---- x = chi0 q + [i in S_l] dchi (p0 + q)
    // slice positions of this lane's four sites (-1: outside S_l); the same for every channel
    int sidx[4];
    {
      const int lo = sg.x - l * A.w_c, W = sg.y + 2 * l * A.w_c + 1;
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        int sx = s0 + n - lo;
        if (A.periodic) { sx %= N; if (sx < 0) sx += N; }
        sidx[n] = (s0 + n < N && sx >= 0 && sx < W) ? sx : -1;
      }
    }
    const bool in_slice = sidx[0] >= 0 || sidx[1] >= 0 || sidx[2] >= 0 || sidx[3] >= 0;
    const T* dchi_l = A.dchi + ((long)g * A.L + (l - 1)) * A.Wmax * DP;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ch = 16 * mt + M::row(lane, r);
        const int uo = (16 * mt + M::r_row(r)) * Np;  // lane-independent part of the offset
        V4<T> c;
        if constexpr (PFC || EC) c = cb[mt * 4 + r];
        else c = ld4(A.chi + bo + lo_off + uo);
        T x[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) x[n] = c.v[n] * acc[mt][n][r];
        if (in_slice) {
          // the four sites' operands requested together (a site outside S_l reads the
          // vertex change at position 0 and weights it by zero)
          const V4<T> pv = ld4(A.p0 + bo + lo_off + uo);
          T dv[4];
#pragma unroll
          for (int n = 0; n < 4; ++n) dv[n] = dchi_l[max(sidx[n], 0) * DP + ch];
#pragma unroll
          for (int n = 0; n < 4; ++n) x[n] += (sidx[n] >= 0 ? dv[n] : T(0)) * (pv.v[n] + acc[mt][n][r]);
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[mt][n][r] = (!MXI || s0 + n < N) ? x[n] : T(0);
        if (r == 3) __builtin_amdgcn_sched_barrier(0);
      }
    // sites past the chain end hold zeros (only the workgroups of the last tile position
    // have any; the blocks between first and last mask as they go, since their register
    // budget has no room for this separate pass)
    if (!MXI && !full) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[mt][n][r] = (s0 + n < N) ? acc[mt][n][r] : T(0);
    }
    // the next tile's input travels while this one is mixed and stored
    if (PF && g + gstride < g_hi) prefetch(g + gstride);
    // BF: x as bf16 operands of phase 2, in accumulator channel order (step sk: channels
    // 16 (2 sk + e / 4) + row(lane, e mod 4))
    bf8 xh[BFM ? NS : 1][BFM ? KB : 1][4];
    if constexpr (BFM) {
#pragma unroll
      for (int sk = 0; sk < KB; ++sk)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            // slots e, e + 1: accumulator entries r, r + 1 of one tile, converted together
            const f2v pr{acc[2 * sk + (e >> 2)][n][e & 3], acc[2 * sk + (e >> 2)][n][(e & 3) + 1]};
            bf2 bq[NS];
            splitnx2<NS>(pr, bq);
#pragma unroll
            for (int q = 0; q < NS; ++q) { xh[q][sk][n][e] = bq[q][0]; xh[q][sk][n][e + 1] = bq[q][1]; }
          }
    }
    // ---- phase 2 per 16-channel output tile: du = U x, stored, and read out
    double part0 = 0.0, part1 = 0.0;
    int loL = 0;
    if (LAST) {
      loL = sg.x - A.L * A.w_c;
      if (A.periodic) { loL %= N; if (loL < 0) loL += N; }
    }
    constexpr int GM = LAST ? CPG / 16 : 1;  // output tiles per group
    // LAST, float: lane (c, hp) of the slice below takes channel c over the tile sites
    // hp K .. hp K + K - 1 (K = CPG); the taps it needs, h(u - k) for those sites k and
    // u < NU, are fetched into registers before the group's products
    constexpr bool TPR = LAST && sizeof(T) == 4;
    constexpr int NTP = TPR ? CPG + NU - 1 : 1;
    static_assert(!LAST || CPG == 16 || CPG == 32, "the tile's parts are lanes 16 or 32 apart");
#pragma unroll 1
    for (int mg = 0; mg < MT; mg += GM) {
      T tp[NTP];  // tp[m] = tc[m - (K - 1) - hp K], tc the window of the slice below
      if constexpr (TPR) {
        const int c = lane % CPG, hp = lane / CPG;
        const T* tc = A.tapsL + (long)(16 * mg + c) * TS + TO + loL - 64 * t - hp * CPG - (CPG - 1);
#pragma unroll
        for (int m = 0; m < NTP; ++m) tp[m] = tc[m];
      }
#pragma unroll 1
      for (int mo = mg; mo < mg + GM; ++mo) {
        // LAST, float: the read-out weights tau of this output tile travel during its products
        constexpr bool TWP = LAST && sizeof(T) == 4;
        V4<T> tw[TWP ? 8 : 1];
        if constexpr (TWP) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const long o = 2 * bo + lo_off + (16 * mo + M::r_row(r)) * Np;
            tw[2 * r] = ld4(A.tau + o);
            tw[2 * r + 1] = ld4(A.tau + (long)DP * Np + o);
          }
        }
        acc_t a2[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) a2[n] = acc_t{0, 0, 0, 0};
        if constexpr (BFM) {
#pragma unroll
          for (int sk = 0; sk < KB; ++sk) {
            bf8 af[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) af[q] = reinterpret_cast<const bf8*>(F2h + q * DP * DP)[(mo * KB + sk) * 64 + lane];
#pragma unroll
            for (int sum = NS - 1; sum >= 0; --sum)
#pragma unroll
              for (int a = 0; a <= sum; ++a)
#pragma unroll
                for (int n = 0; n < 4; ++n) a2[n] = mma_bf16(af[a], xh[sum - a][sk][n], a2[n]);
          }
        } else {
#pragma unroll
          for (int mi = 0; mi < MT; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const T af = F2[((mo * MT + mi) * 64 + lane) * 4 + r];
#pragma unroll
              for (int n = 0; n < 4; ++n) a2[n] = M::mma(af, acc[mi][n][r], a2[n]);
              if (r == 3) __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long o = lo_off + (16 * mo + M::r_row(r)) * Np;
          // sites past the chain end: x is zero there, so du is too
          T y[4];
#pragma unroll
          for (int n = 0; n < 4; ++n) y[n] = a2[n][r];
          if constexpr (LAST) {
            // read-out with Wk + tau (tau already carries Wk when L >= 2)
            V4<T> w0, w1;
            if constexpr (TWP) {
              w0 = tw[2 * r];
              w1 = tw[2 * r + 1];
            } else {
              w0 = ld4(A.tau + 2 * bo + o);
              w1 = ld4(A.tau + 2 * bo + (long)DP * Np + o);
            }
            // the lane's four sites in the field precision, the tile's sum in float64
            T s0w = 0, s1w = 0;
#pragma unroll
            for (int n = 0; n < 4; ++n) {
              s0w += w0.v[n] * y[n];
              s1w += w1.v[n] * y[n];
            }
            part0 += (double)s0w;
            part1 += (double)s1w;
          } else {
            // read-out with Wk = A^T omega / N: one site vector of omega / N per channel,
            // both from LDS; the lane's four sites in the field precision, the rest in float64
            const int ch = 16 * mo + M::row(lane, r);
            const V4<T> wo = ld4(om_s + ch * 64 + 4 * j);
            T swt = 0;
#pragma unroll
            for (int n = 0; n < 4; ++n) swt += wo.v[n] * y[n];
            const double sw = (double)swt;
            part0 += ac_s[ch] * sw;
            part1 += ac_s[DP + ch] * sw;
          }
          if (LAST) {
            const int cl = 16 * (mo - mg) + M::row(lane, r);
#pragma unroll
            for (int n = 0; n < 4; ++n) dh[cl * DH_LD + 4 * j + n] = y[n];
            __builtin_amdgcn_sched_barrier(0);
          } else {
            st4_stream(A.out + fo + o, y);
          }
        }
      }
      if (LAST) {
        // partial slice of the last mixer's output from this tile and channel group; the
        // window holds h(x) = g^(L)(loL + x): tc[u - k] = h(u - ib - k)
        wave_sync();
        constexpr int NPART = 64 / CPG, K = CPG;  // lanes (c, h): sites h K .. h K + K - 1
        const int c = lane % CPG, hp = lane / CPG, cg = 16 * mg + c;
        const int ib = 64 * t, cnt = min(64, N - ib), k0 = hp * K;
        T ya[NU], rg[SLICE_WIN];
#pragma unroll
        for (int u = 0; u < NU; ++u) ya[u] = 0;
        if constexpr (TPR) {
          // every site of the tile: those past the chain end hold zeros
          const T* xr = dh + c * DH_LD + k0;
#pragma unroll
          for (int kk = 0; kk < K; ++kk) {
            const T v = xr[kk];
#pragma unroll
            for (int u = 0; u < NU; ++u) ya[u] += tp[u - kk + K - 1] * v;
          }
        } else {
          // float64: a sliding register window over the taps
          const T* tc = A.tapsL + (long)cg * TS + TO + loL - ib;
#pragma unroll
          for (int u = 0; u < SLICE_WIN; ++u) rg[u] = tc[u - k0];
          const T* xr = dh + c * DH_LD;
          for (int kb = k0; kb < k0 + K && kb < cnt; kb += SLICE_WIN) {
#pragma unroll
            for (int u = 0; u < SLICE_WIN; ++u) {
              const int k = kb + u;
              if (k < cnt) {
                const T v = xr[k];
#pragma unroll
                for (int tt = 0; tt < SLICE_WIN; ++tt) ya[tt] += rg[(tt - u + SLICE_WIN * 4) % SLICE_WIN] * v;
                rg[(SLICE_WIN * 4 - u - 1) % SLICE_WIN] = tc[-(k + 1)];
              }
            }
          }
        }
        // the parts of the tile (lanes CPG apart) are added with row swaps
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          if constexpr (CPG <= 16) ya[u] = swap_sum<16>(ya[u]);
          ya[u] = swap_sum<32>(ya[u]);
        }
        {
          // every part holds the sums after the row swaps: lane (c, hp) stores the rows
          // u = hp, hp + NPART, ... of channel cg
          T* pp = A.slice_part + ((long)g * nt + t) * SLICE_WIN * DP + cg;
#pragma unroll
          for (int u0 = 0; u0 < NU; u0 += NPART) {
            T v = ya[u0];
#pragma unroll
            for (int q = 1; q < NPART; ++q)
              if (u0 + q < NU) v = (hp == q) ? ya[u0 + q] : v;
            if (u0 + hp < NU) pp[(u0 + hp) * DP] = v;
          }
        }
        wave_sync();  // the copy in LDS is free for the next group
      }
    }
    part0 = wave_sum(part0);
    part1 = wave_sum(part1);
    if (lane == 0) {
      double* rp = A.rho + (long)(l - 1) * A.rho_blk + ((long)g * nt + t) * 2;
      rp[0] = part0;
      rp[1] = part1;
    }
  }
}

// Finishes each flip after the tiled last block (one wave per flip): sums the tiles' partial
// slices into y_L, forms e^(L) = U (dchi^(L) * (p0^(L) + V y_L)) on S_L, reads out e^(L)
// and e^(0), adds the deep blocks' read-outs rho[l][f][t] and writes
// log psi(s')/psi(s) = sum_k lcd(Omega0_k, dOmega_k) in float64 (complex read-out: put_ratio).
// INJ (phi injected into the h stream, Fig. 1c): the input change of block L is
// dh^(L-1) + dphi^(L); the tiled block read dh^(L-1) out and mixed it, here the dphi^(L) part
// joins y_L (its mixer output on S_L, the taps g^(L)(t - t') of slice positions t, t') and
// the read-out through tau = G^(L)T D0^(L)T Wk alone (phi is not part of the residual sum).
// With one block there is no tiled block: the input change is e^(0) + dphi^(1), all of it
// taken here (no partial slices).
// e^(0) of channel c at the q-th flipped spin of a cluster (zero for an absent second spin):
// -2 s_j E_(k(j), c), k(j) the spin's position in its token.
template <typename T, int DP>
__device__ inline T inj_e0(const MixArgs<T>& A, int4 sg, int bg, int q, int c) {
  const int js = q == 0 ? sg.z : sg.w;
  if (js < 0) return T(0);
  return (T)(-2 * A.spins[(long)bg * A.N * A.tok + js]) * A.tb.E[(js % A.tok) * DP + c];
}

template <typename T, int DP, bool INJ = false>
__global__ __launch_bounds__(64) void last_finish_kernel(MixArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MT = DP / 16, KS = DP / 4;
  const int g = blockIdx.x;
  if (g >= A.dyn.count(A.C)) return;
  const int cfg0 = A.dyn.first(A.cfg0);
  const int lane = threadIdx.x, j = lane & 15, kq = lane >> 4;
  const int N = A.N, Np = A.Np, nt = Np / 64;
  const int4 sg = A.geom[g];
  const int bg = A.map.cb[cfg0 + g], m = A.map.cm[cfg0 + g];
  const long bL = (long)(bg - A.b0) * DP * Np;
  int loL = sg.x - A.L * A.w_c;
  const int WL = sg.y + 2 * A.L * A.w_c + 1;
  if (A.periodic) { loL %= N; if (loL < 0) loL += N; }
  T* Y = reinterpret_cast<T*>(smem_raw);  // [DP][16]: Y[c][t]
  T* X2 = Y + DP * SLICE_WIN;             // [DP][16]
  const T* pp = A.slice_part + (long)g * nt * SLICE_WIN * DP;
  // float: the V operand does not depend on the partials and is requested before them
  constexpr bool VH = sizeof(T) == 4;
  const T* Vt = A.tb.Vt + (long)(A.L - 1) * DP * DP;
  T vf[VH ? KS : 1][VH ? MT : 1];
  if constexpr (VH) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) vf[ks][mt] = Vt[(4 * ks + kq) * DP + 16 * mt + j];
  }
  for (int c = lane; c < DP; c += 64) {
    // a tile's partials are requested together; rows past the slice (which the last block
    // may not have written) re-read its last row and are dropped below
    T s[SLICE_WIN];
#pragma unroll
    for (int t = 0; t < SLICE_WIN; ++t) s[t] = 0;
    for (int tile = 0; tile < ((!INJ || A.L > 1) ? nt : 0); ++tile) {
      T v[SLICE_WIN];
#pragma unroll
      for (int t = 0; t < SLICE_WIN; ++t) v[t] = pp[((long)tile * SLICE_WIN + min(t, WL - 1)) * DP + c];
#pragma unroll
      for (int t = 0; t < SLICE_WIN; ++t) s[t] += v[t];
    }
    if constexpr (INJ) {
      // the channel's taps g^(L)(t - t') for |t - t'| < SLICE_WIN, held in registers
      const T* dp = A.dphi + ((long)g * A.L + (A.L - 1)) * A.Wmax * DP + c;
      const T* tc = A.tapsL + (long)c * tap_stride(Np) + tap_off(Np) - (SLICE_WIN - 1);
      T tw[2 * SLICE_WIN - 1];
#pragma unroll
      for (int k = 0; k < 2 * SLICE_WIN - 1; ++k) tw[k] = tc[k];
      const T ea = A.L == 1 ? inj_e0<T, DP>(A, sg, bg, 0, c) : T(0);
      const T eb = A.L == 1 ? inj_e0<T, DP>(A, sg, bg, 1, c) : T(0);
#pragma unroll
      for (int t2 = 0; t2 < SLICE_WIN; ++t2) {
        if (t2 < WL) {
          T x = dp[(long)t2 * DP];
          if (t2 == A.w_c) x += ea;
          if (t2 == A.w_c + sg.y) x += eb;
#pragma unroll
          for (int t = 0; t < SLICE_WIN; ++t) s[t] += tw[t - t2 + SLICE_WIN - 1] * x;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < SLICE_WIN; ++t) Y[c * SLICE_WIN + t] = (t < WL) ? s[t] : T(0);
  }
  wave_sync();
  const T* Ut = A.tb.Ut + (long)(A.L - 1) * DP * DP;
  acc_t a2[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) a2[mt] = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int kc = 4 * ks + kq;
    const T bvv = Y[kc * SLICE_WIN + j];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) a2[mt] = M::mma(VH ? vf[VH ? ks : 0][VH ? mt : 0] : Vt[kc * DP + 16 * mt + j], bvv, a2[mt]);
  }
  const int t_me = j;  // this lane's slice position (matrix-core column)
  int site = loL + t_me;
  bool valid = t_me < WL;
  if (A.periodic) site %= N;
  else valid = valid && site >= 0 && site < N;
  const T* dchiL = A.dchi + ((long)g * A.L + (A.L - 1)) * A.Wmax * DP;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ch = 16 * mt + M::row(lane, r);
      T x = 0;
      if (valid) x = dchiL[t_me * DP + ch] * (A.p0L[bL + (long)ch * Np + site] + a2[mt][r]);
      X2[ch * SLICE_WIN + t_me] = x;
    }
  wave_sync();
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) a2[mt] = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int kc = 4 * ks + kq;
    const T bvv = X2[kc * SLICE_WIN + j];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) a2[mt] = M::mma(Ut[kc * DP + 16 * mt + j], bvv, a2[mt]);
  }
  double o0 = 0.0, o1 = 0.0;
  if (valid) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ch = 16 * mt + M::row(lane, r);
        const long o = (long)ch * Np + site;
        o0 += (double)A.tb.Wk[o] * (double)a2[mt][r];
        o1 += (double)A.tb.Wk[(long)DP * Np + o] * (double)a2[mt][r];
      }
  }
  // e^(0) = -2 s_j E on the cluster, read out directly (lanes over channels)
  {
    const int8_t* spb = A.spins + (long)bg * N * A.tok;
    for (int q = 0; q < 2; ++q) {
      const int js = q == 0 ? sg.z : sg.w;  // a flipped spin: its token jt, its position jk
      if (js < 0) continue;
      const int jt = js / A.tok, jk = js - jt * A.tok;
      for (int c = lane; c < DP; c += 64) {
        const double e0 = (double)(-2 * spb[js]) * (double)A.tb.E[jk * DP + c];
        o0 += (double)A.tb.Wk[(long)c * Np + jt] * e0;
        o1 += (double)A.tb.Wk[(long)DP * Np + (long)c * Np + jt] * e0;
      }
    }
  }
  if constexpr (INJ) {  // dphi^(L) read out through tau = (Wk + tau) - Wk
    // lanes (channel c0 + lane / 16, slice position lane % 16): contiguous sites per channel
    const T* dp = A.dphi + ((long)g * A.L + (A.L - 1)) * A.Wmax * DP;
    const int t = lane & 15;
    int st = loL + t;
    bool ok = t < WL;
    if (A.periodic) st %= N;
    else ok = ok && st >= 0 && st < N;
    if (ok)
      for (int c = lane >> 4; c < DP; c += 4) {
        const long o = (long)c * Np + st;
        T xz = dp[(long)t * DP + c];
        if (A.L == 1 && t == A.w_c) xz += inj_e0<T, DP>(A, sg, bg, 0, c);
        if (A.L == 1 && t == A.w_c + sg.y) xz += inj_e0<T, DP>(A, sg, bg, 1, c);
        const double x = (double)xz;
        o0 += ((double)A.tau[2 * bL + o] - (double)A.tb.Wk[o]) * x;
        o1 += ((double)A.tau[2 * bL + (long)DP * Np + o] - (double)A.tb.Wk[(long)DP * Np + o]) * x;
      }
  }
  // read-outs of the tiled deep blocks 1 .. L-1, lanes over (block, tile)
  for (int bt = lane; bt < (A.L - 1) * nt; bt += 64) {
    const double* rp = A.rho + (long)(bt / nt) * A.rho_blk + ((long)g * nt + bt % nt) * 2;
    o0 += rp[0];
    o1 += rp[1];
  }
  o0 = wave_sum(o0);
  o1 = wave_sum(o1);
  if (lane == 0) {
    const long o = (long)bg * A.map.M_max + m;
    put_ratio(A.logratio, o, A.Om0[2 * bg], A.Om0[2 * bg + 1], o0, o1, A.cplx);
    if (A.dom) { A.dom[2 * o] = o0; A.dom[2 * o + 1] = o1; }
  }
}

// phi injected into the h stream (Fig. 1c): the input change of block 1 is
// z = e^(0) + dphi^(1) on S_1 (e^(0)_c = -2 s_j E_(k(j), c) at the tokens of the flipped
// spins), and block 1 mixes it: w(i) = sum_(t in S_1) g^(1)(i - site_t) z_t, written as the
// whole field [F][DP][Np] (zero past the chain end) that the mixer would produce from z,
// without forming z as a field. A lane takes four sites of one channel.
constexpr int INJ_W1 = 9;  // widest S_1: a pair cluster two sites wide and w_c = 3
template <typename T, int DP>
__global__ __launch_bounds__(256) void inject_w1_kernel(MixArgs<T> A) {
  const int F = A.dyn.count(A.C), cfg0 = A.dyn.first(A.cfg0);
  const int N = A.N, Np = A.Np, wc = A.w_c, q4 = Np / 4;
  const int TO = tap_off(Np), TS = tap_stride(Np);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // one flip per workgroup step: waves over channels, lanes over four-site groups
  for (int f = blockIdx.x; f < F; f += gridDim.x) {
    const int4 sg = A.geom[f];
    const int W1 = sg.y + 2 * wc + 1, lo = sg.x - wc;
    const int8_t* sp = A.spins + (long)A.map.cb[cfg0 + f] * N * A.tok;
    // slot t holds site lo + t unwrapped (the taps of a ring are periodic; an open chain's
    // slots outside it hold zero); e^(0) sits at the slots of the cluster's tokens, w_c (the
    // first flipped spin's token clo) and w_c + ext (the second's)
    const int t_a = wc, ka = sg.z % A.tok;
    const int t_b = sg.w >= 0 ? wc + sg.y : -1, kb = sg.w >= 0 ? sg.w % A.tok : 0;
    const T ca = (T)(-2 * sp[sg.z]), cbv = sg.w >= 0 ? (T)(-2 * sp[sg.w]) : T(0);
    const T* dp = A.dphi + (long)f * A.L * A.Wmax * DP;  // block 1's slot
    for (int c = wave; c < DP; c += 4) {
      T z[INJ_W1];
#pragma unroll
      for (int t = 0; t < INJ_W1; ++t) {
        T x = t < W1 ? dp[(long)t * DP + c] : T(0);
        if (t == t_a) x += ca * A.tb.E[ka * DP + c];
        if (t == t_b) x += cbv * A.tb.E[kb * DP + c];
        z[t] = x;
      }
      const T* tcc = A.taps1 + (long)c * TS + TO - lo - (INJ_W1 - 1);
      for (int i4 = lane; i4 < q4; i4 += 64) {
        // tw[k] = g^(1)(4 i4 + k - (INJ_W1 - 1) - lo): site 4 i4 + e against slot t at k = e - t + 8
        T tw[INJ_W1 + 3];
        const T* tc = tcc + 4 * i4;
#pragma unroll
        for (int k = 0; k < INJ_W1 + 3; ++k) tw[k] = tc[k];
        T v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          T acc = 0;
#pragma unroll
          for (int t = 0; t < INJ_W1; ++t) acc += tw[e - t + INJ_W1 - 1] * z[t];
          v[e] = 4 * i4 + e < N ? acc : T(0);
        }
        st4(A.out + ((long)f * DP + c) * Np + 4 * i4, v);
      }
    }
  }
}

// phi injected: the input change of block l + 1 is the tiled block's dh^(l) plus
// dphi^(l+1) on S_(l+1); adds the latter to A.out (A.l = l). One flip per workgroup step,
// lanes (channel 4 w + lane / 16 + 16 k, slice position lane % 16): contiguous sites.
template <typename T, int DP>
__global__ __launch_bounds__(256) void inject_add_kernel(MixArgs<T> A) {
  const int F = A.dyn.count(A.C);
  const int N = A.N, Np = A.Np, wc = A.w_c, l1 = A.l + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = lane & 15;
  for (int f = blockIdx.x; f < F; f += gridDim.x) {
    const int4 sg = A.geom[f];
    if (t >= sg.y + 2 * l1 * wc + 1) continue;
    int i = sg.x - l1 * wc + t;
    if (A.periodic) i = ((i % N) + N) % N;
    else if (i < 0 || i >= N) continue;
    const T* dp = A.dphi + (((long)f * A.L + (l1 - 1)) * A.Wmax + t) * DP;
    T* o = A.out + (long)f * DP * Np + i;
    for (int c = 4 * wave + (lane >> 4); c < DP; c += 16) o[(long)c * Np] += dp[c];
  }
}

// ---------------------------------------------------------------------------------------
// Per-flip slice recompute of the phi stream and vertices (ABACUS, Sec. III: the vertex
// changes only on S_l = sites within l*w_c of the cluster). Writes dchi^(l) = chi'^(l) -
// chi0^(l) on S_l for l = 1..L and the cluster geometry (clo, ext, j0, j1): S_l covers sites
// clo - l*w_c .. clo + ext + l*w_c.
template <typename T> struct SliceArgs {
  Tables<T> tb;
  int N, Np, L, w_c, periodic, act;
  int F, f0, b0, Bc;      // flips [f0, f0+F), chunk's first sample b0, samples in chunk
  CfgMap map;
  const int8_t* spins;
  const T* a0;            // [L][Bc][DP][Np]
  const T* chi0;          // [L][Bc][DP][Np]
  T* dchi;                // [F][L][Wmax][DP]
  int4* geom;             // [F]
  int Wmax;
  int* err;               // set to 1 for a cluster the slice recurrence does not cover
  int ext_max;            // widest cluster extent the launch's links were built for
  DynRange dyn;           // flips counted on the device (nullable)
  int tok;                // spins per token (spins: [B][N * tok]; sites index spins)
  const T* phi0;          // phi injected: background phi^(l), l = 1..L [L][Bc][DP][Np]
  T* dphi;                // phi injected: dphi^(l) = phi'^(l) - phi0^(l) on S_l [F][L][Wmax][DP]
};

// The slice recompute with its two channel mixes on the matrix cores. A workgroup takes
// P flips at a time and lays them side by side as the columns of one SLM_CAP-column product
// per mix: block l forms a' = W_D phi'^(l-1) + w on S_{l-1} (block 1: from s'), the phi
// stream on S_l from a' with its background halo, and chi' = g(A_D phi'^(l) + b) on S_l,
// column j = p * W + t for flip p and slice position t (W: the launch's widest slice of
// that block). Wave w owns output channels 16 w .. 16 w + 15 of both products and holds
// those rows of W_D and A_D in registers; the element-wise steps use every thread.
constexpr int SLM_NT = 4;              // 16-column tiles per product
constexpr int SLM_CAP = 16 * SLM_NT;   // columns per product
constexpr int SLM_LDC = SLM_CAP + 17;  // odd LDS row stride of the product operand
constexpr int SLM_GS = 8;              // per flip: b (-1: none), clo, ext, j0, j1, f, c_a, c_b

// Flips per workgroup for slices of at most Wc sites (0: too wide for one product).
__host__ __device__ inline int slm_flips(int Wc) { return SLM_CAP / Wc; }

// Workgroups for G flip groups: a multiple of the XCD count. Workgroup i runs on XCD i % NXCD,
// so group (i % NXCD) * (grid / NXCD) + i / NXCD keeps consecutive groups -- mostly the flips
// of one sample, which read the same per-sample caches -- on one XCD and its L2.
__host__ __device__ inline int slm_grid(int G) { return (G + NXCD - 1) / NXCD * NXCD; }
__device__ inline int slm_group() {
  return (int)(blockIdx.x % NXCD) * (int)(gridDim.x / NXCD) + (int)(blockIdx.x / NXCD);
}

// LDS bytes: phi' [DP][SLM_LDC], a' with halo [DP][lda], geometry [P][SLM_GS].
// (at least SLM_CAP columns, so that a product may also read its operand from this buffer)
__host__ __device__ inline int slm_lda(int P, int Wc, int wc) {
  const int w = P * (Wc + 2 * wc);
  return (w > SLM_CAP ? w : SLM_CAP) | 1;
}
template <typename T> __host__ __device__ inline size_t slm_lds_bytes(int DP, int P, int Wc, int wc) {
  return ((size_t)DP * (SLM_LDC + slm_lda(P, Wc, wc))) * sizeof(T) + (size_t)P * SLM_GS * sizeof(int);
}

// acc[n] = W x over the first NTU column tiles of x (row stride ldx; the other tiles are zero).
template <typename T, int DP, int NTU>
__device__ inline void slm_prod(const T (&w)[DP / 4], const T* x, int ldx, int q, int col,
                                typename Mma<T>::acc (&acc)[SLM_NT]) {
#pragma unroll
  for (int n = 0; n < SLM_NT; ++n) acc[n] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < DP / 4; ++ks)
#pragma unroll
    for (int n = 0; n < NTU; ++n) acc[n] = Mma<T>::mma(w[ks], x[(4 * ks + q) * ldx + 16 * n + col], acc[n]);
}
template <typename T, int DP>
__device__ inline void slm_prod_n(int nt, const T (&w)[DP / 4], const T* x, int ldx, int q, int col,
                                  typename Mma<T>::acc (&acc)[SLM_NT]) {
  switch (nt) {
    case 1: slm_prod<T, DP, 1>(w, x, ldx, q, col, acc); break;
    case 2: slm_prod<T, DP, 2>(w, x, ldx, q, col, acc); break;
    case 3: slm_prod<T, DP, 3>(w, x, ldx, q, col, acc); break;
    default: slm_prod<T, DP, SLM_NT>(w, x, ldx, q, col, acc); break;
  }
}

// This wave's 16 rows of a weight operand table (row = input channel) in operand-A order.
template <typename T, int DP> __device__ inline void slm_rows(const T* Wt, int wave, int lane, T (&w)[DP / 4]) {
#pragma unroll
  for (int ks = 0; ks < DP / 4; ++ks) w[ks] = Wt[(4 * ks + (lane >> 4)) * DP + 16 * wave + (lane & 15)];
}

// Cluster geometry of flips fg .. fg + P - 1 into gs (threads < P; c_a, c_b = -2 s at the
// cluster sites, c_b = 0 for one site). Clusters the slice recurrence does not cover set err.
template <bool TOK, typename T>
__device__ inline void slm_geometry(const SliceArgs<T>& A, int* gs, int P, int fg, int nfl, int f0, bool write_geom) {
  const int N = A.N, L = A.L, wc = A.w_c;
  const bool per = A.periodic != 0;
  const int tid = threadIdx.x;
  if (tid >= P) return;
  const int f = fg + tid;
  int* g = gs + SLM_GS * tid;
  if (f >= nfl) {
    g[0] = -1; g[1] = 0; g[2] = 0; g[3] = -1; g[4] = -1; g[5] = -1; g[6] = 0; g[7] = 0;
    return;
  }
  const int b = A.map.cb[f0 + f], m = A.map.cm[f0 + f];
  const int j0 = A.map.sites[((long)b * A.map.M_max + m) * 2];
  const int j1 = A.map.sites[((long)b * A.map.M_max + m) * 2 + 1];
  // the cluster in tokens: clo its first token, ext its extent; ja flips a spin of token clo,
  // jb (or -1) the other flipped spin, of token clo + ext
  const int tk = TOK ? A.tok : 1, NS = N * tk, z0 = j0 / tk;
  int clo = z0, ext = 0, ja = j0, jb = j1;
  if (j1 >= 0) {
    const int z1 = j1 / tk;
    int ds = j1 > j0 ? j1 - j0 : j0 - j1;  // spin distance: at most 2
    if (per && NS - ds < ds) ds = NS - ds;
    if (ds > 2) {
      ext = -1;
    } else if (per) {
      const int d1 = ((z1 - z0) % N + N) % N, d2 = ((z0 - z1) % N + N) % N;
      if (d1 <= d2) { clo = z0; ext = d1; }
      else { clo = z1; ext = d2; ja = j1; jb = j0; }
    } else if (z1 < z0) {
      clo = z1; ext = z0 - z1; ja = j1; jb = j0;
    } else {
      ext = z1 - z0;
    }
  }
  if (ext < 0 || ext > A.ext_max || (per && ext + 2 * L * wc + 1 > N)) {
    atomicOr(A.err, 1);
    ext = 0;
  }
  if (write_geom) A.geom[f] = make_int4(clo, ext, ja, jb);
  const int8_t* sp = A.spins + (long)b * NS;
  g[0] = b; g[1] = clo; g[2] = ext; g[3] = ja; g[4] = jb; g[5] = f;
  g[6] = -2 * sp[ja];
  g[7] = jb >= 0 ? -2 * sp[jb] : 0;
}

// Blocks 1 .. L of the slice recompute (L = LF when LF > 0). epi(l, n, r, v) receives the
// vertex change v = chi'(l) - chi0(l) of the lane's channel 16 w + row(lane, r) at its
// column 16 n + lane % 16 of S_l (zero for columns that hold no slice site of a flip).
// INJ: the phi-stream change dphi^(l) on S_l is also written (zero outside an open chain).
template <typename T, int DP, int LF, bool TOK, bool INJ = false, typename EPI>
__device__ inline void slm_layers(const SliceArgs<T>& A, T* ph, T* ab, const int* gs, int P, int lda, EPI&& epi) {
  constexpr int NTH = 4 * DP;
  const int N = A.N, Np = A.Np, wc = A.w_c;
  const int L = LF > 0 ? LF : A.L;
  const int Wc = A.ext_max + 2 * L * wc + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool per = A.periodic != 0;
  auto wrap = [&](int i) { if (per) { i %= N; if (i < 0) i += N; } return i; };
  auto inside = [&](int i) { return per || (i >= 0 && i < N); };
  using M = Mma<T>;
  using acc_t = typename M::acc;
  const int col = lane & 15, q = lane >> 4;
  const int AW = Wc + 2 * wc;  // a' block of a flip (the widest)
#pragma unroll
  for (int l = 1; l <= (LF > 0 ? LF : A.L); ++l) {
    const int lp = l - 1;
    const int WPm = A.ext_max + 2 * lp * wc + 1;  // column stride of S_{l-1}
    const int Wlm = WPm + 2 * wc;                 // column stride of S_l
    // this wave's rows of the block's weights, requested first
    T wa[DP / 4], wd[DP / 4];
    slm_rows<T, DP>(A.tb.ADt + (long)lp * DP * DP, wave, lane, wa);
    if (l > 1) slm_rows<T, DP>(A.tb.WDt + (long)lp * DP * DP, wave, lane, wd);
    // the lane's output columns of the A_D product (flip, slice position) and the background
    // gate of its channels there
    int pq[SLM_NT], tq[SLM_NT];
    T c0v[SLM_NT][4];
#pragma unroll
    for (int n = 0; n < SLM_NT; ++n) {
      const int j = 16 * n + col;
      int p = j / Wlm, t = j - p * Wlm;
      bool ok = p < P;
      const int* g = gs + SLM_GS * (ok ? p : 0);
      ok = ok && g[0] >= 0 && t < g[2] + 2 * l * wc + 1;
      const int ii = g[1] - l * wc + t;
      const int site = ok && inside(ii) ? wrap(ii) : g[1];
      const int bb = g[0] >= 0 ? g[0] - A.b0 : 0;
      pq[n] = ok ? p : -1;
      tq[n] = t;
      const T* chi0 = A.chi0 + ((long)lp * A.Bc + bb) * DP * Np + site;
#pragma unroll
      for (int r = 0; r < 4; ++r) c0v[n][r] = chi0[(long)(16 * wave + M::row(lane, r)) * Np];
    }
    // a' on S_{l-1} at block columns 2 w_c + t
    if (l == 1) {
      const int nt1 = A.ext_max + 1;
#pragma unroll 2
      for (int idx = tid; idx < DP * P * nt1; idx += NTH) {
        const int c = idx % DP, pt = idx / DP;
        const int p = pt / nt1, t = pt - p * nt1;
        const int* g = gs + SLM_GS * p;
        if (g[0] < 0 || t > g[2]) continue;
        const int site = wrap(g[1] + t);  // a token of the cluster
        T v = 0;
        if (inside(g[1] + t)) {
          const int tk = TOK ? A.tok : 1, s0 = site * tk;
          const int8_t* sr = A.spins + (long)g[0] * N * tk + s0;
          T sv = (T)sr[0];
          if (s0 == g[3] || s0 == g[4]) sv = -sv;
          v = sv * A.tb.wE1[c] + A.tb.wv[c];
          for (int k = 1; k < tk; ++k) {
            T sk = (T)sr[k];
            if (s0 + k == g[3] || s0 + k == g[4]) sk = -sk;
            v += sk * A.tb.wE1[k * DP + c];
          }
        }
        ab[c * lda + p * AW + 2 * wc + t] = v;
      }
    } else {
      acc_t acc[SLM_NT];
      slm_prod_n<T, DP>((P * WPm + 15) / 16, wd, ph, SLM_LDC, q, col, acc);
#pragma unroll
      for (int n = 0; n < SLM_NT; ++n) {
        const int j = 16 * n + col;
        const int p = j / WPm, t = j - p * WPm;
        if (p < P) {
          const int* g = gs + SLM_GS * p;
          const int WP = g[2] + 2 * lp * wc + 1;
          const int lo = g[1] - lp * wc;
          if (g[0] >= 0 && t < WP) {
            const bool in = inside(lo + t);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ch = 16 * wave + M::row(lane, r);
              ab[ch * lda + p * AW + 2 * wc + t] = in ? acc[n][r] + A.tb.wv[lp * DP + ch] : T(0);
            }
          }
        }
      }
    }
    // the background halo: 2 w_c sites on either side of S_{l-1}
    {
      const int nh = 4 * wc;
#pragma unroll 4
      for (int idx = tid; idx < DP * P * nh; idx += NTH) {
        const int c = idx % DP, hp = idx / DP;
        const int p = hp / nh, h = hp - p * nh;
        const int* g = gs + SLM_GS * p;
        if (g[0] < 0) continue;
        const int WP = g[2] + 2 * lp * wc + 1;
        const int u = h < 2 * wc ? h : WP + h;
        const int jj = g[1] - lp * wc - 2 * wc + u;  // block column 0 is site clo - (l + 1) w_c
        ab[c * lda + p * AW + u] =
            inside(jj) ? A.a0[(((long)lp * A.Bc + (g[0] - A.b0)) * DP + c) * Np + wrap(jj)] : T(0);
      }
    }
    __syncthreads();
    // phi' on S_l: thread (channel c, part k) takes columns k, k + 4, ... of the channel;
    // the channel's taps in registers (w_c <= 3)
    {
      const int c = tid % DP, part = tid / DP;
      T kr[7];
#pragma unroll
      for (int u = 0; u < 7; ++u) kr[u] = u <= 2 * wc ? A.tb.Kc[((long)lp * (2 * wc + 1) + u) * DP + c] : T(0);
      const T kv = A.tb.kv[lp * DP + c];
      const T* ar = ab + c * lda;
      T* pr = ph + c * SLM_LDC;
      for (int j = part; j < P * Wlm; j += 4) {
        const int p = j / Wlm, t = j - p * Wlm;
        const int* g = gs + SLM_GS * p;
        if (g[0] < 0 || t >= g[2] + 2 * l * wc + 1) continue;
        const T* a = ar + p * AW + t;
        T sacc = kv;
#pragma unroll
        for (int u = 0; u < 7; ++u)
          if (u <= 2 * wc) sacc += kr[u] * a[u];
        const int ii = g[1] - l * wc + t;
        const T v = inside(ii) ? act_fn<T>(A.act, sacc) : T(0);
        pr[j] = v;
        if constexpr (INJ) {
          const T v0 = inside(ii) ? A.phi0[(((long)lp * A.Bc + (g[0] - A.b0)) * DP + c) * Np + wrap(ii)] : T(0);
          A.dphi[(((long)g[5] * A.L + lp) * A.Wmax + t) * DP + c] = v - v0;
        }
      }
    }
    __syncthreads();
    // chi' and dchi = chi' - chi0 on S_l
    {
      acc_t acc[SLM_NT];
      slm_prod_n<T, DP>((P * Wlm + 15) / 16, wa, ph, SLM_LDC, q, col, acc);
#pragma unroll
      for (int n = 0; n < SLM_NT; ++n) {
        const bool ok = pq[n] >= 0;
        const int* g = gs + SLM_GS * (ok ? pq[n] : 0);
        const bool in = ok && inside(g[1] - l * wc + tq[n]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ch = 16 * wave + M::row(lane, r);
          epi(l, n, r, in ? act_fn<T>(A.act, acc[n][r] + A.tb.bv[lp * DP + ch]) - c0v[n][r] : T(0));
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int DP, bool INJ = false>
__global__ __launch_bounds__(4 * DP) void slice_mma_kernel(SliceArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int Wc = A.ext_max + 2 * A.L * A.w_c + 1;  // widest S_L of the launch
  const int P = slm_flips(Wc);
  const int lda = slm_lda(P, Wc, A.w_c);
  T* ph = reinterpret_cast<T*>(smem_raw);      // phi' [DP][SLM_LDC], column p * W + t
  T* ab = ph + DP * SLM_LDC;                   // a' [DP][lda], flip p at columns p * AW ..
  int* gs = reinterpret_cast<int*>(ab + DP * lda);
  const int nfl = A.dyn.count(A.F);
  const int fg = slm_group() * P;
  if (fg >= nfl) return;
  slm_geometry<true>(A, gs, P, fg, nfl, A.dyn.first(A.f0), true);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, wc = A.w_c;
  slm_layers<T, DP, 0, true, INJ>(A, ph, ab, gs, P, lda, [&](int l, int n, int r, T v) {
    const int Wlm = A.ext_max + 2 * l * wc + 1;
    const int j = 16 * n + col;
    const int p = j / Wlm, t = j - p * Wlm;
    if (p >= P) return;
    const int* g = gs + SLM_GS * p;
    if (g[0] < 0 || t >= g[2] + 2 * l * wc + 1) return;
    const int ch = 16 * wave + Mma<T>::row(lane, r);
    A.dchi[(((long)g[5] * A.L + (l - 1)) * A.Wmax + t) * DP + ch] = v;
  });
}

}  // namespace dn
