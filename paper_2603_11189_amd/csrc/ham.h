// Hamiltonian connected elements, local energy and the work lists of the estimator.
#pragma once
#include "common.h"

namespace dn {

// Diagonal pair weights of the Ising chain: Jr[r] = c_zz / dist(r)^alpha for r = 1..N-1,
// with c_zz = J (plain form) or -2 J / N_alpha (the paper's Kac-normalised form; the sum over
// ordered pairs i != j counts each unordered pair twice), N_alpha = 2 sum_{r<=N/2} r^-alpha.
__global__ void ising_table_kernel(int N, int periodic, double J, double alpha, int paper_form,
                                   double* __restrict__ Jr) {
  const int t = threadIdx.x;
  double kac = 0.0;
  for (int r = 1 + t; r <= N / 2; r += WAVE) kac += pow((double)r, -alpha);
  kac = 2.0 * wave_sum(kac);
  const double czz = paper_form ? -2.0 * J / kac : J;
  for (int r = t; r < N; r += WAVE) {
    int dist = r;
    if (periodic && N - r < dist) dist = N - r;
    Jr[r] = (r == 0) ? 0.0 : czz / pow((double)dist, alpha);
  }
}

// One wave per sample. Ising: element m flips site m, helem = c_x (h or -h), and
// hdiag = sum_{i<j} Jr[j-i] s_i s_j. J1-J2: bonds (i, i+delta), delta = 1, 2, in the order
// i = 0..N-1 then delta; antiparallel bonds are emitted (ballot + prefix count keeps the
// order) with element J_delta/2; hdiag = sum over bonds of (J_delta/4) s_i s_j.
__global__ __launch_bounds__(64) void connected_kernel(int kind, int periodic, double cx_elem,
                                                       double J1, double J2,
                                                       const double* __restrict__ Jr,
                                                       const int8_t* __restrict__ spins, int N,
                                                       int M_max, int32_t* __restrict__ sites,
                                                       double* __restrict__ helem,
                                                       int32_t* __restrict__ n_conn,
                                                       double* __restrict__ hdiag) {
  const int b = blockIdx.x, t = threadIdx.x;
  const int8_t* s = spins + (long)b * N;
  int32_t* st = sites + (long)b * M_max * 2;
  double* he = helem + (long)b * M_max;
  for (int m = t; m < M_max; m += WAVE) { st[2 * m] = -1; st[2 * m + 1] = -1; he[m] = 0.0; }
  __syncthreads();
  double e = 0.0;
  if (kind == 0) {
    for (int i = t; i < N; i += WAVE) {
      double acc = 0.0;
      for (int j = i + 1; j < N; ++j) acc += Jr[j - i] * (double)(s[j]);
      e += acc * (double)s[i];
      st[2 * i] = i;
      he[i] = cx_elem;
    }
    e = wave_sum(e);
    if (t == 0) { n_conn[b] = N; hdiag[b] = e; }
    return;
  }
  int base = 0;
  for (int i0 = 0; i0 < N; i0 += WAVE) {
    const int i = i0 + t;
    int f1 = 0, f2 = 0, j1 = -1, j2 = -1;
    if (i < N) {
      j1 = i + 1; j2 = i + 2;
      if (j1 >= N) j1 = periodic ? j1 - N : -1;
      if (j2 >= N) j2 = periodic ? j2 - N : -1;
      if (j1 >= 0) { e += 0.25 * J1 * s[i] * s[j1]; f1 = s[i] != s[j1]; }
      if (j2 >= 0) { e += 0.25 * J2 * s[i] * s[j2]; f2 = s[i] != s[j2]; }
    }
    int cnt = f1 + f2;
    // inclusive prefix over the wave
    int inc = cnt;
    for (int off = 1; off < WAVE; off <<= 1) {
      int v = __shfl_up(inc, off, WAVE);
      if (t >= off) inc += v;
    }
    int pos = base + inc - cnt;
    if (f1) { if (pos < M_max) { st[2 * pos] = i; st[2 * pos + 1] = j1; he[pos] = 0.5 * J1; } ++pos; }
    if (f2) { if (pos < M_max) { st[2 * pos] = i; st[2 * pos + 1] = j2; he[pos] = 0.5 * J2; } }
    base += __shfl(inc, WAVE - 1, WAVE);
  }
  e = wave_sum(e);
  if (t == 0) { n_conn[b] = base < M_max ? base : M_max; hdiag[b] = e; }
}

// E_loc = hdiag + sum_{m < n_conn} helem_m exp(logratio_m), one wave per sample. cplx = 1: the
// log-ratios are complex (re, im pairs) and so is E_loc ([B][2]).
__global__ __launch_bounds__(64) void eloc_kernel(const double* __restrict__ hdiag,
                                                  const double* __restrict__ helem,
                                                  const int32_t* __restrict__ n_conn,
                                                  const double* __restrict__ lr, int M_max,
                                                  double* __restrict__ eloc, int cplx) {
  const int b = blockIdx.x, t = threadIdx.x;
  const int n = n_conn[b];
  double acc = 0.0, acc_i = 0.0;
  if (cplx) {
    for (int m = t; m < n; m += WAVE) {
      const long o = (long)b * M_max + m;
      const double mag = helem[o] * exp(lr[2 * o]);
      acc += mag * cos(lr[2 * o + 1]);
      acc_i += mag * sin(lr[2 * o + 1]);
    }
    acc_i = wave_sum(acc_i);
  } else {
    for (int m = t; m < n; m += WAVE) acc += helem[(long)b * M_max + m] * exp(lr[(long)b * M_max + m]);
  }
  acc = wave_sum(acc);
  if (t == 0) {
    if (cplx) {
      eloc[2 * b] = hdiag[b] + acc;
      eloc[2 * b + 1] = acc_i;
    } else {
      eloc[b] = hdiag[b] + acc;
    }
  }
}

// Work list: for each sample b, (with_base ? 1 : 0) + n_conn[b] entries (b, m), m = -1 for the
// unflipped sample; offs[b] = first entry of sample b, offs[B] = total. The inputs are
// validated on the way (the host reads offs[B+1] before any other launch): offs[B+1] gets bit
// 1 if some n_conn is outside [0, M_max], bit 2 if a listed site is outside the chain (the
// second site may be -1, and must differ from the first), bit 8 if a spin is not +-1
// (spin_check_kernel). plan_kernel (one block) counts and
// scans; plan_fill_kernel (one thread per (sample, slot)) writes the entries, checks the
// sites (bit 2 of the error word) and notes whether any cluster has two sites (bit 4).
__global__ __launch_bounds__(1024) void plan_kernel(const int32_t* __restrict__ n_conn, int B, int M_max,
                                                    int with_base, int32_t* __restrict__ offs) {
  __shared__ int part[1024];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  const int per = (B + 1023) / 1024;
  const int b0 = t * per, b1 = min(B, b0 + per);
  int cnt = 0;
  for (int b = b0; b < b1; ++b) {
    int n = n_conn[b];
    if (n < 0 || n > M_max) { atomicOr(&bad, 1); n = n < 0 ? 0 : M_max; }
    cnt += with_base + n;
  }
  part[t] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int pos = part[t] - cnt;
  for (int b = b0; b < b1; ++b) {
    int n = n_conn[b];
    n = n < 0 ? 0 : (n > M_max ? M_max : n);
    offs[b] = pos;
    pos += with_base + n;
  }
  if (t == 1023) { offs[B] = part[1023]; offs[B + 1] = bad; }
}

__global__ void plan_fill_kernel(const int32_t* __restrict__ n_conn, const int32_t* __restrict__ sites, int B,
                                 int N, int M_max, int with_base, int32_t* __restrict__ offs,
                                 int32_t* __restrict__ cb, int32_t* __restrict__ cm) {
  const int S = M_max + with_base;  // slots per sample
  bool any_pair = false;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)B * S; i += (long)gridDim.x * blockDim.x) {
    const int b = (int)(i / S), slot = (int)(i % S);
    int n = n_conn[b];
    n = n < 0 ? 0 : (n > M_max ? M_max : n);
    if (slot >= with_base + n) continue;
    const int pos = offs[b] + slot, m = slot - with_base;
    cb[pos] = b;
    cm[pos] = m;
    if (m >= 0) {
      const int j0 = sites[((long)b * M_max + m) * 2], j1 = sites[((long)b * M_max + m) * 2 + 1];
      if (j0 < 0 || j0 >= N || j1 < -1 || j1 >= N || j1 == j0) atomicOr(&offs[B + 1], 2);
      any_pair = any_pair || j1 >= 0;
    }
  }
  // bit 4: the list holds two-site clusters (one request per wave)
  if (__ballot(any_pair) && (threadIdx.x & 63) == 0) atomicOr(&offs[B + 1], 4);
}

// Bit 8 of the work list's error word when a spin is neither +1 nor -1 (one request per wave).
__global__ void spin_check_kernel(const int8_t* __restrict__ spins, long n, int32_t* __restrict__ err) {
  bool bad = false;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int v = spins[i];
    bad = bad || (v != 1 && v != -1);
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(err, 8);
}

// Probe configurations for launch tuning: spin i = +-1 from the low bit of a 32-bit integer
// hash of (i, seed) (a multiply-xorshift mixer); only timings are taken from them.
__global__ void probe_spins_kernel(int8_t* __restrict__ spins, long n, uint32_t seed) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i * 2654435761u ^ seed;
    x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
    spins[i] = (x & 1u) ? 1 : -1;
  }
}

// Identity work list: entry b is sample b, unflipped.
__global__ void identity_map_kernel(int32_t* __restrict__ cb, int32_t* __restrict__ cm, int B) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    cb[b] = b;
    cm[b] = -1;
  }
}

template <typename T> __global__ void fill_kernel(T* __restrict__ x, long n, T v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}

// log psi = sum_k logcosh(Omega_k) (or the complex unit's log cosh, cplx = 1) for B samples
// whose Omega sits at rows idx[b] (or b).
__global__ void logpsi_kernel(const double* __restrict__ Om, const int32_t* __restrict__ idx, int B,
                              double* __restrict__ logpsi, int cplx) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    const int r = idx ? idx[b] : b;
    put_logpsi(logpsi, b, Om[2 * r], Om[2 * r + 1], cplx);
  }
}

// Plain path: logratio[b, m] = sum_k lcd(Omega(s)_k, Omega(s'_m)_k - Omega(s)_k).
__global__ void plain_ratio_kernel(const double* __restrict__ Om, const int32_t* __restrict__ offs,
                                   const int32_t* __restrict__ cb, const int32_t* __restrict__ cm,
                                   int total, int M_max, double* __restrict__ lr, int cplx) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
    const int m = cm[g];
    if (m < 0) continue;
    const int b = cb[g];
    const int base = offs[b];
    const double a0 = Om[2 * base], a1 = Om[2 * base + 1];
    put_ratio(lr, (long)b * M_max + m, a0, a1, Om[2 * g] - a0, Om[2 * g + 1] - a1, cplx);
  }
}

}  // namespace dn
