// Screened typewriter Metropolis sampler (Sec. IV, Algorithm 2; App. "Screened Metropolis
// sampler is exact"; App. "Practical implementation of the screened typewriter sampler").
//
// One half-sweep over B independent chains: the chain is cut into blocks of `spacing` sites,
// every other block (parity 0: blocks 0, 2, ...; 1: blocks 1, 3, ...) proposes one single-site
// flip at floor(r * width) inside it (r uniform in [0, 1), an input). The proposals' output
// changes dOmega_k come from ABACUS against one background configuration; proposal k is then
// judged with the independent-scattering ratio R~ = |f(Omega + dOmega_k) / f(Omega)|^2, Omega
// being the background's output plus the changes of the flips accepted since, f = prod cosh, so
// R~ = exp(2 sum_units lcd(Omega, dOmega_k)). With P = min(1, R~) a draw u with |u - P| <= eps is
// ambiguous: the chain freezes there (masking, the other chains go on), its background is
// rebuilt at its current configuration and the remaining proposals' changes are recomputed;
// the frozen proposal is then decided with its exact ratio. Otherwise accept iff u < P. When eps
// bounds |R~ - R| the decisions are those of exact Metropolis-Hastings for the same draws.
// The tolerance is one eps, or (the appendix's practical schedule) eps_buf[min(n, n_eps - 1)]
// with n the flips accepted since the chain's current background. Each refresh then records the
// event (n at the freeze, |min(1, R~) - min(1, R)|) with R the frozen proposal's exact ratio, and
// after the half-sweep sweep_eps_kernel applies the events, chain by chain in chain order, to
// the buffer: an entry still at its default takes the error, any other max(entry, gamma error).
#pragma once
#include "common.h"

namespace dn {

struct SweepArgs {
  int B, N, K, spacing, parity;
  int rows;              // chains this round (all of them in the first round, then the frozen ones)
  const int32_t* chain;  // [rows] chain of each row (nullable: row b is chain b)
  double eps;
  const double* r_site;  // [B][K] proposal draws
  const double* u;       // [B][K] acceptance draws
  int8_t* spins;         // [B][N] chains, updated in place
  int32_t* sites;        // [B][K][2] proposals (second site -1)
  int32_t* sites_r;      // [rows][K][2] this round's remaining proposals, from kstart
  int32_t* n_conn;       // [rows] this round's count
  int32_t* kstart;       // [B] first proposal not yet decided (K: done)
  int32_t* pending;      // [B] 1: the proposal at kstart froze the chain (decide it exactly next)
  int32_t* accepted;     // [B][K] 0/1
  int32_t* refreshes;    // [B]
  int32_t* frozen;       // [1] chains that froze in this round
  const double* Om0;     // [rows][2] output of this round's background
  const double* dom;     // [rows][K][2] this round's changes (index k - kstart)
  int cplx;              // 1: complex read-out unit (|psi|^2 decides: the ratio's real part)
  const double* eps_buf;  // nullable: tolerance buffer [n_eps] indexed by n (else eps)
  int n_eps;
  int32_t* nfrz;          // [B] n when the chain froze
  double* pfrz;           // [B] min(1, R~) of the proposal that froze it
  int32_t* ev_n;          // [B][K] refresh events of this half-sweep: n
  double* ev_e;           // [B][K] and the empirical error
  int32_t* ev_cnt;        // [B]
};

// Proposals of the half-sweep and the initial state of every chain.
__global__ void sweep_init_kernel(SweepArgs a) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)a.B * a.K; i += (long)gridDim.x * blockDim.x) {
    const int b = (int)(i / a.K), k = (int)(i % a.K);
    const int lo = (a.parity + 2 * k) * a.spacing;
    const int width = min(a.spacing, a.N - lo);
    const int off = min((int)floor(a.r_site[i] * width), width - 1);
    a.sites[2 * i] = lo + max(off, 0);
    a.sites[2 * i + 1] = -1;
    a.accepted[i] = 0;
    if (k == 0) {
      a.kstart[b] = 0;
      a.pending[b] = 0;
      a.refreshes[b] = 0;
      if (a.eps_buf) a.ev_cnt[b] = 0;
    }
  }
}

// The rows of the next round: the chains that froze, in chain order (one workgroup scans).
__global__ __launch_bounds__(1024) void sweep_list_kernel(const int32_t* __restrict__ kstart, int B, int K,
                                                          int32_t* __restrict__ chain) {
  __shared__ int part[1024];
  const int t = threadIdx.x, per = (B + 1023) / 1024;
  const int b0 = t * per, b1 = min(B, b0 + per);
  int cnt = 0;
  for (int b = b0; b < b1; ++b) cnt += kstart[b] < K;
  part[t] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int pos = part[t] - cnt;
  for (int b = b0; b < b1; ++b)
    if (kstart[b] < K) chain[pos++] = b;
}

// The remaining proposals of every row's chain as this round's work list, and the row's
// configuration (rows that are not chains of the same index take a copy of their chain).
__global__ void sweep_round_kernel(SweepArgs a, int8_t* __restrict__ row_spins) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)a.rows * a.K; i += (long)gridDim.x * blockDim.x) {
    const int row = (int)(i / a.K), m = (int)(i % a.K);
    const int b = a.chain ? a.chain[row] : row;
    const int k0 = a.kstart[b];
    const int k = k0 + m;
    a.sites_r[2 * i] = k < a.K ? a.sites[2 * ((long)b * a.K + k)] : -1;
    a.sites_r[2 * i + 1] = -1;
    if (m == 0) a.n_conn[row] = a.K - min(k0, a.K);
  }
  if (a.chain)
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)a.rows * a.N; i += (long)gridDim.x * blockDim.x)
      row_spins[i] = a.spins[(long)a.chain[i / a.N] * a.N + i % a.N];
  if (blockIdx.x == 0 && threadIdx.x == 0) a.frozen[0] = 0;
}

// Sequential screened acceptance, one thread per row (chain).
__global__ void sweep_accept_kernel(SweepArgs a) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= a.rows) return;
  const int b = a.chain ? a.chain[row] : row;
  const int k0 = a.kstart[b];
  if (k0 >= a.K) return;
  double om0 = a.Om0[2 * row], om1 = a.Om0[2 * row + 1];
  const bool exact_first = a.pending[b] != 0;
  int n = 0;  // flips accepted since this round's background
  for (int k = k0; k < a.K; ++k) {
    const long o = (long)row * a.K + (k - k0);
    const double d0 = a.dom[2 * o], d1 = a.dom[2 * o + 1];
    const double P = fmin(1.0, exp(2.0 * ratio_re(om0, om1, d0, d1, a.cplx)));
    const double uu = a.u[(long)b * a.K + k];
    if (exact_first && k == k0) {
      if (a.eps_buf) {  // the frozen proposal's exact probability against the approximate one
        const int e = a.ev_cnt[b]++;
        a.ev_n[(long)b * a.K + e] = a.nfrz[b];
        a.ev_e[(long)b * a.K + e] = fabs(a.pfrz[b] - P);
      }
    } else {
      const double tol = a.eps_buf ? a.eps_buf[min(n, a.n_eps - 1)] : a.eps;
      if (fabs(uu - P) <= tol) {
        a.kstart[b] = k;
        a.pending[b] = 1;
        a.refreshes[b] += 1;
        if (a.eps_buf) {
          a.nfrz[b] = n;
          a.pfrz[b] = P;
        }
        atomicAdd(a.frozen, 1);
        return;
      }
    }
    if (uu < P) {
      a.accepted[(long)b * a.K + k] = 1;
      const int j = a.sites[2 * ((long)b * a.K + k)];
      a.spins[(long)b * a.N + j] = (int8_t)(-a.spins[(long)b * a.N + j]);
      om0 += d0;
      om1 += d1;
      ++n;
    }
  }
  a.kstart[b] = a.K;
  a.pending[b] = 0;
}

// The half-sweep's refresh events applied to the tolerance buffer in chain order (one thread:
// a few events per chain, and the order fixes the result).
__global__ void sweep_eps_kernel(double* __restrict__ eps_buf, int32_t* __restrict__ eps_set, int n_eps,
                                 double gamma, const int32_t* __restrict__ ev_n, const double* __restrict__ ev_e,
                                 const int32_t* __restrict__ ev_cnt, int B, int K) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int b = 0; b < B; ++b)
    for (int e = 0; e < ev_cnt[b]; ++e) {
      const int i = min(ev_n[(long)b * K + e], n_eps - 1);
      const double err = ev_e[(long)b * K + e];
      if (!eps_set[i]) {
        eps_buf[i] = err;
        eps_set[i] = 1;
      } else {
        eps_buf[i] = fmax(eps_buf[i], gamma * err);
      }
    }
}

}  // namespace dn
