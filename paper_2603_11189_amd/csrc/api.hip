// C ABI of the DysonNet local-estimator library (declared in include/dysonnet.h).
//
// Host orchestration only: argument checks, workspace management, and the order of kernel
// launches on the caller's stream. Every arithmetic step runs in the kernels of
// s4gen.h, kernels.h and ham.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/dysonnet.h"
#include "common.h"
#include "ham.h"
#include "kernels.h"
#include "s4gen.h"
#include "grad.h"
#include "link2.h"
#include "sampler.h"
#include "sr.h"

using namespace dn;

namespace {

thread_local std::string g_err = "no error";
// true while this thread records launches into a graph (profiling events are skipped)
thread_local bool g_capturing = false;
// true while this thread runs the entry point that allocates nothing (no profiling events)
thread_local bool g_noalloc = false;
std::atomic<uint64_t> g_next_uid{1};

dn_status fail(dn_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(DN_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

#define STCHK(expr)                     \
  do {                                  \
    dn_status s_ = (expr);              \
    if (s_ != DN_OK) return s_;         \
  } while (0)

int pad_to(int x, int m) { return (x + m - 1) / m * m; }

struct Layout {
  long off_layers, off_s4, off_A, P;
};

bool layout_of(const dn_model_desc& d, Layout* lo) {
  if (d.N < 1 || d.L < 1 || d.d < 1 || d.s < 1 || d.d_out < 1 || d.w_c < 0) return false;
  const long dd = d.d, Wc = 2 * d.w_c + 1;
  lo->off_layers = 2 * dd * (d.token > 1 ? d.token : 1);  // E, E_phi: one vector per token position
  const long lay = 4 * dd * dd + 3 * dd + Wc * dd;
  lo->off_s4 = lo->off_layers + d.L * lay;
  lo->off_A = lo->off_s4 + (long)(d.L + 1) * dd * (12L * d.s + 1);
  lo->P = lo->off_A + dd * d.d_out;
  return true;
}

// Parameter-derived tables in one element type.
template <typename T> struct TableBufs {
  std::vector<void*> owned;
  Tables<T> tb{};
  T *E, *Ephi, *wE1, *WDt, *ADt, *Ut, *Vt, *Um, *Vm, *wv, *Kc, *kv, *bv, *taps, *tapsR, *Wk, *ADm, *WDm, *Pq, *omN,
      *Ac;
};

struct ProfRec {
  int kind;
  hipEvent_t a, b;
  double flops, bytes;
};

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> free_ev;
  std::vector<ProfRec> pending;
  double ms[DN_K_COUNT] = {}, fl[DN_K_COUNT] = {}, by[DN_K_COUNT] = {};
  long n[DN_K_COUNT] = {};
  ~Prof() {
    for (auto e : free_ev) (void)hipEventDestroy(e);
    for (auto& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  }
};

struct Workspace {
  std::map<std::string, std::pair<void*, size_t>> slots;
  size_t limit = 0, used = 0;
  ~Workspace() {
    for (auto& kv : slots) if (kv.second.first) (void)hipFree(kv.second.first);
  }
};

}  // namespace

struct dn_model {
  uint64_t uid = g_next_uid.fetch_add(1);  // never reused, unlike the address
  uint64_t ws_gen = 0;                     // bumped whenever a workspace buffer moves
  dn_model_desc desc{};
  Layout lay{};
  int DP = 0, Np = 0, Wc = 0;
  bool have_params = false;
  double* params = nullptr;   // [P]
  double* taps64 = nullptr;   // [L+1][d][2N-1]
  double* A64 = nullptr;      // [DP][2]
  double* omega = nullptr;    // [DP][Np]
  // float64 tables (always) and float32 tables (FP32 / BF16 modes)
  TableBufs<double> t64;
  TableBufs<float> t32;
  Workspace ws;
  Prof prof;
  // S4 tap Jacobian (float64 master + float32 copy), valid for the current parameters
  bool have_jac = false;
  // launch shapes (dn_autotune): 16-site output tiles per wave of the Toeplitz kernel
  // (0 = by chain length) and the bytes of flip fields per ABACUS chunk
  int conv_nt = 0;
  bool split3 = true;  // DN_PRODUCT_SPLIT3: three-term bf16 splits (conv_split_kernel, deep_kernel BF = 3)
  size_t flip_budget = (size_t)3 << 30;
  bool tuned = false;
  double* jac64 = nullptr;
  float* jac32 = nullptr;
  // pivot-0 link of block 2 (two-block networks): parameter-only spectra for the offsets
  // [lam_dlo, lam_dlo + lam_nd) (clusters up to two sites apart), float64 and, for float
  // models, float copies; transform length 2^lam_logn
  int lam_logn = 0, lam_nd = 0, lam_dlo = 0;
  double *lamM64r = nullptr, *lamM64i = nullptr;
  float *lamM32r = nullptr, *lamM32i = nullptr;
  std::vector<void*> owned;
  ~dn_model() {
    if (jac64) (void)hipFree(jac64);
    if (jac32) (void)hipFree(jac32);
    for (void* p : owned) (void)hipFree(p);
    for (void* p : t64.owned) (void)hipFree(p);
    for (void* p : t32.owned) (void)hipFree(p);
  }
};

namespace {

dn_status ws_get(dn_model* m, const char* name, size_t bytes, void** out) {
  bytes = std::max<size_t>(bytes, 256);
  auto& slot = m->ws.slots[name];
  if (slot.second >= bytes) { *out = slot.first; return DN_OK; }
  size_t newused = m->ws.used - slot.second + bytes;
  if (m->ws.limit && newused > m->ws.limit)
    return fail(DN_ENOMEM, std::string("workspace limit exceeded for ") + name);
  if (slot.first) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipFree(slot.first));
    m->ws.used -= slot.second;
    slot = {nullptr, 0};
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(DN_ENOMEM, std::string("hipMalloc failed for ") + name);
  slot = {p, bytes};
  m->ws.used += bytes;
  ++m->ws_gen;
  *out = p;
  return DN_OK;
}

hipEvent_t prof_event(dn_model* m) {
  hipEvent_t e = nullptr;
  if (!m->prof.free_ev.empty()) { e = m->prof.free_ev.back(); m->prof.free_ev.pop_back(); }
  else (void)hipEventCreate(&e);
  return e;
}

// Brackets one launch with events on its stream while profiling is on.
struct PScope {
  dn_model* m;
  int kind;
  hipStream_t st;
  double fl, by;
  hipEvent_t a = nullptr;
  PScope(dn_model* m_, int k, hipStream_t s, double f, double b) : m(m_), kind(k), st(s), fl(f), by(b) {
    if (m && m->prof.on && !g_capturing && !g_noalloc) { a = prof_event(m); (void)hipEventRecord(a, st); }
  }
  ~PScope() {
    if (a) {
      hipEvent_t b = prof_event(m);
      (void)hipEventRecord(b, st);
      m->prof.pending.push_back({kind, a, b, fl, by});
    }
  }
};

dn_status prof_harvest(dn_model* m) {
  HIPCHK(hipDeviceSynchronize());
  for (auto& r : m->prof.pending) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    m->prof.ms[r.kind] += ms;
    m->prof.fl[r.kind] += r.flops;
    m->prof.by[r.kind] += r.bytes;
    m->prof.n[r.kind] += 1;
    m->prof.free_ev.push_back(r.a);
    m->prof.free_ev.push_back(r.b);
  }
  m->prof.pending.clear();
  return DN_OK;
}

template <typename T> dn_status alloc_tables(TableBufs<T>& tb, const dn_model& m) {
  const long DP = m.DP, Np = m.Np, L = m.desc.L, Wc = m.Wc;
  auto get = [&](T** p, long n) -> bool {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<long>(n, 1) * sizeof(T)) != hipSuccess) return false;
    tb.owned.push_back(q);
    *p = (T*)q;
    return true;
  };
  const int tk = m.desc.token;
  bool ok = get(&tb.E, tk * DP) && get(&tb.Ephi, tk * DP) && get(&tb.wE1, tk * DP) && get(&tb.WDt, L * DP * DP) &&
            get(&tb.ADt, L * DP * DP) && get(&tb.Ut, L * DP * DP) && get(&tb.Vt, L * DP * DP) &&
            get(&tb.Um, L * DP * DP) && get(&tb.Vm, L * DP * DP) && get(&tb.wv, L * DP) &&
            get(&tb.Kc, L * Wc * DP) && get(&tb.kv, L * DP) && get(&tb.bv, L * DP) &&
            get(&tb.taps, L * DP * tap_stride(Np)) && get(&tb.tapsR, L * DP * tap_stride(Np)) &&
            get(&tb.Wk, 2 * DP * Np) && get(&tb.ADm, L * DP * DP) && get(&tb.WDm, L * DP * DP) &&
            get(&tb.Pq, tk * 4 * DP * tap_stride(Np)) && get(&tb.omN, DP * Np) && get(&tb.Ac, 2 * DP);
  if (!ok) return fail(DN_ENOMEM, "hipMalloc failed for parameter tables");
  tb.tb = Tables<T>{tb.E, tb.Ephi, tb.wE1, tb.WDt, tb.ADt, tb.Ut, tb.Vt, tb.Um, tb.Vm,
                    tb.wv, tb.Kc, tb.kv, tb.bv, tb.taps, tb.tapsR, tb.Wk, tb.ADm, tb.WDm, tb.Pq, tb.omN, tb.Ac};
  return DN_OK;
}

long table_elems(const dn_model& m) {
  const long DP = m.DP, Np = m.Np, L = m.desc.L, Wc = m.Wc, tk = m.desc.token;
  return 3 * tk * DP + 8 * L * DP * DP + 3 * L * DP + L * Wc * DP + (2 * L + 4 * tk) * DP * tap_stride(Np) +
         2 * DP * Np;
}

// Copy double tables into float tables (same member order).
dn_status convert_tables(dn_model* m, hipStream_t st) {
  TableBufs<double>& a = m->t64;
  TableBufs<float>& b = m->t32;
  const long DP = m->DP, Np = m->Np, L = m->desc.L, Wc = m->Wc, tk = m->desc.token;
  struct P { double* s; float* d; long n; } items[] = {
      {a.E, b.E, tk * DP}, {a.Ephi, b.Ephi, tk * DP}, {a.wE1, b.wE1, tk * DP}, {a.WDt, b.WDt, L * DP * DP},
      {a.ADt, b.ADt, L * DP * DP}, {a.Ut, b.Ut, L * DP * DP}, {a.Vt, b.Vt, L * DP * DP},
      {a.Um, b.Um, L * DP * DP}, {a.Vm, b.Vm, L * DP * DP}, {a.wv, b.wv, L * DP},
      {a.Kc, b.Kc, L * Wc * DP}, {a.kv, b.kv, L * DP}, {a.bv, b.bv, L * DP},
      {a.taps, b.taps, L * DP * tap_stride(Np)}, {a.tapsR, b.tapsR, L * DP * tap_stride(Np)}, {a.Wk, b.Wk, 2 * DP * Np},
      {a.ADm, b.ADm, L * DP * DP}, {a.WDm, b.WDm, L * DP * DP}, {a.Pq, b.Pq, tk * 4 * DP * tap_stride(Np)},
      {a.omN, b.omN, DP * Np}, {a.Ac, b.Ac, 2 * DP}};
  for (auto& it : items) {
    int grid = (int)std::min<long>(1024, (it.n + 255) / 256);
    convert_kernel<<<grid, 256, 0, st>>>(it.s, it.d, it.n);
  }
  HIPCHK(hipGetLastError());
  return DN_OK;
}

// Raises a kernel's dynamic LDS limit once (the value only grows).
template <typename K> void allow_lds(K kernel, size_t bytes) {
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  if (bytes <= 64 * 1024) return;
  std::lock_guard<std::mutex> g(mu);
  size_t& have = done[(const void*)kernel];
  if (have >= bytes) return;
  if (hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
    have = bytes;
}

constexpr size_t LDS_MAX = 160 * 1024;

// Compute units of the current device (cached per device; 256 if the query fails).
static int cu_count() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int c = cached[dev].load();
  if (c <= 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cached[dev].store(c);
  }
  return c;
}

// ------------------------------------------------------------------------------------------
// Network passes, templated on element type T and padded channel count DP.

template <typename T> const Tables<T>& tables_of(dn_model* m);
template <> const Tables<double>& tables_of<double>(dn_model* m) { return m->t64.tb; }
template <> const Tables<float>& tables_of<float>(dn_model* m) { return m->t32.tb; }

template <typename T> dn_status launch_conv(dn_model* m, const T* X, T* Y, const T* taps, int C, hipStream_t st,
                                            DynRange dyn = DynRange{nullptr, 0, 0}, const T* add = nullptr,
                                            bool exact = false) {
  if (C <= 0) return DN_OK;
  const int Np = m->Np;
  ConvArgs<T> a{X, Y, taps, m->desc.N, Np, C, m->DP, dyn, add};
  const double Nr = m->desc.N, dr = m->desc.d;
  PScope ps(m, DN_K_CONV, st, 2.0 * C * Nr * Nr * dr, 2.0 * C * Nr * dr * sizeof(T));
  const size_t lds = (CONV_MC * CONV_LD + 2 * Np) * sizeof(T);
  // 16-site tiles per wave; a wave's 16 nt sites must tile Np (so no wave straddles its end)
  int nt = m->conv_nt ? m->conv_nt : (Np >= 256 ? 4 : Np / 64);
  if (nt < 1 || nt > 4 || Np % (16 * nt) != 0) nt = Np >= 256 ? 4 : Np / 64;
  dim3 grid((C + CONV_MC - 1) / CONV_MC, m->DP, (Np + 64 * nt - 1) / (64 * nt));
  if constexpr (std::is_same<T, float>::value) {
    if (m->split3) {
      // BF16-mixed models: hi + lo terms (three partial products); float models and the
      // gradients of any model (exact): the three-term split (six)
      const int ns = m->desc.prec == DN_PREC_BF16_MIXED && !exact ? 2 : 3;
      const size_t lds3 = (ns * (size_t)CONV_MC * CS_LD + ns * 8 * (size_t)(2 * Np + 16)) * sizeof(__bf16);
      // workgroups run over configuration blocks: about two per CU in all (the split taps
      // are then built once per workgroup)
      const long nblk = grid.x;
      grid.x = (unsigned)std::max<long>(1, std::min<long>(nblk, (2L * cu_count() + (long)m->DP * grid.z - 1) / ((long)m->DP * grid.z)));
      if (ns == 2) {
        switch (nt) {
          case 1: allow_lds(conv_split_kernel<1, 2>, lds3); conv_split_kernel<1, 2><<<grid, 256, lds3, st>>>(a); break;
          case 2: allow_lds(conv_split_kernel<2, 2>, lds3); conv_split_kernel<2, 2><<<grid, 256, lds3, st>>>(a); break;
          case 3: allow_lds(conv_split_kernel<3, 2>, lds3); conv_split_kernel<3, 2><<<grid, 256, lds3, st>>>(a); break;
          default: allow_lds(conv_split_kernel<4, 2>, lds3); conv_split_kernel<4, 2><<<grid, 256, lds3, st>>>(a); break;
        }
      } else {
        switch (nt) {
          case 1: allow_lds(conv_split_kernel<1>, lds3); conv_split_kernel<1><<<grid, 256, lds3, st>>>(a); break;
          case 2: allow_lds(conv_split_kernel<2>, lds3); conv_split_kernel<2><<<grid, 256, lds3, st>>>(a); break;
          case 3: allow_lds(conv_split_kernel<3>, lds3); conv_split_kernel<3><<<grid, 256, lds3, st>>>(a); break;
          default: allow_lds(conv_split_kernel<4>, lds3); conv_split_kernel<4><<<grid, 256, lds3, st>>>(a); break;
        }
      }
      HIPCHK(hipGetLastError());
      return DN_OK;
    }
  }
  switch (nt) {
    case 1: allow_lds(conv_kernel<T, 1>, lds); conv_kernel<T, 1><<<grid, 256, lds, st>>>(a); break;
    case 2: allow_lds(conv_kernel<T, 2>, lds); conv_kernel<T, 2><<<grid, 256, lds, st>>>(a); break;
    case 3: allow_lds(conv_kernel<T, 3>, lds); conv_kernel<T, 3><<<grid, 256, lds, st>>>(a); break;
    default: allow_lds(conv_kernel<T, 4>, lds); conv_kernel<T, 4><<<grid, 256, lds, st>>>(a); break;
  }
  HIPCHK(hipGetLastError());
  return DN_OK;
}

template <typename T, int DP, int NT> void phi_go(const PhiArgs<T>& a, int C, size_t lds, hipStream_t st) {
  if (a.tok > 1) {  // tokens of several spins: the general embedding
    allow_lds(phi_kernel<T, DP, NT, true>, lds);
    phi_kernel<T, DP, NT, true><<<C, 256, lds, st>>>(a);
    return;
  }
  allow_lds(phi_kernel<T, DP, NT>, lds);
  phi_kernel<T, DP, NT><<<C, 256, lds, st>>>(a);
}

template <typename T, int DP> dn_status launch_phi(dn_model* m, const PhiArgs<T>& a, int C, hipStream_t st) {
  if (C <= 0) return DN_OK;
  const size_t lds =
      ((size_t)DP * (m->Np + 2 * m->desc.w_c + 1) + (size_t)m->desc.token * m->Np + (2 * m->desc.w_c + 2) * DP) *
      sizeof(T);
  if (lds > LDS_MAX) return fail(DN_EUNSUPPORTED, "phi stream tile exceeds LDS");
  const double Nr = m->desc.N, dr = m->desc.d, e = sizeof(T);
  const double nfield = (a.first ? 0 : 1) + (a.phi_out ? 1 : 0) + 1 + (a.a_out ? 1 : 0) + (a.first ? 1 : 0);
  PScope ps(m, DN_K_PHI, st, (a.first ? 2.0 : 4.0) * C * Nr * dr * dr, nfield * C * Nr * dr * e);
  if constexpr (std::is_same<T, double>::value) {
    phi_go<T, DP, 1>(a, C, lds, st);
  } else {
    // 64 channels: at most two site tiles per wave (four leave one wave per SIMD)
    switch (DP >= 64 ? std::min(2, tiles_per_wave(m->Np)) : tiles_per_wave(m->Np)) {
      case 1: phi_go<T, DP, 1>(a, C, lds, st); break;
      case 2: phi_go<T, DP, 2>(a, C, lds, st); break;
      case 3: phi_go<T, DP, 3>(a, C, lds, st); break;
      default: phi_go<T, DP, 4>(a, C, lds, st); break;
    }
  }
  HIPCHK(hipGetLastError());
  return DN_OK;
}

// Channel mixing on the bf16 matrix cores (DN_PREC_BF16_MIXED; float fields, d > 16).
bool use_bf16(const dn_model* m) { return m->desc.prec == DN_PREC_BF16_MIXED; }

template <typename T, int DP, int MODE>
dn_status launch_mix(dn_model* m, const MixArgs<T>& a, int C, hipStream_t st, bool allow_bf = true) {
  if (C <= 0) return DN_OK;
  const int nw = m->Np / 64;
  const double Nr = m->desc.N, dr = m->desc.d, e = sizeof(T), fld = Nr * dr * e;
  const double fl = 4.0 * C * Nr * dr * dr;
  int kind;
  double by;
  if (MODE == MIX_FWD) {
    kind = DN_K_MIX_FWD;
    by = C * fld * (2 + (a.out ? 1 : 0) + (a.p0_out ? 1 : 0) + (a.inject ? 1 : 0));
  } else {
    kind = DN_K_MIX_TAU;
    by = C * fld + (C / 2) * fld;
  }
  PScope ps(m, kind, st, fl, by);
  bool done = false;
  if constexpr (std::is_same<T, float>::value && DP >= 32) {
    if (allow_bf && use_bf16(m)) {
      mix_kernel<T, DP, MODE, true><<<C, 64 * nw, 0, st>>>(a);
      done = true;
    }
  }
  if (!done) mix_kernel<T, DP, MODE, false><<<C, 64 * nw, 0, st>>>(a);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

// Persistent tiled launch of a deep block (see deep_kernel); the last one is followed by
// last_finish_kernel, one wave per flip.
template <typename T, int DP, bool FIRST, bool LAST, int BF, int NU = SLICE_WIN>
dn_status launch_deep(dn_model* m, const MixArgs<T>& a, int F, hipStream_t st, int Bc) {
  if (F <= 0) return DN_OK;
  // F1 (not in the first block) and F2, then the last block's per-wave copies of dh or the
  // read-out weights of one tile position
  const size_t lds = (size_t)deep_wbytes(DP, sizeof(T), FIRST, BF) +
                     (LAST ? (size_t)DEEP_WAVES * deep_cpg(DP, BF) * DH_LD * sizeof(T)
                           : (size_t)DP * 64 * sizeof(T) + 2 * DP * sizeof(double));
  static int per_cu = 0, cus = 0;
  if (!per_cu) {
    allow_lds(deep_kernel<T, DP, FIRST, LAST, BF, NU>, lds);
    int dev = 0, n = 0, c = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, deep_kernel<T, DP, FIRST, LAST, BF, NU>, 256, lds));
    cus = std::max(c, 1);
    per_cu = std::max(n, 1);
  }
  const int nt = m->Np / 64;
  const long tiles = (long)F * nt;
  long grid = std::min<long>((tiles + DEEP_WAVES - 1) / DEEP_WAVES, (long)cus * per_cu);
  // workgroups per XCD: a multiple of the tile positions (each workgroup keeps one)
  const long nbx = std::max<long>(nt, grid / NXCD / nt * nt);
  grid = nbx * NXCD;
  const double Nr = m->desc.N, dr = m->desc.d, fld = Nr * dr * sizeof(T);
  const int WL = 2 + 2 * m->desc.L * m->desc.w_c + 1;
  {
    // the first block forms its V product from the unit-flip table (only U is a product);
    // the last block also forms the tiles' partial slices of the last mixer's output
    const double fl = (FIRST ? 2.0 : 4.0) * F * Nr * dr * dr + (LAST ? 2.0 * F * WL * Nr * dr : 0.0);
    const double by = F * fld * ((FIRST ? 0 : 1) + (LAST ? 0 : 1)) + (double)Bc * fld * (LAST ? 4 : 2);
    PScope ps(m, DN_K_MIX_DEEP, st, fl, by);
    deep_kernel<T, DP, FIRST, LAST, BF, NU><<<(int)grid, 256, lds, st>>>(a);
    HIPCHK(hipGetLastError());
  }
  if (LAST) {
    PScope ps(m, DN_K_TAIL, st, 4.0 * F * WL * dr * dr,
              (double)F * (m->Np / 64) * SLICE_WIN * dr * sizeof(T) + (double)F * WL * dr * sizeof(T) * 2);
    if (a.dphi) last_finish_kernel<T, DP, true><<<F, 64, 2 * DP * SLICE_WIN * sizeof(T), st>>>(a);
    else last_finish_kernel<T, DP><<<F, 64, 2 * DP * SLICE_WIN * sizeof(T), st>>>(a);
    HIPCHK(hipGetLastError());
  }
  return DN_OK;
}

// The last block of a float model computes its partial slices only over the widest slice
// S_L any flip can have (2 + 2 L w_c + 1 sites), rounded up to 8, 12 or 16.
template <typename T, int DP, bool FIRST, int BF>
dn_status launch_deep_last(dn_model* m, const MixArgs<T>& a, int F, hipStream_t st, int Bc) {
  if constexpr (sizeof(T) == 4) {
    const int WL = 2 + 2 * m->desc.L * m->desc.w_c + 1;
    if (WL <= 8) return launch_deep<T, DP, FIRST, true, BF, 8>(m, a, F, st, Bc);
    if (WL <= 12) return launch_deep<T, DP, FIRST, true, BF, 12>(m, a, F, st, Bc);
  }
  return launch_deep<T, DP, FIRST, true, BF>(m, a, F, st, Bc);
}

template <typename T, int DP, int BF>
dn_status launch_deep_mode(dn_model* m, const MixArgs<T>& a, int F, hipStream_t st, int Bc, bool first, bool last) {
  if (first && last) return launch_deep_last<T, DP, true, BF>(m, a, F, st, Bc);
  if (last) return launch_deep_last<T, DP, false, BF>(m, a, F, st, Bc);
  if (first) return launch_deep<T, DP, true, false, BF>(m, a, F, st, Bc);
  return launch_deep<T, DP, false, false, BF>(m, a, F, st, Bc);
}

template <typename T, int DP>
dn_status launch_deep_any(dn_model* m, const MixArgs<T>& a, int F, hipStream_t st, int Bc, bool first, bool last) {
  if constexpr (std::is_same<T, float>::value && DP >= 32) {
    if (use_bf16(m)) return launch_deep_mode<T, DP, 2>(m, a, F, st, Bc, first, last);
    if (m->split3) return launch_deep_mode<T, DP, 3>(m, a, F, st, Bc, first, last);
  }
  return launch_deep_mode<T, DP, 0>(m, a, F, st, Bc, first, last);
}

// Forward of C configurations listed by `map` entries [cfg0, cfg0+C). rho[C][2] receives
// Omega. With caches (ABACUS background), a/chi/p0 of every block (and phi^(1..L) when
// cache_phi is given) are written layer-major [L][C][DP][Np].
// Checkpoints of the gradient forward: h^(l) for l = 0..L-1 and phi^(l) for l = 1..L-1
// ([L][C][DP][Np] each, phi slot 0 unused) and the residual sum R ([C][DP][Np]).
template <typename T> struct Ckpt {
  T *h = nullptr, *phi = nullptr, *R = nullptr;
};

// fields: nullable; five [C][DP][Np] fields the caller provides (otherwise the workspace's).
template <typename T, int DP>
dn_status forward_chunk(dn_model* m, const int8_t* spins, CfgMap map, int cfg0, int C, double* rho,
                        T* cache_a, T* cache_chi, T* cache_p0, hipStream_t st, Ckpt<T> ck = Ckpt<T>(),
                        T* fields = nullptr, T* cache_phi = nullptr) {
  const dn_model_desc& d = m->desc;
  const int Np = m->Np, L = d.L;
  const long fld = (long)C * DP * Np;
  void *pphi, *pchi0, *pchi1, *pu, *pv;
  if (fields) {
    pphi = fields; pchi0 = fields + fld; pchi1 = fields + 2 * fld; pu = fields + 3 * fld; pv = fields + 4 * fld;
  } else {
    STCHK(ws_get(m, "fw_phi", fld * sizeof(T), &pphi));
    STCHK(ws_get(m, "fw_chi0", fld * sizeof(T), &pchi0));
    STCHK(ws_get(m, "fw_chi1", fld * sizeof(T), &pchi1));
    STCHK(ws_get(m, "fw_u", fld * sizeof(T), &pu));
    STCHK(ws_get(m, "fw_v", fld * sizeof(T), &pv));
  }
  T* phi = (T*)pphi;
  T* chib[2] = {(T*)pchi0, (T*)pchi1};
  T* u = (T*)pu;
  T* v = (T*)pv;
  const Tables<T>& tb = tables_of<T>(m);
  auto chi_of = [&](int l) -> T* { return cache_chi ? cache_chi + (long)l * fld : chib[l & 1]; };
  auto phi_pass = [&](int l) -> dn_status {
    PhiArgs<T> a{};
    a.tb = tb; a.N = d.N; a.Np = Np; a.l = l; a.w_c = d.w_c; a.periodic = d.bc == DN_BC_PERIODIC;
    a.act = d.act; a.inject = d.inject_phi; a.first = (l == 0); a.spins = spins; a.map = map; a.tok = d.token;
    a.cfg0 = cfg0; a.C = C; a.phi_in = phi;
    a.phi_out = (l + 1 < L || d.inject_phi) ? phi : nullptr;
    a.chi_out = chi_of(l);
    a.a_out = cache_a ? cache_a + (long)l * fld : nullptr;
    a.u_out = ck.h ? ck.h : u; a.rho = rho; a.R_out = ck.R;
    if (ck.phi && l >= 1) a.phi_in = ck.phi + (long)l * fld;       // phi^(l) checkpoint (block l+1 reads it)
    if (ck.phi && l + 1 < L) a.phi_out = ck.phi + (long)(l + 1) * fld;
    STCHK((launch_phi<T, DP>(m, a, C, st)));
    // phi^(l+1) of the background (phi injected: ABACUS needs it on the slices)
    if (cache_phi) HIPCHK(hipMemcpyAsync(cache_phi + (long)l * fld, phi, fld * sizeof(T), hipMemcpyDeviceToDevice, st));
    return DN_OK;
  };
  STCHK(phi_pass(0));
  for (int l = 0; l < L; ++l) {
    const T* hin = ck.h ? ck.h + (long)l * fld : u;
    STCHK(launch_conv<T>(m, hin, v, tb.taps + (long)l * DP * tap_stride(Np), C, st, DynRange{nullptr, 0, 0}, nullptr,
                         ck.h != nullptr));
    if (l + 1 < L) STCHK(phi_pass(l + 1));
    MixArgs<T> a{};
    a.tb = tb; a.N = d.N; a.Np = Np; a.l = l; a.L = L; a.w_c = d.w_c;
    a.periodic = d.bc == DN_BC_PERIODIC; a.inject = d.inject_phi; a.C = C; a.cfg0 = cfg0;
    a.X = v; a.chi = chi_of(l); a.p0_out = cache_p0 ? cache_p0 + (long)l * fld : nullptr;
    // phi^(l+2) (injected into the next mixer input): the checkpoint slot when it has one
    a.phi_next = (ck.phi && l + 2 < L) ? ck.phi + (long)(l + 2) * fld : phi;
    a.out = (l + 1 < L) ? (ck.h ? ck.h + (long)(l + 1) * fld : u) : nullptr; a.rho = rho;
    a.R_acc = ck.R;
    // the gradient's forward (checkpoints) stays in float: its backward is float
    STCHK((launch_mix<T, DP, MIX_FWD>(m, a, C, st, ck.h == nullptr)));
  }
  return DN_OK;
}

// Builds the (sample, element) work list on the device and validates n_conn and sites
// (error bits in offs[B + 1]).
dn_status plan_launch(dn_model* m, const int32_t* n_conn, const int32_t* sites, int B, int M_max, int with_base,
                      int32_t** offs, int32_t** cb, int32_t** cm, int upper, hipStream_t st) {
  void *po, *pb, *pm;
  STCHK(ws_get(m, "plan_offs", (size_t)(B + 2) * 4, &po));
  STCHK(ws_get(m, "plan_cb", (size_t)upper * 4, &pb));
  STCHK(ws_get(m, "plan_cm", (size_t)upper * 4, &pm));
  *offs = (int32_t*)po; *cb = (int32_t*)pb; *cm = (int32_t*)pm;
  plan_kernel<<<1, 1024, 0, st>>>(n_conn, B, M_max, with_base, *offs);
  const long slots = (long)B * (M_max + with_base);
  plan_fill_kernel<<<(int)std::min<long>(4096, (slots + 255) / 256), 256, 0, st>>>(n_conn, sites, B,
                                                                                  m->desc.N * m->desc.token, M_max,
                                                                                  with_base, *offs, *cb, *cm);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

dn_status plan_errors(int bits) {
  if (bits & 1) return fail(DN_EINVAL, "n_conn outside [0, M_max]");
  if (bits & 2) return fail(DN_EINVAL, "a site index is outside the chain (or a pair repeats a site)");
  if (bits & 8) return fail(DN_EINVAL, "a spin is neither +1 nor -1");
  return DN_OK;
}

// The work list with its offsets brought back to the host (one stream synchronisation) to
// size the launches exactly.
// The spins of the batch are checked on the way (bit 8 of the error word).
dn_status plan(dn_model* m, const int32_t* n_conn, const int32_t* sites, int B, int M_max, int with_base,
               int32_t** offs, int32_t** cb, int32_t** cm, int upper, std::vector<int32_t>* h_offs,
               hipStream_t st, const int8_t* spins = nullptr) {
  STCHK(plan_launch(m, n_conn, sites, B, M_max, with_base, offs, cb, cm, upper, st));
  if (spins) {
    const long n = (long)B * m->desc.N * m->desc.token;
    spin_check_kernel<<<(int)std::min<long>(1024, (n + 1023) / 1024), 256, 0, st>>>(spins, n, *offs + B + 1);
    HIPCHK(hipGetLastError());
  }
  h_offs->resize(B + 2);
  HIPCHK(hipMemcpyAsync(h_offs->data(), *offs, (size_t)(B + 2) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return plan_errors((*h_offs)[B + 1]);
}

// Identity work list over B samples in the named workspace slots.
dn_status identity_map(dn_model* m, const char* nb, const char* nm, int B, int32_t** cb, int32_t** cm,
                       hipStream_t st) {
  void *pb, *pm;
  STCHK(ws_get(m, nb, (size_t)B * 4, &pb));
  STCHK(ws_get(m, nm, (size_t)B * 4, &pm));
  *cb = (int32_t*)pb;
  *cm = (int32_t*)pm;
  identity_map_kernel<<<(B + 255) / 256, 256, 0, st>>>(*cb, *cm, B);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

size_t chunk_configs(const dn_model* m, size_t elem, int fields, size_t budget) {
  size_t per = (size_t)m->DP * m->Np * elem * fields;
  size_t c = budget / std::max<size_t>(per, 1);
  return std::max<size_t>(64, std::min<size_t>(c, 1 << 20) / 64 * 64);
}

template <typename T, int DP>
dn_status logratio_full(dn_model* m, const int8_t* spins, int B, const int32_t* sites, const int32_t* n_conn,
                        int M_max, double* logpsi, double* logratio, hipStream_t st) {
  int32_t *offs, *cb, *cm;
  std::vector<int32_t> h_offs;
  STCHK(plan(m, n_conn, sites, B, M_max, 1, &offs, &cb, &cm, B * (M_max + 1), &h_offs, st, spins));
  const int total = h_offs[B];
  void* prho;
  STCHK(ws_get(m, "full_rho", (size_t)std::max(total, 1) * 2 * sizeof(double), &prho));
  double* rho = (double*)prho;
  CfgMap map{cb, cm, sites, M_max};
  const size_t chunk = chunk_configs(m, sizeof(T), 5, (size_t)6 << 30);
  for (int c0 = 0; c0 < total; c0 += (int)chunk) {
    const int C = (int)std::min<size_t>(chunk, total - c0);
    STCHK((forward_chunk<T, DP>(m, spins, map, c0, C, rho + 2L * c0, nullptr, nullptr, nullptr, st)));
  }
  fill_kernel<double><<<256, 256, 0, st>>>(logratio, (long)B * M_max * (1 + m->desc.complex_out), 0.0);
  plain_ratio_kernel<<<(total + 255) / 256, 256, 0, st>>>(rho, offs, cb, cm, total, M_max, logratio,
                                                          m->desc.complex_out);
  if (logpsi) logpsi_kernel<<<(B + 255) / 256, 256, 0, st>>>(rho, offs, B, logpsi, m->desc.complex_out);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

// Parameter-only spectra of block 2's pivot-0 link (two-block networks), float64, and float
// copies for float models (see lam_param_kernel). Transform length: the power of two >= 2N - 1.
dn_status build_lam_tables(dn_model* m, hipStream_t st) {
  const dn_model_desc& d = m->desc;
  if (d.L != 2) return DN_OK;
  int logn = 1;
  while ((1 << logn) < 2 * d.N - 1) ++logn;
  const int nd = lam_nd(d.w_c, 2), n = 1 << logn, nh = n / 2 + 1;
  const size_t per_k = (size_t)nd * nh * m->DP * m->DP;  // one position inside a token
  const size_t elems = per_k * d.token;
  if (!m->lamM64r) {
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, elems * 8) != hipSuccess || hipMalloc(&b, elems * 8) != hipSuccess) {
      if (a) (void)hipFree(a);
      return fail(DN_ENOMEM, "hipMalloc failed for the pivot-0 link spectra");
    }
    m->owned.push_back(a);
    m->owned.push_back(b);
    m->lamM64r = (double*)a;
    m->lamM64i = (double*)b;
    if (d.prec != DN_PREC_FP64) {
      void *c = nullptr, *e = nullptr;
      if (hipMalloc(&c, elems * 4) != hipSuccess || hipMalloc(&e, elems * 4) != hipSuccess) {
        if (c) (void)hipFree(c);
        return fail(DN_ENOMEM, "hipMalloc failed for the pivot-0 link spectra");
      }
      m->owned.push_back(c);
      m->owned.push_back(e);
      m->lamM32r = (float*)c;
      m->lamM32i = (float*)e;
    }
  }
  m->lam_logn = logn;
  m->lam_nd = nd;
  m->lam_dlo = -(2 * d.w_c + 2);
  const int nseq = std::max(1, std::min(m->DP, 4096 >> logn));
  const size_t lds = ((size_t)2 * nseq * (n + 1) + n) * sizeof(double);
  allow_lds(lam_param_kernel, lds);
  for (int k = 0; k < d.token; ++k) {  // the composite spectra of each position's unit flip
    LamParamArgs a{};
    a.taps = m->t64.taps; a.Pq = m->t64.Pq + (long)k * 4 * m->DP * tap_stride(m->Np); a.Ut = m->t64.Ut;
    a.N = d.N; a.Np = m->Np; a.d = d.d; a.DP = m->DP; a.logn = logn; a.ND = nd; a.dlo = m->lam_dlo;
    a.periodic = d.bc == DN_BC_PERIODIC; a.Mr = m->lamM64r + k * per_k; a.Mi = m->lamM64i + k * per_k;
    PScope ps(m, DN_K_PREP, st, 5.0 * n * logn * (double)nd * m->DP * m->DP, (double)per_k * 16);
    lam_param_kernel<<<dim3(nd, m->DP), 256, lds, st>>>(a);
  }
  HIPCHK(hipGetLastError());
  if (d.prec != DN_PREC_FP64) {
    convert_kernel<<<1024, 256, 0, st>>>(m->lamM64r, m->lamM32r, (long)elems);
    convert_kernel<<<1024, 256, 0, st>>>(m->lamM64i, m->lamM32i, (long)elems);
    HIPCHK(hipGetLastError());
  }
  return DN_OK;
}

template <typename T> void lam_spectra(const dn_model* m, const T** r, const T** i);
template <> void lam_spectra<double>(const dn_model* m, const double** r, const double** i) { *r = m->lamM64r; *i = m->lamM64i; }
template <> void lam_spectra<float>(const dn_model* m, const float** r, const float** i) { *r = m->lamM32r; *i = m->lamM32i; }

// Channels per workgroup of the per-sample transforms: pairs of channels per complex
// transform, a power of two that keeps the transforms' LDS within 64 KB.
int lam_chf(int DP, int logn, size_t elem) {
  const size_t per_pair = (size_t)2 * ((1 << logn) + 1) * elem;
  int np = 1;
  while (2 * np <= DP / 2 && (size_t)(2 * np) * per_pair <= 65536) np *= 2;
  return 2 * np;
}

// Block 2's pivot-0 link for the background samples of one forward chunk: lam[b][z][delta][c]
// for delta in [dlo, dlo + ND), in passes that keep the spectra of a pass within ~1 GiB.
template <typename T, int DP>
dn_status build_lam(dn_model* m, const T* chi1, int Bf, int ND, int dlo, T* lam, hipStream_t st) {
  const dn_model_desc& d = m->desc;
  const int logn = m->lam_logn, n = 1 << logn, nh = n / 2 + 1;
  const size_t per = (size_t)(ND + 1) * nh * DP * 2 * sizeof(T);
  const int Bs_max = (int)std::max<size_t>(64, std::min<size_t>(Bf, ((size_t)1 << 30) / per));
  void *pxr, *pxi, *pzr, *pzi;
  const size_t nx = (size_t)nh * Bs_max * DP, nz = (size_t)ND * nx;
  STCHK(ws_get(m, "lam_Xr", nx * sizeof(T), &pxr));
  STCHK(ws_get(m, "lam_Xi", nx * sizeof(T), &pxi));
  STCHK(ws_get(m, "lam_Zr", nz * sizeof(T), &pzr));
  STCHK(ws_get(m, "lam_Zi", nz * sizeof(T), &pzi));
  const T *Mr0, *Mi0;
  lam_spectra<T>(m, &Mr0, &Mi0);
  const size_t per_k = (size_t)m->lam_nd * nh * DP * DP;  // spectra of one position in a token
  const long lamk = (long)Bf * d.N * ND * DP;             // links of one position
  const int chf = lam_chf(DP, logn, sizeof(T));
  const size_t lds_t = ((size_t)chf * (n + 1) + n) * sizeof(T);
  const size_t lds_g = ((size_t)2 * DP * 65 + 2 * DP * DP) * sizeof(T);
  allow_lds(lam_fwd_kernel<T>, lds_t);
  allow_lds(lam_inv_kernel<T>, lds_t);
  allow_lds(lam_gemm_kernel<T, DP>, lds_g);
  const double dr = d.d, fft = 5.0 * n * logn;  // flops of one complex transform
  for (int s0 = 0; s0 < Bf; s0 += Bs_max) {
    const int Bs = std::min(Bs_max, Bf - s0);
    LamArgs<T> a{};
    a.N = d.N; a.Np = m->Np; a.DP = DP; a.logn = logn; a.ND = ND; a.periodic = d.bc == DN_BC_PERIODIC;
    a.di0 = dlo - m->lam_dlo; a.Bc = Bs; a.chf = chf;
    a.chi1 = chi1 + (long)s0 * DP * m->Np;
    a.Xr = (T*)pxr; a.Xi = (T*)pxi; a.Zr = (T*)pzr; a.Zi = (T*)pzi;
    {
      PScope ps(m, DN_K_LINK, st, Bs * (dr / 2) * fft, (double)Bs * (d.N * dr + 2.0 * nh * dr) * sizeof(T));
      lam_fwd_kernel<T><<<dim3(Bs, DP / chf), 256, lds_t, st>>>(a);
    }
    for (int k = 0; k < d.token; ++k) {  // the spectra of chi0 serve every position's link
    a.Mr = Mr0 + k * per_k; a.Mi = Mi0 + k * per_k;
    a.lam = lam + k * lamk + (long)s0 * d.N * ND * DP;
    {
      PScope ps(m, DN_K_LINK, st, 8.0 * ND * nh * dr * dr * Bs,
                (double)(2.0 * nh * dr * Bs + 2.0 * ND * nh * dr * dr + 2.0 * ND * nh * dr * Bs) * sizeof(T));
      lam_gemm_kernel<T, DP><<<dim3(nh, (Bs + 63) / 64), 256, lds_g, st>>>(a);
    }
    {
      PScope ps(m, DN_K_LINK, st, (double)Bs * ND * (dr / 2) * fft,
                (double)Bs * ND * (2.0 * nh * dr + d.N * dr) * sizeof(T));
      lam_inv_kernel<T><<<dim3(Bs, ND, DP / chf), 256, lds_t, st>>>(a);
    }
    }
    HIPCHK(hipGetLastError());
  }
  return DN_OK;
}

// The fused slice recompute + per-flip update of one- and two-block networks (shallow_kernel):
// one workgroup of DP / 16 waves per P flips.
template <typename T, int DP, bool TWO>
dn_status launch_shallow(dn_model* m, const SliceArgs<T>& sa, Flip12Args<T> a, int F, int P, int Wc, double slice_fl,
                         hipStream_t st, int ext) {
  if (F <= 0) return DN_OK;
  // plus block 2's taps over the offsets between S_1 and S_2 (two blocks)
  const int W1m = ext + 2 * m->desc.w_c + 1, W2m = W1m + 2 * m->desc.w_c;
  const size_t lds = slm_lds_bytes<T>(DP, P, Wc, m->desc.w_c) + (TWO ? (size_t)DP * (W1m + W2m - 1) * sizeof(T) : 0);
  if (lds > LDS_MAX) return fail(DN_EUNSUPPORTED, "ABACUS slice too wide for one matrix-core product");
  allow_lds(shallow_kernel<T, DP, TWO>, lds);
  allow_lds(shallow_kernel<T, DP, TWO, true>, lds);
  const dn_model_desc& d = m->desc;
  const double dr = d.d, W1 = ext + 2 * d.w_c + 1, W2 = ext + 4 * d.w_c + 1;
  const double fl = 2.0 * dr * dr * (W1 + (TWO ? 2.0 * W2 : 0.0)) + (TWO ? 2.0 * dr * W1 * W2 : 0.0);
  const double by = (TWO ? (2.0 * W1 + 4.0 * W2 + 2.0 * 5) : (3.0 * W1 + 2.0)) * dr * sizeof(T);
  PScope ps(m, DN_K_TAIL, st, (fl + slice_fl) * F, by * F);
  if (sa.tok > 1)  // tokens of several spins: per-position tables and links
    shallow_kernel<T, DP, TWO, true><<<slm_grid((F + P - 1) / P), 4 * DP, lds, st>>>(sa, a);
  else
    shallow_kernel<T, DP, TWO><<<slm_grid((F + P - 1) / P), 4 * DP, lds, st>>>(sa, a);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

// ABACUS: background forward with caches, the output links, the slice recompute and the
// per-flip update, then the float64 log-ratio. With h_offs the flip counts of each chunk are
// host values; without it every flip launch is sized for Bc * M_max and reads its count from
// the device work list, so the sequence has no host round trip. The error word ab_err is set
// for clusters wider than the slice recurrence covers. ext_max: the widest cluster extent in
// the work list (0 single flips, 2 pairs up to two sites apart).
//   L <= 2: per-sample output links T^(0), T^(1) and block 2's pivot-0 link Lam, then
//           shallow_kernel: per-flip work on the slices only (independent of N).
//   L >= 3: the adjoint tau of the last block, then the exact background propagation of each
//           flip's perturbation through blocks 1..L-1 (deep_kernel), finished per flip.
template <typename T, int DP>
dn_status abacus_exec(dn_model* m, const int8_t* spins, int B, const int32_t* sites, int M_max,
                      const int32_t* offs, const int32_t* cb, const int32_t* cm, const int32_t* h_offs,
                      double* logpsi, double* logratio, int ext_max, hipStream_t st, double* dom = nullptr,
                      bool few = false) {
  const dn_model_desc& d = m->desc;
  const int Np = m->Np, L = d.L, wc = d.w_c;
  // phi injected into the h stream: the input change of block l + 1 is dh^(l) + dphi^(l+1),
  // a vector on S_(l+1) rather than a multiple of E at the cluster, so every depth takes the
  // full-chain propagation (one block: the slices and the per-flip finish)
  const bool inj = d.inject_phi != 0;
  // few: a handful of flips per sample (the sampler's proposals), where building block 2's
  // pivot-0 link per sample costs more than propagating each flip through block 1
  const bool shallow = L <= 2 && !inj && !(few && L == 2);
  // identity map for the background forward
  int32_t *idb, *idm;
  STCHK(identity_map(m, "ab_idb", "ab_idm", B, &idb, &idm, st));
  void *pOm, *perr;
  STCHK(ws_get(m, "ab_Om0", (size_t)B * 2 * sizeof(double), &pOm));
  STCHK(ws_get(m, "ab_err", 4, &perr));
  fill_kernel<int><<<1, 64, 0, st>>>((int*)perr, 1, 0);
  double* Om0 = (double*)pOm;
  CfgMap idmap{idb, idm, sites, M_max};
  CfgMap fmap{cb, cm, sites, M_max};
  fill_kernel<double><<<256, 256, 0, st>>>(logratio, (long)B * M_max * (1 + m->desc.complex_out), 0.0);
  const Tables<T>& tb = tables_of<T>(m);
  const int Wmax = 2 + 2 * L * wc + 1;
  const int ND = lam_nd(wc, ext_max), dlo = -(2 * wc + ext_max);
  // samples per chunk: the flip fields dominate (deep networks: 2 fields of [F][DP][Np])
  const size_t per_flip = shallow ? (size_t)L * Wmax * DP * sizeof(T) + sizeof(int4)
                                  : (size_t)DP * Np * sizeof(T) * 2 + (size_t)(inj ? 2 : 1) * L * Wmax * DP * sizeof(T) +
                                        (size_t)(Np / 64) * SLICE_WIN * DP * sizeof(T);
  const size_t flips_budget = std::max<size_t>(1024, m->flip_budget / per_flip);
  const int Bc_max = (int)std::max<size_t>(1, std::min<size_t>(shallow ? 4096 : 1024, flips_budget / std::max(M_max, 1)));
  // background samples per forward chunk: its caches (a0, chi0, p0 per block, tau and its
  // mixer input; two-block networks also T^(0) with its mixer input and Lam) per sample; a
  // large chunk keeps the forward launches wide, the flips then run in chunks of Bc_max
  // samples inside it
  const bool two = shallow && L == 2;
  const size_t per_sample = (size_t)((inj ? 4 : 3) * L + 4 + (two ? 4 : 0)) * DP * Np * sizeof(T) +
                            (two ? (size_t)d.token * d.N * ND * DP * sizeof(T) : 0);
  const int Bf_max = (int)std::max<size_t>(1, std::min<size_t>(B, ((size_t)6 << 30) / per_sample));
  for (int bf0 = 0; bf0 < B; bf0 += Bf_max) {
  const int Bf = std::min(Bf_max, B - bf0);
  const long fldB = (long)Bf * DP * Np;
  void *pa, *pc, *pp, *ptz, *ptau;
  STCHK(ws_get(m, "ab_a0", (size_t)L * fldB * sizeof(T), &pa));
  STCHK(ws_get(m, "ab_chi0", (size_t)L * fldB * sizeof(T), &pc));
  STCHK(ws_get(m, "ab_p0", (size_t)L * fldB * sizeof(T), &pp));
  STCHK(ws_get(m, "ab_tz", (size_t)2 * fldB * sizeof(T), &ptz));
  STCHK(ws_get(m, "ab_tau", (size_t)2 * fldB * sizeof(T), &ptau));
  T *a0 = (T*)pa, *chi0 = (T*)pc, *p0 = (T*)pp, *tz = (T*)ptz, *tau = (T*)ptau;
  T* phi0 = nullptr;
  if (inj) {
    void* pph;
    STCHK(ws_get(m, "ab_phi0", (size_t)L * fldB * sizeof(T), &pph));
    phi0 = (T*)pph;
  }
  STCHK((forward_chunk<T, DP>(m, spins, idmap, bf0, Bf, Om0 + 2L * bf0, a0, chi0, p0, st, Ckpt<T>(), nullptr, phi0)));
  // tau = G^(L)T D0^(L)T Wk; deep networks read out the last block with Wk + tau, and for
  // shallow ones Wk + tau is the output link of the input (L = 1) or of block 1 (L = 2): the
  // conv adds Wk
  {
    MixArgs<T> a{};
    a.tb = tb; a.N = d.N; a.Np = Np; a.l = L - 1; a.L = L; a.w_c = wc;
    a.periodic = d.bc == DN_BC_PERIODIC; a.C = 2 * Bf; a.chi = chi0 + (long)(L - 1) * fldB; a.out = tz;
    STCHK((launch_mix<T, DP, MIX_TAU>(m, a, 2 * Bf, st)));
    STCHK(launch_conv<T>(m, tz, tau, tb.tapsR + (long)(L - 1) * DP * tap_stride(Np), 2 * Bf, st,
                         DynRange{nullptr, 0, 0}, tb.Wk));
  }
  T* T0 = tau;  // output link of the input change
  T* lam = nullptr;
  if (two) {
    // T^(0) = Wk + G^(1)T D0^(1)T T^(1), T^(1) = Wk + tau
    void *pt0z, *pt0, *plam;
    STCHK(ws_get(m, "ab_t0z", (size_t)2 * fldB * sizeof(T), &pt0z));
    STCHK(ws_get(m, "ab_t0", (size_t)2 * fldB * sizeof(T), &pt0));
    STCHK(ws_get(m, "ab_lam", (size_t)d.token * Bf * d.N * ND * DP * sizeof(T), &plam));
    MixArgs<T> a{};
    a.tb = tb; a.N = d.N; a.Np = Np; a.l = 0; a.L = L; a.w_c = wc;
    a.periodic = d.bc == DN_BC_PERIODIC; a.C = 2 * Bf; a.chi = chi0; a.X = tau; a.out = (T*)pt0z;
    STCHK((launch_mix<T, DP, MIX_TAU>(m, a, 2 * Bf, st)));
    STCHK(launch_conv<T>(m, (T*)pt0z, (T*)pt0, tb.tapsR, 2 * Bf, st, DynRange{nullptr, 0, 0}, tb.Wk));
    T0 = (T*)pt0;
    lam = (T*)plam;
    STCHK((build_lam<T, DP>(m, chi0, Bf, ND, dlo, lam, st)));
  }
  for (int b0 = bf0; b0 < bf0 + Bf; b0 += Bc_max) {
    const int Bc = std::min(Bc_max, bf0 + Bf - b0);
    const int f0 = h_offs ? h_offs[b0] : 0;
    const int F = h_offs ? h_offs[b0 + Bc] - f0 : Bc * M_max;
    const DynRange dyn{h_offs ? nullptr : offs, b0, Bc};
    if (F == 0) continue;
    void *pdchi = nullptr, *pgeom = nullptr, *prho, *pdu, *pw, *pdphi = nullptr;
    if (!shallow) {  // the deep path keeps the slices and the cluster geometry for its later kernels
      STCHK(ws_get(m, "ab_dchi", (size_t)F * L * Wmax * DP * sizeof(T), &pdchi));
      STCHK(ws_get(m, "ab_geom", (size_t)F * sizeof(int4), &pgeom));
    }
    if (inj) STCHK(ws_get(m, "ab_dphi", (size_t)F * L * Wmax * DP * sizeof(T), &pdphi));
    const int nt = Np / 64;
    T* dchi = (T*)pdchi;
    int4* geom = (int4*)pgeom;
    SliceArgs<T> sa{};
    sa.tb = tb; sa.N = d.N; sa.Np = Np; sa.L = L; sa.w_c = wc; sa.periodic = d.bc == DN_BC_PERIODIC;
    sa.act = d.act; sa.F = F; sa.f0 = f0; sa.b0 = bf0; sa.Bc = Bf; sa.map = fmap; sa.spins = spins;
    sa.a0 = a0; sa.chi0 = chi0; sa.dchi = dchi; sa.geom = geom; sa.Wmax = Wmax; sa.err = (int*)perr;
    sa.ext_max = ext_max; sa.dyn = dyn; sa.tok = d.token; sa.phi0 = phi0; sa.dphi = (T*)pdphi;
    double slice_fl = 0.0;
    for (int l = 1; l <= L; ++l) slice_fl += 2.0 * (2 * (l - 1) * wc + 1 + 2 * l * wc + 1) * d.d * d.d;
    // P flips side by side per product (slices are at most 16 sites wide: P >= 4)
    const int Wc = ext_max + 2 * L * wc + 1;
    const int P = slm_flips(Wc);
    const size_t slds = slm_lds_bytes<T>(DP, P, Wc, wc);
    if (P < 1 || slds > LDS_MAX) return fail(DN_EUNSUPPORTED, "ABACUS slice too wide for one matrix-core product");
    if (shallow) {  // slice recompute and per-flip update in one kernel
      Flip12Args<T> a{};
      a.p0 = p0; a.fldB = fldB; a.T0 = T0; a.T1 = tau; a.lam = lam; a.ND = ND; a.dlo = dlo;
      a.lamk = (long)Bf * d.N * ND * DP;
      a.Om0 = Om0; a.logratio = logratio; a.dom = dom; a.cplx = d.complex_out;
      if (L == 2) STCHK((launch_shallow<T, DP, true>(m, sa, a, F, P, Wc, slice_fl, st, ext_max)));
      else STCHK((launch_shallow<T, DP, false>(m, sa, a, F, P, Wc, slice_fl, st, ext_max)));
      continue;
    }
    {
      PScope ps(m, DN_K_SLICE, st, slice_fl * F, (double)F * L * Wmax * d.d * sizeof(T));
      if (inj) {
        allow_lds(slice_mma_kernel<T, DP, true>, slds);
        slice_mma_kernel<T, DP, true><<<slm_grid((F + P - 1) / P), 4 * DP, slds, st>>>(sa);
      } else {
        allow_lds(slice_mma_kernel<T, DP>, slds);
        slice_mma_kernel<T, DP><<<slm_grid((F + P - 1) / P), 4 * DP, slds, st>>>(sa);
      }
      HIPCHK(hipGetLastError());
    }
    if (L == 1) {  // phi injected, one block: no tiled block, the finish takes e^(0) + dphi^(1)
      MixArgs<T> a{};
      a.tb = tb; a.N = d.N; a.Np = Np; a.l = 0; a.L = L; a.w_c = wc;
      a.periodic = d.bc == DN_BC_PERIODIC; a.C = F; a.cfg0 = f0; a.dyn = dyn;
      a.map = fmap; a.b0 = bf0; a.spins = spins; a.geom = geom; a.dchi = dchi; a.Wmax = Wmax;
      a.tau = tau; a.tapsL = tb.taps; a.p0L = p0; a.Om0 = Om0; a.logratio = logratio; a.dom = dom;
      a.cplx = d.complex_out; a.tok = d.token; a.dphi = (T*)pdphi;
      const int WL = 2 + 2 * wc + 1;
      PScope ps(m, DN_K_TAIL, st, 4.0 * F * WL * d.d * d.d + 2.0 * F * WL * WL * d.d, (double)F * WL * d.d * sizeof(T) * 6);
      last_finish_kernel<T, DP, true><<<F, 64, 2 * DP * SLICE_WIN * sizeof(T), st>>>(a);
      HIPCHK(hipGetLastError());
      continue;
    }
    // read-outs of the deep blocks 1 .. L-1 per flip and tile, each stored once
    STCHK(ws_get(m, "ab_rho", (size_t)std::max(L - 1, 1) * F * nt * 2 * sizeof(double), &prho));
    double* rho = (double*)prho;
    void* psp;
    STCHK(ws_get(m, "ab_du", (size_t)F * DP * Np * sizeof(T), &pdu));
    STCHK(ws_get(m, "ab_w", (size_t)F * DP * Np * sizeof(T), &pw));
    STCHK(ws_get(m, "ab_spart", (size_t)F * nt * SLICE_WIN * DP * sizeof(T), &psp));
    T* du = (T*)pdu;
    T* w = (T*)pw;
    for (int l = 1; l <= L - 1; ++l) {
      MixArgs<T> a{};
      a.tb = tb; a.N = d.N; a.Np = Np; a.l = l; a.L = L; a.w_c = wc;
      a.periodic = d.bc == DN_BC_PERIODIC; a.C = F; a.cfg0 = f0; a.dyn = dyn; a.rho_blk = 2L * F * nt;
      a.X = w; a.chi = chi0 + (long)(l - 1) * fldB; a.p0 = p0 + (long)(l - 1) * fldB;
      a.out = du; a.rho = rho; a.map = fmap; a.b0 = bf0; a.spins = spins; a.geom = geom;
      a.dchi = dchi; a.Wmax = Wmax; a.tau = tau;
      a.tapsL = tb.taps + (long)(L - 1) * DP * tap_stride(Np); a.taps1 = tb.taps;
      a.p0L = p0 + (long)(L - 1) * fldB; a.Om0 = Om0; a.logratio = logratio; a.dom = dom; a.slice_part = (T*)psp;
      a.cplx = d.complex_out;
      a.tok = d.token;
      a.dphi = (T*)pdphi;
      // phi injected: block 1's mixer output G^(1) (e^(0) + dphi^(1)) is formed from the taps
      // on S_1, then block 1 runs like any later block
      const bool first = (l == 1) && !inj, last = (l == L - 1);
      if (inj && l == 1) {
        MixArgs<T> aw = a;
        aw.out = w;
        const double Wl = 2 * wc + 1 + ext_max;
        PScope ps(m, DN_K_CONV, st, 2.0 * F * Wl * d.N * d.d, (double)F * d.N * d.d * sizeof(T));
        if (ext_max + 2 * wc + 1 > INJ_W1) return fail(DN_EUNSUPPORTED, "slice S_1 wider than the injected source handles");
        inject_w1_kernel<T, DP><<<std::min(F, 16384), 256, 0, st>>>(aw);
        HIPCHK(hipGetLastError());
      } else if (!first) {
        STCHK(launch_conv<T>(m, du, w, tb.taps + (long)(l - 1) * DP * tap_stride(Np), F, st, dyn));
      }
      STCHK((launch_deep_any<T, DP>(m, a, F, st, Bc, first, last)));
      if (inj && !last) {
        const double Wl = 2 * (l + 1) * wc + 1 + ext_max;
        PScope ps(m, DN_K_MIX_DEEP, st, (double)F * Wl * d.d, 3.0 * F * Wl * d.d * sizeof(T));
        inject_add_kernel<T, DP><<<std::min(F, 16384), 256, 0, st>>>(a);
        HIPCHK(hipGetLastError());
      }
    }
  }
  }
  if (logpsi) logpsi_kernel<<<(B + 255) / 256, 256, 0, st>>>(Om0, nullptr, B, logpsi, m->desc.complex_out);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

dn_status abacus_supported(const dn_model* m) {
  const dn_model_desc& d = m->desc;
  if (2 + 2 * d.L * d.w_c + 1 > SLICE_WIN) return fail(DN_EUNSUPPORTED, "ABACUS slice wider than 16 sites (needs L * w_c <= 6)");
  return DN_OK;
}

// Reads the error word of the last ABACUS pass (synchronises the stream).
dn_status abacus_check(dn_model* m, hipStream_t st) {
  void* perr;
  STCHK(ws_get(m, "ab_err", 4, &perr));
  int herr = 0;
  HIPCHK(hipMemcpyAsync(&herr, perr, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (herr) return fail(DN_EUNSUPPORTED, "a cluster is wider than the ABACUS slice recurrence supports (pairs at distance <= 2, slice narrower than the ring)");
  return DN_OK;
}

template <typename T, int DP>
dn_status logratio_abacus(dn_model* m, const int8_t* spins, int B, const int32_t* sites, const int32_t* n_conn,
                          int M_max, double* logpsi, double* logratio, hipStream_t st) {
  STCHK(abacus_supported(m));
  int32_t *offs, *cb, *cm;
  std::vector<int32_t> h_offs;
  STCHK(plan(m, n_conn, sites, B, M_max, 0, &offs, &cb, &cm, std::max(B * M_max, 1), &h_offs, st, spins));
  const int ext_max = (h_offs[B + 1] & 4) ? (m->desc.token > 1 ? 1 : 2) : 0;
  STCHK((abacus_exec<T, DP>(m, spins, B, sites, M_max, offs, cb, cm, h_offs.data(), logpsi, logratio, ext_max, st)));
  return abacus_check(m, st);
}

template <typename T, int DP>
dn_status logpsi_only(dn_model* m, const int8_t* spins, int B, double* logpsi, hipStream_t st) {
  int32_t *idb, *idm;
  STCHK(identity_map(m, "lp_idb", "lp_idm", B, &idb, &idm, st));
  void* prho;
  STCHK(ws_get(m, "lp_rho", (size_t)B * 2 * sizeof(double), &prho));
  CfgMap idmap{idb, idm, nullptr, 0};
  const size_t chunk = chunk_configs(m, sizeof(T), 5, (size_t)4 << 30);
  for (int c0 = 0; c0 < B; c0 += (int)chunk) {
    const int C = (int)std::min<size_t>(chunk, B - c0);
    STCHK((forward_chunk<T, DP>(m, spins, idmap, c0, C, (double*)prho + 2L * c0, nullptr, nullptr, nullptr, st)));
  }
  logpsi_kernel<<<(B + 255) / 256, 256, 0, st>>>((double*)prho, nullptr, B, logpsi, m->desc.complex_out);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

// ------------------------------------------------------------------------------------------
// Per-sample log-derivatives (hand-written reverse mode with layer-boundary checkpoints).

dn_status ensure_jac(dn_model* m, hipStream_t st) {
  if (m->have_jac) return DN_OK;
  const dn_model_desc& d = m->desc;
  const long nch = (long)(d.L + 1) * d.d, TG = 2L * d.N - 1, NP = 12L * d.s + 1;
  const long n = nch * TG * NP;
  if (!m->jac64 && hipMalloc(&m->jac64, n * sizeof(double)) != hipSuccess)
    return fail(DN_ENOMEM, "hipMalloc failed for the S4 tap Jacobian");
  if (d.prec != DN_PREC_FP64 && !m->jac32 && hipMalloc(&m->jac32, n * sizeof(float)) != hipSuccess)
    return fail(DN_ENOMEM, "hipMalloc failed for the S4 tap Jacobian");
  void* pws;
  const bool per_bc = d.bc == DN_BC_PERIODIC;
  const long per = per_bc ? 2L * (4L * d.s * d.s + d.s + (long)d.s * (9L * d.N + 3))
                          : 2L * (2L * d.s * d.s + d.s + 5L * d.N * d.s);
  // The direction kernels keep 3N (open) or 7N (periodic) complex projections in LDS; the
  // periodic prep kernel adds 2(N+1) doubles to its static arrays. Within the model's N limit
  // both fit; the check keeps a raised limit from turning into a failed launch.
  const size_t dir_lds = (per_bc ? 7 : 3) * (size_t)d.N * sizeof(cx);
  const size_t prep_lds = per_bc ? 2 * ((size_t)d.N + 1) * sizeof(double) : 0;
  if (S4JAC_DIR_STATIC_LDS + dir_lds > LDS_MAX || S4JACP_STATIC_LDS + prep_lds > LDS_MAX)
    return fail(DN_EUNSUPPORTED, "the S4 tap Jacobian of this chain length does not fit in LDS");
  STCHK(ws_get(m, "jac_ws", (size_t)nch * per * sizeof(double), &pws));
  {
    PScope ps(m, DN_K_S4GEN, st, 8.0 * nch * (double)d.N * d.s * d.s * 6, (double)n * 8);
    if (per_bc) {  // the aliased kernel of periodic chains
      allow_lds(s4jacp_prep_kernel, prep_lds);
      allow_lds(s4jacp_dir_kernel, dir_lds);
      s4jacp_prep_kernel<<<nch, S4_THREADS, prep_lds, st>>>(m->params, m->lay.off_s4, d.N, d.d, d.s, (double*)pws,
                                                            m->jac64);
      s4jacp_dir_kernel<<<dim3(nch, 12 * d.s), 256, dir_lds, st>>>(m->params, m->lay.off_s4, d.N, d.d, d.s,
                                                                   (double*)pws, m->jac64);
    } else {
      allow_lds(s4jac_dir_kernel, dir_lds);
      s4jac_prep_kernel<<<nch, S4_THREADS, 0, st>>>(m->params, m->lay.off_s4, d.N, d.d, d.s, (double*)pws, m->jac64);
      s4jac_dir_kernel<<<dim3(nch, 12 * d.s), 256, dir_lds, st>>>(m->params, m->lay.off_s4, d.N, d.d, d.s,
                                                                  (double*)pws, m->jac64);
    }
  }
  if (d.prec != DN_PREC_FP64) convert_kernel<<<1024, 256, 0, st>>>(m->jac64, m->jac32, n);
  HIPCHK(hipGetLastError());
  m->have_jac = true;
  return DN_OK;
}

template <typename T> const T* jac_of(dn_model* m);
template <> const double* jac_of<double>(dn_model* m) { return m->jac64; }
template <> const float* jac_of<float>(dn_model* m) { return m->jac32; }

template <typename T, int DP>
dn_status grad_chunk(dn_model* m, const int8_t* spins, CfgMap idmap, int b0, int Bc, double* logpsi, T* grads,
                     hipStream_t st, int part = 0) {
  const dn_model_desc& d = m->desc;
  const int N = d.N, Np = m->Np, L = d.L, wc = d.w_c, dd = d.d, Wc = 2 * wc + 1;
  const long fld = (long)Bc * DP * Np;
  const long Pn = m->lay.P;
  const long lay = 4L * dd * dd + 3L * dd + (long)Wc * dd;
  const int TG = 2 * N - 1, NPc = 12 * d.s + 1, nmix = L + 1;
  const Tables<T>& tb = tables_of<T>(m);
  auto field = [&](const char* name, long nfields, T** out) -> dn_status {
    void* p;
    STCHK(ws_get(m, name, (size_t)nfields * fld * sizeof(T), &p));
    *out = (T*)p;
    return DN_OK;
  };
  T *ckh, *ckphi, *R, *ta, *tphi, *tchi, *tz, *tzeta, *tv, *tq, *dh, *dq, *dchi, *dv, *du[2], *dzeta, *dz, *da, *dph[2];
  STCHK(field("g_ckh", L, &ckh));
  STCHK(field("g_ckphi", L, &ckphi));
  STCHK(field("g_R", 1, &R));
  T* tmp;
  STCHK(field("g_tmp", 18, &tmp));
  T** slots[] = {&ta, &tphi, &tchi, &tz, &tzeta, &tv, &tq, &dh, &dq, &dchi, &dv, &du[0], &du[1], &dzeta, &dz, &da, &dph[0], &dph[1]};
  for (int i = 0; i < 18; ++i) *slots[i] = tmp + i * fld;
  void *prho, *prho2, *pdom, *pdg;
  STCHK(ws_get(m, "g_rho", (size_t)Bc * 2 * sizeof(double), &prho));
  STCHK(ws_get(m, "g_rho2", (size_t)Bc * 2 * sizeof(double), &prho2));
  STCHK(ws_get(m, "g_dom", (size_t)Bc * 2 * sizeof(double), &pdom));
  STCHK(ws_get(m, "g_dg", (size_t)Bc * nmix * dd * TG * sizeof(T), &pdg));
  double *rho = (double*)prho, *rho2 = (double*)prho2, *dOm = (double*)pdom;
  T* dg = (T*)pdg;
  // forward with checkpoints
  Ckpt<T> ck;
  ck.h = ckh; ck.phi = ckphi; ck.R = R;
  STCHK((forward_chunk<T, DP>(m, spins, idmap, b0, Bc, rho, nullptr, nullptr, nullptr, st, ck)));
  if (logpsi)
    logpsi_kernel<<<(Bc + 255) / 256, 256, 0, st>>>(rho, nullptr, Bc, logpsi + (long)b0 * (1 + m->desc.complex_out),
                                                    m->desc.complex_out);
  // read-out: dOmega, dA and the final mixer's tap gradients
  {
    ReadoutGradArgs<T> a{R, rho, m->omega, m->A64, N, Np, dd, DP, nmix, grads, Pn, m->lay.off_A, dg, dOm};
    a.cplx = d.complex_out;
    a.part = part;
    PScope ps(m, DN_K_OTHER, st, 4.0 * Bc * dd * (double)N, (double)fld * sizeof(T));
    readout_grad_kernel<T><<<dim3(Bc, dd), 256, (size_t)(Np + 1) * sizeof(double), st>>>(a);
  }
  auto outer = [&](const T* P, const T* Q1, const T* Q2, const T* emb, long off) {
    OuterArgs<T> a{P, Q1, Q2, emb, spins, b0, N, Np, dd, DP, grads, Pn, off, d.token};
    PScope ps(m, DN_K_OTHER, st, 2.0 * Bc * dd * dd * (double)N, 2.0 * fld * sizeof(T));
    outer_kernel<T, DP><<<Bc, 256, 0, st>>>(a);
  };
  auto rowdot = [&](const T* P, const T* Q, int use_spins, int shift0, int nshift, long off, const double* dom,
                    int kpos = 0) {
    RowdotArgs<T> a{P, Q, spins, use_spins, b0, N, Np, dd, DP, d.bc == DN_BC_PERIODIC, shift0, nshift, grads, Pn,
                    off, 0, dom ? tb.Wk : nullptr, dom, d.token, kpos};
    rowdot_kernel<T><<<dim3(Bc, dd), 64, 0, st>>>(a);
  };
  T* du_next = nullptr;
  T* dph_next = nullptr;
  int flip = 0;
  for (int l = L; l >= 1; --l) {
    const int tl = l - 1;
    const long base = m->lay.off_layers + (long)tl * lay;
    const long offWD = base, offw = base + dd * dd, offK = offw + dd, offk = offK + (long)Wc * dd,
               offAD = offk + dd, offb = offAD + (long)dd * dd, offU = offb + dd, offV = offU + (long)dd * dd;
    // recompute block l from its checkpoints
    {
      PhiArgs<T> a{};
      a.tb = tb; a.N = N; a.Np = Np; a.l = tl; a.w_c = wc; a.periodic = d.bc == DN_BC_PERIODIC; a.act = d.act;
      a.inject = 0; a.first = (l == 1); a.spins = spins; a.map = idmap; a.cfg0 = b0; a.C = Bc; a.tok = d.token;
      a.phi_in = (l >= 2) ? ckphi + (long)(l - 1) * fld : nullptr;
      a.phi_out = tphi; a.chi_out = tchi; a.a_out = ta; a.u_out = tq; a.rho = rho2;
      a.z_out = tz; a.zeta_out = tzeta;
      STCHK((launch_phi<T, DP>(m, a, Bc, st)));
    }
    STCHK(launch_conv<T>(m, ckh + (long)tl * fld, tv, tb.taps + (long)tl * DP * tap_stride(Np), Bc, st,
                         DynRange{nullptr, 0, 0}, nullptr, true));
    {
      MixArgs<T> a{};
      a.tb = tb; a.N = N; a.Np = Np; a.l = tl; a.L = L; a.w_c = wc; a.periodic = d.bc == DN_BC_PERIODIC;
      a.C = Bc; a.cfg0 = b0; a.X = tv; a.chi = tchi; a.p0_out = tq; a.out = nullptr; a.rho = rho2;
      STCHK((launch_mix<T, DP, MIX_FWD>(m, a, Bc, st, false)));
    }
    // vertex and channel mixing backward
    {
      MixBwdArgs<T> a{tb.Um + (long)tl * DP * DP, tb.Vm + (long)tl * DP * DP, tb.Wk, N, Np, du_next, dOm,
                      tchi, tq, dh, dq, dchi, dv};
      const int nw = Np / 64;
      const size_t lds = (size_t)nw * DP * MIX_XS * sizeof(T);
      allow_lds(mixbwd_kernel<T, DP>, lds);
      PScope ps(m, DN_K_OTHER, st, 4.0 * Bc * (double)N * dd * dd, 6.0 * fld * sizeof(T));
      mixbwd_kernel<T, DP><<<Bc, 64 * nw, lds, st>>>(a);
    }
    outer(dh, tchi, tq, nullptr, offU);
    outer(dq, tv, nullptr, nullptr, offV);
    {
      TapGradArgs<T> a{dv, ckh + (long)tl * fld, N, Np, dd, DP, dg, tl, nmix};
      PScope ps(m, DN_K_OTHER, st, 2.0 * Bc * dd * (double)N * N, 2.0 * fld * sizeof(T));
      tapgrad_kernel<T><<<dim3(Bc, dd), 256, 2 * (size_t)Np * sizeof(T), st>>>(a);
    }
    T* du_cur = du[flip];
    STCHK(launch_conv<T>(m, dv, du_cur, tb.tapsR + (long)tl * DP * tap_stride(Np), Bc, st, DynRange{nullptr, 0, 0},
                         nullptr, true));
    // phi stream backward
    T* dph_cur = dph[flip];
    {
      PhiBwdArgs<T> a{tb.ADm + (long)tl * DP * DP, tb.WDm + (long)tl * DP * DP, tb.Kc + (long)tl * Wc * DP,
                      N, Np, wc, d.bc == DN_BC_PERIODIC, d.act, dchi, tzeta, tz, dph_next, dzeta, dz, da, dph_cur,
                      d.inject_phi ? du_cur : nullptr};
      const size_t lds = (size_t)DP * (Np + 2 * wc + 1) * sizeof(T);
      PScope ps(m, DN_K_OTHER, st, 4.0 * Bc * (double)N * dd * dd, 7.0 * fld * sizeof(T));
      if constexpr (std::is_same<T, double>::value) {
        allow_lds(phibwd_kernel<T, DP, 1>, lds);
        phibwd_kernel<T, DP, 1><<<Bc, 256, lds, st>>>(a);
      } else {
        switch (tiles_per_wave(Np)) {
          case 1: allow_lds(phibwd_kernel<T, DP, 1>, lds); phibwd_kernel<T, DP, 1><<<Bc, 256, lds, st>>>(a); break;
          case 2: allow_lds(phibwd_kernel<T, DP, 2>, lds); phibwd_kernel<T, DP, 2><<<Bc, 256, lds, st>>>(a); break;
          case 3: allow_lds(phibwd_kernel<T, DP, 3>, lds); phibwd_kernel<T, DP, 3><<<Bc, 256, lds, st>>>(a); break;
          default: allow_lds(phibwd_kernel<T, DP, 4>, lds); phibwd_kernel<T, DP, 4><<<Bc, 256, lds, st>>>(a); break;
        }
      }
    }
    outer(dzeta, tphi, nullptr, nullptr, offAD);
    if (l >= 2) outer(da, ckphi + (long)(l - 1) * fld, nullptr, nullptr, offWD);
    else outer(da, nullptr, nullptr, tb.Ephi, offWD);
    rowdot(dzeta, nullptr, 0, 0, 1, offb, nullptr);
    rowdot(dz, nullptr, 0, 0, 1, offk, nullptr);
    rowdot(da, nullptr, 0, 0, 1, offw, nullptr);
    rowdot(dz, ta, 0, -wc, Wc, offK, nullptr);
    du_next = du_cur;
    dph_next = dph_cur;
    flip ^= 1;
  }
  // dE_k: h^(0) = sum_k E_k s(tok i + k) gets du^(1) + the read-out adjoint; dE_phi,k likewise
  for (int k = 0; k < d.token; ++k) {
    rowdot(du_next, nullptr, 1, 0, 1, (long)k * dd, dOm, k);
    rowdot(dph_next, nullptr, 1, 0, 1, (long)(d.token + k) * dd, nullptr, k);
  }
  {
    S4GradArgs<T> a{dg, jac_of<T>(m), Bc, nmix * dd, TG, NPc, grads, Pn, m->lay.off_s4};
    PScope ps(m, DN_K_OTHER, st, 2.0 * Bc * nmix * dd * (double)TG * NPc, (double)Bc * nmix * dd * TG * sizeof(T));
    s4grad_kernel<T><<<dim3(nmix * dd, (Bc + 63) / 64, (NPc + 63) / 64), 256, 0, st>>>(a);
  }
  if (d.d_block > 0 && d.d_block < dd)
    for (int tl = 0; tl < L; ++tl) {
      const long offU = m->lay.off_layers + (long)tl * lay + 2L * dd * dd + 3L * dd + (long)Wc * dd;
      block_grad_mask_kernel<T><<<256, 256, 0, st>>>(grads, Bc, Pn, offU, dd, d.d_block);
    }
  HIPCHK(hipGetLastError());
  return DN_OK;
}

template <typename T, int DP>
dn_status grad_logpsi(dn_model* m, const int8_t* spins, int B, double* logpsi, void* grads_out, const double* w,
                      double* wsum, hipStream_t st) {
  const dn_model_desc& d = m->desc;
  STCHK(ensure_jac(m, st));
  T* grads = (T*)grads_out;
  const long Pn = m->lay.P;
  const int parts = 1 + d.complex_out;  // a complex read-out: real part, then imaginary part
  if (!grads) {
    void* p;
    STCHK(ws_get(m, "g_out", (size_t)parts * B * Pn * sizeof(T), &p));
    grads = (T*)p;
  }
  int32_t *idb, *idm;
  STCHK(identity_map(m, "g_idb", "g_idm", B, &idb, &idm, st));
  CfgMap idmap{idb, idm, nullptr, 0};
  const size_t per = (size_t)DP * m->Np * sizeof(T) * (2 * d.L + 19) +
                     (size_t)(d.L + 1) * d.d * (2 * d.N - 1) * sizeof(T);
  const int Bc_max = (int)std::max<size_t>(1, std::min<size_t>(1024, ((size_t)2 << 30) / per));
  for (int part = 0; part < parts; ++part)
    for (int b0 = 0; b0 < B; b0 += Bc_max) {
      const int Bc = std::min(Bc_max, B - b0);
      STCHK((grad_chunk<T, DP>(m, spins, idmap, b0, Bc, part ? nullptr : logpsi,
                               grads + ((long)part * B + b0) * Pn, st, part)));
    }
  if (w && wsum)
    for (int part = 0; part < parts; ++part)
      wsum_kernel<T><<<(int)std::min<long>(4096, (Pn + 255) / 256), 256, 0, st>>>(grads + (long)part * B * Pn, w, B,
                                                                                     Pn, wsum + (long)part * Pn);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

template <typename T, int DP> struct RunGrad {
  static dn_status run(dn_model* m, const int8_t* s, int B, double* lp, void* g, const double* w, double* ws,
                       hipStream_t st) {
    return grad_logpsi<T, DP>(m, s, B, lp, g, w, ws, st);
  }
};

// Dispatch on element type and padded width.
template <template <typename, int> class F, typename... Args>
dn_status dispatch(dn_model* m, Args... args) {
  const bool dbl = m->desc.prec == DN_PREC_FP64;
  switch (m->DP) {
    case 16: return dbl ? F<double, 16>::run(m, args...) : F<float, 16>::run(m, args...);
    case 32: return dbl ? F<double, 32>::run(m, args...) : F<float, 32>::run(m, args...);
    case 64: return dbl ? F<double, 64>::run(m, args...) : F<float, 64>::run(m, args...);
  }
  return fail(DN_EUNSUPPORTED, "channel width");
}

template <typename T, int DP> struct RunFull {
  static dn_status run(dn_model* m, const int8_t* s, int B, const int32_t* si, const int32_t* nc, int M,
                       double* lp, double* lr, hipStream_t st) {
    return logratio_full<T, DP>(m, s, B, si, nc, M, lp, lr, st);
  }
};
// One half-sweep of the screened typewriter sampler over B chains (see sampler.h): rounds of
// (background + ABACUS changes of every chain's remaining proposals, sequential screened
// acceptance per chain) until no chain froze; one host synchronisation per round.
// Proposals per chain and half-sweep up to which a two-block network's sweep propagates each
// proposal through block 1 rather than building block 2's pivot-0 link per chain.
constexpr int SWEEP_FEW = 32;

template <typename T, int DP> struct RunSweep {
  static dn_status run(dn_model* m, int8_t* spins, int B, int spacing, int parity, const double* r_site,
                       const double* u, double eps, int32_t* accepted, int32_t* refreshes, hipStream_t st,
                       double* eps_buf = nullptr, int32_t* eps_set = nullptr, int n_eps = 0, double gamma = 1.0) {
    const int N = m->desc.N * m->desc.token;  // spins per chain
    const int nblk = (N + spacing - 1) / spacing;
    const int K = (nblk - parity + 1) / 2;
    if (K <= 0) return DN_OK;
    void *psi, *psr, *pnc, *pks, *ppe, *pfr, *plr, *pdom, *pch, *prs;
    STCHK(ws_get(m, "sw_sites", (size_t)B * K * 2 * 4, &psi));
    STCHK(ws_get(m, "sw_sites_r", (size_t)B * K * 2 * 4, &psr));
    STCHK(ws_get(m, "sw_nconn", (size_t)B * 4, &pnc));
    STCHK(ws_get(m, "sw_kstart", (size_t)B * 4, &pks));
    STCHK(ws_get(m, "sw_pending", (size_t)B * 4, &ppe));
    STCHK(ws_get(m, "sw_frozen", 4, &pfr));
    STCHK(ws_get(m, "sw_lr", (size_t)B * K * 8 * (1 + m->desc.complex_out), &plr));
    STCHK(ws_get(m, "sw_dom", (size_t)B * K * 2 * 8, &pdom));
    STCHK(ws_get(m, "sw_chain", (size_t)B * 4, &pch));
    STCHK(ws_get(m, "sw_rows", (size_t)B * N, &prs));
    SweepArgs a{};
    a.B = B; a.N = N; a.K = K; a.spacing = spacing; a.parity = parity; a.eps = eps; a.r_site = r_site; a.u = u;
    a.spins = spins; a.sites = (int32_t*)psi; a.sites_r = (int32_t*)psr; a.n_conn = (int32_t*)pnc;
    a.kstart = (int32_t*)pks; a.pending = (int32_t*)ppe; a.accepted = accepted; a.refreshes = refreshes;
    a.frozen = (int32_t*)pfr; a.dom = (double*)pdom; a.cplx = m->desc.complex_out;
    if (eps_buf) {  // the tolerance buffer and this half-sweep's refresh events
      void *pnf, *ppf, *pen, *pee, *pec;
      STCHK(ws_get(m, "sw_nfrz", (size_t)B * 4, &pnf));
      STCHK(ws_get(m, "sw_pfrz", (size_t)B * 8, &ppf));
      STCHK(ws_get(m, "sw_evn", (size_t)B * K * 4, &pen));
      STCHK(ws_get(m, "sw_eve", (size_t)B * K * 8, &pee));
      STCHK(ws_get(m, "sw_evc", (size_t)B * 4, &pec));
      a.eps_buf = eps_buf; a.n_eps = n_eps;
      a.nfrz = (int32_t*)pnf; a.pfrz = (double*)ppf; a.ev_n = (int32_t*)pen; a.ev_e = (double*)pee;
      a.ev_cnt = (int32_t*)pec;
    }
    const int gs = (int)std::min<long>(4096, ((long)B * K + 255) / 256);
    sweep_init_kernel<<<gs, 256, 0, st>>>(a);
    HIPCHK(hipGetLastError());
    // the first round takes every chain; a refresh round only the chains that froze, gathered
    // into rows of their own (so the background forward and links are rebuilt for them alone)
    int rows = B;
    for (int round = 0;; ++round) {
      a.rows = rows;
      a.chain = round == 0 ? nullptr : (const int32_t*)pch;
      if (round > 0) sweep_list_kernel<<<1, 1024, 0, st>>>(a.kstart, B, K, (int32_t*)pch);
      const int gr = (int)std::min<long>(4096, ((long)rows * std::max(K, N) + 255) / 256);
      sweep_round_kernel<<<gr, 256, 0, st>>>(a, (int8_t*)prs);
      HIPCHK(hipGetLastError());
      const int8_t* rs = round == 0 ? spins : (const int8_t*)prs;
      int32_t *offs, *cb, *cm;
      std::vector<int32_t> h_offs;
      STCHK(plan(m, a.n_conn, a.sites_r, rows, K, 0, &offs, &cb, &cm, std::max(rows * K, 1), &h_offs, st));
      STCHK((abacus_exec<T, DP>(m, rs, rows, a.sites_r, K, offs, cb, cm, h_offs.data(), nullptr, (double*)plr, 0, st,
                                (double*)pdom, K <= SWEEP_FEW)));
      void* pOm;
      STCHK(ws_get(m, "ab_Om0", (size_t)rows * 2 * sizeof(double), &pOm));
      a.Om0 = (const double*)pOm;
      sweep_accept_kernel<<<(rows + 255) / 256, 256, 0, st>>>(a);
      HIPCHK(hipGetLastError());
      int frozen = 0;
      HIPCHK(hipMemcpyAsync(&frozen, a.frozen, 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (!frozen) break;
      rows = frozen;  // the chains that froze are exactly those with proposals left
    }
    if (eps_buf) {
      sweep_eps_kernel<<<1, 1, 0, st>>>(eps_buf, eps_set, n_eps, gamma, a.ev_n, a.ev_e, a.ev_cnt, B, K);
      HIPCHK(hipGetLastError());
    }
    return abacus_check(m, st);
  }
};

// Stochastic-reconfiguration update by conjugate gradients (see sr.h); the residual norm is
// checked on the host every 8 iterations (one synchronisation each).
template <typename T, int DP> struct RunSR {
  static dn_status run(dn_model* m, const void* Ov, const double* E, const double* w, int B, double shift, double eta,
                       int max_iter, double tol, double* delta, double* energy, int32_t* iters, hipStream_t st) {
    const T* O = (const T*)Ov;
    const long P = m->lay.P;
    const int parts = 1 + m->desc.complex_out;  // complex: rows Or then Oi, energies Re E then Im E
    void *pv, *pb, *psc;
    STCHK(ws_get(m, "sr_vec", (size_t)(5 + parts) * P * 8, &pv));
    STCHK(ws_get(m, "sr_smp", (size_t)(1 + 2 * parts) * B * 8, &pb));
    STCHK(ws_get(m, "sr_sc", (8 + SR_DOT_WG) * 8, &psc));
    double *x = (double*)pv, *r = x + P, *p = r + P, *Ap = p + P, *F = Ap + P, *Ob = F + P;  // Ob [parts][P]
    double *wv = (double*)pb, *we = wv + B, *t = we + (long)parts * B, *sc = (double*)psc, *dpart = sc + 8;
    const int rows = parts * B;
    auto dot = [&](const double* u, const double* v, double* out) {
      sr_dot_kernel<<<SR_DOT_WG, 256, 0, st>>>(u, v, P, dpart);
      sr_dot_sum_kernel<<<1, 256, 0, st>>>(dpart, out);
    };
    const int gp = (int)((P + 255) / 256), gv = (int)std::min<long>(1024, (P + 255) / 256);
    // partial sums of the split passes over O (column slices or row segments, one at a time)
    void* ppart;
    STCHK(ws_get(m, "sr_part", (size_t)std::max<long>((long)SR_ROW_SLICES * P, (long)B * SR_ROW_SEGS) * 8, &ppart));
    double* part = (double*)ppart;
    auto colsum = [&](const T* Oq, int nrows, const double* coef, const double* v, double sh, double* out) {
      sr_colsum_part_kernel<T><<<dim3(gp, SR_ROW_SLICES), 256, 0, st>>>(Oq, P, nrows, coef, part);
      sr_colsum_fin_kernel<<<gv, 256, 0, st>>>(part, P, v, sh, out);
    };
    auto rowdot = [&](const T* Oq, const double* v, const double* sub, double* tq) {
      sr_rowdot_part_kernel<T><<<dim3((B + SR_ROW_BLK - 1) / SR_ROW_BLK, SR_ROW_SEGS), 256, 0, st>>>(Oq, P, B, v, part);
      sr_rowdot_fin_kernel<<<(B + 255) / 256, 256, 0, st>>>(part, B, sub, wv, tq);
    };
    for (int q = 0; q < parts; ++q) {
      sr_energy_kernel<<<1, 1024, 0, st>>>(E + q, parts, w, B, wv, we + (long)q * B, sc + 5 + q);
      colsum(O + (long)q * B * P, B, wv, nullptr, 0.0, Ob + (long)q * P);
    }
    colsum(O, rows, we, nullptr, 0.0, F);
    sr_init_kernel<<<gv, 256, 0, st>>>(x, r, p, F, P);
    dot(F, F, sc + 0);
    dot(F, F, sc + 4);
    HIPCHK(hipGetLastError());
    double h[8] = {};
    HIPCHK(hipMemcpyAsync(h, sc, 8 * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double fnorm = std::sqrt(h[4]);
    int it = 0;
    if (fnorm > 0.0) {
      for (it = 1; it <= max_iter; ++it) {
        for (int q = 0; q < parts; ++q) {
          double* sub = sc + (q ? 7 : 3);
          dot(Ob + (long)q * P, p, sub);
          rowdot(O + (long)q * B * P, p, sub, t + (long)q * B);
        }
        colsum(O, rows, t, p, shift, Ap);
        dot(p, Ap, sc + 1);
        sr_step_kernel<<<gv, 256, 0, st>>>(x, r, p, Ap, P, sc);
        dot(r, r, sc + 2);
        sr_dir_kernel<<<gv, 256, 0, st>>>(p, r, P, sc);
        sr_roll_kernel<<<1, 1, 0, st>>>(sc);
        HIPCHK(hipGetLastError());
        if (it % 8 == 0 || it == max_iter) {
          HIPCHK(hipMemcpyAsync(h, sc, 8 * 8, hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          if (std::sqrt(h[0]) <= tol * fnorm) break;
        }
      }
      if (it > max_iter) it = max_iter;
    }
    sr_scale_kernel<<<gv, 256, 0, st>>>(x, eta, P, delta);
    if (energy) HIPCHK(hipMemcpyAsync(energy, sc + 5, 8 * parts, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipGetLastError());
    if (iters) *iters = it;
    return DN_OK;
  }
};

template <typename T, int DP> struct RunAbacus {
  static dn_status run(dn_model* m, const int8_t* s, int B, const int32_t* si, const int32_t* nc, int M,
                       double* lp, double* lr, hipStream_t st) {
    return logratio_abacus<T, DP>(m, s, B, si, nc, M, lp, lr, st);
  }
};
// ------------------------------------------------------------------------------------------
// Entry point that allocates nothing: log psi with its forward fields, work list and read-out
// sums in a file-scope device array. Each GPU holds its own copy for the life of the process;
// host code uses the address hipGetSymbolAddress reports for the current device, never the
// array's name.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The current device's scratch address, taken once per device with that device current.
dn_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(DN_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DN_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DN_OK;
}

// Bytes of scratch one configuration of this model needs: the five forward fields, its
// work-list entry and its two read-out sums.
size_t noalloc_bytes_per_config(const dn_model* m) {
  const size_t elem = m->desc.prec == DN_PREC_FP64 ? 8 : 4;
  return 5 * (size_t)m->DP * m->Np * elem + 2 * sizeof(int32_t) + 2 * sizeof(double);
}

// log psi of B configurations in chunks that fit the scratch array (layout per chunk of C:
// fields [5][C][DP][Np], read-out sums [C][2] float64, work list cb [C], cm [C]).
template <typename T, int DP> struct RunLogpsiNoAlloc {
  static dn_status run(dn_model* m, const int8_t* spins, int B, double* logpsi, hipStream_t st) {
    void* base;
    STCHK(scratch_address(&base));
    const int C_max = (int)std::min<size_t>(B, NOALLOC_SCRATCH_BYTES / noalloc_bytes_per_config(m));
    const long fld = (long)C_max * DP * m->Np;
    T* fields = (T*)base;
    double* rho = (double*)(fields + 5 * fld);
    int32_t* cb = (int32_t*)(rho + 2L * C_max);
    int32_t* cm = cb + C_max;
    for (int c0 = 0; c0 < B; c0 += C_max) {
      const int C = std::min(C_max, B - c0);
      identity_map_kernel<<<(C + 255) / 256, 256, 0, st>>>(cb, cm, C);
      CfgMap idmap{cb, cm, nullptr, 0};
      STCHK((forward_chunk<T, DP>(m, spins + (long)c0 * m->desc.N * m->desc.token, idmap, 0, C, rho, nullptr, nullptr,
                                  nullptr, st,
                                  Ckpt<T>(), fields)));
      logpsi_kernel<<<(C + 255) / 256, 256, 0, st>>>(rho, nullptr, C, logpsi + (long)c0 * (1 + m->desc.complex_out),
                                                     m->desc.complex_out);
      HIPCHK(hipGetLastError());
    }
    return DN_OK;
  }
};

template <typename T, int DP> struct RunLogpsi {
  static dn_status run(dn_model* m, const int8_t* s, int B, double* lp, hipStream_t st) {
    return logpsi_only<T, DP>(m, s, B, lp, st);
  }
};

bool check_desc(const dn_model_desc* d, std::string* why) {
  if (!d) { *why = "null descriptor"; return false; }
  if (d->N < 2 || d->N > 512) { *why = "N must be in [2, 512]"; return false; }
  if (d->L < 1 || d->L > 8) { *why = "L must be in [1, 8]"; return false; }
  if (d->d < 1 || d->d > 64) { *why = "d must be in [1, 64]"; return false; }
  if (d->s < 1 || d->s > S4_SMAX) { *why = "s must be in [1, 32]"; return false; }
  if (d->d_out != 2) { *why = "d_out must be 2"; return false; }
  if (d->w_c < 0 || d->w_c > 3) { *why = "w_c must be in [0, 3]"; return false; }
  if (d->N <= 2 * d->w_c) { *why = "N must exceed 2 w_c"; return false; }
  if (d->bc != DN_BC_OPEN && d->bc != DN_BC_PERIODIC) { *why = "bad bc"; return false; }
  if (d->act < 0 || d->act > 2) { *why = "bad act"; return false; }
  if (d->inject_phi != 0 && d->inject_phi != 1) { *why = "inject_phi must be 0 or 1"; return false; }
  if (d->prec < 0 || d->prec > 2) { *why = "bad prec"; return false; }
  if (d->complex_out != 0 && d->complex_out != 1) { *why = "complex_out must be 0 or 1"; return false; }
  if (d->token < 0 || d->token > 4) { *why = "token must be in [0, 4] (0 = 1)"; return false; }
  if (d->d_block < 0 || (d->d_block > 0 && d->d % d->d_block != 0)) {
    *why = "d_block must be 0 or divide d";
    return false;
  }
  return true;
}

// Connected elements with a caller-provided coupling table Jr [N].
dn_status connected_launch(const dn_ham_desc* ham, const int8_t* spins, int B, int N, int M_max, double* Jr,
                           int32_t* sites, double* helem, int32_t* n_conn, double* hdiag, hipStream_t st) {
  if (ham->kind == DN_H_LRTFIM)
    ising_table_kernel<<<1, 64, 0, st>>>(N, ham->bc == DN_BC_PERIODIC, ham->J, ham->alpha, ham->paper_form, Jr);
  const double cx = ham->paper_form ? -ham->h : ham->h;
  connected_kernel<<<B, 64, 0, st>>>(ham->kind, ham->bc == DN_BC_PERIODIC, cx, ham->J1, ham->J2, Jr, spins, N,
                                     M_max, sites, helem, n_conn, hdiag);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

dn_status check_ham(const dn_ham_desc* ham, int N, int M_max) {
  if (ham->kind != DN_H_LRTFIM && ham->kind != DN_H_J1J2) return fail(DN_EINVAL, "bad Hamiltonian kind");
  if (ham->bc != DN_BC_OPEN && ham->bc != DN_BC_PERIODIC) return fail(DN_EINVAL, "bad Hamiltonian bc");
  if (ham->kind == DN_H_LRTFIM && M_max < N) return fail(DN_EINVAL, "M_max must be >= N for the Ising chain");
  if (ham->kind == DN_H_J1J2 && M_max < 2 * N) return fail(DN_EINVAL, "M_max must be >= 2N for the J1-J2 chain");
  if (ham->kind == DN_H_J1J2 && N < 5) return fail(DN_EINVAL, "the J1-J2 chain needs N >= 5");
  return DN_OK;
}

// ------------------------------------------------------------------------------------------
// Ragged batches: instances of different shapes, one model each, in one submission.

struct RaggedInst {
  dn_model* m;
  dn_ham_desc ham;
  const int8_t* spins;
  int B, M_max;
  double* logpsi;  // nullable
  double* eloc;
};

// One instance: generator, work list, ABACUS log-ratios and E_loc, every flip launch
// counted on the device. No host round trip; nothing is allocated once the model's
// workspace has reached this instance's size.
template <typename T, int DP> struct RunInst {
  static dn_status run(dn_model* m, const RaggedInst* in, hipStream_t st) {
    const int B = in->B, M = in->M_max, N = m->desc.N * m->desc.token;  // spins
    void *ps, *ph, *pn, *pd, *pl, *pj;
    STCHK(ws_get(m, "rg_sites", (size_t)B * M * 2 * 4, &ps));
    STCHK(ws_get(m, "rg_helem", (size_t)B * M * 8, &ph));
    STCHK(ws_get(m, "rg_nconn", (size_t)B * 4, &pn));
    STCHK(ws_get(m, "rg_hdiag", (size_t)B * 8, &pd));
    STCHK(ws_get(m, "rg_lr", (size_t)B * M * 8 * (1 + m->desc.complex_out), &pl));
    STCHK(ws_get(m, "rg_Jr", (size_t)N * 8, &pj));
    int32_t* sites = (int32_t*)ps;
    int32_t* nconn = (int32_t*)pn;
    {
      const double Nr = N;
      PScope g(m, DN_K_GEN, st, in->ham.kind == DN_H_LRTFIM ? (double)B * Nr * Nr : (double)B * 8 * Nr,
               (double)B * (Nr + M * 16.0 + 12));
      STCHK(connected_launch(&in->ham, in->spins, B, N, M, (double*)pj, sites, (double*)ph, nconn, (double*)pd, st));
    }
    int32_t *offs, *cb, *cm;
    STCHK(plan_launch(m, nconn, sites, B, M, 0, &offs, &cb, &cm, std::max(B * M, 1), st));
    // the J1-J2 generator emits pairs up to two sites apart, the Ising one single flips
    const int ext_max = in->ham.kind == DN_H_J1J2 ? (m->desc.token > 1 ? 1 : 2) : 0;
    STCHK((abacus_exec<T, DP>(m, in->spins, B, sites, M, offs, cb, cm, nullptr, in->logpsi, (double*)pl, ext_max, st)));
    PScope e(m, DN_K_ELOC, st, 3.0 * B * M, (double)B * M * 16.0 + B * 20.0);
    eloc_kernel<<<B, 64, 0, st>>>((double*)pd, (double*)ph, nconn, (double*)pl, M, in->eloc, m->desc.complex_out);
    HIPCHK(hipGetLastError());
    return DN_OK;
  }
};

// Synchronises st and reads an instance's error words (work list, then ABACUS).
dn_status inst_check(dn_model* m, int B, hipStream_t st) {
  void* po;
  STCHK(ws_get(m, "plan_offs", (size_t)(B + 2) * 4, &po));
  int bits = 0;
  HIPCHK(hipMemcpyAsync(&bits, (int32_t*)po + B + 1, 4, hipMemcpyDeviceToHost, st));
  STCHK(abacus_check(m, st));
  return plan_errors(bits);
}

// Cost model of one instance (for the eager schedule): background forward plus, per flip,
// the deep propagation (full-chain channel mixing and Toeplitz products of blocks 2..L).
double inst_cost(const RaggedInst& in) {
  const double Np = in.m->Np, d = in.m->DP, L = in.m->desc.L;
  const double fwd = L * (8.0 * Np * d * d + 2.0 * Np * Np * d);
  const double flip = 4.0 * Np * d * d * std::max(1.0, L - 1) + 2.0 * Np * Np * d * std::max(0.0, L - 2);
  return in.B * (fwd + in.M_max * flip);
}

// Heaviest first onto the least-loaded of K lanes.
std::vector<std::vector<int>> lpt_lanes(const std::vector<double>& cost, int K) {
  std::vector<int> order(cost.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<std::vector<int>> lanes(K);
  std::vector<double> load(K, 0.0);
  for (int i : order) {
    int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lanes[k].push_back(i);
    load[k] += cost[i];
  }
  return lanes;
}

// Library streams and events of one device (created on first use, kept until exit).
struct StreamPool {
  int dev = -1;
  std::vector<hipStream_t> st;
  std::vector<hipEvent_t> ev;
};

struct RaggedPlan {
  std::vector<uint64_t> key, uids;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t stamp = 0;
  ~RaggedPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

std::mutex g_rg_mu;
std::vector<StreamPool> g_pools;
std::vector<RaggedPlan*> g_rg_cache;  // at most RG_CACHE plans, least recently used dropped
uint64_t g_rg_clock = 0;
constexpr size_t RG_CACHE = 8;

dn_status get_pool(int dev, int K, StreamPool** out) {
  StreamPool* p = nullptr;
  for (auto& q : g_pools) if (q.dev == dev) p = &q;
  if (!p) { g_pools.push_back(StreamPool{}); p = &g_pools.back(); p->dev = dev; }
  while ((int)p->st.size() < K) {
    hipStream_t s;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    p->st.push_back(s);
  }
  while ((int)p->ev.size() < K + 1) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    p->ev.push_back(e);
  }
  *out = p;
  return DN_OK;
}

uint64_t dbits(double x) {
  uint64_t u;
  std::memcpy(&u, &x, 8);
  return u;
}

std::vector<uint64_t> ragged_key(const std::vector<RaggedInst>& ins, int K, int dev) {
  std::vector<uint64_t> k{(uint64_t)ins.size(), (uint64_t)K, (uint64_t)dev};
  for (auto& in : ins) {
    const dn_ham_desc& h = in.ham;
    // launch shapes and the product mode are recorded into the graph as well
    k.insert(k.end(), {(uint64_t)in.m->conv_nt, (uint64_t)in.m->flip_budget, (uint64_t)in.m->split3});
    k.insert(k.end(), {in.m->uid, in.m->ws_gen, (uint64_t)in.B, (uint64_t)(uintptr_t)in.spins,
                       (uint64_t)(uintptr_t)in.logpsi, (uint64_t)(uintptr_t)in.eloc, (uint64_t)h.kind,
                       (uint64_t)h.bc, (uint64_t)h.paper_form, dbits(h.J), dbits(h.alpha), dbits(h.h),
                       dbits(h.J1), dbits(h.J2)});
  }
  return k;
}

// Instances on K lanes: lane 0 is `main`, lanes 1..K-1 the pool's streams, forked from
// and joined back into `main` by events.
dn_status ragged_lanes(std::vector<RaggedInst>& ins, const std::vector<std::vector<int>>& lanes, StreamPool* pool,
                       hipStream_t main) {
  const int K = (int)lanes.size();
  if (K > 1) HIPCHK(hipEventRecord(pool->ev[0], main));
  for (int k = 1; k < K; ++k) HIPCHK(hipStreamWaitEvent(pool->st[k], pool->ev[0], 0));
  for (int k = 0; k < K; ++k) {
    hipStream_t sk = k == 0 ? main : pool->st[k];
    for (int i : lanes[k]) STCHK(dispatch<RunInst>(ins[i].m, (const RaggedInst*)&ins[i], sk));
  }
  for (int k = 1; k < K; ++k) {
    HIPCHK(hipEventRecord(pool->ev[k], pool->st[k]));
    HIPCHK(hipStreamWaitEvent(main, pool->ev[k], 0));
  }
  return DN_OK;
}

// Records the submission into a graph on the pool's capture stream.
dn_status ragged_capture(std::vector<RaggedInst>& ins, const std::vector<std::vector<int>>& lanes, StreamPool* pool,
                         hipGraph_t* out) {
  *out = nullptr;
  hipStream_t cap = pool->st[0];
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  g_capturing = true;
  dn_status s = ragged_lanes(ins, lanes, pool, cap);
  g_capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cap, &g);
  if (s != DN_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  HIPCHK(e);
  *out = g;
  return DN_OK;
}

// First call of a graph-mode submission: every instance in turn on `st`, timed, checked.
dn_status ragged_first(std::vector<RaggedInst>& ins, hipStream_t st, std::vector<double>* ms) {
  std::vector<hipEvent_t> ev(ins.size() + 1, nullptr);
  dn_status s = DN_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) s = fail(DN_EHIP, "hipEventCreate failed");
  if (s == DN_OK && hipEventRecord(ev[0], st) != hipSuccess) s = fail(DN_EHIP, "hipEventRecord failed");
  for (size_t i = 0; i < ins.size() && s == DN_OK; ++i) {
    s = dispatch<RunInst>(ins[i].m, (const RaggedInst*)&ins[i], st);
    if (s == DN_OK && hipEventRecord(ev[i + 1], st) != hipSuccess) s = fail(DN_EHIP, "hipEventRecord failed");
  }
  for (size_t i = 0; i < ins.size() && s == DN_OK; ++i) s = inst_check(ins[i].m, ins[i].B, st);
  ms->assign(ins.size(), 0.0);
  for (size_t i = 0; i < ins.size() && s == DN_OK; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) s = fail(DN_EHIP, "hipEventElapsedTime failed");
    (*ms)[i] = t;
  }
  for (auto e : ev) if (e) (void)hipEventDestroy(e);
  return s;
}

void ragged_forget(uint64_t uid) {
  std::lock_guard<std::mutex> g(g_rg_mu);
  for (size_t i = 0; i < g_rg_cache.size();) {
    auto& u = g_rg_cache[i]->uids;
    if (std::find(u.begin(), u.end(), uid) != u.end()) {
      delete g_rg_cache[i];
      g_rg_cache.erase(g_rg_cache.begin() + i);
    } else {
      ++i;
    }
  }
}

}  // namespace

extern "C" {

int64_t dn_param_count(const dn_model_desc* desc) {
  Layout lo;
  if (!desc || !layout_of(*desc, &lo)) return -1;
  return lo.P;
}

const char* dn_last_error(void) { return g_err.c_str(); }

dn_status dn_model_create(const dn_model_desc* desc, dn_model** out) {
  std::string why;
  if (!out) return fail(DN_EINVAL, "null output handle");
  *out = nullptr;
  if (!check_desc(desc, &why)) return fail(desc ? DN_EUNSUPPORTED : DN_EINVAL, why);
  if (desc->prec == DN_PREC_BF16_MIXED && desc->d <= 16)
    return fail(DN_EUNSUPPORTED, "BF16-mixed precision needs d > 16 (k-steps of 32 channels)");
  dn_model* m = new dn_model();
  m->desc = *desc;
  if (m->desc.token < 1) m->desc.token = 1;
  layout_of(*desc, &m->lay);
  m->DP = desc->d <= 16 ? 16 : desc->d <= 32 ? 32 : 64;
  m->Np = pad_to(desc->N, 64);
  m->Wc = 2 * desc->w_c + 1;
  const size_t elem = desc->prec == DN_PREC_FP64 ? 8 : 4;
  if ((size_t)m->DP * (m->Np + 2 * desc->w_c) * elem + m->Np * elem > LDS_MAX) {
    delete m;
    return fail(DN_EUNSUPPORTED, "one configuration's field does not fit the on-chip tile at this precision");
  }
  auto get = [&](double** p, long n) -> bool {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<long>(n, 1) * sizeof(double)) != hipSuccess) return false;
    m->owned.push_back(q);
    *p = (double*)q;
    return true;
  };
  const long L = desc->L;
  bool ok = get(&m->params, m->lay.P) && get(&m->taps64, (L + 1) * desc->d * (2L * desc->N - 1)) &&
            get(&m->A64, 2L * m->DP) && get(&m->omega, (long)m->DP * m->Np);
  if (!ok) { delete m; return fail(DN_ENOMEM, "hipMalloc failed for model storage"); }
  if (alloc_tables(m->t64, *m) != DN_OK) { delete m; return DN_ENOMEM; }
  if (desc->prec != DN_PREC_FP64 && alloc_tables(m->t32, *m) != DN_OK) { delete m; return DN_ENOMEM; }
  *out = m;
  return DN_OK;
}

dn_status dn_set_workspace_limit(dn_model* m, size_t bytes) {
  if (!m) return fail(DN_EINVAL, "null model");
  m->ws.limit = bytes;
  return DN_OK;
}

dn_status dn_model_set_params(dn_model* m, const double* params, int on_device, void* stream) {
  if (!m || !params) return fail(DN_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const dn_model_desc& d = m->desc;
  HIPCHK(hipMemcpyAsync(m->params, params, m->lay.P * sizeof(double),
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  const size_t lds = 2 * (size_t)(d.N + 1) * sizeof(double);
  {
    // N state-matrix products of s x s complex entries (8 real flops per complex MAC)
    PScope ps(m, DN_K_S4GEN, st, 8.0 * (d.L + 1) * d.d * (double)d.N * d.s * d.s,
              (d.L + 1.0) * d.d * (2.0 * d.N - 1) * 8);
    s4_taps_kernel<<<(d.L + 1) * d.d, S4_THREADS, lds, st>>>(m->params, m->lay.off_s4, d.N, d.d, d.s,
                                                             d.bc == DN_BC_PERIODIC, m->taps64);
  }
  HIPCHK(hipGetLastError());
  PrepArgs a{};
  a.params = m->params; a.taps64 = m->taps64; a.N = d.N; a.Np = m->Np; a.L = d.L; a.d = d.d; a.DP = m->DP;
  a.s = d.s; a.w_c = d.w_c; a.d_out = d.d_out; a.periodic = d.bc == DN_BC_PERIODIC; a.off_layers = m->lay.off_layers; a.off_A = m->lay.off_A;
  a.tok = d.token;
  a.dblk = d.d_block;
  TableBufs<double>& t = m->t64;
  a.E = t.E; a.Ephi = t.Ephi; a.wE1 = t.wE1; a.WDt = t.WDt; a.ADt = t.ADt; a.Ut = t.Ut; a.Vt = t.Vt;
  a.Um = t.Um; a.Vm = t.Vm; a.wv = t.wv; a.Kc = t.Kc; a.kv = t.kv; a.bv = t.bv; a.taps = t.taps;
  a.tapsR = t.tapsR; a.omega = m->omega; a.Wk = t.Wk; a.A = m->A64; a.ADm = t.ADm; a.WDm = t.WDm;
  a.omN = t.omN; a.Ac = t.Ac;
  {
    PScope ps(m, DN_K_PREP, st, 0.0, (double)table_elems(*m) * 8);
    prep_kernel<<<256, 256, 0, st>>>(a);
    for (int k = 0; k < d.token; ++k)  // one unit-flip table per position inside a token
      ptab_kernel<<<256, 256, 0, st>>>(t.taps, t.Vt, t.E + (long)k * m->DP, m->DP, tap_stride(m->Np),
                                       t.Pq + (long)k * 4 * m->DP * tap_stride(m->Np));
  }
  HIPCHK(hipGetLastError());
  if (d.prec != DN_PREC_FP64) STCHK(convert_tables(m, st));
  STCHK(build_lam_tables(m, st));
  void* pbad;
  STCHK(ws_get(m, "sp_bad", 4, &pbad));
  fill_kernel<int><<<1, 64, 0, st>>>((int*)pbad, 1, 0);
  const long nt = (d.L + 1L) * d.d * (2L * d.N - 1);
  finite_check_kernel<<<256, 256, 0, st>>>(m->taps64, nt, (int*)pbad);
  int hbad = 0;
  HIPCHK(hipMemcpyAsync(&hbad, pbad, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hbad) return fail(DN_EINVAL, "Green's-function taps are not finite (unstable state matrix?)");
  m->have_params = true;
  m->have_jac = false;
  return DN_OK;
}

dn_status dn_model_get_taps(dn_model* m, double* taps_out, void* stream) {
  if (!m || !taps_out) return fail(DN_EINVAL, "null argument");
  if (!m->have_params) return fail(DN_ESTATE, "parameters not set");
  const long n = (m->desc.L + 1L) * m->desc.d * (2L * m->desc.N - 1);
  HIPCHK(hipMemcpyAsync(taps_out, m->taps64, n * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return DN_OK;
}

dn_status dn_logpsi(dn_model* m, const int8_t* spins, int32_t B, double* logpsi, void* stream) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (B < 0) return fail(DN_EINVAL, "B < 0");
  if (!m->have_params) return fail(DN_ESTATE, "parameters not set");
  if (B == 0) return DN_OK;
  if (!spins || !logpsi) return fail(DN_EINVAL, "null argument");
  return dispatch<RunLogpsi>(m, spins, (int)B, logpsi, (hipStream_t)stream);
}

dn_status dn_screened_sweep(dn_model* m, int8_t* spins, int32_t B, int32_t spacing, int32_t parity, const double* r_site,
                            const double* u, double eps, int32_t* accepted, int32_t* refreshes, void* stream) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (B < 0 || spacing < 1 || (parity != 0 && parity != 1) || !(eps >= 0.0))
    return fail(DN_EINVAL, "bad B, spacing, parity or eps");
  if (!m->have_params) return fail(DN_ESTATE, "parameters not set");
  if (B == 0) return DN_OK;
  if (!spins || !r_site || !u || !accepted || !refreshes) return fail(DN_EINVAL, "null argument");
  STCHK(abacus_supported(m));
  return dispatch<RunSweep>(m, spins, (int)B, (int)spacing, (int)parity, r_site, u, eps, accepted, refreshes,
                            (hipStream_t)stream);
}

dn_status dn_screened_sweep_adaptive(dn_model* m, int8_t* spins, int32_t B, int32_t spacing, int32_t parity,
                                     const double* r_site, const double* u, double* eps_buf, int32_t* eps_set,
                                     int32_t n_eps, double gamma, int32_t* accepted, int32_t* refreshes,
                                     void* stream) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (B < 0 || spacing < 1 || (parity != 0 && parity != 1) || n_eps < 1 || !(gamma >= 1.0) || !std::isfinite(gamma))
    return fail(DN_EINVAL, "bad B, spacing, parity, n_eps or gamma");
  if (!m->have_params) return fail(DN_ESTATE, "parameters not set");
  if (B == 0) return DN_OK;
  if (!spins || !r_site || !u || !eps_buf || !eps_set || !accepted || !refreshes) return fail(DN_EINVAL, "null argument");
  STCHK(abacus_supported(m));
  return dispatch<RunSweep>(m, spins, (int)B, (int)spacing, (int)parity, r_site, u, 0.0, accepted, refreshes,
                            (hipStream_t)stream, eps_buf, eps_set, (int)n_eps, gamma);
}

dn_status dn_sr_update(dn_model* m, const void* O, const double* eloc, const double* weights, int32_t B, double shift,
                       double eta, int32_t max_iter, double tol, double* delta, double* energy, int32_t* iters,
                       void* stream) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (B < 1 || !(shift >= 0.0) || !std::isfinite(eta) || max_iter < 1 || !(tol >= 0.0))
    return fail(DN_EINVAL, "bad B, shift, eta, max_iter or tol");
  if (!O || !eloc || !delta) return fail(DN_EINVAL, "null argument");
  return dispatch<RunSR>(m, O, eloc, weights, (int)B, shift, eta, (int)max_iter, tol, delta, energy, iters,
                         (hipStream_t)stream);
}

dn_status dn_logpsi_noalloc(dn_model* m, const int8_t* spins, int32_t B, double* logpsi, void* stream) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (B < 0) return fail(DN_EINVAL, "B < 0");
  if (!m->have_params) return fail(DN_ESTATE, "parameters not set");
  if (B == 0) return DN_OK;
  if (!spins || !logpsi) return fail(DN_EINVAL, "null argument");
  const size_t per = noalloc_bytes_per_config(m);
  if (per > NOALLOC_SCRATCH_BYTES)
    return fail(DN_EUNSUPPORTED, "one configuration needs " + std::to_string(per) + " bytes of scratch; the array holds " +
                                     std::to_string(NOALLOC_SCRATCH_BYTES));
  g_noalloc = true;
  const dn_status st = dispatch<RunLogpsiNoAlloc>(m, spins, (int)B, logpsi, (hipStream_t)stream);
  g_noalloc = false;
  return st;
}

dn_status dn_connected(const dn_ham_desc* ham, const int8_t* spins, int32_t B, int32_t N, int32_t M_max,
                       int32_t* sites, double* helem, int32_t* n_conn, double* hdiag, void* stream) {
  if (!ham) return fail(DN_EINVAL, "null argument");
  if (B < 0 || N < 2) return fail(DN_EINVAL, "bad B or N");
  if (B > 0 && (!spins || !sites || !helem || !n_conn || !hdiag)) return fail(DN_EINVAL, "null argument");
  STCHK(check_ham(ham, N, M_max));
  if (B == 0) return DN_OK;
  hipStream_t st = (hipStream_t)stream;
  thread_local double* tl_Jr = nullptr;
  thread_local int tl_N = 0;
  if (ham->kind == DN_H_LRTFIM && tl_N < N) {
    if (tl_Jr) { HIPCHK(hipStreamSynchronize(st)); HIPCHK(hipFree(tl_Jr)); tl_Jr = nullptr; tl_N = 0; }
    if (hipMalloc(&tl_Jr, (size_t)N * sizeof(double)) != hipSuccess) return fail(DN_ENOMEM, "coupling table");
    tl_N = N;
  }
  return connected_launch(ham, spins, B, N, M_max, tl_Jr, sites, helem, n_conn, hdiag, st);
}

dn_status dn_logratio(dn_model* m, int32_t path, const int8_t* spins, int32_t B, const int32_t* sites,
                      const int32_t* n_conn, int32_t M_max, double* logpsi, double* logratio, void* stream) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (B < 0 || M_max < 1) return fail(DN_EINVAL, "bad B or M_max");
  if (path != DN_PATH_ABACUS && path != DN_PATH_FULL) return fail(DN_EINVAL, "bad path");
  if (!m->have_params) return fail(DN_ESTATE, "parameters not set");
  if ((long)B * (M_max + 1) > (1L << 31) - 1) return fail(DN_EINVAL, "B * (M_max + 1) too large");
  if (B == 0) return DN_OK;
  if (!spins || !sites || !n_conn || !logratio) return fail(DN_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  if (path == DN_PATH_FULL) return dispatch<RunFull>(m, spins, (int)B, sites, n_conn, (int)M_max, logpsi, logratio, st);
  return dispatch<RunAbacus>(m, spins, (int)B, sites, n_conn, (int)M_max, logpsi, logratio, st);
}

dn_status dn_local_energy(const double* hdiag, const double* helem, const int32_t* n_conn, const double* logratio,
                          int32_t B, int32_t M_max, double* eloc, void* stream) {
  if (B < 0 || M_max < 1) return fail(DN_EINVAL, "bad B or M_max");
  if (B == 0) return DN_OK;
  if (!hdiag || !helem || !n_conn || !logratio || !eloc) return fail(DN_EINVAL, "null argument");
  eloc_kernel<<<B, 64, 0, (hipStream_t)stream>>>(hdiag, helem, n_conn, logratio, M_max, eloc, 0);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

dn_status dn_local_energy_complex(const double* hdiag, const double* helem, const int32_t* n_conn,
                                  const double* logratio, int32_t B, int32_t M_max, double* eloc, void* stream) {
  if (B < 0 || M_max < 1) return fail(DN_EINVAL, "bad B or M_max");
  if (B == 0) return DN_OK;
  if (!hdiag || !helem || !n_conn || !logratio || !eloc) return fail(DN_EINVAL, "null argument");
  eloc_kernel<<<B, 64, 0, (hipStream_t)stream>>>(hdiag, helem, n_conn, logratio, M_max, eloc, 1);
  HIPCHK(hipGetLastError());
  return DN_OK;
}

dn_status dn_eloc(dn_model* m, int32_t path, const dn_ham_desc* ham, const int8_t* spins, int32_t B, int32_t M_max,
                  double* logpsi, double* logratio, double* eloc, void* stream) {
  if (!m || !ham) return fail(DN_EINVAL, "null argument");
  if (B < 0) return fail(DN_EINVAL, "B < 0");
  if (B == 0) return DN_OK;
  if (!spins || !logpsi || !eloc) return fail(DN_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  void *ps, *ph, *pn, *pd, *pl;
  STCHK(ws_get(m, "el_sites", (size_t)B * M_max * 2 * 4, &ps));
  STCHK(ws_get(m, "el_helem", (size_t)B * M_max * 8, &ph));
  STCHK(ws_get(m, "el_nconn", (size_t)B * 4, &pn));
  STCHK(ws_get(m, "el_hdiag", (size_t)B * 8, &pd));
  if (!logratio) {
    STCHK(ws_get(m, "el_lr", (size_t)B * M_max * 8 * (1 + m->desc.complex_out), &pl));
    logratio = (double*)pl;
  }
  {
    const double N = m->desc.N;
    PScope g(m, DN_K_GEN, st, ham->kind == DN_H_LRTFIM ? (double)B * N * N : (double)B * 8 * N,
             (double)B * (N + M_max * 16.0 + 12));
    STCHK(dn_connected(ham, spins, B, m->desc.N * m->desc.token, M_max, (int32_t*)ps, (double*)ph, (int32_t*)pn,
                       (double*)pd, stream));
  }
  STCHK(dn_logratio(m, path, spins, B, (int32_t*)ps, (int32_t*)pn, M_max, logpsi, logratio, stream));
  PScope e(m, DN_K_ELOC, st, 3.0 * B * M_max, (double)B * M_max * 16.0 + B * 20.0);
  if (m->desc.complex_out)
    return dn_local_energy_complex((double*)pd, (double*)ph, (int32_t*)pn, logratio, B, M_max, eloc, stream);
  return dn_local_energy((double*)pd, (double*)ph, (int32_t*)pn, logratio, B, M_max, eloc, stream);
}

dn_status dn_grad_logpsi(dn_model* m, const int8_t* spins, int32_t B, double* logpsi, void* grads,
                         const double* weights, double* wsum, void* stream) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (B < 0) return fail(DN_EINVAL, "B < 0");
  if (!m->have_params) return fail(DN_ESTATE, "parameters not set");
  if (B == 0) return DN_OK;
  if (!spins) return fail(DN_EINVAL, "null spins");
  if ((weights == nullptr) != (wsum == nullptr)) return fail(DN_EINVAL, "weights and wsum go together");
  return dispatch<RunGrad>(m, spins, (int)B, logpsi, grads, weights, wsum, (hipStream_t)stream);
}

dn_status dn_profile_enable(dn_model* m, int enable) {
  if (!m) return fail(DN_EINVAL, "null model");
  STCHK(prof_harvest(m));
  if (enable) {
    for (int k = 0; k < DN_K_COUNT; ++k) { m->prof.ms[k] = m->prof.fl[k] = m->prof.by[k] = 0.0; m->prof.n[k] = 0; }
  }
  m->prof.on = enable != 0;
  return DN_OK;
}

dn_status dn_profile_read(dn_model* m, int32_t kind, double* total_ms, int64_t* launches, double* flops,
                          double* bytes) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (kind < 0 || kind >= DN_K_COUNT) return fail(DN_EINVAL, "bad kernel kind");
  STCHK(prof_harvest(m));
  if (total_ms) *total_ms = m->prof.ms[kind];
  if (launches) *launches = m->prof.n[kind];
  if (flops) *flops = m->prof.fl[kind];
  if (bytes) *bytes = m->prof.by[kind];
  return DN_OK;
}

dn_status dn_autotune(dn_model* m, const dn_ham_desc* ham, int32_t B_probe, int32_t* conv_nt_out,
                      int64_t* flip_budget_out, void* stream) {
  if (!m || !ham) return fail(DN_EINVAL, "null argument");
  if (B_probe < 1) return fail(DN_EINVAL, "B_probe < 1");
  if (!m->have_params) return fail(DN_ESTATE, "parameters not set");
  const int N = m->desc.N * m->desc.token, M = ham->kind == DN_H_J1J2 ? 2 * N : N;  // spins
  STCHK(check_ham(ham, N, M));
  STCHK(abacus_supported(m));
  hipStream_t st = (hipStream_t)stream;
  void *ps, *pl, *pe;
  STCHK(ws_get(m, "tu_spins", (size_t)B_probe * N, &ps));
  STCHK(ws_get(m, "tu_lp", (size_t)B_probe * 8 * (1 + m->desc.complex_out), &pl));
  STCHK(ws_get(m, "tu_el", (size_t)B_probe * 8 * (1 + m->desc.complex_out), &pe));
  probe_spins_kernel<<<256, 256, 0, st>>>((int8_t*)ps, (long)B_probe * N, 0x9e3779b9u);
  HIPCHK(hipGetLastError());
  const bool prof = m->prof.on;
  m->prof.on = false;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto run = [&](int nt, size_t budget, float* ms) -> dn_status {
    m->conv_nt = nt;
    m->flip_budget = budget;
    auto once = [&]() {
      return dn_eloc(m, DN_PATH_ABACUS, ham, (const int8_t*)ps, B_probe, M, (double*)pl, nullptr, (double*)pe, st);
    };
    STCHK(once());  // sizes the workspace for this shape
    HIPCHK(hipEventRecord(e0, st));
    STCHK(once());
    STCHK(once());
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    return DN_OK;
  };
  // coordinate search: tiles of the Toeplitz kernel first, then the flip chunk size
  const int Np = m->Np;
  int best_nt = Np >= 256 ? 4 : Np / 64;
  size_t best_budget = (size_t)3 << 30;
  float best = 1e30f, t = 0.f;
  dn_status s = DN_OK;
  for (int nt = 1; nt <= 4 && s == DN_OK; ++nt) {
    if (Np % (16 * nt) != 0) continue;  // the waves' site spans must tile the padded chain
    s = run(nt, best_budget, &t);
    if (s == DN_OK && t < best) { best = t; best_nt = nt; }
  }
  const size_t budgets[] = {(size_t)256 << 20, (size_t)1 << 30, (size_t)3 << 30};
  for (size_t bud : budgets) {
    if (s != DN_OK || bud == ((size_t)3 << 30)) continue;  // 3 GiB was timed above
    s = run(best_nt, bud, &t);
    if (s == DN_OK && t < best) { best = t; best_budget = bud; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  m->prof.on = prof;
  m->conv_nt = best_nt;
  m->flip_budget = best_budget;
  if (s != DN_OK) return s;
  m->tuned = true;
  if (conv_nt_out) *conv_nt_out = best_nt;
  if (flip_budget_out) *flip_budget_out = (int64_t)best_budget;
  return DN_OK;
}

dn_status dn_set_launch_shapes(dn_model* m, int32_t conv_nt, int64_t flip_budget) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (conv_nt < 0 || conv_nt > 4 || (conv_nt && m->Np % (16 * conv_nt) != 0))
    return fail(DN_EINVAL, "conv_nt must be 0 or 1..4 with the padded chain a multiple of 16 conv_nt");
  if (flip_budget < 0) return fail(DN_EINVAL, "flip_budget < 0");
  m->conv_nt = conv_nt;
  m->flip_budget = flip_budget ? (size_t)flip_budget : ((size_t)3 << 30);
  m->tuned = true;
  return DN_OK;
}

dn_status dn_set_product_mode(dn_model* m, int32_t mode) {
  if (!m) return fail(DN_EINVAL, "null model");
  if (mode != DN_PRODUCT_SPLIT3 && mode != DN_PRODUCT_FP32) return fail(DN_EINVAL, "unknown product mode");
  m->split3 = mode == DN_PRODUCT_SPLIT3;
  return DN_OK;
}

dn_status dn_ragged_eloc(int32_t n_inst, dn_model* const* models, const dn_ham_desc* hams,
                         const int8_t* const* spins, const int32_t* B, double* const* logpsi,
                         double* const* eloc, int32_t n_streams, int32_t mode, void* stream) {
  if (n_inst < 0) return fail(DN_EINVAL, "n_inst < 0");
  if (n_inst == 0) return DN_OK;
  if (!models || !hams || !spins || !B || !eloc) return fail(DN_EINVAL, "null argument");
  if (n_streams < 0 || n_streams > 8) return fail(DN_EINVAL, "n_streams must be in [0, 8]");
  if (mode != DN_RAGGED_EAGER && mode != DN_RAGGED_GRAPH) return fail(DN_EINVAL, "bad ragged mode");
  std::vector<RaggedInst> ins;
  for (int i = 0; i < n_inst; ++i) {
    dn_model* m = models[i];
    const std::string at = " (instance " + std::to_string(i) + ")";
    if (!m) return fail(DN_EINVAL, "null model" + at);
    for (int j = 0; j < i; ++j)
      if (models[j] == m) return fail(DN_EINVAL, "each instance needs its own model" + at);
    if (!m->have_params) return fail(DN_ESTATE, "parameters not set" + at);
    const int N = m->desc.N * m->desc.token;  // spins
    const int M = hams[i].kind == DN_H_J1J2 ? 2 * N : N;
    STCHK(check_ham(&hams[i], N, M));
    STCHK(abacus_supported(m));
    if (B[i] < 0) return fail(DN_EINVAL, "B < 0" + at);
    if ((long)B[i] * (M + 1) > (1L << 31) - 1) return fail(DN_EINVAL, "B * (M_max + 1) too large" + at);
    if (B[i] == 0) continue;
    if (!spins[i] || !eloc[i]) return fail(DN_EINVAL, "null spins or eloc" + at);
    ins.push_back(RaggedInst{m, hams[i], spins[i], B[i], M, logpsi ? logpsi[i] : nullptr, eloc[i]});
  }
  if (ins.empty()) return DN_OK;
  hipStream_t st = (hipStream_t)stream;
  const int K = std::min<int>(n_streams == 0 ? 4 : n_streams, (int)ins.size());
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> guard(g_rg_mu);
  StreamPool* pool;
  STCHK(get_pool(dev, K, &pool));
  if (mode == DN_RAGGED_EAGER) {
    std::vector<double> cost;
    for (auto& in : ins) cost.push_back(inst_cost(in));
    return ragged_lanes(ins, lpt_lanes(cost, K), pool, st);
  }
  const std::vector<uint64_t> key = ragged_key(ins, K, dev);
  for (RaggedPlan* p : g_rg_cache) {
    if (p->key == key) {
      p->stamp = ++g_rg_clock;
      HIPCHK(hipGraphLaunch(p->exec, st));
      return DN_OK;
    }
  }
  for (auto& in : ins)
    if (!in.m->tuned) STCHK(dn_autotune(in.m, &in.ham, std::min(in.B, 256), nullptr, nullptr, st));
  std::vector<double> ms;
  STCHK(ragged_first(ins, st, &ms));
  std::vector<uint64_t> gen;
  for (auto& in : ins) gen.push_back(in.m->ws_gen);
  RaggedPlan* p = new RaggedPlan();
  dn_status s = ragged_capture(ins, lpt_lanes(ms, K), pool, &p->graph);
  for (size_t i = 0; s == DN_OK && i < ins.size(); ++i)
    if (ins[i].m->ws_gen != gen[i]) s = fail(DN_EHIP, "workspace moved while recording the ragged graph");
  if (s == DN_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
    s = fail(DN_EHIP, "hipGraphInstantiate failed");
  if (s != DN_OK) { delete p; return s; }
  p->key = ragged_key(ins, K, dev);
  for (auto& in : ins) p->uids.push_back(in.m->uid);
  p->stamp = ++g_rg_clock;
  if (g_rg_cache.size() >= RG_CACHE) {
    auto old = std::min_element(g_rg_cache.begin(), g_rg_cache.end(),
                                [](RaggedPlan* a, RaggedPlan* b) { return a->stamp < b->stamp; });
    delete *old;
    g_rg_cache.erase(old);
  }
  g_rg_cache.push_back(p);
  return DN_OK;
}

void dn_model_destroy(dn_model* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  ragged_forget(m->uid);
  delete m;
}

}  // extern "C"
