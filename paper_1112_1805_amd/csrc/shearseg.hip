// Host side of the shearlet-segmentation library: plan (filter bank, its pruned layout
// and the column work lists on the device), workspace layout, launch orchestration of the
// ADMM of Section 3, and the C ABI declared in include/shearseg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "shearseg.h"
#include "kernels.hpp"
#include "generic.hpp"
#include "grouped.hpp"
#include "tv.hpp"
#include "nl.hpp"

using namespace shs;

struct shs_plan {
  int n, C, q, J, store, eta, M, P, PP, W, NS, device;
  int generic;         // 1: mixed-radix path (N not a power of two)
  int rpb;             // rows per row-pass block
  int rw;              // generic path: rows per wave of the row pass (1, 2 or 4)
  int wpb;             // generic path: waves per row-pass block (1, 2 or 4)
  FftPlan prow, pcol;  // mixed-radix stage lists (generic path)
  float* psi;          // [eta][N][PP] dense filter bank (half spectrum)
  float2* tw;          // [N] exp(-2 pi i m / N), then (power-of-two N) the FFT stage tables
  float* eig;          // [N] 4 sin^2(pi k / N): DFT eigenvalues of one forward-difference pair (TV)
  // pruned layout
  float* psiw;         // filter values inside each column window
  int4* pwin;          // [eta][M+1] {a, L, value offset, 0}
  int4* tcol;          // [eta] {cb, pitch, off_lo, off_hi} of the filtered spectra
  long long t_ls;      // label stride of the filtered spectra (float2)
  // column work lists
  int4* items_syn;     // {strip, flist offset, count, -1}
  int4* items_ana;     // {strip, flist offset, count, partial slot or -1}
  int* flist;          // filter ids, grouped by strip
  int2* strips_ana;    // per strip {first analysis item, items}
  int n_syn, n_ana, n_part;
  int fc_syn;          // filters per synthesis work item
  long long nnz;       // stored filter values
  struct GraphCache* graphs;  // captured steady-state iterations of shs_solve
  char schedule[256];  // chosen launch schedule (shs_plan_describe)
};

// Executable graphs of steady-state ADMM iterations, keyed by everything the captured
// launches bake in (workspace, data term, history, thresholds, iteration count).  Captured
// on a stream of the plan's own and launched on the caller's stream; a few entries, least
// recently used dropped first.  The mutex makes lookups, captures and launches of one plan
// safe from several host threads.
struct GraphCache {
  struct Entry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
  };
  std::mutex mu;
  hipStream_t cap = nullptr;
  std::vector<Entry> entries;   // most recently used last
  static constexpr size_t kMax = 6;
  ~GraphCache() {
    for (Entry& e : entries) (void)hipGraphExecDestroy(e.exec);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

thread_local std::string g_err;

shs_status fail(shs_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(SHS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK(what)                                                                   \
  do {                                                                                    \
    hipError_t e_ = hipGetLastError();                                                    \
    if (e_ != hipSuccess) return fail(SHS_E_DEVICE, std::string("launch ") + what + ": " + hipGetErrorString(e_)); \
  } while (0)

// Makes the plan's device current for the duration of a call and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------- kernel timing
enum KClass {
  KC_ROW_SOLVE, KC_COL_SYN, KC_COL_ANA, KC_COL_FINAL, KC_COL_FWD, KC_ROW_C2R, KC_ROW_R2C, KC_ROW_PRIME,
  KC_ROW_ENERGY, KC_PIXEL, KC_REDUCE, KC_OTHER, KC_BATCH, KC_ROW_SHRINK, KC_ROW_PD, KC_TV_RHS, KC_TV_UPDATE,
  KC_COL_SOLVE, KC_NL_DUAL, KC_NL_PRIMAL, KC_COUNT
};
const char* const kKClassName[KC_COUNT] = {"row_solve", "col_syn", "col_ana", "col_final", "col_fwd", "row_c2r",
                                           "row_r2c", "row_prime", "row_energy", "pixel", "reduce", "other",
                                           "batch_solve", "row_shrink", "row_pd", "tv_rhs", "tv_update",
                                           "col_solve", "nl_dual", "nl_primal"};

struct Prof {
  std::mutex mu;
  bool on = false;
  uint32_t mask = ~0u;                 // kernel classes that are timed (bit per class)
  std::vector<hipEvent_t> pool;        // reused across sessions
  size_t used = 0;
  std::vector<int> cls;                // class of event pair i (events 2i, 2i+1)
};
Prof& prof() {
  static Prof p;
  return p;
}
bool profiling_on() {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  return P.on;
}
// Set while a batch graph is being captured: no timing events inside graphs.
thread_local int g_capturing = 0;
struct CaptureScope {
  CaptureScope() { ++g_capturing; }
  ~CaptureScope() { --g_capturing; }
};

// Brackets the launches made during its lifetime with HIP events on stream s (when on).
struct Timed {
  hipStream_t s;
  hipEvent_t stop = nullptr;
  Timed(hipStream_t s_, int cls) : s(s_) {
    Prof& P = prof();
    if (!P.on || g_capturing || !((P.mask >> cls) & 1u)) return;
    std::lock_guard<std::mutex> g(P.mu);
    while (P.pool.size() < P.used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      P.pool.push_back(e);
    }
    hipEvent_t start = P.pool[P.used];
    stop = P.pool[P.used + 1];
    P.used += 2;
    P.cls.push_back(cls);
    (void)hipEventRecord(start, s);
  }
  ~Timed() {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

size_t store_bytes(int store) { return store == SHS_STORE_F32 ? 4 : 2; }

template <template <int> class F>
int by_size(int n) {
  switch (n) {
    case 64: return F<64>::value;
    case 128: return F<128>::value;
    case 256: return F<256>::value;
    case 512: return F<512>::value;
    case 1024: return F<1024>::value;
    case 2048: return F<2048>::value;
  }
  return 0;
}
template <int N> struct RpbOf { static constexpr int value = RowGeom<N>::RPB; };

// Stage twiddle table of fft_run<L, R, RM> (thread read order), copied from the base table
// exp(-2 pi i m / NT) so both hold identical values.
template <int L, int R, int RM>
void fill_stage_tw(const std::vector<float2>& tw, int NT, float2* out) {
  constexpr int T = L / R;
  const int step = NT / L;
  for (int r = 1; r < R; ++r)
    for (int t = 0; t < T; ++t) out[(r - 1) * T + t] = tw[(r * t * step) % NT];
  for (int r = 1; r < RM; ++r)
    for (int tr = 0; tr < R; ++tr) out[(R - 1) * T + (r - 1) * R + tr] = tw[(r * tr * (L / (R * RM)) * step) % NT];
}
template <int N>
void fill_plan_tw(std::vector<float2>& tw) {
  tw.resize(tw_table_size<N>());
  fill_stage_tw<N / 2, RowGeom<N>::R, RowGeom<N>::RM>(tw, N, tw.data() + row_sw_off<N>());
  fill_stage_tw<N, ColGeom<N>::R, ColGeom<N>::RM>(tw, N, tw.data() + col_sw_off<N>());
}
// Stage table of a mixed-radix transform of length L (gstage): W_{Ns R}^{i k} at
// i Ns + k - 1, copied from the base table of NT = L * step entries.
void fill_stage_tw_g(const FftPlan& pl, const std::vector<float2>& tw, int NT, float2* out) {
  const int L = pl.L, step = NT / L;
  for (int e = 0; e < L; ++e) out[e] = tw[0];
  int Ns = 1;
  for (int s = 0; s < pl.ns; ++s) {
    const int R = pl.radix[s];
    for (int i = 1; i < R; ++i)
      for (int k = 0; k < Ns; ++k)
        if (Ns > 1) out[i * Ns + k - 1] = tw[(long long)i * k * (L / (Ns * R)) * step % NT];
    Ns *= R;
  }
}
void fill_stage_tables(int n, std::vector<float2>& tw) {
  switch (n) {
    case 64: fill_plan_tw<64>(tw); break;
    case 128: fill_plan_tw<128>(tw); break;
    case 256: fill_plan_tw<256>(tw); break;
    case 512: fill_plan_tw<512>(tw); break;
    case 1024: fill_plan_tw<1024>(tw); break;
    case 2048: fill_plan_tw<2048>(tw); break;
  }
}
template <int N> struct WOf { static constexpr int value = ColGeom<N>::W; };

constexpr int kRed1Blocks = 256;
constexpr int kDotBlocks = 1024;

struct Layout {
  size_t g, w, bw, state_end;
  size_t t1, t2, v, z, zs, us, part, parts, red1, sdev, hctr, total;
  long long nrow_parts, nparts;
};

Layout make_layout(const shs_plan* p) {
  Layout L{};
  const size_t n = p->n, nn = n * n, q = p->q, eta = p->eta, P = p->P;
  const size_t plane = n * P;  // float2 per dense spectrum
  size_t off = 0;
  L.g = off;   off = align256(off + q * eta * nn * store_bytes(p->store));
  L.w = off;   off = align256(off + q * nn * 4);
  L.bw = off;  off = align256(off + q * nn * 4);
  L.state_end = off;
  L.t1 = off;  off = align256(off + q * size_t(p->t_ls) * 8);
  L.t2 = off;  off = align256(off + q * size_t(p->t_ls) * 8);
  L.v = off;   off = align256(off + q * plane * 8);
  L.z = off;   off = align256(off + q * plane * 8);
  L.zs = off;  off = align256(off + q * nn * 4);
  L.us = off;  off = align256(off + q * nn * 4);
  L.part = off; off = align256(off + size_t(std::max(p->n_part, 1)) * q * n * p->W * 8);
  L.nrow_parts = (long long)(q * eta) * (n / p->rpb);
  const long long npix = (long long)((nn + 255) / 256);
  L.nparts = L.nrow_parts + std::max<long long>(2 * npix, kDotBlocks);
  L.parts = off; off = align256(off + size_t(L.nparts) * 4 * 8);
  L.red1 = off;  off = align256(off + kRed1Blocks * 4 * 8);
  L.sdev = off;  off = align256(off + 8 * 8);   // totals [0, 5), history row counter at [6]
  L.hctr = L.sdev + 6 * 8;
  L.total = off;
  return L;
}

// ---------------------------------------------------------------- launch recording (batches)
// While a Recorder is installed (this thread), the launchers below append a description of
// each launch, with the grouped kernel of its configuration, instead of launching; the
// batch solve turns one iteration's records of all images into grouped launches.  Each
// record carries the step of the iteration it belongs to.
enum BatchStep { BS_ANA, BS_FINAL, BS_C2R, BS_PIXEL, BS_R2C, BS_FWD, BS_SYN, BS_ROW, BS_REDUCE, BS_COUNT };
enum RecKind { RK_ROW, RK_COL, RK_PIX, RK_REDUCE };
struct LaunchRec {
  int step = 0, kind = 0;
  const void* fn = nullptr;    // grouped kernel of the launch's configuration
  int threads = 0, gx = 0, gy = 0;
  size_t lds = 0;              // dynamic LDS bytes
  RowParams rp{};
  ColParams cp{};
  PixParams pp{};
  GenParams gp{};
  // RK_REDUCE (one image's two-level FP64 reduction)
  double* parts = nullptr;
  long long nparts = 0;
  double* red1 = nullptr;
  double* sdev = nullptr;
  double gamma = 1.0;
};
struct Recorder {
  std::vector<LaunchRec> recs;
  int step = 0;
};
thread_local Recorder* g_rec = nullptr;
void rec_step(int s) {
  if (g_rec) g_rec->step = s;
}
template <class F>
LaunchRec& rec_add(int kind, F fn, int threads, int gx, int gy, size_t lds) {
  LaunchRec r;
  r.step = g_rec->step;
  r.kind = kind;
  r.fn = reinterpret_cast<const void*>(fn);
  r.threads = threads;
  r.gx = gx;
  r.gy = gy;
  r.lds = lds;
  g_rec->recs.push_back(r);
  return g_rec->recs.back();
}

// ---------------------------------------------------------------- per-size launchers
template <int N>
struct Pipe {
  using RG = RowGeom<N>;
  using CG = ColCfg<N>;

  template <int MODE, int ST, bool STATS>
  static void row_t(const RowParams& rp, int channels, hipStream_t s) {
    dim3 grid(N / RG::RPB, channels);
    if (g_rec) {
      rec_add(RK_ROW, &kg_row<N, MODE, ST, STATS>, RG::THREADS, N / RG::RPB, channels, 0).rp = rp;
      return;
    }
    hipLaunchKernelGGL((k_row<N, MODE, ST, STATS>), grid, dim3(RG::THREADS), 0, s, rp);
  }
  static void row(const shs_plan*, int mode, int store, bool stats, const RowParams& rp, int channels, hipStream_t s) {
    switch (mode) {
      case ROW_SOLVE:
        if (store == ST_F32) { stats ? row_t<ROW_SOLVE, ST_F32, true>(rp, channels, s) : row_t<ROW_SOLVE, ST_F32, false>(rp, channels, s); }
        else if (store == ST_BF16) { stats ? row_t<ROW_SOLVE, ST_BF16, true>(rp, channels, s) : row_t<ROW_SOLVE, ST_BF16, false>(rp, channels, s); }
        else { stats ? row_t<ROW_SOLVE, ST_F16, true>(rp, channels, s) : row_t<ROW_SOLVE, ST_F16, false>(rp, channels, s); }
        break;
      case ROW_PRIME:
        if (store == ST_F32) row_t<ROW_PRIME, ST_F32, false>(rp, channels, s);
        else if (store == ST_BF16) row_t<ROW_PRIME, ST_BF16, false>(rp, channels, s);
        else row_t<ROW_PRIME, ST_F16, false>(rp, channels, s);
        break;
      case ROW_C2R: row_t<ROW_C2R, ST_F32, false>(rp, channels, s); break;
      case ROW_R2C: row_t<ROW_R2C, ST_F32, false>(rp, channels, s); break;
      case ROW_ENERGY: row_t<ROW_ENERGY, ST_F32, true>(rp, channels, s); break;
      case ROW_SHRINK: row_t<ROW_SHRINK, ST_F32, false>(rp, channels, s); break;
      case ROW_PD:
        if (store == ST_F32) { stats ? row_t<ROW_PD, ST_F32, true>(rp, channels, s) : row_t<ROW_PD, ST_F32, false>(rp, channels, s); }
        else if (store == ST_BF16) { stats ? row_t<ROW_PD, ST_BF16, true>(rp, channels, s) : row_t<ROW_PD, ST_BF16, false>(rp, channels, s); }
        else { stats ? row_t<ROW_PD, ST_F16, true>(rp, channels, s) : row_t<ROW_PD, ST_F16, false>(rp, channels, s); }
        break;
    }
  }
  static void col(const shs_plan*, int kind, const ColParams& cp, int nblocks, int labels, hipStream_t s) {
    const dim3 grid(nblocks, labels), block(CG::THREADS);
    if (g_rec) {
      LaunchRec* r = nullptr;
      switch (kind) {
        case 0: r = &rec_add(RK_COL, &kg_col_fwd<N>, CG::THREADS, nblocks, labels, 0); break;
        case 1: r = &rec_add(RK_COL, &kg_col_syn<N>, CG::THREADS, nblocks, labels, 0); break;
        case 2: r = &rec_add(RK_COL, &kg_col_ana<N>, CG::THREADS, nblocks, labels, 0); break;
        case 3: r = &rec_add(RK_COL, &kg_col_final<N>, CG::THREADS, nblocks, labels, 0); break;
      }
      if (r) r->cp = cp;
      return;
    }
    switch (kind) {
      case 0: hipLaunchKernelGGL((k_col_fwd<N>), grid, block, 0, s, cp); break;
      case 1: hipLaunchKernelGGL((k_col_syn<N>), grid, block, 0, s, cp); break;
      case 2: hipLaunchKernelGGL((k_col_ana<N>), grid, block, 0, s, cp); break;
      case 3: hipLaunchKernelGGL((k_col_final<N>), grid, block, 0, s, cp); break;
    }
  }
};
enum { COL_FWD = 0, COL_SYN = 1, COL_ANA = 2, COL_FINAL = 3 };

// Dynamic LDS of a generic row-pass block: two half-length buffers of rw rows per wave,
// then the twiddle tables.
size_t row_g_lds_bytes(int M, int rw, int wpb, int n) {
  return (size_t(wpb) * 2 * M * rw + row_tab_len(n)) * sizeof(float2);
}
constexpr size_t kRowGLdsMax = 64 * 1024;   // dynamic LDS a generic row block may take

// Mixed-radix (generic) launchers: runtime N, one row per wave, LDS-resident transforms.
struct GenPipe {
  static GenParams gp(const shs_plan* p) { return GenParams{p->prow, p->pcol, p->n, p->wpb}; }
  template <int MODE, int ST, bool STATS>
  static void row_t(const shs_plan* p, const RowParams& rp, int channels, hipStream_t s) {
    // p->wpb waves per block, p->rw rows per wave
    const dim3 grid(p->n / p->rpb, channels);
    const int threads = 64 * p->wpb;
    const size_t lds = row_g_lds_bytes(p->M, p->rw, p->wpb, p->n);
    if (g_rec) {
      LaunchRec* r = nullptr;
      switch (p->rw) {
        case 4: r = &rec_add(RK_ROW, &kg_row_g<MODE, ST, STATS, 4>, threads, p->n / p->rpb, channels, lds); break;
        case 2: r = &rec_add(RK_ROW, &kg_row_g<MODE, ST, STATS, 2>, threads, p->n / p->rpb, channels, lds); break;
        default: r = &rec_add(RK_ROW, &kg_row_g<MODE, ST, STATS, 1>, threads, p->n / p->rpb, channels, lds); break;
      }
      r->rp = rp;
      r->gp = gp(p);
      return;
    }
    switch (p->rw) {
      case 4: hipLaunchKernelGGL((k_row_g<MODE, ST, STATS, 4>), grid, dim3(threads), lds, s, rp, gp(p)); break;
      case 2: hipLaunchKernelGGL((k_row_g<MODE, ST, STATS, 2>), grid, dim3(threads), lds, s, rp, gp(p)); break;
      default: hipLaunchKernelGGL((k_row_g<MODE, ST, STATS, 1>), grid, dim3(threads), lds, s, rp, gp(p)); break;
    }
  }
  static void row(const shs_plan* p, int mode, int store, bool stats, const RowParams& rp, int channels,
                  hipStream_t s) {
    switch (mode) {
      case ROW_SOLVE:
        if (store == ST_F32) { stats ? row_t<ROW_SOLVE, ST_F32, true>(p, rp, channels, s) : row_t<ROW_SOLVE, ST_F32, false>(p, rp, channels, s); }
        else if (store == ST_BF16) { stats ? row_t<ROW_SOLVE, ST_BF16, true>(p, rp, channels, s) : row_t<ROW_SOLVE, ST_BF16, false>(p, rp, channels, s); }
        else { stats ? row_t<ROW_SOLVE, ST_F16, true>(p, rp, channels, s) : row_t<ROW_SOLVE, ST_F16, false>(p, rp, channels, s); }
        break;
      case ROW_PRIME:
        if (store == ST_F32) row_t<ROW_PRIME, ST_F32, false>(p, rp, channels, s);
        else if (store == ST_BF16) row_t<ROW_PRIME, ST_BF16, false>(p, rp, channels, s);
        else row_t<ROW_PRIME, ST_F16, false>(p, rp, channels, s);
        break;
      case ROW_C2R: row_t<ROW_C2R, ST_F32, false>(p, rp, channels, s); break;
      case ROW_R2C: row_t<ROW_R2C, ST_F32, false>(p, rp, channels, s); break;
      case ROW_ENERGY: row_t<ROW_ENERGY, ST_F32, true>(p, rp, channels, s); break;
      case ROW_SHRINK: row_t<ROW_SHRINK, ST_F32, false>(p, rp, channels, s); break;
      case ROW_PD:
        if (store == ST_F32) { stats ? row_t<ROW_PD, ST_F32, true>(p, rp, channels, s) : row_t<ROW_PD, ST_F32, false>(p, rp, channels, s); }
        else if (store == ST_BF16) { stats ? row_t<ROW_PD, ST_BF16, true>(p, rp, channels, s) : row_t<ROW_PD, ST_BF16, false>(p, rp, channels, s); }
        else { stats ? row_t<ROW_PD, ST_F16, true>(p, rp, channels, s) : row_t<ROW_PD, ST_F16, false>(p, rp, channels, s); }
        break;
    }
  }
  static void col(const shs_plan* p, int kind, const ColParams& cp, int nblocks, int labels, hipStream_t s) {
    const dim3 grid(nblocks, labels), block(256);
    const size_t e = size_t(p->n) * kGW * sizeof(float2);
    const size_t t = size_t(col_tab_len(p->n)) * sizeof(float2);
    if (g_rec) {
      LaunchRec* r = nullptr;
      switch (kind) {
        case 0: r = &rec_add(RK_COL, &kg_colg_fwd, 256, nblocks, labels, t + 2 * e); break;
        case 1: r = &rec_add(RK_COL, &kg_colg_syn, 256, nblocks, labels, t + 3 * e); break;
        case 2: r = &rec_add(RK_COL, &kg_colg_ana, 256, nblocks, labels, t + 3 * e); break;
        case 3: r = &rec_add(RK_COL, &kg_colg_final, 256, nblocks, labels, t + 2 * e); break;
      }
      if (r) {
        r->cp = cp;
        r->gp = gp(p);
      }
      return;
    }
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_colg_fwd, grid, block, t + 2 * e, s, cp, gp(p)); break;
      case 1: hipLaunchKernelGGL(k_colg_syn, grid, block, t + 3 * e, s, cp, gp(p)); break;
      case 2: hipLaunchKernelGGL(k_colg_ana, grid, block, t + 3 * e, s, cp, gp(p)); break;
      case 3: hipLaunchKernelGGL(k_colg_final, grid, block, t + 2 * e, s, cp, gp(p)); break;
    }
  }
};

struct Ops {
  void (*row)(const shs_plan*, int, int, bool, const RowParams&, int, hipStream_t);
  void (*col)(const shs_plan*, int, const ColParams&, int, int, hipStream_t);
};

template <int N>
Ops ops_for() {
  return Ops{&Pipe<N>::row, &Pipe<N>::col};
}

constexpr int kGenericMaxN = 1024;   // largest image side of the mixed-radix path

// Stage list of a mixed-radix transform of length L (radices 16, 8, 4, 2, 9, 3 and the
// primes 5..23); false if L has a larger prime factor.
// Default stage list of length L: empty if L has a prime factor above 23.
std::vector<int> fft_factors(int L) {
  int m = L;
  std::vector<int> rs;
  for (int pr : {23, 19, 17, 13, 11, 7, 5}) while (m % pr == 0) { rs.push_back(pr); m /= pr; }
  while (m % 9 == 0) { rs.push_back(9); m /= 9; }
  while (m % 3 == 0) { rs.push_back(3); m /= 3; }
  while (m % 16 == 0) { rs.insert(rs.begin(), 16); m /= 16; }
  if (m == 2 || m == 4 || m == 8) { rs.insert(rs.begin(), m); m = 1; }
  if (m != 1) rs.clear();
  return rs;
}

// Plan of the stages `rs` (in this order; their product is L).
bool fft_plan_from(int L, const std::vector<int>& rs, FftPlan& pl) {
  pl = FftPlan{};
  pl.L = L;
  long long prod = 1;
  for (int r : rs) prod *= r;
  if (rs.empty() || prod != L || int(rs.size()) > kMaxStages) return false;
  pl.ns = int(rs.size());
  int ns = 1;
  for (int i = 0; i < pl.ns; ++i) {
    pl.radix[i] = rs[i];
    // x / ns = (umulhi(x, mag) + x) >> sh with sh = ceil(log2 ns), mag = floor(2^32 (2^sh - ns) / ns) + 1;
    // exact for every ns <= 2048 and x < 2^21 (x < L * strip width here)
    int sh = 0;
    while ((1 << sh) < ns) ++sh;
    pl.sh[i] = sh;
    pl.mag[i] = ns == 1 ? 0u : unsigned((((unsigned long long)1 << 32) * ((1ull << sh) - ns)) / ns + 1);
    ns *= rs[i];
  }
  return true;
}

bool make_fft_plan(int L, FftPlan& pl) { return fft_plan_from(L, fft_factors(L), pl); }

bool get_ops_pow2(int n, Ops& o);

bool get_ops(const shs_plan* p, Ops& o) {
  if (p->generic) { o = Ops{&GenPipe::row, &GenPipe::col}; return true; }
  return get_ops_pow2(p->n, o);
}

bool get_ops_pow2(int n, Ops& o) {
  switch (n) {
    case 64: o = ops_for<64>(); return true;
    case 128: o = ops_for<128>(); return true;
    case 256: o = ops_for<256>(); return true;
    case 512: o = ops_for<512>(); return true;
    case 1024: o = ops_for<1024>(); return true;
    case 2048: o = ops_for<2048>(); return true;
  }
  return false;
}

int row_class(int mode) {
  switch (mode) {
    case ROW_SOLVE: return KC_ROW_SOLVE;
    case ROW_C2R: return KC_ROW_C2R;
    case ROW_R2C: return KC_ROW_R2C;
    case ROW_PRIME: return KC_ROW_PRIME;
    case ROW_ENERGY: return KC_ROW_ENERGY;
    case ROW_SHRINK: return KC_ROW_SHRINK;
    case ROW_PD: return KC_ROW_PD;
  }
  return KC_OTHER;
}

// Everything a compute call needs, resolved from plan + workspace.
struct Ctx {
  const shs_plan* p;
  Layout L;
  Ops ops;
  char* ws;
  hipStream_t s;
  FilterWeights fw;
  template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

shs_status make_ctx(const shs_plan* p, void* ws, size_t ws_bytes, void* stream, Ctx& c) {
  if (!p) return fail(SHS_E_INVALID, "null plan");
  c.p = p;
  c.L = make_layout(p);
  if (!get_ops(p, c.ops)) return fail(SHS_E_UNSUPPORTED, "unsupported size");
  if (!ws) return fail(SHS_E_WORKSPACE, "null workspace");
  if (ws_bytes < c.L.total)
    return fail(SHS_E_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                                     std::to_string(c.L.total));
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(SHS_E_WORKSPACE, "workspace must be 256-byte aligned");
  c.ws = static_cast<char*>(ws);
  c.s = static_cast<hipStream_t>(stream);
  std::memset(&c.fw, 0, sizeof(c.fw));
  return SHS_OK;
}

SpecLayout dense_layout(const shs_plan* p) { return SpecLayout{nullptr, (long long)p->n * p->P, 1, p->P}; }
SpecLayout pruned_layout(const shs_plan* p) { return SpecLayout{p->tcol, p->t_ls, p->eta, p->P}; }

void run_row(const Ctx& c, int mode, int store, bool stats, RowParams rp, int channels) {
  rp.tw = c.p->tw;
  rp.eta = c.p->eta;
  rp.real_cs = (long long)c.p->n * c.p->n;
  rp.fw = c.fw;
  rp.partials = c.at<double>(c.L.parts);
  Timed tm(c.s, row_class(mode));
  c.ops.row(c.p, mode, store, stats, rp, channels, c.s);
}

ColParams col_params(const Ctx& c, int labels) {
  const shs_plan* p = c.p;
  ColParams cp{};
  cp.psiw = p->psiw;
  cp.pwin = p->pwin;
  cp.tl = pruned_layout(p);
  cp.flist = p->flist;
  cp.strips = p->strips_ana;
  cp.part = c.at<float2>(c.L.part);
  cp.tw = p->tw;
  cp.P = p->P;
  cp.eta = p->eta;
  cp.labels = labels;
  cp.nnz = int(p->nnz);
  cp.inv_n2 = 1.0f / (float(p->n) * float(p->n));
  return cp;
}

void run_col(const Ctx& c, int kind, const ColParams& cp, int nblocks, int labels) {
  static const int cls[4] = {KC_COL_FWD, KC_COL_SYN, KC_COL_ANA, KC_COL_FINAL};
  Timed tm(c.s, cls[kind]);
  c.ops.col(c.p, kind, cp, nblocks, labels, c.s);
}

template <int N>
void launch_col_solve(const ColParams& cp, const float* eig, int nblocks, int labels, hipStream_t s) {
  hipLaunchKernelGGL(k_col_solve<N>, dim3(nblocks, labels), dim3(ColCfg<N>::THREADS), 0, s, cp, eig);
}

// u-step of the TV model on per-label spectra: Z = V / (1 + eigenvalues) column-wise.
void run_col_solve(const Ctx& c, const ColParams& cp, int labels) {
  const shs_plan* p = c.p;
  Timed tm(c.s, KC_COL_SOLVE);
  if (p->generic) {
    const size_t e = size_t(p->n) * kGW * sizeof(float2);
    hipLaunchKernelGGL(k_colg_solve, dim3(p->NS, labels), dim3(256), 2 * e, c.s, cp,
                       GenParams{p->prow, p->pcol, p->n}, p->eig);
    return;
  }
  switch (p->n) {
    case 64: launch_col_solve<64>(cp, p->eig, p->NS, labels, c.s); break;
    case 128: launch_col_solve<128>(cp, p->eig, p->NS, labels, c.s); break;
    case 256: launch_col_solve<256>(cp, p->eig, p->NS, labels, c.s); break;
    case 512: launch_col_solve<512>(cp, p->eig, p->NS, labels, c.s); break;
    case 1024: launch_col_solve<1024>(cp, p->eig, p->NS, labels, c.s); break;
    case 2048: launch_col_solve<2048>(cp, p->eig, p->NS, labels, c.s); break;
  }
}

// S: real images [count][N][N] -> pruned coefficient spectra T1 (count * eta planes).
void enqueue_synthesis(const Ctx& c, const float* real_in, int count) {
  const shs_plan* p = c.p;
  RowParams rp{};
  rp.real_in = real_in;
  rp.spec_out = c.at<float2>(c.L.v);
  rp.lout = dense_layout(p);
  rec_step(BS_R2C);
  run_row(c, ROW_R2C, ST_F32, false, rp, count);
  ColParams cp = col_params(c, count);
  cp.in = c.at<float2>(c.L.v);
  cp.out = c.at<float2>(c.L.v);          // column FFT in place: V -> U
  rec_step(BS_FWD);
  run_col(c, COL_FWD, cp, p->NS, count);
  cp.in = c.at<float2>(c.L.v);
  cp.out = c.at<float2>(c.L.t1);
  cp.items = p->items_syn;
  rec_step(BS_SYN);
  run_col(c, COL_SYN, cp, p->n_syn, count);
}

// Adjoint column side: pruned spectra T2 (count * eta planes) -> Z (count dense planes).
void enqueue_analysis(const Ctx& c, int count) {
  const shs_plan* p = c.p;
  ColParams cp = col_params(c, count);
  cp.in = c.at<float2>(c.L.t2);
  cp.out = c.at<float2>(c.L.z);
  cp.items = p->items_ana;
  rec_step(BS_ANA);
  run_col(c, COL_ANA, cp, p->n_ana, count);
  rec_step(BS_FINAL);
  if (p->n_part > 0) run_col(c, COL_FINAL, cp, p->NS, count);
}

// hist_ctr: NULL (hist_row is the row itself) or the device row counter (hist_row is the
// history's first row).
void enqueue_reduce(const Ctx& c, long long nparts, double* hist_row, double gamma, int* hist_ctr = nullptr) {
  if (g_rec) {
    rec_step(BS_REDUCE);
    LaunchRec& r = rec_add(RK_REDUCE, &k_reduce2, 256, 1, 1, 0);
    r.parts = c.at<double>(c.L.parts);
    r.nparts = nparts;
    r.red1 = c.at<double>(c.L.red1);
    r.sdev = c.at<double>(c.L.sdev);
    r.gamma = gamma;
    return;
  }
  Timed tm(c.s, KC_REDUCE);
  const long long per = (nparts + kRed1Blocks - 1) / kRed1Blocks;
  hipLaunchKernelGGL(k_reduce1, dim3(kRed1Blocks), dim3(256), 0, c.s, c.at<double>(c.L.parts), nparts,
                     std::max<long long>(per, 1), c.at<double>(c.L.red1));
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(256), 0, c.s, c.at<double>(c.L.red1), kRed1Blocks,
                     c.at<double>(c.L.sdev), hist_row, gamma, hist_ctr);
}

// Per-filter weights and thresholds from a host Lambda (J+1 per-scale or eta per-filter).
shs_status set_lambda(Ctx& c, const shs_params* prm) {
  const int eta = c.p->eta, J = c.p->J;
  if (!prm->lambda) return fail(SHS_E_INVALID, "null lambda");
  float lam_f[kMaxFilters] = {};   // eta <= kMaxFilters (J <= 6); no heap allocation
  if (prm->lambda_len == eta) {
    for (int f = 0; f < eta; ++f) lam_f[f] = prm->lambda[f];
  } else if (prm->lambda_len == J + 1) {
    int f = 0;
    lam_f[f++] = prm->lambda[0];
    for (int j = 0; j < J; ++j)
      for (int i = 0; i < (4 << j); ++i) lam_f[f++] = prm->lambda[j + 1];
  } else {
    return fail(SHS_E_INVALID, "lambda_len must be J+1 or eta");
  }
  for (int f = 0; f < eta; ++f)
    if (!(lam_f[f] >= 0.f) || !std::isfinite(lam_f[f]))
      return fail(SHS_E_INVALID, "lambda entries must be finite and >= 0");
  std::memset(&c.fw, 0, sizeof(c.fw));
  for (int f = 0; f < eta; ++f) {
    c.fw.lam[f] = lam_f[f];
    c.fw.thr[f] = prm->gamma * lam_f[f];
  }
  return SHS_OK;
}

// Exact energy <u, s> + sum_l sum_j lambda_j ||S_j u_l||_1 of u [q][N][N] (device), FP64.
shs_status energy_of(const Ctx& c, const float* d_u, const float* d_s, double* out) {
  const shs_plan* p = c.p;
  enqueue_synthesis(c, d_u, p->q);
  RowParams rp{};
  rp.spec_in = c.at<float2>(c.L.t1);
  rp.lin = pruned_layout(p);
  run_row(c, ROW_ENERGY, ST_F32, true, rp, p->q * p->eta);
  LAUNCHCHK("energy rows");
  const long long nn = (long long)p->n * p->n * p->q;
  {
    Timed tm(c.s, KC_OTHER);
    hipLaunchKernelGGL(k_dot, dim3(kDotBlocks), dim3(256), 0, c.s, d_u, d_s, nn,
                       c.at<double>(c.L.parts) + c.L.nrow_parts * 4);
  }
  enqueue_reduce(c, c.L.nrow_parts + kDotBlocks, nullptr, 1.0);
  LAUNCHCHK("energy reduce");
  double tot[8];
  HIPCHK(hipMemcpyAsync(tot, c.at<double>(c.L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  if (tot[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite energy");
  *out = tot[SLOT_WS] + tot[SLOT_L1];
  return SHS_OK;
}

// ---------------------------------------------------------------- plan construction
void free_plan(shs_plan* p) {
  if (!p) return;
  delete p->graphs;
  void* bufs[] = {p->psi, p->tw, p->eig, p->psiw, p->pwin, p->tcol, p->items_syn, p->items_ana, p->flist,
                  p->strips_ana};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete p;
}

template <class T>
shs_status upload(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
  if (hipMalloc(dst, bytes) != hipSuccess) return fail(SHS_E_NOMEM, "plan table allocation");
  if (!v.empty()) HIPCHK(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return SHS_OK;
}

// Column work list: per strip, the filters whose column range meets it, cut into runs of
// at most `fc` filters.  Analysis lists also assign partial-accumulator slots.
void build_items(const std::vector<std::vector<int>>& per_strip, const std::vector<int>& strip_flist_off, int fc,
                 bool with_parts, std::vector<int4>& items, std::vector<int2>* strips, int* nparts) {
  items.clear();
  int slot = 0;
  for (size_t s = 0; s < per_strip.size(); ++s) {
    const int nf = int(per_strip[s].size());
    const int nit = (nf + fc - 1) / fc;
    if (strips) strips->push_back(make_int2(int(items.size()), nit));
    for (int i = 0; i < nit; ++i) {
      const int cnt = std::min(fc, nf - i * fc);
      int part = -1;
      if (with_parts && nit > 1) part = slot++;
      items.push_back(make_int4(int(s), strip_flist_off[s] + i * fc, cnt, part));
    }
  }
  if (nparts) *nparts = slot;
}

// Filters meeting each strip (grouped by strip in flist), kept for re-cutting the synthesis
// work items while the plan is tuned.
struct StripLists {
  std::vector<std::vector<int>> per_strip;
  std::vector<int> strip_off;
};

shs_status build_pruned_layout(shs_plan* p, StripLists* keep) {
  const int n = p->n, half = p->M + 1, eta = p->eta, W = p->W;
  // 1. column windows of every filter
  int2* dwin = nullptr;
  if (hipMalloc(&dwin, size_t(eta) * half * sizeof(int2)) != hipSuccess) return fail(SHS_E_NOMEM, "window scratch");
  hipLaunchKernelGGL(k_filter_windows, dim3((eta * half + 255) / 256), dim3(256), 0, 0, p->psi, n, p->PP, eta, dwin);
  std::vector<int2> win(size_t(eta) * half);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipMemcpy(win.data(), dwin, win.size() * sizeof(int2), hipMemcpyDeviceToHost);
  (void)hipFree(dwin);
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(SHS_E_DEVICE, "filter window scan");
  // 2. compact value offsets and per-filter column ranges (whole strips)
  std::vector<int4> pwin(win.size());
  std::vector<int4> tcol(eta);
  std::vector<int> s0(eta), s1(eta);
  long long off = 0, toff = 0;
  for (int j = 0; j < eta; ++j) {
    int c0 = -1, c1 = -1;
    for (int k1 = 0; k1 < half; ++k1) {
      const int2 w = win[size_t(j) * half + k1];
      pwin[size_t(j) * half + k1] = make_int4(w.x, w.y, int(off), 0);
      off += w.y;
      if (w.y > 0) { if (c0 < 0) c0 = k1; c1 = k1; }
    }
    if (c0 < 0) c0 = c1 = 0;
    s0[j] = c0 / W;
    s1[j] = c1 / W;
    const int cb = s0[j] * W, pitch = (s1[j] - s0[j] + 1) * W;
    tcol[j] = make_int4(cb, pitch, int(toff & 0xffffffffLL), int(toff >> 32));
    toff += (long long)n * pitch;
  }
  if (off >= (1LL << 29)) return fail(SHS_E_UNSUPPORTED, "filter bank too large");
  p->nnz = off;
  p->t_ls = toff;
  // 3. work lists
  std::vector<std::vector<int>> per_strip(p->NS);
  std::vector<int> flist, strip_off(p->NS);
  for (int s = 0; s < p->NS; ++s) {
    for (int j = 0; j < eta; ++j)
      if (s >= s0[j] && s <= s1[j]) per_strip[s].push_back(j);
    strip_off[s] = int(flist.size());
    flist.insert(flist.end(), per_strip[s].begin(), per_strip[s].end());
  }
  const long long pairs = (long long)flist.size();
  const int fc_syn = int(std::min<long long>(kItemMax, std::max<long long>(1, (pairs * p->q + 1249) / 2500)));
  const int fc_ana = int(std::min<long long>(kItemMax, std::max<long long>(2, (pairs * p->q + 749) / 1500)));
  std::vector<int4> isyn, iana;
  std::vector<int2> strips;
  build_items(per_strip, strip_off, fc_syn, false, isyn, nullptr, nullptr);
  build_items(per_strip, strip_off, fc_ana, true, iana, &strips, &p->n_part);
  p->n_syn = int(isyn.size());
  p->n_ana = int(iana.size());
  p->fc_syn = fc_syn;
  if (keep) {
    keep->per_strip = per_strip;
    keep->strip_off = strip_off;
  }
  shs_status st;
  if ((st = upload(&p->pwin, pwin)) != SHS_OK) return st;
  if ((st = upload(&p->tcol, tcol)) != SHS_OK) return st;
  if ((st = upload(&p->items_syn, isyn)) != SHS_OK) return st;
  if ((st = upload(&p->items_ana, iana)) != SHS_OK) return st;
  if ((st = upload(&p->flist, flist)) != SHS_OK) return st;
  if ((st = upload(&p->strips_ana, strips)) != SHS_OK) return st;
  // 4. compact filter values
  if (hipMalloc(&p->psiw, size_t(std::max<long long>(off, 1)) * 4) != hipSuccess) return fail(SHS_E_NOMEM, "psiw");
  hipLaunchKernelGGL(k_filter_compact, dim3(4, std::min(eta * half, 65535)), dim3(256), 0, 0, p->psi, n, p->PP, eta,
                     p->pwin, p->psiw);
  LAUNCHCHK("filter compaction");
  HIPCHK(hipDeviceSynchronize());
  return SHS_OK;
}


shs_status check_params(const shs_params* prm) {
  if (!(prm->gamma > 0.f) || !std::isfinite(prm->gamma)) return fail(SHS_E_INVALID, "gamma must be > 0");
  if (prm->iters < 0) return fail(SHS_E_INVALID, "iters must be >= 0");
  if (prm->tol < 0.0 || (prm->tol > 0.0 && prm->check_every < 1)) return fail(SHS_E_INVALID, "bad tol/check_every");
  return SHS_OK;
}

// Zero ADMM state (v = w = b = 0) with a fill kernel, so that it can be captured in a graph.
void enqueue_zero_state(const Ctx& c) {
  const long long words = (long long)(c.L.state_end / 4);
  hipLaunchKernelGGL(k_fill_u32, dim3(unsigned((words + 255) / 256)), dim3(256), 0, c.s,
                     reinterpret_cast<uint32_t*>(c.ws + c.L.g), words, 0u);
}

void enqueue_epilogue(const Ctx& c, float* d_u, int32_t* d_labels) {
  if (!d_u && !d_labels) return;
  const long long n2 = (long long)c.p->n * c.p->n;
  Timed tm(c.s, KC_OTHER);
  hipLaunchKernelGGL(k_epilogue, dim3(unsigned((n2 + 255) / 256)), dim3(256), 0, c.s, c.at<float>(c.L.w), c.p->q, n2,
                     d_u, d_labels);
}

// One ADMM iteration of one image (Section 3): u-update from the adjoint of the previous
// iteration's (v - b_v) (absent on the first iteration), w/b_w update, forward transform,
// v/b_v update fused with the next adjoint's row FFT (when `emit`), optional FP64 residual
// reduction into `hist_row`.  Enqueues only; no host synchronisation.
void enqueue_iteration(const Ctx& c, const float* d_s, float gamma, bool have_adjoint_input, bool stats, bool emit,
                       double* hist_row, int* hist_ctr = nullptr) {
  const shs_plan* p = c.p;
  const Layout& L = c.L;
  const int q = p->q;
  const long long n2 = (long long)p->n * p->n;
  const long long npix_blocks = (n2 + 255) / 256;
  if (have_adjoint_input) {
    enqueue_analysis(c, q);
    RowParams rz{};
    rz.spec_in = c.at<float2>(L.z);
    rz.lin = dense_layout(p);
    rz.real_out = c.at<float>(L.zs);
    rec_step(BS_C2R);
    run_row(c, ROW_C2R, ST_F32, false, rz, q);
  }
  PixParams pp{};
  pp.z = c.at<float>(L.zs);
  pp.w = c.at<float>(L.w);
  pp.bw = c.at<float>(L.bw);
  pp.s = d_s;
  pp.u = c.at<float>(L.us);
  pp.partials = c.at<double>(L.parts) + L.nrow_parts * 4;
  pp.n2 = n2;
  pp.gamma = gamma;
  pp.q = q;
  rec_step(BS_PIXEL);
  if (g_rec) {
    auto fn = have_adjoint_input ? (stats ? &kg_pixel<true, true> : &kg_pixel<false, true>)
                                 : (stats ? &kg_pixel<true, false> : &kg_pixel<false, false>);
    rec_add(RK_PIX, fn, 256, int(npix_blocks), 1, 0).pp = pp;
  } else {
    Timed tm(c.s, KC_PIXEL);
    const dim3 g{unsigned(npix_blocks)}, b{256};
    if (have_adjoint_input) {
      if (stats) hipLaunchKernelGGL((k_pixel<true, true>), g, b, 0, c.s, pp);
      else hipLaunchKernelGGL((k_pixel<false, true>), g, b, 0, c.s, pp);
    } else {
      if (stats) hipLaunchKernelGGL((k_pixel<true, false>), g, b, 0, c.s, pp);
      else hipLaunchKernelGGL((k_pixel<false, false>), g, b, 0, c.s, pp);
    }
  }
  enqueue_synthesis(c, c.at<float>(L.us), q);
  RowParams rp{};
  rp.spec_in = c.at<float2>(L.t1);
  rp.lin = pruned_layout(p);
  rp.spec_out = c.at<float2>(L.t2);
  rp.lout = pruned_layout(p);
  rp.g = c.ws + L.g;
  rp.emit = emit ? 1 : 0;
  rec_step(BS_ROW);
  run_row(c, ROW_SOLVE, p->store, stats, rp, q * p->eta);
  if (stats) enqueue_reduce(c, L.nrow_parts + npix_blocks, hist_row, gamma, hist_ctr);
}

template <int ST>
void launch_tv_update(bool stats, dim3 grid, hipStream_t s, const TvParams& tp) {
  if (stats) hipLaunchKernelGGL((k_tv_update<ST, true>), grid, dim3(256), 0, s, tp);
  else hipLaunchKernelGGL((k_tv_update<ST, false>), grid, dim3(256), 0, s, tp);
}

TvParams tv_params(const Ctx& c, const float* d_s, float lambda, float gamma) {
  const shs_plan* p = c.p;
  TvParams tp{};
  tp.g = c.ws + c.L.g;
  tp.g_out = c.ws + c.L.g;
  tp.w = c.at<float>(c.L.w);
  tp.bw = c.at<float>(c.L.bw);
  tp.s = d_s;
  tp.u = c.at<float>(c.L.zs);
  tp.rhs = c.at<float>(c.L.us);
  tp.partials = c.at<double>(c.L.parts);
  tp.n = p->n;
  tp.q = p->q;
  tp.gamma = gamma;
  tp.lambda = lambda;
  tp.radius = gamma * lambda;
  return tp;
}

// One ADMM iteration of the TV model: right-hand side (grad^T of v - b_v, w - b_w, data
// term), the u-solve on the DFT (row R2C, column FFT / divide / inverse, row C2R), then
// the pixel update of g, w, b_w with residual partials.
void enqueue_tv_iteration(const Ctx& c, const float* d_s, float lambda, float gamma, bool stats, double* hist_row) {
  const shs_plan* p = c.p;
  const Layout& L = c.L;
  const int q = p->q;
  const long long n2 = (long long)p->n * p->n;
  const dim3 gpix{unsigned((n2 + 255) / 256)}, bpix{256};
  const TvParams tp = tv_params(c, d_s, lambda, gamma);
  {
    Timed tm(c.s, KC_TV_RHS);
    switch (p->store) {
      case ST_F32: hipLaunchKernelGGL((k_tv_rhs<ST_F32>), gpix, bpix, 0, c.s, tp); break;
      case ST_BF16: hipLaunchKernelGGL((k_tv_rhs<ST_BF16>), gpix, bpix, 0, c.s, tp); break;
      default: hipLaunchKernelGGL((k_tv_rhs<ST_F16>), gpix, bpix, 0, c.s, tp); break;
    }
  }
  RowParams rp{};
  rp.real_in = c.at<float>(L.us);
  rp.spec_out = c.at<float2>(L.v);
  rp.lout = dense_layout(p);
  run_row(c, ROW_R2C, ST_F32, false, rp, q);
  ColParams cp = col_params(c, q);
  cp.in = c.at<float2>(L.v);
  cp.out = c.at<float2>(L.z);
  run_col_solve(c, cp, q);
  RowParams rz{};
  rz.spec_in = c.at<float2>(L.z);
  rz.lin = dense_layout(p);
  rz.real_out = c.at<float>(L.zs);
  run_row(c, ROW_C2R, ST_F32, false, rz, q);
  {
    Timed tm(c.s, KC_TV_UPDATE);
    switch (p->store) {
      case ST_F32: launch_tv_update<ST_F32>(stats, gpix, c.s, tp); break;
      case ST_BF16: launch_tv_update<ST_BF16>(stats, gpix, c.s, tp); break;
      default: launch_tv_update<ST_F16>(stats, gpix, c.s, tp); break;
    }
  }
  if (stats) enqueue_reduce(c, (n2 + 255) / 256, hist_row, gamma);
}

// <w, s> + lambda TV(w) (FP64), synchronising.
shs_status tv_energy_of(const Ctx& c, const float* d_s, float lambda, double* out) {
  const long long n2 = (long long)c.p->n * c.p->n;
  TvParams tp = tv_params(c, d_s, lambda, 1.f);
  {
    Timed tm(c.s, KC_OTHER);
    hipLaunchKernelGGL(k_tv_energy, dim3(unsigned((n2 + 255) / 256)), dim3(256), 0, c.s, tp);
  }
  enqueue_reduce(c, (n2 + 255) / 256, nullptr, 1.0);
  LAUNCHCHK("tv energy");
  double tot[8];
  HIPCHK(hipMemcpyAsync(tot, c.at<double>(c.L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  if (tot[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite energy");
  *out = tot[SLOT_WS] + tot[SLOT_L1];
  return SHS_OK;
}

// One primal-dual iteration (Chambolle-Pock for the functional of Section 3):
// K ubar (synthesis), the dual step fused into the row pass (y <- clip(y + sigma K ubar),
// then the row FFT of y), K^T y (analysis), the primal step and extrapolation per pixel.
void enqueue_pd_iteration(const Ctx& c, const float* d_s, float tau, float sigma, bool stats, double* hist_row) {
  const shs_plan* p = c.p;
  const Layout& L = c.L;
  const int q = p->q;
  const long long n2 = (long long)p->n * p->n;
  const long long npix_blocks = (n2 + 255) / 256;
  enqueue_synthesis(c, c.at<float>(L.us), q);
  RowParams rp{};
  rp.spec_in = c.at<float2>(L.t1);
  rp.lin = pruned_layout(p);
  rp.spec_out = c.at<float2>(L.t2);
  rp.lout = pruned_layout(p);
  rp.g = c.ws + L.g;
  rp.emit = 1;
  rp.sigma = sigma;
  run_row(c, ROW_PD, p->store, stats, rp, q * p->eta);
  enqueue_analysis(c, q);
  RowParams rz{};
  rz.spec_in = c.at<float2>(L.z);
  rz.lin = dense_layout(p);
  rz.real_out = c.at<float>(L.zs);
  run_row(c, ROW_C2R, ST_F32, false, rz, q);
  PixParams pp{};
  pp.z = c.at<float>(L.zs);
  pp.w = c.at<float>(L.w);
  pp.s = d_s;
  pp.u = c.at<float>(L.us);
  pp.partials = c.at<double>(L.parts) + L.nrow_parts * 4;
  pp.n2 = n2;
  pp.gamma = tau;
  pp.q = q;
  {
    Timed tm(c.s, KC_PIXEL);
    const dim3 g{unsigned(npix_blocks)}, b{256};
    if (stats) hipLaunchKernelGGL((k_pixel_pd<true>), g, b, 0, c.s, pp);
    else hipLaunchKernelGGL((k_pixel_pd<false>), g, b, 0, c.s, pp);
  }
  if (stats) enqueue_reduce(c, L.nrow_parts + npix_blocks, hist_row, 1.0);
}

// KIND 0: dual step, 1: primal step of the NL primal-dual iteration.
template <int ST, int KIND>
void launch_nl(bool stats, long long npix, hipStream_t s, const NlParams& p) {
  const dim3 g{unsigned(npix)}, b{256};
  if constexpr (KIND == 0) {
    if (stats) hipLaunchKernelGGL((k_nl_dual<ST, true>), g, b, 0, s, p);
    else hipLaunchKernelGGL((k_nl_dual<ST, false>), g, b, 0, s, p);
  } else {
    if (stats) hipLaunchKernelGGL((k_nl_primal<ST, true>), g, b, 0, s, p);
    else hipLaunchKernelGGL((k_nl_primal<ST, false>), g, b, 0, s, p);
  }
}

}  // namespace

// A batch of images of different sizes and label counts (one plan per distinct shape).
// A solve of the whole batch is one captured graph, replayed on the caller's stream with a
// single launch.  Images are split into lanes by kernel class (the same kernels and the same
// occupancy); in a lane every step of an iteration is one grouped launch covering all its
// images (grouped.hpp), and the lanes are independent branches of the graph that run side by
// side.
struct shs_batch {
  int count = 0, device = 0;
  std::vector<shs_plan*> plans;
  std::vector<int> plan_of;
  std::vector<size_t> ws_off;
  size_t ws_total = 0;
  std::vector<std::vector<int>> lanes; // images by kernel class (see batch_class)
  hipStream_t main = nullptr;          // capture stream (default priority)
  std::vector<hipStream_t> lane_s;     // one capture branch per lane (default priority)
  std::vector<hipEvent_t> lane_e;
  hipEvent_t fork = nullptr;
  std::vector<double> key;             // pointers and parameters baked into the graph
  hipGraphExec_t graph = nullptr;      // the whole solve
  void* arena = nullptr;               // device task tables of the grouped launches

  void drop_graph() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
    if (arena) (void)hipFree(arena);
    arena = nullptr;
    key.clear();
  }
};

namespace {
// One iteration of a batch as launches: grouped launches (tables at arena offsets) and the
// per-image FP64 reductions, in the order of the iteration's steps.
struct BatchItem {
  bool group = true;
  const void* fn = nullptr;
  int threads = 0;
  size_t lds = 0;
  unsigned blocks = 0;
  size_t tasks_off = 0, bt_off = 0;
  LaunchRec red;       // !group: one image's reduction
};
using BatchIter = std::vector<BatchItem>;

size_t arena_put(std::vector<char>& a, const void* data, size_t bytes) {
  const size_t off = align256(a.size());
  a.resize(off + bytes);
  std::memcpy(a.data() + off, data, bytes);
  return off;
}

template <class P>
void put_group(const std::vector<const LaunchRec*>& recs, P LaunchRec::*field, std::vector<char>& arena,
               BatchItem& it) {
  std::vector<GroupTask<P>> tasks(recs.size());
  std::vector<uint16_t> bt;
  unsigned start = 0;
  for (size_t k = 0; k < recs.size(); ++k) {
    const LaunchRec& r = *recs[k];
    GroupTask<P>& T = tasks[k];
    std::memset(static_cast<void*>(&T), 0, sizeof(T));
    T.p = r.*field;
    T.gp = r.gp;
    T.gx = r.gx;
    T.gy = r.gy;
    T.start = int(start);
    const unsigned nb = unsigned(r.gx) * unsigned(r.gy);
    bt.insert(bt.end(), nb, uint16_t(k));
    start += nb;
    it.lds = std::max(it.lds, r.lds);
  }
  it.blocks = start;
  it.tasks_off = arena_put(arena, tasks.data(), tasks.size() * sizeof(GroupTask<P>));
  it.bt_off = arena_put(arena, bt.data(), bt.size() * sizeof(uint16_t));
}

// Groups one iteration's records of all images (image order) by step, then by kernel.
void build_batch_iter(const std::vector<LaunchRec>& recs, std::vector<char>& arena, BatchIter& out) {
  for (int step = 0; step < BS_COUNT; ++step) {
    std::vector<std::pair<const void*, int>> keys;
    std::vector<std::vector<const LaunchRec*>> groups;
    for (const LaunchRec& r : recs) {
      if (r.step != step) continue;
      if (r.kind == RK_REDUCE) {
        BatchItem it;
        it.group = false;
        it.red = r;
        out.push_back(it);
        continue;
      }
      size_t g = 0;
      while (g < keys.size() && !(keys[g].first == r.fn && keys[g].second == r.threads)) ++g;
      if (g == keys.size()) {
        keys.emplace_back(r.fn, r.threads);
        groups.emplace_back();
      }
      groups[g].push_back(&r);
    }
    for (size_t g = 0; g < groups.size(); ++g) {
      BatchItem it;
      it.fn = keys[g].first;
      it.threads = keys[g].second;
      const int kind = groups[g][0]->kind;
      if (kind == RK_ROW) put_group(groups[g], &LaunchRec::rp, arena, it);
      else if (kind == RK_COL) put_group(groups[g], &LaunchRec::cp, arena, it);
      else put_group(groups[g], &LaunchRec::pp, arena, it);
      out.push_back(it);
    }
  }
}

// Kernel class of an image: the power-of-two side, or for the mixed-radix path the rows per
// wave of its row pass and the blocks per CU its column passes' LDS allows (a grouped launch
// takes its largest image's LDS, so only images of one occupancy share a launch).
int batch_class(const shs_plan* p) {
  if (!p->generic) return p->n;
  const int lds3 = (3 * p->n * kGW + col_tab_len(p->n)) * int(sizeof(float2));
  const int bpc = std::min(4, (160 * 1024) / lds3);
  return 100000 + p->wpb * 100 + p->rw * 10 + bpc;
}

void launch_batch_iter(const BatchIter& iter, char* dbase, hipStream_t s) {
  for (const BatchItem& it : iter) {
    if (it.group) {
      void* tasks = dbase + it.tasks_off;
      void* bt = dbase + it.bt_off;
      void* args[] = {&tasks, &bt};
      (void)hipLaunchKernel(it.fn, dim3(it.blocks), dim3(it.threads), args, it.lds, s);
    } else {
      const LaunchRec& r = it.red;
      const long long per = std::max<long long>((r.nparts + kRed1Blocks - 1) / kRed1Blocks, 1);
      hipLaunchKernelGGL(k_reduce1, dim3(kRed1Blocks), dim3(256), 0, s, r.parts, r.nparts, per, r.red1);
      hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(256), 0, s, r.red1, kRed1Blocks, r.sdev, nullptr, r.gamma,
                         nullptr);
    }
  }
}
}  // namespace

// ---------------------------------------------------------------- schedule tuning
// Mixed-radix plans pick their launch schedule by timing candidates on their own kernels
// at plan creation: rows per wave and waves per block of the row pass, the stage order of
// the row FFT, the stage order of the column FFT, and the filters per synthesis work item.
// The row-pass geometry and the synthesis item size leave the solution bit-identical (the
// residual partial sums are grouped by block, so the histories can differ in the last
// bits); the stage order changes the FFT's rounding (results stay within the parity
// bounds, and are fixed for a given schedule).  The choice is cached per (arch, N, J, q, store) for the process, and in the
// file named by SHEARSEG_TUNE_CACHE when set (one line per key); SHEARSEG_TUNE=0 keeps the
// default schedule.
struct TuneCfg {
  int rw = 1, wpb = 4, fc_syn = 1;
  std::vector<int> prow, pcol;
};
std::mutex g_tune_mu;
std::vector<std::pair<std::string, TuneCfg>> g_tune;   // process cache
bool g_tune_loaded = false;

std::string join_radices(const std::vector<int>& v, char sep) {
  std::string out;
  for (size_t i = 0; i < v.size(); ++i) out += (i ? std::string(1, sep) : std::string()) + std::to_string(v[i]);
  return out;
}
std::vector<int> split_radices(const std::string& t) {
  std::vector<int> v;
  size_t i = 0;
  while (i < t.size()) {
    size_t j = t.find(',', i);
    if (j == std::string::npos) j = t.size();
    v.push_back(std::atoi(t.substr(i, j - i).c_str()));
    i = j + 1;
  }
  return v;
}

void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("SHEARSEG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[128], prow[128], pcol[128];
  int rw, wpb, fc;
  while (std::fscanf(f, "%127s %d %d %d %127s %127s", key, &rw, &wpb, &fc, prow, pcol) == 6) {
    TuneCfg c;
    c.rw = rw;
    c.wpb = wpb;
    c.fc_syn = fc;
    c.prow = split_radices(prow);
    c.pcol = split_radices(pcol);
    g_tune.emplace_back(key, c);
  }
  std::fclose(f);
}
void tune_cache_store(const std::string& key, const TuneCfg& c) {
  g_tune.emplace_back(key, c);
  const char* path = std::getenv("SHEARSEG_TUNE_CACHE");
  if (!path || !*path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%s %d %d %d %s %s\n", key.c_str(), c.rw, c.wpb, c.fc_syn, join_radices(c.prow, ',').c_str(),
                 join_radices(c.pcol, ',').c_str());
    std::fclose(f);
  }
}

// Stage orders worth timing: the default, reversed, radix 16 as 4 x 4, powers of two last.
std::vector<std::vector<int>> order_candidates(const std::vector<int>& d) {
  std::vector<std::vector<int>> out{d};
  auto add = [&](const std::vector<int>& v) {
    if (int(v.size()) <= kMaxStages && std::find(out.begin(), out.end(), v) == out.end()) out.push_back(v);
  };
  add(std::vector<int>(d.rbegin(), d.rend()));
  std::vector<int> split;
  for (int r : d) {
    if (r == 16) { split.push_back(4); split.push_back(4); }
    else split.push_back(r);
  }
  add(split);
  std::vector<int> odd_first;
  for (int r : d) if (r & 1) odd_first.push_back(r);
  for (int r : d) if (!(r & 1)) odd_first.push_back(r);
  add(odd_first);
  return out;
}

// Installs a schedule in the plan: FFT plans and their twiddle tables, rows per wave, and
// the synthesis work items.
shs_status apply_schedule(shs_plan* p, const TuneCfg& c, const StripLists& sl) {
  FftPlan pr, pc;
  if (!fft_plan_from(p->M, c.prow, pr) || !fft_plan_from(p->n, c.pcol, pc)) return fail(SHS_E_DEVICE, "bad schedule");
  const int n = p->n;
  std::vector<float2> tw(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * double(m) / double(n);
    tw[m] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }
  std::vector<float2> tabs(size_t(n) / 2 + n);
  fill_stage_tw_g(pr, tw, n, tabs.data());
  fill_stage_tw_g(pc, tw, n, tabs.data() + n / 2);
  HIPCHK(hipMemcpy(p->tw + n, tabs.data(), tabs.size() * sizeof(float2), hipMemcpyHostToDevice));
  p->prow = pr;
  p->pcol = pc;
  p->rw = c.rw;
  p->wpb = c.wpb;
  p->rpb = c.wpb * c.rw;
  if (c.fc_syn != p->fc_syn) {
    std::vector<int4> isyn;
    build_items(sl.per_strip, sl.strip_off, c.fc_syn, false, isyn, nullptr, nullptr);
    int4* d = nullptr;
    const shs_status st = upload(&d, isyn);
    if (st != SHS_OK) return st;
    (void)hipFree(p->items_syn);
    p->items_syn = d;
    p->n_syn = int(isyn.size());
    p->fc_syn = c.fc_syn;
  }
  return SHS_OK;
}

shs_status tune_schedule(shs_plan* p, const StripLists& sl) {
  hipDeviceProp_t prop{};
  HIPCHK(hipGetDeviceProperties(&prop, p->device));
  const std::string key = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':')) +
                          "/n" + std::to_string(p->n) + "/J" + std::to_string(p->J) + "/q" + std::to_string(p->q) +
                          "/s" + std::to_string(p->store);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_cache_load();
  TuneCfg base;
  base.rw = p->rw;
  base.wpb = p->wpb;
  base.fc_syn = p->fc_syn;
  base.prow = fft_factors(p->M);
  base.pcol = fft_factors(p->n);
  for (auto& e : g_tune)
    if (e.first == key) {
      const shs_status st = apply_schedule(p, e.second, sl);
      if (st == SHS_OK)
        std::snprintf(p->schedule, sizeof(p->schedule), "%s: rows/wave %d, waves/block %d, row radices %s, "
                      "column radices %s, synthesis run %d (cached)", key.c_str(), p->rw, p->wpb,
                      join_radices(e.second.prow, 'x').c_str(),
                      join_radices(e.second.pcol, 'x').c_str(), p->fc_syn);
      return st;
    }
  const char* off = std::getenv("SHEARSEG_TUNE");
  if (off && std::string(off) == "0") {
    std::snprintf(p->schedule, sizeof(p->schedule), "%s: rows/wave %d, waves/block %d, row radices %s, "
                  "column radices %s, synthesis run %d (default)", key.c_str(), p->rw, p->wpb,
                  join_radices(base.prow, 'x').c_str(),
                  join_radices(base.pcol, 'x').c_str(), p->fc_syn);
    return SHS_OK;
  }
  const auto t0 = std::chrono::steady_clock::now();
  // a workspace for one label's channels, sized for the smallest rows per block
  const int rw0 = p->rw, rpb0 = p->rpb;
  p->rw = 1;
  p->rpb = 1;
  const Layout L = make_layout(p);
  p->rw = rw0;
  p->rpb = rpb0;
  void* ws = nullptr;
  if (hipMalloc(&ws, L.total) != hipSuccess) return fail(SHS_E_NOMEM, "tuning workspace");
  struct Free {
    void* w;
    ~Free() { (void)hipFree(w); }
  } fr{ws};
  HIPCHK(hipMemset(ws, 0, L.total));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  struct FreeEv {
    hipEvent_t a, b;
    ~FreeEv() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } fe{e0, e1};
  CaptureScope cs;   // no profiling events while tuning
  auto time_ms = [&](auto&& launch) -> float {
    launch();
    (void)hipEventRecord(e0, 0);
    for (int r = 0; r < 3; ++r) launch();
    (void)hipEventRecord(e1, 0);
    float ms = 1e30f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1e30f;
    return ms;
  };
  TuneCfg best = base;
  int tried = 0;
  // row pass: rows per wave x row stage order (one label's channels, state update on)
  float best_row = 1e30f;
  for (int rw : {1, 2, 4})
   for (int wpb : {4, 2, 1}) {
    // a block's rows divide N and its LDS stays within the limit; one wave per block only
    // where four rows per wave would not otherwise fit
    if (p->n % (rw * wpb) != 0 || row_g_lds_bytes(p->M, rw, wpb, p->n) > kRowGLdsMax) continue;
    if (wpb == 1 && rw < 4) continue;
    for (const auto& ord : order_candidates(base.prow)) {
      TuneCfg c = best;
      c.rw = rw;
      c.wpb = wpb;
      c.prow = ord;
      shs_status st = apply_schedule(p, c, sl);
      if (st != SHS_OK) return st;
      Ctx cx;
      if ((st = make_ctx(p, ws, L.total, nullptr, cx)) != SHS_OK) return st;
      RowParams rp{};
      rp.spec_in = cx.at<float2>(cx.L.t1);
      rp.lin = pruned_layout(p);
      rp.spec_out = cx.at<float2>(cx.L.t2);
      rp.lout = pruned_layout(p);
      rp.g = cx.ws + cx.L.g;
      rp.emit = 1;
      const float ms = time_ms([&] { run_row(cx, ROW_SOLVE, p->store, false, rp, p->eta); });
      ++tried;
      if (ms < best_row) { best_row = ms; best.rw = rw; best.wpb = wpb; best.prow = ord; }
    }
   }
  // column passes: column stage order x synthesis run length (one label)
  float best_col = 1e30f;
  std::vector<int> fcs;
  for (int fc : {1, 2, 4, 8, 16}) if (fc <= kItemMax) fcs.push_back(fc);
  for (const auto& ord : order_candidates(base.pcol)) {
    for (int fc : fcs) {
      TuneCfg c = best;
      c.pcol = ord;
      c.fc_syn = fc;
      shs_status st = apply_schedule(p, c, sl);
      if (st != SHS_OK) return st;
      Ctx cx;
      if ((st = make_ctx(p, ws, L.total, nullptr, cx)) != SHS_OK) return st;
      ColParams cp = col_params(cx, 1);
      const float ms = time_ms([&] {
        ColParams a = cp;
        a.in = cx.at<float2>(cx.L.v);
        a.out = cx.at<float2>(cx.L.t1);
        a.items = p->items_syn;
        run_col(cx, COL_SYN, a, p->n_syn, 1);
        ColParams b = cp;
        b.in = cx.at<float2>(cx.L.t2);
        b.out = cx.at<float2>(cx.L.z);
        b.items = p->items_ana;
        run_col(cx, COL_ANA, b, p->n_ana, 1);
      });
      ++tried;
      if (ms < best_col) { best_col = ms; best.pcol = ord; best.fc_syn = fc; }
    }
  }
  LAUNCHCHK("schedule tuning");
  shs_status st = apply_schedule(p, best, sl);
  if (st != SHS_OK) return st;
  tune_cache_store(key, best);
  const double tms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  std::snprintf(p->schedule, sizeof(p->schedule), "%s: rows/wave %d, waves/block %d, row radices %s, column "
                "radices %s, synthesis run %d (tuned: %d candidates, %.0f ms)", key.c_str(), p->rw, p->wpb,
                join_radices(best.prow, 'x').c_str(),
                join_radices(best.pcol, 'x').c_str(), p->fc_syn, tried, tms);
  return SHS_OK;
}

// ---------------------------------------------------------------- graph replay
constexpr int kGraphIters = 8;   // ADMM iterations per captured graph

namespace {
// Enqueues `reps` x `k` steady-state ADMM iterations (adjoint input present, next adjoint
// input emitted, statistics only when a history is kept) on c.s by replaying a captured
// graph of k iterations.  The graph is captured on first use for this key.
shs_status replay_iterations(const Ctx& c, const float* d_s, float gamma, double* d_hist, int* hctr, int k, int reps) {
  const shs_plan* p = c.p;
  GraphCache& G = *p->graphs;
  std::vector<uint64_t> key;
  key.reserve(8 + 2 * kMaxFilters);
  auto put = [&](const void* ptr) { key.push_back(uint64_t(reinterpret_cast<uintptr_t>(ptr))); };
  put(c.ws); put(d_s); put(d_hist); put(hctr);
  key.push_back(uint64_t(k));
  uint32_t gb;
  std::memcpy(&gb, &gamma, 4);
  key.push_back(gb);
  for (int f = 0; f < p->eta; ++f) {
    uint32_t a, b;
    std::memcpy(&a, &c.fw.thr[f], 4);
    std::memcpy(&b, &c.fw.lam[f], 4);
    key.push_back((uint64_t(a) << 32) | b);
  }
  std::lock_guard<std::mutex> lock(G.mu);
  hipGraphExec_t exec = nullptr;
  for (size_t i = 0; i < G.entries.size(); ++i) {
    if (G.entries[i].key == key) {
      GraphCache::Entry e = G.entries[i];
      G.entries.erase(G.entries.begin() + long(i));
      G.entries.push_back(e);
      exec = e.exec;
      break;
    }
  }
  if (!exec) {
    if (!G.cap) HIPCHK(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
    Ctx cc = c;
    cc.s = G.cap;
    {
      CaptureScope cs;
      HIPCHK(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < k; ++i) enqueue_iteration(cc, d_s, gamma, true, d_hist != nullptr, true, d_hist, hctr);
      const hipError_t el = hipGetLastError();
      hipGraph_t g = nullptr;
      const hipError_t ee = hipStreamEndCapture(G.cap, &g);
      if (el != hipSuccess || ee != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return fail(SHS_E_DEVICE, "capture of the iteration graph failed");
      }
      const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) return fail(SHS_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    if (G.entries.size() >= GraphCache::kMax) {
      (void)hipGraphExecDestroy(G.entries.front().exec);
      G.entries.erase(G.entries.begin());
    }
    G.entries.push_back(GraphCache::Entry{key, exec});
  }
  for (int r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(exec, c.s));
  return SHS_OK;
}
}  // namespace

// ---------------------------------------------------------------- allocation-free solve
// Workspace of shs_solve_noalloc: one file-scope device array per GPU, held until the
// process ends.  Host code never passes `scratch` itself (on the host it is only a stand-in
// for the symbol); it uses the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device on the first call there.
static __device__ __align__(256) unsigned char scratch[SHS_NOALLOC_MAX_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on `device` (which must be current).
shs_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kScratchDevices) return fail(SHS_E_UNSUPPORTED, "device ordinal too large");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SHS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return SHS_OK;
}
}  // namespace

// ===================================================================== C ABI
extern "C" {

const char* shs_status_str(shs_status s) {
  switch (s) {
    case SHS_OK: return "ok";
    case SHS_E_INVALID: return "invalid argument";
    case SHS_E_UNSUPPORTED: return "unsupported";
    case SHS_E_NOMEM: return "out of device memory";
    case SHS_E_DEVICE: return "device error";
    case SHS_E_NUMERIC: return "non-finite value";
    case SHS_E_WORKSPACE: return "workspace too small or missing";
  }
  return "unknown status";
}

const char* shs_last_error(void) { return g_err.c_str(); }

shs_status shs_profile_begin(void) { return shs_profile_begin_classes(nullptr); }

shs_status shs_profile_begin_classes(const char* classes) {
  uint32_t mask = 0;
  if (!classes || !*classes) {
    mask = ~0u;
  } else {
    // comma-separated names, matched in place (no allocation)
    const char* p = classes;
    for (;;) {
      const char* e = p;
      while (*e && *e != ',') ++e;
      const size_t len = size_t(e - p);
      int c = 0;
      while (c < KC_COUNT && !(std::strlen(kKClassName[c]) == len && std::strncmp(kKClassName[c], p, len) == 0)) ++c;
      if (c == KC_COUNT) {
        g_err.assign("unknown kernel class '").append(p, len).append("'");
        return SHS_E_INVALID;
      }
      mask |= 1u << c;
      if (!*e) break;
      p = e + 1;
    }
  }
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.on = true;
  P.mask = mask;
  P.used = 0;
  P.cls.clear();
  return SHS_OK;
}

int32_t shs_profile_end(shs_kernel_time* out, int32_t max_entries) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.on = false;
  double ms[KC_COUNT] = {0};
  int64_t cnt[KC_COUNT] = {0};
  for (size_t i = 0; i < P.cls.size(); ++i) {
    if (hipEventSynchronize(P.pool[2 * i + 1]) != hipSuccess) { g_err = "event synchronize"; return -1; }
    float t = 0.f;
    if (hipEventElapsedTime(&t, P.pool[2 * i], P.pool[2 * i + 1]) != hipSuccess) { g_err = "event elapsed"; return -1; }
    ms[P.cls[i]] += t;
    cnt[P.cls[i]] += 1;
  }
  int32_t k = 0;
  for (int c = 0; c < KC_COUNT && k < max_entries; ++c) {
    if (!cnt[c]) continue;
    if (out) {
      std::memset(out[k].name, 0, sizeof(out[k].name));
      std::strncpy(out[k].name, kKClassName[c], sizeof(out[k].name) - 1);
      out[k].launches = cnt[c];
      out[k].total_ms = ms[c];
    }
    ++k;
  }
  P.used = 0;
  P.cls.clear();
  return k;
}

int32_t shs_num_filters(int32_t J) { return J < 1 || J > 12 ? -1 : 1 + 4 * ((1 << J) - 1); }

shs_status shs_plan_create(const shs_shape* shape, int device, shs_plan** out) {
  if (!shape || !out) return fail(SHS_E_INVALID, "null argument");
  *out = nullptr;
  const int n = shape->n;
  if (n < 2) return fail(SHS_E_INVALID, "n must be >= 2");
  if (shape->q < 1 || shape->q > SHS_MAX_LABELS) return fail(SHS_E_INVALID, "q must be in 1..8");
  if (shape->channels < 1 || shape->channels > SHS_MAX_CHANNELS) return fail(SHS_E_INVALID, "channels must be in 1..4");
  if (shape->J < 1 || shape->J > 6 || (1LL << (2 * shape->J)) > 2LL * n)
    return fail(SHS_E_INVALID, "J must satisfy J >= 1 and 4^J <= 2N");
  if (shape->store < SHS_STORE_F32 || shape->store > SHS_STORE_F16) return fail(SHS_E_INVALID, "bad store type");
  Ops o;
  FftPlan prow{}, pcol{};
  const bool pow2 = get_ops_pow2(n, o);
  if (!pow2) {
    // mixed-radix path: N a multiple of 8 in [64, 1024] whose prime factors are <= 23
    if (n % 8 != 0 || n < 64 || n > kGenericMaxN || !make_fft_plan(n / 2, prow) || !make_fft_plan(n, pcol))
      return fail(SHS_E_UNSUPPORTED,
                  "n must be a power of two in 64..2048 or a multiple of 8 in 64..1024 with prime factors <= 23");
  }
  if (device < 0) return fail(SHS_E_INVALID, "bad device");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return fail(SHS_E_DEVICE, "no such HIP device");
  DeviceGuard dg(device);
  if (!dg.ok) return fail(SHS_E_DEVICE, "hipSetDevice failed");

  shs_plan* p = new (std::nothrow) shs_plan{};
  if (!p) return fail(SHS_E_NOMEM, "host allocation");
  p->graphs = new (std::nothrow) GraphCache();
  if (!p->graphs) { delete p; return fail(SHS_E_NOMEM, "host allocation"); }
  p->n = n; p->C = shape->channels; p->q = shape->q; p->J = shape->J; p->store = shape->store;
  p->eta = shs_num_filters(shape->J);
  p->M = n / 2;
  p->generic = pow2 ? 0 : 1;
  p->prow = prow;
  p->pcol = pcol;
  p->W = pow2 ? by_size<WOf>(n) : kGW;
  // generic rows: several rows per wave keep the lanes busy in stages with few butterflies;
  // the two LDS buffers of a block (4 waves, 64 M rw bytes) stay at or below 48 KB, beside
  // the 8 N bytes of twiddle tables
  p->rw = pow2 ? 1 : (n % 16 == 0 && p->M <= 192) ? 4 : (p->M <= 384 ? 2 : 1);
  p->wpb = 4;
  p->rpb = pow2 ? by_size<RpbOf>(n) : p->wpb * p->rw;
  p->NS = p->M / p->W + 1;
  p->P = p->NS * p->W;  // columns of a dense spectrum plane (strip tiled); columns M+1.. unused
  p->PP = p->M + 16;    // row pitch of the dense filter bank
  p->device = device;
  const size_t psi_bytes = size_t(p->eta) * n * p->PP * 4;
  if (hipMalloc(&p->psi, psi_bytes) != hipSuccess) { free_plan(p); return fail(SHS_E_NOMEM, "filter bank allocation"); }
  std::vector<float2> tw(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * double(m) / double(n);
    tw[m] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }
  // append the row and column stage tables
  if (pow2) {
    fill_stage_tables(n, tw);
  } else {
    tw.resize(size_t(n) + n / 2 + n);
    fill_stage_tw_g(prow, tw, n, tw.data() + n);
    fill_stage_tw_g(pcol, tw, n, tw.data() + n + n / 2);
  }
  if (hipMalloc(&p->tw, tw.size() * 8) != hipSuccess) { free_plan(p); return fail(SHS_E_NOMEM, "twiddle allocation"); }
  std::vector<float> eig(n);
  for (int k = 0; k < n; ++k) {
    const double sn = std::sin(M_PI * double(k) / double(n));
    eig[k] = float(4.0 * sn * sn);
  }
  if (hipMalloc(&p->eig, size_t(n) * 4) != hipSuccess) { free_plan(p); return fail(SHS_E_NOMEM, "eigenvalue table"); }
  if (hipMemcpy(p->eig, eig.data(), size_t(n) * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(p->psi, 0, psi_bytes) != hipSuccess) {
    free_plan(p);
    return fail(SHS_E_DEVICE, "plan initialisation copy");
  }
  const long long total = (long long)p->eta * n * (p->M + 1);
  hipLaunchKernelGGL(k_filter_gen, dim3(unsigned((total + 255) / 256)), dim3(256), 0, 0, p->psi, n, p->J, p->PP,
                     p->eta);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    free_plan(p);
    return fail(SHS_E_DEVICE, "filter generation failed");
  }
  if (p->generic) {
    // generic column passes hold their twiddle table and 3 strips of N x 4 bins in dynamic
    // LDS (up to 104 KB); the cap is set for the largest supported N, so plans of any size
    // can be created in any order
    const int lds3 = (3 * kGenericMaxN * kGW + col_tab_len(kGenericMaxN)) * int(sizeof(float2));
    const int lds2 = (2 * kGenericMaxN * kGW + col_tab_len(kGenericMaxN)) * int(sizeof(float2));
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colg_syn), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds3) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colg_ana), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds3) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colg_fwd), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds2) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colg_final), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds2) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colg_solve), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds2) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&kg_colg_syn), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds3) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&kg_colg_ana), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds3) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&kg_colg_fwd), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds2) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&kg_colg_final), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds2) != hipSuccess) {
      free_plan(p);
      return fail(SHS_E_DEVICE, "cannot reserve LDS for the mixed-radix column passes");
    }
  }
  StripLists sl;
  shs_status st = build_pruned_layout(p, &sl);
  if (st == SHS_OK && p->generic) st = tune_schedule(p, sl);
  if (st != SHS_OK) {
    free_plan(p);
    return st;
  }
  if (!p->generic)
    std::snprintf(p->schedule, sizeof(p->schedule), "n%d: power-of-two path, row FFT %d-point (compile-time "
                  "radices), column strips of %d, synthesis run %d", n, p->M, p->W, p->fc_syn);
  *out = p;
  return SHS_OK;
}

shs_status shs_plan_destroy(shs_plan* p) {
  if (!p) return SHS_OK;
  DeviceGuard dg(p->device);
  free_plan(p);
  return SHS_OK;
}

size_t shs_workspace_bytes(const shs_plan* p) { return p ? make_layout(p).total : 0; }
size_t shs_state_bytes(const shs_plan* p) { return p ? make_layout(p).state_end : 0; }

const char* shs_plan_describe(const shs_plan* p) { return p ? p->schedule : ""; }

shs_status shs_filters(const shs_plan* p, float* d_psi, void* stream) {
  if (!p || !d_psi) return fail(SHS_E_INVALID, "null argument");
  DeviceGuard dg(p->device);
  const size_t w = size_t(p->M + 1) * 4;
  HIPCHK(hipMemcpy2DAsync(d_psi, w, p->psi, size_t(p->PP) * 4, w, size_t(p->eta) * p->n, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(stream)));
  return SHS_OK;
}

shs_status shs_datacost(const shs_plan* p, const float* d_img, const float* h_codebook, float pw, float* d_s,
                        void* stream) {
  if (!p || !d_img || !h_codebook || !d_s) return fail(SHS_E_INVALID, "null argument");
  if (!(pw > 0.f) || !std::isfinite(pw)) return fail(SHS_E_INVALID, "p must be > 0");
  DeviceGuard dg(p->device);
  Codebook cb{};
  for (int k = 0; k < p->q; ++k)
    for (int c = 0; c < p->C; ++c) cb.c[k * 4 + c] = h_codebook[k * p->C + c];
  const long long n2 = (long long)p->n * p->n;
  hipLaunchKernelGGL(k_datacost, dim3(unsigned((n2 + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     d_img, p->C, cb, p->q, pw, d_s, n2);
  LAUNCHCHK("datacost");
  return SHS_OK;
}

shs_status shs_solve_pd(const shs_plan* p, const shs_pd_params* prm, const float* d_s, void* d_ws, size_t ws_bytes,
                        float* d_u, int32_t* d_labels, double* d_hist, shs_stats* h_stats, void* stream) {
  if (!p || !prm || !d_s) return fail(SHS_E_INVALID, "null argument");
  if (!(prm->tau > 0.f) || !(prm->sigma > 0.f) || !std::isfinite(prm->tau) || !std::isfinite(prm->sigma))
    return fail(SHS_E_INVALID, "tau and sigma must be finite and > 0");
  if (double(prm->tau) * double(prm->sigma) > 1.0 + 1e-6)
    return fail(SHS_E_INVALID, "tau * sigma must be <= 1 (||K|| = 1)");
  if (prm->iters < 0) return fail(SHS_E_INVALID, "iters must be >= 0");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  shs_params lp{};
  lp.lambda = prm->lambda;
  lp.lambda_len = prm->lambda_len;
  lp.gamma = 1.f;                        // thresholds = lambda_j (the dual box)
  if ((st = set_lambda(c, &lp)) != SHS_OK) return st;
  const long long n2 = (long long)p->n * p->n;
  // zero start: y (in the g array), u (in w) and ubar
  enqueue_zero_state(c);
  {
    const long long words = (long long)p->q * n2;
    hipLaunchKernelGGL(k_fill_u32, dim3(unsigned((words + 255) / 256)), dim3(256), 0, c.s,
                       reinterpret_cast<uint32_t*>(c.at<float>(c.L.us)), words, 0u);
  }
  LAUNCHCHK("initial state");
  double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool have = false;
  for (int it = 0; it < prm->iters; ++it) {
    const bool last = it == prm->iters - 1;
    const bool stats = d_hist != nullptr || (last && h_stats != nullptr);
    enqueue_pd_iteration(c, d_s, prm->tau, prm->sigma, stats, d_hist ? d_hist + 4LL * it : nullptr);
    LAUNCHCHK("primal-dual iteration");
    if (last && h_stats) {
      HIPCHK(hipMemcpyAsync(tot, c.at<double>(c.L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
      HIPCHK(hipStreamSynchronize(c.s));
      have = true;
      if (tot[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite value in the primal-dual iteration");
    }
  }
  enqueue_epilogue(c, d_u, d_labels);
  LAUNCHCHK("epilogue");
  if (h_stats) {
    shs_stats out{};
    out.iters_done = prm->iters;
    if (have) {
      out.r_primal = std::sqrt(tot[SLOT_DB2]);
      out.r_dual = std::sqrt(tot[SLOT_DY2]);
      out.r_combined = tot[SLOT_DY2] + tot[SLOT_DB2];
      out.energy_surrogate = tot[SLOT_WS] + tot[SLOT_L1];
    }
    double e = 0.0;
    st = energy_of(c, c.at<float>(c.L.w), d_s, &e);
    if (st != SHS_OK) return st;
    out.energy = e;
    *h_stats = out;
  }
  return SHS_OK;
}

shs_status shs_solve_tv(const shs_plan* p, const shs_params* prm, const float* d_s, void* d_ws, size_t ws_bytes,
                        float* d_u, int32_t* d_labels, double* d_hist, shs_stats* h_stats, void* stream) {
  if (!p || !prm || !d_s || !prm->lambda) return fail(SHS_E_INVALID, "null argument");
  shs_status st = check_params(prm);
  if (st != SHS_OK) return st;
  if (prm->lambda_len != 1) return fail(SHS_E_INVALID, "the TV model takes one weight (lambda_len = 1)");
  const float lam = prm->lambda[0];
  if (!(lam >= 0.f) || !std::isfinite(lam)) return fail(SHS_E_INVALID, "lambda must be finite and >= 0");
  if (prm->resume) return fail(SHS_E_INVALID, "the TV solver starts from the zero state only");
  if (p->q > kTvMaxLabels) return fail(SHS_E_UNSUPPORTED, "too many labels for the TV solver");
  DeviceGuard dg(p->device);
  Ctx c;
  st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  const long long n2 = (long long)p->n * p->n;
  enqueue_zero_state(c);
  LAUNCHCHK("initial state");
  const double rnorm = std::sqrt(double(p->q) * double(n2));
  double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool have = false;
  int done = 0;
  for (int it = 0; it < prm->iters; ++it) {
    const bool last = it == prm->iters - 1;
    const bool check = prm->tol > 0.0 && ((it + 1) % prm->check_every == 0 || last);
    const bool stats = d_hist != nullptr || check || (last && h_stats != nullptr);
    enqueue_tv_iteration(c, d_s, lam, prm->gamma, stats, d_hist ? d_hist + 4LL * it : nullptr);
    LAUNCHCHK("TV iteration");
    done = it + 1;
    if (check || (last && h_stats)) {
      HIPCHK(hipMemcpyAsync(tot, c.at<double>(c.L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
      HIPCHK(hipStreamSynchronize(c.s));
      have = true;
      if (tot[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite residual at iteration " + std::to_string(it + 1));
      if (check && std::sqrt(tot[SLOT_DY2] + tot[SLOT_DB2]) <= prm->tol * rnorm) break;
    }
  }
  enqueue_epilogue(c, d_u, d_labels);
  LAUNCHCHK("epilogue");
  if (h_stats) {
    shs_stats out{};
    out.iters_done = done;
    if (have) {
      out.r_primal = std::sqrt(tot[SLOT_DB2]);
      out.r_dual = std::sqrt(tot[SLOT_DY2]) / prm->gamma;
      out.r_combined = tot[SLOT_DY2] + tot[SLOT_DB2];
      out.energy_surrogate = tot[SLOT_WS] + tot[SLOT_L1];
    }
    double e = 0.0;
    if ((st = tv_energy_of(c, d_s, lam, &e)) != SHS_OK) return st;
    out.energy = e;
    *h_stats = out;
  }
  return SHS_OK;
}

shs_status shs_nl_graph(int32_t n, int32_t channels, const float* h_img, const shs_nl_graph_params* prm,
                        int32_t* h_nbr, int32_t* h_rev, int32_t* h_max_degree) {
  if (!h_img || !prm || !h_nbr || !h_rev) return fail(SHS_E_INVALID, "null argument");
  if (channels < 1 || channels > SHS_MAX_CHANNELS) return fail(SHS_E_INVALID, "channels must be 1..4");
  if (prm->patch < 1 || prm->patch % 2 == 0) return fail(SHS_E_INVALID, "patch must be odd and >= 1");
  if (prm->window < 3 || prm->window % 2 == 0) return fail(SHS_E_INVALID, "window must be odd and >= 3");
  if (n < prm->window || n > 4096) return fail(SHS_E_INVALID, "n must be in window..4096");
  if (prm->m < 1 || 2 * prm->m > kNlMaxBlocks) return fail(SHS_E_INVALID, "m must be 1..8");
  if (!(prm->a > 0.f) || !std::isfinite(prm->a)) return fail(SHS_E_INVALID, "a must be finite and > 0");
  NlGraphCfg g{n, channels, prm->patch, prm->window, prm->m, double(prm->a)};
  const int md = nl_build_graph(g, h_img, h_nbr, h_rev);
  if (h_max_degree) *h_max_degree = md;
  return SHS_OK;
}

shs_status shs_solve_nl(const shs_plan* p, const shs_nl_params* prm, const float* d_s, const int32_t* d_nbr,
                        const int32_t* d_rev, void* d_ws, size_t ws_bytes, float* d_u, int32_t* d_labels,
                        double* d_hist, shs_stats* h_stats, void* stream) {
  if (!p || !prm || !d_s || !d_nbr || !d_rev) return fail(SHS_E_INVALID, "null argument");
  if (prm->blocks < 1 || prm->blocks > kNlMaxBlocks) return fail(SHS_E_INVALID, "blocks must be 1..16");
  if (prm->blocks > p->eta) return fail(SHS_E_UNSUPPORTED, "the plan's state holds q * eta images: need eta >= blocks");
  if (prm->max_degree < 0 || prm->max_degree > prm->blocks) return fail(SHS_E_INVALID, "bad max_degree");
  if (!(prm->tau > 0.f) || !(prm->sigma > 0.f) || !std::isfinite(prm->tau) || !std::isfinite(prm->sigma))
    return fail(SHS_E_INVALID, "tau and sigma must be finite and > 0");
  if (double(prm->tau) * double(prm->sigma) * 4.0 * std::max(prm->max_degree, 1) > 1.0 + 1e-6)
    return fail(SHS_E_INVALID, "tau * sigma * 4 * max_degree must be <= 1 (||D||^2 <= 4 max_degree)");
  if (!(prm->lambda >= 0.f) || !std::isfinite(prm->lambda)) return fail(SHS_E_INVALID, "lambda must be >= 0");
  if (prm->iters < 0) return fail(SHS_E_INVALID, "iters must be >= 0");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  const long long n2 = (long long)p->n * p->n;
  const long long npix = (n2 + 255) / 256;
  enqueue_zero_state(c);
  {
    const long long words = (long long)p->q * n2;
    hipLaunchKernelGGL(k_fill_u32, dim3(unsigned((words + 255) / 256)), dim3(256), 0, c.s,
                       reinterpret_cast<uint32_t*>(c.at<float>(c.L.us)), words, 0u);
  }
  LAUNCHCHK("initial state");
  NlParams np{};
  np.y = c.ws + c.L.g;
  np.u = c.at<float>(c.L.w);
  np.ubar = c.at<float>(c.L.us);
  np.s = d_s;
  np.nbr = d_nbr;
  np.rev = d_rev;
  np.n2 = n2;
  np.q = p->q;
  np.M2 = prm->blocks;
  np.lambda = prm->lambda;
  np.tau = prm->tau;
  np.sigma = prm->sigma;
  double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool have = false;
  for (int it = 0; it < prm->iters; ++it) {
    const bool last = it == prm->iters - 1;
    const bool stats = d_hist != nullptr || (last && h_stats != nullptr);
    NlParams pd = np, pp = np;
    pd.partials = c.at<double>(c.L.parts);
    pp.partials = c.at<double>(c.L.parts) + npix * 4;
    {
      Timed tm(c.s, KC_NL_DUAL);
      switch (p->store) {
        case ST_F32: launch_nl<ST_F32, 0>(stats, npix, c.s, pd); break;
        case ST_BF16: launch_nl<ST_BF16, 0>(stats, npix, c.s, pd); break;
        default: launch_nl<ST_F16, 0>(stats, npix, c.s, pd); break;
      }
    }
    {
      Timed tm(c.s, KC_NL_PRIMAL);
      switch (p->store) {
        case ST_F32: launch_nl<ST_F32, 1>(stats, npix, c.s, pp); break;
        case ST_BF16: launch_nl<ST_BF16, 1>(stats, npix, c.s, pp); break;
        default: launch_nl<ST_F16, 1>(stats, npix, c.s, pp); break;
      }
    }
    if (stats) enqueue_reduce(c, 2 * npix, d_hist ? d_hist + 4LL * it : nullptr, 1.0);
    LAUNCHCHK("NL primal-dual iteration");
    if (last && h_stats) {
      HIPCHK(hipMemcpyAsync(tot, c.at<double>(c.L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
      HIPCHK(hipStreamSynchronize(c.s));
      have = true;
      if (tot[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite value in the NL iteration");
    }
  }
  enqueue_epilogue(c, d_u, d_labels);
  LAUNCHCHK("epilogue");
  if (h_stats) {
    shs_stats out{};
    out.iters_done = prm->iters;
    if (have) {
      out.r_primal = std::sqrt(tot[SLOT_DB2]);
      out.r_dual = std::sqrt(tot[SLOT_DY2]);
      out.r_combined = tot[SLOT_DY2] + tot[SLOT_DB2];
      out.energy_surrogate = tot[SLOT_WS] + tot[SLOT_L1];
    }
    NlParams pe = np;
    pe.partials = c.at<double>(c.L.parts);
    {
      Timed tm(c.s, KC_OTHER);
      hipLaunchKernelGGL(k_nl_energy, dim3(unsigned(npix)), dim3(256), 0, c.s, pe);
    }
    enqueue_reduce(c, npix, nullptr, 1.0);
    LAUNCHCHK("NL energy");
    double e[8];
    HIPCHK(hipMemcpyAsync(e, c.at<double>(c.L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
    HIPCHK(hipStreamSynchronize(c.s));
    if (e[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite energy");
    out.energy = e[SLOT_WS] + e[SLOT_L1];
    *h_stats = out;
  }
  return SHS_OK;
}

// The transform entry points take any number of images and run them in groups of at
// most q (the plan's label count sizes the workspace's spectra).
shs_status shs_shearlet_forward(const shs_plan* p, int32_t count, const float* d_f, float* d_c, void* d_ws,
                                size_t ws_bytes, void* stream) {
  if (!p || !d_f || !d_c) return fail(SHS_E_INVALID, "null argument");
  if (count < 1) return fail(SHS_E_INVALID, "count must be >= 1");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  const long long n2 = (long long)p->n * p->n;
  for (int i0 = 0; i0 < count; i0 += p->q) {
    const int k = std::min(p->q, count - i0);
    enqueue_synthesis(c, d_f + i0 * n2, k);
    RowParams rp{};
    rp.spec_in = c.at<float2>(c.L.t1);
    rp.lin = pruned_layout(p);
    rp.real_out = d_c + (long long)i0 * p->eta * n2;
    run_row(c, ROW_C2R, ST_F32, false, rp, k * p->eta);
    LAUNCHCHK("forward");
  }
  return SHS_OK;
}

shs_status shs_shearlet_adjoint(const shs_plan* p, int32_t count, const float* d_c, float* d_f, void* d_ws,
                                size_t ws_bytes, void* stream) {
  if (!p || !d_f || !d_c) return fail(SHS_E_INVALID, "null argument");
  if (count < 1) return fail(SHS_E_INVALID, "count must be >= 1");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  const long long n2 = (long long)p->n * p->n;
  for (int i0 = 0; i0 < count; i0 += p->q) {
    const int k = std::min(p->q, count - i0);
    RowParams rp{};
    rp.real_in = d_c + (long long)i0 * p->eta * n2;
    rp.spec_out = c.at<float2>(c.L.t2);
    rp.lout = pruned_layout(p);
    run_row(c, ROW_R2C, ST_F32, false, rp, k * p->eta);
    enqueue_analysis(c, k);
    RowParams rz{};
    rz.spec_in = c.at<float2>(c.L.z);
    rz.lin = dense_layout(p);
    rz.real_out = d_f + i0 * n2;
    run_row(c, ROW_C2R, ST_F32, false, rz, k);
    LAUNCHCHK("adjoint");
  }
  return SHS_OK;
}

// S^T S_lambda S: forward transform, soft shrinkage of every coefficient and the adjoint,
// with the shrinkage inside the row pass between the two column passes (the coefficient
// images are never stored).
shs_status shs_shearlet_denoise(const shs_plan* p, int32_t count, const float* h_lambda, int32_t lambda_len,
                                const float* d_f, float* d_out, void* d_ws, size_t ws_bytes, void* stream) {
  if (!p || !d_f || !d_out || !h_lambda) return fail(SHS_E_INVALID, "null argument");
  if (count < 1) return fail(SHS_E_INVALID, "count must be >= 1");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  shs_params prm{};
  prm.lambda = h_lambda;
  prm.lambda_len = lambda_len;
  prm.gamma = 1.f;
  if ((st = set_lambda(c, &prm)) != SHS_OK) return st;
  const long long n2 = (long long)p->n * p->n;
  for (int i0 = 0; i0 < count; i0 += p->q) {
    const int k = std::min(p->q, count - i0);
    enqueue_synthesis(c, d_f + i0 * n2, k);
    RowParams rp{};
    rp.spec_in = c.at<float2>(c.L.t1);
    rp.lin = pruned_layout(p);
    rp.spec_out = c.at<float2>(c.L.t2);
    rp.lout = pruned_layout(p);
    run_row(c, ROW_SHRINK, ST_F32, false, rp, k * p->eta);
    enqueue_analysis(c, k);
    RowParams rz{};
    rz.spec_in = c.at<float2>(c.L.z);
    rz.lin = dense_layout(p);
    rz.real_out = d_out + i0 * n2;
    run_row(c, ROW_C2R, ST_F32, false, rz, k);
    LAUNCHCHK("denoise");
  }
  return SHS_OK;
}

shs_status shs_energy(const shs_plan* p, const shs_params* prm, const float* d_s, const float* d_u, void* d_ws,
                      size_t ws_bytes, double* h_energy, void* stream) {
  if (!p || !prm || !d_s || !d_u || !h_energy) return fail(SHS_E_INVALID, "null argument");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  shs_params tmp = *prm;
  if (!(tmp.gamma > 0.f)) tmp.gamma = 1.f;
  st = set_lambda(c, &tmp);
  if (st != SHS_OK) return st;
  return energy_of(c, d_u, d_s, h_energy);
}

}  // extern "C"

namespace {
// shs_solve; allow_graphs = false keeps every launch eager (no graph capture or
// instantiation, which may allocate).
shs_status solve_impl(const shs_plan* p, const shs_params* prm, const float* d_s, void* d_ws, size_t ws_bytes,
                      float* d_u, int32_t* d_labels, double* d_hist, shs_stats* h_stats, void* stream,
                      bool allow_graphs) {
  if (!p || !prm || !d_s) return fail(SHS_E_INVALID, "null argument");
  shs_status st = check_params(prm);
  if (st != SHS_OK) return st;
  DeviceGuard dg(p->device);
  Ctx c;
  st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  st = set_lambda(c, prm);
  if (st != SHS_OK) return st;

  const int q = p->q;
  const long long n2 = (long long)p->n * p->n;
  if (!prm->resume) {
    enqueue_zero_state(c);
  } else {
    RowParams rp{};
    rp.g = c.ws + c.L.g;
    rp.spec_out = c.at<float2>(c.L.t2);
    rp.lout = pruned_layout(p);
    run_row(c, ROW_PRIME, p->store, false, rp, q * p->eta);
  }
  LAUNCHCHK("initial state");

  const double rnorm = std::sqrt(double(q) * double(n2));
  int done = 0;
  bool have_adjoint_input = prm->resume != 0;
  double last_tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool have_last = false;
  // History rows are addressed through a device counter (reset here), so the launches of
  // every steady-state iteration are identical.
  int* hctr = d_hist ? c.at<int>(c.L.hctr) : nullptr;
  if (hctr) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c.s, reinterpret_cast<uint32_t*>(hctr), 1LL, 0u);
  // FP16 state overflows to inf beyond 65504: the last iteration's non-finite flag is
  // always reduced and checked for it (one synchronisation), also without h_stats.
  const bool f16_guard = p->store == SHS_STORE_F16;
  // Steady-state iterations (not the first, not the last; no host check in between) are
  // replayed from captured graphs of kGraphIters iterations unless kernel timing is on.
  const bool graphs = allow_graphs && prm->tol == 0.0 && prm->iters >= 4 && !profiling_on();
  for (int it = 0; it < prm->iters; ++it) {
    const bool last = it == prm->iters - 1;
    if (graphs && it >= 1 && it + kGraphIters < prm->iters) {
      const int reps = (prm->iters - 1 - it) / kGraphIters;
      st = replay_iterations(c, d_s, prm->gamma, d_hist, hctr, kGraphIters, reps);
      if (st != SHS_OK) return st;
      it += reps * kGraphIters - 1;
      have_adjoint_input = true;
      done = it + 1;
      continue;
    }
    const bool check = prm->tol > 0.0 && ((it + 1) % prm->check_every == 0 || last);
    const bool want_last = last && (h_stats != nullptr || f16_guard);
    const bool stats = d_hist != nullptr || check || want_last;
    enqueue_iteration(c, d_s, prm->gamma, have_adjoint_input, stats, !last, d_hist, hctr);
    LAUNCHCHK("iteration");
    have_adjoint_input = true;
    done = it + 1;
    if (check || want_last) {
      HIPCHK(hipMemcpyAsync(last_tot, c.at<double>(c.L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
      HIPCHK(hipStreamSynchronize(c.s));
      have_last = true;
      if (last_tot[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite residual at iteration " + std::to_string(it + 1));
      if (check && std::sqrt(last_tot[SLOT_DY2] + last_tot[SLOT_DB2]) <= prm->tol * rnorm) break;
    }
  }
  enqueue_epilogue(c, d_u, d_labels);
  LAUNCHCHK("epilogue");
  if (h_stats) {
    shs_stats out{};
    out.iters_done = done;
    if (have_last) {
      out.r_primal = std::sqrt(last_tot[SLOT_DB2]);
      out.r_dual = std::sqrt(last_tot[SLOT_DY2]) / prm->gamma;
      out.r_combined = last_tot[SLOT_DY2] + last_tot[SLOT_DB2];
      out.energy_surrogate = last_tot[SLOT_WS] + last_tot[SLOT_L1];
    }
    double e = 0.0;
    st = energy_of(c, c.at<float>(c.L.w), d_s, &e);
    if (st != SHS_OK) return st;
    out.energy = e;
    *h_stats = out;
  }
  return SHS_OK;
}

}  // namespace

extern "C" {

shs_status shs_solve(const shs_plan* p, const shs_params* prm, const float* d_s, void* d_ws, size_t ws_bytes,
                     float* d_u, int32_t* d_labels, double* d_hist, shs_stats* h_stats, void* stream) {
  return solve_impl(p, prm, d_s, d_ws, ws_bytes, d_u, d_labels, d_hist, h_stats, stream, true);
}

shs_status shs_solve_noalloc(const shs_plan* p, const shs_params* prm, const float* d_s, float* d_u,
                             int32_t* d_labels, double* d_hist, shs_stats* h_stats, void* stream) {
  if (!p || !prm || !d_s) return fail(SHS_E_INVALID, "null argument");
  const size_t need = shs_workspace_bytes(p);
  if (need > SHS_NOALLOC_MAX_BYTES)
    return fail(SHS_E_WORKSPACE, "this plan needs " + std::to_string(need) + " bytes of workspace; the "
                "allocation-free solve holds at most " + std::to_string((unsigned long long)SHS_NOALLOC_MAX_BYTES));
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(SHS_E_DEVICE, "hipSetDevice failed");
  void* ws = nullptr;
  const shs_status st = scratch_address(p->device, &ws);
  if (st != SHS_OK) return st;
  return solve_impl(p, prm, d_s, ws, need, d_u, d_labels, d_hist, h_stats, stream, false);
}

shs_status shs_batch_create(int32_t count, const shs_shape* shapes, int device, shs_batch** out) {
  if (!out || !shapes || count < 1) return fail(SHS_E_INVALID, "null argument or count < 1");
  if (count > 65535) return fail(SHS_E_UNSUPPORTED, "at most 65535 images per batch");
  *out = nullptr;
  shs_batch* b = new (std::nothrow) shs_batch{};
  if (!b) return fail(SHS_E_NOMEM, "host allocation");
  b->count = count;
  b->device = device;
  for (int i = 0; i < count; ++i) {
    const shs_shape& s = shapes[i];
    int found = -1;
    for (size_t k = 0; k < b->plans.size(); ++k) {
      const shs_plan* p = b->plans[k];
      if (p->n == s.n && p->C == s.channels && p->q == s.q && p->J == s.J && p->store == s.store) found = int(k);
    }
    if (found < 0) {
      shs_plan* p = nullptr;
      const shs_status st = shs_plan_create(&s, device, &p);
      if (st != SHS_OK) {
        const std::string msg = g_err;
        shs_batch_destroy(b);
        return fail(st, "image " + std::to_string(i) + ": " + msg);
      }
      b->plans.push_back(p);
      found = int(b->plans.size()) - 1;
    }
    b->plan_of.push_back(found);
    b->ws_off.push_back(b->ws_total);
    b->ws_total += align256(shs_workspace_bytes(b->plans[found]));
  }
  {
    std::vector<int> keys;
    for (int i = 0; i < count; ++i) {
      const int k = batch_class(b->plans[b->plan_of[i]]);
      size_t l = 0;
      while (l < keys.size() && keys[l] != k) ++l;
      if (l == keys.size()) {
        keys.push_back(k);
        b->lanes.emplace_back();
      }
      b->lanes[l].push_back(i);
    }
  }
  DeviceGuard dg(device);
  bool ok = hipStreamCreateWithFlags(&b->main, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (size_t l = 0; ok && l < b->lanes.size(); ++l) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    if (st) b->lane_s.push_back(st);
    if (ev) b->lane_e.push_back(ev);
  }
  if (!ok) {
    shs_batch_destroy(b);
    return fail(SHS_E_DEVICE, "batch stream creation");
  }
  *out = b;
  return SHS_OK;
}

shs_status shs_batch_destroy(shs_batch* b) {
  if (!b) return SHS_OK;
  DeviceGuard dg(b->device);
  b->drop_graph();
  if (b->main) (void)hipStreamDestroy(b->main);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipStream_t st : b->lane_s) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->lane_e) (void)hipEventDestroy(ev);
  for (shs_plan* p : b->plans) shs_plan_destroy(p);
  delete b;
  return SHS_OK;
}

size_t shs_batch_workspace_bytes(const shs_batch* b) { return b ? b->ws_total : 0; }

shs_status shs_solve_batch(shs_batch* b, const shs_params* params, const float* const* d_s, void* d_ws,
                           size_t ws_bytes, float* const* d_u, int32_t* const* d_labels, double* d_stats,
                           void* stream) {
  if (!b || !params || !d_s) return fail(SHS_E_INVALID, "null argument");
  if (!d_ws || ws_bytes < b->ws_total) return fail(SHS_E_WORKSPACE, "batch workspace too small");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return fail(SHS_E_WORKSPACE, "workspace must be 256-byte aligned");
  const int iters = params[0].iters;
  for (int i = 0; i < b->count; ++i) {
    const shs_status st = check_params(&params[i]);
    if (st != SHS_OK) return fail(st, "image " + std::to_string(i) + ": " + g_err);
    if (!d_s[i]) return fail(SHS_E_INVALID, "null data term of image " + std::to_string(i));
    if (params[i].iters != iters) return fail(SHS_E_UNSUPPORTED, "all images of a batch run the same iteration count");
    if (params[i].tol != 0.0 || params[i].resume) return fail(SHS_E_UNSUPPORTED, "batch solves take no tol / resume");
  }
  DeviceGuard dg(b->device);
  // per-image contexts, all on the capture stream
  std::vector<Ctx> ctx(b->count);
  for (int i = 0; i < b->count; ++i) {
    const shs_plan* p = b->plans[b->plan_of[i]];
    shs_status st = make_ctx(p, static_cast<char*>(d_ws) + b->ws_off[i], shs_workspace_bytes(p), nullptr, ctx[i]);
    if (st == SHS_OK) st = set_lambda(ctx[i], &params[i]);
    if (st != SHS_OK) return fail(st, "image " + std::to_string(i) + ": " + g_err);
    ctx[i].s = b->main;
  }
  // graph cache key: every pointer and parameter baked into the graph
  std::vector<double> key;
  key.push_back(double(reinterpret_cast<uintptr_t>(d_ws)));
  key.push_back(double(reinterpret_cast<uintptr_t>(d_stats)));
  key.push_back(iters);
  for (int i = 0; i < b->count; ++i) {
    key.push_back(double(reinterpret_cast<uintptr_t>(d_s[i])));
    key.push_back(double(reinterpret_cast<uintptr_t>(d_u ? d_u[i] : nullptr)));
    key.push_back(double(reinterpret_cast<uintptr_t>(d_labels ? d_labels[i] : nullptr)));
    key.push_back(params[i].gamma);
    for (int f = 0; f < ctx[i].p->eta; ++f) key.push_back(ctx[i].fw.lam[f]);
  }
  if (key != b->key || !b->graph) {
    b->drop_graph();
    // the iteration variants, recorded for all images and grouped
    struct Variant {
      bool adj, stats, emit;
    };
    std::vector<Variant> vars;
    if (iters == 1) vars = {{false, true, false}};
    else if (iters == 2) vars = {{false, false, true}, {true, true, false}};
    else if (iters >= 3) vars = {{false, false, true}, {true, false, true}, {true, true, false}};
    std::vector<char> arena;
    const size_t nl = b->lanes.size();
    std::vector<std::vector<BatchIter>> its(nl, std::vector<BatchIter>(vars.size()));
    for (size_t l = 0; l < nl; ++l) {
      for (size_t v = 0; v < vars.size(); ++v) {
        Recorder rec;
        CaptureScope cs;        // no timing events while recording
        g_rec = &rec;
        for (int i : b->lanes[l])
          enqueue_iteration(ctx[i], d_s[i], params[i].gamma, vars[v].adj, vars[v].stats, vars[v].emit, nullptr);
        g_rec = nullptr;
        build_batch_iter(rec.recs, arena, its[l][v]);
      }
    }
    if (!arena.empty()) {
      if (hipMalloc(&b->arena, arena.size()) != hipSuccess) return fail(SHS_E_NOMEM, "batch task tables");
      HIPCHK(hipMemcpy(b->arena, arena.data(), arena.size(), hipMemcpyHostToDevice));
    }
    char* dbase = static_cast<char*>(b->arena);
    auto tail = [&](int i) {   // epilogue + statistics of image i (zeros when no iteration ran)
      const Ctx& c = ctx[i];
      enqueue_epilogue(c, d_u ? d_u[i] : nullptr, d_labels ? d_labels[i] : nullptr);
      if (d_stats && iters > 0)
        hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(64), 0, c.s, c.at<double>(c.L.sdev), 5, d_stats + 5LL * i);
      else if (d_stats)
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c.s, reinterpret_cast<uint32_t*>(d_stats + 5LL * i),
                           10LL, 0u);
    };
    {
      CaptureScope cs;
      HIPCHK(hipStreamBeginCapture(b->main, hipStreamCaptureModeThreadLocal));
      bool ok = hipEventRecord(b->fork, b->main) == hipSuccess;
      for (size_t l = 0; ok && l < nl; ++l) {
        hipStream_t ls = b->lane_s[l];
        ok = hipStreamWaitEvent(ls, b->fork, 0) == hipSuccess;
        for (int i : b->lanes[l]) {
          ctx[i].s = ls;
          enqueue_zero_state(ctx[i]);
        }
        if (iters >= 1) launch_batch_iter(its[l][0], dbase, ls);
        for (int it = 1; it + 1 < iters; ++it) launch_batch_iter(its[l][1], dbase, ls);
        if (iters >= 2) launch_batch_iter(its[l].back(), dbase, ls);
        for (int i : b->lanes[l]) tail(i);
        ok = ok && hipEventRecord(b->lane_e[l], ls) == hipSuccess &&
             hipStreamWaitEvent(b->main, b->lane_e[l], 0) == hipSuccess;
      }
      const hipError_t el = ok ? hipGetLastError() : hipErrorUnknown;
      hipGraph_t g = nullptr;
      const hipError_t ee = hipStreamEndCapture(b->main, &g);
      if (el != hipSuccess || ee != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        b->drop_graph();
        return fail(SHS_E_DEVICE, "capture of the batch graph failed");
      }
      const hipError_t ei = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        b->graph = nullptr;
        b->drop_graph();
        return fail(SHS_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
      }
    }
    b->key = key;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Timed tm(s, KC_BATCH);
  HIPCHK(hipGraphLaunch(b->graph, s));
  return SHS_OK;
}

}  // extern "C"
