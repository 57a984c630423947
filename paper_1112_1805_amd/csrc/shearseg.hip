// Host side of the shearlet-segmentation library: plan (filter bank + twiddles on the
// device), workspace layout, launch orchestration of the ADMM of Section 3, and the C ABI
// declared in include/shearseg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "shearseg.h"
#include "kernels.hpp"

using namespace shs;

struct shs_plan {
  int n, C, q, J, store, eta, M, P, device;
  float* psi;      // [eta][N][P] filter bank (half spectrum)
  float2* tw;      // [N] exp(-2 pi i m / N)
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

size_t store_bytes(int store) { return store == SHS_STORE_F32 ? 4 : 2; }

int row_rpb(int n) {
  switch (n) {
    case 64: return RowGeom<64>::RPB;
    case 128: return RowGeom<128>::RPB;
    case 256: return RowGeom<256>::RPB;
    case 512: return RowGeom<512>::RPB;
    case 1024: return RowGeom<1024>::RPB;
    case 2048: return RowGeom<2048>::RPB;
  }
  return 1;
}
int col_w(int n) {
  switch (n) {
    case 64: return ColGeom<64>::W;
    case 128: return ColGeom<128>::W;
    case 256: return ColGeom<256>::W;
    case 512: return ColGeom<512>::W;
    case 1024: return ColGeom<1024>::W;
    case 2048: return ColGeom<2048>::W;
  }
  return 1;
}

constexpr int kRed1Blocks = 256;
constexpr int kDotBlocks = 1024;
constexpr int kTargetBlocks = 2048;   // aim for >> 256 CUs worth of column blocks

struct Layout {
  size_t g, w, bw, state_end;
  size_t t1, t2, v, z, zs, us, accp, parts, red1, sdev, total;
  long long nrow_parts, nparts;
  int nstrips, fc_syn, nch_syn, fc_ana, nch_ana;
};

void chunking(int eta, int blocks_per_filterless, int cap, int& fc, int& nch) {
  int want = (kTargetBlocks + blocks_per_filterless - 1) / blocks_per_filterless;
  want = std::max(1, std::min(want, std::min(cap, eta)));
  fc = (eta + want - 1) / want;
  nch = (eta + fc - 1) / fc;
}

Layout make_layout(const shs_plan* p) {
  Layout L{};
  const size_t n = p->n, nn = n * n, q = p->q, eta = p->eta, P = p->P;
  const size_t plane = n * P;  // float2 per spectrum
  L.nstrips = int(p->M / col_w(p->n) + 1);
  chunking(p->eta, L.nstrips * p->q, p->eta, L.fc_syn, L.nch_syn);
  chunking(p->eta, L.nstrips * p->q, 16, L.fc_ana, L.nch_ana);
  size_t off = 0;
  L.g = off;   off = align256(off + q * eta * nn * store_bytes(p->store));
  L.w = off;   off = align256(off + q * nn * 4);
  L.bw = off;  off = align256(off + q * nn * 4);
  L.state_end = off;
  L.t1 = off;  off = align256(off + q * eta * plane * 8);
  L.t2 = off;  off = align256(off + q * eta * plane * 8);
  L.v = off;   off = align256(off + q * plane * 8);
  L.z = off;   off = align256(off + q * plane * 8);
  L.zs = off;  off = align256(off + q * nn * 4);
  L.us = off;  off = align256(off + q * nn * 4);
  L.accp = off;
  if (L.nch_ana > 1) off = align256(off + size_t(L.nch_ana) * q * plane * 8);
  L.nrow_parts = (long long)(q * eta) * (n / row_rpb(p->n));
  const long long npix = (long long)((nn + 255) / 256);
  L.nparts = L.nrow_parts + std::max<long long>(npix, kDotBlocks);
  L.parts = off; off = align256(off + size_t(L.nparts) * 4 * 8);
  L.red1 = off;  off = align256(off + kRed1Blocks * 4 * 8);
  L.sdev = off;  off = align256(off + 8 * 8);
  L.total = off;
  return L;
}

// ---------------------------------------------------------------- per-size launchers
template <int N>
struct Pipe {
  using RG = RowGeom<N>;
  using CG = ColCfg<N>;

  template <int MODE, int ST, bool STATS>
  static void row_t(const RowParams& rp, int channels, hipStream_t s) {
    dim3 grid(N / RG::RPB, channels);
    hipLaunchKernelGGL((k_row<N, MODE, ST, STATS>), grid, dim3(256), 0, s, rp);
  }
  static void row(int mode, int store, bool stats, const RowParams& rp, int channels, hipStream_t s) {
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
    }
  }
  static void col_syn(const ColParams& cp, int labels, int nstrips, int nch, hipStream_t s) {
    hipLaunchKernelGGL((k_col_syn<N>), dim3(nstrips, labels, nch), dim3(CG::THREADS), 0, s, cp);
  }
  static void col_ana(const ColParams& cp, int labels, int nstrips, int nch, hipStream_t s) {
    hipLaunchKernelGGL((k_col_ana<N>), dim3(nstrips, labels, nch), dim3(CG::THREADS), 0, s, cp);
    if (nch > 1) hipLaunchKernelGGL((k_col_final<N>), dim3(nstrips, labels), dim3(CG::THREADS), 0, s, cp);
  }
};

struct Ops {
  void (*row)(int, int, bool, const RowParams&, int, hipStream_t);
  void (*col_syn)(const ColParams&, int, int, int, hipStream_t);
  void (*col_ana)(const ColParams&, int, int, int, hipStream_t);
};

template <int N>
Ops ops_for() {
  return Ops{&Pipe<N>::row, &Pipe<N>::col_syn, &Pipe<N>::col_ana};
}

bool get_ops(int n, Ops& o) {
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
  if (!get_ops(p->n, c.ops)) return fail(SHS_E_UNSUPPORTED, "unsupported size");
  if (!ws) return fail(SHS_E_WORKSPACE, "null workspace");
  if (ws_bytes < c.L.total)
    return fail(SHS_E_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                                     std::to_string(c.L.total));
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(SHS_E_WORKSPACE, "workspace must be 256-byte aligned");
  c.ws = static_cast<char*>(ws);
  c.s = static_cast<hipStream_t>(stream);
  return SHS_OK;
}

RowParams row_params(const Ctx& c) {
  RowParams rp{};
  rp.tw = c.p->tw;
  rp.P = c.p->P;
  rp.eta = c.p->eta;
  rp.spec_cs = (long long)c.p->n * c.p->P;
  rp.real_cs = (long long)c.p->n * c.p->n;
  rp.fw = c.fw;
  rp.partials = c.at<double>(c.L.parts);
  rp.emit = 1;
  return rp;
}

ColParams col_params(const Ctx& c, int labels) {
  ColParams cp{};
  cp.psi = c.p->psi;
  cp.tw = c.p->tw;
  cp.accp = c.at<float2>(c.L.accp);
  cp.P = c.p->P;
  cp.eta = c.p->eta;
  cp.labels = labels;
  cp.inv_n2 = 1.0f / (float(c.p->n) * float(c.p->n));
  return cp;
}

// S: real images [count][N][N] -> coefficient spectra T1 (and optionally real coefficients).
void enqueue_synthesis(const Ctx& c, const float* real_in, int count) {
  RowParams rp = row_params(c);
  rp.real_in = real_in;
  rp.spec_out = c.at<float2>(c.L.v);
  c.ops.row(ROW_R2C, ST_F32, false, rp, count, c.s);
  ColParams cp = col_params(c, count);
  cp.in = c.at<float2>(c.L.v);
  cp.out = c.at<float2>(c.L.t1);
  cp.fc = c.L.fc_syn;
  cp.nchunks = c.L.nch_syn;
  c.ops.col_syn(cp, count, c.L.nstrips, c.L.nch_syn, c.s);
}

// Adjoint column side: spectra T2 (count*eta channels) -> Z (count labels).
void enqueue_analysis(const Ctx& c, int count) {
  ColParams cp = col_params(c, count);
  cp.in = c.at<float2>(c.L.t2);
  cp.out = c.at<float2>(c.L.z);
  cp.fc = c.L.fc_ana;
  cp.nchunks = c.L.nch_ana;
  c.ops.col_ana(cp, count, c.L.nstrips, c.L.nch_ana, c.s);
}

void enqueue_reduce(const Ctx& c, long long nparts, double* hist_row, double gamma) {
  const long long per = (nparts + kRed1Blocks - 1) / kRed1Blocks;
  hipLaunchKernelGGL(k_reduce1, dim3(kRed1Blocks), dim3(256), 0, c.s, c.at<double>(c.L.parts), nparts,
                     std::max<long long>(per, 1), c.at<double>(c.L.red1));
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(256), 0, c.s, c.at<double>(c.L.red1), kRed1Blocks,
                     c.at<double>(c.L.sdev), hist_row, gamma);
}

// Per-filter weights and thresholds from a host Lambda (J+1 per-scale or eta per-filter).
shs_status set_lambda(Ctx& c, const shs_params* prm) {
  const int eta = c.p->eta, J = c.p->J;
  if (!prm->lambda) return fail(SHS_E_INVALID, "null lambda");
  std::vector<float> lam_f(eta, 0.f);
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
  for (float v : lam_f)
    if (!(v >= 0.f) || !std::isfinite(v)) return fail(SHS_E_INVALID, "lambda entries must be finite and >= 0");
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
  RowParams rp = row_params(c);
  rp.spec_in = c.at<float2>(c.L.t1);
  c.ops.row(ROW_ENERGY, ST_F32, true, rp, p->q * p->eta, c.s);
  LAUNCHCHK("energy rows");
  const long long nn = (long long)p->n * p->n * p->q;
  hipLaunchKernelGGL(k_dot, dim3(kDotBlocks), dim3(256), 0, c.s, d_u, d_s, nn,
                     c.at<double>(c.L.parts) + c.L.nrow_parts * 4);
  enqueue_reduce(c, c.L.nrow_parts + kDotBlocks, nullptr, 1.0);
  LAUNCHCHK("energy reduce");
  double tot[8];
  HIPCHK(hipMemcpyAsync(tot, c.at<double>(c.L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  if (tot[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite energy");
  *out = tot[SLOT_WS] + tot[SLOT_L1];
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
  if (!get_ops(n, o)) return fail(SHS_E_UNSUPPORTED, "n must be one of 64, 128, 256, 512, 1024, 2048");
  if (device < 0) return fail(SHS_E_INVALID, "bad device");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return fail(SHS_E_DEVICE, "no such HIP device");
  DeviceGuard dg(device);
  if (!dg.ok) return fail(SHS_E_DEVICE, "hipSetDevice failed");

  shs_plan* p = new (std::nothrow) shs_plan{};
  if (!p) return fail(SHS_E_NOMEM, "host allocation");
  p->n = n; p->C = shape->channels; p->q = shape->q; p->J = shape->J; p->store = shape->store;
  p->eta = shs_num_filters(shape->J);
  p->M = n / 2;
  p->P = p->M + 16;  // 128-byte aligned rows; columns M+1.. are padding
  p->device = device;
  const size_t psi_bytes = size_t(p->eta) * n * p->P * 4;
  if (hipMalloc(&p->psi, psi_bytes) != hipSuccess) { delete p; return fail(SHS_E_NOMEM, "filter bank allocation"); }
  if (hipMalloc(&p->tw, size_t(n) * 8) != hipSuccess) {
    (void)hipFree(p->psi); delete p; return fail(SHS_E_NOMEM, "twiddle allocation");
  }
  std::vector<float2> tw(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * double(m) / double(n);
    tw[m] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }
  shs_status st = SHS_OK;
  if (hipMemcpy(p->tw, tw.data(), size_t(n) * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(p->psi, 0, psi_bytes) != hipSuccess) {
    st = fail(SHS_E_DEVICE, "plan initialisation copy");
  } else {
    const long long total = (long long)p->eta * n * (p->M + 1);
    hipLaunchKernelGGL(k_filter_gen, dim3(unsigned((total + 255) / 256)), dim3(256), 0, 0, p->psi, n, p->J, p->P,
                       p->eta);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
      st = fail(SHS_E_DEVICE, "filter generation failed");
  }
  if (st != SHS_OK) {
    (void)hipFree(p->psi); (void)hipFree(p->tw); delete p;
    return st;
  }
  *out = p;
  return SHS_OK;
}

shs_status shs_plan_destroy(shs_plan* p) {
  if (!p) return SHS_OK;
  DeviceGuard dg(p->device);
  (void)hipFree(p->psi);
  (void)hipFree(p->tw);
  delete p;
  return SHS_OK;
}

size_t shs_workspace_bytes(const shs_plan* p) { return p ? make_layout(p).total : 0; }
size_t shs_state_bytes(const shs_plan* p) { return p ? make_layout(p).state_end : 0; }

shs_status shs_filters(const shs_plan* p, float* d_psi, void* stream) {
  if (!p || !d_psi) return fail(SHS_E_INVALID, "null argument");
  DeviceGuard dg(p->device);
  const size_t w = size_t(p->M + 1) * 4;
  HIPCHK(hipMemcpy2DAsync(d_psi, w, p->psi, size_t(p->P) * 4, w, size_t(p->eta) * p->n, hipMemcpyDeviceToDevice,
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

shs_status shs_shearlet_forward(const shs_plan* p, int32_t count, const float* d_f, float* d_c, void* d_ws,
                                size_t ws_bytes, void* stream) {
  if (!p || !d_f || !d_c) return fail(SHS_E_INVALID, "null argument");
  if (count < 1 || count > p->q) return fail(SHS_E_INVALID, "count must be in 1..q");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  enqueue_synthesis(c, d_f, count);
  RowParams rp = row_params(c);
  rp.spec_in = c.at<float2>(c.L.t1);
  rp.real_out = d_c;
  c.ops.row(ROW_C2R, ST_F32, false, rp, count * p->eta, c.s);
  LAUNCHCHK("forward");
  return SHS_OK;
}

shs_status shs_shearlet_adjoint(const shs_plan* p, int32_t count, const float* d_c, float* d_f, void* d_ws,
                                size_t ws_bytes, void* stream) {
  if (!p || !d_f || !d_c) return fail(SHS_E_INVALID, "null argument");
  if (count < 1 || count > p->q) return fail(SHS_E_INVALID, "count must be in 1..q");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  RowParams rp = row_params(c);
  rp.real_in = d_c;
  rp.spec_out = c.at<float2>(c.L.t2);
  c.ops.row(ROW_R2C, ST_F32, false, rp, count * p->eta, c.s);
  enqueue_analysis(c, count);
  RowParams rz = row_params(c);
  rz.spec_in = c.at<float2>(c.L.z);
  rz.real_out = d_f;
  c.ops.row(ROW_C2R, ST_F32, false, rz, count, c.s);
  LAUNCHCHK("adjoint");
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

shs_status shs_solve(const shs_plan* p, const shs_params* prm, const float* d_s, void* d_ws, size_t ws_bytes,
                     float* d_u, int32_t* d_labels, double* d_hist, shs_stats* h_stats, void* stream) {
  if (!p || !prm || !d_s) return fail(SHS_E_INVALID, "null argument");
  if (!(prm->gamma > 0.f) || !std::isfinite(prm->gamma)) return fail(SHS_E_INVALID, "gamma must be > 0");
  if (prm->iters < 0) return fail(SHS_E_INVALID, "iters must be >= 0");
  if (prm->tol < 0.0 || (prm->tol > 0.0 && prm->check_every < 1)) return fail(SHS_E_INVALID, "bad tol/check_every");
  DeviceGuard dg(p->device);
  Ctx c;
  shs_status st = make_ctx(p, d_ws, ws_bytes, stream, c);
  if (st != SHS_OK) return st;
  st = set_lambda(c, prm);
  if (st != SHS_OK) return st;

  const int q = p->q, eta = p->eta;
  const long long n2 = (long long)p->n * p->n;
  const long long npix_blocks = (n2 + 255) / 256;
  const Layout& L = c.L;
  float* W = c.at<float>(L.w);
  float* BW = c.at<float>(L.bw);

  if (!prm->resume) {
    HIPCHK(hipMemsetAsync(c.ws + L.g, 0, L.w - L.g, c.s));
    HIPCHK(hipMemsetAsync(W, 0, size_t(q) * n2 * 4, c.s));
    HIPCHK(hipMemsetAsync(BW, 0, size_t(q) * n2 * 4, c.s));
  } else {
    RowParams rp = row_params(c);
    rp.g = c.ws + L.g;
    rp.spec_out = c.at<float2>(L.t2);
    c.ops.row(ROW_PRIME, p->store, false, rp, q * eta, c.s);
    LAUNCHCHK("prime");
  }

  const double rnorm = std::sqrt(double(q) * double(n2));
  int done = 0;
  bool have_adjoint_input = prm->resume != 0;
  double last_tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool have_last = false;
  for (int it = 0; it < prm->iters; ++it) {
    const bool last = it == prm->iters - 1;
    const bool check = prm->tol > 0.0 && ((it + 1) % prm->check_every == 0 || last);
    const bool stats = d_hist != nullptr || check || (last && h_stats != nullptr);
    // ---- u-update: z = S^T (v - b_v) per label
    if (have_adjoint_input) {
      enqueue_analysis(c, q);
      RowParams rz = row_params(c);
      rz.spec_in = c.at<float2>(L.z);
      rz.real_out = c.at<float>(L.zs);
      c.ops.row(ROW_C2R, ST_F32, false, rz, q, c.s);
    }
    PixParams pp{};
    pp.z = c.at<float>(L.zs);
    pp.w = W;
    pp.bw = BW;
    pp.s = d_s;
    pp.u = c.at<float>(L.us);
    pp.partials = c.at<double>(L.parts) + L.nrow_parts * 4;
    pp.n2 = n2;
    pp.gamma = prm->gamma;
    pp.q = q;
    if (have_adjoint_input) {
      if (stats) hipLaunchKernelGGL((k_pixel<true, true>), dim3(unsigned(npix_blocks)), dim3(256), 0, c.s, pp);
      else hipLaunchKernelGGL((k_pixel<false, true>), dim3(unsigned(npix_blocks)), dim3(256), 0, c.s, pp);
    } else {
      if (stats) hipLaunchKernelGGL((k_pixel<true, false>), dim3(unsigned(npix_blocks)), dim3(256), 0, c.s, pp);
      else hipLaunchKernelGGL((k_pixel<false, false>), dim3(unsigned(npix_blocks)), dim3(256), 0, c.s, pp);
    }
    // ---- v-update and b_v-update with S u, fused with the next adjoint's row FFT
    enqueue_synthesis(c, c.at<float>(L.us), q);
    RowParams rp = row_params(c);
    rp.spec_in = c.at<float2>(L.t1);
    rp.spec_out = c.at<float2>(L.t2);
    rp.g = c.ws + L.g;
    rp.emit = last ? 0 : 1;
    c.ops.row(ROW_SOLVE, p->store, stats, rp, q * eta, c.s);
    LAUNCHCHK("iteration");
    have_adjoint_input = true;
    if (stats) {
      enqueue_reduce(c, L.nrow_parts + npix_blocks, d_hist ? d_hist + 4LL * it : nullptr, prm->gamma);
      LAUNCHCHK("reduce");
    }
    done = it + 1;
    if (check || (last && h_stats)) {
      HIPCHK(hipMemcpyAsync(last_tot, c.at<double>(L.sdev), 5 * 8, hipMemcpyDeviceToHost, c.s));
      HIPCHK(hipStreamSynchronize(c.s));
      have_last = true;
      if (last_tot[4] != 0.0) return fail(SHS_E_NUMERIC, "non-finite residual at iteration " + std::to_string(it + 1));
      if (check && std::sqrt(last_tot[SLOT_DY2] + last_tot[SLOT_DB2]) <= prm->tol * rnorm) break;
    }
  }
  if (d_u || d_labels) {
    hipLaunchKernelGGL(k_epilogue, dim3(unsigned(npix_blocks)), dim3(256), 0, c.s, W, q, n2, d_u, d_labels);
    LAUNCHCHK("epilogue");
  }
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
    st = energy_of(c, W, d_s, &e);
    if (st != SHS_OK) return st;
    out.energy = e;
    *h_stats = out;
  }
  return SHS_OK;
}

}  // extern "C"
