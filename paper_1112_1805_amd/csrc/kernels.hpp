// HIP kernels for gfx950 implementing the ADMM hot path of the shearlet-regularised
// multi-label segmentation (Haeuser & Steidl, arXiv 1112.1805, Sections 2-3).
//
// Data layout (all row-major):
//   real images          [channel][N][N]          float (state: float / bf16 / f16)
//   half spectra         [channel][N][P] float2   bins (k0, k1), k1 = 0..N/2, P >= N/2+1
//   filter bank          [eta][N][P]     float    real spectra on the half grid
// A 2-D DFT is a row pass (real <-> half spectrum along k1) and a column pass (complex
// FFT along k0).  The row pass of the ADMM fuses: inverse row FFT of the synthesised
// coefficient spectrum, the shrinkage/multiplier update of the state, and the forward
// row FFT of the next adjoint input, so the state is read and written once per
// iteration.  Column passes stream strips of W adjacent columns (coalesced) and loop
// over filters with the spectrum of u (synthesis) or the adjoint accumulator (analysis)
// held in registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.hpp"

namespace shs {

// ---------------------------------------------------------------- storage types
enum StoreKind { ST_F32 = 0, ST_BF16 = 1, ST_F16 = 2 };

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
// float -> bf16, round to nearest even (the gfx950 conversion instruction)
__device__ __forceinline__ uint16_t f_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f2_to_bf16x2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}
__device__ __forceinline__ float f16_to_f(uint16_t h) {
  _Float16 v = __builtin_bit_cast(_Float16, h);
  return float(v);
}
__device__ __forceinline__ uint16_t f_to_f16(float f) {
  _Float16 v = _Float16(f);
  return __builtin_bit_cast(uint16_t, v);
}

// Load / store a pixel pair (x, x+1), x even, of a state image.
template <int ST> struct Store;
template <> struct Store<ST_F32> {
  using T = float;
  using Pair = float2;
  __device__ __forceinline__ static Pair load_pair(const T* p) { return *reinterpret_cast<const float2*>(p); }
  __device__ __forceinline__ static void unpack(Pair v, float& a, float& b) { a = v.x; b = v.y; }
  __device__ __forceinline__ static void store2(T* p, float a, float b) {
    *reinterpret_cast<float2*>(p) = make_float2(a, b);
  }
  __device__ __forceinline__ static float round(float a) { return a; }
  // round a and b to the storage type in place; returns the stored pair
  __device__ __forceinline__ static Pair round2(float& a, float& b) { return make_float2(a, b); }
  __device__ __forceinline__ static void store_pair(T* p, Pair v) { *reinterpret_cast<float2*>(p) = v; }
  __device__ __forceinline__ static float to_float(T a) { return a; }
  __device__ __forceinline__ static T from_float(float a) { return a; }
};
template <> struct Store<ST_BF16> {
  using T = uint16_t;
  using Pair = uint32_t;
  __device__ __forceinline__ static Pair load_pair(const T* p) { return *reinterpret_cast<const uint32_t*>(p); }
  __device__ __forceinline__ static void unpack(Pair v, float& a, float& b) {
    a = bf16_to_f(uint16_t(v & 0xffffu)); b = bf16_to_f(uint16_t(v >> 16));
  }
  __device__ __forceinline__ static void store2(T* p, float a, float b) {
    *reinterpret_cast<uint32_t*>(p) = f2_to_bf16x2(a, b);
  }
  __device__ __forceinline__ static float round(float a) { return bf16_to_f(f_to_bf16(a)); }
  __device__ __forceinline__ static Pair round2(float& a, float& b) {
    const uint32_t v = f2_to_bf16x2(a, b);
    a = __uint_as_float(v << 16);
    b = __uint_as_float(v & 0xffff0000u);
    return v;
  }
  __device__ __forceinline__ static void store_pair(T* p, Pair v) { *reinterpret_cast<uint32_t*>(p) = v; }
  __device__ __forceinline__ static float to_float(T a) { return bf16_to_f(a); }
  __device__ __forceinline__ static T from_float(float a) { return f_to_bf16(a); }
};
template <> struct Store<ST_F16> {
  using T = uint16_t;
  using Pair = uint32_t;
  __device__ __forceinline__ static Pair load_pair(const T* p) { return *reinterpret_cast<const uint32_t*>(p); }
  __device__ __forceinline__ static void unpack(Pair v, float& a, float& b) {
    a = f16_to_f(uint16_t(v & 0xffffu)); b = f16_to_f(uint16_t(v >> 16));
  }
  __device__ __forceinline__ static void store2(T* p, float a, float b) {
    *reinterpret_cast<uint32_t*>(p) = uint32_t(f_to_f16(a)) | (uint32_t(f_to_f16(b)) << 16);
  }
  __device__ __forceinline__ static float round(float a) { return f16_to_f(f_to_f16(a)); }
  __device__ __forceinline__ static Pair round2(float& a, float& b) {
    // one packed conversion (round to nearest even) for both values
    const f16x2_t h = __builtin_convertvector((f32x2_t){a, b}, f16x2_t);
    a = float(h[0]);
    b = float(h[1]);
    return __builtin_bit_cast(uint32_t, h);
  }
  __device__ __forceinline__ static void store_pair(T* p, Pair v) { *reinterpret_cast<uint32_t*>(p) = v; }
  __device__ __forceinline__ static float to_float(T a) { return f16_to_f(a); }
  __device__ __forceinline__ static T from_float(float a) { return f_to_f16(a); }
};

// x clipped to [-th, th] (th >= 0): one median-of-three instruction
__device__ __forceinline__ float clip(float x, float th) { return __builtin_amdgcn_fmed3f(x, -th, th); }

// 16 bytes of stored pairs (2 FP32 pairs or 4 16-bit pairs), moved with one vector access.
template <class Pair>
struct PairVec {
  static constexpr int V = 16 / int(sizeof(Pair));
  __device__ __forceinline__ static void load(const void* p, Pair (&out)[V]) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    const unsigned w[4] = {v.x, v.y, v.z, v.w};
    if constexpr (V == 4) {
      for (int i = 0; i < 4; ++i) out[i] = __builtin_bit_cast(Pair, w[i]);
    } else {
      for (int i = 0; i < 2; ++i) out[i] = make_float2(__uint_as_float(w[2 * i]), __uint_as_float(w[2 * i + 1]));
    }
  }
  __device__ __forceinline__ static void store(void* p, const Pair (&in)[V]) {
    uint4 v;
    if constexpr (V == 4) {
      v.x = __builtin_bit_cast(unsigned, in[0]); v.y = __builtin_bit_cast(unsigned, in[1]);
      v.z = __builtin_bit_cast(unsigned, in[2]); v.w = __builtin_bit_cast(unsigned, in[3]);
    } else {
      v.x = __float_as_uint(in[0].x); v.y = __float_as_uint(in[0].y);
      v.z = __float_as_uint(in[1].x); v.w = __float_as_uint(in[1].y);
    }
    *reinterpret_cast<uint4*>(p) = v;
  }
};

// ---------------------------------------------------------------- FP64 block reduction
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Deterministic sum of 4 values over a block of NWAVES waves; result valid in thread 0.
template <int NWAVES>
__device__ __forceinline__ void block_sum4(double (&v)[4], double* sh) {
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) sh[wave * 4 + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double s = 0.0;
      for (int w = 0; w < NWAVES; ++w) s += sh[w * 4 + i];
      v[i] = s;
    }
  }
}
// The same over a block of `nwaves` waves (a launch-time block size).
__device__ __forceinline__ void block_sum4_n(double (&v)[4], double* sh, int nwaves) {
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) sh[wave * 4 + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double s = 0.0;
      for (int w = 0; w < nwaves; ++w) s += sh[w * 4 + i];
      v[i] = s;
    }
  }
}
// Partial-sum slots: 0 = |dy|^2, 1 = |db|^2, 2 = <w, s>, 3 = sum lambda |v| (or energy l1).
enum { SLOT_DY2 = 0, SLOT_DB2 = 1, SLOT_WS = 2, SLOT_L1 = 3 };

// ---------------------------------------------------------------- filter bank (FP64)
// Meyer building blocks of Section 2 (eq. (psi1_psi2), the auxiliary polynomial v, the
// profile b and the scaling-function profile), evaluated in double precision.
__device__ __forceinline__ double mey_v(double x) {
  if (x < 0.0) return 0.0;
  if (x > 1.0) return 1.0;
  const double x2 = x * x;
  return x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
}
__device__ __forceinline__ double mey_b(double x) {
  const double a = fabs(x);
  if (a >= 1.0 && a <= 2.0) return sin(0.5 * M_PI * mey_v(a - 1.0));
  if (a > 2.0 && a <= 4.0) return cos(0.5 * M_PI * mey_v(0.5 * a - 1.0));
  return 0.0;
}
__device__ __forceinline__ double mey_psi1(double w) {
  const double b2 = mey_b(2.0 * w), b1 = mey_b(w);
  return sqrt(b2 * b2 + b1 * b1);
}
__device__ __forceinline__ double mey_psi2(double w) { return w <= 0.0 ? sqrt(mey_v(1.0 + w)) : sqrt(mey_v(1.0 - w)); }
__device__ __forceinline__ double mey_phi(double w) {
  const double a = fabs(w);
  if (a <= 0.5) return 1.0;
  if (a < 1.0) return cos(0.5 * M_PI * mey_v(2.0 * a - 1.0));
  return 0.0;
}

// Decode filter index f (documented order) into kind (0 low, 1 h, 2 v, 3 seam), scale, shear.
__device__ __forceinline__ void decode_filter(int f, int& kind, int& j, int& k) {
  if (f == 0) { kind = 0; j = 0; k = 0; return; }
  int rem = f - 1;
  j = 0;
  while (rem >= (4 << j)) { rem -= (4 << j); ++j; }
  const int ns = (2 << j) - 1;      // shears per cone at scale j
  const int half = (1 << j) - 1;
  if (rem < ns) { kind = 1; k = rem - half; }
  else if (rem < 2 * ns) { kind = 2; k = rem - ns - half; }
  else { kind = 3; k = (rem == 2 * ns) ? -(1 << j) : (1 << j); }
}

// psi1(4^-j a) psi2(2^j b/a + k): the sheared, dilated shearlet of Section 2 (a != 0).
__device__ __forceinline__ double shear_val(double a, double b, int j, int k) {
  return mey_psi1(a / double(1 << (2 * j))) * mey_psi2(double(1 << j) * b / a + double(k));
}

// Filter value at integer frequencies (o1, o2) with xi = rho * omega.
__device__ double filter_value(int kind, int j, int k, int o1, int o2, double rho) {
  const double x1 = rho * o1, x2 = rho * o2;
  const int a1 = o1 < 0 ? -o1 : o1, a2 = o2 < 0 ? -o2 : o2;
  if (kind == 0) return mey_phi(fmax(fabs(x1), fabs(x2)));
  double v = 0.0;
  if (kind != 2 && a2 < a1) v += shear_val(x1, x2, j, k);         // horizontal cone
  if (kind != 1 && a1 < a2) v += shear_val(x2, x1, j, k);         // vertical cone
  if (kind == 3 && a1 == a2 && a1 > 0) v += shear_val(x1, x2, j, k);  // seam line
  return v;
}

__device__ __forceinline__ int freq_of(int idx, int n) { return idx < (n + 1) / 2 ? idx : idx - n; }

// One thread per (filter, k0, k1) of the half spectrum (k1 <= N/2).
__global__ void k_filter_gen(float* __restrict__ psi, int n, int J, int P, int eta) {
  const int half = n / 2 + 1;
  const long long total = (long long)eta * n * half;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int k1 = int(i % half);
  const int k0 = int((i / half) % n);
  const int f = int(i / ((long long)half * n));
  int kind, j, k;
  decode_filter(f, kind, j, k);
  const double rho = double(1 << (2 * J)) / double(n);
  const int o1 = freq_of(k0, n), o2 = freq_of(k1, n);
  double v = filter_value(kind, j, k, o1, o2, rho);
  if ((n % 2 == 0) && (k0 == n / 2 || k1 == n / 2)) {
    // Nyquist bins: energy-symmetrise with the mirror bin -omega (mod N).
    const int m0 = (n - k0) % n, m1 = (n - k1) % n;
    const double w = filter_value(kind, j, k, freq_of(m0, n), freq_of(m1, n), rho);
    v = sqrt(0.5 * (v * v + w * w));
  }
  psi[((long long)f * n + k0) * P + k1] = float(v);
}

// ---------------------------------------------------------------- data term
struct Codebook { float c[8 * 4]; };
// s[k][p] = sum_c |f[c][p] - cb[k][c]|^p (eq. (computationOfs), colour form of Section 4).
__global__ void k_datacost(const float* __restrict__ img, int C, Codebook cb, int q, float pw,
                           float* __restrict__ s, long long n2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  float f[4];
  for (int c = 0; c < C; ++c) f[c] = img[c * n2 + i];
  for (int k = 0; k < q; ++k) {
    float acc = 0.f;
    for (int c = 0; c < C; ++c) {
      const float d = f[c] - cb.c[k * 4 + c];
      acc += (pw == 2.0f) ? d * d : powf(fabsf(d), pw);
    }
    s[k * n2 + i] = acc;
  }
}

// ---------------------------------------------------------------- strip geometry
// Column FFTs have complex length N: radix R (and middle radix RM), one strip of W
// adjacent columns per block, W * T threads.  Strip s holds columns [s W, s W + W) (only
// those <= N/2 exist).  Strips are stored as contiguous blocks, so W only trades block
// size against occupancy (W = 4 at N = 1024: 256 threads, 34 KB of LDS with the pad
// slots, four blocks per CU).
// WPE is the occupancy hint of the filtered column passes (waves per SIMD).  At N = 2048
// they run at two waves and load the next filter's spectrum column and filter values
// during the current FFT (PREFETCH); with more waves per SIMD those extra registers would
// spill.
template <int N> struct ColGeom;
template <> struct ColGeom<64>   { static constexpr int R = 8,  RM = 1, W = 16, WPE = 3; };
template <> struct ColGeom<128>  { static constexpr int R = 8,  RM = 2, W = 16, WPE = 3; };
template <> struct ColGeom<256>  { static constexpr int R = 16, RM = 1, W = 16, WPE = 3; };
template <> struct ColGeom<512>  { static constexpr int R = 16, RM = 2, W = 8,  WPE = 3; };
template <> struct ColGeom<1024> { static constexpr int R = 16, RM = 4, W = 4,  WPE = 4; };
template <> struct ColGeom<2048> { static constexpr int R = 16, RM = 8, W = 4,  WPE = 2; };
template <int N> struct ColCfg : ColGeom<N> {
  static constexpr int T = N / ColGeom<N>::R;
  static constexpr int THREADS = ColGeom<N>::W * T;
  static constexpr bool PREFETCH = ColGeom<N>::WPE <= 2;
};

// Half-spectrum planes are stored in strips: strip s of a plane (columns [s W, s W + W))
// is one contiguous block of N * W bins, bin (k0, k1) at k0 * W + (k1 mod W).  A column
// pass streams a whole block; a row pass (8 consecutive rows per block) reads 8 * W
// contiguous bins per strip.  tix gives the bin offset of column ip of a plane, with
// floor division for negative ip: a plane of `pitch` columns (pitch a multiple of W)
// spans offsets [0, pitch * N), and every ip outside [0, pitch) lands outside that span
// (negative offsets wrap to above 2^31 as unsigned byte offsets).
template <int N>
__device__ __forceinline__ int tix(int ip, int row) {
  constexpr int W = ColGeom<N>::W;
  constexpr int S = W == 4 ? 2 : W == 8 ? 3 : 4;
  static_assert((1 << S) == W, "strip width");
  return (ip >> S) * (N * W) + row * W + (ip & (W - 1));
}

// A bin index whose byte offset (times 8, modulo 2^32) stays far above any plane size,
// also after adding a row or column stride: loads from it read zero.
constexpr int kOutOfPlane = -(1 << 26);

// Raw buffer view of one spectrum plane.  The hardware range check of buffer accesses
// (offset >= size) makes loads outside the plane return zero and drops such stores, so
// the wedge window of a row needs no branches.
struct PlaneBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ PlaneBuf(const float2* base, int bins)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(base), short(0), bins * 8, 0x00020000)) {}
  __device__ __forceinline__ cpx load(int bin) const {
    // (elements are taken by value: a bit cast of a vector-element lvalue would read
    // element 0 for both)
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, unsigned(bin) * 8u, 0, 0);
    const unsigned lo = v[0], hi = v[1];
    return cpx{__uint_as_float(lo), __uint_as_float(hi)};
  }
  __device__ __forceinline__ void store(int bin, cpx x) const {
    using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0, 0));
    u2 v;
    v[0] = __float_as_uint(x.x);
    v[1] = __float_as_uint(x.y);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, unsigned(bin) * 8u, 0, 0);
  }
};

// Block coordinates of a kernel body: its own grid's blockIdx.x / blockIdx.y / gridDim.x,
// or the block's place inside one image's part of a grouped launch (see grouped.hpp).
struct BlockId {
  int x, y, gx;
};
__device__ __forceinline__ BlockId own_block() { return BlockId{int(blockIdx.x), int(blockIdx.y), int(gridDim.x)}; }

// ---------------------------------------------------------------- row pass
enum RowMode { ROW_SOLVE = 0, ROW_C2R = 1, ROW_R2C = 2, ROW_PRIME = 3, ROW_ENERGY = 4, ROW_SHRINK = 5, ROW_PD = 6 };

// Row FFTs have complex length M = N/2: (R, RM) with R * R * RM = M.
template <int M> struct RowFft;
template <> struct RowFft<32>   { static constexpr int R = 4,  RM = 2; };
template <> struct RowFft<64>   { static constexpr int R = 8,  RM = 1; };
template <> struct RowFft<128>  { static constexpr int R = 8,  RM = 2; };
template <> struct RowFft<256>  { static constexpr int R = 16, RM = 1; };
template <> struct RowFft<512>  { static constexpr int R = 16, RM = 2; };
template <> struct RowFft<1024> { static constexpr int R = 16, RM = 4; };

// The row FFT's twiddles sit in LDS, copied once per block: the real-FFT pre/post factors
// W_N^k (k < M for N <= 512; for larger N only W_N^t, t < T, and the other factors are
// W_N^t times a compile-time constant) followed by the stage table of fft_run.  Reading
// every stage power from LDS needs no products and takes those loads off the vector-memory
// data path, which the row pass keeps busy.  Sizes keep four waves per SIMD: four blocks
// of four waves per CU up to N = 1024, two blocks of eight waves at N = 2048.
template <int N> struct RowGeom {
  static constexpr int M = N / 2;
  static constexpr int R = RowFft<M>::R;
  static constexpr int RM = RowFft<M>::RM;
  static constexpr int T = M / R;
  static constexpr int RPW = 64 / T;          // rows per wave
  static constexpr int WAVES = N >= 2048 ? 8 : 4;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int RPB = RPW * WAVES;     // rows per block
  static constexpr int LROW = M + M / R;      // LDS float2 per row (padded)
  static constexpr bool PREFULL = N <= 512;   // all M pre/post factors in LDS
  static constexpr int TW_PRE = PREFULL ? M : T;
  static constexpr int TW_STAGE = stage_tw_size<M, R, RM>();
  static constexpr int TW_LDS = TW_PRE + TW_STAGE;
};

// Twiddle tables of a power-of-two plan, one device array: [0, N) holds exp(-2 pi i m / N);
// then the stage table of the row FFTs (length N/2), then that of the column FFTs
// (length N).
template <int N> constexpr int row_sw_off() { return N; }
template <int N> constexpr int col_sw_off() {
  return N + stage_tw_size<N / 2, RowGeom<N>::R, RowGeom<N>::RM>();
}
template <int N> constexpr int tw_table_size() {
  return col_sw_off<N>() + stage_tw_size<N, ColGeom<N>::R, ColGeom<N>::RM>();
}

constexpr int kMaxFilters = 256;
struct FilterWeights {
  float thr[kMaxFilters];   // per-filter threshold gamma * lambda_j
  float lam[kMaxFilters];   // per-filter weight lambda_j
};

// A family of half-spectrum planes.  Plane (l, f) at base + l * ls + off_f keeps the
// columns [cb_f, cb_f + pitch_f) (whole strips, cb_f and pitch_f multiples of W) in strip
// blocks: bin (k0, k1) at tix(k1 - cb_f, k0).  The filtered spectra (synthesis input /
// adjoint output of filter f) keep only the strips where filter f is nonzero (wedge
// pruning); per-label spectra are dense (one plane, cb 0, all P = NS * W columns).
struct SpecLayout {
  const int4* tab;   // per filter {cb, pitch, off_lo, off_hi}; null = dense
  long long ls;      // label stride (float2)
  int nf;            // planes per label (eta, or 1 when dense)
  int P;             // columns of a dense plane (NS * W)
};
__device__ __forceinline__ void plane_geom(const SpecLayout& L, int f, int& cb, int& pitch, long long& off) {
  if (L.tab) {
    // f is uniform over the block: keep the entry in scalar registers
    const int4 e = L.tab[f];
    cb = __builtin_amdgcn_readfirstlane(e.x);
    pitch = __builtin_amdgcn_readfirstlane(e.y);
    off = (long long)(unsigned)__builtin_amdgcn_readfirstlane(e.z) |
          ((long long)__builtin_amdgcn_readfirstlane(e.w) << 32);
  } else {
    cb = 0; pitch = L.P; off = 0;
  }
}

struct RowParams {
  const float2* spec_in;   // half spectra read (SOLVE, C2R, ENERGY)
  float2* spec_out;        // half spectra written (SOLVE, R2C, PRIME)
  SpecLayout lin, lout;    // their layouts
  const float* real_in;    // real rows read (R2C)
  float* real_out;         // real rows written (C2R)
  void* g;                 // ADMM state g_v (SOLVE, PRIME)
  const float2* tw;        // exp(-2 pi i m / N), m < N
  double* partials;        // [blocks][4] FP64 partial sums (STATS)
  long long real_cs;       // channel stride of real rows (floats)
  int eta;                 // filters per label: filter of channel ch is ch % eta
  int emit;                // SOLVE: write the next adjoint input spectrum
  float sigma;             // PD: dual step size
  FilterWeights fw;        // passed by value (kernel argument memory)
};

// Column offset of the row bins at k = t + r*T, k - cb and M - k - cb, as strip-tiled
// bin offsets: when T is a whole number of strips they step by a constant.
template <int N, int SIGN>
__device__ __forceinline__ int row_bin(int base_ip, int base_off, int r, int row) {
  using G = RowGeom<N>;
  constexpr int W = ColGeom<N>::W;
  if constexpr (G::T % W == 0) {
    return base_off + SIGN * r * (G::T * N);
  } else {
    return tix<N>(base_ip + SIGN * r * G::T, row);
  }
}

// W_N^k for k = t + r*T from the row pass's LDS twiddle table.
template <int N, int r>
__device__ __forceinline__ cpx pre_twiddle(const float2* twl, int t) {
  using G = RowGeom<N>;
  if constexpr (G::PREFULL) return ld(twl + t + r * G::T);
  else return twc<r * G::T, N, false>(ld(twl + t));
}

// Inverse real FFT of a half-spectrum row (unnormalised): X[0..M] -> x[0..N) with
// point pair (2p, 2p+1) of p = t + r*T in a[r] = (x[2p], x[2p+1]).  The plane holds the
// columns [cb, cb + pitch); other bins are zero.  twl: the block's LDS twiddle table.
template <int N, class Addr>
__device__ __forceinline__ void row_c2r(cpx (&a)[RowGeom<N>::R], const float2* __restrict__ X, int row, int cb,
                                        int pitch, const Addr& A, int t, const float2* twl) {
  using G = RowGeom<N>;
  const PlaneBuf B(X, pitch * N);
  const int ip0 = t - cb, im0 = G::M - t - cb;
  const int op0 = tix<N>(ip0, row), om0 = tix<N>(im0, row);
  // Chunk r covers k in [r T, r T + T) for every row of the wave; whether it meets the
  // window (directly or mirrored) is uniform, so chunks outside it are skipped whole.  Bins
  // of a partly covered chunk outside the plane's columns map below 0 or at or above
  // pitch * N: their loads are out of range and read zero.  (Issuing every load instead of
  // branching was measured slower: this pass keeps the vector-memory data path near
  // saturation.)
  cpx xp[G::R], xm[G::R];
  const auto in_p = [&](int k0) { return k0 < cb + pitch && k0 + G::T > cb; };
  const auto in_m = [&](int k0) { return k0 <= G::M - cb && k0 + G::T > G::M - cb - pitch; };
  static_for<G::R>([&](auto r) {
    constexpr int k0 = r * G::T;
    xp[r] = cpx{0.f, 0.f};
    if (in_p(k0)) xp[r] = B.load(row_bin<N, 1>(ip0, op0, r, row));
  });
  // Each bin is loaded once.  The mirrored bins X[M - k] come from the lanes that loaded
  // them, through the LDS crossbar (ds_bpermute) instead of the vector-memory path: for
  // t > 0, bin M - t - r T = (T - t) + (R - 1 - r) T is lane T - t's xp[R - 1 - r] (zero
  // where that chunk was not loaded: outside the window); lane t = 0 holds X[M - r T]
  // itself as xp[R - r] and loads X[M].
  const int src = (int(threadIdx.x & 63u) - t + ((G::T - t) & (G::T - 1))) << 2;
  cpx xnyq = cpx{0.f, 0.f};
  if (t == 0 && in_m(0)) xnyq = B.load(om0);
  static_for<G::R>([&](auto r) {
    constexpr int k0 = r * G::T;
    constexpr int rs = G::R - 1 - r;
    xm[r] = cpx{0.f, 0.f};
    if (in_m(k0)) {
      cpx v = cpx{__int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(xp[rs].x))),
                  __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(xp[rs].y)))};
      if (t == 0) {
        if constexpr (r == 0) v = xnyq;
        else v = xp[G::R - r];
      }
      xm[r] = v;
    }
  });
  // z[k] = s + i d W_N^{-k} with s = X[k] + conj(X[M-k]), d = X[k] - conj(X[M-k]): the
  // product folded into FMAs; chunks with neither bin range in the window are zero.
  static_for<G::R>([&](auto r) {
    constexpr int k0 = r * G::T;
    if (in_p(k0) || in_m(k0)) {
      const cpx s = xp[r] + conj(xm[r]), d = xp[r] - conj(xm[r]);
      const cpx w = pre_twiddle<N, r>(twl, t);   // W_N^{k}
      a[r] = cpx{fmaf(d.x, w.y, fmaf(-d.y, w.x, s.x)), fmaf(d.x, w.x, fmaf(d.y, w.y, s.y))};
    } else {
      a[r] = cpx{0.f, 0.f};
    }
  });
  fft_run<G::M, G::R, G::RM, true, SYNC_WAVE, Addr, 1>(a, A, t, twl + G::TW_PRE);
}

// Forward real FFT of a row held as pairs a[r] = (x[2p], x[2p+1]); writes the bins of
// X[0..M] that fall in [cb, cb + pitch).  HALF: the row was passed in halved, which takes
// the post-processing's factor 1/2 (exact: a power of two commutes with the FFT's
// rounding).
template <int N, bool HALF, class Addr>
__device__ __forceinline__ void row_r2c(cpx (&a)[RowGeom<N>::R], float2* __restrict__ X, int row, int cb, int pitch,
                                        const Addr& A, int t, const float2* twl) {
  using G = RowGeom<N>;
  fft_run<G::M, G::R, G::RM, false, SYNC_WAVE, Addr, 1>(a, A, t, twl + G::TW_PRE);
  const int tq = int(unsigned(t) / G::R), tr = int(unsigned(t) % G::R);
  fft_sync<SYNC_WAVE>();
  static_for<G::R>([&](auto r) { st(A.template at<G::R>(tq + r * G::RM, tr), a[r]); });
  fft_sync<SYNC_WAVE>();
  const PlaneBuf B(X, pitch * N);
  const int ip0 = t - cb, op0 = tix<N>(ip0, row);
  static_for<G::R>([&](auto r) {
    constexpr int k0 = r * G::T;
    if (k0 < cb + pitch && k0 + G::T > cb) {
      const int k = t + k0;
      const cpx yk = a[r];
      const cpx ym = conj(ld(A(unsigned(G::M - k) & unsigned(G::M - 1))));
      const cpx s = yk + ym, d = yk - ym;
      const cpx w = pre_twiddle<N, r>(twl, t);   // W_N^{k}
      // (s - i d w) / 2, the product folded into FMAs
      cpx x = cpx{fmaf(d.x, w.y, fmaf(d.y, w.x, s.x)), fmaf(-d.x, w.x, fmaf(d.y, w.y, s.y))};
      if constexpr (!HALF) x = x * 0.5f;
      B.store(row_bin<N, 1>(ip0, op0, r, row), x);
    }
  });
  if (t == 0) B.store(tix<N>(G::M - cb, row), cpx{HALF ? 2.f * (a[0].x - a[0].y) : a[0].x - a[0].y, 0.f});
}

template <int N, int MODE, int ST, bool STATS>
__device__ __forceinline__ void row_body(const RowParams& p, BlockId bid) {
  using G = RowGeom<N>;
  using S = Store<ST>;
  using PV = PairVec<typename S::Pair>;
  static_assert(G::R % PV::V == 0, "a thread's pairs fill whole 16-byte groups");
  __shared__ float2 lds[G::RPB * G::LROW];
  __shared__ float2 twl[G::TW_LDS];
  __shared__ double red[G::WAVES * 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane / G::T, t = lane % G::T;
  const int rowl = wave * G::RPW + sub;
  const int row = bid.x * G::RPB + rowl;
  const int ch = bid.y;
  const int j = ch % p.eta;
  const RowAddr<G::R> A{lds + rowl * G::LROW};
  cpx a[G::R];
  float acc[4] = {0.f, 0.f, 0.f, 0.f};   // per-thread partial sums of one row segment
  typename S::T* gp = nullptr;
  typename S::Pair gv[G::R];
  if constexpr (MODE == ROW_SOLVE || MODE == ROW_PRIME || MODE == ROW_PD) {
    // The state does not depend on the inverse FFT below: load it first so its latency
    // overlaps the FFT.  A row of the state is stored in the order the row pass holds it:
    // thread t's pairs r = V i .. V i + V - 1 (points 2p, 2p+1 of p = t + r T) are the 16
    // bytes at pair offset (i T + t) V, so each of the R / V loads (and stores) of a wave is
    // one contiguous run per row.  Only this pass reads or writes the state.
    gp = reinterpret_cast<typename S::T*>(p.g) + (long long)ch * N * N + (long long)row * N;
    static_for<G::R / PV::V>([&](auto i) {
      typename S::Pair v[PV::V];
      PV::load(gp + 2 * PV::V * (i * G::T + t), v);
      static_for<PV::V>([&](auto e) { gv[i * PV::V + e] = v[e]; });
    });
  }
  // the block's twiddle table (pre/post factors, then the FFT stage table)
  for (int e = threadIdx.x; e < G::TW_LDS; e += G::THREADS)
    twl[e] = p.tw[e < G::TW_PRE ? e : row_sw_off<N>() + (e - G::TW_PRE)];
  __syncthreads();

  if constexpr (MODE == ROW_SOLVE || MODE == ROW_C2R || MODE == ROW_ENERGY || MODE == ROW_SHRINK || MODE == ROW_PD) {
    int cb, pitch;
    long long off;
    const int f = ch % p.lin.nf;
    plane_geom(p.lin, f, cb, pitch, off);
    const float2* X = p.spec_in + (ch / p.lin.nf) * p.lin.ls + off;
    row_c2r<N>(a, X, row, cb, pitch, A, t, twl);
  }
  if constexpr (MODE == ROW_C2R) {
    float* out = p.real_out + ch * p.real_cs + (long long)row * N;
    static_for<G::R>([&](auto r) {
      const int k = t + r * G::T;
      *reinterpret_cast<float2*>(out + 2 * k) = make_float2(a[r].x, a[r].y);
    });
    return;
  }
  if constexpr (MODE == ROW_ENERGY) {
    static_for<G::R>([&](auto r) { acc[SLOT_L1] += fabsf(a[r].x) + fabsf(a[r].y); });
  }
  if constexpr (MODE == ROW_R2C) {
    const float* in = p.real_in + ch * p.real_cs + (long long)row * N;
    static_for<G::R>([&](auto r) {
      const int k = t + r * G::T;
      const float2 v = *reinterpret_cast<const float2*>(in + 2 * k);
      a[r] = cpx{v.x, v.y};
    });
  }
  if constexpr (MODE == ROW_SOLVE || MODE == ROW_PRIME) {
    const float th = p.fw.thr[j];
    typename S::Pair nv[PV::V];
    static_for<G::R>([&](auto r) {
      float g0, g1;
      S::unpack(gv[r], g0, g1);
      const float b0 = clip(g0, th), b1 = clip(g1, th);
      float n0 = g0, n1 = g1;
      if constexpr (MODE == ROW_SOLVE) {
        // g <- clip(g) + S_j u  (v = shrink(g), b_v = clip(g); Section 3 v- and b_v-updates)
        n0 = b0 + a[r].x;
        n1 = b1 + a[r].y;
        nv[r % PV::V] = S::round2(n0, n1);
        if constexpr (r % PV::V == PV::V - 1) PV::store(gp + 2 * PV::V * ((r / PV::V) * G::T + t), nv);
      }
      const float nb0 = clip(n0, th), nb1 = clip(n1, th);
      if constexpr (STATS && MODE == ROW_SOLVE) {
        const float dv0 = (n0 - nb0) - (g0 - b0), dv1 = (n1 - nb1) - (g1 - b1);
        const float db0 = nb0 - b0, db1 = nb1 - b1;
        acc[SLOT_DY2] = fmaf(dv0, dv0, acc[SLOT_DY2]);
        acc[SLOT_DY2] = fmaf(dv1, dv1, acc[SLOT_DY2]);
        acc[SLOT_DB2] = fmaf(db0, db0, acc[SLOT_DB2]);
        acc[SLOT_DB2] = fmaf(db1, db1, acc[SLOT_DB2]);
        acc[SLOT_L1] += fabsf(n0 - nb0);
        acc[SLOT_L1] += fabsf(n1 - nb1);
      }
      // next adjoint input v - b_v = g - 2 clip(g), passed on halved (see row_r2c)
      a[r] = cpx{fmaf(0.5f, n0, -nb0), fmaf(0.5f, n1, -nb1)};
    });
    // Complete the residual partial sums here (an empty asm that reads and writes them):
    // otherwise the compiler sinks them past the forward FFT and keeps every per-pixel
    // term live, doubling the register footprint.
    if constexpr (STATS && MODE == ROW_SOLVE) __asm__ volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[3]));
  }
  if constexpr (MODE == ROW_PD) {
    // dual step of the primal-dual iteration: y <- clip(y + sigma c, +-lambda_j), c = (K ubar)_j
    const float th = p.fw.thr[j];
    typename S::Pair nv[PV::V];
    static_for<G::R>([&](auto r) {
      float y0, y1;
      S::unpack(gv[r], y0, y1);
      float n0 = clip(fmaf(p.sigma, a[r].x, y0), th);
      float n1 = clip(fmaf(p.sigma, a[r].y, y1), th);
      nv[r % PV::V] = S::round2(n0, n1);
      if constexpr (r % PV::V == PV::V - 1) PV::store(gp + 2 * PV::V * ((r / PV::V) * G::T + t), nv);
      if constexpr (STATS) {
        const float d0 = n0 - y0, d1 = n1 - y1;
        acc[SLOT_DY2] += d0 * d0 + d1 * d1;
        acc[SLOT_L1] += fabsf(a[r].x) + fabsf(a[r].y);
      }
      a[r] = cpx{n0, n1};
    });
    if constexpr (STATS) __asm__ volatile("" : "+v"(acc[0]), "+v"(acc[3]));
  }
  if constexpr (MODE == ROW_SHRINK) {
    // soft shrinkage of the coefficient row (Section 3's S_lambda, threshold thr_j)
    const float th = p.fw.thr[j];
    static_for<G::R>([&](auto r) {
      a[r] = cpx{a[r].x - clip(a[r].x, th), a[r].y - clip(a[r].y, th)};
    });
  }
  if constexpr (MODE == ROW_R2C || MODE == ROW_PRIME || MODE == ROW_SOLVE || MODE == ROW_SHRINK || MODE == ROW_PD) {
    bool emit = true;
    if constexpr (MODE == ROW_SOLVE) emit = p.emit != 0;
    if (emit) {
      int cb, pitch;
      long long off;
      const int f = ch % p.lout.nf;
      plane_geom(p.lout, f, cb, pitch, off);
      float2* X = p.spec_out + (ch / p.lout.nf) * p.lout.ls + off;
      row_r2c<N, MODE == ROW_SOLVE || MODE == ROW_PRIME>(a, X, row, cb, pitch, A, t, twl);
    }
  }
  if constexpr (STATS) {
    // FP32 partials of one row segment (2R pixels) per thread, FP64 from here on.
    double d[4] = {double(acc[0]), double(acc[1]), double(acc[2]), double(acc[3])};
    d[SLOT_L1] *= double(p.fw.lam[j]);
    block_sum4<G::WAVES>(d, red);
    if (threadIdx.x == 0) {
      double* o = p.partials + ((long long)bid.y * bid.gx + bid.x) * 4;
      o[0] = d[0]; o[1] = d[1]; o[2] = d[2]; o[3] = d[3];
    }
  }
}

template <int N, int MODE, int ST, bool STATS>
__global__ __launch_bounds__(RowGeom<N>::THREADS) void k_row(RowParams p) {
  row_body<N, MODE, ST, STATS>(p, own_block());
}

// ---------------------------------------------------------------- column passes
// Work item of a column pass: strip, a run of filters (indices into flist) whose
// column range meets the strip, and the partial-accumulator slot (analysis; -1 when the
// strip has a single item and the item finalises directly).
struct ColParams {
  const float2* in;       // spectra read
  float2* out;            // spectra written
  const float* psiw;      // filter values inside each column window (compact)
  const int4* pwin;       // [eta][N/2+1] {window start a, length L, value offset, 0}
  SpecLayout tl;          // layout of the filtered spectra (compact)
  const int4* items;      // {strip, first flist index, count, partial slot}
  const int* flist;       // filter ids
  const int2* strips;     // per strip {first analysis item, number of items}
  float2* part;           // partial accumulators [slot][labels][N][W]
  const float2* tw;       // exp(-2 pi i m / N)
  int P, eta, labels;
  int nnz;                // stored filter values in psiw (< 2^29)
  float inv_n2;           // 1 / N^2 (normalisation of the inverse 2-D DFT)
};

constexpr int kItemMax = 16;   // filters per column work item

// A work item's per-filter data, staged in LDS once per block: the column window of
// every (filter, column) pair and the plane geometry {cb, pitch, off_lo, off_hi} of
// every filter.  Without it each filter step waits on three dependent loads.
template <int W> struct ItemStage {
  int4 win[kItemMax][W];
  int4 geo[kItemMax];
};
template <int N>
__device__ __forceinline__ void stage_item(const ColParams& p, int4 it, ItemStage<ColCfg<N>::W>& st) {
  constexpr int W = ColCfg<N>::W, M = N / 2;
  for (int e = threadIdx.x; e < it.z * W; e += ColCfg<N>::THREADS) {
    const int i = e / W, cc = e % W;
    const int j = p.flist[it.y + i];
    const int k1 = it.x * W + cc;
    st.win[i][cc] = k1 <= M ? p.pwin[j * (M + 1) + k1] : make_int4(0, 0, 0, 0);
    if (cc == 0) st.geo[i] = p.tl.tab[j];
  }
}
__device__ __forceinline__ long long geo_off(int4 g) { return (long long)(unsigned)g.z | ((long long)g.w << 32); }

// Filter values of one column window, psi_j(k0, k1) for k0 = t + r T (zero outside the
// window; a wave with no lane inside the window for some r skips that load).
struct PsiBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ explicit PsiBuf(const ColParams& p)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p.psiw), short(0), p.nnz * 4, 0x00020000)) {}
  template <int N, int R, int T>
  __device__ __forceinline__ void load(int4 win, int t, float (&v)[R]) const {
    const unsigned base = unsigned(t - win.x);
    static_for<R>([&](auto rr) {
      const unsigned rel = (base + unsigned(rr * T)) & unsigned(N - 1);
      v[rr] = 0.f;
      if (rel < unsigned(win.y)) v[rr] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (unsigned(win.z) + rel) * 4u, 0, 0));
    });
  }
};

// psi_j(k0, k1) from the compact window of column k1 (zero outside the window).
template <int N>
__device__ __forceinline__ float psi_at(const ColParams& p, int4 win, int k0) {
  const unsigned rel = unsigned(k0 - win.x) & unsigned(N - 1);
  return rel < unsigned(win.y) ? p.psiw[win.z + rel] : 0.f;
}

// Dense column FFT of per-label spectra: U_l = colFFT(V_l) (forward) on every column.
template <int N>
__device__ __forceinline__ void col_fwd_body(const ColParams& p, BlockId bid) {
  using G = ColCfg<N>;
  constexpr int R = G::R, T = G::T, W = G::W, M = N / 2;
  __shared__ float2 lds[col_lds_points<N, R>() * W];
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int k1 = bid.x * W + c;
  const bool valid = k1 <= M;
  const int l = bid.y;
  const ColAddr<W, R> A{lds + c};
  const long long strip = l * (long long)N * p.P + (long long)bid.x * (N * W) + c;
  cpx a[R];
  static_for<R>([&](auto r) { a[r] = valid ? ld(p.in + strip + (t + r * T) * W) : cpx{0.f, 0.f}; });
  fft_run<N, R, G::RM, false, SYNC_BLOCK>(a, A, t, p.tw + col_sw_off<N>());
  if (valid) {
    static_for<R>([&](auto r) { st(p.out + strip + (t + r * T) * W, a[r]); });
  }
}

template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_col_fwd(ColParams p) {
  col_fwd_body<N>(p, own_block());
}

// Synthesis: for every filter j of the item, T1[l, j] = colIFFT(psi_j * U_l / N^2) on the
// item's strip (only columns inside filter j's range exist in T1).  With PREFETCH the next
// filter's values are loaded while the current inverse FFT runs.
template <int N>
__device__ __forceinline__ void col_syn_body(const ColParams& p, BlockId bid) {
  using G = ColCfg<N>;
  constexpr int R = G::R, T = G::T, W = G::W, M = N / 2;
  __shared__ float2 lds[col_lds_points<N, R>() * W];
  __shared__ ItemStage<W> stg;
  __shared__ float2 ctw[stage_tw_pow2_size<N, R, G::RM>()];   // packed stage twiddles
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int4 it = p.items[bid.x];
  const int k1 = it.x * W + c;
  const bool valid = k1 <= M;
  const int l = bid.y;
  const ColAddr<W, R> A{lds + c};
  stage_item<N>(p, it, stg);
  load_stage_tw_pow2<N, R, G::RM>(ctw, p.tw + col_sw_off<N>(), threadIdx.x, G::THREADS);
  cpx uh[R];
  const float2* U = p.in + l * (long long)N * p.P + (long long)it.x * (N * W) + c;
  static_for<R>([&](auto r) { uh[r] = valid ? ld(U + (t + r * T) * W) : cpx{0.f, 0.f}; });
  __syncthreads();
  const PsiBuf PB(p);
  float ps[R];
  if constexpr (G::PREFETCH) PB.load<N, R, T>(stg.win[0][c], t, ps);
  for (int i = 0; i < it.z; ++i) {
    if constexpr (!G::PREFETCH) PB.load<N, R, T>(stg.win[i][c], t, ps);
    cpx a[R];
    static_for<R>([&](auto r) { a[r] = uh[r] * (ps[r] * p.inv_n2); });
    if constexpr (G::PREFETCH) {
      if (i + 1 < it.z) PB.load<N, R, T>(stg.win[i + 1][c], t, ps);
    }
    fft_run<N, R, G::RM, true, SYNC_BLOCK, ColAddr<W, R>, 2>(a, A, t, ctw);
    const int4 geo = stg.geo[i];
    float2* o = p.out + l * p.tl.ls + geo_off(geo) + (long long)(it.x - geo.x / W) * (N * W) + c;
    if (valid) {
      static_for<R>([&](auto r) { st(o + (t + r * T) * W, a[r]); });
    }
  }
}

template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(ColGeom<N>::WPE))) void k_col_syn(ColParams p) {
  col_syn_body<N>(p, own_block());
}

template <int N>
__device__ __forceinline__ void col_finish(const ColParams& p, cpx (&acc)[ColCfg<N>::R], int t, int k1, bool valid,
                                           int l, const ColAddr<ColCfg<N>::W, ColCfg<N>::R>& A) {
  using G = ColCfg<N>;
  constexpr int R = G::R, T = G::T;
  static_for<R>([&](auto r) { acc[r] = acc[r] * p.inv_n2; });
  fft_run<N, R, G::RM, true, SYNC_BLOCK>(acc, A, t, p.tw + col_sw_off<N>());
  float2* o = p.out + l * (long long)N * p.P + (long long)(k1 / G::W) * (N * G::W) + (k1 & (G::W - 1));
  if (valid) {
    static_for<R>([&](auto r) { st(o + (t + r * T) * G::W, acc[r]); });
  }
}

// Analysis: ACC = sum_j psi_j * colFFT(T2[l, j]) over the item's filters.  A strip with a
// single item finishes here (Z_l = colIFFT(ACC / N^2)); otherwise the item's partial
// accumulator is stored and k_col_final sums the strip's items in order.  With PREFETCH
// the next filter's spectrum column is loaded while the current FFT runs.
template <int N>
__device__ __forceinline__ void col_ana_body(const ColParams& p, BlockId bid) {
  using G = ColCfg<N>;
  constexpr int R = G::R, T = G::T, W = G::W, M = N / 2;
  __shared__ float2 lds[col_lds_points<N, R>() * W];
  __shared__ ItemStage<W> stg;
  __shared__ float2 ctw[stage_tw_pow2_size<N, R, G::RM>()];   // packed stage twiddles
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int4 it = p.items[bid.x];
  const int k1 = it.x * W + c;
  const bool valid = k1 <= M;
  const int l = bid.y;
  const ColAddr<W, R> A{lds + c};
  stage_item<N>(p, it, stg);
  load_stage_tw_pow2<N, R, G::RM>(ctw, p.tw + col_sw_off<N>(), threadIdx.x, G::THREADS);
  __syncthreads();
  // T2 column of item filter i; columns past N/2 are never written and read as zero
  auto load_col = [&](int i, cpx (&v)[R]) {
    const int4 geo = stg.geo[i];
    const PlaneBuf B(p.in + l * p.tl.ls + geo_off(geo), geo.y * N);
    const int base = valid ? (it.x - geo.x / W) * (N * W) + t * W + c : kOutOfPlane;
    static_for<R>([&](auto r) { v[r] = B.load(base + r * (T * W)); });
  };
  cpx acc[R], nx[R];
  static_for<R>([&](auto r) { acc[r] = cpx{0.f, 0.f}; });
  if constexpr (G::PREFETCH) load_col(0, nx);
  const PsiBuf PB(p);
  for (int i = 0; i < it.z; ++i) {
    cpx a[R];
    if constexpr (G::PREFETCH) {
      static_for<R>([&](auto r) { a[r] = nx[r]; });
      if (i + 1 < it.z) load_col(i + 1, nx);
    } else {
      load_col(i, a);
    }
    float ps[R];
    PB.load<N, R, T>(stg.win[i][c], t, ps);
    fft_run<N, R, G::RM, false, SYNC_BLOCK, ColAddr<W, R>, 2>(a, A, t, ctw);
    static_for<R>([&](auto r) { acc[r] = acc[r] + a[r] * ps[r]; });
  }
  if (it.w < 0) {
    col_finish<N>(p, acc, t, k1, valid, l, A);
  } else {
    float2* o = p.part + ((long long)it.w * p.labels + l) * (N * W);
    static_for<R>([&](auto r) { st(o + (t + r * T) * W + c, acc[r]); });
  }
}

template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(ColGeom<N>::WPE))) void k_col_ana(ColParams p) {
  col_ana_body<N>(p, own_block());
}

template <int N>
__device__ __forceinline__ void col_final_body(const ColParams& p, BlockId bid) {
  using G = ColCfg<N>;
  constexpr int R = G::R, T = G::T, W = G::W, M = N / 2;
  __shared__ float2 lds[col_lds_points<N, R>() * W];
  const int2 si = p.strips[bid.x];
  if (si.y <= 1) return;
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int k1 = bid.x * W + c;
  const bool valid = k1 <= M;
  const int l = bid.y;
  const ColAddr<W, R> A{lds + c};
  cpx acc[R];
  static_for<R>([&](auto r) { acc[r] = cpx{0.f, 0.f}; });
  for (int i = 0; i < si.y; ++i) {
    const int slot = p.items[si.x + i].w;
    const float2* in = p.part + ((long long)slot * p.labels + l) * (N * W);
    static_for<R>([&](auto r) { acc[r] = acc[r] + ld(in + (t + r * T) * W + c); });
  }
  col_finish<N>(p, acc, t, k1, valid, l, A);
}

template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_col_final(ColParams p) {
  col_final_body<N>(p, own_block());
}

// ---------------------------------------------------------------- plan-time filter windows
// For filter j and column k1: the shortest circular interval of k0 holding every nonzero
// of the column (start a, length L; L = 0 for an all-zero column).
__global__ void k_filter_windows(const float* __restrict__ psi, int n, int P, int eta, int2* __restrict__ win) {
  const int half = n / 2 + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= eta * half) return;
  const int j = i / half, k1 = i % half;
  const float* col = psi + (long long)j * n * P + k1;
  int first = -1, last = -1, prev = -1, gap_best = -1, gap_end = 0;
  for (int k0 = 0; k0 < n; ++k0) {
    if (col[(long long)k0 * P] != 0.f) {
      if (first < 0) first = k0;
      if (prev >= 0 && k0 - prev - 1 > gap_best) { gap_best = k0 - prev - 1; gap_end = k0; }
      prev = k0;
      last = k0;
    }
  }
  if (first < 0) { win[i] = make_int2(0, 0); return; }
  const int wrap = first + n - last - 1;          // zero run across the end of the column
  if (wrap >= gap_best) win[i] = make_int2(first, last - first + 1);
  else win[i] = make_int2(gap_end, n - gap_best);
}

// Gathers the window values: psiw[off + r] = psi[j][(a + r) mod N][k1].
__global__ void k_filter_compact(const float* __restrict__ psi, int n, int P, int eta, const int4* __restrict__ pwin,
                                 float* __restrict__ psiw) {
  const int half = n / 2 + 1;
  for (int i = blockIdx.y; i < eta * half; i += gridDim.y) {   // (j, k1) pair
    const int j = i / half, k1 = i % half;
    const int4 w = pwin[i];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < w.y; r += gridDim.x * blockDim.x)
      psiw[w.z + r] = psi[((long long)j * n + ((w.x + r) % n)) * P + k1];
  }
}

// ---------------------------------------------------------------- per-pixel u / w step
struct PixParams {
  const float* z;      // S^T (v - b_v) per label [q][N^2] (null on the first iteration)
  float* w;            // w   [q][N^2]  (read, written)
  float* bw;           // b_w [q][N^2]  (read, written)
  const float* s;      // data term [q][N^2]
  float* u;            // u   [q][N^2]  (written)
  double* partials;    // [blocks][4]
  long long n2;
  float gamma;
  int q;
};

// Projection of one label vector onto the simplex C, in place: the paper's procedure
// (project onto the hyperplane sum = 1, drop the entries that are not positive,
// re-project the rest, until none is dropped; at most q rounds).
template <int MQ>
__device__ __forceinline__ void simplex_project(float (&g)[MQ], int q) {
  bool act[MQ];
  int cnt = q;
#pragma unroll
  for (int l = 0; l < MQ; ++l) act[l] = l < q;
  float tau = 0.f;
  for (int round = 0; round < MQ; ++round) {
    float sum = 0.f;
#pragma unroll
    for (int l = 0; l < MQ; ++l) sum += act[l] ? g[l] : 0.f;
    tau = (sum - 1.f) / float(cnt);
    bool dropped = false;
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      if (act[l] && g[l] - tau <= 0.f) { act[l] = false; --cnt; dropped = true; }
    }
    if (!dropped) break;
  }
  // a single remaining entry is the vertex: exactly 1 (g - (g - 1) need not round to 1)
#pragma unroll
  for (int l = 0; l < MQ; ++l) g[l] = act[l] ? (cnt == 1 ? 1.f : g[l] - tau) : 0.f;
}

// u = 1/2 [z + (w - b_w) - gamma s]  (Section 3 u-update, A^T A = 2I);
// g_w = b_w + u;  w = P_C(g_w) (pixelwise simplex);  b_w = g_w - w.
template <bool STATS, bool HAVE_Z>
__device__ __forceinline__ void pixel_body(const PixParams& p, BlockId bid) {
  constexpr int MQ = 8;
  __shared__ double red[4 * 4];
  const long long i = (long long)bid.x * 256 + threadIdx.x;
  const bool active = i < p.n2;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (active) {
    float gw[MQ], wn[MQ], wo[MQ], bo[MQ], sv[MQ];
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      gw[l] = 0.f;
      if (l < p.q) {
        const long long o = l * p.n2 + i;
        const float z = HAVE_Z ? p.z[o] : 0.f;
        wo[l] = p.w[o]; bo[l] = p.bw[o]; sv[l] = p.s[o];
        const float u = 0.5f * (z + (wo[l] - bo[l]) - p.gamma * sv[l]);
        p.u[o] = u;
        gw[l] = bo[l] + u;
      }
      wn[l] = gw[l];
    }
    simplex_project<MQ>(wn, p.q);
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      if (l < p.q) {
        const long long o = l * p.n2 + i;
        const float bn = gw[l] - wn[l];
        p.w[o] = wn[l];
        p.bw[o] = bn;
        if constexpr (STATS) {
          const float dw = wn[l] - wo[l], db = bn - bo[l];
          acc[SLOT_DY2] += double(dw) * dw;
          acc[SLOT_DB2] += double(db) * db;
          acc[SLOT_WS] += double(wn[l]) * double(sv[l]);
        }
      }
    }
  }
  if constexpr (STATS) {
    block_sum4<4>(acc, red);
    if (threadIdx.x == 0) {
      double* o = p.partials + (long long)bid.x * 4;
      o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2]; o[3] = acc[3];
    }
  }
}

template <bool STATS, bool HAVE_Z>
__global__ __launch_bounds__(256) void k_pixel(PixParams p) {
  pixel_body<STATS, HAVE_Z>(p, own_block());
}

// Primal step of the primal-dual iteration: u_new = P_C(u - tau (K^T y + s)) and the
// extrapolation ubar = 2 u_new - u.  Here w holds u (read, written), u receives ubar, z
// holds K^T y, gamma is the primal step tau.  Partials: ||u_new - u||^2, <u_new, s>.
template <bool STATS>
__global__ __launch_bounds__(256) void k_pixel_pd(PixParams p) {
  constexpr int MQ = 8;
  __shared__ double red[4 * 4];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool active = i < p.n2;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (active) {
    float un[MQ], uo[MQ], sv[MQ];
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      un[l] = 0.f;
      if (l < p.q) {
        const long long o = l * p.n2 + i;
        uo[l] = p.w[o];
        sv[l] = p.s[o];
        un[l] = uo[l] - p.gamma * (p.z[o] + sv[l]);
      }
    }
    simplex_project<MQ>(un, p.q);
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      if (l < p.q) {
        const long long o = l * p.n2 + i;
        p.w[o] = un[l];
        p.u[o] = 2.f * un[l] - uo[l];
        if constexpr (STATS) {
          const float du = un[l] - uo[l];
          acc[SLOT_DB2] += double(du) * du;
          acc[SLOT_WS] += double(un[l]) * double(sv[l]);
        }
      }
    }
  }
  if constexpr (STATS) {
    block_sum4<4>(acc, red);
    if (threadIdx.x == 0) {
      double* o = p.partials + (long long)blockIdx.x * 4;
      o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2]; o[3] = acc[3];
    }
  }
}

// <u, s> partial sums (energy), one per block.
__global__ __launch_bounds__(256) void k_dot(const float* __restrict__ u, const float* __restrict__ s,
                                             long long n, double* partials) {
  __shared__ double red[4 * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    acc[SLOT_WS] += double(u[i]) * double(s[i]);
  block_sum4<4>(acc, red);
  if (threadIdx.x == 0) {
    double* o = partials + (long long)blockIdx.x * 4;
    o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2]; o[3] = acc[3];
  }
}

// Relaxed labelling and label map: u* = w, label = first index of the largest entry.
__global__ __launch_bounds__(256) void k_epilogue(const float* __restrict__ w, int q, long long n2,
                                                  float* __restrict__ u_out, int32_t* __restrict__ labels) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n2) return;
  float best = w[i];
  int arg = 0;
  if (u_out) u_out[i] = best;
  for (int l = 1; l < q; ++l) {
    const float v = w[l * n2 + i];
    if (u_out) u_out[l * n2 + i] = v;
    if (v > best) { best = v; arg = l; }
  }
  if (labels) labels[i] = arg;
}

// ---------------------------------------------------------------- reductions
// Level 1: block b sums partial rows [b*per, min((b+1)*per, n)) in a fixed order.
__global__ __launch_bounds__(256) void k_reduce1(const double* __restrict__ parts, long long n, long long per,
                                                 double* __restrict__ out) {
  __shared__ double red[4 * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const long long b0 = blockIdx.x * per, b1 = min(b0 + per, n);
  for (long long r = b0 + threadIdx.x; r < b1; r += 256) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += parts[r * 4 + i];
  }
  block_sum4<4>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) out[blockIdx.x * 4 + i] = acc[i];
  }
}

// Level 2: one block; writes totals[0..3], the history row (r_primal, r_dual, r_combined,
// surrogate energy) and a non-finite flag in totals[4].  With hist_ctr the row is
// hist_row + 4 * (*hist_ctr) and the counter advances by one, so one launch sequence (a
// captured graph) serves every iteration of a solve.
__global__ __launch_bounds__(256) void k_reduce2(const double* __restrict__ in, int n, double* __restrict__ totals,
                                                 double* __restrict__ hist_row, double gamma, int* hist_ctr) {
  __shared__ double red[4 * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = threadIdx.x; r < n; r += 256) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += in[r * 4 + i];
  }
  block_sum4<4>(acc, red);
  if (threadIdx.x == 0) {
    const double dy2 = acc[SLOT_DY2], db2 = acc[SLOT_DB2];
    totals[0] = acc[0]; totals[1] = acc[1]; totals[2] = acc[2]; totals[3] = acc[3];
    const double comb = dy2 + db2;
    totals[4] = (isfinite(comb) && isfinite(acc[2]) && isfinite(acc[3])) ? 0.0 : 1.0;
    if (hist_row && hist_ctr) hist_row += 4LL * (*hist_ctr)++;
    if (hist_row) {
      hist_row[0] = sqrt(db2);
      hist_row[1] = sqrt(dy2) / gamma;
      hist_row[2] = comb;
      hist_row[3] = acc[SLOT_WS] + acc[SLOT_L1];
    }
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, long long n, uint32_t v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_copy_f64(const double* __restrict__ src, int n, double* __restrict__ dst) {
  if (int(threadIdx.x) < n) dst[threadIdx.x] = src[threadIdx.x];
}

}  // namespace shs
