// Device-side FFT building blocks for gfx950 (CDNA4, wave64).
//
// The shearlet transform of the paper (Section 2, eq. (wichtig) and the inverse
// paragraph) is realised by 2-D DFTs; here every 2-D DFT is a pass over rows and a
// pass over columns, and each 1-D DFT of length L is a Stockham auto-sort FFT run by
// T = L/R threads that each hold R points in registers:
//
//   stage 0   radix R,  reads positions t + r*T (natural order), no twiddle
//   [stage 1] radix RM, optional middle stage (RM divides R)
//   stage 2   radix R,  writes positions t + r*T (natural order)
//
// so a thread's input positions equal its output positions: a forward FFT, a
// pointwise product and an inverse FFT chain in registers without extra exchange.
// Between stages the points travel through LDS.  Inter-stage twiddles come from a table
// per FFT configuration, laid out in the order the threads read them (values
// exp(-2 pi i m / NT) computed in FP64 on the host, rounded to FP32); twiddles inside a
// register DFT are compile-time constants.
#pragma once
#include <hip/hip_runtime.h>
#include <utility>
#include <type_traits>

namespace shs {

// ---------------------------------------------------------------- complex helpers
struct cpx { float x, y; };
__device__ __forceinline__ cpx mk(float a, float b) { return cpx{a, b}; }
__device__ __forceinline__ cpx operator+(cpx a, cpx b) { return cpx{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cpx operator-(cpx a, cpx b) { return cpx{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cpx operator*(cpx a, float s) { return cpx{a.x * s, a.y * s}; }
__device__ __forceinline__ cpx cmul(cpx a, cpx b) {
  return cpx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cpx cmulc(cpx a, cpx b) {  // a * conj(b)
  return cpx{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ cpx conj(cpx a) { return cpx{a.x, -a.y}; }
__device__ __forceinline__ cpx mul_i(cpx a) { return cpx{-a.y, a.x}; }      //  i * a
__device__ __forceinline__ cpx mul_mi(cpx a) { return cpx{a.y, -a.x}; }     // -i * a
__device__ __forceinline__ cpx ld(const float2* p) { float2 v = *p; return cpx{v.x, v.y}; }
__device__ __forceinline__ void st(float2* p, cpx v) { *p = make_float2(v.x, v.y); }

// ---------------------------------------------------------------- compile-time loops
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------- constexpr trig
// cos / sin of 2*pi*e/n for integer e and power-of-two n, by octant reduction and a
// Taylor series on [0, pi/4] (evaluated by the compiler in double precision).
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) { term *= -x2 / double((2 * k) * (2 * k + 1)); sum += term; }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) { term *= -x2 / double((2 * k - 1) * (2 * k)); sum += term; }
  return sum;
}
// cos(2 pi f) for f in [0, 1)
constexpr double cos2pi_frac(double f) {
  if (f > 0.5) f = 1.0 - f;                        // cos(2pi f) = cos(2pi(1-f))
  double sgn = 1.0;
  if (f > 0.25) { f = 0.5 - f; sgn = -1.0; }       // cos(2pi f) = -cos(2pi(1/2-f))
  if (f > 0.125) return sgn * taylor_sin(2.0 * kPi * (0.25 - f));
  return sgn * taylor_cos(2.0 * kPi * f);
}
constexpr double cos2pi(int e, int n) {
  int m = ((e % n) + n) % n;
  return cos2pi_frac(double(m) / double(n));
}
constexpr double sin2pi(int e, int n) {  // sin(2pi e/n) = cos(2pi (e/n - 1/4))
  return cos2pi(4 * e - n, 4 * n);
}

// x * W_n^e with W_n = exp(-2 pi i / n) (forward) or its conjugate (inverse).
template <int E, int NN, bool INV>
__device__ __forceinline__ cpx twc(cpx x) {
  constexpr int e = ((E % NN) + NN) % NN;
  if constexpr (e == 0) {
    return x;
  } else if constexpr (4 * e == NN) {
    return INV ? mul_i(x) : mul_mi(x);
  } else if constexpr (2 * e == NN) {
    return cpx{-x.x, -x.y};
  } else if constexpr (4 * e == 3 * NN) {
    return INV ? mul_mi(x) : mul_i(x);
  } else {
    constexpr float c = float(cos2pi(e, NN));
    constexpr float s = float(INV ? sin2pi(e, NN) : -sin2pi(e, NN));
    return cpx{x.x * c - x.y * s, x.x * s + x.y * c};
  }
}

// ---------------------------------------------------------------- register DFTs
// In-place DFT of R points held in registers (natural order in and out), unnormalised,
// forward = exp(-2 pi i jk/R), inverse = exp(+2 pi i jk/R).
template <int R, bool INV> struct RegDFT {
  __device__ __forceinline__ static void run(cpx (&a)[R]);
};

// ---------------------------------------------------------------- twiddled butterflies
// A butterfly (p, q) -> (p + q w, p - q w) costs four FMAs for the sum (the product folded
// into the additions) and two for the difference, taken as 2 p - (p + q w): six
// instructions instead of the eight of a complex product followed by two complex
// additions (the FMA formulation of Linzer and Feig, IBM J. Res. Dev. 37(5), 1993).
// INV multiplies by conj(w).
template <bool INV>
__device__ __forceinline__ cpx mul_tw(cpx q, cpx w) { return INV ? cmulc(q, w) : cmul(q, w); }
template <bool INV>
__device__ __forceinline__ cpx fmac_tw(cpx p, cpx q, cpx w) {   // p + q w
  if constexpr (INV) return cpx{fmaf(q.x, w.x, fmaf(q.y, w.y, p.x)), fmaf(q.y, w.x, fmaf(-q.x, w.y, p.y))};
  else return cpx{fmaf(q.x, w.x, fmaf(-q.y, w.y, p.x)), fmaf(q.y, w.x, fmaf(q.x, w.y, p.y))};
}
__device__ __forceinline__ cpx twice_minus(cpx p, cpx s) {      // 2 p - s
  return cpx{fmaf(2.f, p.x, -s.x), fmaf(2.f, p.y, -s.y)};
}
template <bool INV>
__device__ __forceinline__ void bfly_tw(cpx& p, cpx& q, cpx w) {
  const cpx s = fmac_tw<INV>(p, q, w);
  q = twice_minus(p, s);
  p = s;
}
// The same with the compile-time twiddle W_NN^E; the multiples of a quarter turn need no
// product and keep the plain additions.
template <int E, int NN>
constexpr bool quarter_turn() {
  constexpr int e = ((E % NN) + NN) % NN;
  return e == 0 || 4 * e == NN || 2 * e == NN || 4 * e == 3 * NN;
}
template <int E, int NN, bool INV>
__device__ __forceinline__ void bfly_twc(cpx& p, cpx& q) {
  if constexpr (quarter_turn<E, NN>()) {
    const cpx u = twc<E, NN, INV>(q);
    q = p - u;
    p = p + u;
  } else {
    constexpr int e = ((E % NN) + NN) % NN;
    constexpr float c = float(cos2pi(e, NN));
    constexpr float sn = float(INV ? sin2pi(e, NN) : -sin2pi(e, NN));
    const cpx s = cpx{fmaf(q.x, c, fmaf(-q.y, sn, p.x)), fmaf(q.x, sn, fmaf(q.y, c, p.y))};
    q = twice_minus(p, s);
    p = s;
  }
}

// 4-point DFT (natural order) of x[j] * W_NN^{j K}: compile-time twiddles.
template <int NN, int K, bool INV>
__device__ __forceinline__ void dft4_twc(cpx (&z)[4]) {
  bfly_twc<2 * K, NN, INV>(z[0], z[2]);                 // s0, d0
  z[1] = twc<K, NN, INV>(z[1]);
  bfly_twc<3 * K, NN, INV>(z[1], z[3]);                 // s1, d1 before the quarter turn
  const cpx d1 = INV ? mul_i(z[3]) : mul_mi(z[3]);
  const cpx s0 = z[0], d0 = z[2], s1 = z[1];
  z[0] = s0 + s1;
  z[2] = s0 - s1;
  z[1] = d0 + d1;
  z[3] = d0 - d1;
}

// A-point DFT of z[j] * W_NN^{j K} (folded butterflies for A = 2 and 4).
template <int A, int NN, int K, bool INV>
__device__ __forceinline__ void dft_twc(cpx (&z)[A]) {
  if constexpr (A == 2) {
    bfly_twc<K, NN, INV>(z[0], z[1]);
  } else if constexpr (A == 4) {
    dft4_twc<NN, K, INV>(z);
  } else {
    static_for<A>([&](auto j) { z[j] = twc<int(j) * K, NN, INV>(z[j]); });
    RegDFT<A, INV>::run(z);
  }
}

// R = A * B split in registers (four-step): B-point DFTs over the A interleaved
// subsequences x[j + A m], then A-point DFTs across j of the outputs twiddled by W_R^{j k2}
// (the twiddles folded into the butterflies).
template <int R, int A, int B, bool INV>
__device__ __forceinline__ void reg_dft_split(cpx (&a)[R]) {
  cpx y[A][B];
  static_for<A>([&](auto j) {
    static_for<B>([&](auto m) { y[j][m] = a[j + A * m]; });
    RegDFT<B, INV>::run(y[j]);
  });
  static_for<B>([&](auto k2) {
    cpx z[A];
    static_for<A>([&](auto j) { z[j] = y[j][k2]; });
    dft_twc<A, R, int(k2), INV>(z);
    static_for<A>([&](auto k1) { a[k2 + B * k1] = z[k1]; });
  });
}

template <int R, bool INV>
__device__ __forceinline__ void RegDFT<R, INV>::run(cpx (&a)[R]) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    cpx t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  } else if constexpr (R == 3) {
    // X0 = a0 + s, X1,2 = a0 - s/2 -+ i (sqrt(3)/2) d  (forward), s = a1 + a2, d = a1 - a2
    constexpr float h = 0.86602540378443864676f;
    const cpx s = a[1] + a[2], d = a[1] - a[2];
    const cpx t = cpx{a[0].x - 0.5f * s.x, a[0].y - 0.5f * s.y};
    const cpx r = INV ? mul_i(d * h) : mul_mi(d * h);
    a[0] = a[0] + s;
    a[1] = t + r;
    a[2] = t - r;
  } else if constexpr (R == 4) {
    cpx s0 = a[0] + a[2], d0 = a[0] - a[2];
    cpx s1 = a[1] + a[3], d1 = a[1] - a[3];
    d1 = INV ? mul_i(d1) : mul_mi(d1);
    a[0] = s0 + s1;
    a[2] = s0 - s1;
    a[1] = d0 + d1;
    a[3] = d0 - d1;
  } else if constexpr (R == 8) {
    reg_dft_split<8, 2, 4, INV>(a);
  } else if constexpr (R == 16) {
    reg_dft_split<16, 4, 4, INV>(a);
  } else {
    static_assert(R == 32, "register DFT sizes 1..32");
    reg_dft_split<32, 4, 8, INV>(a);
  }
}

// R-point DFT (natural order) of a[0] and a[r] * w[r], r >= 1 (INV: conj(w[r])), with the
// runtime twiddles folded into the first butterfly layer.  TW0: a[0] is twiddled by w[0]
// as well.  Same split as RegDFT.
template <int R, bool INV, bool TW0 = false>
__device__ __forceinline__ void dft_tw(cpx (&a)[R], const cpx (&w)[R]) {
  if constexpr (R == 2) {
    if constexpr (TW0) a[0] = mul_tw<INV>(a[0], w[0]);
    bfly_tw<INV>(a[0], a[1], w[1]);
  } else if constexpr (R == 4) {
    if constexpr (TW0) a[0] = mul_tw<INV>(a[0], w[0]);
    bfly_tw<INV>(a[0], a[2], w[2]);                     // s0, d0
    a[1] = mul_tw<INV>(a[1], w[1]);
    bfly_tw<INV>(a[1], a[3], w[3]);                     // s1, d1 before the quarter turn
    const cpx d1 = INV ? mul_i(a[3]) : mul_mi(a[3]);
    const cpx s0 = a[0], d0 = a[2], s1 = a[1];
    a[0] = s0 + s1;
    a[2] = s0 - s1;
    a[1] = d0 + d1;
    a[3] = d0 - d1;
  } else {
    static_assert(R == 8 || R == 16 || R == 32, "twiddled register DFT sizes 2, 4, 8, 16, 32");
    constexpr int A = R == 8 ? 2 : 4, B = R / A;
    cpx y[A][B];
    static_for<A>([&](auto j) {
      cpx wj[B];
      static_for<B>([&](auto m) {
        y[j][m] = a[j + A * m];
        wj[m] = w[j + A * m];
      });
      dft_tw<B, INV, TW0 || (int(j) > 0)>(y[j], wj);
    });
    static_for<B>([&](auto k2) {
      cpx z[A];
      static_for<A>([&](auto j) { z[j] = y[j][k2]; });
      dft_twc<A, R, int(k2), INV>(z);
      static_for<A>([&](auto k1) { a[k2 + B * k1] = z[k1]; });
    });
  }
}

// An FFT of complex length L = R * R * RM (RM = 1 means two stages) is run by T = L / R
// threads; R and RM are chosen per use (row or column pass) by the caller.

enum SyncKind { SYNC_WAVE = 0, SYNC_BLOCK = 1 };

template <int SK>
__device__ __forceinline__ void fft_sync() {
  if constexpr (SK == SYNC_BLOCK) {
    __syncthreads();
  } else {
    // All lanes of one FFT live in one wavefront: order the LDS traffic of the wave.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// LDS addressing of one FFT's points.  `at<R>(q, rr)` is point q * R + rr (rr < R); the
// FFT stages below only use that form, with q = a per-thread base plus a compile-time
// constant, so every LDS access is one base register plus an immediate offset.
// Row style: points contiguous with one pad slot per R points.
template <int R>
struct RowAddr {
  float2* base;
  __device__ __forceinline__ float2* operator()(unsigned pos) const { return base + (pos + pos / R); }
  template <int RQ>
  __device__ __forceinline__ float2* at(int q, int rr) const {
    static_assert(RQ == R, "row addressing pads every R points");
    return base + (q * (R + 1) + rr);
  }
};
// Column style: W FFTs interleaved, point pos of FFT c at (pos + pos/R)*W + c.  The pad
// slot every R points keeps the first stage's writes (lane stride R points) off a single
// bank group: without it a stride of R*W*8 bytes, a multiple of the 256-byte bank width,
// sends every lane of a column to the same banks.
template <int W, int R>
struct ColAddr {
  float2* base;  // already offset by the column c
  __device__ __forceinline__ float2* operator()(unsigned pos) const { return base + (pos + pos / R) * W; }
  template <int RQ>
  __device__ __forceinline__ float2* at(int q, int rr) const {
    static_assert(RQ == R, "column addressing pads every R points");
    return base + (q * (R + 1) + rr) * W;
  }
};
// LDS points (per column) of a padded column FFT of length L with radix R.
template <int L, int R>
constexpr int col_lds_points() { return L + L / R; }

// The Q - 1 twiddles w[r] = z^r (1 <= r < Q, Q a power of two) of one butterfly: the
// powers z^1, z^2, z^4, z^8 are loaded (entry (r-1)*stride of `p`), the others are
// products of two of them (at most three roundings from the table values).  Loads go
// through the vector-memory data path, which the row pass keeps near saturation; the
// products cost a few FMAs each.
template <int Q>
__device__ __forceinline__ void pow2_twiddles(const float2* __restrict__ p, int stride, cpx (&w)[Q]) {
  w[0] = cpx{1.f, 0.f};
  static_for<Q>([&](auto r) {
    if constexpr (r > 0 && (r & (r - 1)) == 0) w[r] = ld(p + (r - 1) * stride);
  });
  static_for<Q>([&](auto r) {
    if constexpr (r > 0 && (r & (r - 1)) != 0) {
      constexpr int hi = 1 << (31 - __builtin_clz(unsigned(r)));
      w[r] = cmul(w[hi], w[r - hi]);
    }
  });
}

// The same Q - 1 twiddles read directly, entry (r-1)*stride each: used when the table
// sits in LDS, where a read costs no vector-memory bandwidth and no products are needed.
template <int Q>
__device__ __forceinline__ void all_twiddles(const float2* p, int stride, cpx (&w)[Q]) {
  w[0] = cpx{1.f, 0.f};
  static_for<Q>([&](auto r) {
    if constexpr (r > 0) w[r] = ld(p + (r - 1) * stride);
  });
}

// Inter-stage twiddles of one FFT configuration, stored in the order the threads read
// them so that the lanes of a wave load consecutive entries (a table indexed by the
// exponent r*t would be read with stride r and touch up to one cache line per lane):
//   last stage   sw[(r-1) T + t]              = W_L^{r t},       1 <= r < R, t < T
//   middle stage sw[(R-1) T + (r-1) R + tr]   = W_{R RM}^{r tr}, 1 <= r < RM, tr < R
// with W_n = exp(-2 pi i / n).  The values are those of the plan's table exp(-2 pi i m / NT)
// at m = exponent * NT / n, copied on the host.
template <int L, int R, int RM>
constexpr int stage_tw_size() { return (R - 1) * (L / R) + (RM - 1) * R; }

// The power-of-two rows of that table only (r = 1, 2, 4, ...), packed: last stage
// cw[log2(r) T + t], then middle stage cw[log2(R) T + log2(r) R + tr].  The other powers
// are products of two of them, as in pow2_twiddles.
constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
template <int L, int R, int RM>
constexpr int stage_tw_pow2_size() { return ilog2c(R) * (L / R) + ilog2c(RM) * R; }
// Copies the packed power-of-two rows of the stage table `sw` (global) into `cw` (LDS);
// threads tid = 0, nthr, 2 nthr, ... of the block share the copy.  The caller synchronises.
template <int L, int R, int RM>
__device__ __forceinline__ void load_stage_tw_pow2(float2* cw, const float2* __restrict__ sw, int tid, int nthr) {
  constexpr int T = L / R, LAST = ilog2c(R) * T;
  for (int e = tid; e < stage_tw_pow2_size<L, R, RM>(); e += nthr) {
    int src;
    if (e < LAST) {
      src = ((1 << (e / T)) - 1) * T + e % T;
    } else {
      const int e2 = e - LAST;
      src = (R - 1) * T + ((1 << (e2 / R)) - 1) * R + e2 % R;
    }
    cw[e] = sw[src];
  }
}
// Q - 1 twiddles from the packed rows (entry log2(r) * stride for r = 1, 2, 4, ...; the
// others products of two of them).
template <int Q>
__device__ __forceinline__ void pow2_twiddles_packed(const float2* p, int stride, cpx (&w)[Q]) {
  w[0] = cpx{1.f, 0.f};
  static_for<Q>([&](auto r) {
    if constexpr (r > 0 && (r & (r - 1)) == 0) w[r] = ld(p + ilog2c(r) * stride);
  });
  static_for<Q>([&](auto r) {
    if constexpr (r > 0 && (r & (r - 1)) != 0) {
      constexpr int hi = 1 << (31 - __builtin_clz(unsigned(r)));
      w[r] = cmul(w[hi], w[r - hi]);
    }
  });
}

// In-register/LDS Stockham FFT of length L.  On entry a[r] holds point t + r*T; on exit
// a[r] holds output bin t + r*T.  `sw` is the stage twiddle table of (L, R, RM) above.
// The caller must have synchronised any earlier reader of the LDS region before the call
// (the routine synchronises before its first LDS write).  TWL = 0: `sw` is the table in
// global memory (power-of-two powers loaded, the others formed by products); 1: `sw` points
// to a copy of the table in LDS and every power is read from it; 2: `sw` points to the
// packed power-of-two rows in LDS (load_stage_tw_pow2), the others formed by products.
template <int L, int R, int RM, bool INV, int SK, class Addr, int TWL = 0>
__device__ __forceinline__ void fft_run(cpx (&a)[R], const Addr& lds, int t, const float2* __restrict__ sw) {
  static_assert(R * R * RM == L && R % RM == 0, "FFT configuration");
  constexpr int T = L / R;                 // = R * RM
  const int tq = int(unsigned(t) / R);     // t = tq * R + tr
  const int tr = int(unsigned(t) % R);
  // stage 0: radix R, Ns = 1; point r of this thread goes to position t * R + r
  RegDFT<R, INV>::run(a);
  fft_sync<SK>();
  static_for<R>([&](auto r) { st(lds.template at<R>(t, r), a[r]); });
  fft_sync<SK>();
  if constexpr (RM > 1) {
    // middle stage: radix RM, Ns = R; this thread runs R/RM butterflies bf = t + u*T with
    // inputs bf + r*L/RM = (tq + u*RM + r*R) * R + tr and twiddle index k = bf mod R = tr
    constexpr int U = R / RM;
    cpx b[R];
    static_for<U>([&](auto u) {
      static_for<RM>([&](auto r) { b[u * RM + r] = ld(lds.template at<R>(tq + u * RM + r * R, tr)); });
    });
    fft_sync<SK>();
    cpx w[RM];
    if constexpr (TWL == 1) all_twiddles<RM>(sw + (R - 1) * T + tr, R, w);
    else if constexpr (TWL == 2) pow2_twiddles_packed<RM>(sw + ilog2c(R) * T + tr, R, w);
    else pow2_twiddles<RM>(sw + (R - 1) * T + tr, R, w);
    static_for<U>([&](auto u) {
      cpx c[RM];
      static_for<RM>([&](auto r) { c[r] = b[u * RM + r]; });
      dft_tw<RM, INV>(c, w);
      // outputs (bf / R) * R * RM + k + r * R = ((tq + u*RM) * RM + r) * R + tr
      static_for<RM>([&](auto r) { st(lds.template at<R>((tq + u * RM) * RM + r, tr), c[r]); });
    });
    fft_sync<SK>();
  }
  // last stage: radix R, Ns = L/R, butterfly bf = t; input t + r*T = (tq + r*RM) * R + tr
  cpx wl[R];
  if constexpr (TWL == 1) all_twiddles<R>(sw + t, T, wl);
  else if constexpr (TWL == 2) pow2_twiddles_packed<R>(sw + t, T, wl);
  else pow2_twiddles<R>(sw + t, T, wl);
  static_for<R>([&](auto r) { a[r] = ld(lds.template at<R>(tq + r * RM, tr)); });
  dft_tw<R, INV>(a, wl);
}

}  // namespace shs
