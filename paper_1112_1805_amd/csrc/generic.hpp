// Row and column passes for image sizes that are not a power of two (N = 2^a * m with
// m's prime factors in {3, 5, 7, 11, 13, 17, 19, 23}), e.g. the 32 * {3..24} sizes of a
// batch of mixed images.  The data of a transform stays in LDS between stages; every stage
// of the mixed-radix Stockham FFT has a runtime radix from a small set, each with a
// compile-time butterfly: power-of-two radices use the register DFTs of fft.hpp, radix 9 a
// 3 x 3 split, odd primes the symmetric-pair form
//   X[k]   = a0 + sum_n (a_n + a_{P-n}) cos(2 pi n k/P) - i (a_n - a_{P-n}) sin(2 pi n k/P)
//   X[P-k] = a0 + sum_n (a_n + a_{P-n}) cos(2 pi n k/P) + i (a_n - a_{P-n}) sin(2 pi n k/P)
// (forward; the inverse swaps the signs of the sine terms).
#pragma once
#include "kernels.hpp"

namespace shs {

constexpr int kMaxStages = 10;
struct FftPlan {
  int L;                     // transform length
  int ns;                    // number of stages
  int radix[kMaxStages];     // product = L
  // Division by the stage stride Ns_s = radix[0] * ... * radix[s-1] without a divide:
  // x / Ns_s = (umulhi(x, mag[s]) + x) >> sh[s] for x < 2^21 (constants from the host).
  unsigned mag[kMaxStages];
  int sh[kMaxStages];
};

// ---------------------------------------------------------------- small DFTs
template <int P, bool INV>
__device__ __forceinline__ void dft_odd_prime(cpx (&a)[P]) {
  constexpr int H = (P - 1) / 2;
  cpx s[H], d[H];
  cpx sum = a[0];
  static_for<H>([&](auto i) {
    s[i] = a[i + 1] + a[P - 1 - i];
    d[i] = a[i + 1] - a[P - 1 - i];
    sum = sum + s[i];
  });
  const cpx a0 = a[0];
  a[0] = sum;
  static_for<H>([&](auto kk) {
    constexpr int k = kk + 1;
    cpx re = a0, im = cpx{0.f, 0.f};
    static_for<H>([&](auto i) {
      constexpr int n = i + 1;
      constexpr float c = float(cos2pi(n * k, P));
      constexpr float sn = float(sin2pi(n * k, P));
      re = cpx{fmaf(s[i].x, c, re.x), fmaf(s[i].y, c, re.y)};
      im = cpx{fmaf(d[i].x, sn, im.x), fmaf(d[i].y, sn, im.y)};
    });
    // forward: X[k] = re - i im, X[P-k] = re + i im
    const cpx t = INV ? mul_i(im) : mul_mi(im);
    a[k] = re + t;
    a[P - k] = re - t;
  });
}

template <int R, bool INV>
__device__ __forceinline__ void dft_any(cpx (&a)[R]) {
  if constexpr (R == 2 || R == 4 || R == 8 || R == 16) {
    RegDFT<R, INV>::run(a);
  } else if constexpr (R == 9) {
    reg_dft_split<9, 3, 3, INV>(a);
  } else {
    dft_odd_prime<R, INV>(a);
  }
}

// ---------------------------------------------------------------- one Stockham stage
// `items` = W interleaved transforms x (L / R) butterflies, spread over nthr threads.
// Element `pos` of transform c lives at buf[pos * W + c].
// sw: stage twiddles of the whole transform in thread read order, W_{Ns R}^{i k} at
// sw[i Ns + k - 1] (1 <= i < R, k < Ns) for the stage of stride Ns and radix R; the stages'
// ranges [Ns - 1, Ns R - 1) tile [0, L - 1), and consecutive butterflies read consecutive
// entries.
// TWL: sw is a copy of the table in LDS and every twiddle power is read from it (no
// products, no vector-memory loads); otherwise the power-of-two exponents are loaded from
// global memory and the others formed by products.
template <int R, bool INV, int W, bool TWL>
__device__ __forceinline__ void gstage(const float2* __restrict__ src, float2* __restrict__ dst, int L, int Ns,
                                       unsigned mag, int sh, int nthr, int tid, const float2* __restrict__ sw) {
  static_assert((W & (W - 1)) == 0, "strip width is a power of two");
  const int nb = L / R;
  const int items = nb * W;
  for (int it = tid; it < items; it += nthr) {
    const int c = it & (W - 1);
    const unsigned bf = unsigned(it) / W;
    const unsigned g = (__umulhi(bf, mag) + bf) >> sh;     // bf / Ns
    const int k = int(bf - g * unsigned(Ns));
    cpx a[R];
    static_for<R>([&](auto i) { a[i] = ld(src + (int(bf) + i * nb) * W + c); });
    if (Ns > 1) {
      // z^i with z = W_{Ns R}^k: the power-of-two exponents are loaded, the others are
      // products of two of them (fewer loads through the vector-memory data path)
      cpx w[R];
      if constexpr (TWL) {
        static_for<R>([&](auto i) {
          if constexpr (i > 0) w[i] = ld(sw + (i * Ns + k - 1));
        });
      } else {
        static_for<R>([&](auto i) {
          if constexpr (i > 0 && (i & (i - 1)) == 0) w[i] = ld(sw + (i * Ns + k - 1));
        });
        static_for<R>([&](auto i) {
          if constexpr (i > 0 && (i & (i - 1)) != 0) {
            constexpr int hi = 1 << (31 - __builtin_clz(unsigned(i)));
            w[i] = cmul(w[hi], w[i - hi]);
          }
        });
      }
      static_for<R - 1>([&](auto i1) {
        constexpr int i = i1 + 1;
        a[i] = INV ? cmulc(a[i], w[i]) : cmul(a[i], w[i]);
      });
    }
    dft_any<R, INV>(a);
    const int ob = int(g) * Ns * R + k;
    static_for<R>([&](auto i) { st(dst + (ob + i * Ns) * W + c, a[i]); });
  }
}

// Full transform: data in b0 (natural order) -> result (natural order) in the returned buffer.
template <bool INV, int SK, int W, bool TWL = false>
__device__ __forceinline__ float2* gfft(float2* b0, float2* b1, const FftPlan& pl, int nthr, int tid, const float2* __restrict__ sw) {
  float2* src = b0;
  float2* dst = b1;
  int Ns = 1;
  for (int s = 0; s < pl.ns; ++s) {
    const int r = pl.radix[s];
    const unsigned mg = pl.mag[s];
    const int sh = pl.sh[s];
    switch (r) {
      case 2: gstage<2, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 3: gstage<3, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 4: gstage<4, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 5: gstage<5, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 7: gstage<7, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 8: gstage<8, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 9: gstage<9, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 11: gstage<11, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 13: gstage<13, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 16: gstage<16, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 17: gstage<17, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 19: gstage<19, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      case 23: gstage<23, INV, W, TWL>(src, dst, pl.L, Ns, mg, sh, nthr, tid, sw); break;
      default: break;
    }
    fft_sync<SK>();
    float2* t = src;
    src = dst;
    dst = t;
    Ns *= r;
  }
  return src;
}

// ---------------------------------------------------------------- generic geometry
constexpr int kGW = 4;          // strip width of the generic path


struct GenParams {
  FftPlan prow;   // length N/2
  FftPlan pcol;   // length N
  int n;
  int wpb;        // waves per row-pass block (1, 2 or 4; the block is 64 wpb threads)
};
// Twiddle table of a mixed-radix plan, one device array: [0, N) exp(-2 pi i m / N), then
// the stage table of the row FFT (N/2 entries), then that of the column FFT (N entries).
__device__ __forceinline__ const float2* row_sw_g(const float2* tw, int n) { return tw + n; }
__device__ __forceinline__ const float2* col_sw_g(const float2* tw, int n) { return tw + n + n / 2; }

// The kernels below keep their twiddles in LDS, at the start of the dynamic shared memory
// (loaded once per block): the mixed-radix stages read one table entry per twiddle, where
// loads from global memory would compete with the data for the vector-memory path.
//   row pass:     exp(-2 pi i k / N) for k <= N/2, then the row FFT's stage table
//   column pass:  the column FFT's stage table (N - 1 entries, padded to N)
__host__ __device__ constexpr int row_tab_len(int n) { return n; }       // (N/2 + 1) + (N/2 - 1)
__host__ __device__ constexpr int col_tab_len(int n) { return n; }
__device__ __forceinline__ void load_table(float2* dst, const float2* __restrict__ src, int len) {
  for (int e = threadIdx.x; e < len; e += blockDim.x) dst[e] = src[e];
}

// ---------------------------------------------------------------- generic row pass
// Same modes and data contract as k_row.  Each wave transforms RW rows at once, stored
// interleaved in LDS (bin k of row c at k * RW + c, two half-length complex buffers per
// wave, dynamic shared memory), so that a stage's butterflies of all RW rows share the
// wave's lanes; memory phases walk one row at a time (coalesced along the row).  A block
// holds gp.wpb waves: more rows per wave fill the lanes in stages with few butterflies
// (a large radix), fewer waves per block keep such blocks within their LDS share.
__device__ __forceinline__ int tix_g(int ip, int row, int n) {
  return (ip >> 2) * (n * kGW) + row * kGW + (ip & (kGW - 1));     // floor for negative ip
}

template <int MODE, int ST, bool STATS, int RW>
__device__ __forceinline__ void row_g_body(const RowParams& p, const GenParams& gp, BlockId bid) {
  static_assert(kGW == 4, "tix_g assumes strips of 4 columns");
  using S = Store<ST>;
  extern __shared__ float2 gsm[];
  __shared__ double red[4 * 4];
  const int n = gp.n, M = n / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = (bid.x * gp.wpb + wave) * RW;
  const int ch = bid.y;
  const int j = ch % p.eta;
  float2* ltw = gsm;                 // exp(-2 pi i k / N), k <= M
  float2* lsw = gsm + M + 1;         // row FFT stage table
  load_table(ltw, p.tw, M + 1);
  load_table(lsw, row_sw_g(p.tw, n), M - 1);
  float2* b0 = gsm + row_tab_len(n) + wave * 2 * M * RW;
  float2* b1 = b0 + M * RW;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  float2* res = b0;
  __syncthreads();

  if constexpr (MODE == ROW_SOLVE || MODE == ROW_C2R || MODE == ROW_ENERGY || MODE == ROW_SHRINK || MODE == ROW_PD) {
    int cb, pitch;
    long long off;
    plane_geom(p.lin, ch % p.lin.nf, cb, pitch, off);
    const PlaneBuf B(p.spec_in + (ch / p.lin.nf) * p.lin.ls + off, pitch * n);
    for (int c = 0; c < RW; ++c) {
      const int row = row0 + c;
      for (int k = lane; k < M; k += 64) {
        // bins outside the plane's columns are out-of-range buffer loads: zero
        const cpx xp = B.load(tix_g(k - cb, row, n));
        const cpx xm = conj(B.load(tix_g(M - k - cb, row, n)));
        const cpx s = xp + xm, d = xp - xm;
        const cpx w = conj(ld(ltw + k));
        st(b0 + k * RW + c, s + mul_i(cmul(d, w)));
      }
    }
    fft_sync<SYNC_WAVE>();
    res = gfft<true, SYNC_WAVE, RW, true>(b0, b1, gp.prow, 64, lane, lsw);
  }
  if constexpr (MODE == ROW_C2R) {
    for (int c = 0; c < RW; ++c) {
      float* out = p.real_out + ch * p.real_cs + (long long)(row0 + c) * n;
      for (int k = lane; k < M; k += 64) *reinterpret_cast<float2*>(out + 2 * k) = res[k * RW + c];
    }
    return;
  }
  if constexpr (MODE == ROW_ENERGY) {
    for (int e = lane; e < M * RW; e += 64) acc[SLOT_L1] += fabsf(res[e].x) + fabsf(res[e].y);
  }
  if constexpr (MODE == ROW_R2C) {
    for (int c = 0; c < RW; ++c) {
      const float* in = p.real_in + ch * p.real_cs + (long long)(row0 + c) * n;
      for (int k = lane; k < M; k += 64) res[k * RW + c] = *reinterpret_cast<const float2*>(in + 2 * k);
    }
  }
  if constexpr (MODE == ROW_SOLVE || MODE == ROW_PRIME) {
    const float th = p.fw.thr[j];
    for (int c = 0; c < RW; ++c) {
      typename S::T* g = reinterpret_cast<typename S::T*>(p.g) + (long long)ch * n * n + (long long)(row0 + c) * n;
      for (int k = lane; k < M; k += 64) {
        float g0, g1;
        S::unpack(S::load_pair(g + 2 * k), g0, g1);
        const float b0v = clip(g0, th), b1v = clip(g1, th);
        float n0 = g0, n1 = g1;
        if constexpr (MODE == ROW_SOLVE) {
          const float2 cc = res[k * RW + c];
          n0 = b0v + cc.x;
          n1 = b1v + cc.y;
          S::store_pair(g + 2 * k, S::round2(n0, n1));
        }
        const float nb0 = clip(n0, th), nb1 = clip(n1, th);
        if constexpr (STATS && MODE == ROW_SOLVE) {
          const float dv0 = (n0 - nb0) - (g0 - b0v), dv1 = (n1 - nb1) - (g1 - b1v);
          const float db0 = nb0 - b0v, db1 = nb1 - b1v;
          acc[SLOT_DY2] = fmaf(dv0, dv0, acc[SLOT_DY2]);
          acc[SLOT_DY2] = fmaf(dv1, dv1, acc[SLOT_DY2]);
          acc[SLOT_DB2] = fmaf(db0, db0, acc[SLOT_DB2]);
          acc[SLOT_DB2] = fmaf(db1, db1, acc[SLOT_DB2]);
          acc[SLOT_L1] += fabsf(n0 - nb0);
          acc[SLOT_L1] += fabsf(n1 - nb1);
        }
        res[k * RW + c] = make_float2(n0 - 2.f * nb0, n1 - 2.f * nb1);
      }
    }
  }
  if constexpr (MODE == ROW_PD) {
    const float th = p.fw.thr[j];
    for (int c = 0; c < RW; ++c) {
      typename S::T* g = reinterpret_cast<typename S::T*>(p.g) + (long long)ch * n * n + (long long)(row0 + c) * n;
      for (int k = lane; k < M; k += 64) {
        float y0, y1;
        S::unpack(S::load_pair(g + 2 * k), y0, y1);
        const float2 cc = res[k * RW + c];
        float n0 = clip(fmaf(p.sigma, cc.x, y0), th);
        float n1 = clip(fmaf(p.sigma, cc.y, y1), th);
        S::store_pair(g + 2 * k, S::round2(n0, n1));
        if constexpr (STATS) {
          const float d0 = n0 - y0, d1 = n1 - y1;
          acc[SLOT_DY2] += d0 * d0 + d1 * d1;
          acc[SLOT_L1] += fabsf(cc.x) + fabsf(cc.y);
        }
        res[k * RW + c] = make_float2(n0, n1);
      }
    }
  }
  if constexpr (MODE == ROW_SHRINK) {
    const float th = p.fw.thr[j];
    for (int e = lane; e < M * RW; e += 64) {
      const float2 c = res[e];
      res[e] = make_float2(c.x - clip(c.x, th), c.y - clip(c.y, th));
    }
  }
  if constexpr (MODE == ROW_R2C || MODE == ROW_PRIME || MODE == ROW_SOLVE || MODE == ROW_SHRINK || MODE == ROW_PD) {
    bool emit = true;
    if constexpr (MODE == ROW_SOLVE) emit = p.emit != 0;
    if (emit) {
      fft_sync<SYNC_WAVE>();
      float2* other = res == b0 ? b1 : b0;
      float2* Y = gfft<false, SYNC_WAVE, RW, true>(res, other, gp.prow, 64, lane, lsw);
      int cb, pitch;
      long long off;
      plane_geom(p.lout, ch % p.lout.nf, cb, pitch, off);
      const PlaneBuf B(p.spec_out + (ch / p.lout.nf) * p.lout.ls + off, pitch * n);
      for (int c = 0; c < RW; ++c) {
        const int row = row0 + c;
        for (int k = lane; k <= M; k += 64) {
          // stores of bins outside the plane's columns are dropped (out-of-range buffer stores)
          const cpx yk = ld(Y + (k == M ? 0 : k) * RW + c);
          const cpx ym = conj(ld(Y + (k == 0 ? 0 : M - k) * RW + c));
          const cpx s = yk + ym, d = yk - ym;
          const cpx w = ld(ltw + k);
          B.store(tix_g(k - cb, row, n), (s - mul_i(cmul(d, w))) * 0.5f);
        }
      }
    }
  }
  if constexpr (STATS) {
    double dd[4] = {double(acc[0]), double(acc[1]), double(acc[2]), double(acc[3])};
    dd[SLOT_L1] *= double(p.fw.lam[j]);
    block_sum4_n(dd, red, gp.wpb);
    if (threadIdx.x == 0) {
      double* o = p.partials + ((long long)bid.y * bid.gx + bid.x) * 4;
      o[0] = dd[0]; o[1] = dd[1]; o[2] = dd[2]; o[3] = dd[3];
    }
  }
}

template <int MODE, int ST, bool STATS, int RW>
__global__ __launch_bounds__(256) void k_row_g(RowParams p, GenParams gp) {
  row_g_body<MODE, ST, STATS, RW>(p, gp, own_block());
}

// ---------------------------------------------------------------- generic column passes
// One strip (kGW columns) per block of 256 threads; a strip's N x kGW bins are one
// contiguous block in memory and in LDS (bin (k0, c) at k0 * kGW + c).
__device__ __forceinline__ float psi_at_rt(const ColParams& p, int4 win, int k0, int n) {
  int rel = k0 - win.x;
  if (rel < 0) rel += n;
  return rel < win.y ? p.psiw[win.z + rel] : 0.f;
}

// The item's filter windows and plane geometry in LDS (as stage_item of the fixed sizes).
__device__ __forceinline__ void stage_item_g(const ColParams& p, int4 it, int M, ItemStage<kGW>& st) {
  for (int e = threadIdx.x; e < it.z * kGW; e += 256) {
    const int i = e / kGW, cc = e % kGW;
    const int j = p.flist[it.y + i];
    const int k1 = it.x * kGW + cc;
    st.win[i][cc] = k1 <= M ? p.pwin[j * (M + 1) + k1] : make_int4(0, 0, 0, 0);
    if (cc == 0) st.geo[i] = p.tl.tab[j];
  }
}

__device__ __forceinline__ void colg_fwd_body(const ColParams& p, const GenParams& gp, BlockId bid) {
  extern __shared__ float2 gsm[];
  const int n = gp.n, E = n * kGW;
  float2* lsw = gsm;
  float2* b0 = gsm + col_tab_len(n);
  float2* b1 = b0 + E;
  load_table(lsw, col_sw_g(p.tw, n), n - 1);
  const long long strip = bid.y * (long long)n * p.P + (long long)bid.x * E;
  for (int e = threadIdx.x; e < E; e += 256) b0[e] = p.in[strip + e];
  __syncthreads();
  float2* r = gfft<false, SYNC_BLOCK, kGW, true>(b0, b1, gp.pcol, 256, threadIdx.x, lsw);
  const int M = n / 2;
  for (int e = threadIdx.x; e < E; e += 256)
    if (bid.x * kGW + (e % kGW) <= M) p.out[strip + e] = r[e];
}

__global__ __launch_bounds__(256) void k_colg_fwd(ColParams p, GenParams gp) {
  colg_fwd_body(p, gp, own_block());
}

__device__ __forceinline__ void colg_syn_body(const ColParams& p, const GenParams& gp, BlockId bid) {
  extern __shared__ float2 gsm[];
  const int n = gp.n, E = n * kGW, M = n / 2;
  float2* lsw = gsm;
  float2* bu = gsm + col_tab_len(n);
  float2* b0 = bu + E;
  float2* b1 = bu + 2 * E;
  __shared__ ItemStage<kGW> stg;
  const int4 it = p.items[bid.x];
  const int l = bid.y;
  load_table(lsw, col_sw_g(p.tw, n), n - 1);
  stage_item_g(p, it, M, stg);
  const float2* U = p.in + l * (long long)n * p.P + (long long)it.x * E;
  for (int e = threadIdx.x; e < E; e += 256) bu[e] = U[e];
  __syncthreads();
  for (int i = 0; i < it.z; ++i) {
    for (int e = threadIdx.x; e < E; e += 256) {
      const float f = psi_at_rt(p, stg.win[i][e % kGW], e / kGW, n);   // zero window past N/2
      b0[e] = make_float2(bu[e].x * f * p.inv_n2, bu[e].y * f * p.inv_n2);
    }
    __syncthreads();
    float2* r = gfft<true, SYNC_BLOCK, kGW, true>(b0, b1, gp.pcol, 256, threadIdx.x, lsw);
    const int4 geo = stg.geo[i];
    float2* o = p.out + l * p.tl.ls + geo_off(geo) + (long long)(it.x - geo.x / kGW) * E;
    for (int e = threadIdx.x; e < E; e += 256)
      if (it.x * kGW + (e % kGW) <= M) o[e] = r[e];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_colg_syn(ColParams p, GenParams gp) {
  colg_syn_body(p, gp, own_block());
}

__device__ __forceinline__ void colg_finish(const ColParams& p, const GenParams& gp, const float2* lsw, float2* acc,
                                            float2* b1, int strip, int l) {
  const int n = gp.n, E = n * kGW, M = n / 2;
  for (int e = threadIdx.x; e < E; e += 256) acc[e] = make_float2(acc[e].x * p.inv_n2, acc[e].y * p.inv_n2);
  __syncthreads();
  float2* r = gfft<true, SYNC_BLOCK, kGW, true>(acc, b1, gp.pcol, 256, threadIdx.x, lsw);
  float2* o = p.out + l * (long long)n * p.P + (long long)strip * E;
  for (int e = threadIdx.x; e < E; e += 256)
    if (strip * kGW + (e % kGW) <= M) o[e] = r[e];
}

__device__ __forceinline__ void colg_ana_body(const ColParams& p, const GenParams& gp, BlockId bid) {
  extern __shared__ float2 gsm[];
  const int n = gp.n, E = n * kGW, M = n / 2;
  float2* lsw = gsm;
  float2* ba = gsm + col_tab_len(n);
  float2* b0 = ba + E;
  float2* b1 = ba + 2 * E;
  __shared__ ItemStage<kGW> stg;
  const int4 it = p.items[bid.x];
  const int l = bid.y;
  load_table(lsw, col_sw_g(p.tw, n), n - 1);
  stage_item_g(p, it, M, stg);
  for (int e = threadIdx.x; e < E; e += 256) ba[e] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int i = 0; i < it.z; ++i) {
    const int4 geo = stg.geo[i];
    const float2* in = p.in + l * p.tl.ls + geo_off(geo) + (long long)(it.x - geo.x / kGW) * E;
    for (int e = threadIdx.x; e < E; e += 256) {
      const int k1 = it.x * kGW + (e % kGW);
      b0[e] = k1 <= M ? in[e] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    float2* r = gfft<false, SYNC_BLOCK, kGW, true>(b0, b1, gp.pcol, 256, threadIdx.x, lsw);
    for (int e = threadIdx.x; e < E; e += 256) {
      const float f = psi_at_rt(p, stg.win[i][e % kGW], e / kGW, n);   // zero window past N/2
      ba[e] = make_float2(ba[e].x + r[e].x * f, ba[e].y + r[e].y * f);
    }
    __syncthreads();
  }
  if (it.w < 0) {
    colg_finish(p, gp, lsw, ba, b1, it.x, l);
  } else {
    float2* o = p.part + ((long long)it.w * p.labels + l) * E;
    for (int e = threadIdx.x; e < E; e += 256) o[e] = ba[e];
  }
}

__global__ __launch_bounds__(256) void k_colg_ana(ColParams p, GenParams gp) {
  colg_ana_body(p, gp, own_block());
}

__device__ __forceinline__ void colg_final_body(const ColParams& p, const GenParams& gp, BlockId bid) {
  extern __shared__ float2 gsm[];
  const int n = gp.n, E = n * kGW;
  const int2 si = p.strips[bid.x];
  if (si.y <= 1) return;
  float2* lsw = gsm;
  float2* ba = gsm + col_tab_len(n);
  float2* b1 = ba + E;
  const int l = bid.y;
  load_table(lsw, col_sw_g(p.tw, n), n - 1);
  for (int e = threadIdx.x; e < E; e += 256) ba[e] = make_float2(0.f, 0.f);
  for (int i = 0; i < si.y; ++i) {
    const float2* in = p.part + ((long long)p.items[si.x + i].w * p.labels + l) * E;
    for (int e = threadIdx.x; e < E; e += 256) ba[e] = make_float2(ba[e].x + in[e].x, ba[e].y + in[e].y);
  }
  __syncthreads();
  colg_finish(p, gp, lsw, ba, b1, bid.x, l);
}

__global__ __launch_bounds__(256) void k_colg_final(ColParams p, GenParams gp) {
  colg_final_body(p, gp, own_block());
}

}  // namespace shs
