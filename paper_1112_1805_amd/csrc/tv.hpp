// TV comparison model of Section 4 (labels coupled per pixel), solved by the ADMM of
// Section 3 with the periodic forward-difference gradient in place of S:
//   u   = (I + grad^T grad)^{-1} [grad^T (v - b_v) + (w - b_w) - gamma s]
//   v   = shrink_{gamma lambda}(b_v + grad u)   (isotropic over the 2q-vector of a pixel)
//   w   = P_C(b_w + u),  b_v, b_w as in Section 3.
// The state keeps g = b_v + grad u ([q][2][N][N]) as for the shearlet model: with P the
// projection onto the ball of radius gamma lambda, v = g - P(g), b_v = P(g), and
// v - b_v = g - 2 P(g).  The u-step runs on the DFT: grad^T grad has the eigenvalues
// e(k0) + e(k1), e(k) = 4 sin^2(pi k / N).
#pragma once
#include "generic.hpp"

namespace shs {

constexpr int kTvMaxLabels = 8;

struct TvParams {
  const void* g;      // state g [q][2][N][N] (rhs: read)
  void* g_out;        // state g (update: read and written)
  float* w;           // [q][N^2]
  float* bw;          // [q][N^2]
  const float* s;     // [q][N^2]
  const float* u;     // u [q][N^2] (update: read)
  float* rhs;         // [q][N^2] (rhs: written)
  double* partials;   // [blocks][4]
  int n, q;
  float gamma, radius, lambda;   // radius = gamma * lambda
};

// Scale of the ball projection of a 2q-vector with squared norm nn: P(x) = x min(1, r/|x|).
__device__ __forceinline__ float ball_scale(float nn, float r) {
  return nn > r * r ? r * rsqrtf(nn) : 1.f;
}

template <int ST>
__device__ __forceinline__ void tv_load_pixel(const typename Store<ST>::T* g, long long n2, int q, long long o,
                                              float (&v)[2 * kTvMaxLabels], float& nn) {
  using S = Store<ST>;
  nn = 0.f;
#pragma unroll
  for (int k = 0; k < 2 * kTvMaxLabels; ++k) {
    v[k] = 0.f;
    if (k < 2 * q) {
      v[k] = S::to_float(g[k * n2 + o]);
      nn = fmaf(v[k], v[k], nn);
    }
  }
}

// rhs_l = grad^T d_l + (w - b_w)_l - gamma s_l with d = g - 2 P(g) per pixel:
// (grad^T d)(r, c) = d_0(r-1, c) - d_0(r, c) + d_1(r, c-1) - d_1(r, c)  (periodic).
template <int ST>
__global__ __launch_bounds__(256) void k_tv_rhs(TvParams p) {
  using S = Store<ST>;
  const long long n2 = (long long)p.n * p.n;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n2) return;
  const int r = int(i / p.n), c = int(i - (long long)r * p.n);
  const long long iu = (long long)(r == 0 ? p.n - 1 : r - 1) * p.n + c;   // (r-1, c)
  const long long il = (long long)r * p.n + (c == 0 ? p.n - 1 : c - 1);   // (r, c-1)
  const typename S::T* g = reinterpret_cast<const typename S::T*>(p.g);
  float x[2 * kTvMaxLabels], xu[2 * kTvMaxLabels], xl[2 * kTvMaxLabels];
  float nn, nu, nl;
  tv_load_pixel<ST>(g, n2, p.q, i, x, nn);
  tv_load_pixel<ST>(g, n2, p.q, iu, xu, nu);
  tv_load_pixel<ST>(g, n2, p.q, il, xl, nl);
  const float m = 1.f - 2.f * ball_scale(nn, p.radius);
  const float mu = 1.f - 2.f * ball_scale(nu, p.radius);
  const float ml = 1.f - 2.f * ball_scale(nl, p.radius);
#pragma unroll
  for (int l = 0; l < kTvMaxLabels; ++l) {
    if (l < p.q) {
      const long long o = l * n2 + i;
      const float div = (mu * xu[2 * l] - m * x[2 * l]) + (ml * xl[2 * l + 1] - m * x[2 * l + 1]);
      p.rhs[o] = div + (p.w[o] - p.bw[o]) - p.gamma * p.s[o];
    }
  }
}

// g <- P(g) + grad u (the v / b_v update), w = P_C(b_w + u), b_w += u - w, and the
// residual partials (||v' - v||^2 + ||w' - w||^2, ||b' - b||^2, <w', s>, lambda sum |v'|).
template <int ST, bool STATS>
__global__ __launch_bounds__(256) void k_tv_update(TvParams p) {
  using S = Store<ST>;
  constexpr int MQ = kTvMaxLabels;
  __shared__ double red[4 * 4];
  const long long n2 = (long long)p.n * p.n;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n2) {
    const int r = int(i / p.n), c = int(i - (long long)r * p.n);
    const long long id = (long long)(r == p.n - 1 ? 0 : r + 1) * p.n + c;   // (r+1, c)
    const long long ir = (long long)r * p.n + (c == p.n - 1 ? 0 : c + 1);   // (r, c+1)
    typename S::T* g = reinterpret_cast<typename S::T*>(p.g_out);
    float x[2 * MQ], nn;
    tv_load_pixel<ST>(g, n2, p.q, i, x, nn);
    const float b_old = ball_scale(nn, p.radius);
    float xn[2 * MQ], mm = 0.f;
    float gw[MQ], wn[MQ], wo[MQ], bo[MQ], sv[MQ];
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      gw[l] = 0.f;
      xn[2 * l] = xn[2 * l + 1] = 0.f;
      if (l < p.q) {
        const long long o = l * n2;
        const float uc = p.u[o + i];
        xn[2 * l] = S::round(fmaf(b_old, x[2 * l], p.u[o + id] - uc));
        xn[2 * l + 1] = S::round(fmaf(b_old, x[2 * l + 1], p.u[o + ir] - uc));
        mm = fmaf(xn[2 * l], xn[2 * l], fmaf(xn[2 * l + 1], xn[2 * l + 1], mm));
        g[(2 * l) * n2 + i] = S::from_float(xn[2 * l]);
        g[(2 * l + 1) * n2 + i] = S::from_float(xn[2 * l + 1]);
        wo[l] = p.w[o + i];
        bo[l] = p.bw[o + i];
        sv[l] = p.s[o + i];
        gw[l] = bo[l] + uc;
      }
      wn[l] = gw[l];
    }
    simplex_project<MQ>(wn, p.q);
    const float b_new = ball_scale(mm, p.radius);
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      if (l < p.q) {
        const long long o = l * n2 + i;
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
    if constexpr (STATS) {
      // v = (1 - b) x, b_v = b x, for the old and the new state vector
      double dv = 0.0, dbv = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * MQ; ++k) {
        if (k < 2 * p.q) {
          const float e1 = (1.f - b_new) * xn[k] - (1.f - b_old) * x[k];
          const float e2 = b_new * xn[k] - b_old * x[k];
          dv += double(e1) * e1;
          dbv += double(e2) * e2;
        }
      }
      acc[SLOT_DY2] += dv;
      acc[SLOT_DB2] += dbv;
      acc[SLOT_L1] += double(p.lambda) * double(1.f - b_new) * sqrt(double(mm));
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

// Exact energy partials of w: <w, s> and lambda sum_pixels (sum_l |grad w_l|^2)^(1/2).
__global__ __launch_bounds__(256) void k_tv_energy(TvParams p) {
  __shared__ double red[4 * 4];
  const long long n2 = (long long)p.n * p.n;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n2) {
    const int r = int(i / p.n), c = int(i - (long long)r * p.n);
    const long long id = (long long)(r == p.n - 1 ? 0 : r + 1) * p.n + c;
    const long long ir = (long long)r * p.n + (c == p.n - 1 ? 0 : c + 1);
    double nn = 0.0;
    for (int l = 0; l < p.q; ++l) {
      const long long o = l * n2;
      const double wc = p.w[o + i];
      const double d0 = double(p.w[o + id]) - wc, d1 = double(p.w[o + ir]) - wc;
      nn += d0 * d0 + d1 * d1;
      acc[SLOT_WS] += wc * double(p.s[o + i]);
    }
    acc[SLOT_L1] = double(p.lambda) * sqrt(nn);
  }
  block_sum4<4>(acc, red);
  if (threadIdx.x == 0) {
    double* o = p.partials + (long long)blockIdx.x * 4;
    o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2]; o[3] = acc[3];
  }
}

// u-step on the spectrum: Z = colIFFT( colFFT(V) / (N^2 (1 + e(k0) + e(k1))) ) for every
// column of q per-label half spectra (eig[k] = e(k), computed on the host in FP64).
template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_col_solve(
    ColParams p, const float* __restrict__ eig) {
  using G = ColCfg<N>;
  constexpr int R = G::R, T = G::T, W = G::W, M = N / 2;
  __shared__ float2 lds[col_lds_points<N, R>() * W];
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int k1 = blockIdx.x * W + c;
  const bool valid = k1 <= M;
  const int l = blockIdx.y;
  const ColAddr<W, R> A{lds + c};
  const long long strip = l * (long long)N * p.P + (long long)blockIdx.x * (N * W) + c;
  cpx a[R];
  static_for<R>([&](auto r) { a[r] = valid ? ld(p.in + strip + (t + r * T) * W) : cpx{0.f, 0.f}; });
  fft_run<N, R, G::RM, false, SYNC_BLOCK>(a, A, t, p.tw + col_sw_off<N>());
  const float e1 = valid ? eig[k1] : 0.f;
  static_for<R>([&](auto r) { a[r] = a[r] * (p.inv_n2 / (1.f + eig[t + r * T] + e1)); });
  fft_run<N, R, G::RM, true, SYNC_BLOCK>(a, A, t, p.tw + col_sw_off<N>());
  if (valid) {
    static_for<R>([&](auto r) { st(p.out + strip + (t + r * T) * W, a[r]); });
  }
}

__global__ __launch_bounds__(256) void k_colg_solve(ColParams p, GenParams gp, const float* __restrict__ eig) {
  extern __shared__ float2 gsm[];
  const int n = gp.n, E = n * kGW, M = n / 2;
  float2* b0 = gsm;
  float2* b1 = gsm + E;
  const long long strip = blockIdx.y * (long long)n * p.P + (long long)blockIdx.x * E;
  for (int e = threadIdx.x; e < E; e += 256) b0[e] = p.in[strip + e];
  __syncthreads();
  float2* r = gfft<false, SYNC_BLOCK, kGW>(b0, b1, gp.pcol, 256, threadIdx.x, col_sw_g(p.tw, gp.n));
  float2* o = r == b0 ? b1 : b0;
  for (int e = threadIdx.x; e < E; e += 256) {
    const int k1 = blockIdx.x * kGW + (e % kGW);
    const float m = k1 <= M ? p.inv_n2 / (1.f + eig[e / kGW] + eig[k1]) : 0.f;
    r[e] = make_float2(r[e].x * m, r[e].y * m);
  }
  __syncthreads();
  float2* z = gfft<true, SYNC_BLOCK, kGW>(r, o, gp.pcol, 256, threadIdx.x, col_sw_g(p.tw, gp.n));
  for (int e = threadIdx.x; e < E; e += 256)
    if (blockIdx.x * kGW + (e % kGW) <= M) p.out[strip + e] = z[e];
}

}  // namespace shs
