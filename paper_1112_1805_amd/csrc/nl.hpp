// Nonlocal regulariser of Section 4: the NL-means neighbour graph (host, built once per
// image) and the primal-dual iteration for  <u, s> + lambda sum_i ||(D u)(i)|| + iota_C(u)
// with D the graph's difference operator (device kernels).
//
// Graph: for every pixel i in row-major order, with l its number of weights already set,
// pick k = min(m, 2m - l) eligible pixels j of smallest Gaussian-weighted patch distance
//   d(i, j) = sum_{t1, t2} G(t) sum_c (f_c(i + t) - f_c(j + t))^2
// in the search window, and set w(i, j) = w(j, i) = 1.  Eligible: j != i, not yet a
// neighbour of i, fewer than 2m weights; ties go to the smaller linear index; periodic
// boundary.  D has 2m blocks: block b row i = u(j_b(i)) - u(i) for the b-th neighbour of i
// (in the order the weights were set), zero if i has fewer neighbours.
#pragma once
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "kernels.hpp"

namespace shs {

// ---------------------------------------------------------------- host graph builder
struct NlGraphCfg {
  int n, channels, patch, window, m;
  double a;
};

// Patch distances of the pixels of row r to all window offsets: dist[k * n + c] =
// d(i, i + offs[k]) for i = (r, c).  `pad` is the image periodically padded by `ph`
// pixels on each side (channel-major, side n + 2 ph).  The sum runs over t1, t2, channel
// with one rounding per operation (no contraction), as the definition is written; the
// innermost loop runs along the row so that it vectorises.
#pragma clang fp contract(off)
inline void nl_distances_row(const NlGraphCfg& g, const std::vector<double>& pad, int ph,
                             const std::vector<double>& G, const std::vector<int2>& offs, int r, double* dist) {
  const int n = g.n, h = (g.patch - 1) / 2, K = int(offs.size()), W = n + 2 * ph;
  const size_t plane = size_t(W) * W;
  for (int k = 0; k < K; ++k) {
    const int o1 = offs[k].x, o2 = offs[k].y;
    double* acc = dist + size_t(k) * n;
    for (int c = 0; c < n; ++c) acc[c] = 0.0;
    for (int t1 = -h; t1 <= h; ++t1) {
      for (int t2 = -h; t2 <= h; ++t2) {
        const double gw = G[size_t(t1 + h) * g.patch + (t2 + h)];
        for (int ch = 0; ch < g.channels; ++ch) {
          const double* pa = pad.data() + ch * plane + size_t(r + t1 + ph) * W + (t2 + ph);
          const double* pb = pad.data() + ch * plane + size_t(r + o1 + t1 + ph) * W + (o2 + t2 + ph);
          for (int c = 0; c < n; ++c) {
            const double diff = pa[c] - pb[c];
            const double sq = diff * diff;
            const double term = gw * sq;
            acc[c] = acc[c] + term;
          }
        }
      }
    }
  }
}
#pragma clang fp contract(on)

// Builds the graph: nbr[b * n^2 + i] = b-th neighbour of i or -1; rev[b * n^2 + i] = the
// block b' with nbr[b' * n^2 + nbr[b * n^2 + i]] = i (or -1).  Returns the largest degree.
inline int nl_build_graph(const NlGraphCfg& g, const float* img, int32_t* nbr, int32_t* rev) {
  const int n = g.n, m = g.m, M2 = 2 * m, h = (g.patch - 1) / 2, rr = (g.window - 1) / 2;
  const size_t n2 = size_t(n) * n;
  // normalised Gaussian on the patch
  std::vector<double> G(size_t(g.patch) * g.patch);
  double gs = 0.0;
  for (int t1 = -h; t1 <= h; ++t1)
    for (int t2 = -h; t2 <= h; ++t2) {
      const double v = std::exp(-double(t1 * t1 + t2 * t2) / (2.0 * g.a * g.a));
      G[size_t(t1 + h) * g.patch + (t2 + h)] = v;
      gs += v;
    }
  for (double& v : G) v /= gs;
  std::vector<int2> offs;
  for (int o1 = -rr; o1 <= rr; ++o1)
    for (int o2 = -rr; o2 <= rr; ++o2)
      if (o1 != 0 || o2 != 0) offs.push_back(make_int2(o1, o2));
  const int K = int(offs.size());
  std::vector<std::vector<int>> nb(n2);
  for (auto& v : nb) v.reserve(M2);
  // periodic padding by ph = h + rr pixels so that no index wraps in the distance loop
  const int ph = h + rr, W = n + 2 * ph;
  std::vector<double> pad(size_t(g.channels) * W * W);
  for (int ch = 0; ch < g.channels; ++ch)
    for (int y = 0; y < W; ++y)
      for (int x = 0; x < W; ++x)
        pad[(size_t(ch) * W + y) * W + x] =
            double(img[(size_t(ch) * n + size_t(((y - ph) % n + n) % n)) * n + size_t(((x - ph) % n + n) % n)]);
  const int rows_per_chunk = std::max(1, std::min(n, int((size_t(64) << 20) / (size_t(n) * K * sizeof(double)))));
  std::vector<double> dist(size_t(rows_per_chunk) * n * K);
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  // Selection state: weights set per pixel, and per pixel a mask of the window offsets that
  // land on its current neighbours (those candidates are excluded).  The k smallest
  // (distance, index) pairs are kept in insertion order of that pair ordering.
  std::vector<int> deg(n2, 0);
  const int Wd = 2 * rr + 1, center = rr * Wd + rr;
  auto kidx = [&](int o1, int o2) { const int e = (o1 + rr) * Wd + (o2 + rr); return e > center ? e - 1 : e; };
  std::vector<uint64_t> excl((size_t(K) + 63) / 64);
  std::vector<double> bd(size_t(std::max(m, 1)));
  std::vector<int> bj(size_t(std::max(m, 1)));
  std::vector<int> rowb(Wd, 0), colw(Wd, 0);   // wrapped row offsets / columns in the window
  for (int r0 = 0; r0 < n; r0 += rows_per_chunk) {
    const int r1 = std::min(n, r0 + rows_per_chunk);
    // distances of this chunk of rows in parallel (row-interleaved over threads)
    std::vector<std::thread> pool;
    const int rows = r1 - r0;
    const unsigned nt = std::min<unsigned>(hw, unsigned(rows));
    for (unsigned t = 0; t < nt; ++t)
      pool.emplace_back([&, t]() {
        // a row's distances come out offset-major (vectorised along the row) and are stored
        // pixel-major, so that the selection reads each pixel's K candidates contiguously
        std::vector<double> tmp(size_t(n) * K);
        for (int r = r0 + int(t); r < r1; r += int(nt)) {
          nl_distances_row(g, pad, ph, G, offs, r, tmp.data());
          double* out = dist.data() + size_t(r - r0) * n * K;
          constexpr int B = 16;
          for (int c0 = 0; c0 < n; c0 += B)
            for (int k0 = 0; k0 < K; k0 += B)
              for (int c = c0; c < std::min(n, c0 + B); ++c)
                for (int kk = k0; kk < std::min(K, k0 + B); ++kk) out[size_t(c) * K + kk] = tmp[size_t(kk) * n + c];
        }
      });
    for (auto& th : pool) th.join();
    // the sequential selection over the chunk's pixels
    for (int r = r0; r < r1; ++r) {
      for (int o = -rr; o <= rr; ++o) rowb[size_t(o + rr)] = ((r + o) % n + n) % n * n;
      for (int c = 0; c < n; ++c) {
        const int i = r * n + c;
        const int k = std::min(m, M2 - deg[i]);
        if (k <= 0) continue;
        for (int o = -rr; o <= rr; ++o) colw[size_t(o + rr)] = ((c + o) % n + n) % n;
        // offsets landing on a current neighbour x of i (every o = x - i mod n in the window)
        std::fill(excl.begin(), excl.end(), uint64_t(0));
        for (const int x : nb[i]) {
          const int d1 = ((x / n - r) % n + n) % n, d2 = ((x % n - c) % n + n) % n;
          for (int o1 = d1 - n * ((d1 + rr) / n); o1 <= rr; o1 += n)
            for (int o2 = d2 - n * ((d2 + rr) / n); o2 <= rr; o2 += n)
              if (o1 != 0 || o2 != 0) {
                const int e = kidx(o1, o2);
                excl[size_t(e) >> 6] |= uint64_t(1) << (e & 63);
              }
        }
        const double* d = dist.data() + (size_t(r - r0) * n + c) * K;
        int nbest = 0;
        for (int kk = 0; kk < K; ++kk) {
          if ((excl[size_t(kk) >> 6] >> (kk & 63)) & 1) continue;
          const int j = rowb[size_t(offs[kk].x + rr)] + colw[size_t(offs[kk].y + rr)];
          if (j == i || deg[j] >= M2) continue;
          const double dv = d[kk];
          auto before = [&](int p) { return dv < bd[p] || (dv == bd[p] && j < bj[p]); };
          if (nbest == k && !before(k - 1)) continue;
          int pos = nbest < k ? nbest++ : k - 1;
          while (pos > 0 && before(pos - 1)) {
            bd[pos] = bd[pos - 1];
            bj[pos] = bj[pos - 1];
            --pos;
          }
          bd[pos] = dv;
          bj[pos] = j;
        }
        for (int t = 0; t < nbest; ++t) {
          nb[i].push_back(bj[t]);
          nb[bj[t]].push_back(i);
          ++deg[i];
          ++deg[bj[t]];
        }
      }
    }
  }
  int maxdeg = 0;
  for (size_t i = 0; i < n2; ++i) {
    maxdeg = std::max(maxdeg, int(nb[i].size()));
    for (int b = 0; b < M2; ++b) {
      nbr[size_t(b) * n2 + i] = b < int(nb[i].size()) ? nb[i][b] : -1;
      rev[size_t(b) * n2 + i] = -1;
      if (b < int(nb[i].size())) {
        const auto& o = nb[nb[i][b]];
        rev[size_t(b) * n2 + i] = int(std::find(o.begin(), o.end(), int(i)) - o.begin());
      }
    }
  }
  return maxdeg;
}

// ---------------------------------------------------------------- device iteration
constexpr int kNlMaxBlocks = 16;

struct NlParams {
  void* y;              // dual variable [q][M2][n^2] (storage type)
  float* u;             // primal u [q][n^2] (read, written)
  float* ubar;          // extrapolation [q][n^2] (read by the dual step, written by the primal step)
  const float* s;       // data term [q][n^2]
  const int32_t* nbr;   // [M2][n^2]
  const int32_t* rev;   // [M2][n^2]
  double* partials;     // [blocks][4]
  long long n2;
  int q, M2;
  float lambda, tau, sigma;
};

// y <- P_ball(y + sigma D ubar) per pixel over (label, block), radius lambda.  Partials:
// ||y' - y||^2 and lambda ||(D ubar)(i)||.  Two passes over the pixel's entries (norm,
// then scaled store) keep the register footprint independent of q * M2.
template <int ST, bool STATS>
__global__ __launch_bounds__(256) void k_nl_dual(NlParams p) {
  using S = Store<ST>;
  __shared__ double red[4 * 4];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < p.n2) {
    typename S::T* y = reinterpret_cast<typename S::T*>(p.y);
    int nj[kNlMaxBlocks];
#pragma unroll
    for (int b = 0; b < kNlMaxBlocks; ++b) nj[b] = b < p.M2 ? p.nbr[b * p.n2 + i] : -1;
    float nn = 0.f, kk = 0.f;
    for (int l = 0; l < p.q; ++l) {
      const float* ub = p.ubar + l * p.n2;
      const float ui = ub[i];
#pragma unroll
      for (int b = 0; b < kNlMaxBlocks; ++b) {
        if (b < p.M2) {
          const float z = nj[b] >= 0 ? ub[nj[b]] - ui : 0.f;
          const float v = fmaf(p.sigma, z, S::to_float(y[(l * p.M2 + b) * p.n2 + i]));
          nn = fmaf(v, v, nn);
          kk = fmaf(z, z, kk);
        }
      }
    }
    const float sc = nn > p.lambda * p.lambda ? p.lambda * rsqrtf(nn) : 1.f;
    float d2 = 0.f;
    for (int l = 0; l < p.q; ++l) {
      const float* ub = p.ubar + l * p.n2;
      const float ui = ub[i];
#pragma unroll
      for (int b = 0; b < kNlMaxBlocks; ++b) {
        if (b < p.M2) {
          const long long o = (l * p.M2 + b) * p.n2 + i;
          const float z = nj[b] >= 0 ? ub[nj[b]] - ui : 0.f;
          const float yo = S::to_float(y[o]);
          const float yn = S::round(fmaf(p.sigma, z, yo) * sc);
          y[o] = S::from_float(yn);
          d2 = fmaf(yn - yo, yn - yo, d2);
        }
      }
    }
    if constexpr (STATS) {
      acc[SLOT_DY2] = d2;
      acc[SLOT_L1] = double(p.lambda) * sqrt(double(kk));
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

// u' = P_C(u - tau (D^T y + s)), ubar = 2 u' - u, with
// (D^T y)(j) = sum_c [j has a c-th neighbour i] (y_{rev_c(j)}(i) - y_c(j)).
template <int ST, bool STATS>
__global__ __launch_bounds__(256) void k_nl_primal(NlParams p) {
  using S = Store<ST>;
  constexpr int MQ = 8;
  __shared__ double red[4 * 4];
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < p.n2) {
    const typename S::T* y = reinterpret_cast<const typename S::T*>(p.y);
    int ni[kNlMaxBlocks], rb[kNlMaxBlocks];
#pragma unroll
    for (int c = 0; c < kNlMaxBlocks; ++c) {
      ni[c] = c < p.M2 ? p.nbr[c * p.n2 + j] : -1;
      rb[c] = c < p.M2 ? p.rev[c * p.n2 + j] : 0;
    }
    float un[MQ], uo[MQ], sv[MQ];
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      un[l] = 0.f;
      if (l < p.q) {
        float kt = 0.f;
#pragma unroll
        for (int c = 0; c < kNlMaxBlocks; ++c) {
          if (ni[c] >= 0) {
            kt += S::to_float(y[(l * p.M2 + rb[c]) * p.n2 + ni[c]]) - S::to_float(y[(l * p.M2 + c) * p.n2 + j]);
          }
        }
        uo[l] = p.u[l * p.n2 + j];
        sv[l] = p.s[l * p.n2 + j];
        un[l] = uo[l] - p.tau * (kt + sv[l]);
      }
    }
    simplex_project<MQ>(un, p.q);
#pragma unroll
    for (int l = 0; l < MQ; ++l) {
      if (l < p.q) {
        const long long o = l * p.n2 + j;
        p.u[o] = un[l];
        p.ubar[o] = 2.f * un[l] - uo[l];
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

// Energy partials of u: <u, s> and lambda sum_i (sum_{l, b} (D_b u_l)(i)^2)^(1/2), FP64.
__global__ __launch_bounds__(256) void k_nl_energy(NlParams p) {
  __shared__ double red[4 * 4];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < p.n2) {
    double nn = 0.0;
    for (int l = 0; l < p.q; ++l) {
      const float* u = p.u + l * p.n2;
      const double ui = u[i];
      acc[SLOT_WS] += ui * double(p.s[l * p.n2 + i]);
      for (int b = 0; b < p.M2; ++b) {
        const int jb = p.nbr[b * p.n2 + i];
        if (jb >= 0) {
          const double d = double(u[jb]) - ui;
          nn += d * d;
        }
      }
    }
    acc[SLOT_L1] = double(p.lambda) * sqrt(nn);
  }
  block_sum4<4>(acc, red);
  if (threadIdx.x == 0) {
    double* o = p.partials + (long long)blockIdx.x * 4;
    o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2]; o[3] = acc[3];
  }
}

}  // namespace shs
