// Host build of the register DFTs of the FFT engine (paper_1112_1805_amd/csrc/fft.hpp): the
// untwiddled DFTs and the DFTs with runtime twiddles folded into their butterflies, for
// every size the engine uses, forward and inverse, against a direct FP64 DFT of the same
// (twiddled) inputs.  Prints one line per case and exits non-zero if any case is off.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>

#include <hip/hip_runtime.h>
// The device synchronisation calls of fft.hpp are not used by the register DFTs.
static inline void __syncthreads() {}
static inline void __builtin_amdgcn_fence(int, const char*) {}
static inline void __builtin_amdgcn_wave_barrier() {}
#include "fft.hpp"

using namespace shs;

template <int R, bool INV, bool TW>
double worst(std::mt19937& g, int trials) {
  std::uniform_real_distribution<float> U(-1.f, 1.f);
  double out = 0.0;
  for (int n = 0; n < trials; ++n) {
    cpx a[R], w[R];
    std::complex<double> x[R];
    for (int r = 0; r < R; ++r) {
      a[r] = cpx{U(g), U(g)};
      const double ang = 3.141592653589793 * U(g);
      w[r] = cpx{float(std::cos(ang)), float(std::sin(ang))};
      const std::complex<double> wr(w[r].x, INV ? -w[r].y : w[r].y);
      x[r] = std::complex<double>(a[r].x, a[r].y) * ((TW && r > 0) ? wr : std::complex<double>(1.0));
    }
    if constexpr (TW) dft_tw<R, INV>(a, w);
    else RegDFT<R, INV>::run(a);
    double err = 0.0, nrm = 0.0;
    for (int k = 0; k < R; ++k) {
      std::complex<double> s = 0.0;
      for (int j = 0; j < R; ++j) s += x[j] * std::polar(1.0, (INV ? 2.0 : -2.0) * M_PI * j * k / R);
      err = std::max(err, std::abs(s - std::complex<double>(a[k].x, a[k].y)));
      nrm = std::max(nrm, std::abs(s));
    }
    out = std::max(out, err / nrm);
  }
  return out;
}

int main() {
  std::mt19937 g(12345);
  const double tol = 1e-6;   // FP32 register DFTs of at most 32 points
  int bad = 0;
  auto report = [&](const char* what, int R, bool inv, double e) {
    std::printf("%s R=%d %s max_rel_err=%.3e\n", what, R, inv ? "inverse" : "forward", e);
    if (!(e <= tol)) ++bad;
  };
#define CASE(R)                                                   \
  report("plain", R, false, worst<R, false, false>(g, 500));      \
  report("plain", R, true, worst<R, true, false>(g, 500));        \
  report("twiddled", R, false, worst<R, false, true>(g, 500));    \
  report("twiddled", R, true, worst<R, true, true>(g, 500));
  CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
  report("plain", 3, false, worst<3, false, false>(g, 500));
  report("plain", 3, true, worst<3, true, false>(g, 500));
  std::printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}
