// Host-side check of the register FFTs that every imaging engine runs
// (fft_reg<N, S>, N = 8 ... 64, both signs; N = 64 is the FMA-folded split):
// each is compared with a direct double-precision DFT of the same input,
// X[k] = sum_n x[n] exp(S 2 pi i n k / N), over random and sparse inputs.
// Prints the worst error relative to max |X| per size and sign and exits
// nonzero if any exceeds 1e-6 (single precision, at most 6 radix levels).
#include "fft_reg.h"

#include <cmath>
#include <cstdio>
#include <random>

using namespace epic;

template <int N, int S>
static int check(std::mt19937& g) {
  std::normal_distribution<double> nd;
  double worst = 0.0;
  for (int trial = 0; trial < 500; ++trial) {
    float2 v[64];
    double xr[64], xi[64];
    for (int n = 0; n < N; ++n) {
      v[n] = make_float2(float(nd(g)), float(nd(g)));
      if (trial % 5 == 0 && n % 3 != 0) v[n] = make_float2(0.f, 0.f);   // sparse rows, as gridded apertures are
      xr[n] = v[n].x;
      xi[n] = v[n].y;
    }
    fft_reg<N, S>(v);
    double peak = 0.0, err = 0.0;
    for (int k = 0; k < N; ++k) {
      double sr = 0.0, si = 0.0;
      for (int n = 0; n < N; ++n) {
        const double ang = S * 2.0 * M_PI * double((n * k) % N) / double(N);
        sr += xr[n] * std::cos(ang) - xi[n] * std::sin(ang);
        si += xr[n] * std::sin(ang) + xi[n] * std::cos(ang);
      }
      peak = std::fmax(peak, std::hypot(sr, si));
      err = std::fmax(err, std::hypot(double(v[k].x) - sr, double(v[k].y) - si));
    }
    if (peak > 0.0) worst = std::fmax(worst, err / peak);
  }
  std::printf("N=%2d S=%+d worst |X - DFT| / max|DFT| = %.3e\n", N, S, worst);
  return worst <= 1e-6 ? 0 : 1;
}

int main() {
  std::mt19937 g(20160307);
  int bad = 0;
  bad |= check<8, 1>(g) | check<8, -1>(g);
  bad |= check<16, 1>(g) | check<16, -1>(g);
  bad |= check<32, 1>(g) | check<32, -1>(g);
  bad |= check<64, 1>(g) | check<64, -1>(g);
  std::printf(bad ? "FAIL\n" : "fft_reg check passed\n");
  return bad;
}
