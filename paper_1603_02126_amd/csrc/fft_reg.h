// Register-resident radix-2/4/8 FFTs for gfx950 wavefronts.
//
// One lane owns one pencil of N <= 64 complex values (float2) and transforms
// it entirely in VGPRs: a two-level Cooley-Tukey split N = R1 * R2 with
// radix-2/4/8 butterflies and compile-time twiddles.  Every index is a
// compile-time constant (static_for), so the arrays live in registers and
// trivial twiddles (1, +-i, (+-1 +-i)/sqrt 2) cost no multiplies.
//
// Sign convention: fft_reg<N, S> computes X[k] = sum_n x[n] exp(S 2 pi i n k / N),
// natural order in and out, no normalisation.  The image transform of the
// paper (Sec. 2.1, MOFF summary equation) uses S = +1; its adjoint S = -1.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace epic {

template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// ---- compile-time trigonometry (Taylor series on a quadrant-reduced angle) --
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 24; ++k) {
    term *= -x * x / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 24; ++k) {
    term *= -x * x / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi m / n, reduced exactly to phi in [0, pi/2) by quadrant.
constexpr double cos2pi(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m) / n, r = 4 * m - q * n;
  const double phi = (kPi / 2) * double(r) / double(n);
  const double c = taylor_cos(phi), s = taylor_sin(phi);
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
constexpr double sin2pi(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m) / n, r = 4 * m - q * n;
  const double phi = (kPi / 2) * double(r) / double(n);
  const double c = taylor_cos(phi), s = taylor_sin(phi);
  return q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
}

constexpr float kInvSqrt2 = 0.70710678118654752440f;

// ---- complex helpers ------------------------------------------------------
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// acc[i] += |v[i]|^2 for i < M, as two fused multiply-adds into each
// accumulator (one instruction fewer per value than squaring into a sum)
template <int M, int A, int V>
__host__ __device__ __forceinline__ void add_norms(float (&acc)[A], const float2 (&v)[V]) {
  static_assert(M <= A && M <= V, "accumulators and values for every index");
  static_for<0, M>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    acc[i] = fmaf(v[i].y, v[i].y, fmaf(v[i].x, v[i].x, acc[i]));
  });
}

// multiply by S*i
template <int S>
__host__ __device__ __forceinline__ float2 mul_si(float2 a) {
  if constexpr (S > 0) return make_float2(-a.y, a.x);
  else return make_float2(a.y, -a.x);
}

// v * exp(S 2 pi i M / N), special-casing the multiples of 2 pi / 8
template <int M, int N, int S>
__host__ __device__ __forceinline__ float2 twiddle(float2 v) {
  constexpr int m = ((M % N) + N) % N;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (2 * m == N) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * m == N) {
    return mul_si<S>(v);
  } else if constexpr (4 * m == 3 * N) {
    return mul_si<-S>(v);
  } else if constexpr (8 * m == N) {  // (1 + S i) / sqrt2
    return make_float2((v.x - S * v.y) * kInvSqrt2, (v.y + S * v.x) * kInvSqrt2);
  } else if constexpr (8 * m == 3 * N) {  // (-1 + S i) / sqrt2
    return make_float2((-v.x - S * v.y) * kInvSqrt2, (S * v.x - v.y) * kInvSqrt2);
  } else if constexpr (8 * m == 5 * N) {  // -(1 + S i) / sqrt2
    return make_float2((S * v.y - v.x) * kInvSqrt2, (-v.y - S * v.x) * kInvSqrt2);
  } else if constexpr (8 * m == 7 * N) {  // (1 - S i) / sqrt2
    return make_float2((v.x + S * v.y) * kInvSqrt2, (v.y - S * v.x) * kInvSqrt2);
  } else {
    constexpr float c = float(cos2pi(m, N));
    constexpr float s = float(S * sin2pi(m, N));
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// ---- small DFTs, natural order in place -----------------------------------
template <int S>
__host__ __device__ __forceinline__ void dft2(float2* x) {
  const float2 a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <int S>
__host__ __device__ __forceinline__ void dft4(float2* x) {
  const float2 s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
  const float2 s13 = cadd(x[1], x[3]), d13 = mul_si<S>(csub(x[1], x[3]));
  x[0] = cadd(s02, s13);
  x[2] = csub(s02, s13);
  x[1] = cadd(d02, d13);
  x[3] = csub(d02, d13);
}

template <int S>
__host__ __device__ __forceinline__ void dft8(float2* x) {
  float2 e[4] = {x[0], x[2], x[4], x[6]};
  float2 o[4] = {x[1], x[3], x[5], x[7]};
  dft4<S>(e);
  dft4<S>(o);
  static_for<0, 4>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const float2 t = twiddle<k, 8, S>(o[k]);
    x[k] = cadd(e[k], t);
    x[k + 4] = csub(e[k], t);
  });
}

template <int R, int S>
__host__ __device__ __forceinline__ void dft_small(float2* x) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<S>(x);
  } else if constexpr (R == 4) {
    dft4<S>(x);
  } else if constexpr (R == 8) {
    dft8<S>(x);
  } else {
    static_assert(R == 8, "radix must be 1, 2, 4 or 8");
  }
}

template <int N>
struct FftSplit {
  static constexpr int R1 = (N >= 64) ? 8 : (N == 32) ? 4 : (N == 16) ? 4 : (N == 8) ? 8 : N;
  static constexpr int R2 = N / R1;
};

// ---- 64 points with the twiddles folded into fused multiply-adds ----------
// The split 64 = 8 x 8 of fft_reg below, with each inter-stage twiddle
// w = exp(i theta) written as sigma * (1 + i tau) (tau = tan theta, sigma =
// cos theta, where |cos theta| >= |sin theta|) or sigma * (kappa + i)
// (kappa = cot theta, sigma = sin theta, otherwise).  The first stage applies
// only the unit-diagonal factor (two FMAs instead of a complex multiply of
// four instructions); the scales sigma, all compile-time constants of
// magnitude in [1/sqrt 2, 1], are carried into the second stage's 8-point
// transforms as ratios in the FMAs that replace their additions (the
// scaled-twiddle method for fused multiply-add hardware of Linzer and Feig).
// Every ratio has a magnitude between 1/2 and 2; the input of index 0 of each
// second-stage transform is never twiddled, so its outputs carry no residual
// scale.
struct Tw {
  int kind;       // 0: sigma * p with p = z; 1: p = i z; 2: p = -i z; 3: tangent; 4: cotangent
  double sigma, t;
};
constexpr Tw tw64(int m) {
  m = ((m % 64) + 64) % 64;
  if (m == 0) return Tw{0, 1.0, 0.0};
  if (m == 32) return Tw{0, -1.0, 0.0};
  if (m == 16) return Tw{1, 1.0, 0.0};
  if (m == 48) return Tw{2, 1.0, 0.0};
  const double c = cos2pi(m, 64), s = sin2pi(m, 64);
  const double ac = c < 0 ? -c : c, as = s < 0 ? -s : s;
  if (ac >= as) return Tw{3, c, s / c};
  return Tw{4, s, c / s};
}

// p such that w * z = sigma * p for w = exp(2 pi i m / 64)
template <int M>
__host__ __device__ __forceinline__ float2 tw_unit(float2 z) {
  constexpr Tw w = tw64(M);
  if constexpr (w.kind == 0) {
    return z;
  } else if constexpr (w.kind == 1) {
    return make_float2(-z.y, z.x);
  } else if constexpr (w.kind == 2) {
    return make_float2(z.y, -z.x);
  } else if constexpr (w.kind == 3) {
    constexpr float t = float(w.t);
    return make_float2(fmaf(-t, z.y, z.x), fmaf(t, z.x, z.y));
  } else {
    constexpr float k = float(w.t);
    return make_float2(fmaf(k, z.x, -z.y), fmaf(k, z.y, z.x));
  }
}

// a + r * b and a - r * b
__host__ __device__ __forceinline__ void fma_pm(float2 a, float2 b, float r, float2& sum, float2& dif) {
  sum = make_float2(fmaf(r, b.x, a.x), fmaf(r, b.y, a.y));
  dif = make_float2(fmaf(-r, b.x, a.x), fmaf(-r, b.y, a.y));
}

template <int S>
__host__ __device__ __forceinline__ float2 si_mul(float2 a) {   // (S i) * a
  if constexpr (S > 0) return make_float2(-a.y, a.x);
  else return make_float2(a.y, -a.x);
}

template <int S>
__host__ __device__ __forceinline__ void fft64_scaled(float2* v) {
  float2 p[8][8];   // [n2][k1]: first-stage outputs times the unit-diagonal twiddle factor
  static_for<0, 8>([&](auto n2c) {
    constexpr int n2 = decltype(n2c)::value;
    float2 t[8];
    static_for<0, 8>([&](auto n1c) { t[decltype(n1c)::value] = v[8 * decltype(n1c)::value + n2]; });
    dft8<S>(t);
    static_for<0, 8>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      p[n2][k1] = tw_unit<S * n2 * k1>(t[k1]);
    });
  });
  static_for<0, 8>([&](auto k1c) {
    constexpr int k1 = decltype(k1c)::value;
    constexpr double sg[8] = {tw64(0).sigma,          tw64(S * 1 * k1).sigma, tw64(S * 2 * k1).sigma,
                              tw64(S * 3 * k1).sigma, tw64(S * 4 * k1).sigma, tw64(S * 5 * k1).sigma,
                              tw64(S * 6 * k1).sigma, tw64(S * 7 * k1).sigma};
    // level 1: pairs (a, a + 4), scale sg[a]
    float2 sp[4], dp[4];
    static_for<0, 4>([&](auto ac) {
      constexpr int a = decltype(ac)::value;
      fma_pm(p[a][k1], p[a + 4][k1], float(sg[a + 4] / sg[a]), sp[a], dp[a]);
    });
    // level 2: the even (0, 2; scale sg[0] = 1) and odd (1, 3; scale sg[1]) 4-point transforms
    float2 E[4], O[4];
    fma_pm(sp[0], sp[2], float(sg[2] / sg[0]), E[0], E[2]);
    fma_pm(dp[0], si_mul<S>(dp[2]), float(sg[2] / sg[0]), E[1], E[3]);
    fma_pm(sp[1], sp[3], float(sg[3] / sg[1]), O[0], O[2]);
    fma_pm(dp[1], si_mul<S>(dp[3]), float(sg[3] / sg[1]), O[1], O[3]);
    // level 3: X[k] = E[k] +- w8^(S k) sg[1] O[k]
    constexpr float r1 = float(sg[1] / sg[0]);
    constexpr float r1h = float(sg[1] / sg[0] * 0.70710678118654752440);
    float2 X[8];
    fma_pm(E[0], O[0], r1, X[0], X[4]);
    fma_pm(E[1], make_float2(O[1].x - S * O[1].y, O[1].y + S * O[1].x), r1h, X[1], X[5]);
    fma_pm(E[2], si_mul<S>(O[2]), r1, X[2], X[6]);
    fma_pm(E[3], make_float2(-O[3].x - S * O[3].y, S * O[3].x - O[3].y), r1h, X[3], X[7]);
    static_for<0, 8>([&](auto k2c) { v[k1 + 8 * decltype(k2c)::value] = X[decltype(k2c)::value]; });
  });
}

// In-register FFT of one pencil of N <= 64 values.
// N = R1 * R2, n = R2 n1 + n2, k = k1 + R1 k2:
//   X[k1 + R1 k2] = sum_n2 w_R2^(n2 k2) w_N^(n2 k1) [sum_n1 x[R2 n1 + n2] w_R1^(n1 k1)]
// (64 points: fft64_scaled, the same split with the twiddles in FMAs).
template <int N, int S>
__host__ __device__ __forceinline__ void fft_reg(float2* v) {
  if constexpr (N == 64) {
    fft64_scaled<S>(v);
  } else if constexpr (N <= 8) {
    dft_small<N, S>(v);
  } else {
    constexpr int R1 = FftSplit<N>::R1, R2 = FftSplit<N>::R2;
    float2 y[R2][R1];
    static_for<0, R2>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      float2 t[R1];
      static_for<0, R1>([&](auto n1c) { t[decltype(n1c)::value] = v[R2 * decltype(n1c)::value + n2]; });
      dft_small<R1, S>(t);
      static_for<0, R1>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        y[n2][k1] = twiddle<n2 * k1, N, S>(t[k1]);
      });
    });
    static_for<0, R1>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      float2 t[R2];
      static_for<0, R2>([&](auto n2c) { t[decltype(n2c)::value] = y[decltype(n2c)::value][k1]; });
      dft_small<R2, S>(t);
      static_for<0, R2>([&](auto k2c) { v[k1 + R1 * decltype(k2c)::value] = t[decltype(k2c)::value]; });
    });
  }
}

}  // namespace epic
