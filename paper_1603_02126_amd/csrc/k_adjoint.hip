// HIP kernels (gfx950): adjoint of fixed-gain imaging with respect to the gains.
#include "engine.h"

namespace epic {

// ---------------------------------------------------------------------------
// Adjoint of fixed-gain imaging: gradient of a real loss with respect to the
// gains.  Per frame the forward transform is recomputed (no per-sample
// storage), multiplied by R = dL/dI, transformed back with the conjugate
// sign, degridded at each antenna's cells and correlated with the
// uncalibrated E-field:
//   partial_a += conj(E_a(t)) sum_k w_ak DFT-(R . DFT+(G_t))[cell_ak]
// The host-side reduction applies 2 conj(-1/g^2) / (T Na^2).
// ---------------------------------------------------------------------------
template <int N, int APL>
__global__ __launch_bounds__(256) void k_adjoint(AdjointArgs a) {
  using G = Geo<N>;
  constexpr int P = G::PITCH;
  __shared__ float2 lds[G::LDS];
  __shared__ float2 lds_e[G::SLOTS * APL * N];
  __shared__ uint2 stab[Budget<N, APL>::TAB_SLOTS * N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane / N, lam = lane % N;
  const int slot = wave * G::FPW + h;
  const int f = blockIdx.x % a.F;
  const int s = blockIdx.x / a.F;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* buf = lds + slot * G::FRAME;
  float2* epr = lds_e + slot * (APL * N);

  load_slot_table(stab, a.slots, a.n_slots, N);
  constexpr int K2 = 4;  // device cell tables are padded to four cells
  DegridTable<N, K2, APL> dg;
  dg.load(a.cell_ixy, a.cell_w, lam, a.Na);
  float r[N];
  static_for<0, N>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    r[y] = a.R[(int64_t(f) * N + y) * N + lam];
  });
  static_for<0, N>([&](auto xc) { buf[lam * P + decltype(xc)::value] = make_float2(0.f, 0.f); });
  __syncthreads();
  double2 du[APL];
  static_for<0, APL>([&](auto ic) { du[decltype(ic)::value] = make_double2(0.0, 0.0); });

  const int64_t iters = (te - tb + G::SLOTS - 1) / G::SLOTS;
  Raw raw[APL], rawc[APL];
  float2 uu[APL];
  {
    const int64_t t = tb + slot;
    fetch_frame<N, APL>(raw, uu, a.efield, a.u, t, kNoInterval, f, a.F, a.Na, a.fmt, lam, t < te);
  }
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + it * G::SLOTS + slot;
    const bool active = t < te;
    stage_frame<N, APL>(epr, raw, uu, lam, a.Na, a.fmt, active);
    static_for<0, APL>([&](auto ic) { rawc[decltype(ic)::value] = raw[decltype(ic)::value]; });
    {
      const int64_t tn = t + G::SLOTS;
      fetch_frame<N, APL>(raw, uu, a.efield, a.u, tn, kNoInterval, f, a.F, a.Na, a.fmt, lam, tn < te);
    }
    wave_lds_sync();
    grid_frame(buf, epr, stab, a.n_slots, N, lam);
    wave_lds_sync();
    float2 v[N];
    transform_frame<N, +1>(buf, v, lam);
    static_for<0, N>([&](auto yc) { v[decltype(yc)::value] = cscale(v[decltype(yc)::value], r[decltype(yc)::value]); });
    fft_reg<N, -1>(v);
    wave_lds_sync();
    static_for<0, N>([&](auto yc) { buf[decltype(yc)::value * P + lam] = v[decltype(yc)::value]; });
    wave_lds_sync();
    static_for<0, N>([&](auto xc) { v[decltype(xc)::value] = buf[lam * P + decltype(xc)::value]; });
    fft_reg<N, -1>(v);
    static_for<0, N>([&](auto xc) { buf[lam * P + decltype(xc)::value] = v[decltype(xc)::value]; });
    wave_lds_sync();
    static_for<0, APL>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if (active && lam + N * i < a.Na) {
        float2 gb = make_float2(0.f, 0.f);
        static_for<0, K2>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const float2 c = buf[dg.off[i][k]];
          gb.x = fmaf(dg.w[i][k], c.x, gb.x);
          gb.y = fmaf(dg.w[i][k], c.y, gb.y);
        });
        const float2 e = unpack_raw(rawc[i], a.fmt);
        // conj(e) * gb
        du[i].x += double(e.x * gb.x + e.y * gb.y);
        du[i].y += double(e.x * gb.y - e.y * gb.x);
      }
    });
    wave_lds_sync();
    static_for<0, N>([&](auto xc) { buf[lam * P + decltype(xc)::value] = make_float2(0.f, 0.f); });
  }
  __syncthreads();
  double2* red = reinterpret_cast<double2*>(lds);   // [SLOTS][APL*N]
  static_for<0, APL>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    red[slot * (APL * N) + lam + N * i] = du[i];
  });
  __syncthreads();
  for (int an = threadIdx.x; an < a.Na; an += 256) {
    double2 sum = make_double2(0.0, 0.0);
    for (int q = 0; q < G::SLOTS; ++q) {
      const double2 d = red[q * (APL * N) + an];
      sum.x += d.x;
      sum.y += d.y;
    }
    a.partial[(int64_t(s) * a.F + f) * a.Na + an] = sum;
  }
}

// dL/dg = 2 conj(-1/g^2) scale sum_s partial  (FP64)
__global__ __launch_bounds__(256) void k_adjoint_reduce(const double2* partial, int splits, int F, int Na,
                                                        const double2* gains, double scale, double2* out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t n = int64_t(F) * Na;
  if (i >= n) return;
  double2 sum = make_double2(0.0, 0.0);
  for (int k = 0; k < splits; ++k) {
    const double2 d = partial[int64_t(k) * n + i];
    sum.x += d.x;
    sum.y += d.y;
  }
  const double2 g = gains[i];
  const double2 g2 = zmul(g, g);
  const double2 m = zrecip(g2);                        // 1 / g^2
  const double2 c = make_double2(-m.x, m.y);          // conj(-1 / g^2)
  const double2 d = zmul(c, make_double2(sum.x * scale, sum.y * scale));
  out[i] = make_double2(2.0 * d.x, 2.0 * d.y);
}

// u = 1/g in FP32 (zero for flagged antennas).
__global__ __launch_bounds__(256) void k_recip(const double2* gains, const uint8_t* flag, int F, int Na, float2* u) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= int64_t(F) * Na) return;
  const double2 r = zrecip(gains[i]);
  u[i] = flag[i % Na] ? make_float2(0.f, 0.f) : make_float2(float(r.x), float(r.y));
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N, int APL>
struct LaunchAdjoint {
  static hipError_t run(const AdjointArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_adjoint<N, APL>), dim3(a.F * a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
  }
};
hipError_t launch_adjoint(int N, const AdjointArgs& a, hipStream_t s) {
  return dispatch_n<LaunchAdjoint>(N, a.Na, a, s);
}
hipError_t launch_adjoint_reduce(const double2* partial, int splits, int F, int Na, const double2* gains,
                                 double scale, double2* dL_dg, hipStream_t s) {
  const int64_t n = int64_t(F) * Na;
  hipLaunchKernelGGL(k_adjoint_reduce, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, partial, splits, F, Na,
                     gains, scale, dL_dg);
  return hipGetLastError();
}
hipError_t launch_recip(const double2* gains, const uint8_t* flag, int F, int Na, float2* u, hipStream_t s) {
  const int64_t n = int64_t(F) * Na;
  hipLaunchKernelGGL(k_recip, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, gains, flag, F, Na, u);
  return hipGetLastError();
}


}  // namespace epic
