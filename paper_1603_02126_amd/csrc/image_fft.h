// N <= 64 FFT imaging engine (work-item body), shared by the per-array kernel
// and the batched persistent kernel.
#pragma once
#include "engine.h"

namespace epic {

// LDS layout of the FFT engine: frame buffers, E' staging, slot table.
template <int N, int APL>
struct FftSmem {
  static constexpr int E_OFF = Geo<N>::LDS * 8;
  static constexpr int T_OFF = E_OFF + Geo<N>::SLOTS * APL * N * 8;
  static constexpr int BYTES = T_OFF + Budget<N, APL>::TAB_SLOTS * N * 8;
};

// One work item of the N <= 64 FFT engine: channel f, time split s.
template <int N, int APL>
__device__ __forceinline__ void image_item(const ImageArgs& a, int f, int s, uint8_t* smem) {
  using G = Geo<N>;
  float2* lds = reinterpret_cast<float2*>(smem);
  float2* lds_e = reinterpret_cast<float2*>(smem + FftSmem<N, APL>::E_OFF);
  uint2* stab = reinterpret_cast<uint2*>(smem + FftSmem<N, APL>::T_OFF);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane / N, lam = lane % N;
  const int slot = wave * G::FPW + h;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* buf = lds + slot * G::FRAME;
  float2* epr = lds_e + slot * (APL * N);

  load_slot_table(stab, a.slots, a.n_slots, N);
  static_for<0, N>([&](auto xc) { buf[lam * G::PITCH + decltype(xc)::value] = make_float2(0.f, 0.f); });
  __syncthreads();

  float acc[N];
  static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });

  const int64_t iters = (te - tb + G::SLOTS - 1) / G::SLOTS;
  Raw raw[APL];
  float2 uu[APL];
  {
    const int64_t t = tb + slot;
    fetch_frame<N, APL>(raw, uu, a.efield, a.u, t, a.t_cal, f, a.F, a.Na, a.fmt, lam, t < te);
  }
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + it * G::SLOTS + slot;
    stage_frame<N, APL>(epr, raw, uu, lam, a.Na, a.fmt, t < te);
    {
      const int64_t tn = t + G::SLOTS;
      fetch_frame<N, APL>(raw, uu, a.efield, a.u, tn, a.t_cal, f, a.F, a.Na, a.fmt, lam, tn < te);
    }
    wave_lds_sync();
    grid_frame(buf, epr, stab, a.n_slots, N, lam);
    wave_lds_sync();
    float2 v[N];
    transform_frame<N, +1>(buf, v, lam);
    static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] += cnorm(v[decltype(yc)::value]); });
  }

  // workgroup reduction of the SLOTS accumulators
  __syncthreads();
  float* red = reinterpret_cast<float*>(lds);
  static_for<0, N>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    red[(slot * N + y) * N + lam] = acc[y];
  });
  __syncthreads();
  float* out = a.partial + (int64_t(s) * a.F + f) * (N * N);
  for (int idx = threadIdx.x; idx < N * N; idx += 256) {
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < G::SLOTS; ++q) sum += red[q * N * N + idx];
    out[idx] = sum;
  }
  __syncthreads();
}

}  // namespace epic
