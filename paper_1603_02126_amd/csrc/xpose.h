// In-register transpose of a 64 x 64 complex matrix held one row per lane of
// a wave64 (gfx950): on entry lane y holds v[k] = M[y][k], on exit lane k
// holds v[y] = M[y][k].
//
// Lane index and register index are both 6-bit numbers; transposing swaps
// them bit for bit, and the three swaps below commute:
//   bits 0..3  through a small LDS staging area, one group of 16 registers
//              at a time (a 16 x 16 transpose inside each group of 16
//              lanes; the registers of a group only exchange among
//              themselves, so no extra registers are needed);
//   bit 4      v_permlane16_swap between registers k and k + 16;
//   bit 5      v_permlane32_swap between registers k and k + 32.
// The staging area holds 64 x 17 complex values (a pitch of 17 keeps the
// stores and loads within two-way bank conflicts).
#pragma once
#include "fft_reg.h"

namespace epic {

constexpr int kXposePitch = 17;
constexpr int kXposeFloat2 = 64 * kXposePitch;   // staging area per wave, in float2

__device__ __forceinline__ void xpose_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void swap16(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

__device__ __forceinline__ void swap32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

__device__ __forceinline__ void transpose64(float2 (&v)[64], float2* T, int lane) {
  const int wbase = lane * kXposePitch;
  const int rbase = (lane & ~15) * kXposePitch + (lane & 15);
  static_for<0, 4>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    static_for<0, 16>([&](auto mc) { T[wbase + decltype(mc)::value] = v[16 * j + decltype(mc)::value]; });
    xpose_lds_sync();
    static_for<0, 16>([&](auto ic) {
      v[16 * j + decltype(ic)::value] = T[rbase + decltype(ic)::value * kXposePitch];
    });
    xpose_lds_sync();
  });
  static_for<0, 64>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr ((k & 16) == 0) {
      swap16(v[k].x, v[k + 16].x);
      swap16(v[k].y, v[k + 16].y);
    }
  });
  static_for<0, 32>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    swap32(v[k].x, v[k + 32].x);
    swap32(v[k].y, v[k + 32].y);
  });
}

}  // namespace epic
