// Transpose of a 64 x 64 complex matrix held one row per lane of a wave64
// (gfx950): on entry lane y holds v[k] = M[y][k], on exit lane k holds
// v[y] = M[y][k].
//
// The matrix goes through an LDS staging area one component at a time: each
// lane stores its row of real parts (64 x 65 floats: the odd pitch puts both
// the row stores and the column loads of a wave on 64 distinct banks), loads
// its column, and the same for the imaginary parts.  The staging area is
// zero again on exit: the imaginary parts are loaded by LDS exchanges with
// zero (lds_take).  Exchanging the
// upper index bits with v_permlane16_swap / v_permlane32_swap instead, with
// LDS only for the low four bits, measured 9% slower on the 64 x 64 imaging
// kernel: a wave spent about ten SIMD cycles per swap.
#pragma once
#include "engine.h"

namespace epic {

constexpr int kXposePitch = 65;                      // floats
constexpr int kXposeFloat2 = (64 * kXposePitch + 1) / 2;   // staging area per wave, in float2

__device__ __forceinline__ void xpose_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void transpose64(float2 (&v)[64], float2* T, int lane) {
  float* F = reinterpret_cast<float*>(T);
  const int wbase = lane * kXposePitch;
  static_for<0, 64>([&](auto kc) { F[wbase + decltype(kc)::value] = v[decltype(kc)::value].x; });
  xpose_lds_sync();
  static_for<0, 64>([&](auto yc) { v[decltype(yc)::value].x = F[decltype(yc)::value * kXposePitch + lane]; });
  xpose_lds_sync();
  static_for<0, 64>([&](auto kc) { F[wbase + decltype(kc)::value] = v[decltype(kc)::value].y; });
  xpose_lds_sync();
  static_for<0, 64>([&](auto yc) { v[decltype(yc)::value].y = lds_take(F + decltype(yc)::value * kXposePitch + lane); });
}

}  // namespace epic
