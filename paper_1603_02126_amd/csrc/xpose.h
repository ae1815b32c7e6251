// Transpose of a 64 x 64 complex matrix held one row per lane of a wave64
// (gfx950): on entry lane y holds v[k] = M[y][k], on exit lane k holds
// v[y] = M[y][k].
//
// The matrix goes through an LDS staging area one component at a time,
// element (y, k) at F[66 k + y]: each lane stores its row of real parts one
// value per column (the 64 lanes of one store hit 64 consecutive words), then
// loads its column as 32 pairs of consecutive rows (64-bit loads; the even
// pitch keeps them aligned, and the lanes of one load cover every bank twice);
// the same for the imaginary parts, which are loaded by 64-bit LDS exchanges
// with zero, so that the staging area is zero again on exit.  Exchanging the
// upper index bits with v_permlane16_swap / v_permlane32_swap instead, with
// LDS only for the low four bits, measured 9% slower on the 64 x 64 imaging
// kernel (a wave spent about ten SIMD cycles per swap); loading the columns one
// value at a time, 2% slower.
#pragma once
#include "engine.h"

namespace epic {

constexpr int kXposePitch = 66;                      // floats
constexpr int kXposeFloat2 = 64 * kXposePitch / 2;   // staging area per wave, in float2

__device__ __forceinline__ void xpose_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void transpose64(float2 (&v)[64], float2* T, int lane) {
  float* F = reinterpret_cast<float*>(T);
  static_for<0, 64>([&](auto kc) { F[decltype(kc)::value * kXposePitch + lane] = v[decltype(kc)::value].x; });
  xpose_lds_sync();
  const float2* C = reinterpret_cast<const float2*>(F + lane * kXposePitch);
  static_for<0, 32>([&](auto yc) {
    constexpr int y = 2 * decltype(yc)::value;
    const float2 p = C[y / 2];
    v[y].x = p.x;
    v[y + 1].x = p.y;
  });
  xpose_lds_sync();
  static_for<0, 64>([&](auto kc) { F[decltype(kc)::value * kXposePitch + lane] = v[decltype(kc)::value].y; });
  xpose_lds_sync();
  static_for<0, 32>([&](auto yc) {
    constexpr int y = 2 * decltype(yc)::value;
    const float2 p = lds_take(reinterpret_cast<float2*>(F + lane * kXposePitch + y));
    v[y].y = p.x;
    v[y + 1].y = p.y;
  });
}

}  // namespace epic
