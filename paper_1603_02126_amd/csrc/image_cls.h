// Imaging of N = 64 R grids (R = 2, 4) by output residue classes (work-item
// body shared by the per-array kernels and the batched persistent kernel).
//
// With k = R m + c and j = 64 p + q (m, q < 64; c, p < R) the transform
// splits into R x R independent 64 x 64 transforms:
//   X(R m + c) = sum_q exp(+2 pi i q.m / 64) H_c(q),
//   H_c(q)    = sum_{j = q mod 64} G(j) exp(+2 pi i j.c / N)
// so class c is the 64 x 64 engine applied to the grid folded modulo 64 with
// the phase exp(+2 pi i j.c / N) on every contribution.  One wave owns one
// class; the four waves of a workgroup image four classes of the same frame
// from one shared E' staging area, and each class writes its own interleaved
// subset of the partial image.
// Slot code: antenna | qx << 12 | qy << 18 | px << 24 | py << 26 | valid << 30
//            | first << 31.
//
// Two variants: the slot table copied to LDS with a double-buffered staging
// area (Na <= 512, one barrier per frame), and the "big" variant for dense
// arrays (Na <= 2048) that reads the table from memory (L1/L2 resident, the
// same rows for the four waves) with a single staging buffer (two barriers
// per frame).
#pragma once
#include "engine.h"

namespace epic {

constexpr int kClsMaxAnt = 512;
constexpr int kClsMaxAntBig = 2048;
constexpr int kClsTabSlots =
    (kLdsBytes - 4 * Geo<64>::FRAME * 8 - 2 * kClsMaxAnt * 8 - 256 * 8) / (64 * 8);

template <int R, bool BIG>
struct ClsSmem {
  static constexpr int FRAMES = 4 * Geo<64>::FRAME * 8;
  static constexpr int E_OFF = FRAMES;
  static constexpr int E_BYTES = BIG ? kClsMaxAntBig * 8 : 2 * kClsMaxAnt * 8;
  static constexpr int TW_OFF = E_OFF + E_BYTES;
  static constexpr int T_OFF = TW_OFF + 64 * R * 8;
  static constexpr int BYTES = T_OFF + (BIG ? 0 : kClsTabSlots * 64 * 8);
};

// One work item: channel f, class group cg (four classes), time split s.
template <int R, bool BIG>
__device__ __forceinline__ void image_cls_item(const ImageArgs& a, int f, int cg, int s, uint8_t* smem) {
  constexpr int N = 64 * R;
  constexpr int MAXI = BIG ? kClsMaxAntBig / 256 : kClsMaxAnt / 256;   // antennas per thread
  using G = Geo<64>;
  using L = ClsSmem<R, BIG>;
  constexpr int P = G::PITCH;
  float2* lds = reinterpret_cast<float2*>(smem);
  float2* epr_base = reinterpret_cast<float2*>(smem + L::E_OFF);
  float2* tw = reinterpret_cast<float2*>(smem + L::TW_OFF);
  const uint2* stab = BIG ? a.slots : reinterpret_cast<const uint2*>(smem + L::T_OFF);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = cg * 4 + wave, cx = c % R, cy = c / R;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* buf = lds + wave * G::FRAME;

  if constexpr (!BIG) load_slot_table(reinterpret_cast<uint2*>(smem + L::T_OFF), a.slots, a.n_slots, 64);
  for (int k = tid; k < N; k += 256) {
    double sn, cs;
    sincospi(2.0 * double(k) / double(N), &sn, &cs);
    tw[k] = make_float2(float(cs), float(sn));
  }
  static_for<0, 64>([&](auto xc) { buf[lane * P + decltype(xc)::value] = make_float2(0.f, 0.f); });
  float acc[64];
  static_for<0, 64>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });

  Raw raw[MAXI];
  float2 uu[MAXI];
  auto fetch = [&](int64_t t, bool active) {
    const int bpe = a.fmt == kCF32 ? 8 : a.fmt == kCI8 ? 2 : 1;
    const uint8_t* row = a.efield + (t * a.F + f) * int64_t(a.Na) * bpe;
    const float2* urow = a.u + ((t / a.t_cal) * a.F + f) * int64_t(a.Na);
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
      const int an = tid + 256 * i;
      if (active && an < a.Na) {
        raw[i] = load_raw(row, an, a.fmt);
        uu[i] = urow[an];
      } else {
        raw[i] = Raw{0u, 0u};
        uu[i] = make_float2(0.f, 0.f);
      }
    }
  };
  fetch(tb, tb < te);
  __syncthreads();
  for (int64_t t = tb; t < te; ++t) {
    float2* epr = BIG ? epr_base : epr_base + ((t - tb) & 1) * kClsMaxAnt;
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
      const int an = tid + 256 * i;
      if (an < a.Na) epr[an] = cmul(unpack_raw(raw[i], a.fmt), uu[i]);
    }
    fetch(t + 1, t + 1 < te);
    __syncthreads();
    // grid class (cx, cy): owned sub-cells, each contribution phased by exp(+2 pi i j.c / N)
    float2 sum = make_float2(0.f, 0.f);
#pragma unroll 4
    for (int k = 0; k < a.n_slots; ++k) {
      const uint2 e = stab[k * 64 + lane];
      const uint32_t code = e.x;
      const int qx = (code >> 12) & 63, qy = (code >> 18) & 63;
      const int jx = qx + 64 * int((code >> 24) & 3), jy = qy + 64 * int((code >> 26) & 3);
      const float2 ph = tw[(jx * cx + jy * cy) & (N - 1)];
      const float w = __uint_as_float(e.y);
      const float2 ev = cmul(epr[code & kSlotAntMask], make_float2(w * ph.x, w * ph.y));
      const bool first = int(code) < 0;
      sum.x = first ? ev.x : sum.x + ev.x;
      sum.y = first ? ev.y : sum.y + ev.y;
      const int off = (code >> 30) & 1 ? qy * P + qx : 64;
      buf[off] = sum;
    }
    if constexpr (BIG) __syncthreads();   // the single staging buffer is rewritten next
    else wave_lds_sync();
    float2 v[64];
    transform_frame<64, +1>(buf, v, lane);
    static_for<0, 64>([&](auto yc) { acc[decltype(yc)::value] += cnorm(v[decltype(yc)::value]); });
  }
  // class pixels: (R ky + cy, R kx + cx) with kx = lane
  float* out = a.partial + (int64_t(s) * a.F + f) * (int64_t(N) * N);
  static_for<0, 64>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    out[(R * y + cy) * N + R * lane + cx] = acc[y];
  });
  __syncthreads();
}

}  // namespace epic
