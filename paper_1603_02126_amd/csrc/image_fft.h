// N <= 64 FFT imaging engine (work-item body), shared by the per-array kernel
// and the batched persistent kernel.
#pragma once
#include "engine.h"
#include "xpose.h"

namespace epic {

// LDS layout of the FFT engine with W waves: frame buffers, E' staging, slot table.
template <int N, int APL, int W = 4>
struct FftSmem {
  static constexpr int E_OFF = Geo<N, W>::LDS * 8;
  static constexpr int T_OFF = E_OFF + Geo<N, W>::SLOTS * APL * N * 8;
  static constexpr int BYTES = T_OFF + Budget<N, APL, W>::TAB_SLOTS * N * 8;
};

// One work item of the N <= 64 FFT engine: channel f, time split s; W waves
// (4 in its own kernel; 8, two per SIMD, in the persistent batched kernel,
// for N <= 32 where eight waves' frame buffers fit).
template <int N, int APL, int W = 4>
__device__ __forceinline__ void image_item(const ImageArgs& a, int f, int s, uint8_t* smem) {
  using G = Geo<N, W>;
  float2* lds = reinterpret_cast<float2*>(smem);
  float2* lds_e = reinterpret_cast<float2*>(smem + FftSmem<N, APL, W>::E_OFF);
  uint2* stab = reinterpret_cast<uint2*>(smem + FftSmem<N, APL, W>::T_OFF);
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
    add_norms<N>(acc, v);
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
  for (int idx = threadIdx.x; idx < N * N; idx += 64 * W) {
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < G::SLOTS; ++q) sum += red[q * N * N + idx];
    gstore(out + idx, sum);
  }
  __syncthreads();
}

}  // namespace epic

namespace epic {

// ---------------------------------------------------------------------------
// 64 x 64 engine with two waves per SIMD ("paired" engine).
//
// A wave64 issues a VALU instruction at most every other cycle of its SIMD's
// FP32 pipeline, so the pipeline only runs at full rate with two waves
// computing at the same time.  The one-wave engine above needs a 33 KB frame
// buffer per wave, which leaves room for one wave per SIMD; here each of the
// eight waves of a workgroup (two per SIMD) images its own frames with 19 KB:
//   * gridding goes through half a frame (32 columns): the columns 0..31 are
//     gridded, then every lane loads the half of its row y = lane and clears
//     it; then the columns 32..63 (two schedules, built on the host);
//   * after the row FFTs the frame is transposed (xpose.h) through the same
//     half buffer, one component at a time, which leaves it zero;
//   * column FFTs and |X|^2 accumulation as in the one-wave engine.
// Waves never wait for each other inside the frame loop.  Integer E-field
// formats (ci4, ci8) with 129..256 antennas (four per lane).
// ---------------------------------------------------------------------------
constexpr int kPairThreads = 512;

template <int APL>
struct PairSmem {
  static constexpr int HALF = 64 * kHalfPitch;            // float2: half frame
  static constexpr int WAVE = HALF + APL * 64;            // float2 per wave: half frame + E' staging
  static constexpr int T_OFF = 8 * WAVE * 8;              // bytes: slot table
  static constexpr int TAB_SLOTS = (kLdsBytes - T_OFF) / (64 * 8);
  static constexpr int BYTES = T_OFF + TAB_SLOTS * 64 * 8;
  static_assert(HALF >= kXposeFloat2, "the transpose staging reuses the half frame");
  static_assert(8 * 64 * 64 * 4 <= T_OFF, "the accumulator reduction reuses the wave areas");
};

// The eight waves' share of the frames [tb, te) of channel f: wave w images
// tb + w, tb + w + 8, ... and adds |X|^2 into acc (lane = kx, acc[y] = ky).
// The wave's half frame is zero on entry and on exit.
template <int APL, int FMT>
__device__ __forceinline__ void pair_frames(const ImageArgs& a, int f, int64_t tb, int64_t te, float (&acc)[64],
                                            float2* H, float2* epr, const uint2* stab, int lam, int wave) {
  static_assert(FMT == kCI4 || FMT == kCI8, "integer E-field formats");
  constexpr int N = 64, INFLIGHT = 8;
  const int S0 = a.n_slots_h0, S1 = a.n_slots_h1;
  float2 v[N];
  uint32_t raw[APL];   // integer formats only: one packed sample per register
  const int64_t iters = (te - tb + INFLIGHT - 1) / INFLIGHT;
  constexpr int bpe = FMT == kCI4 ? 1 : 2;
  // the packed samples of a frame are requested at the end of the previous
  // frame; u (constant over an interval, cache resident) is loaded when the
  // frame is staged
  auto fetch_raw = [&](int64_t t) {
    const uint8_t* row = a.efield + (t * a.F + f) * int64_t(a.Na) * bpe;
    static_for<0, APL>([&](auto ic) {
      const int an = lam + N * decltype(ic)::value;
      raw[decltype(ic)::value] = (t < te && an < a.Na) ? load_raw_global(row, an, FMT).x : 0u;
    });
  };
  fetch_raw(tb + wave);
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + it * INFLIGHT + wave;
    // the LDS-bound phases of staging and gridding run at a raised wave
    // priority so that they advance while the other wave of the SIMD is in an
    // FFT (raising it for the transpose as well measured slower)
    __builtin_amdgcn_s_setprio(1);
    // calibrate: all u loads are issued before any is used (one memory
    // latency per frame)
    const float2* urow = a.u + (((t < te ? t : tb) / a.t_cal) * a.F + f) * int64_t(a.Na);
    float2 uu[APL];
    static_for<0, APL>([&](auto ic) {
      const int an = lam + N * decltype(ic)::value;
      uu[decltype(ic)::value] = gload(urow + (an < a.Na ? an : a.Na - 1));
    });
    static_for<0, APL>([&](auto ic) {
      const int an = lam + N * decltype(ic)::value;
      if (an < a.Na) epr[an] = t < te ? cmul(unpack_raw(Raw{raw[decltype(ic)::value], 0u}, FMT),
                                             uu[decltype(ic)::value])
                                      : make_float2(0.f, 0.f);
    });
    wave_lds_sync();
    // columns 0..31: grid, every lane loads its row's half and clears it
    grid_frame_fit(H, epr, stab, S0, N, lam);
    wave_lds_sync();
    take_half_row<0>(v, H, lam);
    wave_lds_sync();
    // columns 32..63
    grid_frame_fit(H, epr, stab + S0 * N, S1, N, lam);
    wave_lds_sync();
    take_half_row<32>(v, H, lam);
    wave_lds_sync();
    __builtin_amdgcn_s_setprio(0);
    fft_reg<N, +1>(v);            // along x: lane = row y
    transpose64(v, H, lam);       // lane = column kx (normal priority: measured faster)
    fft_reg<N, +1>(v);            // along y
    // the next frame's samples are requested here rather than at staging:
    // their registers would otherwise stay live through both FFTs
    fetch_raw(t + INFLIGHT);
    add_norms<N>(acc, v);
  }
}

// Workgroup sum of the eight waves' accumulators, times `scale`, into
// out[64 * 64] (row-major ky, kx); the accumulators are zeroed.  The sums go
// through the wave areas, whose half frames are cleared again afterwards.
template <int APL>
__device__ __forceinline__ void pair_reduce(float (&acc)[64], float* out, float scale, uint8_t* smem, int lam,
                                            int wave) {
  constexpr int N = 64;
  __syncthreads();
  float* red = reinterpret_cast<float*>(smem);
  static_for<0, N>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    red[(wave * N + y) * N + lam] = acc[y];
    acc[y] = 0.f;
  });
  __syncthreads();
  for (int idx = threadIdx.x; idx < N * N; idx += kPairThreads) {
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) sum += red[q * N * N + idx];
    gstore(out + idx, sum * scale);
  }
  __syncthreads();
  clear_half_row(reinterpret_cast<float2*>(smem) + wave * PairSmem<APL>::WAVE, lam);
}

template <int APL, int FMT>
__device__ __forceinline__ void image_item_pair(const ImageArgs& a, int f, int s, uint8_t* smem) {
  using L = PairSmem<APL>;
  const int lam = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float2* H = reinterpret_cast<float2*>(smem) + wave * L::WAVE;
  uint2* stab = reinterpret_cast<uint2*>(smem + L::T_OFF);
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;

  load_slot_table(stab, a.slots_h, a.n_slots_h0 + a.n_slots_h1, 64);
  clear_half_row(H, lam);
  __syncthreads();
  float acc[64];
  static_for<0, 64>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });
  pair_frames<APL, FMT>(a, f, tb, te, acc, H, H + L::HALF, stab, lam, wave);
  pair_reduce<APL>(acc, a.partial + (int64_t(s) * a.F + f) * (64 * 64), 1.f, smem, lam, wave);
  __syncthreads();
}

}  // namespace epic

namespace epic {

// ---------------------------------------------------------------------------
// Snapshot forms of the two N <= 64 engines: one image per window of t_acc
// consecutive samples (the short-timescale images of transient science)
// instead of the average over the run.  The windows of a channel are split
// over the workgroups; each frame slot (a lane group of the one-wave engine,
// a wave of the paired engine) takes whole windows in turn, accumulates their
// frames in registers and stores the window's image itself: no reduction
// between slots, no atomics, and every store writes a row of N contiguous
// pixels.  Long windows would leave most of the paired engine's waves idle
// (a channel split has few of them); there its eight waves share each
// window and sum it through LDS.
// ---------------------------------------------------------------------------

// Walks one slot's frames: windows j = j0, j0 + stride, ... below j_end
// (j_end <= the number of windows), the samples of each window in order (the
// last window of the run may be short).  `valid`: the cursor is on a sample;
// `last`: that sample ends its window.
struct SnapCursor {
  int64_t j, i, j_end, stride, t_acc, n_t;
  __device__ __forceinline__ int64_t t() const { return j * t_acc + i; }
  __device__ __forceinline__ int64_t len() const { return min(t_acc, n_t - j * t_acc); }
  __device__ __forceinline__ bool valid() const { return j < j_end; }
  __device__ __forceinline__ bool last() const { return i == len() - 1; }
  __device__ __forceinline__ void next() {
    if (++i >= len()) {
      i = 0;
      j += stride;
    }
  }
};

template <int N>
__device__ __forceinline__ void snap_store(const ImageArgs& a, int f, int64_t j, float (&acc)[N], int lam) {
  const int64_t len = min(a.t_acc, a.n_t - j * a.t_acc);
  const float sc = float(a.snap_scale / double(len));
  // the images are not read again by this kernel: streaming (nontemporal)
  // stores keep them from displacing the E-field stream and u in the caches
  __attribute__((address_space(1))) float* out =
      (__attribute__((address_space(1))) float*)(a.snap + (j * a.F + f) * int64_t(N * N));
  static_for<0, N>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    __builtin_nontemporal_store(acc[y] * sc, out + y * N + lam);
    acc[y] = 0.f;
  });
}

template <int N, int APL>
__device__ __forceinline__ void image_item_snap(const ImageArgs& a, int f, int s, uint8_t* smem) {
  using G = Geo<N>;
  float2* lds = reinterpret_cast<float2*>(smem);
  float2* lds_e = reinterpret_cast<float2*>(smem + FftSmem<N, APL>::E_OFF);
  uint2* stab = reinterpret_cast<uint2*>(smem + FftSmem<N, APL>::T_OFF);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane / N, lam = lane % N;
  const int slot = wave * G::FPW + h;
  const int64_t W = (a.n_t + a.t_acc - 1) / a.t_acc;
  const int64_t wb = W * s / a.splits, we = W * (s + 1) / a.splits;
  float2* buf = lds + slot * G::FRAME;
  float2* epr = lds_e + slot * (APL * N);

  load_slot_table(stab, a.slots, a.n_slots, N);
  static_for<0, N>([&](auto xc) { buf[lam * G::PITCH + decltype(xc)::value] = make_float2(0.f, 0.f); });
  __syncthreads();

  float acc[N];
  static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });
  // every slot walks the same number of steps (the slots of one wave stay in
  // step; frames past a slot's windows are empty)
  const int64_t steps = (we - wb + G::SLOTS - 1) / G::SLOTS * a.t_acc;
  SnapCursor cur{wb + slot, 0, we, G::SLOTS, a.t_acc, a.n_t};
  SnapCursor nxt = cur;
  Raw raw[APL];
  float2 uu[APL];
  fetch_frame<N, APL>(raw, uu, a.efield, a.u, cur.t(), a.t_cal, f, a.F, a.Na, a.fmt, lam, cur.valid());
  for (int64_t q = 0; q < steps; ++q) {
    stage_frame<N, APL>(epr, raw, uu, lam, a.Na, a.fmt, cur.valid());
    nxt.next();
    fetch_frame<N, APL>(raw, uu, a.efield, a.u, nxt.t(), a.t_cal, f, a.F, a.Na, a.fmt, lam, nxt.valid());
    wave_lds_sync();
    grid_frame(buf, epr, stab, a.n_slots, N, lam);
    wave_lds_sync();
    float2 v[N];
    transform_frame<N, +1>(buf, v, lam);
    add_norms<N>(acc, v);
    if (cur.valid() && cur.last()) snap_store<N>(a, f, cur.j, acc, lam);
    cur = nxt;
  }
  __syncthreads();
}

template <int APL, int FMT>
__device__ __forceinline__ void image_item_pair_snap(const ImageArgs& a, int f, int s, uint8_t* smem) {
  static_assert(FMT == kCI4 || FMT == kCI8, "integer E-field formats");
  constexpr int N = 64, INFLIGHT = 8;
  using L = PairSmem<APL>;
  float2* lds = reinterpret_cast<float2*>(smem);
  const int lam = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float2* H = lds + wave * L::WAVE;
  float2* epr = H + L::HALF;
  uint2* stab = reinterpret_cast<uint2*>(smem + L::T_OFF);
  const int S0 = a.n_slots_h0, S1 = a.n_slots_h1;
  const int64_t W = (a.n_t + a.t_acc - 1) / a.t_acc;
  const int64_t wb = W * s / a.splits, we = W * (s + 1) / a.splits;

  load_slot_table(stab, a.slots_h, S0 + S1, N);
  clear_half_row(H, lam);
  __syncthreads();

  float acc[N];
  static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });
  float2 v[N];
  uint32_t raw[APL];
  constexpr int bpe = FMT == kCI4 ? 1 : 2;
  auto fetch_raw = [&](const SnapCursor& c) {
    const bool ok = c.valid();
    const uint8_t* row = a.efield + (c.t() * a.F + f) * int64_t(a.Na) * bpe;
    static_for<0, APL>([&](auto ic) {
      const int an = lam + N * decltype(ic)::value;
      raw[decltype(ic)::value] = (ok && an < a.Na) ? load_raw_global(row, an, FMT).x : 0u;
    });
  };
  // the waves are independent: each walks its own windows
  SnapCursor cur{wb + wave, 0, we, INFLIGHT, a.t_acc, a.n_t};
  fetch_raw(cur);
  while (cur.valid()) {
    const int64_t t = cur.t();
    __builtin_amdgcn_s_setprio(1);
    const float2* urow = a.u + ((t / a.t_cal) * a.F + f) * int64_t(a.Na);
    float2 uu[APL];
    static_for<0, APL>([&](auto ic) {
      const int an = lam + N * decltype(ic)::value;
      uu[decltype(ic)::value] = gload(urow + (an < a.Na ? an : a.Na - 1));
    });
    static_for<0, APL>([&](auto ic) {
      const int an = lam + N * decltype(ic)::value;
      if (an < a.Na) epr[an] = cmul(unpack_raw(Raw{raw[decltype(ic)::value], 0u}, FMT), uu[decltype(ic)::value]);
    });
    wave_lds_sync();
    grid_frame_fit(H, epr, stab, S0, N, lam);
    wave_lds_sync();
    take_half_row<0>(v, H, lam);
    wave_lds_sync();
    grid_frame_fit(H, epr, stab + S0 * N, S1, N, lam);
    wave_lds_sync();
    take_half_row<32>(v, H, lam);
    wave_lds_sync();
    __builtin_amdgcn_s_setprio(0);
    fft_reg<N, +1>(v);
    transpose64(v, H, lam);
    fft_reg<N, +1>(v);
    SnapCursor nxt = cur;
    nxt.next();
    fetch_raw(nxt);
    add_norms<N>(acc, v);
    if (cur.last()) snap_store<N>(a, f, cur.j, acc, lam);
    cur = nxt;
  }
  __syncthreads();
}

// Long windows (t_acc >= kSnapGroupWindow) on the paired engine: the eight
// waves share each window's frames, as in the averaging engine, and the
// workgroup sums them into the window's image.
template <int APL, int FMT>
__device__ __forceinline__ void image_item_pair_snap_group(const ImageArgs& a, int f, int s, uint8_t* smem) {
  using L = PairSmem<APL>;
  const int lam = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float2* H = reinterpret_cast<float2*>(smem) + wave * L::WAVE;
  uint2* stab = reinterpret_cast<uint2*>(smem + L::T_OFF);
  const int64_t W = (a.n_t + a.t_acc - 1) / a.t_acc;
  const int64_t wb = W * s / a.splits, we = W * (s + 1) / a.splits;

  load_slot_table(stab, a.slots_h, a.n_slots_h0 + a.n_slots_h1, 64);
  clear_half_row(H, lam);
  __syncthreads();
  float acc[64];
  static_for<0, 64>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });
  for (int64_t j = wb; j < we; ++j) {
    const int64_t t0 = j * a.t_acc, t1 = min(t0 + a.t_acc, a.n_t);
    pair_frames<APL, FMT>(a, f, t0, t1, acc, H, H + L::HALF, stab, lam, wave);
    pair_reduce<APL>(acc, a.snap + (j * a.F + f) * int64_t(64 * 64), float(a.snap_scale / double(t1 - t0)), smem,
                     lam, wave);
  }
  __syncthreads();
}

}  // namespace epic
