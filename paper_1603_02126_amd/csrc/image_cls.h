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
#include "xpose.h"

namespace epic {

constexpr int kClsMaxAnt = 512;
constexpr int kClsGridBatch = 8;   // gridding slots per batch in the one-wave class engines
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
// GB: gridding slots per batch; 0 grids one slot at a time (the persistent
// multi-array kernel, where that form measured faster).
template <int R, bool BIG, int GB = kClsGridBatch>
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
        raw[i] = load_raw_global(row, an, a.fmt);
        uu[i] = gload(urow + an);
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
    if constexpr (GB > 0) {
      // slots in batches: the batch's table entries are all requested before the
      // first is used (from memory for the dense variant), so one wait covers them
      const int S = a.n_slots;
      for (int k0 = 0; k0 < S; k0 += GB) {
        uint2 e[GB];
        static_for<0, GB>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          const int k = k0 + j < S ? k0 + j : S - 1;
          e[j] = BIG ? gload(a.slots + k * 64 + lane) : stab[k * 64 + lane];
        });
        static_for<0, GB>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          const uint32_t code = e[j].x;
          const int qx = (code >> 12) & 63, qy = (code >> 18) & 63;
          const int jx = qx + 64 * int((code >> 24) & 3), jy = qy + 64 * int((code >> 26) & 3);
          const float2 ph = tw[(jx * cx + jy * cy) & (N - 1)];
          const float w = __uint_as_float(e[j].y);
          const float2 ev = cmul(epr[code & kSlotAntMask], make_float2(w * ph.x, w * ph.y));
          const float keep = int(code) < 0 ? 0.f : 1.f;   // a cell's first contribution restarts the sum
          sum.x = fmaf(sum.x, keep, ev.x);
          sum.y = fmaf(sum.y, keep, ev.y);
          const int off = (code >> 30) & 1 ? qy * P + qx : 64;
          if (k0 + j < S) buf[off] = sum;
        });
      }
    } else {
#pragma unroll 4
      for (int k = 0; k < a.n_slots; ++k) {
        const uint2 e = BIG ? gload(a.slots + k * 64 + lane) : stab[k * 64 + lane];
        const uint32_t code = e.x;
        const int qx = (code >> 12) & 63, qy = (code >> 18) & 63;
        const int jx = qx + 64 * int((code >> 24) & 3), jy = qy + 64 * int((code >> 26) & 3);
        const float2 ph = tw[(jx * cx + jy * cy) & (N - 1)];
        const float w = __uint_as_float(e.y);
        const float2 ev = cmul(epr[code & kSlotAntMask], make_float2(w * ph.x, w * ph.y));
        const float keep = int(code) < 0 ? 0.f : 1.f;
        sum.x = fmaf(sum.x, keep, ev.x);
        sum.y = fmaf(sum.y, keep, ev.y);
        const int off = (code >> 30) & 1 ? qy * P + qx : 64;
        buf[off] = sum;
      }
    }
    if constexpr (BIG) __syncthreads();   // the single staging buffer is rewritten next
    else wave_lds_sync();
    float2 v[64];
    transform_frame<64, +1>(buf, v, lane);
    add_norms<64>(acc, v);
  }
  // class pixels: (R ky + cy, R kx + cx) with kx = lane
  float* out = a.partial + (int64_t(s) * a.F + f) * (int64_t(N) * N);
  static_for<0, 64>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    gstore(out + (R * y + cy) * N + R * lane + cx, acc[y]);
  });
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Residue-class engine with two waves per SIMD (integer E-fields, Na <= 512).
//
// Eight waves: two frames (samples t, t + 1) x four classes of the class
// group.  Each wave grids its class of its frame through half a 64 x 64 frame
// (sub-cell columns 0..31, then 32..63, two schedules built on the host), runs
// the row FFTs, transposes through the half frame (xpose.h)
// and runs the column FFTs, as the 64 x 64 paired engine does.  The E' of the
// two frames is staged once per frame by its four waves; two workgroup
// barriers per pair of samples order the staging against the gridding.
// Waves w and w + 4 image the same class and are summed at the end.
// ---------------------------------------------------------------------------
constexpr int kClsPairThreads = 512;

// DB: the staged E' is double buffered (two pairs of frames; arrays of at
// most kClsPairMaxAntDB antennas), so that no workgroup barrier has to keep a
// pair's E' alive until every wave has gridded it: one barrier per pair of
// samples instead of two.
constexpr int kClsPairMaxAntDB = 384;

template <int R, bool DB = false>
struct ClsPairSmem {
  static constexpr int N = 64 * R;
  static constexpr int HALF = 64 * kHalfPitch;                   // float2 per wave
  static constexpr int MAXA = DB ? kClsPairMaxAntDB : kClsMaxAnt;   // E' per frame
  static constexpr int E_OFF = 8 * HALF * 8;                     // bytes
  static constexpr int TW_OFF = E_OFF + (DB ? 4 : 2) * MAXA * 8;
  static constexpr int T_OFF = TW_OFF + N * 8;
  static constexpr int TAB_SLOTS = (kLdsBytes - T_OFF) / (64 * 8);
  static constexpr int BYTES = T_OFF + TAB_SLOTS * 64 * 8;
  static_assert(HALF >= kXposeFloat2, "the transpose staging reuses the half frame");
  static_assert(4 * 64 * 64 * 4 <= E_OFF, "the class reduction reuses the half frames");
};

// Grid sub-cell columns [32 hf, 32 hf + 32) of class (cx, cy) into the half
// frame H (column qx - 32 hf), slots in batches of B.
template <int R, int B>
__device__ __forceinline__ void grid_cls_half(float2* H, const float2* epr, const float2* tw, const uint2* stab,
                                              int S, int hf, int cx, int cy, int lam) {
  constexpr int N = 64 * R;
  int lo = lam;                 // opaque copy: no per-slot table address held across the frame loop
  asm volatile("" : "+v"(lo));
  const uint2* col = stab + lo;
  float2 sum = make_float2(0.f, 0.f);
  for (int s0 = 0; s0 < S; s0 += B) {
    uint2 e[B];
    float2 ev[B], ph[B];
    static_for<0, B>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      e[k] = col[(s0 + k < S ? s0 + k : S - 1) * 64];
    });
    static_for<0, B>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const uint32_t code = e[k].x;
      const int jx = int((code >> 12) & 63) + 64 * int((code >> 24) & 3);
      const int jy = int((code >> 18) & 63) + 64 * int((code >> 26) & 3);
      ph[k] = tw[(jx * cx + jy * cy) & (N - 1)];
      ev[k] = epr[code & kSlotAntMask];
    });
    static_for<0, B>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const uint32_t code = e[k].x;
      const float w = __uint_as_float(e[k].y);
      const float2 c = cmul(ev[k], make_float2(w * ph[k].x, w * ph[k].y));
      const float keep = int(code) < 0 ? 0.f : 1.f;   // a cell's first contribution restarts the sum
      sum.x = fmaf(sum.x, keep, c.x);
      sum.y = fmaf(sum.y, keep, c.y);
      const int qx = (code >> 12) & 63, qy = (code >> 18) & 63;
      const int off = (code >> 30) & 1 ? qy * kHalfPitch + qx - 32 * hf : 32;
      if (s0 + k < S) H[off] = sum;
    });
  }
}

// grid_cls_half with the batch chosen from the half's schedule length: a
// schedule of up to 12 slots goes in one batch (two LDS round trips) rather
// than in three of 4.
template <int R>
__device__ __forceinline__ void grid_cls_half_fit(float2* H, const float2* epr, const float2* tw, const uint2* stab,
                                                  int S, int hf, int cx, int cy, int lam) {
  if (S <= 4) grid_cls_half<R, 4>(H, epr, tw, stab, S, hf, cx, cy, lam);
  else if (S <= 8) grid_cls_half<R, 8>(H, epr, tw, stab, S, hf, cx, cy, lam);
  else if (S <= 12) grid_cls_half<R, 12>(H, epr, tw, stab, S, hf, cx, cy, lam);
  else grid_cls_half<R, 4>(H, epr, tw, stab, S, hf, cx, cy, lam);
}

template <int R, int FMT, bool DB>
__device__ __forceinline__ void image_cls_pair_item(const ImageArgs& a, int f, int cg, int s, uint8_t* smem) {
  static_assert(FMT == kCI4 || FMT == kCI8, "integer E-field formats");
  constexpr int N = 64 * R, NF = 64;
  using L = ClsPairSmem<R, DB>;
  float2* lds = reinterpret_cast<float2*>(smem);
  const int tid = threadIdx.x, lam = tid & 63, wave = tid >> 6;
  const int fs = wave >> 2, ci = wave & 3;          // frame slot, class within the group
  const int c = cg * 4 + ci, cx = c % R, cy = c / R;
  const int gt = tid & 255;                         // thread within the frame's four waves
  float2* H = lds + wave * L::HALF;
  float2* const e_base = reinterpret_cast<float2*>(smem + L::E_OFF);
  float2* tw = reinterpret_cast<float2*>(smem + L::TW_OFF);
  uint2* stab = reinterpret_cast<uint2*>(smem + L::T_OFF);
  const int S0 = a.n_slots_h0, S1 = a.n_slots_h1;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  constexpr int bpe = FMT == kCI4 ? 1 : 2;
  constexpr int APT = kClsMaxAnt / 256;             // antennas per staging thread

  load_slot_table(stab, a.slots_h, S0 + S1, 64);
  for (int k = tid; k < N; k += kClsPairThreads) {
    double sn, cs;
    sincospi(2.0 * double(k) / double(N), &sn, &cs);
    tw[k] = make_float2(float(cs), float(sn));
  }
  clear_half_row(H, lam);

  float acc[NF];
  static_for<0, NF>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });
  float2 v[NF];
  uint32_t raw[APT];
  auto fetch_raw = [&](int64_t t) {
    const uint8_t* row = a.efield + (t * a.F + f) * int64_t(a.Na) * bpe;
    static_for<0, APT>([&](auto ic) {
      const int an = gt + 256 * decltype(ic)::value;
      raw[decltype(ic)::value] = (t < te && an < a.Na) ? load_raw_global(row, an, FMT).x : 0u;
    });
  };
  const int64_t iters = (te - tb + 1) / 2;
  fetch_raw(tb + fs);
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + 2 * it + fs;
    float2* epr = e_base + ((DB ? int(it & 1) * 2 : 0) + fs) * L::MAXA;
    __builtin_amdgcn_s_setprio(1);   // LDS-bound phases at raised priority (see the 64 x 64 paired engine)
    // stage E' of this frame (its four waves)
    const float2* urow = a.u + (((t < te ? t : tb) / a.t_cal) * a.F + f) * int64_t(a.Na);
    float2 uu[APT];
    static_for<0, APT>([&](auto ic) {
      const int an = gt + 256 * decltype(ic)::value;
      uu[decltype(ic)::value] = gload(urow + (an < a.Na ? an : a.Na - 1));
    });
    static_for<0, APT>([&](auto ic) {
      const int an = gt + 256 * decltype(ic)::value;
      if (an < a.Na) epr[an] = t < te ? cmul(unpack_raw(Raw{raw[decltype(ic)::value], 0u}, FMT),
                                             uu[decltype(ic)::value])
                                      : make_float2(0.f, 0.f);
    });
    __syncthreads();
    grid_cls_half_fit<R>(H, epr, tw, stab, S0, 0, cx, cy, lam);
    wave_lds_sync();
    take_half_row<0>(v, H, lam);
    wave_lds_sync();
    grid_cls_half_fit<R>(H, epr, tw, stab + S0 * 64, S1, 1, cx, cy, lam);
    wave_lds_sync();
    take_half_row<32>(v, H, lam);
    // single buffer: every wave must be done with this pair's E' before the
    // next pair is staged; double buffered, the next pair goes to the other
    // buffer, and the pair after it is staged only after the barrier that
    // follows the next staging, which every wave reaches after gridding this one
    if constexpr (!DB) __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    fft_reg<NF, +1>(v);
    __builtin_amdgcn_s_setprio(1);
    transpose64(v, H, lam);
    __builtin_amdgcn_s_setprio(0);
    fft_reg<NF, +1>(v);
    fetch_raw(t + 2);
    add_norms<NF>(acc, v);
  }
  // sum the two frame slots of each class, then write the class pixels
  // (R y + cy, R kx + cx) with kx = lam
  __syncthreads();
  float* red = reinterpret_cast<float*>(lds);
  if (fs == 1)
    static_for<0, NF>([&](auto yc) { red[(ci * NF + decltype(yc)::value) * NF + lam] = acc[decltype(yc)::value]; });
  __syncthreads();
  if (fs == 0) {
    float* out = a.partial + (int64_t(s) * a.F + f) * (int64_t(N) * N);
    static_for<0, NF>([&](auto yc) {
      constexpr int y = decltype(yc)::value;
      gstore(out + (R * y + cy) * N + R * lam + cx, acc[y] + red[(ci * NF + y) * NF + lam]);
    });
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Residue-class engine with two waves per SIMD for dense arrays (integer
// E-fields; 513..2048 antennas at 256 x 256, up to 1024 at 128 x 128).
//
// Eight waves, one class each: at R = 4 the eight classes (cy = 2 cg + j,
// j = 0, 1; cx = 0..3) of one frame, at R = 2 the four classes of two frames
// (samples t, t + 1).  The gridding serves all classes of a frame at once:
// the frame's sub-cells are owned by the lanes of all its waves (a host
// schedule per half of the sub-cell columns), and every contribution
// z = w E'_a to sub-cell q = j mod 64 is added, for each class c, as
//   z exp(+2 pi i jy cy / N) exp(+2 pi i jx cx / N)
// into the owner's register sums, which go to the classes' half frames when
// the sub-cell's last contribution has been added.  One table entry, one E'
// and three twiddle loads (the column twiddles' higher powers are products)
// serve eight classes (R = 4), against one table entry, one
// E' and one twiddle per contribution and class when each wave grids its own
// class.  Each wave then takes its class's half rows, runs the row FFTs,
// transposes through the half frame and runs the column FFTs, as the paired engines do.
// The E' of a frame (up to 2048 complex values) and the eight half frames
// fill the LDS, so the schedules are read from memory (the same rows for
// every workgroup of the array: cache resident), each batch of entries
// requested while the previous one is gridded.  Workgroup barriers order the
// staging, the two gridding passes and the row loads.
// Multi-class slot code: antenna | qx << 12 | qy << 18 | px << 24 | py << 26
//                        | last << 30 | first << 31
// (padding slots: weight 0, first and not last, never stored).
// ---------------------------------------------------------------------------
constexpr int kClsDenseThreads = 512;

template <int R>
struct ClsDenseSmem {
  static constexpr int N = 64 * R;
  static constexpr int CPW = R == 4 ? 8 : 4;            // classes per frame (= per workgroup)
  static constexpr int NF = 8 / CPW;                     // frames per step
  static constexpr int NCY = CPW / R;                    // cy values per workgroup
  static constexpr int OWNERS = 64 * CPW;                // lanes owning a frame's sub-cells
  static constexpr int MAXA = R == 4 ? 2048 : 1024;      // E' per frame
  static constexpr int HALF = 64 * kHalfPitch;           // float2 per wave
  static constexpr int E_OFF = 8 * HALF * 8;             // bytes
  static constexpr int TW_OFF = E_OFF + NF * MAXA * 8;
  static constexpr int BYTES = TW_OFF + N * 8;
  static_assert(BYTES <= kLdsBytes, "half frames, E' staging and twiddles fit the LDS");
  static_assert(HALF >= kXposeFloat2, "the transpose staging reuses the half frame");
  static_assert(4 * 64 * 64 * 4 <= E_OFF, "the class reduction reuses the half frames");
};

// Grid sub-cell columns [32 hf, 32 hf + 32) of all classes of a frame: the
// owner's slots from `tab` (S rows of OWNERS entries, this owner's column),
// B per batch, the next batch requested before the current one is gridded.
// Class (cy0 + jc, cx) goes to the half frame H0 + (jc R + cx) * HALF.
template <int R, int B>
__device__ __forceinline__ void grid_dense_half(float2* H0, const float2* epr, const float2* tw, const uint2* tab,
                                                int S, int hf, int cy0, int owner) {
  using L = ClsDenseSmem<R>;
  constexpr int N = 64 * R, NCY = L::NCY, OW = L::OWNERS;
  if (S <= 0) return;
  float2 acc[NCY][R];
  static_for<0, NCY>([&](auto jc) {
    static_for<0, R>([&](auto mc) { acc[decltype(jc)::value][decltype(mc)::value] = make_float2(0.f, 0.f); });
  });
  int ow = owner;               // opaque copy: no per-slot table address held across the frame loop
  asm volatile("" : "+v"(ow));
  tab += ow;
  uint2 nxt[B];
  static_for<0, B>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    nxt[k] = gload(tab + (k < S ? k : S - 1) * OW);
  });
  for (int s0 = 0; s0 < S; s0 += B) {
    uint2 e[B];
    static_for<0, B>([&](auto kc) { e[decltype(kc)::value] = nxt[decltype(kc)::value]; });
    if (s0 + B < S) {
      static_for<0, B>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        nxt[k] = gload(tab + (s0 + B + k < S ? s0 + B + k : S - 1) * OW);
      });
    }
    static_for<0, B>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const uint32_t code = e[k].x;
      const int qx = (code >> 12) & 63, qy = (code >> 18) & 63;
      const int jx = qx + 64 * int((code >> 24) & 3), jy = qy + 64 * int((code >> 26) & 3);
      const float2 ev = epr[code & kSlotAntMask];
      float2 tx[R], ty[NCY];
      // tx[m] = e^{+2 pi i jx m / N}: one gather, the higher powers by products
      tx[1] = tw[jx & (N - 1)];
      static_for<2, R>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        tx[m] = cmul(tx[m - 1], tx[1]);
      });
      static_for<0, NCY>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        ty[j] = tw[(jy * (cy0 + j)) & (N - 1)];
      });
      const float w = __uint_as_float(e[k].y);
      const float2 z = make_float2(w * ev.x, w * ev.y);
      // a cell's first contribution restarts its sums: acc * 0 + c, one FMA
      // per component instead of an add and a select
      const float keep = int(code) < 0 ? 0.f : 1.f;
      const bool last = (code >> 30) & 1;
      static_for<0, NCY>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const float2 zy = cmul(z, ty[j]);
        static_for<0, R>([&](auto mc) {
          constexpr int m = decltype(mc)::value;
          float2 c;
          if constexpr (m == 0) c = zy;
          else c = cmul(zy, tx[m]);
          acc[j][m].x = fmaf(acc[j][m].x, keep, c.x);
          acc[j][m].y = fmaf(acc[j][m].y, keep, c.y);
        });
      });
      if (last && s0 + k < S) {
        const int off = qy * kHalfPitch + qx - 32 * hf;
        static_for<0, NCY>([&](auto jc) {
          static_for<0, R>([&](auto mc) {
            constexpr int j = decltype(jc)::value, m = decltype(mc)::value;
            H0[(j * R + m) * L::HALF + off] = acc[j][m];
          });
        });
      }
    });
  }
}

// GB: gridding slots per batch (2 or 4, an autotuner choice).
template <int R, int FMT, int GB>
__device__ __forceinline__ void image_cls_dense_item(const ImageArgs& a, int f, int cg, int s, uint8_t* smem) {
  static_assert(FMT == kCI4 || FMT == kCI8, "integer E-field formats");
  using L = ClsDenseSmem<R>;
  constexpr int N = 64 * R, NF = L::NF, CPW = L::CPW, OW = L::OWNERS;
  constexpr int APT = L::MAXA / OW;                 // antennas per staging thread
  float2* lds = reinterpret_cast<float2*>(smem);
  const int tid = threadIdx.x, lam = tid & 63, wave = tid >> 6;
  const int fs = wave / CPW, ci = wave % CPW;       // frame slot, class within the frame
  const int cx = ci % R, cy = cg * L::NCY + ci / R, cy0 = cg * L::NCY;
  const int owner = tid % OW;                       // sub-cell owner (and staging thread) of the frame
  float2* H = lds + wave * L::HALF;
  float2* H0 = lds + fs * CPW * L::HALF;            // the frame's first class buffer
  float2* epr = reinterpret_cast<float2*>(smem + L::E_OFF) + fs * L::MAXA;
  float2* tw = reinterpret_cast<float2*>(smem + L::TW_OFF);
  const int S0 = a.n_slots_m0, S1 = a.n_slots_m1;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  constexpr int bpe = FMT == kCI4 ? 1 : 2;

  for (int k = tid; k < N; k += kClsDenseThreads) {
    double sn, cs;
    sincospi(2.0 * double(k) / double(N), &sn, &cs);
    tw[k] = make_float2(float(cs), float(sn));
  }
  clear_half_row(H, lam);

  float acc[64];
  static_for<0, 64>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });
  float2 v[64];
  uint32_t raw[APT];
  auto fetch_raw = [&](int64_t t) {
    const uint8_t* row = a.efield + (t * a.F + f) * int64_t(a.Na) * bpe;
    static_for<0, APT>([&](auto ic) {
      const int an = owner + OW * decltype(ic)::value;
      raw[decltype(ic)::value] = (t < te && an < a.Na) ? load_raw_global(row, an, FMT).x : 0u;
    });
  };
  const int64_t iters = (te - tb + NF - 1) / NF;
  fetch_raw(tb + fs);
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + NF * it + fs;
    const float2* urow = a.u + (((t < te ? t : tb) / a.t_cal) * a.F + f) * int64_t(a.Na);
    float2 uu[APT];
    static_for<0, APT>([&](auto ic) {
      const int an = owner + OW * decltype(ic)::value;
      uu[decltype(ic)::value] = gload(urow + (an < a.Na ? an : a.Na - 1));
    });
    static_for<0, APT>([&](auto ic) {
      const int an = owner + OW * decltype(ic)::value;
      if (an < a.Na) epr[an] = t < te ? cmul(unpack_raw(Raw{raw[decltype(ic)::value], 0u}, FMT),
                                             uu[decltype(ic)::value])
                                      : make_float2(0.f, 0.f);
    });
    __syncthreads();                 // E' staged (and every half frame clear)
    grid_dense_half<R, GB>(H0, epr, tw, a.slots_m, S0, 0, cy0, owner);
    __syncthreads();                 // every class's first half gridded
    take_half_row<0>(v, H, lam);
    __syncthreads();                 // every half frame read and cleared
    grid_dense_half<R, GB>(H0, epr, tw, a.slots_m + S0 * OW, S1, 1, cy0, owner);
    __syncthreads();                 // second halves gridded; E' free for the next step
    take_half_row<32>(v, H, lam);
    fft_reg<64, +1>(v);
    transpose64(v, H, lam);
    fft_reg<64, +1>(v);
    fetch_raw(t + NF);
    add_norms<64>(acc, v);
  }
  // class pixels (R y + cy, R kx + cx), kx = lam; at R = 2 the two frame
  // slots of each class are summed first
  float* out = a.partial + (int64_t(s) * a.F + f) * (int64_t(N) * N);
  if constexpr (NF == 1) {
    static_for<0, 64>([&](auto yc) {
      constexpr int y = decltype(yc)::value;
      gstore(out + (R * y + cy) * N + R * lam + cx, acc[y]);
    });
  } else {
    __syncthreads();
    float* red = reinterpret_cast<float*>(lds);
    if (fs == 1)
      static_for<0, 64>([&](auto yc) { red[(ci * 64 + decltype(yc)::value) * 64 + lam] = acc[decltype(yc)::value]; });
    __syncthreads();
    if (fs == 0) {
      static_for<0, 64>([&](auto yc) {
        constexpr int y = decltype(yc)::value;
        gstore(out + (R * y + cy) * N + R * lam + cx, acc[y] + red[(ci * 64 + y) * 64 + lam]);
      });
    }
  }
  __syncthreads();
}

}  // namespace epic
