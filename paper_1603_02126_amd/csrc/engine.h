// Device building blocks shared by the imaging, adjoint and calibration
// kernels (gfx950, wave64).
#pragma once
#include "epic_internal.h"
#include "fft_reg.h"

namespace epic {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// Global memory accesses with the address space stated.  Where a pointer
// reaches the code through a function boundary (the batched kernel calls the
// engines as functions) the compiler cannot tell that it points to global
// memory and would use FLAT instructions, which also count against the LDS
// wait counter: every LDS wait would then wait for the next frame's
// prefetch as well.
typedef unsigned int gvec2 __attribute__((ext_vector_type(2)));
typedef unsigned int gvec4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  // vector structs (float2, uint2, ...) go through a native vector type: their
  // copy constructor would take the address back to a generic pointer
  if constexpr (sizeof(T) == 8 && alignof(T) >= 8) {
    const gvec2 v = *(const __attribute__((address_space(1))) gvec2*)p;
    T r;
    __builtin_memcpy(&r, &v, 8);
    return r;
  } else if constexpr (sizeof(T) == 16 && alignof(T) >= 16) {
    const gvec4 v = *(const __attribute__((address_space(1))) gvec4*)p;
    T r;
    __builtin_memcpy(&r, &v, 16);
    return r;
  } else {
    return *(const __attribute__((address_space(1))) T*)p;
  }
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  if constexpr (sizeof(T) == 8 && alignof(T) >= 8) {
    gvec2 w;
    __builtin_memcpy(&w, &v, 8);
    *(__attribute__((address_space(1))) gvec2*)p = w;
  } else if constexpr (sizeof(T) == 16 && alignof(T) >= 16) {
    gvec4 w;
    __builtin_memcpy(&w, &v, 16);
    *(__attribute__((address_space(1))) gvec4*)p = w;
  } else {
    *(__attribute__((address_space(1))) T*)p = v;
  }
}

// A raw packed sample held in registers until it is used (so that a prefetch
// does not force the wait for the load at the point of issue).
struct Raw {
  uint32_t x, y;
};

// Sample a of a packed row: load_raw reads a row anywhere (the calibration
// solve reads rows staged in LDS), load_raw_global a row of the E-field
// stream in global memory, with the address space stated.
__device__ __forceinline__ Raw load_raw(const uint8_t* row, int a, int fmt) {
  Raw r;
  if (fmt == kCI4) {
    r.x = row[a];
    r.y = 0;
  } else if (fmt == kCI8) {
    r.x = reinterpret_cast<const uint16_t*>(row)[a];
    r.y = 0;
  } else {
    const uint2 v = reinterpret_cast<const uint2*>(row)[a];
    r.x = v.x;
    r.y = v.y;
  }
  return r;
}

__device__ __forceinline__ Raw load_raw_global(const uint8_t* row, int a, int fmt) {
  Raw r;
  if (fmt == kCI4) {
    r.x = gload(row + a);
    r.y = 0;
  } else if (fmt == kCI8) {
    r.x = gload(reinterpret_cast<const uint16_t*>(row) + a);
    r.y = 0;
  } else {
    const uint2 v = gload(reinterpret_cast<const uint2*>(row) + a);
    r.x = v.x;
    r.y = v.y;
  }
  return r;
}

// Two's complement nibbles / bytes -> float (exact).
__device__ __forceinline__ float2 unpack_raw(Raw r, int fmt) {
  if (fmt == kCI4) {
    const int b = int(int8_t(uint8_t(r.x)));
    return make_float2(float(b >> 4), float(int(int8_t(uint8_t(r.x << 4))) >> 4));
  } else if (fmt == kCI8) {
    return make_float2(float(int8_t(uint8_t(r.x))), float(int8_t(uint8_t(r.x >> 8))));
  }
  return make_float2(__uint_as_float(r.x), __uint_as_float(r.y));
}

__device__ __forceinline__ float2 load_sample(const uint8_t* row, int a, int fmt) {
  return unpack_raw(load_raw(row, a, fmt), fmt);
}

__device__ __forceinline__ float2 load_sample_global(const uint8_t* row, int a, int fmt) {
  return unpack_raw(load_raw_global(row, a, fmt), fmt);
}

// Order LDS traffic of one wavefront: the hardware executes a wave's LDS
// instructions in order; this keeps the compiler from moving them across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float2 shfl_xor2(float2 v, int m) {
  return make_float2(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

template <int N, int W = 4>
struct Geo {
  static constexpr int PITCH = N + 2;       // complex values per LDS row
  static constexpr int FPW = 64 / N;        // frames per wave
  static constexpr int FRAME = N * PITCH;   // float2 per frame buffer
  static constexpr int SLOTS = W * FPW;     // frames in flight per workgroup of W waves
  static constexpr int LDS = SLOTS * FRAME; // float2 per workgroup
};

// Gridding schedule ("owner computes"): every nonzero grid cell is owned by
// exactly one lane of the frame, which sums the cell's kernel contributions
// w * E'_a (E'_a staged in LDS by the antenna lanes) and stores the cell with
// a plain LDS write -- no atomics.  The host builds the schedule, balanced
// over lanes: per lane a list of slots (lane fastest in memory), each
//   code = antenna | cell offset << 12 | first-of-cell << 31,  weight (float)
// A lane's slots of one cell are consecutive; every slot stores the running
// sum, so the cell's last slot leaves the full sum.  Padding slots have zero
// weight and store into a pad column that the transform never reads.  Cells
// nobody owns stay zero.  The table lives in LDS, shared by the workgroup.
constexpr int64_t kNoInterval = 0x7fffffffffffffffLL;  // t_cal of a single interval
constexpr uint32_t kSlotAntMask = 0xfffu, kSlotCellShift = 12, kSlotCellMask = 0x1fffu;
constexpr int kLdsBytes = 163840 - 1024;                // LDS per workgroup on gfx950, minus a margin

// Copy the slot table (S x L entries) into LDS with the whole workgroup.
__device__ __forceinline__ void load_slot_table(uint2* stab, const uint2* slots, int S, int L) {
  for (int i = threadIdx.x; i < S * L; i += blockDim.x) stab[i] = gload(slots + i);
}

// Half-frame buffer of the two-waves-per-SIMD engines (kHalfPitch rows of
// 32 cells): every lane takes the cells of its own row y = lane into
// v[X0 .. X0 + 31] and clears them for the next half.  Each cell is read and
// cleared by one LDS exchange: a load and a separate store of zeros took 7%
// longer on the 64 x 64 imaging kernel, whose LDS traffic bounds it as much
// as its FP32 issue.
__device__ __forceinline__ float2 lds_take(float2* p) {
  const unsigned long long r = __hip_atomic_exchange(reinterpret_cast<unsigned long long*>(p), 0ull,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  return make_float2(__uint_as_float(uint32_t(r)), __uint_as_float(uint32_t(r >> 32)));
}

template <int X0>
__device__ __forceinline__ void take_half_row(float2 (&v)[64], float2* H, int lam) {
  float2* row = H + lam * kHalfPitch;
  static_for<0, 32>([&](auto xc) { v[X0 + decltype(xc)::value] = lds_take(row + decltype(xc)::value); });
}

// Clears the lane's row of a half-frame buffer, pad column included.
__device__ __forceinline__ void clear_half_row(float2* H, int lam) {
  static_for<0, kHalfPitch>([&](auto xc) { H[lam * kHalfPitch + decltype(xc)::value] = make_float2(0.f, 0.f); });
}

// Calibrate (E'_a = u_a E_a) into the frame's E' staging area.
template <int N, int APL>
__device__ __forceinline__ void stage_frame(float2* epr, const Raw (&raw)[APL], const float2 (&uu)[APL], int lam,
                                            int Na, int fmt, bool active) {
  static_for<0, APL>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const int an = lam + N * i;
    if (an < Na) epr[an] = active ? cmul(unpack_raw(raw[i], fmt), uu[i]) : make_float2(0.f, 0.f);
  });
}

// Grid the staged frame into `buf` (owned cells only; the rest stays zero).
// Slots go in batches of B: the B table entries are loaded together, then
// the B staged values, then the B cell stores -- the stores may alias the
// loads as far as the compiler can tell, so without batching every slot
// would wait for two LDS round trips.
template <int B = 4>
__device__ __forceinline__ void grid_frame(float2* buf, const float2* epr, const uint2* stab, int S, int L,
                                           int lam) {
  // the table addresses come from an opaque copy of the lane index: hoisted
  // out of a frame loop as invariants (one per slot) they took registers the
  // FFTs need and were spilled
  int lo = lam;
  asm volatile("" : "+v"(lo));
  const uint2* col = stab + lo;
  float2 acc = make_float2(0.f, 0.f);
  for (int s0 = 0; s0 < S; s0 += B) {
    uint2 e[B];
    float2 ev[B];
    static_for<0, B>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int s = s0 + k < S ? s0 + k : S - 1;
      e[k] = col[s * L];
    });
    static_for<0, B>([&](auto kc) { ev[decltype(kc)::value] = epr[e[decltype(kc)::value].x & kSlotAntMask]; });
    static_for<0, B>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const float w = __uint_as_float(e[k].y);
      const bool first = int(e[k].x) < 0;
      acc.x = fmaf(w, ev[k].x, first ? 0.f : acc.x);
      acc.y = fmaf(w, ev[k].y, first ? 0.f : acc.y);
      if (s0 + k < S) buf[(e[k].x >> kSlotCellShift) & kSlotCellMask] = acc;
    });
  }
}

// grid_frame with a batch that takes a short schedule in one pass: every
// batch costs two LDS round trips, and the slots of a batch past S are loads
// for nothing (a 9-slot half: one batch of 10 instead of two of 8).
__device__ __forceinline__ void grid_frame_fit(float2* buf, const float2* epr, const uint2* stab, int S, int L,
                                               int lam) {
  if (S <= 8) grid_frame<8>(buf, epr, stab, S, L, lam);
  else if (S <= 10) grid_frame<10>(buf, epr, stab, S, L, lam);
  else if (S <= 12) grid_frame<12>(buf, epr, stab, S, L, lam);
  else grid_frame<8>(buf, epr, stab, S, L, lam);
}

template <int N, int APL>
__device__ __forceinline__ void fetch_frame(Raw (&raw)[APL], float2 (&uu)[APL], const uint8_t* efield,
                                            const float2* u, int64_t t, int64_t t_cal, int f, int F,
                                            int Na, int fmt, int lam, bool active) {
  const int bpe = fmt == kCF32 ? 8 : fmt == kCI8 ? 2 : 1;
  const uint8_t* row = efield + (t * F + f) * int64_t(Na) * bpe;
  const float2* urow = u + ((t / t_cal) * F + f) * int64_t(Na);
  static_for<0, APL>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const int a = lam + N * i;
    if (active && a < Na) {
      raw[i] = load_raw_global(row, a, fmt);
      uu[i] = gload(urow + a);
    } else {
      raw[i] = Raw{0u, 0u};
      uu[i] = make_float2(0.f, 0.f);
    }
  });
}

// Row FFT -> transpose through LDS -> column FFT.  On entry buf holds the
// gridded frame; on exit v[ky] = sum_j G_j exp(S 2 pi i j.k / N) for
// kx = lam, and the lane's buffer row is zero again.
template <int N, int S>
__device__ __forceinline__ void transform_frame(float2* buf, float2 (&v)[N], int lam) {
  constexpr int P = Geo<N>::PITCH;
  static_for<0, N>([&](auto xc) { v[decltype(xc)::value] = buf[lam * P + decltype(xc)::value]; });
  fft_reg<N, S>(v);
  wave_lds_sync();
  static_for<0, N>([&](auto xc) { buf[decltype(xc)::value * P + lam] = v[decltype(xc)::value]; });
  wave_lds_sync();
  static_for<0, N>([&](auto yc) { v[decltype(yc)::value] = buf[lam * P + decltype(yc)::value]; });
  static_for<0, N>([&](auto yc) { buf[lam * P + decltype(yc)::value] = make_float2(0.f, 0.f); });
  fft_reg<N, S>(v);
}


// ---------------------------------------------------------------------------
// EPICal: FP64 update helpers (eq. Cna, eq. damping)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  const double2 n = zmul(a, zconj(b));
  return make_double2(n.x / d, n.y / d);
}
__device__ __forceinline__ double2 zrecip(double2 g) {
  const double d = g.x * g.x + g.y * g.y;
  return make_double2(g.x / d, -g.y / d);
}

// One damped update.  Returns the new gain; sets *st bits if held.
__device__ __forceinline__ double2 epical_step(double2 Kbar, double Qbar, double2 A, double2 D, double2 g,
                                               uint8_t hold, double na, double gamma, uint32_t* st) {
  if (hold) {
    *st |= (hold & kHoldFlagged ? 1u : 0u) | (hold & kHoldDZero ? 2u : 0u);
    return g;
  }
  // C = Kbar - conj(A) Qbar / (Na conj(g))
  const double2 t = zdiv(make_double2(A.x * Qbar, -A.y * Qbar), make_double2(na * g.x, -na * g.y));
  const double2 C = make_double2(Kbar.x - t.x, Kbar.y - t.y);
  const double2 sol = zdiv(make_double2(C.x * na, C.y * na), D);
  const double2 gn = make_double2((1.0 - gamma) * sol.x + gamma * g.x, (1.0 - gamma) * sol.y + gamma * g.y);
  if (!isfinite(gn.x) || !isfinite(gn.y)) {
    *st |= 4u;
    return g;
  }
  return gn;
}


// Update from several tapped pixels: the least-squares combination over the
// pixels of Na C_ap = g_a D_ap (C_ap as in epical_step, per pixel), damped.
__device__ __forceinline__ double2 epical_step_multi(const double2 (&Kbar)[kMaxPix], double Qbar,
                                                     const double2 (&A)[kMaxPix], const double2 (&D)[kMaxPix],
                                                     int np, double2 g, uint8_t hold, double na, double gamma,
                                                     uint32_t* st) {
  if (hold) {
    *st |= (hold & kHoldFlagged ? 1u : 0u) | (hold & kHoldDZero ? 2u : 0u);
    return g;
  }
  const double2 inv = zdiv(make_double2(1.0, 0.0), make_double2(na * g.x, -na * g.y));   // 1 / (Na conj g)
  double2 num = make_double2(0.0, 0.0);
  double den = 0.0;
#pragma unroll
  for (int p = 0; p < kMaxPix; ++p) {
    if (p < np) {
      const double2 t = zmul(make_double2(A[p].x * Qbar, -A[p].y * Qbar), inv);
      const double2 C = make_double2(Kbar[p].x - t.x, Kbar[p].y - t.y);
      const double2 dc = zmul(zconj(D[p]), C);
      num.x += dc.x;
      num.y += dc.y;
      den += D[p].x * D[p].x + D[p].y * D[p].y;
    }
  }
  const double2 sol = make_double2(na * num.x / den, na * num.y / den);
  const double2 gn = make_double2((1.0 - gamma) * sol.x + gamma * g.x, (1.0 - gamma) * sol.y + gamma * g.y);
  if (!isfinite(gn.x) || !isfinite(gn.y)) {
    *st |= 4u;
    return g;
  }
  return gn;
}

template <int N, int K2, int APL>
struct DegridTable {
  int off[APL][K2];
  float w[APL][K2];
  __device__ __forceinline__ void load(const uint32_t* cell_ixy, const float* cell_w, int lam, int Na) {
    static_for<0, APL>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const int an = lam + N * i;
      static_for<0, K2>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (an < Na) {
          const uint32_t ixy = cell_ixy[an * K2 + k];
          off[i][k] = int(ixy >> 16) * Geo<N>::PITCH + int(ixy & 0xffffu);
          w[i][k] = cell_w[an * K2 + k];
        } else {
          off[i][k] = 0;
          w[i][k] = 0.f;
        }
      });
    });
  }
};


// ---------------------------------------------------------------------------
// compile-time variants of the N <= 64 engine
//   APL: antennas per lane of the E' staging (Na <= APL * N)
// LDS budget per workgroup: frame buffers, E' staging, then the slot table.
// ---------------------------------------------------------------------------
template <int N, int APL, int W = 4>
struct Budget {
  static constexpr int FRAMES = Geo<N, W>::LDS * 8;
  static constexpr int STAGE = Geo<N, W>::SLOTS * APL * N * 8;
  static constexpr int TAB_SLOTS = (kLdsBytes - FRAMES - STAGE) / (N * 8);   // slot rows that fit
};

inline int apl_for(int N, int na) {
  const int need = (na + N - 1) / N;
  return need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 0;
}

inline int tab_slots_for(int N, int apl) {
  switch (N * 16 + apl) {
    case 16 * 16 + 2: return Budget<16, 2>::TAB_SLOTS;
    case 16 * 16 + 4: return Budget<16, 4>::TAB_SLOTS;
    case 16 * 16 + 8: return Budget<16, 8>::TAB_SLOTS;
    case 32 * 16 + 2: return Budget<32, 2>::TAB_SLOTS;
    case 32 * 16 + 4: return Budget<32, 4>::TAB_SLOTS;
    case 32 * 16 + 8: return Budget<32, 8>::TAB_SLOTS;
    case 64 * 16 + 2: return Budget<64, 2>::TAB_SLOTS;
    case 64 * 16 + 4: return Budget<64, 4>::TAB_SLOTS;
    case 64 * 16 + 8: return Budget<64, 8>::TAB_SLOTS;
    default: return 0;
  }
}

template <int N, template <int, int> class Launch, typename Args>
inline hipError_t dispatch_apl(int na, const Args& a, hipStream_t s) {
  switch (apl_for(N, na)) {
    case 2: return Launch<N, 2>::run(a, s);
    case 4: return Launch<N, 4>::run(a, s);
    case 8: return Launch<N, 8>::run(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <template <int, int> class Launch, typename Args>
inline hipError_t dispatch_n(int N, int na, const Args& a, hipStream_t s) {
  if (N == 16) return dispatch_apl<16, Launch>(na, a, s);
  if (N == 32) return dispatch_apl<32, Launch>(na, a, s);
  if (N == 64) return dispatch_apl<64, Launch>(na, a, s);
  return hipErrorInvalidValue;
}

}  // namespace epic
