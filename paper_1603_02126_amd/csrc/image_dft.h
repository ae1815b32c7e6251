// HIP kernels (gfx950): 2D DFT as two complex GEMMs on the matrix cores, with
// split-precision 16-bit operands and FP32 accumulation (grids of 32 and 64;
// 128 and 256 as residue classes of 64 x 64).
//
// Per frame, with F[j][k] = exp(+2 pi i j k / N) (symmetric):
//   stage 1   Y^T = G^T F      (Y^T[jx][ky] = sum_jy G[jy][jx] F[jy][ky])
//   stage 2   X^T = F Y^T      (X^T[kx][ky] = sum_jx F[kx][jx] Y^T[jx][ky])
// so X[ky][kx] = sum_j G[jy][jx] exp(+2 pi i (jx kx + jy ky) / N), the
// unnormalised image transform of Sec. 2.1.  Every real operand x is split
// into 16-bit parts, x = p0 + p1 (+ p2), p_k the rounding of what the earlier
// parts leave; a real product takes the part products p_i q_j with
// i + j < PARTS (the dropped ones are below the last part's precision), and a
// complex product four real ones, the two that are subtracted accumulated
// apart and subtracted at the end.  Precisions (DftPrec):
//   F16     fp16 hi + lo, 3 part products (22 bits); each frame is scaled by a
//           power of two first (exact, divided out of |X|^2) so that fp16
//           neither overflows nor loses the lo part
//   BF16    bf16 hi + lo, 3 part products (16 bits; FP32 range, no scale)
//   BF16X3  bf16 hi + mid + lo, 6 part products (24 bits; no scale)
// The FP32 accumulator tile of stage 1 is already laid out as the B operand
// of stage 2 once the contraction index is relabelled the same way in both
// operands, so Y never leaves registers.
//
// MFMA v_mfma_f32_32x32x16_{f16,bf16} lane layout (lane l, h = l / 32):
//   A[i][k]: i = l % 32, k = 8 h + e        (e = element 0..7 of the vector)
//   B[k][j]: j = l % 32, k = 8 h + e
//   C[i][j]: j = l % 32, i = 8 (v / 4) + 4 h + v % 4   (v = 0..15)
#pragma once
#include "engine.h"

namespace epic {

constexpr int kDftTabSlots = 32;   // gridding slot rows held in LDS

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float16v mfma(half8 a, half8 b, float16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float16v mfma(bf16x8 a, bf16x8 b, float16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Precision policies (the values of ImageArgs::dft_prec).
enum : int { kDftF16 = 0, kDftBF16 = 1, kDftBF16x3 = 2 };
template <int PREC>
struct DftPrec;
template <>
struct DftPrec<kDftF16> {
  using E = _Float16;
  using V = half8;
  static constexpr int PARTS = 2;
  static constexpr bool SCALE = true;
};
template <>
struct DftPrec<kDftBF16> {
  using E = __bf16;
  using V = bf16x8;
  static constexpr int PARTS = 2;
  static constexpr bool SCALE = false;
};
template <>
struct DftPrec<kDftBF16x3> {
  using E = __bf16;
  using V = bf16x8;
  static constexpr int PARTS = 3;
  static constexpr bool SCALE = false;
};

template <int PREC>
struct SplitV {
  typename DftPrec<PREC>::V p[DftPrec<PREC>::PARTS];
};

template <int PREC>
__device__ __forceinline__ SplitV<PREC> split8(const float (&x)[8]) {
  using P = DftPrec<PREC>;
  SplitV<PREC> s;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float r = x[e];
#pragma unroll
    for (int k = 0; k < P::PARTS; ++k) {
      const typename P::E h = typename P::E(r);
      s.p[k][e] = h;
      r -= float(h);
    }
  }
  return s;
}

// acc += a * b with split operands: the part products p_i q_j, i + j < PARTS,
// smallest first.
template <int PREC>
__device__ __forceinline__ float16v mfma_split(const SplitV<PREC>& a, const SplitV<PREC>& b, float16v acc) {
  constexpr int P = DftPrec<PREC>::PARTS;
#pragma unroll
  for (int d = P - 1; d >= 0; --d)
#pragma unroll
    for (int i = 0; i <= d; ++i) acc = mfma(a.p[i], b.p[d - i], acc);
  return acc;
}

// Real MFMA operations per split product (executed work).
template <int PREC>
constexpr int split_products() {
  return DftPrec<PREC>::PARTS * (DftPrec<PREC>::PARTS + 1) / 2;
}

// F element exp(+2 pi i m / N) in float, from a double-precision angle.
__device__ __forceinline__ float2 froot(int m, int N) {
  double s, c;
  sincospi(2.0 * double(m % N) / double(N), &s, &c);
  return make_float2(float(c), float(s));
}

template <int N>
struct DftGeo {
  static constexpr int T = N / 32;           // 32-wide tiles per dimension
  static constexpr int WPF = T;              // waves per frame (one per column tile)
  static constexpr int FPI = 4 / WPF;        // frames per workgroup iteration
  static constexpr int OWNERS = 64 * WPF;    // lanes gridding a frame
  static constexpr int PITCH = N + 2;        // complex values per G^T row in LDS
  static constexpr int FRAME = N * PITCH;
  static constexpr int KS = N / 16;          // k-steps of stage 1
};

// The stage-2 A operand F[kx][k] in lane order, split: c2 holds, for each
// (tx, ti, sg), the real parts then the imaginary parts, PARTS vectors each.
template <int N, int PREC>
__device__ __forceinline__ void dft_stage2_table(typename DftPrec<PREC>::V* c2, int tid) {
  using D = DftGeo<N>;
  constexpr int PP = DftPrec<PREC>::PARTS;
  for (int q = tid; q < D::T * D::T * 2 * 64; q += 256) {
    const int ln = q % 64, sg = (q / 64) % 2, ti = (q / 128) % D::T, tx = q / (128 * D::T);
    const int hh = ln >> 5, ll = ln & 31;
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = ti * 32 + 16 * sg + 8 * (e / 4) + 4 * hh + (e % 4);
      const float2 w = froot((tx * 32 + ll) * k, N);
      re[e] = w.x;
      im[e] = w.y;
    }
    const SplitV<PREC> r = split8<PREC>(re), i = split8<PREC>(im);
    const int base = ((tx * D::T + ti) * 2 + sg) * 2 * PP * 64;
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      c2[base + k * 64 + ln] = r.p[k];
      c2[base + (PP + k) * 64 + ln] = i.p[k];
    }
  }
}

// The two GEMMs of one frame held transposed in LDS (gt, pitch PITCH), scaled
// by sc, for the column tile ty of this wave: |X^T[tx tile][ty tile]|^2 / sc^2
// is added to acc (when active).
template <int N, int PREC>
__device__ __forceinline__ void dft_frame(const float2* gt, float sc, const SplitV<PREC> (&b1r)[DftGeo<N>::KS],
                                          const SplitV<PREC> (&b1i)[DftGeo<N>::KS],
                                          const typename DftPrec<PREC>::V* c2, float (&acc)[DftGeo<N>::T][16],
                                          bool active, int lane) {
  using D = DftGeo<N>;
  constexpr int P = D::PITCH, PP = DftPrec<PREC>::PARTS;
  const int h = lane >> 5, li = lane & 31;
  // stage 1: Y^T[:, ty tile] = G^T . F; yp - yq and yi per row tile
  float16v yp[D::T], yq[D::T], yi[D::T];
#pragma unroll
  for (int ti = 0; ti < D::T; ++ti) {
    yp[ti] = float16v{};
    yq[ti] = float16v{};
    yi[ti] = float16v{};
#pragma unroll
    for (int ks = 0; ks < D::KS; ++ks) {
      float gr[8], gi[8];
      const float2* src = gt + (ti * 32 + li) * P + ks * 16 + 8 * h;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 g = src[e];
        gr[e] = g.x * sc;
        gi[e] = g.y * sc;
      }
      const SplitV<PREC> Ar = split8<PREC>(gr), Ai = split8<PREC>(gi);
      yp[ti] = mfma_split(Ar, b1r[ks], yp[ti]);
      yq[ti] = mfma_split(Ai, b1i[ks], yq[ti]);
      yi[ti] = mfma_split(Ar, b1i[ks], yi[ti]);
      yi[ti] = mfma_split(Ai, b1r[ks], yi[ti]);
    }
  }
  // stage 2: X^T[tx tile, ty tile] = F . Y^T, B operand straight from the
  // stage-1 accumulators (k relabelled as v = 8 sg + e)
  float16v xp[D::T], xq[D::T], xi[D::T];
#pragma unroll
  for (int tx = 0; tx < D::T; ++tx) {
    xp[tx] = float16v{};
    xq[tx] = float16v{};
    xi[tx] = float16v{};
  }
#pragma unroll
  for (int ti = 0; ti < D::T; ++ti)
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      float br[8], bi[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        br[e] = yp[ti][8 * sg + e] - yq[ti][8 * sg + e];
        bi[e] = yi[ti][8 * sg + e];
      }
      const SplitV<PREC> Br = split8<PREC>(br), Bi = split8<PREC>(bi);
#pragma unroll
      for (int tx = 0; tx < D::T; ++tx) {
        const int base = ((tx * D::T + ti) * 2 + sg) * 2 * PP * 64;
        SplitV<PREC> Fr, Fi;
#pragma unroll
        for (int k = 0; k < PP; ++k) {
          Fr.p[k] = c2[base + k * 64 + lane];
          Fi.p[k] = c2[base + (PP + k) * 64 + lane];
        }
        xp[tx] = mfma_split(Fr, Br, xp[tx]);
        xq[tx] = mfma_split(Fi, Bi, xq[tx]);
        xi[tx] = mfma_split(Fr, Bi, xi[tx]);
        xi[tx] = mfma_split(Fi, Br, xi[tx]);
      }
    }
  const float inv = 1.f / (sc * sc);
#pragma unroll
  for (int tx = 0; tx < D::T; ++tx)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float xr = xp[tx][v] - xq[tx][v];
      acc[tx][v] += active ? (xr * xr + xi[tx][v] * xi[tx][v]) * inv : 0.f;
    }
}

// Stage-1 B operand F[k][ky], k = ks 16 + 8 h + e, ky = ty 32 + li, split.
template <int N, int PREC>
__device__ __forceinline__ void dft_stage1_consts(SplitV<PREC> (&b1r)[DftGeo<N>::KS],
                                                  SplitV<PREC> (&b1i)[DftGeo<N>::KS], int ty, int lane) {
  const int h = lane >> 5, li = lane & 31;
#pragma unroll
  for (int ks = 0; ks < DftGeo<N>::KS; ++ks) {
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float2 w = froot((ks * 16 + 8 * h + e) * (ty * 32 + li), N);
      re[e] = w.x;
      im[e] = w.y;
    }
    b1r[ks] = split8<PREC>(re);
    b1i[ks] = split8<PREC>(im);
  }
}

// Power-of-two frame scale (fp16 only): the largest |component| goes to about 64.
__device__ __forceinline__ float frame_scale(float mx) { return mx > 0.f ? exp2f(6.f - ceilf(log2f(mx))) : 1.f; }

__device__ __forceinline__ float wave_max(float mx) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
  return mx;
}

// Frame engine: the frame's waves grid it together (each owns its lanes of a
// 64 x WPF-lane schedule with transposed cell offsets; the largest stored
// value gives the fp16 scale), then every wave runs the two split GEMMs for
// its column tile.
template <int N, int APL, int PREC>
struct DftSmem {
  using D = DftGeo<N>;
  static constexpr int E_OFF = D::FPI * D::FRAME * 8;
  static constexpr int S_OFF = E_OFF + D::FPI * APL * 64 * 8;
  static constexpr int T_OFF = S_OFF + 64;
  static constexpr int C_OFF = T_OFF + kDftTabSlots * D::OWNERS * 8;
  static constexpr int BYTES = C_OFF + D::T * D::T * 2 * 2 * DftPrec<PREC>::PARTS * 64 * 16;
  static_assert(BYTES <= kLdsBytes, "DFT engine LDS");
};

template <int N, int APL, int PREC>
__device__ __forceinline__ void dft_item(const ImageArgs& a, int f, int s, uint8_t* smem) {
  using D = DftGeo<N>;
  using L = DftSmem<N, APL, PREC>;
  float2* lds = reinterpret_cast<float2*>(smem);
  float2* lds_e = reinterpret_cast<float2*>(smem + L::E_OFF);
  float* scale_l = reinterpret_cast<float*>(smem + L::S_OFF);   // [FPI][WPF] partial maxima
  uint2* stab = reinterpret_cast<uint2*>(smem + L::T_OFF);
  auto* c2 = reinterpret_cast<typename DftPrec<PREC>::V*>(smem + L::C_OFF);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = wave / D::WPF;          // frame within the iteration
  const int ty = wave % D::WPF;          // column tile of this wave
  const int owner = ty * 64 + lane;      // gridding / staging lane of the frame
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* gt = lds + fr * D::FRAME;
  float2* epr = lds_e + fr * (APL * 64);

  load_slot_table(stab, a.slots, a.n_slots, D::OWNERS);
  for (int i = tid; i < D::FPI * D::FRAME; i += 256) lds[i] = make_float2(0.f, 0.f);
  dft_stage2_table<N, PREC>(c2, tid);
  SplitV<PREC> b1r[D::KS], b1i[D::KS];
  dft_stage1_consts<N, PREC>(b1r, b1i, ty, lane);
  float acc[D::T][16];
#pragma unroll
  for (int tx = 0; tx < D::T; ++tx)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[tx][v] = 0.f;

  __syncthreads();
  const int64_t iters = (te - tb + D::FPI - 1) / D::FPI;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + it * D::FPI + fr;
    const bool active = t < te;
    // calibrate into the staging area (the frame's waves share it), grid G^T
    const int bpe = efmt_bytes(a.fmt);
    const uint8_t* row = a.efield + ((active ? t : tb) * a.F + f) * int64_t(a.Na) * bpe;
    const float2* urow = a.u + (((active ? t : tb) / a.t_cal) * a.F + f) * int64_t(a.Na);
    for (int an = owner; an < a.Na; an += D::OWNERS)
      epr[an] = active ? cmul(load_sample_global(row, an, a.fmt), gload(urow + an)) : make_float2(0.f, 0.f);
    __syncthreads();
    float mx = 0.f;
    {
      float2 sum = make_float2(0.f, 0.f);
      for (int k = 0; k < a.n_slots; ++k) {
        const uint2 e = stab[k * D::OWNERS + owner];
        const float w = __uint_as_float(e.y);
        const float2 ev = epr[e.x & kSlotAntMask];
        const bool first = int(e.x) < 0;
        sum.x = fmaf(w, ev.x, first ? 0.f : sum.x);
        sum.y = fmaf(w, ev.y, first ? 0.f : sum.y);
        gt[(e.x >> kSlotCellShift) & kSlotCellMask] = sum;
        mx = fmaxf(mx, fmaxf(fabsf(sum.x), fabsf(sum.y)));
      }
    }
    if constexpr (DftPrec<PREC>::SCALE) {
      mx = wave_max(mx);
      if (lane == 0) scale_l[fr * D::WPF + ty] = mx;
    }
    __syncthreads();
    float sc = 1.f;
    if constexpr (DftPrec<PREC>::SCALE) {
      float m = 0.f;
#pragma unroll
      for (int q = 0; q < D::WPF; ++q) m = fmaxf(m, scale_l[fr * D::WPF + q]);
      sc = frame_scale(m);
    }
    dft_frame<N, PREC>(gt, sc, b1r, b1i, c2, acc, active, lane);
    __syncthreads();   // the next frame rewrites every owned cell (the others stay zero)
  }
  __syncthreads();
  // reduce the frames of the workgroup: slot (fr, ty) -> pixels of tiles (tx, ty)
  float* red = reinterpret_cast<float*>(lds);   // [4][T][16][64], frames are done
  static_assert(4 * D::T * 16 * 64 * 4 <= D::FPI * D::FRAME * 8, "reduction area");
#pragma unroll
  for (int tx = 0; tx < D::T; ++tx)
#pragma unroll
    for (int v = 0; v < 16; ++v) red[((wave * D::T + tx) * 16 + v) * 64 + lane] = acc[tx][v];
  __syncthreads();
  float* out = a.partial + (int64_t(s) * a.F + f) * (N * N);
  for (int idx = tid; idx < N * N; idx += 256) {
    const int ky = idx / N, kx = idx % N;
    const int tyy = ky / 32, jl = ky % 32, tx = kx / 32, r = kx % 32;
    // C layout: r = 8 (v/4) + 4 hh + v%4
    const int hh = (r / 4) % 2, v = 4 * (r / 8) + r % 4;
    const int ln = jl + 32 * hh;
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < D::FPI; ++q) sum += red[(((q * D::WPF + tyy) * D::T + tx) * 16 + v) * 64 + ln];
    gstore(out + idx, sum);
  }
  __syncthreads();
}


// ---------------------------------------------------------------------------
// Grids of N = 64 R (R = 2, 4) by residue classes on the matrix cores: class
// c = (cx, cy) of the output, X(R m + c), is the 64 x 64 DFT of the grid
// folded modulo 64 with the phase exp(+2 pi i j.c / N) on every contribution
// (the decomposition of the residue-class FFT engine), and each 64 x 64 DFT
// is the two split GEMMs above.  A workgroup images two classes of the same
// channel (one per frame slot) for all its samples; both waves of a frame
// slot grid its class together from a schedule in the dense class engine's
// format built for 128 owners over all sub-cell columns (sub-cell q owned by
// one lane, its last contribution marked), read from memory, and store the
// folded grid transposed (G^T).
// ---------------------------------------------------------------------------
constexpr int kDftClsMaxAnt = 512;
constexpr int kDftClsOwners = 128;

template <int R, int PREC>
struct DftClsSmem {
  using D = DftGeo<64>;
  static constexpr int N = 64 * R;
  static constexpr int E_OFF = D::FPI * D::FRAME * 8;
  static constexpr int S_OFF = E_OFF + kDftClsMaxAnt * 8;
  static constexpr int W_OFF = S_OFF + 64;
  static constexpr int C_OFF = W_OFF + N * 8;
  static constexpr int BYTES = C_OFF + D::T * D::T * 2 * 2 * DftPrec<PREC>::PARTS * 64 * 16;
  static_assert(BYTES <= kLdsBytes, "DFT class engine LDS");
};

template <int R, int PREC>
__device__ __forceinline__ void dft_cls_item(const ImageArgs& a, int f, int cp, int s, uint8_t* smem) {
  using D = DftGeo<64>;
  using L = DftClsSmem<R, PREC>;
  constexpr int N = 64 * R, P = D::PITCH, OW = kDftClsOwners;
  float2* lds = reinterpret_cast<float2*>(smem);
  float2* epr = reinterpret_cast<float2*>(smem + L::E_OFF);      // shared by both classes (same frame)
  float* scale_l = reinterpret_cast<float*>(smem + L::S_OFF);
  float2* tw = reinterpret_cast<float2*>(smem + L::W_OFF);
  auto* c2 = reinterpret_cast<typename DftPrec<PREC>::V*>(smem + L::C_OFF);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = wave / D::WPF;          // frame slot = class of the pair
  const int ty = wave % D::WPF;
  const int owner = ty * 64 + lane;
  const int c = 2 * cp + fr, cx = c % R, cy = c / R;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* gt = lds + fr * D::FRAME;
  const int S = a.n_slots_c;             // class schedule, all sub-cell columns, OW owners

  for (int i = tid; i < D::FPI * D::FRAME; i += 256) lds[i] = make_float2(0.f, 0.f);
  for (int k = tid; k < N; k += 256) {
    double sn, cs;
    sincospi(2.0 * double(k) / double(N), &sn, &cs);
    tw[k] = make_float2(float(cs), float(sn));
  }
  dft_stage2_table<64, PREC>(c2, tid);
  SplitV<PREC> b1r[D::KS], b1i[D::KS];
  dft_stage1_consts<64, PREC>(b1r, b1i, ty, lane);
  float acc[D::T][16];
#pragma unroll
  for (int tx = 0; tx < D::T; ++tx)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[tx][v] = 0.f;

  __syncthreads();
  for (int64_t t = tb; t < te; ++t) {
    const int bpe = efmt_bytes(a.fmt);
    const uint8_t* row = a.efield + (t * a.F + f) * int64_t(a.Na) * bpe;
    const float2* urow = a.u + ((t / a.t_cal) * a.F + f) * int64_t(a.Na);
    for (int an = tid; an < a.Na; an += 256) epr[an] = cmul(load_sample_global(row, an, a.fmt), gload(urow + an));
    __syncthreads();
    // fold and phase the class: owned sub-cells, stored transposed at their last contribution
    float mx = 0.f;
    {
      float2 sum = make_float2(0.f, 0.f);
      for (int k = 0; k < S; ++k) {
        const uint2 e = gload(a.slots_c + k * OW + owner);
        const uint32_t code = e.x;
        const int qx = (code >> 12) & 63, qy = (code >> 18) & 63;
        const int jx = qx + 64 * int((code >> 24) & 3), jy = qy + 64 * int((code >> 26) & 3);
        const float2 ph = tw[(jx * cx + jy * cy) & (N - 1)];
        const float w = __uint_as_float(e.y);
        const float2 ev = cmul(epr[code & kSlotAntMask], make_float2(w * ph.x, w * ph.y));
        const float keep = int(code) < 0 ? 0.f : 1.f;   // a cell's first contribution restarts the sum
        sum.x = fmaf(sum.x, keep, ev.x);
        sum.y = fmaf(sum.y, keep, ev.y);
        if ((code >> 30) & 1) {
          gt[qx * P + qy] = sum;
          mx = fmaxf(mx, fmaxf(fabsf(sum.x), fabsf(sum.y)));
        }
      }
    }
    if constexpr (DftPrec<PREC>::SCALE) {
      mx = wave_max(mx);
      if (lane == 0) scale_l[fr * D::WPF + ty] = mx;
    }
    __syncthreads();
    float sc = 1.f;
    if constexpr (DftPrec<PREC>::SCALE) {
      float m = 0.f;
#pragma unroll
      for (int q = 0; q < D::WPF; ++q) m = fmaxf(m, scale_l[fr * D::WPF + q]);
      sc = frame_scale(m);
    }
    dft_frame<64, PREC>(gt, sc, b1r, b1i, c2, acc, true, lane);
    __syncthreads();   // the next frame rewrites every owned sub-cell (the others stay zero)
  }
  __syncthreads();
  // each wave owns distinct class pixels: write them straight out
  // (C layout: row r of a 32 x 32 tile = 8 (v / 4) + 4 h + v % 4, column li)
  const int h = lane >> 5, li = lane & 31;
  float* out = a.partial + (int64_t(s) * a.F + f) * (int64_t(N) * N);
#pragma unroll
  for (int tx = 0; tx < D::T; ++tx)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int kx = tx * 32 + 8 * (v / 4) + 4 * h + v % 4;   // C row = kx of X^T
      const int ky = ty * 32 + li;                            // C column = ky
      gstore(out + (R * ky + cy) * N + R * kx + cx, acc[tx][v]);
    }
  __syncthreads();
}

}  // namespace epic
