// HIP kernels (gfx950): 2D DFT as two complex GEMMs on the matrix cores, with
// split-precision FP16 operands and FP32 accumulation (grids of 32 and 64).
//
// Per frame, with F[j][k] = exp(+2 pi i j k / N) (symmetric):
//   stage 1   Y^T = G^T F      (Y^T[jx][ky] = sum_jy G[jy][jx] F[jy][ky])
//   stage 2   X^T = F Y^T      (X^T[kx][ky] = sum_jx F[kx][jx] Y^T[jx][ky])
// so X[ky][kx] = sum_j G[jy][jx] exp(+2 pi i (jx kx + jy ky) / N), the
// unnormalised image transform of Sec. 2.1.  Every real operand x is split
// x = hi + lo with hi = fp16(x), lo = fp16(x - hi); a real product is
// hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-22 relative, is dropped); a
// complex product takes four real ones.  The FP32 accumulator tile of stage 1
// is already laid out as the B operand of stage 2 once the contraction index
// is relabelled the same way in both operands, so Y never leaves registers.
// Each frame is scaled by a power of two before the split (the scale is
// exact and divided out of |X|^2) so that fp16 neither overflows nor loses
// the lo part.
//
// MFMA v_mfma_f32_32x32x16_f16 lane layout (lane l, h = l / 32):
//   A[i][k]: i = l % 32, k = 8 h + e        (e = element 0..7 of the half8)
//   B[k][j]: j = l % 32, k = 8 h + e
//   C[i][j]: j = l % 32, i = 8 (v / 4) + 4 h + v % 4   (v = 0..15)
#pragma once
#include "engine.h"

namespace epic {


constexpr int kDftTabSlots = 32;   // gridding slot rows held in LDS

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float16v mfma(half8 a, half8 b, float16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// hi/lo split of 8 floats.
struct Split8 {
  half8 hi, lo;
};
__device__ __forceinline__ Split8 split8(const float (&x)[8], float sgn) {
  Split8 s;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float v = sgn * x[e];
    const _Float16 h = _Float16(v);
    s.hi[e] = h;
    s.lo[e] = _Float16(v - float(h));
  }
  return s;
}

// acc += a * b with split operands (3 products).
__device__ __forceinline__ float16v mfma3(const Split8& a, const Split8& b, float16v acc) {
  acc = mfma(a.hi, b.hi, acc);
  acc = mfma(a.hi, b.lo, acc);
  acc = mfma(a.lo, b.hi, acc);
  return acc;
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
  static constexpr int PITCH = N + 2;        // complex values per G^T row in LDS
  static constexpr int FRAME = N * PITCH;
  static constexpr int KS = N / 16;          // k-steps of stage 1
};

// Frame engine: gridding by the frame's lead wave (slot schedule with
// transposed cell offsets), then the two split-precision GEMMs.
template <int N, int APL>
struct DftSmem {
  using D = DftGeo<N>;
  static constexpr int E_OFF = D::FPI * D::FRAME * 8;
  static constexpr int S_OFF = E_OFF + D::FPI * APL * 64 * 8;
  static constexpr int T_OFF = S_OFF + 16;
  static constexpr int C_OFF = T_OFF + kDftTabSlots * 64 * 8;
  static constexpr int BYTES = C_OFF + D::T * D::T * 2 * 2 * 2 * 64 * 16;
};

template <int N, int APL>
__device__ __forceinline__ void dft_item(const ImageArgs& a, int f, int s, uint8_t* smem) {
  using D = DftGeo<N>;
  using L = DftSmem<N, APL>;
  constexpr int P = D::PITCH;
  float2* lds = reinterpret_cast<float2*>(smem);
  float2* lds_e = reinterpret_cast<float2*>(smem + L::E_OFF);
  float* scale_l = reinterpret_cast<float*>(smem + L::S_OFF);
  uint2* stab = reinterpret_cast<uint2*>(smem + L::T_OFF);
  // stage-2 A operand F[kx][k] in lane order: [tx][ti][sg][re/im][hi/lo][lane]
  half8* c2 = reinterpret_cast<half8*>(smem + L::C_OFF);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, li = lane & 31;
  const int fr = wave / D::WPF;          // frame within the iteration
  const int ty = wave % D::WPF;          // column tile of this wave
  const bool lead = ty == 0;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* gt = lds + fr * D::FRAME;
  float2* epr = lds_e + fr * (APL * 64);

  load_slot_table(stab, a.slots, a.n_slots, 64);
  for (int i = tid; i < D::FPI * D::FRAME; i += 256) lds[i] = make_float2(0.f, 0.f);
  // kx = tx*32 + li, k = ti*32 + 16 sg + 8 (e/4) + 4h + e%4 (the stage-1 C-row order)
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
    const Split8 r = split8(re, 1.f), i = split8(im, 1.f);
    const int base = ((tx * D::T + ti) * 2 + sg) * 4 * 64;
    c2[base + 0 * 64 + ln] = r.hi;
    c2[base + 1 * 64 + ln] = r.lo;
    c2[base + 2 * 64 + ln] = i.hi;
    c2[base + 3 * 64 + ln] = i.lo;
  }

  // constants: stage-1 B operand F[k][ky], k = ks*16 + 8h + e, ky = ty*32 + li
  Split8 b1r[D::KS], b1i[D::KS];
#pragma unroll
  for (int ks = 0; ks < D::KS; ++ks) {
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float2 w = froot((ks * 16 + 8 * h + e) * (ty * 32 + li), N);
      re[e] = w.x;
      im[e] = w.y;
    }
    b1r[ks] = split8(re, 1.f);
    b1i[ks] = split8(im, 1.f);
  }
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
    if (lead) {
      // calibrate into the staging area, then grid G^T (owned cells only)
      const int bpe = efmt_bytes(a.fmt);
      const uint8_t* row = a.efield + ((active ? t : tb) * a.F + f) * int64_t(a.Na) * bpe;
      const float2* urow = a.u + (((active ? t : tb) / a.t_cal) * a.F + f) * int64_t(a.Na);
#pragma unroll
      for (int i = 0; i < APL; ++i) {
        const int an = lane + 64 * i;
        if (an < a.Na) epr[an] = active ? cmul(load_sample_global(row, an, a.fmt), gload(urow + an)) : make_float2(0.f, 0.f);
      }
      wave_lds_sync();
      grid_frame(gt, epr, stab, a.n_slots, 64, lane);
      wave_lds_sync();
      // per-frame power-of-two scale: max |component| -> about 64
      float mx = 0.f;
      for (int i = lane; i < N * N; i += 64) {
        const float2 g = gt[(i / N) * P + (i % N)];
        mx = fmaxf(mx, fmaxf(fabsf(g.x), fabsf(g.y)));
      }
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
      if (lane == 0) scale_l[fr] = mx > 0.f ? exp2f(6.f - ceilf(log2f(mx))) : 1.f;
    }
    __syncthreads();
    const float sc = scale_l[fr];
    // stage 1: Y^T[:, ty tile] = G^T . F, one accumulator pair per row tile ti
    float16v yr[D::T], yi[D::T];
#pragma unroll
    for (int ti = 0; ti < D::T; ++ti) {
      yr[ti] = float16v{};
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
        const Split8 Ar = split8(gr, 1.f), Ai = split8(gi, 1.f), An = split8(gi, -1.f);
        yr[ti] = mfma3(Ar, b1r[ks], yr[ti]);
        yr[ti] = mfma3(An, b1i[ks], yr[ti]);
        yi[ti] = mfma3(Ar, b1i[ks], yi[ti]);
        yi[ti] = mfma3(Ai, b1r[ks], yi[ti]);
      }
    }
    // stage 2: X^T[tx tile, ty tile] = F . Y^T, B operand straight from the
    // stage-1 accumulators (k relabelled as v = 8 sg + e)
    float16v xr[D::T], xi[D::T];
#pragma unroll
    for (int tx = 0; tx < D::T; ++tx) {
      xr[tx] = float16v{};
      xi[tx] = float16v{};
    }
#pragma unroll
    for (int ti = 0; ti < D::T; ++ti)
#pragma unroll
      for (int sg = 0; sg < 2; ++sg) {
        float br[8], bi[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          br[e] = yr[ti][8 * sg + e];
          bi[e] = yi[ti][8 * sg + e];
        }
        const Split8 Br = split8(br, 1.f), Bi = split8(bi, 1.f), Bn = split8(bi, -1.f);
#pragma unroll
        for (int tx = 0; tx < D::T; ++tx) {
          const int base = ((tx * D::T + ti) * 2 + sg) * 4 * 64;
          const Split8 Fr{c2[base + 0 * 64 + lane], c2[base + 1 * 64 + lane]};
          const Split8 Fi{c2[base + 2 * 64 + lane], c2[base + 3 * 64 + lane]};
          xr[tx] = mfma3(Fr, Br, xr[tx]);
          xr[tx] = mfma3(Fi, Bn, xr[tx]);
          xi[tx] = mfma3(Fr, Bi, xi[tx]);
          xi[tx] = mfma3(Fi, Br, xi[tx]);
        }
      }
    const float inv = 1.f / (sc * sc);
#pragma unroll
    for (int tx = 0; tx < D::T; ++tx)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        acc[tx][v] += active ? (xr[tx][v] * xr[tx][v] + xi[tx][v] * xi[tx][v]) * inv : 0.f;
    __syncthreads();
  }
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
// is the two split-precision GEMMs above.  A workgroup images two classes
// of the same channel (one per frame slot) for all its samples.  The slot
// table is the residue-class schedule (sub-cell q owned by one lane); the
// folded grid is stored transposed (G^T) for stage 1.
// ---------------------------------------------------------------------------
constexpr int kDftClsMaxAnt = 512;

template <int R>
struct DftClsSmem {
  using D = DftGeo<64>;
  static constexpr int N = 64 * R;
  static constexpr int E_OFF = D::FPI * D::FRAME * 8;
  static constexpr int S_OFF = E_OFF + D::FPI * kDftClsMaxAnt * 8;
  static constexpr int W_OFF = S_OFF + 16;
  static constexpr int T_OFF = W_OFF + N * 8;
  static constexpr int C_OFF = T_OFF + kDftTabSlots * 64 * 8;
  static constexpr int BYTES = C_OFF + D::T * D::T * 2 * 2 * 2 * 64 * 16;
};

template <int R>
__device__ __forceinline__ void dft_cls_item(const ImageArgs& a, int f, int cp, int s, uint8_t* smem) {
  using D = DftGeo<64>;
  using L = DftClsSmem<R>;
  constexpr int N = 64 * R, P = D::PITCH;
  float2* lds = reinterpret_cast<float2*>(smem);
  float2* lds_e = reinterpret_cast<float2*>(smem + L::E_OFF);
  float* scale_l = reinterpret_cast<float*>(smem + L::S_OFF);
  float2* tw = reinterpret_cast<float2*>(smem + L::W_OFF);
  uint2* stab = reinterpret_cast<uint2*>(smem + L::T_OFF);
  half8* c2 = reinterpret_cast<half8*>(smem + L::C_OFF);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, li = lane & 31;
  const int fr = wave / D::WPF;          // frame slot = class of the pair
  const int ty = wave % D::WPF;
  const bool lead = ty == 0;
  const int c = 2 * cp + fr, cx = c % R, cy = c / R;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* gt = lds + fr * D::FRAME;
  float2* epr = lds_e + fr * kDftClsMaxAnt;

  load_slot_table(stab, a.slots, a.n_slots, 64);
  for (int i = tid; i < D::FPI * D::FRAME; i += 256) lds[i] = make_float2(0.f, 0.f);
  for (int k = tid; k < N; k += 256) {
    double sn, cs;
    sincospi(2.0 * double(k) / double(N), &sn, &cs);
    tw[k] = make_float2(float(cs), float(sn));
  }
  for (int q = tid; q < D::T * D::T * 2 * 64; q += 256) {
    const int ln = q % 64, sg = (q / 64) % 2, ti = (q / 128) % D::T, tx = q / (128 * D::T);
    const int hh = ln >> 5, ll = ln & 31;
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = ti * 32 + 16 * sg + 8 * (e / 4) + 4 * hh + (e % 4);
      const float2 w = froot((tx * 32 + ll) * k, 64);
      re[e] = w.x;
      im[e] = w.y;
    }
    const Split8 r = split8(re, 1.f), i = split8(im, 1.f);
    const int base = ((tx * D::T + ti) * 2 + sg) * 4 * 64;
    c2[base + 0 * 64 + ln] = r.hi;
    c2[base + 1 * 64 + ln] = r.lo;
    c2[base + 2 * 64 + ln] = i.hi;
    c2[base + 3 * 64 + ln] = i.lo;
  }
  Split8 b1r[D::KS], b1i[D::KS];
#pragma unroll
  for (int ks = 0; ks < D::KS; ++ks) {
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float2 w = froot((ks * 16 + 8 * h + e) * (ty * 32 + li), 64);
      re[e] = w.x;
      im[e] = w.y;
    }
    b1r[ks] = split8(re, 1.f);
    b1i[ks] = split8(im, 1.f);
  }
  float acc[D::T][16];
#pragma unroll
  for (int tx = 0; tx < D::T; ++tx)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[tx][v] = 0.f;

  __syncthreads();
  for (int64_t t = tb; t < te; ++t) {
    if (lead) {
      const int bpe = efmt_bytes(a.fmt);
      const uint8_t* row = a.efield + (t * a.F + f) * int64_t(a.Na) * bpe;
      const float2* urow = a.u + ((t / a.t_cal) * a.F + f) * int64_t(a.Na);
      for (int an = lane; an < a.Na; an += 64) epr[an] = cmul(load_sample_global(row, an, a.fmt), gload(urow + an));
      wave_lds_sync();
      // fold and phase the class: owned sub-cells, transposed layout
      float2 sum = make_float2(0.f, 0.f);
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
        const int off = (code >> 30) & 1 ? qx * P + qy : 64;
        gt[off] = sum;
      }
      wave_lds_sync();
      float mx = 0.f;
      for (int i = lane; i < 64 * 64; i += 64) {
        const float2 g = gt[(i / 64) * P + (i % 64)];
        mx = fmaxf(mx, fmaxf(fabsf(g.x), fabsf(g.y)));
      }
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
      if (lane == 0) scale_l[fr] = mx > 0.f ? exp2f(6.f - ceilf(log2f(mx))) : 1.f;
    }
    __syncthreads();
    const float sc = scale_l[fr];
    float16v yr[D::T], yi[D::T];
#pragma unroll
    for (int ti = 0; ti < D::T; ++ti) {
      yr[ti] = float16v{};
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
        const Split8 Ar = split8(gr, 1.f), Ai = split8(gi, 1.f), An = split8(gi, -1.f);
        yr[ti] = mfma3(Ar, b1r[ks], yr[ti]);
        yr[ti] = mfma3(An, b1i[ks], yr[ti]);
        yi[ti] = mfma3(Ar, b1i[ks], yi[ti]);
        yi[ti] = mfma3(Ai, b1r[ks], yi[ti]);
      }
    }
    float16v xr[D::T], xi[D::T];
#pragma unroll
    for (int tx = 0; tx < D::T; ++tx) {
      xr[tx] = float16v{};
      xi[tx] = float16v{};
    }
#pragma unroll
    for (int ti = 0; ti < D::T; ++ti)
#pragma unroll
      for (int sg = 0; sg < 2; ++sg) {
        float br[8], bi[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          br[e] = yr[ti][8 * sg + e];
          bi[e] = yi[ti][8 * sg + e];
        }
        const Split8 Br = split8(br, 1.f), Bi = split8(bi, 1.f), Bn = split8(bi, -1.f);
#pragma unroll
        for (int tx = 0; tx < D::T; ++tx) {
          const int base = ((tx * D::T + ti) * 2 + sg) * 4 * 64;
          const Split8 Fr{c2[base + 0 * 64 + lane], c2[base + 1 * 64 + lane]};
          const Split8 Fi{c2[base + 2 * 64 + lane], c2[base + 3 * 64 + lane]};
          xr[tx] = mfma3(Fr, Br, xr[tx]);
          xr[tx] = mfma3(Fi, Bn, xr[tx]);
          xi[tx] = mfma3(Fr, Bi, xi[tx]);
          xi[tx] = mfma3(Fi, Br, xi[tx]);
        }
      }
    const float inv = 1.f / (sc * sc);
#pragma unroll
    for (int tx = 0; tx < D::T; ++tx)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tx][v] += (xr[tx][v] * xr[tx][v] + xi[tx][v] * xi[tx][v]) * inv;
    __syncthreads();
  }
  // each wave owns distinct class pixels: write them straight out
  // (C layout: row r of a 32 x 32 tile = 8 (v / 4) + 4 h + v % 4, column li)
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
