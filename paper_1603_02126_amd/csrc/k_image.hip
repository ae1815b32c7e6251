// HIP kernels (gfx950) for the EPIC direct-imaging loop with EPICal.
//
// Layout of the imaging engine ("one lane = one pencil"): a wave64 owns
// 64 / N frames of an N x N grid (N <= 64); lane lam of a frame owns grid row
// lam.  Per frame:
//   1. calibrate + grid (Sec. 2.1, E'_a = E_a / g_a and eq. gridding): each
//      lane takes antennas lam, lam + N, ... and scatters w * u * E with LDS
//      float atomics into the frame's zeroed LDS buffer;
//   2. lane lam loads row lam into registers and runs an N-point FFT there;
//   3. the row spectrum is written transposed to LDS (lane-consecutive
//      addresses, conflict free) and lane lam reads back column lam (rows of
//      the buffer are padded by two complex values to spread banks), zeroing
//      the buffer for the next frame as it goes;
//   4. an N-point FFT over the other axis gives X(kx = lam, ky), whose |X|^2
//      is accumulated in registers over all frames of the wave (squaring and
//      time averaging, Sec. 2.1).
// Waves of one workgroup share a channel and split its samples; their
// accumulators are summed through LDS into one partial image per workgroup.
//
// The calibration solve runs in its own kernel before imaging: the tapped
// pixel of interval n only needs the gains of interval n, and its value
// X_t(k0) equals the beamformed sum (1/Na) sum_a A_a(k0) u_a E_a(t) (the
// transform of the gridded field evaluated at one pixel), so the feedback
// recursion costs O(Na) per sample and the O(Ng log Ng) imaging of every
// sample becomes independent work.
#include "engine.h"

namespace epic {

// ---------------------------------------------------------------------------
// Fused imaging kernel
// ---------------------------------------------------------------------------
template <int N, int APL>
__global__ __launch_bounds__(256) void k_image(ImageArgs a) {
  using G = Geo<N>;
  __shared__ float2 lds[G::LDS];
  __shared__ float2 lds_e[G::SLOTS * APL * N];
  __shared__ uint2 stab[Budget<N, APL>::TAB_SLOTS * N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane / N, lam = lane % N;
  const int slot = wave * G::FPW + h;
  const int f = blockIdx.x % a.F;
  const int s = blockIdx.x / a.F;
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
}

// ---------------------------------------------------------------------------
// Imaging of N = 64 R grids (R = 2, 4) by output residue classes.
//
// With k = R m + c and j = 64 p + q (m, q < 64; c, p < R) the transform
// splits into R x R independent 64 x 64 transforms:
//   X(R m + c) = sum_q exp(+2 pi i q.m / 64) H_c(q),
//   H_c(q)    = sum_{j = q mod 64} G(j) exp(+2 pi i j.c / N)
// so class c is the 64 x 64 engine applied to the grid folded modulo 64 with
// the phase exp(+2 pi i j.c / N) on every contribution.  One wave owns one
// class; the four waves of a workgroup image four classes of the same frame
// from one shared E' staging area (one barrier per frame), and each class
// writes its own interleaved subset of the partial image.
// Slot code: antenna | qx << 12 | qy << 18 | px << 24 | py << 26 | valid << 30
//            | first << 31.
// ---------------------------------------------------------------------------
constexpr int kClsMaxAnt = 512;
constexpr int kClsTabSlots =
    (kLdsBytes - 4 * Geo<64>::FRAME * 8 - 2 * kClsMaxAnt * 8 - 256 * 8) / (64 * 8);

template <int R>
__global__ __launch_bounds__(256) void k_image_cls(ImageArgs a) {
  constexpr int N = 64 * R, CG = (R * R) / 4;
  using G = Geo<64>;
  constexpr int P = G::PITCH;
  __shared__ float2 lds[4 * G::FRAME];
  __shared__ float2 epr_l[2][kClsMaxAnt];
  __shared__ float2 tw[N];
  __shared__ uint2 stab[kClsTabSlots * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = blockIdx.x % a.F;
  const int rest = blockIdx.x / a.F;
  const int cg = rest % CG, s = rest / CG;
  const int c = cg * 4 + wave, cx = c % R, cy = c / R;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* buf = lds + wave * G::FRAME;

  load_slot_table(stab, a.slots, a.n_slots, 64);
  for (int k = tid; k < N; k += 256) {
    double sn, cs;
    sincospi(2.0 * double(k) / double(N), &sn, &cs);
    tw[k] = make_float2(float(cs), float(sn));
  }
  static_for<0, 64>([&](auto xc) { buf[lane * P + decltype(xc)::value] = make_float2(0.f, 0.f); });
  float acc[64];
  static_for<0, 64>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });

  // antennas staged by this thread: tid and tid + 256
  Raw raw[2];
  float2 uu[2];
  auto fetch = [&](int64_t t, bool active) {
    const int bpe = a.fmt == kCF32 ? 8 : a.fmt == kCI8 ? 2 : 1;
    const uint8_t* row = a.efield + (t * a.F + f) * int64_t(a.Na) * bpe;
    const float2* urow = a.u + ((t / a.t_cal) * a.F + f) * int64_t(a.Na);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
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
    float2* epr = epr_l[(t - tb) & 1];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
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
    wave_lds_sync();
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
}

// ---------------------------------------------------------------------------
// Stage-wise gridding to HBM (one frame per lane group; tables read from
// memory: this is the debugging path, not the timed one)
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_grid(GridArgs a) {
  using G = Geo<N>;
  __shared__ float2 lds[G::LDS];
  __shared__ float2 lds_e[G::SLOTS * 8 * N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane / N, lam = lane % N;
  const int slot = wave * G::FPW + h;
  const int64_t q = int64_t(blockIdx.x) * G::SLOTS + slot;  // frame = t * F + f
  const bool active = q < int64_t(a.nt) * a.F;
  float2* buf = lds + slot * G::FRAME;
  float2* epr = lds_e + slot * (8 * N);
  static_for<0, N>([&](auto xc) { buf[lam * G::PITCH + decltype(xc)::value] = make_float2(0.f, 0.f); });
  const int64_t t = active ? q / a.F : 0;
  const int f = active ? int(q % a.F) : 0;
  const int bpe = efmt_bytes(a.fmt);
  const uint8_t* row = a.efield + ((a.t0 + t) * a.F + f) * int64_t(a.Na) * bpe;
  for (int an = lam; an < a.Na; an += N)
    epr[an] = active ? cmul(load_sample(row, an, a.fmt), a.u[int64_t(f) * a.Na + an]) : make_float2(0.f, 0.f);
  wave_lds_sync();
  grid_frame(buf, epr, a.slots, a.n_slots, N, lam);
  wave_lds_sync();
  if (active) {
    float2* out = a.grid + q * (N * N);
    static_for<0, N>([&](auto yc) {
      constexpr int y = decltype(yc)::value;
      out[y * N + lam] = buf[y * G::PITCH + lam];
    });
  }
}

// ---------------------------------------------------------------------------
// Stage-wise transform + square + accumulate (+ tap) from HBM grids
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_image_acc(ImageAccArgs a) {
  using G = Geo<N>;
  __shared__ float2 lds[G::LDS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane / N, lam = lane % N;
  const int slot = wave * G::FPW + h;
  const int f = blockIdx.x;
  float2* buf = lds + slot * G::FRAME;
  const int kx0 = a.k0 ? a.k0[2 * f] : 0, ky0 = a.k0 ? a.k0[2 * f + 1] : 0;
  float acc[N];
  static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });
  const int iters = (a.nt + G::SLOTS - 1) / G::SLOTS;
  for (int it = 0; it < iters; ++it) {
    const int t = it * G::SLOTS + slot;
    const bool active = t < a.nt;
    float2 v[N];
    const float2* row = a.grid + ((int64_t(active ? t : 0) * a.F + f) * N + lam) * N;
    static_for<0, N>([&](auto xc) {
      constexpr int x = decltype(xc)::value;
      v[x] = active ? row[x] : make_float2(0.f, 0.f);
    });
    wave_lds_sync();
    static_for<0, N>([&](auto xc) { buf[lam * G::PITCH + decltype(xc)::value] = v[decltype(xc)::value]; });
    wave_lds_sync();
    transform_frame<N, +1>(buf, v, lam);
    static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] += cnorm(v[decltype(yc)::value]); });
    if (a.tap && active && lam == kx0) {
      float2 p = make_float2(0.f, 0.f);
      static_for<0, N>([&](auto yc) {
        if (decltype(yc)::value == ky0) p = v[decltype(yc)::value];
      });
      a.tap[int64_t(t) * a.F + f] = cscale(p, a.inv_na);
    }
  }
  __syncthreads();
  float* red = reinterpret_cast<float*>(lds);
  static_for<0, N>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    red[(slot * N + y) * N + lam] = acc[y];
  });
  __syncthreads();
  const float s2 = a.inv_na * a.inv_na;
  float* img = a.image + int64_t(f) * N * N;
  for (int idx = threadIdx.x; idx < N * N; idx += 256) {
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < G::SLOTS; ++q) sum += red[q * N * N + idx];
    img[idx] += sum * s2;
  }
}

// ---------------------------------------------------------------------------
// Partial-image reduction (FP64 sum over splits)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(const float* partial, int splits, int64_t per_split,
                                                double scale, float* image) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= per_split) return;
  double s = 0.0;
  for (int k = 0; k < splits; ++k) s += double(partial[int64_t(k) * per_split + i]);
  image[i] = float(s * scale);
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int grid_lanes(int N) { return N; }
int grid_pitch(int N) { return N + 2; }

int cls_table_slots() { return kClsTabSlots; }

bool image_supported(int N, int na, int n_slots) {
  if (N == 128 || N == 256) return na <= kClsMaxAnt && n_slots <= kClsTabSlots;
  if (!(N == 16 || N == 32 || N == 64) || na > 8 * N) return false;
  const int apl = apl_for(N, na);
  return apl != 0 && n_slots <= tab_slots_for(N, apl);
}

template <int N, int APL>
struct LaunchImage {
  static hipError_t run(const ImageArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_image<N, APL>), dim3(a.F * a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
  }
};

hipError_t launch_image(int N, const ImageArgs& a, hipStream_t s) {
  if (N == 128) {
    hipLaunchKernelGGL((k_image_cls<2>), dim3(a.F * 1 * a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (N == 256) {
    hipLaunchKernelGGL((k_image_cls<4>), dim3(a.F * 4 * a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  return dispatch_n<LaunchImage>(N, a.Na, a, s);
}

hipError_t launch_grid(int N, const GridArgs& a, hipStream_t s) {
  if (a.nt == 0) return hipSuccess;
  const int64_t frames = int64_t(a.nt) * a.F;
  const int slots = 4 * (64 / N);
  const dim3 grid(unsigned((frames + slots - 1) / slots));
  if (N == 16) hipLaunchKernelGGL((k_grid<16>), grid, dim3(256), 0, s, a);
  else if (N == 32) hipLaunchKernelGGL((k_grid<32>), grid, dim3(256), 0, s, a);
  else if (N == 64) hipLaunchKernelGGL((k_grid<64>), grid, dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_image_acc(int N, const ImageAccArgs& a, hipStream_t s) {
  if (a.nt == 0) return hipSuccess;
  if (N == 16) hipLaunchKernelGGL((k_image_acc<16>), dim3(a.F), dim3(256), 0, s, a);
  else if (N == 32) hipLaunchKernelGGL((k_image_acc<32>), dim3(a.F), dim3(256), 0, s, a);
  else if (N == 64) hipLaunchKernelGGL((k_image_acc<64>), dim3(a.F), dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_reduce(const float* partial, int splits, int64_t per_split, double scale, float* image,
                         hipStream_t s) {
  const int64_t blocks = (per_split + 255) / 256;
  hipLaunchKernelGGL(k_reduce, dim3(unsigned(blocks)), dim3(256), 0, s, partial, splits, per_split, scale,
                     image);
  return hipGetLastError();
}

}  // namespace epic
