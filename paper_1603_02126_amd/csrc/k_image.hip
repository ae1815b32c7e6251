// HIP kernels (gfx950) for the EPIC direct-imaging loop with EPICal.
//
// Layout of the imaging engine ("one lane = one pencil"): a wave64 owns
// 64 / N frames of an N x N grid (N <= 64); lane lam of a frame owns grid row
// lam.  Per frame:
//   1. calibrate + grid (Sec. 2.1, E'_a = E_a / g_a and eq. gridding): each
//      lane stages antennas lam, lam + N, ... as E' in LDS, then sums the
//      contributions of the grid cells it owns (a fixed schedule built on the
//      host) and stores them into the frame's LDS buffer;
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
#include "image_cls.h"
#include "image_fft.h"

namespace epic {

// ---------------------------------------------------------------------------
// Fused imaging kernel
// ---------------------------------------------------------------------------
template <int N, int APL>
__global__ __launch_bounds__(256) void k_image(ImageArgs a) {
  __shared__ __align__(16) uint8_t smem[FftSmem<N, APL>::BYTES];
  image_item<N, APL>(a, blockIdx.x % a.F, blockIdx.x / a.F, smem);
}

template <int APL, int FMT>
__global__ __launch_bounds__(kPairThreads) void k_image_pair(ImageArgs a) {
  static_assert(APL == 2 || APL == 4, "instantiated for the register budget checked at two and four antennas per lane");
  __shared__ __align__(16) uint8_t smem[PairSmem<APL>::BYTES];
  image_item_pair<APL, FMT>(a, blockIdx.x % a.F, blockIdx.x / a.F, smem);
}

// Snapshot forms (one image per window of t_acc samples).
template <int N, int APL>
__global__ __launch_bounds__(256) void k_image_snap(ImageArgs a) {
  __shared__ __align__(16) uint8_t smem[FftSmem<N, APL>::BYTES];
  image_item_snap<N, APL>(a, blockIdx.x % a.F, blockIdx.x / a.F, smem);
}

template <int APL, int FMT>
__global__ __launch_bounds__(kPairThreads) void k_image_pair_snap(ImageArgs a) {
  static_assert(APL == 2 || APL == 4, "instantiated for the register budget checked at two and four antennas per lane");
  __shared__ __align__(16) uint8_t smem[PairSmem<APL>::BYTES];
  image_item_pair_snap<APL, FMT>(a, blockIdx.x % a.F, blockIdx.x / a.F, smem);
}

template <int APL, int FMT>
__global__ __launch_bounds__(kPairThreads) void k_image_pair_snap_group(ImageArgs a) {
  static_assert(APL == 2 || APL == 4, "instantiated for the register budget checked at two and four antennas per lane");
  __shared__ __align__(16) uint8_t smem[PairSmem<APL>::BYTES];
  image_item_pair_snap_group<APL, FMT>(a, blockIdx.x % a.F, blockIdx.x / a.F, smem);
}

template <int R>
__global__ __launch_bounds__(256) void k_image_cls(ImageArgs a) {
  __shared__ __align__(16) uint8_t smem[ClsSmem<R, false>::BYTES];
  constexpr int CG = (R * R) / 4;
  const int rest = blockIdx.x / a.F;
  image_cls_item<R, false>(a, blockIdx.x % a.F, rest % CG, rest / CG, smem);
}

template <int R, int FMT, bool DB>
__global__ __launch_bounds__(kClsPairThreads) void k_image_cls_pair(ImageArgs a) {
  __shared__ __align__(16) uint8_t smem[ClsPairSmem<R, DB>::BYTES];
  constexpr int CG = (R * R) / 4;
  const int rest = blockIdx.x / a.F;
  image_cls_pair_item<R, FMT, DB>(a, blockIdx.x % a.F, rest % CG, rest / CG, smem);
}

template <int R, int FMT, int GB>
__global__ __launch_bounds__(kClsDenseThreads) void k_image_cls_dense(ImageArgs a) {
  __shared__ __align__(16) uint8_t smem[ClsDenseSmem<R>::BYTES];
  constexpr int CG = (R * R) / ClsDenseSmem<R>::CPW;
  const int rest = blockIdx.x / a.F;
  image_cls_dense_item<R, FMT, GB>(a, blockIdx.x % a.F, rest % CG, rest / CG, smem);
}

template <int R>
__global__ __launch_bounds__(256) void k_image_cls_big(ImageArgs a) {
  __shared__ __align__(16) uint8_t smem[ClsSmem<R, true>::BYTES];
  constexpr int CG = (R * R) / 4;
  const int rest = blockIdx.x / a.F;
  image_cls_item<R, true>(a, blockIdx.x % a.F, rest % CG, rest / CG, smem);
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
    add_norms<N>(acc, v);
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
// Integer E-field samples decoded by the imaging path's own unpacking
// (load_raw_global + unpack_raw), written as int16 (re, im) pairs
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_unpack(const uint8_t* efield, int64_t n, int fmt, short2* out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const float2 v = unpack_raw(load_raw_global(efield + i * efmt_bytes(fmt), 0, fmt), fmt);
  out[i] = make_short2(short(v.x), short(v.y));
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_unpack(const uint8_t* efield, int64_t n, int fmt, int16_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (fmt != kCI4 && fmt != kCI8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_unpack, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, efield, n, fmt,
                     reinterpret_cast<short2*>(out));
  return hipGetLastError();
}

int grid_lanes(int N) { return N; }
int grid_pitch(int N) { return N + 2; }

int cls_table_slots() { return kClsTabSlots; }

// 1: slot table in LDS, 2: dense-array variant, 0: unsupported
int cls_variant(int na, int n_slots) {
  if (na <= kClsMaxAnt && n_slots <= kClsTabSlots) return 1;
  return na <= kClsMaxAntBig ? 2 : 0;
}

bool image_supported(int N, int na, int n_slots) {
  if (N == 128 || N == 256) return cls_variant(na, n_slots) != 0;
  if (!(N == 16 || N == 32 || N == 64) || na > 8 * N) return false;
  const int apl = apl_for(N, na);
  return apl != 0 && n_slots <= tab_slots_for(N, apl);
}

// The paired 64 x 64 engine: integer E-fields, up to 256 antennas (two or
// four per lane: the register budget of two waves per SIMD is checked
// there), and a half-frame schedule that fits its LDS table.
bool pair_engine(const ImageArgs& a, int N) {
  const int apl = apl_for(N, a.Na);
  return N == 64 && a.fmt != kCF32 && (apl == 2 || apl == 4) && a.slots_h != nullptr &&
         a.n_slots_h0 + a.n_slots_h1 <= (apl == 2 ? PairSmem<2>::TAB_SLOTS : PairSmem<4>::TAB_SLOTS);
}

template <int N, int APL>
struct LaunchImage {
  static hipError_t run(const ImageArgs& a, hipStream_t s) {
    if constexpr (N == 64 && (APL == 2 || APL == 4)) {
      if (pair_engine(a, N)) {
        if (a.fmt == kCI4) hipLaunchKernelGGL((k_image_pair<APL, kCI4>), dim3(a.F * a.splits), dim3(kPairThreads), 0, s, a);
        else hipLaunchKernelGGL((k_image_pair<APL, kCI8>), dim3(a.F * a.splits), dim3(kPairThreads), 0, s, a);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_image<N, APL>), dim3(a.F * a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
  }
};

// The residue-class engine with two waves per SIMD: integer E-fields, at
// most 512 antennas, half-frame schedules that fit its LDS table; with at
// most kClsPairMaxAntDB antennas and a table that still fits, its
// double-buffered form (one barrier per pair of samples).
bool cls_pair_db(const ImageArgs& a, int N) {
  const int cap = N == 128 ? ClsPairSmem<2, true>::TAB_SLOTS : ClsPairSmem<4, true>::TAB_SLOTS;
  return a.Na <= kClsPairMaxAntDB && a.n_slots_h0 + a.n_slots_h1 <= cap;
}

bool cls_pair_engine(const ImageArgs& a, int N) {
  if (!(N == 128 || N == 256) || a.fmt == kCF32 || a.Na > kClsMaxAnt || !a.slots_h || a.grid_batch != 0)
    return false;
  const int cap = N == 128 ? ClsPairSmem<2>::TAB_SLOTS : ClsPairSmem<4>::TAB_SLOTS;
  return a.n_slots_h0 + a.n_slots_h1 <= cap;
}

// The dense residue-class engine with two waves per SIMD: integer E-fields,
// up to 2048 antennas at 256 x 256 and 1024 at 128 x 128 (its E' staging of
// one or two frames); by default the arrays the class-pair engine does not
// take, any of them when a gridding batch is chosen (grid_batch 2 or 4).
bool cls_dense_engine(const ImageArgs& a, int N) {
  if (!(N == 128 || N == 256) || a.fmt == kCF32 || !a.slots_m || cls_pair_engine(a, N)) return false;
  return a.Na <= (N == 256 ? ClsDenseSmem<4>::MAXA : ClsDenseSmem<2>::MAXA);
}

int cls_groups(const ImageArgs& a, int N) {
  if (N == 256) return cls_dense_engine(a, N) ? 16 / ClsDenseSmem<4>::CPW : 4;
  return 1;
}

hipError_t launch_image(int N, const ImageArgs& a, hipStream_t s) {
  if (N == 128 || N == 256) {
    const bool big = cls_variant(a.Na, a.n_slots) == 2;
    const dim3 grid(a.F * cls_groups(a, N) * a.splits);
    if (cls_dense_engine(a, N)) {
      const dim3 blk(kClsDenseThreads);
      if (a.grid_batch == 4) {
        if (N == 128 && a.fmt == kCI4) hipLaunchKernelGGL((k_image_cls_dense<2, kCI4, 4>), grid, blk, 0, s, a);
        else if (N == 128) hipLaunchKernelGGL((k_image_cls_dense<2, kCI8, 4>), grid, blk, 0, s, a);
        else if (a.fmt == kCI4) hipLaunchKernelGGL((k_image_cls_dense<4, kCI4, 4>), grid, blk, 0, s, a);
        else hipLaunchKernelGGL((k_image_cls_dense<4, kCI8, 4>), grid, blk, 0, s, a);
      } else {
        if (N == 128 && a.fmt == kCI4) hipLaunchKernelGGL((k_image_cls_dense<2, kCI4, 2>), grid, blk, 0, s, a);
        else if (N == 128) hipLaunchKernelGGL((k_image_cls_dense<2, kCI8, 2>), grid, blk, 0, s, a);
        else if (a.fmt == kCI4) hipLaunchKernelGGL((k_image_cls_dense<4, kCI4, 2>), grid, blk, 0, s, a);
        else hipLaunchKernelGGL((k_image_cls_dense<4, kCI8, 2>), grid, blk, 0, s, a);
      }
      return hipGetLastError();
    }
    if (cls_pair_engine(a, N)) {
      const dim3 blk(kClsPairThreads);
      if (cls_pair_db(a, N)) {
        if (N == 128 && a.fmt == kCI4) hipLaunchKernelGGL((k_image_cls_pair<2, kCI4, true>), grid, blk, 0, s, a);
        else if (N == 128) hipLaunchKernelGGL((k_image_cls_pair<2, kCI8, true>), grid, blk, 0, s, a);
        else if (a.fmt == kCI4) hipLaunchKernelGGL((k_image_cls_pair<4, kCI4, true>), grid, blk, 0, s, a);
        else hipLaunchKernelGGL((k_image_cls_pair<4, kCI8, true>), grid, blk, 0, s, a);
      } else {
        if (N == 128 && a.fmt == kCI4) hipLaunchKernelGGL((k_image_cls_pair<2, kCI4, false>), grid, blk, 0, s, a);
        else if (N == 128) hipLaunchKernelGGL((k_image_cls_pair<2, kCI8, false>), grid, blk, 0, s, a);
        else if (a.fmt == kCI4) hipLaunchKernelGGL((k_image_cls_pair<4, kCI4, false>), grid, blk, 0, s, a);
        else hipLaunchKernelGGL((k_image_cls_pair<4, kCI8, false>), grid, blk, 0, s, a);
      }
      return hipGetLastError();
    }
    if (N == 128 && !big) hipLaunchKernelGGL((k_image_cls<2>), grid, dim3(256), 0, s, a);
    else if (N == 128) hipLaunchKernelGGL((k_image_cls_big<2>), grid, dim3(256), 0, s, a);
    else if (!big) hipLaunchKernelGGL((k_image_cls<4>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_image_cls_big<4>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  return dispatch_n<LaunchImage>(N, a.Na, a, s);
}

template <int N, int APL>
struct LaunchImageSnap {
  static hipError_t run(const ImageArgs& a, hipStream_t s) {
    if constexpr (N == 64 && (APL == 2 || APL == 4)) {
      if (pair_engine(a, N)) {
        const dim3 grid(a.F * a.splits), block(kPairThreads);
        if (a.t_acc >= kSnapGroupWindow) {
          if (a.fmt == kCI4) hipLaunchKernelGGL((k_image_pair_snap_group<APL, kCI4>), grid, block, 0, s, a);
          else hipLaunchKernelGGL((k_image_pair_snap_group<APL, kCI8>), grid, block, 0, s, a);
        } else {
          if (a.fmt == kCI4) hipLaunchKernelGGL((k_image_pair_snap<APL, kCI4>), grid, block, 0, s, a);
          else hipLaunchKernelGGL((k_image_pair_snap<APL, kCI8>), grid, block, 0, s, a);
        }
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_image_snap<N, APL>), dim3(a.F * a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
  }
};

hipError_t launch_image_snap(int N, const ImageArgs& a, hipStream_t s) {
  if (N > 64 || a.t_acc < 1 || !a.snap || a.splits < 1) return hipErrorInvalidValue;
  return dispatch_n<LaunchImageSnap>(N, a.Na, a, s);
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
