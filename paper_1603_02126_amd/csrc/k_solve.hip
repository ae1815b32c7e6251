// HIP kernels (gfx950): EPICal calibration solve (tap, correlation, damped FP64 update).
#include <algorithm>

#include "solve.h"
#include "solve_band.h"

namespace epic {

template <int J, int PS>
__global__ __launch_bounds__(kSolveMainThreads) void k_solve(SolveArgs a) {
  __shared__ __align__(16) uint8_t smem[SolveSmem::BYTES];
  solve_channel<J, PS>(a, blockIdx.x, smem);
}

template <int PS>
__global__ __launch_bounds__(kSolveThreads) void k_solve_pixels(SolveArgs a) {
  __shared__ __align__(16) uint8_t smem[SolveSmem::BYTES];
  solve_channel_pixels<PS>(a, blockIdx.x, smem);
}

// One wave per channel: small arrays with short intervals.
__global__ __launch_bounds__(64) void k_solve_wave(SolveArgs a) {
  __shared__ float2 ring[kSolveWaveRows * 64];
  if (a.fmt == kCI4) solve_channel_wave<kCI4>(a, blockIdx.x, ring);
  else if (a.fmt == kCI8) solve_channel_wave<kCI8>(a, blockIdx.x, ring);
  else solve_channel_wave<kCF32>(a, blockIdx.x, ring);
}

// ---------------------------------------------------------------------------
// Stage-wise EPICal accumulate / finalize: one workgroup per channel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_update(UpdateArgs a) {
  const int f = blockIdx.x;
  const int bpe = efmt_bytes(a.fmt);
  const int64_t rowstride = int64_t(a.F) * a.Na * bpe;
  const uint8_t* ebase = a.efield + (a.t0 * a.F + f) * int64_t(a.Na) * bpe;
  for (int an = threadIdx.x; an < a.Na; an += 256) {
    double* kq = a.kq + (int64_t(f) * a.Na + an) * 4;
    double kx = 0.0, ky = 0.0, q = 0.0;
    for (int t = 0; t < a.nt; ++t) {
      const float2 e = load_sample(ebase + t * rowstride, an, a.fmt);
      const float2 p = a.tap[int64_t(t) * a.F + f];
      kx += double(e.x) * p.x + double(e.y) * p.y;
      ky += double(e.y) * p.x - double(e.x) * p.y;
      q += double(e.x) * e.x + double(e.y) * e.y;
    }
    kx += kq[0];
    ky += kq[1];
    q += kq[2];
    const double cnt = kq[3] + a.nt;
    if (a.finalize) {
      const int64_t ia = int64_t(f) * a.Na + an;
      uint32_t st = 0u;
      if (cnt > 0) {
        const double inv_n = 1.0 / cnt;
        a.gains[ia] = epical_step(make_double2(kx * inv_n, ky * inv_n), q * inv_n, a.A[ia], a.D[ia],
                                  a.gains[ia], a.hold[ia], a.na_eff, a.gamma, &st);
      }
      if (a.status) a.status[ia] |= st;
      kq[0] = kq[1] = kq[2] = kq[3] = 0.0;
    } else {
      kq[0] = kx;
      kq[1] = ky;
      kq[2] = q;
      kq[3] = cnt;
    }
  }
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int MAXP, int T>
static int stage_cap(int RB) {
  return RB % 16 == 0 ? Stager<16, MAXP, T>::CAP : RB % 4 == 0 ? Stager<4, MAXP, T>::CAP : Stager<1, MAXP, T>::CAP;
}

int solve_main_j(int na) { return na <= kSolveMainThreads ? 1 : na <= 2 * kSolveMainThreads ? 2 : 4; }

bool solve_supported(int na, int fmt, int n_pix) {
  const int RB = na * efmt_bytes(fmt);
  if (n_pix < 1 || n_pix > kMaxPix || na < 1) return false;
  if (n_pix > 1) return na <= kSolveThreads && RB <= stage_cap<8, kSolveThreads>(RB);
  // the single-pixel solve's stager (MainStageMax: 8 pieces per thread at 512 threads)
  return na <= 4 * kSolveMainThreads && RB <= stage_cap<8, kSolveMainThreads>(RB);
}

bool solve_multi_fusable(int na, int fmt) {
  const int RB = na * efmt_bytes(fmt);
  return na >= 1 && na <= kSolveMainThreads && RB <= stage_cap<8, kSolveMainThreads>(RB);
}

template <int J>
static hipError_t launch_solve_j(const SolveArgs& a, hipStream_t s) {
  const int RB = a.Na * efmt_bytes(a.fmt);
  const dim3 blk(kSolveMainThreads);
  if (RB % 16 == 0) hipLaunchKernelGGL((k_solve<J, 16>), dim3(a.F), blk, 0, s, a);
  else if (RB % 4 == 0) hipLaunchKernelGGL((k_solve<J, 4>), dim3(a.F), blk, 0, s, a);
  else hipLaunchKernelGGL((k_solve<J, 1>), dim3(a.F), blk, 0, s, a);
  return hipGetLastError();
}

static hipError_t launch_solve_pixels(const SolveArgs& a, hipStream_t s) {
  const int RB = a.Na * efmt_bytes(a.fmt);
  const dim3 blk(kSolveThreads);
  if (RB % 16 == 0) hipLaunchKernelGGL((k_solve_pixels<16>), dim3(a.F), blk, 0, s, a);
  else if (RB % 4 == 0) hipLaunchKernelGGL((k_solve_pixels<4>), dim3(a.F), blk, 0, s, a);
  else hipLaunchKernelGGL((k_solve_pixels<1>), dim3(a.F), blk, 0, s, a);
  return hipGetLastError();
}

bool solve_by_wave(const SolveArgs& a) {
  return a.Na <= kSolveWaveMaxAnt && a.n_pix == 1 && a.t_cal <= kSolveWaveMaxTcal;
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  if (!solve_supported(a.Na, a.fmt, a.n_pix)) return hipErrorInvalidValue;
  if (solve_by_wave(a)) {
    hipLaunchKernelGGL(k_solve_wave, dim3(a.F), dim3(64), 0, s, a);
    return hipGetLastError();
  }
  if (a.n_pix > 1) return launch_solve_pixels(a, s);
  const int j = solve_main_j(a.Na);
  return j == 1 ? launch_solve_j<1>(a, s) : j == 2 ? launch_solve_j<2>(a, s) : launch_solve_j<4>(a, s);
}
__global__ __launch_bounds__(256) void k_hist_to_u(const double2* g_hist, const uint8_t* hold, int64_t n_elem,
                                                   int64_t per_int, float2* u_hist) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n_elem) return;
  double2 u = zrecip(g_hist[i]);
  if (hold[i % per_int] & kHoldFlagged) u = make_double2(0.0, 0.0);
  u_hist[i] = make_float2(float(u.x), float(u.y));
}

hipError_t launch_hist_to_u(const double2* g_hist, const uint8_t* hold, int64_t n_int, int F, int Na, float2* u_hist,
                            hipStream_t s) {
  const int64_t per = int64_t(F) * Na, n = n_int * per;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hist_to_u, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, g_hist, hold, n, per, u_hist);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gains shared over a band of channels: one cooperative launch, every
// workgroup resident, channels f = blockIdx.x + k * gridDim.x.  Per interval:
// each channel's undamped solution (band_interval), a grid barrier, the band
// model of every antenna (one wave per antenna), a grid barrier, and each
// channel's damped update (band_apply).
// ---------------------------------------------------------------------------
template <int PS, int FMT>
__global__ __launch_bounds__(kSolveThreads) void k_solve_band(BandArgs b) {
  __shared__ __align__(16) uint8_t smem[BandSmem::BYTES];
  __shared__ int s_ok;
  const SolveArgs& a = b.s;
  const int G = gridDim.x;
  uint32_t epoch = 0;
  for (int n = 0; n < a.n_int; ++n) {
    for (int f = blockIdx.x; f < a.F; f += G) band_interval<PS, FMT>(b, f, n, smem);
    if (!grid_barrier(b.bar, ++epoch, &s_ok)) {
      band_abort(b);
      return;
    }
    band_fit_phase(b);
    if (!grid_barrier(b.bar, ++epoch, &s_ok)) {
      band_abort(b);
      return;
    }
    for (int f = blockIdx.x; f < a.F; f += G) band_apply(b, f, n);
    __syncthreads();
  }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

bool band_supported(int na, int fmt) { return na >= 1 && na <= kSolveThreads && solve_supported(na, fmt, 1); }

template <int PS>
static const void* band_kernel(int fmt) {
  if (fmt == kCI4) return reinterpret_cast<const void*>(&k_solve_band<PS, kCI4>);
  if (fmt == kCI8) return reinterpret_cast<const void*>(&k_solve_band<PS, kCI8>);
  return reinterpret_cast<const void*>(&k_solve_band<PS, kCF32>);
}

hipError_t launch_solve_band(const BandArgs& b, int n_cu, hipStream_t s, int* groups) {
  const SolveArgs& a = b.s;
  if (!band_supported(a.Na, a.fmt) || a.n_pix != 1 || b.b0 < 0 || b.b1 <= b.b0 || b.b1 > a.F)
    return hipErrorInvalidValue;
  if (b.mode == kBandPoly && (b.deg_amp < 0 || b.deg_amp > kBandMaxDeg || b.deg_phase < 0 ||
                              b.deg_phase > kBandMaxDeg))
    return hipErrorInvalidValue;
  if (b.mode != kBandMean && b.mode != kBandPoly) return hipErrorInvalidValue;
  const int RB = a.Na * efmt_bytes(a.fmt);
  const void* fn = RB % 16 == 0 ? band_kernel<16>(a.fmt) : RB % 4 == 0 ? band_kernel<4>(a.fmt) : band_kernel<1>(a.fmt);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSolveThreads, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int G = std::min({a.F, per_cu * n_cu, kBandMaxGroups});
  if (groups) *groups = G;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kBandMaxGroups), 0, s, b.bar, kBandMaxGroups);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  BandArgs arg = b;
  void* args[] = {&arg};
  return hipLaunchCooperativeKernel(fn, dim3(G), dim3(kSolveThreads), args, 0, s);
}

hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(a.F), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace epic
