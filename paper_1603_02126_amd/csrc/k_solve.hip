// HIP kernels (gfx950): EPICal calibration solve (tap, correlation, damped FP64 update).
#include "solve.h"

namespace epic {

template <int J, int PS>
__global__ __launch_bounds__(kSolveThreads) void k_solve(SolveArgs a) {
  __shared__ __align__(16) uint8_t smem[SolveSmem::BYTES];
  solve_channel<J, PS>(a, blockIdx.x, smem);
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
template <int MAXP>
static int stage_cap(int RB) {
  return RB % 16 == 0 ? Stager<16, MAXP>::CAP : RB % 4 == 0 ? Stager<4, MAXP>::CAP : Stager<1, MAXP>::CAP;
}

bool solve_supported(int na, int fmt, int n_pix) {
  const int RB = na * efmt_bytes(fmt);
  const int cap = na <= kSolveThreads ? stage_cap<8>(RB) : stage_cap<4>(RB);   // the stagers of J = 1 and 2
  if (n_pix < 1 || n_pix > kMaxPix || (n_pix > 1 && na > kSolveThreads)) return false;
  return na >= 1 && na <= 2 * kSolveThreads && RB <= cap;
}

template <int J>
static hipError_t launch_solve_j(const SolveArgs& a, hipStream_t s) {
  const int RB = a.Na * efmt_bytes(a.fmt);
  if (RB % 16 == 0) hipLaunchKernelGGL((k_solve<J, 16>), dim3(a.F), dim3(kSolveThreads), 0, s, a);
  else if (RB % 4 == 0) hipLaunchKernelGGL((k_solve<J, 4>), dim3(a.F), dim3(kSolveThreads), 0, s, a);
  else hipLaunchKernelGGL((k_solve<J, 1>), dim3(a.F), dim3(kSolveThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  if (!solve_supported(a.Na, a.fmt, a.n_pix)) return hipErrorInvalidValue;
  if (a.Na <= kSolveThreads) return launch_solve_j<1>(a, s);
  return launch_solve_j<2>(a, s);
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

hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(a.F), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace epic
