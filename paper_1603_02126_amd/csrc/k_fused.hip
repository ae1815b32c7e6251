// HIP kernels (gfx950): the fused run, one launch for the EPICal
// calibration solve and the imaging of every array of a plan.
#include "batch_bodies.h"
#include "solve.h"

namespace epic {

// ---------------------------------------------------------------------------
// Fused run: the calibration solve and the imaging of every array in one
// launch (FusedArgs).  The first workgroups to start take the solve tasks
// (tickets 0 .. n_solve-1, one channel each, the single-pixel or the
// several-pixel solve at kSolveMainThreads = kBatchThreads threads publishing
// u interval by interval); a workgroup whose ticket is past the solve tasks
// pulls imaging items and, before each, waits until the channel has published
// every interval its samples fall in.  Tickets are taken by running workgroups
// only, so every solve a wait depends on is already running; the solves
// themselves never wait.
// ---------------------------------------------------------------------------
static_assert(kSolveMainThreads == kBatchThreads, "solve tasks run on the imaging workgroups");
static_assert(SolveSmem::BYTES <= kLdsBytes, "the solve fits the shared LDS arena");
static_assert(sizeof(BatchImageArgs) + sizeof(FusedArgs) <= 4096, "kernel arguments of the fused run");

template <typename T>
__device__ __forceinline__ T uniform_copy(const T& a) {
  static_assert(sizeof(T) % 4 == 0, "word-wise copy");
  T r;
  uint32_t words[sizeof(T) / 4];
  __builtin_memcpy(words, &a, sizeof(T));
  static_for<0, int(sizeof(T) / 4)>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    words[i] = __builtin_amdgcn_readfirstlane(words[i]);
  });
  __builtin_memcpy(&r, words, sizeof(T));
  return r;
}

template <int J, int PS>
__device__ __noinline__ void fused_solve_call(const SolveArgs& a, int f, uint8_t* smem, int* progress) {
  const SolveArgs la = uniform_copy(a);
  f = __builtin_amdgcn_readfirstlane(f);
  if (la.fmt == kCI4) solve_channel_fmt<J, PS, kCI4, kSolveMainThreads, true>(la, f, smem, progress);
  else if (la.fmt == kCI8) solve_channel_fmt<J, PS, kCI8, kSolveMainThreads, true>(la, f, smem, progress);
  else solve_channel_fmt<J, PS, kCF32, kSolveMainThreads, true>(la, f, smem, progress);
}

// Several tapped pixels (arrays of at most kSolveMainThreads antennas).
template <int PS>
__device__ __noinline__ void fused_multi_call(const SolveArgs& a, int f, uint8_t* smem, int* progress) {
  const SolveArgs la = uniform_copy(a);
  f = __builtin_amdgcn_readfirstlane(f);
  if (la.fmt == kCI4) solve_channel_multi<PS, kCI4, kSolveMainThreads, true>(la, f, smem, progress);
  else if (la.fmt == kCI8) solve_channel_multi<PS, kCI8, kSolveMainThreads, true>(la, f, smem, progress);
  else solve_channel_multi<PS, kCF32, kSolveMainThreads, true>(la, f, smem, progress);
}

__device__ __forceinline__ void run_solve(int code, const SolveArgs& a, int f, uint8_t* smem, int* progress) {
  switch (code) {
    case kFusedMultiCode + 16: fused_multi_call<16>(a, f, smem, progress); break;
    case kFusedMultiCode + 4: fused_multi_call<4>(a, f, smem, progress); break;
    case kFusedMultiCode + 1: fused_multi_call<1>(a, f, smem, progress); break;
    case 116: fused_solve_call<1, 16>(a, f, smem, progress); break;
    case 104: fused_solve_call<1, 4>(a, f, smem, progress); break;
    case 101: fused_solve_call<1, 1>(a, f, smem, progress); break;
    case 216: fused_solve_call<2, 16>(a, f, smem, progress); break;
    case 204: fused_solve_call<2, 4>(a, f, smem, progress); break;
    case 201: fused_solve_call<2, 1>(a, f, smem, progress); break;
    case 416: fused_solve_call<4, 16>(a, f, smem, progress); break;
    case 404: fused_solve_call<4, 4>(a, f, smem, progress); break;
    case 401: fused_solve_call<4, 1>(a, f, smem, progress); break;
    default: break;
  }
}

__global__ void k_fused_reset(int* ticket, int* counter, int* error, int* progress, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *ticket = 0;
    *counter = 0;
    *error = 0;
  }
  if (i < n) progress[i] = 0;
}

__global__ __launch_bounds__(kBatchThreads) void k_run_fused(BatchImageArgs b, FusedArgs fa) {
  __shared__ __align__(16) uint8_t smem[kLdsBytes];
  __shared__ int item_l;
  constexpr size_t kRaw = sizeof(ImageArgs) > sizeof(SolveArgs) ? sizeof(ImageArgs) : sizeof(SolveArgs);
  __shared__ __align__(16) uint8_t item_raw[kRaw];
  // solve tasks
  for (;;) {
    if (threadIdx.x == 0) item_l = atomicAdd(fa.ticket, 1);
    __syncthreads();
    const int t = item_l;
    int i = 0;
    while (i + 1 < b.n_arrays && t >= fa.chan_off[i + 1]) ++i;
    if (t < fa.n_solve && threadIdx.x == 0) {
      const ImageArgs& ia = b.arr[i];
      const FusedSolveExtra& x = fa.sx[i];
      SolveArgs sa{};
      sa.efield = ia.efield;
      sa.n_t = ia.n_t;
      sa.F = ia.F;
      sa.Na = ia.Na;
      sa.fmt = ia.fmt;
      sa.t_cal = ia.t_cal;
      sa.n_int = x.n_int;
      sa.A = x.A;
      sa.D = x.D;
      sa.hold = x.hold;
      sa.na_eff = x.na_eff;
      sa.gamma = x.gamma;
      sa.gains = x.gains;
      sa.u_hist = const_cast<float2*>(ia.u);
      sa.g_hist = x.g_hist;
      sa.status = x.status;
      sa.n_pix = x.n_pix;
      __builtin_memcpy(item_raw, &sa, sizeof(SolveArgs));
    }
    __syncthreads();
    if (t >= fa.n_solve) break;   // every wave of the workgroup leaves together
    run_solve(fa.sx[i].code, *reinterpret_cast<const SolveArgs*>(item_raw), t - fa.chan_off[i], smem,
              fa.progress + fa.chan_off[i]);
    __syncthreads();              // item_l and item_raw are rewritten next
  }
  // imaging items
  const ImageArgs& item_args = *reinterpret_cast<const ImageArgs*>(item_raw);
  for (;;) {
    if (threadIdx.x == 0) item_l = atomicAdd(b.counter, 1);
    __syncthreads();
    const int it = item_l;
    if (it < b.n_items && threadIdx.x == 0) {
      const int4 w = b.items[it];
      const ImageArgs one = b.arr[w.x];
      __builtin_memcpy(item_raw, &one, sizeof(ImageArgs));
      // the intervals of samples [tb, te) of this split: u of interval k is
      // published once progress > k
      const int64_t te = one.n_t * (w.w + 1) / one.splits;
      const int need = int((te + one.t_cal - 1) / one.t_cal);
      const int* p = fa.progress + fa.chan_off[w.x] + w.y;
      int polls = 0;
      while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (++polls > fa.max_polls) {
          __hip_atomic_store(fa.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the published u, not a stale cached copy
    }
    __syncthreads();
    if (it >= b.n_items) break;
    const int4 w = b.items[it];
    run_item(item_args, b.code[w.x], w, smem);
  }
}

hipError_t launch_run_fused(const BatchImageArgs& b, const FusedArgs& fa, int n_workgroups, hipStream_t s) {
  hipLaunchKernelGGL(k_fused_reset, dim3(unsigned((fa.n_solve + 255) / 256)), dim3(256), 0, s, fa.ticket, b.counter,
                     fa.error, fa.progress, fa.n_solve);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_run_fused, dim3(n_workgroups), dim3(kBatchThreads), 0, s, b, fa);
  return hipGetLastError();
}

}  // namespace epic
