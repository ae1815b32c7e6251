// HIP kernels (gfx950): one launch per stage for a whole batch of arrays of
// uneven antenna count and grid size.
//
//   k_solve_batch   one 1024-thread workgroup per (array, channel)
//   k_image_batch   persistent: one workgroup per CU pulls work items
//                   {array, channel, class group, time split} from an atomic
//                   counter (items sorted by cost, largest first) and runs the
//                   engine chosen for that array (FFT / DFT-GEMM / residue
//                   classes) in the same LDS arena
//   k_reduce_batch  FP64 reduction of every array's partial images
// Per-array arguments travel in the kernel argument block; the item list is
// plan-owned device memory.  The whole sequence (plus the counter reset) is
// what the library captures in a hipGraph.
#include "epic_internal.h"
#include "image_cls.h"
#include "image_dft.h"
#include "image_fft.h"
#include "solve.h"

namespace epic {

static_assert(FftSmem<64, 8>::BYTES <= kLdsBytes && ClsSmem<4, false>::BYTES <= kLdsBytes &&
                  ClsSmem<4, true>::BYTES <= kLdsBytes && DftSmem<64, 8>::BYTES <= kLdsBytes,
              "every engine fits the shared LDS arena");

__global__ void k_counter_reset(int* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

// Each engine body is its own (non-inlined) function so that the register
// allocation of one engine does not constrain the others.  Through the call
// the arguments arrive as generic pointers: the engines state the address
// space of their global accesses (gload / gstore), and each wrapper copies
// the arguments once, so that the frame loop does not reload them with
// generic (FLAT) loads, which would also count against the LDS wait counter.
template <int N, int APL>
__device__ __noinline__ void fft_call(const ImageArgs& a, int4 w, uint8_t* smem) {
  const ImageArgs la = a;
  image_item<N, APL>(la, w.y, w.w, smem);
}
template <int N, int APL>
__device__ __noinline__ void dft_call(const ImageArgs& a, int4 w, uint8_t* smem) {
  const ImageArgs la = a;
  dft_item<N, APL>(la, w.y, w.w, smem);
}
template <int R, bool BIG>
__device__ __noinline__ void cls_call(const ImageArgs& a, int4 w, uint8_t* smem) {
  const ImageArgs la = a;
  image_cls_item<R, BIG, 0>(la, w.y, w.z, w.w, smem);
}

// engine code: 100 * engine + N / 32 * 10 + param (APL or R)
__device__ __forceinline__ void run_item(const ImageArgs& a, int code, int4 w, uint8_t* smem) {
  switch (code) {
    case 100 * kEngFft + 10 + 2: fft_call<32, 2>(a, w, smem); break;
    case 100 * kEngFft + 10 + 4: fft_call<32, 4>(a, w, smem); break;
    case 100 * kEngFft + 10 + 8: fft_call<32, 8>(a, w, smem); break;
    case 100 * kEngFft + 20 + 2: fft_call<64, 2>(a, w, smem); break;
    case 100 * kEngFft + 20 + 4: fft_call<64, 4>(a, w, smem); break;
    case 100 * kEngFft + 20 + 8: fft_call<64, 8>(a, w, smem); break;
    case 100 * kEngDft + 10 + 2: dft_call<32, 2>(a, w, smem); break;
    case 100 * kEngDft + 10 + 4: dft_call<32, 4>(a, w, smem); break;
    case 100 * kEngDft + 10 + 8: dft_call<32, 8>(a, w, smem); break;
    case 100 * kEngDft + 20 + 2: dft_call<64, 2>(a, w, smem); break;
    case 100 * kEngDft + 20 + 4: dft_call<64, 4>(a, w, smem); break;
    case 100 * kEngDft + 20 + 8: dft_call<64, 8>(a, w, smem); break;
    case 100 * kEngCls + 40 + 2: cls_call<2, false>(a, w, smem); break;
    case 100 * kEngCls + 80 + 4: cls_call<4, false>(a, w, smem); break;
    case 100 * kEngClsBig + 40 + 2: cls_call<2, true>(a, w, smem); break;
    case 100 * kEngClsBig + 80 + 4: cls_call<4, true>(a, w, smem); break;
    default: break;
  }
}

__global__ __launch_bounds__(256) void k_image_batch(BatchImageArgs b) {
  __shared__ __align__(16) uint8_t smem[kLdsBytes];
  __shared__ int item_l;
  for (;;) {
    if (threadIdx.x == 0) item_l = atomicAdd(b.counter, 1);
    __syncthreads();
    const int it = item_l;
    __syncthreads();
    if (it >= b.n_items) break;   // every wave of the workgroup leaves together
    const int4 w = b.items[it];
    run_item(b.arr[w.x], b.code[w.x], w, smem);
  }
}

template <int J, int PS>
__global__ __launch_bounds__(kSolveThreads) void k_solve_batch(BatchSolveArgs b) {
  __shared__ __align__(16) uint8_t smem[SolveSmem::BYTES];
  int i = 0;
  while (i + 1 < b.n_arrays && int(blockIdx.x) >= b.chan_off[i + 1]) ++i;
  solve_channel<J, PS>(b.arr[i], int(blockIdx.x) - b.chan_off[i], smem);
}

__global__ __launch_bounds__(256) void k_reduce_batch(BatchReduceArgs b) {
  const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= b.off[b.n_arrays]) return;
  int i = 0;
  while (i + 1 < b.n_arrays && g >= b.off[i + 1]) ++i;
  const int64_t j = g - b.off[i];
  double s = 0.0;
  for (int k = 0; k < b.splits[i]; ++k) s += double(b.partial[i][int64_t(k) * b.per_split[i] + j]);
  b.image[i][j] = float(s * b.scale[i]);
}

bool batch_engine_supported(int code) {
  switch (code) {
    case 100 * kEngFft + 12: case 100 * kEngFft + 14: case 100 * kEngFft + 18:
    case 100 * kEngFft + 22: case 100 * kEngFft + 24: case 100 * kEngFft + 28:
    case 100 * kEngDft + 12: case 100 * kEngDft + 14: case 100 * kEngDft + 18:
    case 100 * kEngDft + 22: case 100 * kEngDft + 24: case 100 * kEngDft + 28:
    case 100 * kEngCls + 42: case 100 * kEngCls + 84:
    case 100 * kEngClsBig + 42: case 100 * kEngClsBig + 84:
    case 100 * kEngDftCls + 42: case 100 * kEngDftCls + 84:   // own launches in the batched sequence
      return true;
    default:
      return false;
  }
}

hipError_t launch_image_batch(const BatchImageArgs& b, int n_workgroups, hipStream_t s) {
  hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, s, b.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_image_batch, dim3(n_workgroups), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_solve_batch(const BatchSolveArgs& b, int j, int ps, hipStream_t s) {
  const dim3 grid(b.chan_off[b.n_arrays]);
  if (j == 1 && ps == 16) hipLaunchKernelGGL((k_solve_batch<1, 16>), grid, dim3(kSolveThreads), 0, s, b);
  else if (j == 1 && ps == 4) hipLaunchKernelGGL((k_solve_batch<1, 4>), grid, dim3(kSolveThreads), 0, s, b);
  else if (j == 1) hipLaunchKernelGGL((k_solve_batch<1, 1>), grid, dim3(kSolveThreads), 0, s, b);
  else if (ps == 16) hipLaunchKernelGGL((k_solve_batch<2, 16>), grid, dim3(kSolveThreads), 0, s, b);
  else if (ps == 4) hipLaunchKernelGGL((k_solve_batch<2, 4>), grid, dim3(kSolveThreads), 0, s, b);
  else hipLaunchKernelGGL((k_solve_batch<2, 1>), grid, dim3(kSolveThreads), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_reduce_batch(const BatchReduceArgs& b, hipStream_t s) {
  const int64_t n = b.off[b.n_arrays];
  hipLaunchKernelGGL(k_reduce_batch, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, b);
  return hipGetLastError();
}

}  // namespace epic
