// HIP kernels (gfx950): one launch per stage for a whole batch of arrays of
// uneven antenna count and grid size.
//
//   k_solve_batch   one 512-thread workgroup per (array, channel)
//   k_image_batch   persistent, 512 threads (two waves per SIMD): one
//                   workgroup per CU pulls work items {array, channel, class
//                   group, time split} from an atomic counter (items sorted
//                   by cost, largest first) and runs the body chosen for that
//                   array in one LDS arena:
//                     N <= 32     the FFT engine with eight waves
//                     N = 64      the paired engine (integer E-fields, <= 256 antennas)
//                     N = 128/256 the class-pair engine (<= 512 antennas) or the
//                                 dense class engine (<= 2048 / 1024)
//   k_reduce_batch  FP64 reduction of every array's partial images
// Arrays no body covers (complex float E-fields at 64 x 64 and above, the
// DFT-GEMM form) are imaged by their own launches in the same sequence.
// Per-array arguments travel in the kernel argument block; the item list is
// plan-owned device memory.  The whole sequence (plus the counter reset) is
// what the library captures in a hipGraph.  The bodies (batch_bodies.h) are
// shared with the fused solve + imaging kernel of k_fused.hip.
#include "batch_bodies.h"
#include "epic_internal.h"
#include "image_dft.h"
#include "solve.h"

namespace epic {

__global__ void k_counter_reset(int* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

// The item's array arguments are copied from the kernel argument block into
// LDS and handed to the body from there: a reference into the argument block
// itself would make the compiler copy the whole block (every array's
// arguments) into each lane's scratch memory.
__global__ __launch_bounds__(kBatchThreads) void k_image_batch(BatchImageArgs b) {
  __shared__ __align__(16) uint8_t smem[kLdsBytes];
  __shared__ int item_l;
  __shared__ __align__(16) uint8_t item_raw[sizeof(ImageArgs)];
  const ImageArgs& item_args = *reinterpret_cast<const ImageArgs*>(item_raw);
  for (;;) {
    if (threadIdx.x == 0) item_l = atomicAdd(b.counter, 1);
    __syncthreads();
    const int it = item_l;
    if (it < b.n_items && threadIdx.x == 0) {
      const ImageArgs one = b.arr[b.items[it].x];
      __builtin_memcpy(item_raw, &one, sizeof(ImageArgs));
    }
    __syncthreads();
    if (it >= b.n_items) break;   // every wave of the workgroup leaves together
    const int4 w = b.items[it];
    run_item(item_args, b.code[w.x], w, smem);
  }
}

int batch_body(const ImageArgs& a, int N, bool dft) {
  if (dft) return 0;
  const bool integer = a.fmt == kCI4 || a.fmt == kCI8;
  if (N == 16 || N == 32) {
    const int apl = apl_for(N, a.Na);
    const int cap = N == 16 ? (apl == 2 ? Budget<16, 2, 8>::TAB_SLOTS : apl == 4 ? Budget<16, 4, 8>::TAB_SLOTS
                                                                                : Budget<16, 8, 8>::TAB_SLOTS)
                            : (apl == 2 ? Budget<32, 2, 8>::TAB_SLOTS : apl == 4 ? Budget<32, 4, 8>::TAB_SLOTS : 0);
    if (apl == 0 || a.n_slots > cap) return 0;
    return fft8_code(N, apl);
  }
  if (N == 64) return pair_engine(a, N) ? pair_code(apl_for(N, a.Na), a.fmt) : 0;
  if ((N == 128 || N == 256) && integer) {
    const int R = N / 64;
    if (cls_pair_engine(a, N)) return cls_pair_code(R, a.fmt, cls_pair_db(a, N));
    if (cls_dense_engine(a, N)) return dense_code(R, a.fmt, a.grid_batch == 4 ? 4 : 2);
  }
  return 0;
}

template <int J, int PS>
__global__ __launch_bounds__(kSolveMainThreads) void k_solve_batch(BatchSolveArgs b) {
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
  b.image[i][j] = b.error && *b.error ? __builtin_nanf("") : float(s * b.scale[i]);
}

hipError_t launch_image_batch(const BatchImageArgs& b, int n_workgroups, hipStream_t s) {
  hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, s, b.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_image_batch, dim3(n_workgroups), dim3(kBatchThreads), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_solve_batch(const BatchSolveArgs& b, int j, int ps, hipStream_t s) {
  const dim3 grid(b.chan_off[b.n_arrays]), blk(kSolveMainThreads);
  if (j == 1 && ps == 16) hipLaunchKernelGGL((k_solve_batch<1, 16>), grid, blk, 0, s, b);
  else if (j == 1 && ps == 4) hipLaunchKernelGGL((k_solve_batch<1, 4>), grid, blk, 0, s, b);
  else if (j == 1) hipLaunchKernelGGL((k_solve_batch<1, 1>), grid, blk, 0, s, b);
  else if (j == 2 && ps == 16) hipLaunchKernelGGL((k_solve_batch<2, 16>), grid, blk, 0, s, b);
  else if (j == 2 && ps == 4) hipLaunchKernelGGL((k_solve_batch<2, 4>), grid, blk, 0, s, b);
  else if (j == 2) hipLaunchKernelGGL((k_solve_batch<2, 1>), grid, blk, 0, s, b);
  else if (ps == 16) hipLaunchKernelGGL((k_solve_batch<4, 16>), grid, blk, 0, s, b);
  else if (ps == 4) hipLaunchKernelGGL((k_solve_batch<4, 4>), grid, blk, 0, s, b);
  else hipLaunchKernelGGL((k_solve_batch<4, 1>), grid, blk, 0, s, b);
  return hipGetLastError();
}

hipError_t launch_reduce_batch(const BatchReduceArgs& b, hipStream_t s) {
  const int64_t n = b.off[b.n_arrays];
  hipLaunchKernelGGL(k_reduce_batch, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, b);
  return hipGetLastError();
}

}  // namespace epic
