// HIP kernels (gfx950): one launch per stage for a whole batch of arrays of
// uneven antenna count and grid size.
//
//   k_solve_batch   one 1024-thread workgroup per (array, channel)
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
// what the library captures in a hipGraph.
#include "epic_internal.h"
#include "image_cls.h"
#include "image_dft.h"
#include "image_fft.h"
#include "solve.h"

namespace epic {

constexpr int kBatchThreads = 512;

__global__ void k_counter_reset(int* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

// Each body is its own (non-inlined) function so that the register
// allocation of one body does not constrain the others (inlined into one
// kernel, the bodies spilled hundreds of registers).  Through the call the
// arguments arrive as a generic pointer and would be loaded into vector
// registers, turning every address computation of the frame loop into vector
// work: each wrapper copies the arguments once and makes every word uniform
// (readfirstlane), so that they live in scalar registers as a kernel's
// arguments do.  The engines state the address space of their global
// accesses (gload / gstore): generic (FLAT) loads would also count against
// the LDS wait counter.
__device__ __forceinline__ ImageArgs uniform_args(const ImageArgs& a, int4& w) {
  static_assert(sizeof(ImageArgs) % 4 == 0, "word-wise copy");
  ImageArgs r;
  uint32_t words[sizeof(ImageArgs) / 4];
  __builtin_memcpy(words, &a, sizeof(ImageArgs));
  static_for<0, int(sizeof(ImageArgs) / 4)>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    words[i] = __builtin_amdgcn_readfirstlane(words[i]);
  });
  __builtin_memcpy(&r, words, sizeof(ImageArgs));
  w = make_int4(__builtin_amdgcn_readfirstlane(w.x), __builtin_amdgcn_readfirstlane(w.y),
                __builtin_amdgcn_readfirstlane(w.z), __builtin_amdgcn_readfirstlane(w.w));
  return r;
}

template <int N, int APL>
__device__ __noinline__ void fft8_call(const ImageArgs& a, int4 w, uint8_t* smem) {
  const ImageArgs la = uniform_args(a, w);
  image_item<N, APL, 8>(la, w.y, w.w, smem);
}
template <int APL, int FMT>
__device__ __noinline__ void pair_call(const ImageArgs& a, int4 w, uint8_t* smem) {
  const ImageArgs la = uniform_args(a, w);
  image_item_pair<APL, FMT>(la, w.y, w.w, smem);
}
template <int R, int FMT, bool DB>
__device__ __noinline__ void cls_pair_call(const ImageArgs& a, int4 w, uint8_t* smem) {
  const ImageArgs la = uniform_args(a, w);
  image_cls_pair_item<R, FMT, DB>(la, w.y, w.z, w.w, smem);
}
template <int R, int FMT, int GB>
__device__ __noinline__ void dense_call(const ImageArgs& a, int4 w, uint8_t* smem) {
  const ImageArgs la = uniform_args(a, w);
  image_cls_dense_item<R, FMT, GB>(la, w.y, w.z, w.w, smem);
}

// Body codes: 1000 kind + parameters (0: no body, the array has its own launch).
constexpr int fft8_code(int N, int apl) { return 1000 + 10 * N + apl; }
constexpr int pair_code(int apl, int fmt) { return 2000 + 10 * apl + fmt; }
constexpr int cls_pair_code(int R, int fmt, bool db) { return 3000 + 100 * R + 10 * fmt + (db ? 1 : 0); }
constexpr int dense_code(int R, int fmt, int gb) { return 4000 + 100 * R + 10 * fmt + gb; }

static_assert(FftSmem<32, 4, 8>::BYTES <= kLdsBytes && FftSmem<16, 8, 8>::BYTES <= kLdsBytes &&
                  PairSmem<4>::BYTES <= kLdsBytes && ClsPairSmem<4>::BYTES <= kLdsBytes &&
                  ClsPairSmem<4, true>::BYTES <= kLdsBytes && ClsDenseSmem<4>::BYTES <= kLdsBytes,
              "every body fits the shared LDS arena");

__device__ __forceinline__ void run_item(const ImageArgs& a, int code, int4 w, uint8_t* smem) {
  switch (code) {
    case fft8_code(16, 2): fft8_call<16, 2>(a, w, smem); break;
    case fft8_code(16, 4): fft8_call<16, 4>(a, w, smem); break;
    case fft8_code(16, 8): fft8_call<16, 8>(a, w, smem); break;
    case fft8_code(32, 2): fft8_call<32, 2>(a, w, smem); break;
    case fft8_code(32, 4): fft8_call<32, 4>(a, w, smem); break;
    case pair_code(2, kCI8): pair_call<2, kCI8>(a, w, smem); break;
    case pair_code(2, kCI4): pair_call<2, kCI4>(a, w, smem); break;
    case pair_code(4, kCI8): pair_call<4, kCI8>(a, w, smem); break;
    case pair_code(4, kCI4): pair_call<4, kCI4>(a, w, smem); break;
    case cls_pair_code(2, kCI8, false): cls_pair_call<2, kCI8, false>(a, w, smem); break;
    case cls_pair_code(2, kCI4, false): cls_pair_call<2, kCI4, false>(a, w, smem); break;
    case cls_pair_code(2, kCI8, true): cls_pair_call<2, kCI8, true>(a, w, smem); break;
    case cls_pair_code(2, kCI4, true): cls_pair_call<2, kCI4, true>(a, w, smem); break;
    case cls_pair_code(4, kCI8, false): cls_pair_call<4, kCI8, false>(a, w, smem); break;
    case cls_pair_code(4, kCI4, false): cls_pair_call<4, kCI4, false>(a, w, smem); break;
    case cls_pair_code(4, kCI8, true): cls_pair_call<4, kCI8, true>(a, w, smem); break;
    case cls_pair_code(4, kCI4, true): cls_pair_call<4, kCI4, true>(a, w, smem); break;
    case dense_code(2, kCI8, 2): dense_call<2, kCI8, 2>(a, w, smem); break;
    case dense_code(2, kCI4, 2): dense_call<2, kCI4, 2>(a, w, smem); break;
    case dense_code(4, kCI8, 2): dense_call<4, kCI8, 2>(a, w, smem); break;
    case dense_code(4, kCI4, 2): dense_call<4, kCI4, 2>(a, w, smem); break;
    case dense_code(2, kCI8, 4): dense_call<2, kCI8, 4>(a, w, smem); break;
    case dense_code(2, kCI4, 4): dense_call<2, kCI4, 4>(a, w, smem); break;
    case dense_code(4, kCI8, 4): dense_call<4, kCI8, 4>(a, w, smem); break;
    case dense_code(4, kCI4, 4): dense_call<4, kCI4, 4>(a, w, smem); break;
    default: break;
  }
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

hipError_t launch_image_batch(const BatchImageArgs& b, int n_workgroups, hipStream_t s) {
  hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, s, b.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_image_batch, dim3(n_workgroups), dim3(kBatchThreads), 0, s, b);
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
