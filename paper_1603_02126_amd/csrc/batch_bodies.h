// Imaging bodies of the persistent kernels (the batched imaging kernel and
// the fused solve + imaging kernel): each engine as a called function taking
// one work item, and the dispatch on an array's body code.  Included by the
// translation unit of each kernel, so that each kernel gets its own
// instantiations (called from two kernels of one unit, the bodies were
// compiled with stack frames of 760 instead of 464 bytes and the batched
// imaging of the LWA shape took 8.7 instead of 5.6 ms).
#pragma once
#include "epic_internal.h"
#include "image_cls.h"
#include "image_fft.h"

namespace epic {

constexpr int kBatchThreads = 512;

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

}  // namespace epic
