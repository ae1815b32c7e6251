// HIP kernels (gfx950): split-precision DFT-GEMM imaging (see image_dft.h);
// grids of 128 and 256 by residue classes of 64 x 64 DFT-GEMMs.
#include "image_dft.h"

namespace epic {

template <int N, int APL, int PREC>
__global__ __launch_bounds__(256) void k_image_dft(ImageArgs a) {
  __shared__ __align__(16) uint8_t smem[DftSmem<N, APL, PREC>::BYTES];
  dft_item<N, APL, PREC>(a, blockIdx.x % a.F, blockIdx.x / a.F, smem);
}

template <int R, int PREC>
__global__ __launch_bounds__(256) void k_image_dft_cls(ImageArgs a) {
  __shared__ __align__(16) uint8_t smem[DftClsSmem<R, PREC>::BYTES];
  constexpr int CP = R * R / 2;   // class pairs
  const int rest = blockIdx.x / a.F;
  dft_cls_item<R, PREC>(a, blockIdx.x % a.F, rest % CP, rest / CP, smem);
}

int dft_owners(int N) { return N >= 128 ? kDftClsOwners : DftGeo<32>::OWNERS * (N / 32); }

// n_slots: the transposed schedule for N <= 64 (held in LDS), the class
// schedule (read from memory) for N = 128, 256.
bool dft_supported(int N, int na, int n_slots) {
  if (N == 128 || N == 256) return na <= kDftClsMaxAnt;
  return (N == 32 || N == 64) && na <= 8 * 64 && n_slots <= kDftTabSlots;
}

template <int PREC>
static hipError_t launch_dft_prec(int N, const ImageArgs& a, hipStream_t s) {
  const int apl = (a.Na + 63) / 64;
  const dim3 grid(a.F * a.splits);
  if (N == 64) {
    if (apl <= 2) hipLaunchKernelGGL((k_image_dft<64, 2, PREC>), grid, dim3(256), 0, s, a);
    else if (apl <= 4) hipLaunchKernelGGL((k_image_dft<64, 4, PREC>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_image_dft<64, 8, PREC>), grid, dim3(256), 0, s, a);
  } else if (N == 32) {
    if (apl <= 2) hipLaunchKernelGGL((k_image_dft<32, 2, PREC>), grid, dim3(256), 0, s, a);
    else if (apl <= 4) hipLaunchKernelGGL((k_image_dft<32, 4, PREC>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_image_dft<32, 8, PREC>), grid, dim3(256), 0, s, a);
  } else if (N == 128) {
    hipLaunchKernelGGL((k_image_dft_cls<2, PREC>), dim3(a.F * 2 * a.splits), dim3(256), 0, s, a);
  } else if (N == 256) {
    hipLaunchKernelGGL((k_image_dft_cls<4, PREC>), dim3(a.F * 8 * a.splits), dim3(256), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_image_dft(int N, const ImageArgs& a, hipStream_t s) {
  if ((N == 128 || N == 256) && !a.slots_c) return hipErrorInvalidValue;
  switch (a.dft_prec) {
    case kDftF16: return launch_dft_prec<kDftF16>(N, a, s);
    case kDftBF16: return launch_dft_prec<kDftBF16>(N, a, s);
    case kDftBF16x3: return launch_dft_prec<kDftBF16x3>(N, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace epic
