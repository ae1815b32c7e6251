// HIP kernels (gfx950): adjoint of fixed-gain imaging with respect to the gains.
#include "engine.h"
#include "image_fft.h"

namespace epic {

// ---------------------------------------------------------------------------
// Adjoint of fixed-gain imaging: gradient of a real loss with respect to the
// gains.  Per frame the forward transform is recomputed (no per-sample
// storage), multiplied by R = dL/dI, transformed back with the conjugate
// sign, degridded at each antenna's cells and correlated with the
// uncalibrated E-field:
//   partial_a += conj(E_a(t)) sum_k w_ak DFT-(R . DFT+(G_t))[cell_ak]
// The host-side reduction applies 2 conj(-1/g^2) / (T Na^2).
// ---------------------------------------------------------------------------
template <int N, int APL>
__global__ __launch_bounds__(256) void k_adjoint(AdjointArgs a) {
  using G = Geo<N>;
  constexpr int P = G::PITCH;
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
  constexpr int K2 = 4;  // device cell tables are padded to four cells
  DegridTable<N, K2, APL> dg;
  dg.load(a.cell_ixy, a.cell_w, lam, a.Na);
  float r[N];
  static_for<0, N>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    r[y] = a.R[(int64_t(f) * N + y) * N + lam];
  });
  static_for<0, N>([&](auto xc) { buf[lam * P + decltype(xc)::value] = make_float2(0.f, 0.f); });
  __syncthreads();
  double2 du[APL];
  static_for<0, APL>([&](auto ic) { du[decltype(ic)::value] = make_double2(0.0, 0.0); });

  const int64_t iters = (te - tb + G::SLOTS - 1) / G::SLOTS;
  Raw raw[APL], rawc[APL];
  float2 uu[APL];
  {
    const int64_t t = tb + slot;
    fetch_frame<N, APL>(raw, uu, a.efield, a.u, t, kNoInterval, f, a.F, a.Na, a.fmt, lam, t < te);
  }
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + it * G::SLOTS + slot;
    const bool active = t < te;
    stage_frame<N, APL>(epr, raw, uu, lam, a.Na, a.fmt, active);
    static_for<0, APL>([&](auto ic) { rawc[decltype(ic)::value] = raw[decltype(ic)::value]; });
    {
      const int64_t tn = t + G::SLOTS;
      fetch_frame<N, APL>(raw, uu, a.efield, a.u, tn, kNoInterval, f, a.F, a.Na, a.fmt, lam, tn < te);
    }
    wave_lds_sync();
    grid_frame(buf, epr, stab, a.n_slots, N, lam);
    wave_lds_sync();
    float2 v[N];
    transform_frame<N, +1>(buf, v, lam);
    static_for<0, N>([&](auto yc) { v[decltype(yc)::value] = cscale(v[decltype(yc)::value], r[decltype(yc)::value]); });
    fft_reg<N, -1>(v);
    wave_lds_sync();
    static_for<0, N>([&](auto yc) { buf[decltype(yc)::value * P + lam] = v[decltype(yc)::value]; });
    wave_lds_sync();
    static_for<0, N>([&](auto xc) { v[decltype(xc)::value] = buf[lam * P + decltype(xc)::value]; });
    fft_reg<N, -1>(v);
    static_for<0, N>([&](auto xc) { buf[lam * P + decltype(xc)::value] = v[decltype(xc)::value]; });
    wave_lds_sync();
    static_for<0, APL>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if (active && lam + N * i < a.Na) {
        float2 gb = make_float2(0.f, 0.f);
        static_for<0, K2>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const float2 c = buf[dg.off[i][k]];
          gb.x = fmaf(dg.w[i][k], c.x, gb.x);
          gb.y = fmaf(dg.w[i][k], c.y, gb.y);
        });
        const float2 e = unpack_raw(rawc[i], a.fmt);
        // conj(e) * gb
        du[i].x += double(e.x * gb.x + e.y * gb.y);
        du[i].y += double(e.x * gb.y - e.y * gb.x);
      }
    });
    wave_lds_sync();
    static_for<0, N>([&](auto xc) { buf[lam * P + decltype(xc)::value] = make_float2(0.f, 0.f); });
  }
  __syncthreads();
  double2* red = reinterpret_cast<double2*>(lds);   // [SLOTS][APL*N]
  static_for<0, APL>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    red[slot * (APL * N) + lam + N * i] = du[i];
  });
  __syncthreads();
  for (int an = threadIdx.x; an < a.Na; an += 256) {
    double2 sum = make_double2(0.0, 0.0);
    for (int q = 0; q < G::SLOTS; ++q) {
      const double2 d = red[q * (APL * N) + an];
      sum.x += d.x;
      sum.y += d.y;
    }
    a.partial[(int64_t(s) * a.F + f) * a.Na + an] = sum;
  }
}

// ---------------------------------------------------------------------------
// The same adjoint with two waves per SIMD (64 x 64, integer E-fields, 129..256
// antennas), built like the paired imaging engine: eight waves per
// workgroup, each imaging its own frames through half a frame (columns 0..31,
// then 32..63) and transposing through that half buffer (xpose.h).  After R and the conjugate
// transform the frame G' (lane = row y) goes back through the same half
// buffer, one half of the columns at a time, and each lane gathers its
// antennas' kernel cells of that half (the other half's cells carry weight
// zero).  R is read per frame from the cache (16 KiB per channel).
// ---------------------------------------------------------------------------
template <int FMT>
__global__ __launch_bounds__(kPairThreads) void k_adjoint_pair(AdjointArgs a) {
  static_assert(FMT == kCI4 || FMT == kCI8, "integer E-field formats");
  constexpr int N = 64, APL = 4, K2 = 4, INFLIGHT = 8;
  using L = PairSmem<APL>;
  __shared__ __align__(16) uint8_t smem[L::BYTES];
  const int lam = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float2* H = reinterpret_cast<float2*>(smem) + wave * L::WAVE;
  float2* epr = H + L::HALF;
  uint2* stab = reinterpret_cast<uint2*>(smem + L::T_OFF);
  const int S0 = a.n_slots_h0, S1 = a.n_slots_h1;
  const int f = blockIdx.x % a.F, s = blockIdx.x / a.F;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  const float* Rf = a.R + int64_t(f) * N * N;

  load_slot_table(stab, a.slots_h, S0 + S1, N);
  clear_half_row(H, lam);
  __syncthreads();
  // per frame (cache resident, loaded where used: the loop has no registers
  // to keep them): the fixed calibration u and, for antenna lam + 64 i and
  // kernel cell k, the cell's offset in the half buffer (bit 15: the half of
  // the columns it lies in) and its weight
  const float2* urow = a.u + int64_t(f) * a.Na;

  double2 du[APL];
  static_for<0, APL>([&](auto ic) { du[decltype(ic)::value] = make_double2(0.0, 0.0); });
  float2 v[N];
  uint32_t raw[APL], rawc[APL];
  constexpr int bpe = FMT == kCI4 ? 1 : 2;
  auto fetch_raw = [&](int64_t t) {
    const uint8_t* row = a.efield + (t * a.F + f) * int64_t(a.Na) * bpe;
    static_for<0, APL>([&](auto ic) {
      const int an = lam + N * decltype(ic)::value;
      raw[decltype(ic)::value] = (t < te && an < a.Na) ? load_raw_global(row, an, FMT).x : 0u;
    });
  };
  const int64_t iters = (te - tb + INFLIGHT - 1) / INFLIGHT;
  fetch_raw(tb + wave);
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + it * INFLIGHT + wave;
    const bool active = t < te;
    __builtin_amdgcn_s_setprio(1);
    // per-frame addresses come from an opaque copy of the lane index: hoisted
    // out of the loop as invariants they would occupy ~80 registers
    int lo = lam;
    asm volatile("" : "+v"(lo));
    float2 uu[APL];
    static_for<0, APL>([&](auto ic) {
      const int an = lo + N * decltype(ic)::value;
      uu[decltype(ic)::value] = gload(urow + (an < a.Na ? an : a.Na - 1));
    });
    static_for<0, APL>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const int an = lam + N * i;
      rawc[i] = raw[i];
      if (an < a.Na) epr[an] = active ? cmul(unpack_raw(Raw{raw[i], 0u}, FMT), uu[i]) : make_float2(0.f, 0.f);
    });
    wave_lds_sync();
    grid_frame<8>(H, epr, stab, S0, N, lam);
    wave_lds_sync();
    take_half_row<0>(v, H, lam);
    wave_lds_sync();
    grid_frame<8>(H, epr, stab + S0 * N, S1, N, lam);
    wave_lds_sync();
    take_half_row<32>(v, H, lam);
    wave_lds_sync();
    __builtin_amdgcn_s_setprio(0);
    fft_reg<N, +1>(v);            // along x: lane = row y
    __builtin_amdgcn_s_setprio(1);
    transpose64(v, H, lam);       // lane = column kx
    __builtin_amdgcn_s_setprio(0);
    fft_reg<N, +1>(v);            // along y: v[ky] = X(kx = lane, ky)
    fetch_raw(t + INFLIGHT);
    // the loads below stay in their phase: hoisted above the transforms they
    // would hold registers that the transforms need
    __builtin_amdgcn_sched_barrier(0);
    int lr = lam;
    asm volatile("" : "+v"(lr));
    static_for<0, 4>([&](auto cc) {
      constexpr int c0 = 16 * decltype(cc)::value;
      float rr[16];
      static_for<0, 16>([&](auto kc) { rr[decltype(kc)::value] = gload(Rf + (c0 + decltype(kc)::value) * N + lr); });
      static_for<0, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        v[c0 + k] = cscale(v[c0 + k], rr[k]);
      });
    });
    __builtin_amdgcn_sched_barrier(0);
    fft_reg<N, -1>(v);            // conjugate transform along y: v[y], kx = lane
    __builtin_amdgcn_s_setprio(1);
    transpose64(v, H, lam);       // lane = row y, v[kx]
    __builtin_amdgcn_s_setprio(0);
    fft_reg<N, -1>(v);            // along x: v[x] = G'(x, y = lane)
    __builtin_amdgcn_s_setprio(1);
    // degrid: the half of the columns in the buffer, then the other half
    __builtin_amdgcn_sched_barrier(0);
    int doff[APL][K2];
    float dw[APL][K2];
    int ld = lam;
    asm volatile("" : "+v"(ld));
    static_for<0, APL>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const int an = ld + N * i;
      static_for<0, K2>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const int q = (an < a.Na ? an : 0) * K2 + k;
        const uint32_t ixy = gload(a.cell_ixy + q);
        const int ix = int(ixy & 0xffffu), iy = int(ixy >> 16);
        doff[i][k] = iy * kHalfPitch + (ix & 31) + ((ix >> 5) << 15);
        dw[i][k] = an < a.Na ? gload(a.cell_w + q) : 0.f;
      });
    });
    float2 gb[APL];
    static_for<0, APL>([&](auto ic) { gb[decltype(ic)::value] = make_float2(0.f, 0.f); });
    static_for<0, 2>([&](auto hc) {
      constexpr int hf = decltype(hc)::value;
      static_for<0, 32>([&](auto xc) { H[lam * kHalfPitch + decltype(xc)::value] = v[32 * hf + decltype(xc)::value]; });
      wave_lds_sync();
      static_for<0, APL>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        static_for<0, K2>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const float2 c = H[doff[i][k] & 0x7fff];
          const float w = (doff[i][k] >> 15) == hf ? dw[i][k] : 0.f;
          gb[i].x = fmaf(w, c.x, gb[i].x);
          gb[i].y = fmaf(w, c.y, gb[i].y);
        });
      });
      wave_lds_sync();
    });
    static_for<0, 32>([&](auto xc) { H[lam * kHalfPitch + decltype(xc)::value] = make_float2(0.f, 0.f); });
    __builtin_amdgcn_s_setprio(0);
    // correlate with the uncalibrated E-field: du_a += conj(E_a) G'(cells of a)
    static_for<0, APL>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if (active && lam + N * i < a.Na) {
        const float2 e = unpack_raw(Raw{rawc[i], 0u}, FMT);
        du[i].x += double(e.x * gb[i].x + e.y * gb[i].y);
        du[i].y += double(e.x * gb[i].y - e.y * gb[i].x);
      }
    });
  }
  // workgroup sum of the eight waves' partials (FP64) per antenna
  __syncthreads();
  double2* red = reinterpret_cast<double2*>(smem);   // [8][APL * 64]
  static_for<0, APL>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    red[wave * (APL * N) + lam + N * i] = du[i];
  });
  __syncthreads();
  for (int an = threadIdx.x; an < a.Na; an += kPairThreads) {
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double2 d = red[q * (APL * N) + an];
      sum.x += d.x;
      sum.y += d.y;
    }
    a.partial[(int64_t(s) * a.F + f) * a.Na + an] = sum;
  }
}

// dL/dg = 2 conj(-1/g^2) scale sum_s partial  (FP64)
__global__ __launch_bounds__(256) void k_adjoint_reduce(const double2* partial, int splits, int F, int Na,
                                                        const double2* gains, double scale, double2* out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t n = int64_t(F) * Na;
  if (i >= n) return;
  double2 sum = make_double2(0.0, 0.0);
  for (int k = 0; k < splits; ++k) {
    const double2 d = partial[int64_t(k) * n + i];
    sum.x += d.x;
    sum.y += d.y;
  }
  const double2 g = gains[i];
  const double2 g2 = zmul(g, g);
  const double2 m = zrecip(g2);                        // 1 / g^2
  const double2 c = make_double2(-m.x, m.y);          // conj(-1 / g^2)
  const double2 d = zmul(c, make_double2(sum.x * scale, sum.y * scale));
  out[i] = make_double2(2.0 * d.x, 2.0 * d.y);
}

// u = 1/g in FP32 (zero for flagged antennas).
__global__ __launch_bounds__(256) void k_recip(const double2* gains, const uint8_t* flag, int F, int Na, float2* u) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= int64_t(F) * Na) return;
  const double2 r = zrecip(gains[i]);
  u[i] = flag[i % Na] ? make_float2(0.f, 0.f) : make_float2(float(r.x), float(r.y));
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N, int APL>
struct LaunchAdjoint {
  static hipError_t run(const AdjointArgs& a, hipStream_t s) {
    if constexpr (N == 64 && APL == 4) {
      if (a.fmt != kCF32 && a.slots_h && a.n_slots_h0 + a.n_slots_h1 <= PairSmem<4>::TAB_SLOTS && a.k2 <= 4) {
        const dim3 grid(a.F * a.splits), block(kPairThreads);
        if (a.fmt == kCI4) hipLaunchKernelGGL((k_adjoint_pair<kCI4>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_pair<kCI8>), grid, block, 0, s, a);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_adjoint<N, APL>), dim3(a.F * a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
  }
};
hipError_t launch_adjoint(int N, const AdjointArgs& a, hipStream_t s) {
  return dispatch_n<LaunchAdjoint>(N, a.Na, a, s);
}
hipError_t launch_adjoint_reduce(const double2* partial, int splits, int F, int Na, const double2* gains,
                                 double scale, double2* dL_dg, hipStream_t s) {
  const int64_t n = int64_t(F) * Na;
  hipLaunchKernelGGL(k_adjoint_reduce, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, partial, splits, F, Na,
                     gains, scale, dL_dg);
  return hipGetLastError();
}
hipError_t launch_recip(const double2* gains, const uint8_t* flag, int F, int Na, float2* u, hipStream_t s) {
  const int64_t n = int64_t(F) * Na;
  hipLaunchKernelGGL(k_recip, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, gains, flag, F, Na, u);
  return hipGetLastError();
}


}  // namespace epic
