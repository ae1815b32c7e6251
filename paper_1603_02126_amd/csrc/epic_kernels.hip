// HIP kernels (gfx950) for the EPIC direct-imaging loop with EPICal.
//
// Layout of the imaging engine ("one lane = one pencil"): a wave64 owns
// 64 / N frames of an N x N grid (N <= 64); lane lam of a frame owns grid row
// lam.  Per frame:
//   1. calibrate + grid (Sec. 2.1, E'_a = E_a / g_a and eq. gridding): each
//      lane takes antennas lam, lam + N, ... and scatters w * u * E with LDS
//      float atomics into the frame's zeroed LDS buffer;
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
#include "epic_internal.h"
#include "fft_reg.h"

namespace epic {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// A raw packed sample held in registers until it is used (so that a prefetch
// does not force the wait for the load at the point of issue).
struct Raw {
  uint32_t x, y;
};

__device__ __forceinline__ Raw load_raw(const uint8_t* row, int a, int fmt) {
  Raw r;
  if (fmt == kCI4) {
    r.x = row[a];
    r.y = 0;
  } else if (fmt == kCI8) {
    r.x = reinterpret_cast<const uint16_t*>(row)[a];
    r.y = 0;
  } else {
    const uint2 v = reinterpret_cast<const uint2*>(row)[a];
    r.x = v.x;
    r.y = v.y;
  }
  return r;
}

// Two's complement nibbles / bytes -> float (exact).
__device__ __forceinline__ float2 unpack_raw(Raw r, int fmt) {
  if (fmt == kCI4) {
    const int b = int(int8_t(uint8_t(r.x)));
    return make_float2(float(b >> 4), float(int(int8_t(uint8_t(r.x << 4))) >> 4));
  } else if (fmt == kCI8) {
    return make_float2(float(int8_t(uint8_t(r.x))), float(int8_t(uint8_t(r.x >> 8))));
  }
  return make_float2(__uint_as_float(r.x), __uint_as_float(r.y));
}

__device__ __forceinline__ float2 load_sample(const uint8_t* row, int a, int fmt) {
  return unpack_raw(load_raw(row, a, fmt), fmt);
}

__device__ __forceinline__ void lds_add(float2* p, float2 v) {
  __hip_atomic_fetch_add(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_add(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Order LDS traffic of one wavefront: the hardware executes a wave's LDS
// instructions in order; this keeps the compiler from moving them across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float2 shfl_xor2(float2 v, int m) {
  return make_float2(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

template <int N>
struct Geo {
  static constexpr int PITCH = N + 2;       // complex values per LDS row
  static constexpr int FPW = 64 / N;        // frames per wave
  static constexpr int FRAME = N * PITCH;   // float2 per frame buffer
  static constexpr int SLOTS = 4 * FPW;     // frames in flight per workgroup
  static constexpr int LDS = SLOTS * FRAME; // float2 per workgroup
};

// Per-lane antenna tables: LDS offsets of the K2 cells and their weights.
template <int N, int K2, int APL>
struct AntTable {
  int off[APL][K2];
  float w[APL][K2];
  __device__ __forceinline__ void load(const uint32_t* cell_ixy, const float* cell_w, int lam, int Na) {
    static_for<0, APL>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const int a = lam + N * i;
      static_for<0, K2>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (a < Na) {
          const uint32_t ixy = cell_ixy[a * K2 + k];
          off[i][k] = int(ixy >> 16) * Geo<N>::PITCH + int(ixy & 0xffffu);
          w[i][k] = cell_w[a * K2 + k];
        } else {
          off[i][k] = 0;
          w[i][k] = 0.f;
        }
      });
    });
  }
};

// Calibrate and grid one frame into `buf` (zeroed beforehand).
template <int N, int K2, int APL>
__device__ __forceinline__ void scatter_frame(float2* buf, const AntTable<N, K2, APL>& tab,
                                              const Raw (&raw)[APL], const float2 (&uu)[APL],
                                              int lam, int Na, int fmt, bool active) {
  static_for<0, APL>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if (active && lam + N * i < Na) {
      const float2 ec = cmul(unpack_raw(raw[i], fmt), uu[i]);
      static_for<0, K2>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        lds_add(&buf[tab.off[i][k]], cscale(ec, tab.w[i][k]));
      });
    }
  });
}

template <int N, int APL>
__device__ __forceinline__ void fetch_frame(Raw (&raw)[APL], float2 (&uu)[APL], const uint8_t* efield,
                                            const float2* u, int64_t t, int64_t t_cal, int f, int F,
                                            int Na, int fmt, int lam, bool active) {
  const int bpe = fmt == kCF32 ? 8 : fmt == kCI8 ? 2 : 1;
  const uint8_t* row = efield + (t * F + f) * int64_t(Na) * bpe;
  const float2* urow = u + ((t / t_cal) * F + f) * int64_t(Na);
  static_for<0, APL>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const int a = lam + N * i;
    if (active && a < Na) {
      raw[i] = load_raw(row, a, fmt);
      uu[i] = urow[a];
    } else {
      raw[i] = Raw{0u, 0u};
      uu[i] = make_float2(0.f, 0.f);
    }
  });
}

// Row FFT -> transpose through LDS -> column FFT.  On entry buf holds the
// gridded frame; on exit v[ky] = sum_j G_j exp(S 2 pi i j.k / N) for
// kx = lam, and the lane's buffer row is zero again.
template <int N, int S>
__device__ __forceinline__ void transform_frame(float2* buf, float2 (&v)[N], int lam) {
  constexpr int P = Geo<N>::PITCH;
  static_for<0, N>([&](auto xc) { v[decltype(xc)::value] = buf[lam * P + decltype(xc)::value]; });
  fft_reg<N, S>(v);
  wave_lds_sync();
  static_for<0, N>([&](auto xc) { buf[decltype(xc)::value * P + lam] = v[decltype(xc)::value]; });
  wave_lds_sync();
  static_for<0, N>([&](auto yc) { v[decltype(yc)::value] = buf[lam * P + decltype(yc)::value]; });
  static_for<0, N>([&](auto yc) { buf[lam * P + decltype(yc)::value] = make_float2(0.f, 0.f); });
  fft_reg<N, S>(v);
}

// ---------------------------------------------------------------------------
// Fused imaging kernel
// ---------------------------------------------------------------------------
template <int N, int K2, int APL>
__global__ __launch_bounds__(256) void k_image(ImageArgs a) {
  using G = Geo<N>;
  __shared__ float2 lds[G::LDS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane / N, lam = lane % N;
  const int slot = wave * G::FPW + h;
  const int f = blockIdx.x % a.F;
  const int s = blockIdx.x / a.F;
  const int64_t tb = a.n_t * s / a.splits, te = a.n_t * (s + 1) / a.splits;
  float2* buf = lds + slot * G::FRAME;

  AntTable<N, K2, APL> tab;
  tab.load(a.cell_ixy, a.cell_w, lam, a.Na);
  static_for<0, N>([&](auto xc) { buf[lam * G::PITCH + decltype(xc)::value] = make_float2(0.f, 0.f); });

  float acc[N];
  static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] = 0.f; });

  const int64_t iters = (te - tb + G::SLOTS - 1) / G::SLOTS;
  Raw raw[APL];
  float2 uu[APL];
  {
    const int64_t t = tb + slot;
    fetch_frame<N, APL>(raw, uu, a.efield, a.u, t, a.t_cal, f, a.F, a.Na, a.fmt, lam, t < te);
  }
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t t = tb + it * G::SLOTS + slot;
    wave_lds_sync();
    scatter_frame<N, K2, APL>(buf, tab, raw, uu, lam, a.Na, a.fmt, t < te);
    {
      const int64_t tn = t + G::SLOTS;
      fetch_frame<N, APL>(raw, uu, a.efield, a.u, tn, a.t_cal, f, a.F, a.Na, a.fmt, lam, tn < te);
    }
    wave_lds_sync();
    float2 v[N];
    transform_frame<N, +1>(buf, v, lam);
    static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] += cnorm(v[decltype(yc)::value]); });
  }

  // workgroup reduction of the SLOTS accumulators
  __syncthreads();
  float* red = reinterpret_cast<float*>(lds);
  static_for<0, N>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    red[(slot * N + y) * N + lam] = acc[y];
  });
  __syncthreads();
  float* out = a.partial + (int64_t(s) * a.F + f) * (N * N);
  for (int idx = threadIdx.x; idx < N * N; idx += 256) {
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < G::SLOTS; ++q) sum += red[q * N * N + idx];
    out[idx] = sum;
  }
}

// ---------------------------------------------------------------------------
// Stage-wise gridding to HBM
// ---------------------------------------------------------------------------
template <int N, int K2, int APL>
__global__ __launch_bounds__(256) void k_grid(GridArgs a) {
  using G = Geo<N>;
  __shared__ float2 lds[G::LDS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane / N, lam = lane % N;
  const int slot = wave * G::FPW + h;
  const int64_t q = int64_t(blockIdx.x) * G::SLOTS + slot;  // frame = t * F + f
  const bool active = q < int64_t(a.nt) * a.F;
  float2* buf = lds + slot * G::FRAME;
  AntTable<N, K2, APL> tab;
  tab.load(a.cell_ixy, a.cell_w, lam, a.Na);
  static_for<0, N>([&](auto xc) { buf[lam * G::PITCH + decltype(xc)::value] = make_float2(0.f, 0.f); });
  const int64_t t = active ? q / a.F : 0;
  const int f = active ? int(q % a.F) : 0;
  Raw raw[APL];
  float2 uu[APL];
  {
    const int bpe = efmt_bytes(a.fmt);
    const uint8_t* row = a.efield + ((a.t0 + t) * a.F + f) * int64_t(a.Na) * bpe;
    static_for<0, APL>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const int an = lam + N * i;
      raw[i] = Raw{0u, 0u};
      uu[i] = make_float2(0.f, 0.f);
      if (active && an < a.Na) {
        raw[i] = load_raw(row, an, a.fmt);
        uu[i] = a.u[int64_t(f) * a.Na + an];
      }
    });
  }
  wave_lds_sync();
  scatter_frame<N, K2, APL>(buf, tab, raw, uu, lam, a.Na, a.fmt, active);
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
    static_for<0, N>([&](auto yc) { acc[decltype(yc)::value] += cnorm(v[decltype(yc)::value]); });
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
// EPICal: FP64 update helpers (eq. Cna, eq. damping)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  const double2 n = zmul(a, zconj(b));
  return make_double2(n.x / d, n.y / d);
}
__device__ __forceinline__ double2 zrecip(double2 g) {
  const double d = g.x * g.x + g.y * g.y;
  return make_double2(g.x / d, -g.y / d);
}

// One damped update.  Returns the new gain; sets *st bits if held.
__device__ __forceinline__ double2 epical_step(double2 Kbar, double Qbar, double2 A, double2 D, double2 g,
                                               uint8_t hold, double na, double gamma, uint32_t* st) {
  if (hold) {
    *st |= (hold & kHoldFlagged ? 1u : 0u) | (hold & kHoldDZero ? 2u : 0u);
    return g;
  }
  // C = Kbar - conj(A) Qbar / (Na conj(g))
  const double2 t = zdiv(make_double2(A.x * Qbar, -A.y * Qbar), make_double2(na * g.x, -na * g.y));
  const double2 C = make_double2(Kbar.x - t.x, Kbar.y - t.y);
  const double2 sol = zdiv(make_double2(C.x * na, C.y * na), D);
  const double2 gn = make_double2((1.0 - gamma) * sol.x + gamma * g.x, (1.0 - gamma) * sol.y + gamma * g.y);
  if (!isfinite(gn.x) || !isfinite(gn.y)) {
    *st |= 4u;
    return g;
  }
  return gn;
}

// ---------------------------------------------------------------------------
// EPICal solve over all intervals: one workgroup per channel.
// ---------------------------------------------------------------------------
constexpr int kSolveChunk = 256;

template <int J>
__global__ __launch_bounds__(256) void k_solve(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* g_l = reinterpret_cast<double2*>(smem);                   // [Na]
  float2* c_l = reinterpret_cast<float2*>(g_l + a.Na);                // [Na]
  float2* P_l = c_l + a.Na;                                           // [kSolveChunk]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = blockIdx.x;
  const int bpe = efmt_bytes(a.fmt);
  const int64_t rowstride = int64_t(a.F) * a.Na * bpe;
  const uint8_t* ebase = a.efield + int64_t(f) * a.Na * bpe;
  uint32_t st[J];
  uint8_t hold[J];
  double2 A[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int an = tid + 256 * j;
    st[j] = 0u;
    hold[j] = 0;
    A[j] = make_double2(0.0, 0.0);
    if (an < a.Na) {
      g_l[an] = a.gains[int64_t(f) * a.Na + an];
      hold[j] = a.hold[int64_t(f) * a.Na + an];
      A[j] = a.A[int64_t(f) * a.Na + an];
      if (a.g_hist) a.g_hist[int64_t(f) * a.Na + an] = g_l[an];
    }
  }
  __syncthreads();
  for (int n = 0; n < a.n_int; ++n) {
    const int64_t t0 = int64_t(n) * a.t_cal;
    const int64_t t1 = min(t0 + a.t_cal, a.n_t);
    // coefficients c_a = A_a u_a / Na and u_a = 1 / g_a (0 for flagged antennas)
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int an = tid + 256 * j;
      if (an < a.Na) {
        double2 u = zrecip(g_l[an]);
        if (hold[j] & kHoldFlagged) u = make_double2(0.0, 0.0);
        const double2 c = zmul(A[j], u);
        c_l[an] = make_float2(float(c.x / a.na_eff), float(c.y / a.na_eff));
        a.u_hist[(int64_t(n) * a.F + f) * a.Na + an] = make_float2(float(u.x), float(u.y));
      }
    }
    double Kx[J], Ky[J], Q[J];
#pragma unroll
    for (int j = 0; j < J; ++j) Kx[j] = Ky[j] = Q[j] = 0.0;
    __syncthreads();
    for (int64_t tc = t0; tc < t1; tc += kSolveChunk) {
      const int ncur = int(min(int64_t(kSolveChunk), t1 - tc));
      // tapped pixel P(t) = sum_a c_a E_a(t): one wave per sample, lanes over antennas
      for (int tt = wave; tt < ncur; tt += 4) {
        const uint8_t* row = ebase + (tc + tt) * rowstride;
        float2 p = make_float2(0.f, 0.f);
        for (int an = lane; an < a.Na; an += 64) {
          const float2 e = load_sample(row, an, a.fmt);
          p = cadd(p, cmul(c_l[an], e));
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) p = cadd(p, shfl_xor2(p, m));
        if (lane == 0) P_l[tt] = p;
      }
      __syncthreads();
      // K_a += E_a conj(P), Q_a += |E_a|^2 with the uncalibrated E-fields
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int an = tid + 256 * j;
        if (an < a.Na) {
          float kx = 0.f, ky = 0.f, q = 0.f;
          const uint8_t* col = ebase + tc * rowstride;
          for (int tt = 0; tt < ncur; ++tt) {
            const float2 e = load_sample(col + tt * rowstride, an, a.fmt);
            const float2 p = P_l[tt];
            kx += e.x * p.x + e.y * p.y;
            ky += e.y * p.x - e.x * p.y;
            q += e.x * e.x + e.y * e.y;
          }
          Kx[j] += double(kx);
          Ky[j] += double(ky);
          Q[j] += double(q);
        }
      }
      __syncthreads();
    }
    // damped update (FP64)
    const double inv_n = 1.0 / double(t1 - t0);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int an = tid + 256 * j;
      if (an < a.Na) {
        const double2 g = g_l[an];
        const double2 gn = epical_step(make_double2(Kx[j] * inv_n, Ky[j] * inv_n), Q[j] * inv_n, A[j],
                                       a.D[int64_t(f) * a.Na + an], g, hold[j], a.na_eff, a.gamma, &st[j]);
        g_l[an] = gn;
        if (a.g_hist) a.g_hist[(int64_t(n + 1) * a.F + f) * a.Na + an] = gn;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int an = tid + 256 * j;
    if (an < a.Na) {
      a.gains[int64_t(f) * a.Na + an] = g_l[an];
      if (a.status) a.status[int64_t(f) * a.Na + an] |= st[j];
    }
  }
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
static int apl_for(int N, int na) {
  const int need = (na + N - 1) / N;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 0;
}

bool image_supported(int N, int k2, int na) {
  return (N == 16 || N == 32 || N == 64) && (k2 == 1 || k2 == 4) && apl_for(N, na) != 0;
}

template <int N, int K2, template <int, int, int> class Launch, typename Args>
static hipError_t dispatch_apl(int na, const Args& a, hipStream_t s) {
  switch (apl_for(N, na)) {
    case 1: return Launch<N, K2, 1>::run(a, s);
    case 2: return Launch<N, K2, 2>::run(a, s);
    case 4: return Launch<N, K2, 4>::run(a, s);
    case 8: return Launch<N, K2, 8>::run(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <template <int, int, int> class Launch, typename Args>
static hipError_t dispatch_nk(int N, int k2, int na, const Args& a, hipStream_t s) {
  if (k2 == 1) {
    if (N == 16) return dispatch_apl<16, 1, Launch>(na, a, s);
    if (N == 32) return dispatch_apl<32, 1, Launch>(na, a, s);
    if (N == 64) return dispatch_apl<64, 1, Launch>(na, a, s);
  } else if (k2 == 4) {
    if (N == 16) return dispatch_apl<16, 4, Launch>(na, a, s);
    if (N == 32) return dispatch_apl<32, 4, Launch>(na, a, s);
    if (N == 64) return dispatch_apl<64, 4, Launch>(na, a, s);
  }
  return hipErrorInvalidValue;
}

template <int N, int K2, int APL>
struct LaunchImage {
  static hipError_t run(const ImageArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_image<N, K2, APL>), dim3(a.F * a.splits), dim3(256), 0, s, a);
    return hipGetLastError();
  }
};
template <int N, int K2, int APL>
struct LaunchGrid {
  static hipError_t run(const GridArgs& a, hipStream_t s) {
    const int64_t frames = int64_t(a.nt) * a.F;
    const int64_t blocks = (frames + Geo<N>::SLOTS - 1) / Geo<N>::SLOTS;
    hipLaunchKernelGGL((k_grid<N, K2, APL>), dim3(unsigned(blocks)), dim3(256), 0, s, a);
    return hipGetLastError();
  }
};

hipError_t launch_image(int N, int k2, const ImageArgs& a, hipStream_t s) {
  return dispatch_nk<LaunchImage>(N, k2, a.Na, a, s);
}
hipError_t launch_grid(int N, int k2, const GridArgs& a, hipStream_t s) {
  if (a.nt == 0) return hipSuccess;
  return dispatch_nk<LaunchGrid>(N, k2, a.Na, a, s);
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
hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  const size_t shm = size_t(a.Na) * (sizeof(double2) + sizeof(float2)) + kSolveChunk * sizeof(float2);
  const int J = (a.Na + 255) / 256;
  if (J <= 1) hipLaunchKernelGGL((k_solve<1>), dim3(a.F), dim3(256), shm, s, a);
  else if (J <= 2) hipLaunchKernelGGL((k_solve<2>), dim3(a.F), dim3(256), shm, s, a);
  else if (J <= 4) hipLaunchKernelGGL((k_solve<4>), dim3(a.F), dim3(256), shm, s, a);
  else if (J <= 8) hipLaunchKernelGGL((k_solve<8>), dim3(a.F), dim3(256), shm, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(a.F), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace epic
