// EPICal with gains shared over a band of channels: the per-channel
// solutions averaged across channels (Sec. 5) or fitted by low-order
// polynomials in amplitude and phase over frequency (Sec. 6).
#pragma once
#include "solve.h"

namespace epic {

constexpr uint32_t kBandSpinLimit = 1u << 22;   // polls of one grid barrier before giving up

// LDS: the solve's two chunk buffers, taps, and the coefficients c_a (reused
// for the raw solutions once the interval's taps are done).
struct BandSmem {
  static constexpr int P_OFF = 2 * kSolveChunkBytes;
  static constexpr int C_OFF = P_OFF + kSolveMaxRows * 16;
  static constexpr int BYTES = C_OFF + kSolveThreads * 16;
};

__device__ __forceinline__ double2 nan2() { return make_double2(__builtin_nan(""), __builtin_nan("")); }

// Data exchanged between workgroups (the raw solutions and the band model)
// is written and read with agent-scope atomic accesses, which are coherent
// across the XCDs' L2 caches by themselves; no cache write-back or
// invalidation is needed around the barrier.
__device__ __forceinline__ void put_shared(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double get_shared(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_shared2(double2* p, double2 v) {
  put_shared(&p->x, v.x);
  put_shared(&p->y, v.y);
}
__device__ __forceinline__ double2 get_shared2(const double2* p) {
  return make_double2(get_shared(&p->x), get_shared(&p->y));
}

// Grid-wide barrier of a cooperative launch (every workgroup resident), on
// one flag per workgroup: the barrier of epoch e is passed when every flag
// holds e or more.  Every wave first waits until its own memory operations
// have completed (so its shared-data stores are visible at agent scope),
// then lane 0 stores the workgroup's flag and the first wave polls all flags
// with a few wide loads.  Flags only grow, so they are never reset within a
// launch; no workgroup waits on one shared counter (same-address atomics
// from every workgroup are serialised by the memory system).  The poll is
// bounded: a barrier that does not complete within kBandSpinLimit polls
// returns false (the caller then stops), so every wave exits.
constexpr int kBandMaxGroups = 256;

__device__ __forceinline__ bool grid_barrier(uint32_t* flags, uint32_t epoch, int* s_ok) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x, G = gridDim.x;
    if (lane == 0) __hip_atomic_store(flags + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t polls = 0;
    bool done = false;
    while (!done) {
      bool mine = true;
#pragma unroll
      for (int k = 0; k < kBandMaxGroups / 64; ++k) {
        const int w = lane + 64 * k;
        if (w < G) mine = mine && __hip_atomic_load(flags + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      }
      done = __all(mine);
      if (!done) {
        if (++polls >= kBandSpinLimit) break;
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (lane == 0) *s_ok = done ? 1 : 0;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Phase 1: one channel's interval n -- taps, correlations and the undamped
// solution s_a = Na C_a / D_a (eq. Cna, eq. cal_solution), written to
// raw[f][a] (NaN where the antenna is held).  The gain estimate is read
// from gains[f][a] by the thread that applies its update (band_apply).
template <int PS, int FMT>
__device__ __forceinline__ void band_interval(const BandArgs& b, int f, int n, uint8_t* smem) {
  const SolveArgs& a = b.s;
  uint8_t (*chunk)[kSolveChunkBytes] = reinterpret_cast<uint8_t (*)[kSolveChunkBytes]>(smem);
  double2* P_l = reinterpret_cast<double2*>(smem + BandSmem::P_OFF);
  double2* c_l = reinterpret_cast<double2*>(smem + BandSmem::C_OFF);
  const int tid = threadIdx.x;
  constexpr int bpe = FMT == kCF32 ? 8 : FMT == kCI8 ? 2 : 1;
  const int RB = a.Na * bpe;
  const int64_t rowstride = int64_t(a.F) * RB;
  const uint8_t* ebase = a.efield + int64_t(f) * RB;
  using Stage = Stager<PS, 8>;
  int rpc = Stage::CAP / RB;
  rpc = rpc < kSolveMaxRows ? rpc : kSolveMaxRows;
  int NaP = 16;
  while (NaP < a.Na && NaP < kSolveThreads) NaP <<= 1;
  const int RG = kSolveThreads / NaP;
  const int rg = tid % RG, an = tid / RG;
  const bool own = an < a.Na;
  const int64_t ia = int64_t(f) * a.Na + (own ? an : 0);
  const int64_t t0 = int64_t(n) * a.t_cal;
  const int len = int(min(a.t_cal, a.n_t - t0));

  double2 g = make_double2(1.0, 0.0);
  uint8_t hold = 0;
  if (own) {
    g = a.gains[ia];
    hold = a.hold[ia];
    if (rg == 0) {
      if (n == 0) a.g_hist[ia] = g;
      double2 u = zrecip(g);
      if (hold & kHoldFlagged) u = make_double2(0.0, 0.0);
      const double2 c = zmul(a.A[ia], u);
      c_l[an] = make_double2(c.x / a.na_eff, c.y / a.na_eff);
    }
  }
  Stage stg;
  int cur = 0;
  {
    const int nr = min(rpc, len);
    stg.load(ebase, rowstride, t0, nr, RB, tid);
    stg.store(chunk[0], nr, RB, tid);
  }
  __syncthreads();
  double Kx = 0.0, Ky = 0.0, Q = 0.0;
  for (int r0 = 0; r0 < len; r0 += rpc) {
    const int nr = min(rpc, len - r0);
    const bool have_next = r0 + nr < len;
    const int nr_nx = have_next ? min(rpc, len - r0 - nr) : 0;
    if (have_next) stg.load(ebase, rowstride, t0 + r0 + nr, nr_nx, RB, tid);
    const uint8_t* ch = chunk[cur];
    {
      const int q = tid & 15, rr = tid >> 4;
      for (int rb = 0; rb < nr; rb += kSolveThreads / 16) {
        const int r = rb + rr;
        double px = 0.0, py = 0.0;
        if (r < nr) {
          const uint8_t* row = ch + r * RB;
#pragma unroll 4
          for (int k = q; k < a.Na; k += 16) {
            const float2 e = load_sample(row, k, FMT);
            const double2 c = c_l[k];
            px = fma(c.x, double(e.x), fma(-c.y, double(e.y), px));
            py = fma(c.x, double(e.y), fma(c.y, double(e.x), py));
          }
        }
        px = row16_sum_lane15(px);
        py = row16_sum_lane15(py);
        if (q == 15 && r < nr) P_l[r] = make_double2(px, py);
      }
    }
    __syncthreads();
    if (own) {
#pragma unroll 4
      for (int r = rg; r < nr; r += RG) {
        const float2 e = load_sample(ch + r * RB, an, FMT);
        const double ex = e.x, ey = e.y;
        const double2 p = P_l[r];
        Kx = fma(ex, p.x, fma(ey, p.y, Kx));
        Ky = fma(ey, p.x, fma(-ex, p.y, Ky));
        Q = fma(ex, ex, fma(ey, ey, Q));
      }
    }
    if (have_next) stg.store(chunk[cur ^ 1], nr_nx, RB, tid);
    __syncthreads();
    cur ^= 1;
  }
  for (int m = 1; m < RG; m <<= 1) {
    Kx += __shfl_xor(Kx, m);
    Ky += __shfl_xor(Ky, m);
    Q += __shfl_xor(Q, m);
  }
  if (own && rg == 0) {
    double2 s = nan2();
    if (!hold) {
      const double inv_n = 1.0 / double(len);
      const double2 A = a.A[ia], D = a.D[ia];
      const double q = Q * inv_n, na = a.na_eff;
      const double2 t = zdiv(make_double2(A.x * q, -A.y * q), make_double2(na * g.x, -na * g.y));
      const double2 C = make_double2(Kx * inv_n - t.x, Ky * inv_n - t.y);
      s = zdiv(make_double2(C.x * na, C.y * na), D);
    }
    put_shared2(b.raw + ia, s);
  }
}

// Wave-wide sums (all 64 lanes end with the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Least squares by the normal equations: G c = r, G[j][k] = S[j + k]
// (moments of x over the usable channels), Gaussian elimination with
// partial pivoting, m = degree + 1 <= 4 unknowns.
__device__ __noinline__ void normal_solve(const double* S, const double* r, int m, double* c) {
  double M[4][5];
  for (int j = 0; j < m; ++j) {
    for (int k = 0; k < m; ++k) M[j][k] = S[j + k];
    M[j][m] = r[j];
  }
  for (int p = 0; p < m; ++p) {
    int piv = p;
    for (int j = p + 1; j < m; ++j)
      if (fabs(M[j][p]) > fabs(M[piv][p])) piv = j;
    if (piv != p)
      for (int k = 0; k <= m; ++k) {
        const double t = M[p][k];
        M[p][k] = M[piv][k];
        M[piv][k] = t;
      }
    for (int j = p + 1; j < m; ++j) {
      const double l = M[j][p] / M[p][p];
      for (int k = p; k <= m; ++k) M[j][k] -= l * M[p][k];
    }
  }
  for (int p = m - 1; p >= 0; --p) {
    double v = M[p][m];
    for (int k = p + 1; k < m; ++k) v -= M[p][k] * c[k];
    c[p] = v / M[p][p];
  }
}

__device__ __forceinline__ double wrap_pi(double d) {
  const double two_pi = 6.283185307179586476925286766559;
  return d - two_pi * rint(d / two_pi);
}

// Phase 2: the band model of antenna `ant`, by one wave (lanes over the
// band's channels in order).
__device__ __noinline__ void band_fit_antenna(const BandArgs& b, int ant) {
  const SolveArgs& a = b.s;
  const int lane = threadIdx.x & 63;
  double* out = b.coef + int64_t(ant) * kBandCoef;
  if (b.mode == kBandMean) {
    double sx = 0.0, sy = 0.0, cnt = 0.0;
    for (int f = b.b0 + lane; f < b.b1; f += 64) {
      const double2 s = get_shared2(b.raw + int64_t(f) * a.Na + ant);
      if (isfinite(s.x) && isfinite(s.y)) {
        sx += s.x;
        sy += s.y;
        cnt += 1.0;
      }
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    cnt = wave_sum(cnt);
    if (lane == 0) {
      put_shared(out, cnt > 0 ? sx / cnt : __builtin_nan(""));
      put_shared(out + 1, cnt > 0 ? sy / cnt : __builtin_nan(""));
    }
    return;
  }
  // poly: moments of x (up to twice the larger degree), of x^k |s| and of
  // x^k phase, the phase unwrapped along the usable channels in order
  const int da = b.deg_amp, dp = b.deg_phase;
  double S[2 * kBandMaxDeg + 1], T[kBandMaxDeg + 1], U[kBandMaxDeg + 1];
#pragma unroll
  for (int k = 0; k <= 2 * kBandMaxDeg; ++k) S[k] = 0.0;
#pragma unroll
  for (int k = 0; k <= kBandMaxDeg; ++k) T[k] = U[k] = 0.0;
  bool have = false;          // a usable channel before this chunk
  double last_raw = 0.0;      // its wrapped phase
  double last_unw = 0.0;      // its unwrapped phase
  for (int c0 = b.b0; c0 < b.b1; c0 += 64) {
    const int f = c0 + lane;
    double2 s = make_double2(0.0, 0.0);
    bool ok = false;
    if (f < b.b1) {
      s = get_shared2(b.raw + int64_t(f) * a.Na + ant);
      // a solution of exactly zero has no phase: not usable for this model
      ok = isfinite(s.x) && isfinite(s.y) && (s.x != 0.0 || s.y != 0.0);
    }
    const double ph = ok ? atan2(s.y, s.x) : 0.0;
    const uint64_t mask = __ballot(ok);
    const uint64_t below = mask & ((uint64_t(1) << lane) - 1);
    const int prev = below ? 63 - __builtin_clzll(below) : 0;
    const double ph_prev = __shfl(ph, prev);
    double d = 0.0;
    if (ok) d = below ? wrap_pi(ph - ph_prev) : have ? wrap_pi(ph - last_raw) : ph;
    // inclusive prefix sum of d over the lanes
    double scan = d;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      const double o = __shfl_up(scan, m);
      if (lane >= m) scan += o;
    }
    const double unw = (have ? last_unw : 0.0) + scan;
    if (ok) {
      const double x = b.x[f];
      const double amp = sqrt(s.x * s.x + s.y * s.y);
      double xp = 1.0;
#pragma unroll
      for (int k = 0; k <= 2 * kBandMaxDeg; ++k) {
        S[k] += xp;
        if (k <= kBandMaxDeg) {
          T[k] += xp * amp;
          U[k] += xp * unw;
        }
        xp *= x;
      }
    }
    if (mask) {
      const int lastl = 63 - __builtin_clzll(mask);
      last_raw = __shfl(ph, lastl);
      last_unw = __shfl(unw, lastl);
      have = true;
    }
  }
#pragma unroll
  for (int k = 0; k <= 2 * kBandMaxDeg; ++k) S[k] = wave_sum(S[k]);
#pragma unroll
  for (int k = 0; k <= kBandMaxDeg; ++k) {
    T[k] = wave_sum(T[k]);
    U[k] = wave_sum(U[k]);
  }
  if (lane == 0) {
    double ca[kBandMaxDeg + 1] = {0.0, 0.0, 0.0, 0.0}, cp[kBandMaxDeg + 1] = {0.0, 0.0, 0.0, 0.0};
    const int need = (da > dp ? da : dp) + 1;
    if (S[0] < double(need)) {
      ca[0] = __builtin_nan("");
    } else {
      normal_solve(S, T, da + 1, ca);
      normal_solve(S, U, dp + 1, cp);
    }
#pragma unroll
    for (int k = 0; k <= kBandMaxDeg; ++k) {
      put_shared(out + k, ca[k]);
      put_shared(out + kBandMaxDeg + 1 + k, cp[k]);
    }
  }
}

// Phase 2 for one workgroup: the band model of the antennas its waves own.
__device__ __noinline__ void band_fit_phase(const BandArgs& b) {
  const int G = gridDim.x, wave = threadIdx.x >> 6;
  for (int ant = wave * G + blockIdx.x; ant < b.s.Na; ant += (kSolveThreads / 64) * G) band_fit_antenna(b, ant);
}

// Phase 3: the damped update of one channel (eq. damping) towards the band
// model (band channels) or its own solution (other channels); gain history.
__device__ __noinline__ void band_apply(const BandArgs& b, int f, int n) {
  const SolveArgs& a = b.s;
  const int tid = threadIdx.x;
  int NaP = 16;
  while (NaP < a.Na && NaP < kSolveThreads) NaP <<= 1;
  const int RG = kSolveThreads / NaP;
  const int rg = tid % RG, an = tid / RG;
  if (an >= a.Na || rg != 0) return;
  const int64_t ia = int64_t(f) * a.Na + an;
  double2 g = a.gains[ia];
  const uint8_t hold = a.hold[ia];
  const bool in_band = f >= b.b0 && f < b.b1;
  uint32_t st = 0u;
  if (hold & kHoldFlagged) {
    st = 1u;
  } else {
    double2 target;
    const double* cp = b.coef + int64_t(an) * kBandCoef;
    if (!in_band) {
      target = get_shared2(b.raw + ia);
    } else if (b.mode == kBandMean) {
      target = make_double2(get_shared(cp), get_shared(cp + 1));
    } else {
      double c[kBandCoef];
#pragma unroll
      for (int k = 0; k < kBandCoef; ++k) c[k] = get_shared(cp + k);
      const double x = b.x[f];
      double amp = 0.0, ph = 0.0;
#pragma unroll
      for (int k = kBandMaxDeg; k >= 0; --k) {
        amp = fma(amp, x, c[k]);
        ph = fma(ph, x, c[kBandMaxDeg + 1 + k]);
      }
      target = isfinite(c[0]) ? make_double2(amp * cos(ph), amp * sin(ph)) : nan2();
    }
    if (!(isfinite(target.x) && isfinite(target.y))) {
      st = in_band ? 8u : (hold & kHoldDZero ? 2u : 4u);
    } else {
      const double2 gn = make_double2((1.0 - a.gamma) * target.x + a.gamma * g.x,
                                      (1.0 - a.gamma) * target.y + a.gamma * g.y);
      if (isfinite(gn.x) && isfinite(gn.y)) g = gn;
      else st = 4u;
    }
  }
  a.gains[ia] = g;
  a.g_hist[(int64_t(n + 1) * a.F + f) * a.Na + an] = g;
  if (st && a.status) a.status[ia] |= st;
}

// A grid barrier that did not complete: the workgroup's channels get NaN
// gains and status bit 16, and the workgroup stops.
__device__ __noinline__ void band_abort(const BandArgs& b) {
  const SolveArgs& a = b.s;
  for (int f = blockIdx.x; f < a.F; f += gridDim.x)
    for (int an = threadIdx.x; an < a.Na; an += kSolveThreads) {
      const int64_t ia = int64_t(f) * a.Na + an;
      a.gains[ia] = nan2();
      if (a.status) a.status[ia] |= 16u;
    }
}

}  // namespace epic
