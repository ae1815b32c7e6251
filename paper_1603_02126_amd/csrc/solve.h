// EPICal calibration solve of one channel (work-item body shared by the
// per-array kernel and the batched kernel).
#pragma once
#include "engine.h"

namespace epic {

// ---------------------------------------------------------------------------
// EPICal solve over all intervals: one 1024-thread workgroup per channel.
//
// The packed E-fields of the channel stream through LDS in chunks of rows
// (one row = one sample of all antennas), double buffered: the next chunk is
// fetched into registers while the current one is processed.  Per chunk:
//   tap   P(t) = sum_a c_a E_a(t), c_a = A_a(k0) / (Na g_a)   (16 lanes per row)
//   corr  K_a += E_a(t) conj(P(t)),  Q_a += |E_a(t)|^2       (threads over
//         antenna x row-group; row-group partials meet by lane shuffles)
// and at the end of each interval the damped update.  The only global
// stores are the gain history (its data registers stay live for a whole
// interval, so no store ever has to drain before the next interval's
// prefetch); the FP32 u = 1/g of every interval is derived from that
// history afterwards (launch_hist_to_u).  The whole recursion
// (c, P, K, Q and the update) is FP64: where the calibrator is weak the first
// intervals of the recursion amplify a relative perturbation of the tap by
// up to 1e4, so FP32 rounding there would move the converged gains by 1e-3.
// The E-fields are integers (or FP32) and enter exactly.
// ---------------------------------------------------------------------------
constexpr int kSolveThreads = 1024;       // multi-pixel and band solves
constexpr int kSolveMainThreads = 512;    // the single-pixel solve (all its kernels and bodies)
constexpr int kSolveChunkBytes = 32768;   // a whole interval of most arrays: one load latency per interval
constexpr int kSolveMaxRows = 1024;

// One thread's share of a chunk copy, PS bytes per piece, at most MAXP
// pieces (registers) per thread, T threads.
template <int PS, int MAXP, int T = kSolveThreads>
struct Stager {
  static constexpr int PPT0 = kSolveChunkBytes / (T * PS);
  static constexpr int PPT = PPT0 < MAXP ? PPT0 : MAXP;               // pieces per thread
  static constexpr int CAP = T * PS * PPT;                             // bytes per chunk
  static constexpr int WPP = PS >= 4 ? PS / 4 : 1;                     // 32-bit words per piece
  uint32_t v[PPT * WPP];
  __device__ __forceinline__ void load(const uint8_t* ebase, int64_t rowstride, int64_t t_first, int nrows,
                                       int RB, int tid) {
    const int per_row = RB / PS;
    const int total = nrows * per_row;
    // every piece is loaded (pieces past the chunk re-read its first piece)
    // so that the loads are not under branches: the next chunk's loads then
    // stay in flight while the current chunk is processed
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int p0 = tid + k * T;
      const int p = p0 < total ? p0 : 0;
      const int r = p / per_row, c = p - r * per_row;
      const uint8_t* src = ebase + (t_first + r) * rowstride + c * PS;
      if constexpr (PS == 16) {
        const uint4 w = gload(reinterpret_cast<const uint4*>(src));
        v[4 * k] = w.x; v[4 * k + 1] = w.y; v[4 * k + 2] = w.z; v[4 * k + 3] = w.w;
      } else if constexpr (PS == 4) {
        v[k] = gload(reinterpret_cast<const uint32_t*>(src));
      } else {
        v[k] = gload(src);
      }
    }
  }
  __device__ __forceinline__ void store(uint8_t* dst, int nrows, int RB, int tid) const {
    const int per_row = RB / PS;
    const int total = nrows * per_row;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int p = tid + k * T;
      if (p < total) {
        const int r = p / per_row, c = p - r * per_row;
        uint8_t* d = dst + r * RB + c * PS;
        if constexpr (PS == 16) {
          *reinterpret_cast<uint4*>(d) = make_uint4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
        } else if constexpr (PS == 4) {
          *reinterpret_cast<uint32_t*>(d) = v[k];
        } else {
          *d = uint8_t(v[k]);
        }
      }
    }
  }
};

// DPP move of a double (two 32-bit halves); lanes without a source read 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double(static_cast<long long>(static_cast<unsigned>(lo)) |
                              (static_cast<long long>(hi) << 32));
}

// Sum over each row of 16 lanes, complete in the row's lane 15.
__device__ __forceinline__ double row16_sum_lane15(double x) {
  x += dpp_f64<0x111>(x);   // row_shr:1
  x += dpp_f64<0x112>(x);   // row_shr:2
  x += dpp_f64<0x114>(x);   // row_shr:4
  x += dpp_f64<0x118>(x);   // row_shr:8
  return x;
}

// Two's complement nibbles / bytes of one packed integer sample -> int (exact).
__device__ __forceinline__ int2 unpack_int(Raw r, int fmt) {
  if (fmt == kCI4) {
    const int b = int(int8_t(uint8_t(r.x)));
    return make_int2(b >> 4, int(int8_t(uint8_t(r.x << 4))) >> 4);
  }
  return make_int2(int(int8_t(uint8_t(r.x))), int(int8_t(uint8_t(r.x >> 8))));
}

// The damped update of eq. (damping) with the two per-antenna constants
// folded in: r = 1 / (Na |g|^2) of this interval's gain (the same factor
// makes c = A conj(g) r) and invD = Na conj(D) / |D|^2, fixed for the run.
//   C = K - conj(A) Q / (Na conj g) = K - conj(A) g (Q r)     (eq. Cna)
//   g' = (1 - gamma) C invD + gamma g                          (eq. cal_solution)
// One real division per antenna and interval instead of six.
__device__ __forceinline__ double2 epical_step_r(double2 Kbar, double Qbar, double2 A, double2 invD, double2 g,
                                                 double r, uint8_t hold, double gamma, uint32_t* st) {
  if (hold) {
    *st |= (hold & kHoldFlagged ? 1u : 0u) | (hold & kHoldDZero ? 2u : 0u);
    return g;
  }
  const double qr = Qbar * r;
  const double2 t = zmul(zconj(A), make_double2(g.x * qr, g.y * qr));
  const double2 sol = zmul(make_double2(Kbar.x - t.x, Kbar.y - t.y), invD);
  const double2 gn = make_double2((1.0 - gamma) * sol.x + gamma * g.x, (1.0 - gamma) * sol.y + gamma * g.y);
  if (!isfinite(gn.x) || !isfinite(gn.y)) {
    *st |= 4u;
    return g;
  }
  return gn;
}

// J = antennas per thread slot (Na <= T * J), PS = chunk piece size, T =
// threads of the workgroup (kSolveMainThreads for every single-pixel solve,
// so that all of them sum in the same order and give identical gains).
// LDS of one solve workgroup: two chunk buffers, the taps of a chunk and the
// coefficients c_a (up to 2 * kSolveThreads antennas), both FP64.
// With several tapped pixels the same areas hold the taps [kMaxPix][256]
// and the coefficients [kMaxPix][kSolveThreads].
constexpr int kSolveMultiRows = kSolveMaxRows / kMaxPix;
struct SolveSmem {
  static constexpr int P_OFF = 2 * kSolveChunkBytes;
  static constexpr int C_OFF = P_OFF + kSolveMaxRows * 16;
  static constexpr int BYTES = C_OFF + kMaxPix * kSolveThreads * 16;
  static_assert(2 * kSolveThreads <= kMaxPix * kSolveThreads, "coefficients of 2048 antennas fit");
};

// Pieces per thread of the single-pixel solve's stager: registers are
// plentiful at 512 threads (two waves per SIMD), scarcer at 1024.
template <int J, int T>
struct MainStageMax {
  static constexpr int value = (J == 1 || T <= 512) ? 8 : 4;
};

// PUBLISH (the fused run): at the start of each interval the FP32 u = 1/g of
// every antenna (zero when flagged) is written to a.u_hist, the values that
// launch_hist_to_u would derive from the gain history, with coherent (sc1)
// stores; once every wave's stores have completed, progress[f] = intervals
// published, an agent-scope store the imaging workgroups poll.
template <int J, int PS, int FMT, int T = kSolveMainThreads, bool PUBLISH = false>
__device__ __forceinline__ void solve_channel_fmt(const SolveArgs& a, int f, uint8_t* smem, int* progress = nullptr) {
  uint8_t (*chunk)[kSolveChunkBytes] = reinterpret_cast<uint8_t (*)[kSolveChunkBytes]>(smem);
  double2* P_l = reinterpret_cast<double2*>(smem + SolveSmem::P_OFF);
  double2* c_l = reinterpret_cast<double2*>(smem + SolveSmem::C_OFF);
  const int tid = threadIdx.x;
  constexpr int bpe = FMT == kCF32 ? 8 : FMT == kCI8 ? 2 : 1;
  const int RB = a.Na * bpe;
  const int64_t rowstride = int64_t(a.F) * RB;
  const uint8_t* ebase = a.efield + int64_t(f) * RB;
  using Stage = Stager<PS, MainStageMax<J, T>::value, T>;
  int rpc = Stage::CAP / RB;
  rpc = rpc < kSolveMaxRows ? rpc : kSolveMaxRows;

  // thread -> (antenna slot, row group); row groups of one antenna are adjacent lanes
  int NaP = 16;
  while (NaP < a.Na && NaP < T) NaP <<= 1;
  const int RG = T / NaP;  // <= 64
  const int rg = tid % RG;
  const int a0 = tid / RG;

  // invD = Na conj(D) / |D|^2 is loaded and formed once: the per-interval
  // update must not wait on memory or on a division by D
  double2 g[J], A[J], invD[J];
  uint8_t hold[J];
  uint32_t st[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int an = a0 + NaP * j;
    g[j] = A[j] = invD[j] = make_double2(0.0, 0.0);
    hold[j] = 0;
    st[j] = 0u;
    if (an < a.Na) {
      const int64_t ia = int64_t(f) * a.Na + an;
      g[j] = gload(a.gains + ia);
      A[j] = gload(a.A + ia);
      const double2 D = gload(a.D + ia);
      const double d2 = D.x * D.x + D.y * D.y;
      invD[j] = make_double2(a.na_eff * D.x / d2, -a.na_eff * D.y / d2);
      hold[j] = gload(a.hold + ia);
      if (rg == 0) gstore(a.g_hist + ia, g[j]);
    }
  }

  // chunk schedule: (interval n, first row r0 within it)
  auto interval_len = [&](int n) -> int {
    const int64_t t0 = int64_t(n) * a.t_cal;
    return int(min(a.t_cal, a.n_t - t0));
  };
  Stage stg;
  int cur_buf = 0;
  {
    const int nr = min(rpc, interval_len(0));
    stg.load(ebase, rowstride, 0, nr, RB, tid);
    stg.store(chunk[0], nr, RB, tid);
  }
  __syncthreads();

  for (int n = 0; n < a.n_int; ++n) {
    const int64_t t0 = int64_t(n) * a.t_cal;
    const int len = interval_len(n);
    // c_a = A_a u_a / Na = A_a conj(g_a) r_a, u_a = 1 / g_a (zero for flagged antennas)
    double rr[J];
#pragma unroll
    for (int j = 0; j < J; ++j) rr[j] = 1.0 / (a.na_eff * (g[j].x * g[j].x + g[j].y * g[j].y));
    if (rg == 0) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int an = a0 + NaP * j;
        if (an < a.Na) {
          double2 c = zmul(A[j], make_double2(g[j].x * rr[j], -g[j].y * rr[j]));
          if (hold[j] & kHoldFlagged) c = make_double2(0.0, 0.0);
          c_l[an] = c;
          if constexpr (PUBLISH) {
            double2 u = zrecip(g[j]);
            if (hold[j] & kHoldFlagged) u = make_double2(0.0, 0.0);
            const float2 uf = make_float2(float(u.x), float(u.y));
            __hip_atomic_store((__attribute__((address_space(1))) uint64_t*)(a.u_hist + (int64_t(n) * a.F + f) * a.Na + an),
                               __builtin_bit_cast(uint64_t, uf), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
    }
    if constexpr (PUBLISH) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's u stores are done
    double Kx[J], Ky[J], Q[J];
#pragma unroll
    for (int j = 0; j < J; ++j) Kx[j] = Ky[j] = Q[j] = 0.0;
    __syncthreads();
    if constexpr (PUBLISH) {
      if (tid == 0)
        __hip_atomic_store((__attribute__((address_space(1))) int*)(progress + f), n + 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int r0 = 0; r0 < len; r0 += rpc) {
      const int nr = min(rpc, len - r0);
      // prefetch the following chunk (this interval or the next one)
      int n_nx = n, r_nx = r0 + nr;
      if (r_nx >= len) {
        n_nx = n + 1;
        r_nx = 0;
      }
      const bool have_next = n_nx < a.n_int;
      const int nr_nx = have_next ? min(rpc, interval_len(n_nx) - r_nx) : 0;
      if (have_next) stg.load(ebase, rowstride, int64_t(n_nx) * a.t_cal + r_nx, nr_nx, RB, tid);

      const uint8_t* ch = chunk[cur_buf];
      // tapped pixel of each row: 16 lanes per row (antennas strided by 16),
      // 64 rows per pass, sums within each 16-lane DPP row
      {
        const int q = tid & 15, rr = tid >> 4;
        for (int rb = 0; rb < nr; rb += T / 16) {
          const int r = rb + rr;
          double px = 0.0, py = 0.0;
          if (r < nr) {
            const uint8_t* row = ch + r * RB;
#pragma unroll 4
            for (int an = q; an < a.Na; an += 16) {
              double ex, ey;
              if constexpr (FMT == kCF32) {
                const float2 e = load_sample(row, an, FMT);
                ex = e.x;
                ey = e.y;
              } else {
                const int2 e = unpack_int(load_raw(row, an, FMT), FMT);
                ex = e.x;
                ey = e.y;
              }
              const double2 c = c_l[an];
              px = fma(c.x, ex, fma(-c.y, ey, px));
              py = fma(c.x, ey, fma(c.y, ex, py));
            }
          }
          px = row16_sum_lane15(px);
          py = row16_sum_lane15(py);
          if (q == 15 && r < nr) P_l[r] = make_double2(px, py);
        }
      }
      __syncthreads();
      // correlation with the uncalibrated E-fields
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int an = a0 + NaP * j;
        if (an < a.Na) {
          double kx = 0.0, ky = 0.0;
          if constexpr (FMT == kCF32) {
            double q = 0.0;
#pragma unroll 4
            for (int r = rg; r < nr; r += RG) {
              const float2 e = load_sample(ch + r * RB, an, FMT);
              const double ex = e.x, ey = e.y;
              const double2 p = P_l[r];
              kx = fma(ex, p.x, fma(ey, p.y, kx));
              ky = fma(ey, p.x, fma(-ex, p.y, ky));
              q = fma(ex, ex, fma(ey, ey, q));
            }
            Q[j] += q;
          } else {
            // |E|^2 of integer samples summed exactly in integers (at most
            // 1024 rows of 2 * 128^2 per chunk)
            int qi = 0;
#pragma unroll 4
            for (int r = rg; r < nr; r += RG) {
              const int2 e = unpack_int(load_raw(ch + r * RB, an, FMT), FMT);
              const double ex = e.x, ey = e.y;
              const double2 p = P_l[r];
              kx = fma(ex, p.x, fma(ey, p.y, kx));
              ky = fma(ey, p.x, fma(-ex, p.y, ky));
              qi += e.x * e.x + e.y * e.y;
            }
            Q[j] += double(qi);
          }
          Kx[j] += kx;
          Ky[j] += ky;
        }
      }
      if (have_next) stg.store(chunk[cur_buf ^ 1], nr_nx, RB, tid);
      __syncthreads();
      cur_buf ^= 1;
    }
    // combine row groups (adjacent lanes), then the damped update (FP64)
#pragma unroll
    for (int j = 0; j < J; ++j) {
      for (int m = 1; m < RG; m <<= 1) {
        Kx[j] += __shfl_xor(Kx[j], m);
        Ky[j] += __shfl_xor(Ky[j], m);
        Q[j] += __shfl_xor(Q[j], m);
      }
    }
    const double inv_n = 1.0 / double(len);
    (void)t0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int an = a0 + NaP * j;
      if (an < a.Na) {
        const double2 gn = epical_step_r(make_double2(Kx[j] * inv_n, Ky[j] * inv_n), Q[j] * inv_n, A[j],
                                         invD[j], g[j], rr[j], hold[j], a.gamma, &st[j]);
        g[j] = gn;
        if (rg == 0) gstore(a.g_hist + (int64_t(n + 1) * a.F + f) * a.Na + an, gn);
      }
    }
  }
  if (rg == 0) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int an = a0 + NaP * j;
      if (an < a.Na) {
        gstore(a.gains + int64_t(f) * a.Na + an, g[j]);
        if (a.status) {
          uint32_t* sp = a.status + int64_t(f) * a.Na + an;
          gstore(sp, gload(sp) | st[j]);
        }
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// EPICal solve of one channel by a single wave, for small arrays with short
// calibration intervals (Na <= 64, t_cal <= kSolveWaveMaxTcal).  There the
// recursion is a chain of tiny dependent steps and its latency sets the time:
// lane a owns antenna a, the tap of a sample is a wave-wide DPP sum (no
// workgroup barriers), and the samples stream through a 64-row LDS block that
// is requested one block ahead, so no step waits on memory.
// ---------------------------------------------------------------------------
constexpr int kSolveWaveMaxAnt = 64;
constexpr int kSolveWaveMaxTcal = 8;
constexpr int kSolveWaveRows = 64;

// Sum of x over the 64 lanes, returned to every lane.
__device__ __forceinline__ double wave_sum64(double x) {
  x = row16_sum_lane15(x);                       // lane 16 r + 15: sum of row r
  x += dpp_f64<0x142, 0xa>(x);                   // row_bcast:15 -> lanes 31, 63: rows 0+1, 2+3
  x += dpp_f64<0x143, 0xc>(x);                   // row_bcast:31 -> lane 63: all four rows
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(int(b), 63), hi = __builtin_amdgcn_readlane(int(b >> 32), 63);
  return __longlong_as_double(static_cast<long long>(static_cast<unsigned>(lo)) | (static_cast<long long>(hi) << 32));
}

template <int FMT>
__device__ __forceinline__ void solve_channel_wave(const SolveArgs& a, int f, float2* ring) {
  const int lane = threadIdx.x & 63;
  const bool own = lane < a.Na;
  constexpr int bpe = FMT == kCF32 ? 8 : FMT == kCI8 ? 2 : 1;
  const int64_t rowstride = int64_t(a.F) * a.Na * bpe;
  const uint8_t* ebase = a.efield + int64_t(f) * a.Na * bpe;
  const int64_t ia = int64_t(f) * a.Na + (own ? lane : 0);
  // the constants folded as in solve_channel_fmt (epical_step_r): invD once,
  // one real division per update for r = 1 / (Na |g|^2)
  double2 g = make_double2(0.0, 0.0), A = g, invD = g;
  uint8_t hold = 0;
  uint32_t st = 0u;
  if (own) {
    g = a.gains[ia];
    A = a.A[ia];
    const double2 D = a.D[ia];
    const double d2 = D.x * D.x + D.y * D.y;
    invD = make_double2(a.na_eff * D.x / d2, -a.na_eff * D.y / d2);
    hold = a.hold[ia];
    a.g_hist[ia] = g;
  }
  // samples of rows [64 b, 64 b + 64) for this lane's antenna, one block ahead
  float2 pre[kSolveWaveRows];
  auto request = [&](int64_t b) {
    static_for<0, kSolveWaveRows>([&](auto kc) {
      const int64_t t = b * kSolveWaveRows + decltype(kc)::value;
      pre[decltype(kc)::value] = (own && t < a.n_t) ? load_sample_global(ebase + t * rowstride, lane, FMT)
                                                    : make_float2(0.f, 0.f);
    });
  };
  request(0);
  double2 c = make_double2(0.0, 0.0);
  double rr = 0.0;
  // c_a = A_a u_a / Na = A_a conj(g_a) r_a (zero for flagged antennas and idle lanes)
  auto coefficient = [&]() {
    rr = 1.0 / (a.na_eff * (g.x * g.x + g.y * g.y));
    c = zmul(A, make_double2(g.x * rr, -g.y * rr));
    if (!own || (hold & kHoldFlagged)) c = make_double2(0.0, 0.0);
  };
  coefficient();
  double kx = 0.0, ky = 0.0, q = 0.0;
  int n = 0;
  int64_t t_end = min(a.t_cal, a.n_t);
  for (int64_t t = 0; t < a.n_t; ++t) {
    if ((t & (kSolveWaveRows - 1)) == 0) {
      // entering block t / 64: its samples arrived during the previous block
      static_for<0, kSolveWaveRows>([&](auto kc) { ring[decltype(kc)::value * 64 + lane] = pre[decltype(kc)::value]; });
      wave_lds_sync();
      request(t / kSolveWaveRows + 1);
    }
    const float2 e = ring[(t & (kSolveWaveRows - 1)) * 64 + lane];
    const double ex = e.x, ey = e.y;
    // tap P(t) = sum_a c_a E_a(t), then K_a += E_a conj(P), Q_a += |E_a|^2
    const double px = wave_sum64(fma(c.x, ex, -c.y * ey));
    const double py = wave_sum64(fma(c.x, ey, c.y * ex));
    kx = fma(ex, px, fma(ey, py, kx));
    ky = fma(ey, px, fma(-ex, py, ky));
    q = fma(ex, ex, fma(ey, ey, q));
    if (t + 1 == t_end) {
      const double inv_n = 1.0 / double(t_end - int64_t(n) * a.t_cal);
      g = epical_step_r(make_double2(kx * inv_n, ky * inv_n), q * inv_n, A, invD, g, rr, hold, a.gamma, &st);
      if (own) a.g_hist[(int64_t(n + 1) * a.F + f) * a.Na + lane] = g;
      kx = ky = q = 0.0;
      ++n;
      t_end = min(t_end + a.t_cal, a.n_t);
      coefficient();
    }
  }
  if (own) {
    a.gains[ia] = g;
    if (a.status) a.status[ia] |= st;
  }
}

// ---------------------------------------------------------------------------
// EPICal from several tapped pixels (the multiple-pixel extension of Sec. 6):
// per interval the taps P_p(t) = sum_a c_pa E_a(t) of every pixel, the
// correlations K_ap = <E_a P_p*>, and the least-squares update over the
// pixels (epical_step_multi).  Na <= T, at most kMaxPix pixels; the loops
// over pixels are unrolled to kMaxPix with guards.  T threads (kSolveThreads
// in its own launch, kSolveMainThreads as a task of the fused run); PUBLISH
// as in the single-pixel solve: u = 1/g of every antenna is written to
// a.u_hist at the start of each interval and progress[f] raised once every
// wave's stores have completed.
// ---------------------------------------------------------------------------
template <int PS, int FMT, int T = kSolveThreads, bool PUBLISH = false>
__device__ __forceinline__ void solve_channel_multi(const SolveArgs& a, int f, uint8_t* smem, int* progress = nullptr) {
  static_assert(T <= kSolveThreads, "the coefficient table holds kSolveThreads antennas per pixel");
  uint8_t (*chunk)[kSolveChunkBytes] = reinterpret_cast<uint8_t (*)[kSolveChunkBytes]>(smem);
  double2* P_l = reinterpret_cast<double2*>(smem + SolveSmem::P_OFF);   // [kMaxPix][kSolveMultiRows]
  double2* c_l = reinterpret_cast<double2*>(smem + SolveSmem::C_OFF);   // [kMaxPix][kSolveThreads]
  const int tid = threadIdx.x;
  const int np = a.n_pix;
  constexpr int bpe = FMT == kCF32 ? 8 : FMT == kCI8 ? 2 : 1;
  const int RB = a.Na * bpe;
  const int64_t rowstride = int64_t(a.F) * RB;
  const int64_t pstride = int64_t(a.F) * a.Na;
  const uint8_t* ebase = a.efield + int64_t(f) * RB;
  using Stage = Stager<PS, 8, T>;
  int rpc = Stage::CAP / RB;
  rpc = rpc < kSolveMultiRows ? rpc : kSolveMultiRows;

  int NaP = 16;
  while (NaP < a.Na && NaP < T) NaP <<= 1;
  const int RG = T / NaP;
  const int rg = tid % RG;
  const int an = tid / RG;
  const bool own = an < a.Na;
  const int64_t ia = int64_t(f) * a.Na + (own ? an : 0);

  double2 g = make_double2(0.0, 0.0), A[kMaxPix], D[kMaxPix];
  uint8_t hold = 0;
  uint32_t st = 0u;
#pragma unroll
  for (int p = 0; p < kMaxPix; ++p) {
    A[p] = D[p] = make_double2(0.0, 0.0);
    if (own && p < np) {
      A[p] = a.A[p * pstride + ia];
      D[p] = a.D[p * pstride + ia];
    }
  }
  if (own) {
    g = a.gains[ia];
    hold = a.hold[ia];
    if (rg == 0) a.g_hist[ia] = g;
  }

  auto interval_len = [&](int n) -> int {
    const int64_t t0 = int64_t(n) * a.t_cal;
    return int(min(a.t_cal, a.n_t - t0));
  };
  Stage stg;
  int cur_buf = 0;
  {
    const int nr = min(rpc, interval_len(0));
    stg.load(ebase, rowstride, 0, nr, RB, tid);
    stg.store(chunk[0], nr, RB, tid);
  }
  __syncthreads();

  for (int n = 0; n < a.n_int; ++n) {
    const int len = interval_len(n);
    if (rg == 0 && own) {
      double2 u = zrecip(g);
      if (hold & kHoldFlagged) u = make_double2(0.0, 0.0);
#pragma unroll
      for (int p = 0; p < kMaxPix; ++p)
        if (p < np) {
          const double2 c = zmul(A[p], u);
          c_l[p * kSolveThreads + an] = make_double2(c.x / a.na_eff, c.y / a.na_eff);
        }
      if constexpr (PUBLISH) {
        const float2 uf = make_float2(float(u.x), float(u.y));
        __hip_atomic_store((__attribute__((address_space(1))) uint64_t*)(a.u_hist + (int64_t(n) * a.F + f) * a.Na + an),
                           __builtin_bit_cast(uint64_t, uf), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if constexpr (PUBLISH) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's u stores are done
    double Kx[kMaxPix], Ky[kMaxPix], Q = 0.0;
#pragma unroll
    for (int p = 0; p < kMaxPix; ++p) Kx[p] = Ky[p] = 0.0;
    __syncthreads();
    if constexpr (PUBLISH) {
      if (tid == 0)
        __hip_atomic_store((__attribute__((address_space(1))) int*)(progress + f), n + 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int r0 = 0; r0 < len; r0 += rpc) {
      const int nr = min(rpc, len - r0);
      int n_nx = n, r_nx = r0 + nr;
      if (r_nx >= len) {
        n_nx = n + 1;
        r_nx = 0;
      }
      const bool have_next = n_nx < a.n_int;
      const int nr_nx = have_next ? min(rpc, interval_len(n_nx) - r_nx) : 0;
      if (have_next) stg.load(ebase, rowstride, int64_t(n_nx) * a.t_cal + r_nx, nr_nx, RB, tid);
      const uint8_t* ch = chunk[cur_buf];
      // taps of every pixel: 16 lanes per row, DPP sums within the 16-lane row
      {
        const int q = tid & 15, rr = tid >> 4;
        for (int rb = 0; rb < nr; rb += T / 16) {
          const int r = rb + rr;
          double px[kMaxPix], py[kMaxPix];
#pragma unroll
          for (int p = 0; p < kMaxPix; ++p) px[p] = py[p] = 0.0;
          if (r < nr) {
            const uint8_t* row = ch + r * RB;
            for (int k = q; k < a.Na; k += 16) {
              const float2 e = load_sample(row, k, FMT);
              const double ex = e.x, ey = e.y;
#pragma unroll
              for (int p = 0; p < kMaxPix; ++p)
                if (p < np) {
                  const double2 c = c_l[p * kSolveThreads + k];
                  px[p] = fma(c.x, ex, fma(-c.y, ey, px[p]));
                  py[p] = fma(c.x, ey, fma(c.y, ex, py[p]));
                }
            }
          }
#pragma unroll
          for (int p = 0; p < kMaxPix; ++p)
            if (p < np) {
              const double sx = row16_sum_lane15(px[p]), sy = row16_sum_lane15(py[p]);
              if (q == 15 && r < nr) P_l[p * kSolveMultiRows + r] = make_double2(sx, sy);
            }
        }
      }
      __syncthreads();
      if (own) {
#pragma unroll 2
        for (int r = rg; r < nr; r += RG) {
          const float2 e = load_sample(ch + r * RB, an, FMT);
          const double ex = e.x, ey = e.y;
#pragma unroll
          for (int p = 0; p < kMaxPix; ++p)
            if (p < np) {
              const double2 P = P_l[p * kSolveMultiRows + r];
              Kx[p] = fma(ex, P.x, fma(ey, P.y, Kx[p]));
              Ky[p] = fma(ey, P.x, fma(-ex, P.y, Ky[p]));
            }
          Q = fma(ex, ex, fma(ey, ey, Q));
        }
      }
      if (have_next) stg.store(chunk[cur_buf ^ 1], nr_nx, RB, tid);
      __syncthreads();
      cur_buf ^= 1;
    }
    for (int m = 1; m < RG; m <<= 1) {
#pragma unroll
      for (int p = 0; p < kMaxPix; ++p) {
        Kx[p] += __shfl_xor(Kx[p], m);
        Ky[p] += __shfl_xor(Ky[p], m);
      }
      Q += __shfl_xor(Q, m);
    }
    if (own) {
      const double inv_n = 1.0 / double(len);
      double2 Kb[kMaxPix];
#pragma unroll
      for (int p = 0; p < kMaxPix; ++p) Kb[p] = make_double2(Kx[p] * inv_n, Ky[p] * inv_n);
      g = epical_step_multi(Kb, Q * inv_n, A, D, np, g, hold, a.na_eff, a.gamma, &st);
      if (rg == 0) a.g_hist[(int64_t(n + 1) * a.F + f) * a.Na + an] = g;
    }
  }
  if (rg == 0 && own) {
    a.gains[ia] = g;
    if (a.status) a.status[ia] |= st;
  }
  __syncthreads();
}

// Format dispatch of the single-pixel solve (kSolveMainThreads threads): the
// E-field format is a compile-time constant of the inner loops.
template <int J, int PS>
__device__ __forceinline__ void solve_channel(const SolveArgs& a, int f, uint8_t* smem) {
  if (a.fmt == kCI4) solve_channel_fmt<J, PS, kCI4>(a, f, smem);
  else if (a.fmt == kCI8) solve_channel_fmt<J, PS, kCI8>(a, f, smem);
  else solve_channel_fmt<J, PS, kCF32>(a, f, smem);
}

// Several tapped pixels (kSolveThreads threads).
template <int PS>
__device__ __forceinline__ void solve_channel_pixels(const SolveArgs& a, int f, uint8_t* smem) {
  if (a.fmt == kCI4) solve_channel_multi<PS, kCI4>(a, f, smem);
  else if (a.fmt == kCI8) solve_channel_multi<PS, kCI8>(a, f, smem);
  else solve_channel_multi<PS, kCF32>(a, f, smem);
}

}  // namespace epic
