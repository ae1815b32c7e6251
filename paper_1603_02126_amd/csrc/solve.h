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
//   tap   P(t) = sum_a c_a E_a(t), c_a = A_a(k0) / (Na g_a)   (one wave per row)
//   corr  K_a += E_a(t) conj(P(t)),  Q_a += |E_a(t)|^2       (threads over
//         antenna x row-group; row-group partials meet by lane shuffles)
// and at the end of each interval the FP64 damped update.
// ---------------------------------------------------------------------------
constexpr int kSolveThreads = 1024;
constexpr int kSolveChunkBytes = 16384;
constexpr int kSolveMaxRows = 1024;

// One thread's share of a chunk copy, PS bytes per piece.
template <int PS>
struct Stager {
  static constexpr int PPT0 = kSolveChunkBytes / (kSolveThreads * PS);
  static constexpr int PPT = PPT0 < 4 ? PPT0 : 4;                      // pieces per thread
  static constexpr int CAP = kSolveThreads * PS * PPT;                 // bytes per chunk
  static constexpr int WPP = PS >= 4 ? PS / 4 : 1;                     // 32-bit words per piece
  uint32_t v[PPT * WPP];
  __device__ __forceinline__ void load(const uint8_t* ebase, int64_t rowstride, int64_t t_first, int nrows,
                                       int RB, int tid) {
    const int per_row = RB / PS;
    const int total = nrows * per_row;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int p = tid + k * kSolveThreads;
      if (p < total) {
        const int r = p / per_row, c = p - r * per_row;
        const uint8_t* src = ebase + (t_first + r) * rowstride + c * PS;
        if constexpr (PS == 16) {
          const uint4 w = *reinterpret_cast<const uint4*>(src);
          v[4 * k] = w.x; v[4 * k + 1] = w.y; v[4 * k + 2] = w.z; v[4 * k + 3] = w.w;
        } else if constexpr (PS == 4) {
          v[k] = *reinterpret_cast<const uint32_t*>(src);
        } else {
          v[k] = *src;
        }
      }
    }
  }
  __device__ __forceinline__ void store(uint8_t* dst, int nrows, int RB, int tid) const {
    const int per_row = RB / PS;
    const int total = nrows * per_row;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int p = tid + k * kSolveThreads;
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

// J = antennas per thread slot (Na <= 1024 * J), PS = chunk piece size.
// LDS of one solve workgroup: two chunk buffers, the taps of a chunk and the
// FP32 coefficients c_a (up to 2 * kSolveThreads antennas).
struct SolveSmem {
  static constexpr int P_OFF = 2 * kSolveChunkBytes;
  static constexpr int C_OFF = P_OFF + kSolveMaxRows * 8;
  static constexpr int BYTES = C_OFF + 2 * kSolveThreads * 8;
};

template <int J, int PS>
__device__ __forceinline__ void solve_channel(const SolveArgs& a, int f, uint8_t* smem) {
  uint8_t (*chunk)[kSolveChunkBytes] = reinterpret_cast<uint8_t (*)[kSolveChunkBytes]>(smem);
  float2* P_l = reinterpret_cast<float2*>(smem + SolveSmem::P_OFF);
  float2* c_l = reinterpret_cast<float2*>(smem + SolveSmem::C_OFF);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nwaves = kSolveThreads / 64;
  const int bpe = efmt_bytes(a.fmt);
  const int RB = a.Na * bpe;
  const int64_t rowstride = int64_t(a.F) * RB;
  const uint8_t* ebase = a.efield + int64_t(f) * RB;
  int rpc = Stager<PS>::CAP / RB;
  rpc = rpc < kSolveMaxRows ? rpc : kSolveMaxRows;

  // thread -> (antenna slot, row group); row groups of one antenna are adjacent lanes
  int NaP = 16;
  while (NaP < a.Na && NaP < kSolveThreads) NaP <<= 1;
  const int RG = kSolveThreads / NaP;  // <= 64
  const int rg = tid % RG;
  const int a0 = tid / RG;

  double2 g[J], A[J];
  uint8_t hold[J];
  uint32_t st[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int an = a0 + NaP * j;
    g[j] = A[j] = make_double2(0.0, 0.0);
    hold[j] = 0;
    st[j] = 0u;
    if (an < a.Na) {
      const int64_t ia = int64_t(f) * a.Na + an;
      g[j] = a.gains[ia];
      A[j] = a.A[ia];
      hold[j] = a.hold[ia];
      if (a.g_hist && rg == 0) a.g_hist[ia] = g[j];
    }
  }

  // chunk schedule: (interval n, first row r0 within it)
  auto interval_len = [&](int n) -> int {
    const int64_t t0 = int64_t(n) * a.t_cal;
    return int(min(a.t_cal, a.n_t - t0));
  };
  Stager<PS> stg;
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
    // c_a = A_a u_a / Na, u_a = 1 / g_a (zero for flagged antennas)
    if (rg == 0) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int an = a0 + NaP * j;
        if (an < a.Na) {
          double2 u = zrecip(g[j]);
          if (hold[j] & kHoldFlagged) u = make_double2(0.0, 0.0);
          const double2 c = zmul(A[j], u);
          c_l[an] = make_float2(float(c.x / a.na_eff), float(c.y / a.na_eff));
          a.u_hist[(int64_t(n) * a.F + f) * a.Na + an] = make_float2(float(u.x), float(u.y));
        }
      }
    }
    double Kx[J], Ky[J], Q[J];
#pragma unroll
    for (int j = 0; j < J; ++j) Kx[j] = Ky[j] = Q[j] = 0.0;
    __syncthreads();
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
      // tapped pixel of each row
      for (int r = wave; r < nr; r += nwaves) {
        const uint8_t* row = ch + r * RB;
        float2 p = make_float2(0.f, 0.f);
        for (int an = lane; an < a.Na; an += 64) p = cadd(p, cmul(c_l[an], load_sample(row, an, a.fmt)));
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) p = cadd(p, shfl_xor2(p, m));
        if (lane == 0) P_l[r] = p;
      }
      __syncthreads();
      // correlation with the uncalibrated E-fields
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int an = a0 + NaP * j;
        if (an < a.Na) {
          float kx = 0.f, ky = 0.f, q = 0.f;
          for (int r = rg; r < nr; r += RG) {
            const float2 e = load_sample(ch + r * RB, an, a.fmt);
            const float2 p = P_l[r];
            kx += e.x * p.x + e.y * p.y;
            ky += e.y * p.x - e.x * p.y;
            q += e.x * e.x + e.y * e.y;
          }
          Kx[j] += double(kx);
          Ky[j] += double(ky);
          Q[j] += double(q);
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
        const double2 gn = epical_step(make_double2(Kx[j] * inv_n, Ky[j] * inv_n), Q[j] * inv_n, A[j],
                                       a.D[int64_t(f) * a.Na + an], g[j], hold[j], a.na_eff, a.gamma, &st[j]);
        g[j] = gn;
        if (a.g_hist && rg == 0) a.g_hist[(int64_t(n + 1) * a.F + f) * a.Na + an] = gn;
      }
    }
  }
  if (rg == 0) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int an = a0 + NaP * j;
      if (an < a.Na) {
        a.gains[int64_t(f) * a.Na + an] = g[j];
        if (a.status) a.status[int64_t(f) * a.Na + an] |= st[j];
      }
    }
  }
  __syncthreads();
}

}  // namespace epic
