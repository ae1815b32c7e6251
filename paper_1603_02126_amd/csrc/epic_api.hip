// Host side of the EPIC library: argument checks, plan tables (gridding
// cells, calibrator pixel response, model denominator), scratch memory,
// dispatch and the extern "C" entry points declared in include/epic.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/epic.h"
#include "epic_internal.h"

using epic::ImageArgs;
using zc = std::complex<double>;

namespace {

constexpr double kC = 299792458.0;
constexpr double kTwoPi = 6.283185307179586476925286766559;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(EPIC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Validated copy of one epic_array_desc.
struct HostArray {
  int na = 0, F = 0, nx = 0, ny = 0, kernel = 1, efmt = 0, k2 = 1;
  double dx = 0, dy = 0, x0 = 0, y0 = 0;
  std::vector<double> xy, freq;
  std::vector<uint8_t> flag;
  int na_eff = 0;
};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_desc(const epic_array_desc* d, HostArray* out) {
  if (!d) return fail(EPIC_ERR_ARG, "array descriptor is NULL");
  if (d->n_ant < 1) return fail(EPIC_ERR_ARG, "n_ant must be >= 1 (got %d)", d->n_ant);
  if (d->n_chan < 1) return fail(EPIC_ERR_ARG, "n_chan must be >= 1 (got %d)", d->n_chan);
  if (!is_pow2(d->nx) || !is_pow2(d->ny) || d->nx < 2 || d->ny < 2 || d->nx > 4096 || d->ny > 4096)
    return fail(EPIC_ERR_ARG, "nx, ny must be powers of two in [2, 4096] (got %d x %d)", d->nx, d->ny);
  if (d->kernel != 1 && d->kernel != 2) return fail(EPIC_ERR_ARG, "kernel must be 1 or 2 (got %d)", d->kernel);
  if (d->efmt < EPIC_CF32 || d->efmt > EPIC_CI4) return fail(EPIC_ERR_ARG, "unknown efmt %d", d->efmt);
  if (!(d->dx > 0) || !(d->dy > 0) || !std::isfinite(d->dx) || !std::isfinite(d->dy))
    return fail(EPIC_ERR_ARG, "dx, dy must be positive and finite");
  if (!std::isfinite(d->x0) || !std::isfinite(d->y0)) return fail(EPIC_ERR_ARG, "x0, y0 must be finite");
  if (!d->ant_xy) return fail(EPIC_ERR_ARG, "ant_xy is NULL");
  if (!d->freq_hz) return fail(EPIC_ERR_ARG, "freq_hz is NULL");
  HostArray h;
  h.na = d->n_ant;
  h.F = d->n_chan;
  h.nx = d->nx;
  h.ny = d->ny;
  h.kernel = d->kernel;
  h.k2 = d->kernel == 1 ? 1 : 4;
  h.efmt = d->efmt;
  h.dx = d->dx;
  h.dy = d->dy;
  h.x0 = d->x0;
  h.y0 = d->y0;
  h.xy.assign(d->ant_xy, d->ant_xy + 2 * size_t(h.na));
  h.freq.assign(d->freq_hz, d->freq_hz + h.F);
  for (double v : h.xy)
    if (!std::isfinite(v)) return fail(EPIC_ERR_ARG, "antenna positions must be finite");
  for (double v : h.freq)
    if (!(v > 0) || !std::isfinite(v)) return fail(EPIC_ERR_ARG, "frequencies must be positive and finite");
  h.flag.assign(h.na, 0);
  if (d->ant_flag)
    for (int a = 0; a < h.na; ++a) h.flag[a] = d->ant_flag[a] ? 1 : 0;
  h.na_eff = 0;
  for (int a = 0; a < h.na; ++a) h.na_eff += h.flag[a] == 0;
  if (out) *out = std::move(h);
  return EPIC_OK;
}

// Gridding cells and weights (eq. gridding): nearest cell or 2x2 bilinear
// (area overlap of a one-cell tophat); indices wrap modulo the grid size.
void grid_cells(const HostArray& h, std::vector<int32_t>& ix, std::vector<int32_t>& iy, std::vector<double>& w) {
  ix.assign(size_t(h.na) * h.k2, 0);
  iy.assign(size_t(h.na) * h.k2, 0);
  w.assign(size_t(h.na) * h.k2, 0.0);
  auto wrap = [](long long v, int n) { long long r = v % n; return int32_t(r < 0 ? r + n : r); };
  for (int a = 0; a < h.na; ++a) {
    const double px = (h.xy[2 * a] - h.x0) / h.dx;
    const double py = (h.xy[2 * a + 1] - h.y0) / h.dy;
    if (h.kernel == 1) {
      ix[a] = wrap((long long)std::floor(px + 0.5), h.nx);
      iy[a] = wrap((long long)std::floor(py + 0.5), h.ny);
      w[a] = 1.0;
    } else {
      const double fx = std::floor(px), fy = std::floor(py);
      const double ax = px - fx, ay = py - fy;
      const long long i0 = (long long)fx, j0 = (long long)fy;
      const long long cx[4] = {i0, i0 + 1, i0, i0 + 1}, cy[4] = {j0, j0, j0 + 1, j0 + 1};
      const double cw[4] = {(1 - ax) * (1 - ay), ax * (1 - ay), (1 - ax) * ay, ax * ay};
      for (int k = 0; k < 4; ++k) {
        ix[4 * a + k] = wrap(cx[k], h.nx);
        iy[4 * a + k] = wrap(cy[k], h.ny);
        w[4 * a + k] = cw[k];
      }
    }
  }
}

struct ModelTables {
  std::vector<int32_t> k0;   // [n_pix][F][2]
  std::vector<zc> A, D;      // [n_pix][F][Na]
  std::vector<uint8_t> hold; // [F][Na]
};

static int check_pixels(const double* pix_lm, int n_pix) {
  if (!pix_lm) return fail(EPIC_ERR_ARG, "pixel directions are NULL");
  if (n_pix < 1 || n_pix > EPIC_MAX_PIX) return fail(EPIC_ERR_ARG, "n_pix must be in 1..%d (got %d)", EPIC_MAX_PIX, n_pix);
  for (int i = 0; i < 2 * n_pix; ++i)
    if (!std::isfinite(pix_lm[i])) return fail(EPIC_ERR_ARG, "pixel direction not finite");
  return EPIC_OK;
}

int check_model(const epic_model_desc* m) {
  if (!m) return fail(EPIC_ERR_ARG, "model descriptor is NULL");
  if (!m->src_lmS || m->n_src < 1) return fail(EPIC_ERR_ARG, "model needs at least one source");
  if (!(m->gamma >= 0.0 && m->gamma < 1.0)) return fail(EPIC_ERR_ARG, "gamma must be in [0, 1) (got %g)", m->gamma);
  if (m->t_cal < 1) return fail(EPIC_ERR_ARG, "t_cal must be >= 1 (got %d)", m->t_cal);
  if (!std::isfinite(m->cal_l) || !std::isfinite(m->cal_m)) return fail(EPIC_ERR_ARG, "calibrator direction not finite");
  for (int s = 0; s < 3 * m->n_src; ++s)
    if (!std::isfinite(m->src_lmS[s])) return fail(EPIC_ERR_ARG, "model sources must be finite");
  return EPIC_OK;
}

// k0, A_a(k0) and the model denominator D_a per channel.
//   A_a = sum_k w_ak exp(+2 pi i (jx kx / nx + jy ky / ny))
//   D_a = sum_{b != a, unflagged} conj(A_b) V^M_ab,
//   V^M_ab = sum_s S_s e_a(s) conj(e_b(s)),  e_a(s) = exp(-2 pi i f r_a . s / c)
// factored as D_a = sum_s S_s e_a(s) B(s) - [a unflagged] conj(A_a) sum_s S_s
// with B(s) = sum_{b unflagged} conj(A_b) conj(e_b(s)).
// Tapped pixels: pix_lm [n_pix][2] or, when null, the model's calibrator.
void model_tables(const HostArray& h, const epic_model_desc* m, ModelTables& t, const double* pix_lm = nullptr,
                  int n_pix = 1) {
  std::vector<int32_t> ix, iy;
  std::vector<double> w;
  grid_cells(h, ix, iy, w);
  const size_t FN = size_t(h.F) * h.na;
  t.k0.assign(2 * size_t(h.F) * n_pix, 0);
  t.A.assign(FN * n_pix, zc(0, 0));
  t.D.assign(FN * n_pix, zc(0, 0));
  t.hold.assign(FN, 0);
  const int ns = m->n_src;
  double Stot = 0;
  for (int s = 0; s < ns; ++s) Stot += m->src_lmS[3 * s + 2];
  std::vector<zc> e(size_t(h.na) * ns);
  std::vector<double> den(h.na);
  for (int f = 0; f < h.F; ++f) {
    const double fr = h.freq[f];
    for (int a = 0; a < h.na; ++a)
      for (int s = 0; s < ns; ++s) {
        const double l = m->src_lmS[3 * s], mm = m->src_lmS[3 * s + 1];
        const double ph = -kTwoPi * fr * (h.xy[2 * a] * l + h.xy[2 * a + 1] * mm) / kC;
        e[size_t(a) * ns + s] = zc(std::cos(ph), std::sin(ph));
      }
    std::fill(den.begin(), den.end(), 0.0);
    for (int p = 0; p < n_pix; ++p) {
      const double pl = pix_lm ? pix_lm[2 * p] : m->cal_l, pm = pix_lm ? pix_lm[2 * p + 1] : m->cal_m;
      const long long kxs = (long long)std::floor(pl * fr * h.nx * h.dx / kC + 0.5);
      const long long kys = (long long)std::floor(pm * fr * h.ny * h.dy / kC + 0.5);
      const long long kx = ((kxs % h.nx) + h.nx) % h.nx, ky = ((kys % h.ny) + h.ny) % h.ny;
      t.k0[2 * (size_t(p) * h.F + f)] = int32_t(kx);
      t.k0[2 * (size_t(p) * h.F + f) + 1] = int32_t(ky);
      zc* A = &t.A[size_t(p) * FN + size_t(f) * h.na];
      for (int a = 0; a < h.na; ++a) {
        zc s(0, 0);
        for (int k = 0; k < h.k2; ++k) {
          const size_t q = size_t(a) * h.k2 + k;
          const double ph = kTwoPi * (double((ix[q] * kx) % h.nx) / h.nx + double((iy[q] * ky) % h.ny) / h.ny);
          s += w[q] * zc(std::cos(ph), std::sin(ph));
        }
        A[a] = s;
      }
      std::vector<zc> B(ns, zc(0, 0));
      for (int b = 0; b < h.na; ++b) {
        if (h.flag[b]) continue;
        for (int s = 0; s < ns; ++s) B[s] += std::conj(A[b]) * std::conj(e[size_t(b) * ns + s]);
      }
      zc* D = &t.D[size_t(p) * FN + size_t(f) * h.na];
      for (int a = 0; a < h.na; ++a) {
        zc acc(0, 0);
        for (int s = 0; s < ns; ++s) acc += m->src_lmS[3 * s + 2] * e[size_t(a) * ns + s] * B[s];
        if (!h.flag[a]) acc -= std::conj(A[a]) * Stot;
        D[a] = acc;
        den[a] += std::norm(acc);
      }
    }
    const double dmax = *std::max_element(den.begin(), den.end());
    for (int a = 0; a < h.na; ++a) {
      uint8_t hb = 0;
      if (h.flag[a]) hb |= epic::kHoldFlagged;
      if (!(den[a] > 1e-24 * dmax)) hb |= epic::kHoldDZero;   // sum_p |D_ap|^2 vs (1e-12 max)^2
      t.hold[size_t(f) * h.na + a] = hb;
    }
  }
}

// Owner-computes gridding schedule of the N <= 64 imaging engine: every
// nonzero cell goes to one lane (greedy balance of contribution counts); each
// lane gets consecutive slots per owned cell, coded
//   antenna | LDS cell offset << 12 | first-of-cell << 31,  weight bits.
// Padding slots store zero into the pad column (offset = grid size).
// Returns the slot count S; table is [S][L] (lane fastest), 2 words each.
// half >= 0: the columns 32 half <= x < 32 half + 32 only, at offsets
// y * kHalfPitch + x - 32 half of the half-frame buffer (pad: column 32).
int build_slots(const HostArray& h, int L, int pitch, std::vector<uint32_t>& table, bool transposed = false,
                int half = -1) {
  std::vector<int32_t> ix, iy;
  std::vector<double> w;
  grid_cells(h, ix, iy, w);
  std::vector<std::vector<std::pair<int, float>>> cell(size_t(h.nx) * h.ny);
  for (int a = 0; a < h.na; ++a) {
    if (h.flag[a]) continue;
    for (int k = 0; k < h.k2; ++k) {
      const size_t q = size_t(a) * h.k2 + k;
      if (w[q] == 0.0) continue;
      if (half >= 0 && ix[q] / 32 != half) continue;
      cell[size_t(iy[q]) * h.nx + ix[q]].push_back({a, float(w[q])});
    }
  }
  std::vector<int> order;
  for (size_t c = 0; c < cell.size(); ++c)
    if (!cell[c].empty()) order.push_back(int(c));
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cell[x].size() > cell[y].size(); });
  std::vector<std::vector<int>> lane_cells(L);
  std::vector<size_t> load(L, 0);
  for (int c : order) {
    int best = 0;
    for (int l = 1; l < L; ++l)
      if (load[l] < load[best]) best = l;
    lane_cells[best].push_back(c);
    load[best] += cell[c].size();
  }
  size_t S = 0;
  for (int l = 0; l < L; ++l) S = std::max(S, load[l]);
  const uint32_t pad = uint32_t(half >= 0 ? 32 : h.nx) << 12;   // row 0, first pad column
  table.assign(2 * S * L, 0u);
  for (int l = 0; l < L; ++l) {
    size_t s = 0;
    for (int c : lane_cells[l]) {
      const int cy = c / h.nx, cx = c % h.nx;
      const uint32_t off = half >= 0   ? uint32_t(cy * epic::kHalfPitch + cx - 32 * half)
                           : transposed ? uint32_t(cx * pitch + cy)
                                        : uint32_t(cy * pitch + cx);
      const auto& lst = cell[c];
      for (size_t i = 0; i < lst.size(); ++i, ++s) {
        uint32_t code = uint32_t(lst[i].first) | (off << 12);
        if (i == 0) code |= 1u << 31;
        float wf = lst[i].second;
        uint32_t wb;
        std::memcpy(&wb, &wf, 4);
        table[2 * (s * L + l)] = code;
        table[2 * (s * L + l) + 1] = wb;
      }
    }
    for (; s < S; ++s) {
      table[2 * (s * L + l)] = pad | (1u << 31);
      table[2 * (s * L + l) + 1] = 0u;
    }
  }
  return int(S);
}

// Gridding schedule of the residue-class engine (N = 64 R): contributions are
// grouped by sub-cell q = j mod 64 and sub-cells are balanced over 64 lanes;
// each slot keeps the full cell j = 64 p + q so that the kernel can apply the
// class phase exp(+2 pi i j.c / N).
// half >= 0: the sub-cell columns 32 half <= qx < 32 half + 32 only (the
// codes keep the full qx).
int build_slots_cls(const HostArray& h, std::vector<uint32_t>& table, int half = -1) {
  std::vector<int32_t> ix, iy;
  std::vector<double> w;
  grid_cells(h, ix, iy, w);
  struct Contrib { int a, jx, jy; float w; };
  std::vector<std::vector<Contrib>> sub(64 * 64);
  for (int a = 0; a < h.na; ++a) {
    if (h.flag[a]) continue;
    for (int k = 0; k < h.k2; ++k) {
      const size_t q = size_t(a) * h.k2 + k;
      if (w[q] == 0.0) continue;
      if (half >= 0 && (ix[q] % 64) / 32 != half) continue;
      sub[size_t(iy[q] % 64) * 64 + ix[q] % 64].push_back({a, ix[q], iy[q], float(w[q])});
    }
  }
  std::vector<int> order;
  for (int c = 0; c < 64 * 64; ++c)
    if (!sub[c].empty()) order.push_back(c);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return sub[x].size() > sub[y].size(); });
  std::vector<std::vector<int>> lane_cells(64);
  std::vector<size_t> load(64, 0);
  for (int c : order) {
    int best = 0;
    for (int l = 1; l < 64; ++l)
      if (load[l] < load[best]) best = l;
    lane_cells[best].push_back(c);
    load[best] += sub[c].size();
  }
  size_t S = 0;
  for (int l = 0; l < 64; ++l) S = std::max(S, load[l]);
  table.assign(2 * S * 64, 0u);
  for (int l = 0; l < 64; ++l) {
    size_t s = 0;
    for (int c : lane_cells[l]) {
      const auto& lst = sub[c];
      for (size_t i = 0; i < lst.size(); ++i, ++s) {
        const Contrib& q = lst[i];
        uint32_t code = uint32_t(q.a) | uint32_t(q.jx % 64) << 12 | uint32_t(q.jy % 64) << 18 |
                        uint32_t(q.jx / 64) << 24 | uint32_t(q.jy / 64) << 26 | (1u << 30);
        if (i == 0) code |= 1u << 31;
        uint32_t wb;
        std::memcpy(&wb, &q.w, 4);
        table[2 * (s * 64 + l)] = code;
        table[2 * (s * 64 + l) + 1] = wb;
      }
    }
    for (; s < S; ++s) {
      table[2 * (s * 64 + l)] = 1u << 31;   // invalid: zero weight, stores into the pad column
      table[2 * (s * 64 + l) + 1] = 0u;
    }
  }
  return int(S);
}

// Multi-class schedule of the dense residue-class engine (N = 64 R): the
// sub-cells q = j mod 64 of sub-cell columns [32 half, 32 half + 32) (all
// columns for half < 0) are balanced over `owners` lanes (all waves of a frame); a lane's slots of one
// sub-cell are consecutive, the first marked first, the last marked last.
// Padding slots: weight 0, first, not last.
int build_slots_dense(const HostArray& h, int owners, int half, std::vector<uint32_t>& table) {
  std::vector<int32_t> ix, iy;
  std::vector<double> w;
  grid_cells(h, ix, iy, w);
  struct Contrib { int a, jx, jy; float w; };
  std::vector<std::vector<Contrib>> sub(64 * 64);
  for (int a = 0; a < h.na; ++a) {
    if (h.flag[a]) continue;
    for (int k = 0; k < h.k2; ++k) {
      const size_t q = size_t(a) * h.k2 + k;
      if (w[q] == 0.0 || (half >= 0 && (ix[q] % 64) / 32 != half)) continue;
      sub[size_t(iy[q] % 64) * 64 + ix[q] % 64].push_back({a, ix[q], iy[q], float(w[q])});
    }
  }
  std::vector<int> order;
  for (int c = 0; c < 64 * 64; ++c)
    if (!sub[c].empty()) order.push_back(c);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return sub[x].size() > sub[y].size(); });
  std::vector<std::vector<int>> lane_cells(owners);
  std::vector<size_t> load(owners, 0);
  for (int c : order) {
    int best = 0;
    for (int l = 1; l < owners; ++l)
      if (load[l] < load[best]) best = l;
    lane_cells[best].push_back(c);
    load[best] += sub[c].size();
  }
  size_t S = 0;
  for (int l = 0; l < owners; ++l) S = std::max(S, load[l]);
  table.assign(2 * S * owners, 0u);
  for (int l = 0; l < owners; ++l) {
    size_t s = 0;
    for (int c : lane_cells[l]) {
      const auto& lst = sub[c];
      for (size_t i = 0; i < lst.size(); ++i, ++s) {
        const Contrib& q = lst[i];
        uint32_t code = uint32_t(q.a) | uint32_t(q.jx % 64) << 12 | uint32_t(q.jy % 64) << 18 |
                        uint32_t(q.jx / 64) << 24 | uint32_t(q.jy / 64) << 26;
        if (i == 0) code |= 1u << 31;
        if (i + 1 == lst.size()) code |= 1u << 30;
        uint32_t wb;
        std::memcpy(&wb, &q.w, 4);
        table[2 * (s * owners + l)] = code;
        table[2 * (s * owners + l) + 1] = wb;
      }
    }
    for (; s < S; ++s) {
      table[2 * (s * owners + l)] = 1u << 31;
      table[2 * (s * owners + l) + 1] = 0u;
    }
  }
  return int(S);
}

}  // namespace

// ---------------------------------------------------------------------------
// Static device scratch of the allocation-free run (epic_run_noalloc): every
// GPU the library runs on holds one copy of this array, at its own address,
// until the process ends.  Host code never uses the array's name as an
// address: the address on each device comes from hipGetSymbolAddress, taken
// once per device (with that device current) when a plan is created there.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(EPIC_STATIC_SCRATCH_BYTES);
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
bool g_static_done[kMaxDevices];
hipError_t g_static_err[kMaxDevices];
void* g_static_ptr[kMaxDevices];

// The device address of `scratch` on device `dev` (the current device).
hipError_t static_scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_done[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_static_err[dev] = e;
    g_static_ptr[dev] = e == hipSuccess ? ptr : nullptr;
    g_static_done[dev] = true;
  }
  return g_static_err[dev];
}

// The address taken at set-up, or null with the set-up error.
void* static_scratch_ptr(int dev, hipError_t* err) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (dev < 0 || dev >= kMaxDevices || !g_static_done[dev]) {
    *err = hipErrorNotInitialized;
    return nullptr;
  }
  *err = g_static_err[dev];
  return g_static_ptr[dev];
}
}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct ArrayPlan {
  HostArray h;
  uint32_t* d_cell_ixy = nullptr;
  float* d_cell_w = nullptr;
  uint2* d_slots = nullptr;   // gridding schedule of the imaging engine
  int n_slots = 0;
  uint2* d_slots_dft = nullptr;   // schedule of the DFT-GEMM engine (64 lanes, G^T)
  int n_slots_dft = 0;
  uint2* d_slots_h = nullptr;     // 64 x 64: half-frame schedule (two halves of rows)
  int n_slots_h0 = 0, n_slots_h1 = 0;
  uint2* d_slots_m = nullptr;     // 128 / 256, integer formats: multi-class schedules (two halves)
  int n_slots_m0 = 0, n_slots_m1 = 0;
  uint2* d_slots_c = nullptr;     // 128 / 256: class schedule of the DFT-GEMM engine (128 owners)
  int n_slots_c = 0;
  uint8_t* d_flag = nullptr;
  // tuning (0 = plan default): transform 1 FFT / 2 DFT-GEMM, time splits
  int tune_transform = 0;
  int tune_splits = 0;
  int tune_batch = 0;          // dense class engine gridding batch (0 = default)
  double tune_us = 0;
  bool has_model = false;
  double gamma = 0;
  int t_cal = 1;
  int32_t* d_k0 = nullptr;     // [n_pix][F][2]
  double2* d_A = nullptr;      // [n_pix][F][Na]
  double2* d_D = nullptr;      // [n_pix][F][Na]
  uint8_t* d_hold = nullptr;
  int n_pix = 1;
  // gains shared over a band of channels (epical_set_band)
  int band_mode = 0, band_b0 = 0, band_b1 = 0, band_deg_amp = 0, band_deg_phase = 0;
  double* d_band_x = nullptr;  // [F] band coordinate
};

struct TimerRec {
  int kind;
  hipEvent_t a, b;
};

struct GraphKey {
  std::vector<const void*> ptrs;
  int64_t n_samples = -1;
  uint64_t generation = 0;
  bool operator==(const GraphKey& o) const {
    return ptrs == o.ptrs && n_samples == o.n_samples && generation == o.generation;
  }
};

struct epic_plan_s {
  int device = 0;
  int n_cu = 256;
  std::vector<ArrayPlan> arrays;
  // scratch
  void* d_scratch = nullptr;
  size_t scratch_bytes = 0;
  uint64_t generation = 1;   // bumped whenever device tables or scratch move
  // options
  int splits = 0;
  int transform = 0;
  int batch = 0;             // 0 auto (batched when >1 array), 1 on, 2 off
  bool graph = false;
  bool overlap = true;       // the fused solve + imaging launch where every array allows it
  int fused_polls = epic::kFusedWaitPolls;   // bound of one wait of the fused run
  bool timing = false;
  std::vector<TimerRec> timers;
  std::vector<hipEvent_t> event_pool;
  // batched work list
  int4* d_items = nullptr;
  size_t items_cap = 0;
  int n_items = 0;
  std::vector<int> items_key;
  bool items_built = false;
  int* d_counter = nullptr;
  int* d_fused = nullptr;    // fused run: role ticket, error word, per-channel progress
  int fused_cap = 0;
  // captured graph and the private stream it runs on
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph_g = nullptr;
  hipGraphExec_t graph_x = nullptr;
  GraphKey graph_key;
};

namespace {

void free_array(ArrayPlan& p) {
  hipFree(p.d_cell_ixy);
  hipFree(p.d_cell_w);
  hipFree(p.d_slots);
  hipFree(p.d_slots_dft);
  hipFree(p.d_slots_h);
  hipFree(p.d_slots_m);
  hipFree(p.d_slots_c);
  hipFree(p.d_flag);
  hipFree(p.d_k0);
  hipFree(p.d_A);
  hipFree(p.d_D);
  hipFree(p.d_hold);
  hipFree(p.d_band_x);
  p = ArrayPlan{};
}

template <typename T>
int upload(T** dst, const T* src, size_t n) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) return fail(EPIC_ERR_ALLOC, "hipMalloc(%zu bytes): %s", n * sizeof(T), hipGetErrorString(e));
  if (n) {
    e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  return EPIC_OK;
}

int plan_scratch(epic_plan_t p, size_t bytes, void** out) {
  if (bytes > p->scratch_bytes) {
    if (p->d_scratch) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      hipFree(p->d_scratch);
      p->d_scratch = nullptr;
      p->scratch_bytes = 0;
    }
    hipError_t e = hipMalloc(&p->d_scratch, bytes);
    if (e != hipSuccess) return fail(EPIC_ERR_ALLOC, "scratch hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    p->scratch_bytes = bytes;
    p->generation++;
  }
  *out = p->d_scratch;
  return EPIC_OK;
}

int check_plan(epic_plan_t p, int array) {
  if (!p) return fail(EPIC_ERR_ARG, "plan is NULL");
  if (array < 0 || array >= int(p->arrays.size()))
    return fail(EPIC_ERR_ARG, "array index %d out of range [0, %zu)", array, p->arrays.size());
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != p->device) return fail(EPIC_ERR_ARG, "current device %d is not the plan's device %d", dev, p->device);
  return EPIC_OK;
}

// Caller buffers on the device start on a 256-byte boundary (the boundary's
// contract; torch allocations do).  Null pointers pass (optional buffers are
// checked for presence separately).
int check_aligned(std::initializer_list<std::pair<const void*, const char*>> bufs) {
  for (const auto& b : bufs)
    if (b.first && (reinterpret_cast<uintptr_t>(b.first) & 255u) != 0)
      return fail(EPIC_ERR_ARG, "%s (%p) is not 256-byte aligned", b.second, b.first);
  return EPIC_OK;
}

// small = the call needs the N <= 64 engine (stage-wise calls, adjoint).
int check_grid_supported(const ArrayPlan& ap, bool small = false) {
  const HostArray& h = ap.h;
  if (h.nx != h.ny) return fail(EPIC_ERR_UNSUPPORTED, "only square grids are implemented (got %d x %d)", h.nx, h.ny);
  if (small && h.nx > 64)
    return fail(EPIC_ERR_UNSUPPORTED, "this call supports grids up to 64 x 64 (got %d); epic_run and epic_image "
                "support 128 and 256", h.nx);
  if (!epic::image_supported(h.nx, h.na, ap.n_slots))
    return fail(EPIC_ERR_UNSUPPORTED,
                "grid %d with %d antennas is not supported (N in {16,32,64}: Na <= 8N and a gridding schedule "
                "that fits the LDS slot table, here %d slots per lane; N in {128,256}: Na <= 2048)",
                h.nx, h.na, ap.n_slots);
  return EPIC_OK;
}

struct Timed {
  epic_plan_t p;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  bool on;
  Timed(epic_plan_t p_, int kind_, hipStream_t s_, bool enable = true)
      : p(p_), kind(kind_), s(s_), on(enable && p_->timing) {
    if (!on) return;
    a = take();
    b = take();
    if (a) hipEventRecord(a, s);
  }
  hipEvent_t take() {
    if (!p->event_pool.empty()) {
      hipEvent_t e = p->event_pool.back();
      p->event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~Timed() {
    if (!on || !a || !b) return;
    hipEventRecord(b, s);
    p->timers.push_back({kind, a, b});
  }
};

// The dense residue-class engine's schedules in an array's imaging arguments.
void with_dense_slots(ImageArgs& ia, const ArrayPlan& ap) {
  ia.slots_m = ap.d_slots_m;
  ia.n_slots_m0 = ap.n_slots_m0;
  ia.n_slots_m1 = ap.n_slots_m1;
  ia.grid_batch = ap.tune_batch;
}

// The fields of an array's imaging arguments that decide which engine runs it.
ImageArgs engine_probe(const ArrayPlan& ap) {
  ImageArgs ia{};
  ia.Na = ap.h.na;
  ia.fmt = ap.h.efmt;
  ia.slots_h = ap.d_slots_h;
  ia.n_slots_h0 = ap.n_slots_h0;
  ia.n_slots_h1 = ap.n_slots_h1;
  with_dense_slots(ia, ap);
  return ia;
}

// Workgroups of one time split per channel (class groups of the N = 256 engines).
int units_for(const ArrayPlan& ap) { return epic::cls_groups(engine_probe(ap), ap.h.nx); }
// Frames a workgroup images at once.
int slots_for(int N) { return N >= 128 ? 1 : 4 * (64 / N); }

// What a time-split count is for: the separate imaging launch of a run or of
// the stage-wise call, the fused solve + imaging launch, or another kernel
// (snapshots, the adjoint, the autotuner's reference point).
enum class SplitUse { image, fused, other };

// Time splits per channel for a target of `wg` workgroups, keeping >= 8 frames
// per slot; at 64 x 64 (the two-waves-per-SIMD engines: eight waves) >= 16
// frames per wave, which repays a workgroup's set-up and reduction (the
// 1000-sample differentiable workload: 31 splits 1.20 ms, 8 splits 1.08 ms),
// rounded up to whole rounds of workgroups over the CUs (one imaging
// workgroup per CU).
int64_t splits_for_target(epic_plan_t p, const ArrayPlan& ap, int64_t T, int64_t wg) {
  const int N = ap.h.nx;
  const int64_t units = int64_t(ap.h.F) * units_for(ap);
  int64_t s = (wg + units - 1) / units;
  const int64_t per_split = N == 64 ? 8 * 16 : 8 * int64_t(slots_for(N));
  s = std::min<int64_t>(s, std::max<int64_t>(1, T / per_split));
  if (units * s > p->n_cu) {
    const int64_t rounds = (units * s + p->n_cu - 1) / p->n_cu;
    s = std::min<int64_t>((rounds * p->n_cu + units - 1) / units, std::max<int64_t>(1, T));
  }
  return std::max<int64_t>(1, s);
}

int pick_splits(epic_plan_t p, const ArrayPlan& ap, int64_t T, int tuned = 0, SplitUse use = SplitUse::other) {
  const int N = ap.h.nx;
  if (tuned > 0) return int(std::max<int64_t>(1, std::min<int64_t>(tuned, std::max<int64_t>(1, T))));
  if (p->splits > 0) return int(std::max<int64_t>(1, std::min<int64_t>(p->splits, std::max<int64_t>(1, T))));
  if (use == SplitUse::fused) {
    // the fused run pulls items dynamically, solve workgroups joining late:
    // half again the items of 2048 workgroups keep the last ones short, in
    // whole rounds over the CUs (LWA shape, per fused launch: 16 splits
    // 5.16 ms, 20: 5.07, 24: 5.02-5.07, 28: 5.14, 32: 5.17, 48: 5.18)
    const int64_t per_split = N == 64 ? 8 * 16 : 8 * int64_t(slots_for(N));
    const int64_t units = int64_t(ap.h.F) * units_for(ap);
    int64_t sf = (3 * splits_for_target(p, ap, T, 2048) + 1) / 2;
    const int64_t rounds = (units * sf + p->n_cu - 1) / p->n_cu;
    sf = (rounds * p->n_cu + units - 1) / units;
    return int(std::max<int64_t>(1, std::min<int64_t>(sf, std::max<int64_t>(1, T / per_split))));
  }
  // the separate launch of the paired 64 x 64 engine: every workgroup images
  // the same number of frames, so two rounds over the CUs balance as well as
  // eight and set up and reduce a quarter as often (LWA shape, per launch:
  // 16 splits 4.38-4.44 ms, 8: 4.33, 4: 4.31-4.34, 2: 4.27-4.31; 3, one and a
  // half rounds: 5.78); the partial images written drop from 33.6 to 8.4 MB
  if (use == SplitUse::image && N == 64 && epic::pair_engine(engine_probe(ap), N))
    return int(splits_for_target(p, ap, T, 2 * int64_t(p->n_cu)));
  // aim for >= 2048 workgroups (8 per CU on 256 CUs)
  return int(splits_for_target(p, ap, T, 2048));
}

}  // namespace

extern "C" {

int32_t epic_abi_version(void) { return 2; }

const char* epic_last_error(void) { return g_err.c_str(); }

int epic_host_grid_cells(const epic_array_desc* desc, int32_t* ixy, double* w) {
  HostArray h;
  int rc = check_desc(desc, &h);
  if (rc) return rc;
  if (!ixy || !w) return fail(EPIC_ERR_ARG, "output pointers must not be NULL");
  std::vector<int32_t> ix, iy;
  std::vector<double> ww;
  grid_cells(h, ix, iy, ww);
  for (size_t q = 0; q < ix.size(); ++q) {
    ixy[2 * q] = ix[q];
    ixy[2 * q + 1] = iy[q];
    w[q] = ww[q];
  }
  return EPIC_OK;
}

int epic_host_calibrator_pixels(const epic_array_desc* desc, const epic_model_desc* model, const double* pix_lm,
                                int32_t n_pix, int32_t* k0, double* A, double* D) {
  HostArray h;
  int rc = check_desc(desc, &h);
  if (rc) return rc;
  rc = check_model(model);
  if (rc) return rc;
  rc = check_pixels(pix_lm, n_pix);
  if (rc) return rc;
  ModelTables t;
  model_tables(h, model, t, pix_lm, n_pix);
  if (k0) std::memcpy(k0, t.k0.data(), t.k0.size() * sizeof(int32_t));
  if (A) std::memcpy(A, t.A.data(), t.A.size() * sizeof(zc));
  if (D) std::memcpy(D, t.D.data(), t.D.size() * sizeof(zc));
  return EPIC_OK;
}

int epic_host_calibrator(const epic_array_desc* desc, const epic_model_desc* model, int32_t* k0, double* A,
                         double* D) {
  HostArray h;
  int rc = check_desc(desc, &h);
  if (rc) return rc;
  rc = check_model(model);
  if (rc) return rc;
  ModelTables t;
  model_tables(h, model, t);
  if (k0) std::memcpy(k0, t.k0.data(), t.k0.size() * sizeof(int32_t));
  if (A) std::memcpy(A, t.A.data(), t.A.size() * sizeof(zc));
  if (D) std::memcpy(D, t.D.data(), t.D.size() * sizeof(zc));
  return EPIC_OK;
}

// Band coordinate: the band's frequencies mapped linearly onto [-1, 1] in
// channel order (0 outside the band, and for a band of one channel).
static void band_coordinate(const HostArray& h, int b0, int b1, std::vector<double>& x) {
  x.assign(h.F, 0.0);
  const double lo = h.freq[b0], hi = h.freq[b1 - 1];
  const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
  if (half != 0)
    for (int f = b0; f < b1; ++f) x[f] = (h.freq[f] - mid) / half;
}

static int check_band(const HostArray& h, int b0, int b1, int mode, int deg_amp, int deg_phase) {
  if (mode == EPIC_BAND_NONE) return EPIC_OK;
  if (mode != EPIC_BAND_MEAN && mode != EPIC_BAND_POLY) return fail(EPIC_ERR_ARG, "unknown band mode %d", mode);
  if (b0 < 0 || b1 <= b0 || b1 > h.F)
    return fail(EPIC_ERR_ARG, "band [%d, %d) must be a non-empty range of the %d channels", b0, b1, h.F);
  if (mode == EPIC_BAND_POLY) {
    if (deg_amp < 0 || deg_amp > EPIC_BAND_MAX_DEG || deg_phase < 0 || deg_phase > EPIC_BAND_MAX_DEG)
      return fail(EPIC_ERR_ARG, "band polynomial degrees must be in [0, %d]", EPIC_BAND_MAX_DEG);
    const bool up = h.freq[b1 - 1] >= h.freq[b0];
    for (int f = b0 + 1; f < b1; ++f)
      if (up ? !(h.freq[f] > h.freq[f - 1]) : !(h.freq[f] < h.freq[f - 1]))
        return fail(EPIC_ERR_ARG, "the band's frequencies must be strictly monotonic for the polynomial model");
  }
  return EPIC_OK;
}

int epic_host_band_coordinate(const epic_array_desc* desc, int32_t b0, int32_t b1, double* x) {
  HostArray h;
  int rc = check_desc(desc, &h);
  if (rc) return rc;
  if (!x) return fail(EPIC_ERR_ARG, "x must not be NULL");
  if ((rc = check_band(h, b0, b1, EPIC_BAND_MEAN, 0, 0))) return rc;
  std::vector<double> v;
  band_coordinate(h, b0, b1, v);
  std::memcpy(x, v.data(), v.size() * sizeof(double));
  return EPIC_OK;
}

int epic_plan_create(const epic_array_desc* arrays, int32_t n_arrays, epic_plan_t* out) {
  if (!out) return fail(EPIC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!arrays || n_arrays < 1) return fail(EPIC_ERR_ARG, "need at least one array descriptor");
  std::vector<HostArray> hs(n_arrays);
  for (int i = 0; i < n_arrays; ++i) {
    int rc = check_desc(&arrays[i], &hs[i]);
    if (rc) return rc;
  }
  epic_plan_t p = new (std::nothrow) epic_plan_s;
  if (!p) return fail(EPIC_ERR_ALLOC, "host allocation failed");
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  // the allocation-free run's scratch address on this device (its error, if
  // any, is reported by epic_run_noalloc)
  static_scratch_setup(p->device);
  p->arrays.resize(n_arrays);
  for (int i = 0; i < n_arrays; ++i) {
    ArrayPlan& ap = p->arrays[i];
    ap.h = std::move(hs[i]);
    std::vector<int32_t> ix, iy;
    std::vector<double> w;
    grid_cells(ap.h, ix, iy, w);
    // device cell tables: four cells per antenna (the nearest-cell kernel is
    // padded with zero-weight copies of its cell)
    std::vector<uint32_t> packed(size_t(ap.h.na) * 4);
    std::vector<float> wf(size_t(ap.h.na) * 4, 0.f);
    for (int an = 0; an < ap.h.na; ++an)
      for (int k = 0; k < 4; ++k) {
        const size_t q = size_t(an) * ap.h.k2 + (ap.h.k2 == 4 ? k : 0);
        packed[size_t(an) * 4 + k] = (uint32_t(iy[q]) << 16) | uint32_t(ix[q]);
        wf[size_t(an) * 4 + k] = (ap.h.flag[an] || (ap.h.k2 == 1 && k > 0)) ? 0.f : float(w[q]);
      }
    int rc = upload(&ap.d_cell_ixy, packed.data(), packed.size());
    if (!rc) rc = upload(&ap.d_cell_w, wf.data(), wf.size());
    if (!rc) rc = upload(&ap.d_flag, ap.h.flag.data(), ap.h.flag.size());
    if (!rc && ap.h.nx == ap.h.ny && ap.h.nx <= 64 && ap.h.nx >= 16) {
      std::vector<uint32_t> tab;
      const int L = epic::grid_lanes(ap.h.nx);
      ap.n_slots = build_slots(ap.h, L, epic::grid_pitch(ap.h.nx), tab);
      rc = upload(&ap.d_slots, reinterpret_cast<const uint2*>(tab.data()), tab.size() / 2);
      if (!rc && (ap.h.nx == 32 || ap.h.nx == 64)) {
        ap.n_slots_dft = build_slots(ap.h, epic::dft_owners(ap.h.nx), ap.h.nx + 2, tab, true);
        rc = upload(&ap.d_slots_dft, reinterpret_cast<const uint2*>(tab.data()), tab.size() / 2);
      }
      if (!rc && ap.h.nx == 64) {
        std::vector<uint32_t> hi;
        ap.n_slots_h0 = build_slots(ap.h, 64, epic::kHalfPitch, tab, false, 0);
        ap.n_slots_h1 = build_slots(ap.h, 64, epic::kHalfPitch, hi, false, 1);
        tab.insert(tab.end(), hi.begin(), hi.end());
        rc = upload(&ap.d_slots_h, reinterpret_cast<const uint2*>(tab.data()), tab.size() / 2);
      }
    } else if (!rc && ap.h.nx == ap.h.ny && (ap.h.nx == 128 || ap.h.nx == 256)) {
      std::vector<uint32_t> tab;
      ap.n_slots = build_slots_cls(ap.h, tab);
      rc = upload(&ap.d_slots, reinterpret_cast<const uint2*>(tab.data()), tab.size() / 2);
      if (!rc) {
        std::vector<uint32_t> hi;
        ap.n_slots_h0 = build_slots_cls(ap.h, tab, 0);
        ap.n_slots_h1 = build_slots_cls(ap.h, hi, 1);
        tab.insert(tab.end(), hi.begin(), hi.end());
        rc = upload(&ap.d_slots_h, reinterpret_cast<const uint2*>(tab.data()), tab.size() / 2);
      }
      if (!rc) {
        ap.n_slots_c = build_slots_dense(ap.h, epic::dft_owners(ap.h.nx), -1, tab);
        rc = upload(&ap.d_slots_c, reinterpret_cast<const uint2*>(tab.data()), tab.size() / 2);
      }
      if (!rc && ap.h.efmt != EPIC_CF32) {
        std::vector<uint32_t> hi;
        const int owners = 64 * (ap.h.nx == 256 ? 8 : 4);   // the lanes of a frame's waves
        ap.n_slots_m0 = build_slots_dense(ap.h, owners, 0, tab);
        ap.n_slots_m1 = build_slots_dense(ap.h, owners, 1, hi);
        tab.insert(tab.end(), hi.begin(), hi.end());
        rc = upload(&ap.d_slots_m, reinterpret_cast<const uint2*>(tab.data()), tab.size() / 2);
      }
    }
    if (rc) {
      epic_plan_destroy(p);
      return rc;
    }
  }
  *out = p;
  return EPIC_OK;
}

int epic_plan_destroy(epic_plan_t plan) {
  if (!plan) return EPIC_OK;
  hipDeviceSynchronize();
  for (auto& ap : plan->arrays) free_array(ap);
  hipFree(plan->d_scratch);
  for (auto& t : plan->timers) {
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  for (auto e : plan->event_pool) hipEventDestroy(e);
  if (plan->graph_x) hipGraphExecDestroy(plan->graph_x);
  if (plan->graph_g) hipGraphDestroy(plan->graph_g);
  if (plan->ev_in) hipEventDestroy(plan->ev_in);
  if (plan->ev_out) hipEventDestroy(plan->ev_out);
  if (plan->gstream) hipStreamDestroy(plan->gstream);
  hipFree(plan->d_items);
  hipFree(plan->d_counter);
  hipFree(plan->d_fused);
  delete plan;
  return EPIC_OK;
}

static int set_model_tables(epic_plan_t plan, int32_t array, const epic_model_desc* model, const double* pix_lm,
                            int n_pix);

int epical_set_model(epic_plan_t plan, int32_t array, const epic_model_desc* model) {
  return set_model_tables(plan, array, model, nullptr, 1);
}

int epical_set_model_pixels(epic_plan_t plan, int32_t array, const epic_model_desc* model, const double* pix_lm,
                            int32_t n_pix) {
  int rc = check_pixels(pix_lm, n_pix);
  if (rc) return rc;
  return set_model_tables(plan, array, model, pix_lm, n_pix);
}

static int set_model_tables(epic_plan_t plan, int32_t array, const epic_model_desc* model, const double* pix_lm,
                            int n_pix) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  rc = check_model(model);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if (ap.h.na_eff < 2) return fail(EPIC_ERR_ARG, "calibration needs at least two unflagged antennas");
  if (n_pix > 1 && !epic::solve_supported(ap.h.na, ap.h.efmt, n_pix))
    return fail(EPIC_ERR_UNSUPPORTED, "several tapped pixels need Na <= 1024 (got %d)", ap.h.na);
  ModelTables t;
  model_tables(ap.h, model, t, pix_lm, n_pix);
  hipFree(ap.d_k0);
  hipFree(ap.d_A);
  hipFree(ap.d_D);
  hipFree(ap.d_hold);
  ap.d_k0 = nullptr;
  ap.d_A = ap.d_D = nullptr;
  ap.d_hold = nullptr;
  ap.has_model = false;
  rc = upload(&ap.d_k0, t.k0.data(), t.k0.size());
  if (!rc) rc = upload(&ap.d_A, reinterpret_cast<const double2*>(t.A.data()), t.A.size());
  if (!rc) rc = upload(&ap.d_D, reinterpret_cast<const double2*>(t.D.data()), t.D.size());
  if (!rc) rc = upload(&ap.d_hold, t.hold.data(), t.hold.size());
  if (rc) return rc;
  ap.gamma = model->gamma;
  ap.t_cal = model->t_cal;
  ap.n_pix = n_pix;
  ap.has_model = true;
  plan->generation++;
  return EPIC_OK;
}

int epical_set_band(epic_plan_t plan, int32_t array, int32_t b0, int32_t b1, int32_t mode, int32_t deg_amp,
                    int32_t deg_phase) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if ((rc = check_band(ap.h, b0, b1, mode, deg_amp, deg_phase))) return rc;
  if (mode != EPIC_BAND_NONE && !epic::band_supported(ap.h.na, ap.h.efmt))
    return fail(EPIC_ERR_UNSUPPORTED, "gains shared over a band need Na <= 1024 (got %d)", ap.h.na);
  hipFree(ap.d_band_x);
  ap.d_band_x = nullptr;
  ap.band_mode = EPIC_BAND_NONE;
  if (mode != EPIC_BAND_NONE) {
    std::vector<double> x;
    band_coordinate(ap.h, b0, b1, x);
    if ((rc = upload(&ap.d_band_x, x.data(), x.size()))) return rc;
    ap.band_mode = mode;
    ap.band_b0 = b0;
    ap.band_b1 = b1;
    ap.band_deg_amp = mode == EPIC_BAND_POLY ? deg_amp : 0;
    ap.band_deg_phase = mode == EPIC_BAND_POLY ? deg_phase : 0;
  }
  plan->generation++;
  return EPIC_OK;
}

int epical_set_denominator(epic_plan_t plan, int32_t array, const double* D) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if (!ap.has_model) return fail(EPIC_ERR_STATE, "epical_set_model has not been called for array %d", array);
  if (!D) return fail(EPIC_ERR_ARG, "D must not be NULL");
  const HostArray& h = ap.h;
  const size_t FN = size_t(h.F) * h.na, n = FN * ap.n_pix;
  for (size_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(D[i])) return fail(EPIC_ERR_ARG, "D must be finite");
  // hold bits as epical_set_model derives them: flagged, or sum_p |D_ap|^2 at
  // most 1e-24 of its largest value over the channel's antennas
  std::vector<uint8_t> hold(FN, 0);
  std::vector<double> den(h.na);
  for (int f = 0; f < h.F; ++f) {
    for (int a = 0; a < h.na; ++a) {
      double d = 0;
      for (int p = 0; p < ap.n_pix; ++p) {
        const double* z = D + 2 * (size_t(p) * FN + size_t(f) * h.na + a);
        d += z[0] * z[0] + z[1] * z[1];
      }
      den[a] = d;
    }
    const double dmax = *std::max_element(den.begin(), den.end());
    for (int a = 0; a < h.na; ++a) {
      uint8_t hb = h.flag[a] ? epic::kHoldFlagged : 0;
      if (!(den[a] > 1e-24 * dmax)) hb |= epic::kHoldDZero;
      hold[size_t(f) * h.na + a] = hb;
    }
  }
  // runs still in flight read the old tables
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(ap.d_D, D, n * sizeof(double2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ap.d_hold, hold.data(), FN, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "denominator upload");
  plan->generation++;
  return EPIC_OK;
}

int epic_plan_get_cells(epic_plan_t plan, int32_t array, int32_t* ixy, float* w) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  if (!ixy || !w) return fail(EPIC_ERR_ARG, "ixy and w must not be NULL");
  const ArrayPlan& ap = plan->arrays[array];
  const size_t na = size_t(ap.h.na);
  std::vector<uint32_t> cells(na * 4);
  std::vector<float> wt(na * 4);
  hipError_t e = hipMemcpy(cells.data(), ap.d_cell_ixy, cells.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(wt.data(), ap.d_cell_w, wt.size() * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "cell table read-back");
  const int k2 = ap.h.k2;
  for (size_t a = 0; a < na; ++a)
    for (int k = 0; k < k2; ++k) {
      const uint32_t c = cells[4 * a + k];
      ixy[2 * (a * k2 + k)] = int32_t(c & 0xffffu);
      ixy[2 * (a * k2 + k) + 1] = int32_t(c >> 16);
      w[a * k2 + k] = wt[4 * a + k];
    }
  return EPIC_OK;
}

int epic_debug_unpack(epic_plan_t plan, int32_t array, const void* efield, int64_t n, int16_t* out,
                      epic_stream_t stream) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  const ArrayPlan& ap = plan->arrays[array];
  if (ap.h.efmt != EPIC_CI4 && ap.h.efmt != EPIC_CI8)
    return fail(EPIC_ERR_UNSUPPORTED, "epic_debug_unpack decodes the integer formats (ci4, ci8) only");
  if (n < 0) return fail(EPIC_ERR_ARG, "n must be >= 0");
  if (n > 0 && (!efield || !out)) return fail(EPIC_ERR_ARG, "efield and out must not be NULL");
  if ((rc = check_aligned({{efield, "efield"}, {out, "out"}}))) return rc;
  hipError_t e = epic::launch_unpack(static_cast<const uint8_t*>(efield), n, ap.h.efmt, out,
                                     static_cast<hipStream_t>(stream));
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "epic_debug_unpack launch");
}

int epic_plan_set_option(epic_plan_t plan, int32_t key, int64_t value) {
  if (!plan) return fail(EPIC_ERR_ARG, "plan is NULL");
  switch (key) {
    // options that change the launches a run records retire its captured graph
    case EPIC_OPT_SPLITS:
      if (value < 0 || value > (1 << 20)) return fail(EPIC_ERR_ARG, "splits out of range");
      plan->splits = int(value);
      plan->generation++;
      return EPIC_OK;
    case EPIC_OPT_TRANSFORM:
      if (value < 0 || value > 4) return fail(EPIC_ERR_ARG, "transform must be in 0..4");
      plan->transform = int(value);
      plan->generation++;
      return EPIC_OK;
    case EPIC_OPT_TIMING:
      plan->timing = value != 0;
      return EPIC_OK;
    case EPIC_OPT_BATCH:
      if (value < 0 || value > 2) return fail(EPIC_ERR_ARG, "batch must be 0 (auto), 1 (on) or 2 (off)");
      plan->batch = int(value);
      plan->generation++;
      return EPIC_OK;
    case EPIC_OPT_GRAPH:
      plan->graph = value != 0;
      return EPIC_OK;
    case EPIC_OPT_OVERLAP:
      if (value != 0 && value != 1) return fail(EPIC_ERR_ARG, "EPIC_OPT_OVERLAP is 0 or 1");
      if (plan->overlap != (value != 0)) plan->generation++;
      plan->overlap = value != 0;
      return EPIC_OK;
    case EPIC_OPT_WAIT_POLLS:
      if (value < 0 || value > epic::kFusedWaitPolls)
        return fail(EPIC_ERR_ARG, "EPIC_OPT_WAIT_POLLS must be in [0, %d]", epic::kFusedWaitPolls);
      if (value == 0) value = epic::kFusedWaitPolls;
      if (plan->fused_polls != int(value)) plan->generation++;
      plan->fused_polls = int(value);
      return EPIC_OK;
    default:
      return fail(EPIC_ERR_ARG, "unknown option key %d", key);
  }
}

int epic_plan_get_timing(epic_plan_t plan, double* ms, int64_t* launches, int32_t n) {
  if (!plan) return fail(EPIC_ERR_ARG, "plan is NULL");
  if (n < 0 || (n > 0 && (!ms || !launches))) return fail(EPIC_ERR_ARG, "bad output arrays");
  for (int k = 0; k < n; ++k) {
    ms[k] = 0;
    launches[k] = 0;
  }
  int rc = EPIC_OK;
  for (auto& t : plan->timers) {
    hipError_t e = hipEventSynchronize(t.b);
    float el = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&el, t.a, t.b);
    if (e != hipSuccess && rc == EPIC_OK) rc = hip_fail(e, "hipEventElapsedTime");
    if (t.kind < n) {
      ms[t.kind] += el;
      launches[t.kind] += 1;
    }
    plan->event_pool.push_back(t.a);
    plan->event_pool.push_back(t.b);
  }
  plan->timers.clear();
  return rc;
}

int epic_grid(epic_plan_t plan, int32_t array, const void* efield, int64_t t0, int32_t nt, const float* u,
              float* grid, epic_stream_t stream) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if ((rc = check_grid_supported(ap, true))) return rc;
  if (nt < 0 || t0 < 0) return fail(EPIC_ERR_ARG, "t0 and nt must be >= 0");
  if (nt > 0 && (!efield || !u || !grid)) return fail(EPIC_ERR_ARG, "efield, u and grid must not be NULL");
  if ((rc = check_aligned({{efield, "efield"}, {u, "u"}, {grid, "grid"}}))) return rc;
  epic::GridArgs a{static_cast<const uint8_t*>(efield), t0, nt, ap.h.F, ap.h.na, ap.h.efmt,
                   reinterpret_cast<const float2*>(u), ap.d_slots, ap.n_slots, reinterpret_cast<float2*>(grid)};
  hipError_t e = epic::launch_grid(ap.h.nx, a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "epic_grid launch");
}

int epic_image_accumulate(epic_plan_t plan, int32_t array, const float* grid, int32_t nt, float* image, float* tap,
                          epic_stream_t stream) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if ((rc = check_grid_supported(ap, true))) return rc;
  if (nt < 0) return fail(EPIC_ERR_ARG, "nt must be >= 0");
  if (nt > 0 && (!grid || !image)) return fail(EPIC_ERR_ARG, "grid and image must not be NULL");
  if (tap && !ap.has_model) return fail(EPIC_ERR_STATE, "tap requested but no model (calibrator pixel) set");
  if ((rc = check_aligned({{grid, "grid"}, {image, "image"}, {tap, "tap"}}))) return rc;
  if (ap.h.na_eff < 1) return fail(EPIC_ERR_ARG, "all antennas are flagged");
  epic::ImageAccArgs a{reinterpret_cast<const float2*>(grid), nt, ap.h.F, float(1.0 / ap.h.na_eff), image,
                       reinterpret_cast<float2*>(tap), tap ? ap.d_k0 : nullptr};
  hipError_t e = epic::launch_image_acc(ap.h.nx, a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "epic_image_accumulate launch");
}

int epical_update(epic_plan_t plan, int32_t array, const void* efield, int64_t t0, int32_t nt, const float* tap,
                  double* kq, double* gains, int32_t finalize, uint32_t* status, epic_stream_t stream) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if (!ap.has_model) return fail(EPIC_ERR_STATE, "epical_set_model has not been called for array %d", array);
  if (ap.n_pix != 1)
    return fail(EPIC_ERR_UNSUPPORTED, "the stage-wise update takes one tap per sample; this array has %d pixels "
                "(use epic_run)", ap.n_pix);
  if (ap.band_mode != EPIC_BAND_NONE)
    return fail(EPIC_ERR_UNSUPPORTED, "the stage-wise update is per channel; this array shares gains over a band "
                "(use epic_run)");
  if (nt < 0 || t0 < 0) return fail(EPIC_ERR_ARG, "t0 and nt must be >= 0");
  if (!kq || !gains) return fail(EPIC_ERR_ARG, "kq and gains must not be NULL");
  if (nt > 0 && (!efield || !tap)) return fail(EPIC_ERR_ARG, "efield and tap must not be NULL");
  if ((rc = check_aligned({{efield, "efield"}, {tap, "tap"}, {kq, "kq"}, {gains, "gains"}, {status, "status"}})))
    return rc;
  epic::UpdateArgs a{static_cast<const uint8_t*>(efield), t0, nt, ap.h.F, ap.h.na, ap.h.efmt,
                     reinterpret_cast<const float2*>(tap), kq, reinterpret_cast<double2*>(gains), ap.d_A, ap.d_D,
                     ap.d_hold, double(ap.h.na_eff), ap.gamma, finalize ? 1 : 0, status};
  hipError_t e = epic::launch_update(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "epical_update launch");
}

// Slot schedule of the DFT-GEMM engine: its own transposed table for N <= 64,
// the residue-class table for N = 128, 256.
static const uint2* dft_slots(const ArrayPlan& ap) { return ap.h.nx >= 128 ? ap.d_slots_c : ap.d_slots_dft; }
static int dft_nslots(const ArrayPlan& ap) { return ap.h.nx >= 128 ? ap.n_slots_c : ap.n_slots_dft; }

// Whether the array is imaged by the DFT-GEMM form (tuned or plan transform).
static int transform_of(epic_plan_t plan, const ArrayPlan& ap) {
  return ap.tune_transform ? ap.tune_transform : plan->transform;
}
static bool uses_dft(epic_plan_t plan, const ArrayPlan& ap) {
  return transform_of(plan, ap) >= 2 && epic::dft_supported(ap.h.nx, ap.h.na, dft_nslots(ap));
}

// The imaging arguments of one array: the FFT engines' schedules, or the
// DFT-GEMM engine's.
static ImageArgs image_args(epic_plan_t plan, const ArrayPlan& ap, const void* efield, int64_t n_samples,
                            const float2* u, int64_t t_cal, float* partial, int splits) {
  const HostArray& h = ap.h;
  const bool dft = uses_dft(plan, ap);
  ImageArgs ia{static_cast<const uint8_t*>(efield), n_samples, h.F, h.na, h.efmt, u, t_cal,
               dft && h.nx <= 64 ? dft_slots(ap) : ap.d_slots, dft && h.nx <= 64 ? dft_nslots(ap) : ap.n_slots,
               splits, partial, ap.d_slots_h, ap.n_slots_h0, ap.n_slots_h1};
  with_dense_slots(ia, ap);
  if (dft) {
    ia.dft_prec = transform_of(plan, ap) - 2;
    ia.slots_c = ap.d_slots_c;
    ia.n_slots_c = ap.n_slots_c;
  }
  return ia;
}

static int image_pass(epic_plan_t plan, ArrayPlan& ap, const void* efield, int64_t n_samples, const float2* u,
                      int64_t t_cal, float* image, hipStream_t s, float* partial, int splits, bool timed = true) {
  const HostArray& h = ap.h;
  const int N = h.nx;
  const bool dft = uses_dft(plan, ap);
  const ImageArgs ia = image_args(plan, ap, efield, n_samples, u, t_cal, partial, splits);
  {
    Timed tm(plan, EPIC_TIMER_IMAGE, s, timed);
    hipError_t e = dft ? epic::launch_image_dft(N, ia, s) : epic::launch_image(N, ia, s);
    if (e != hipSuccess) return hip_fail(e, "imaging launch");
  }
  {
    Timed tm(plan, EPIC_TIMER_REDUCE, s, timed);
    const double scale = 1.0 / (double(n_samples) * double(h.na_eff) * double(h.na_eff));
    hipError_t e = epic::launch_reduce(partial, splits, int64_t(h.F) * N * N, scale, image, s);
    if (e != hipSuccess) return hip_fail(e, "image reduction launch");
  }
  return EPIC_OK;
}

// Per-array layout of one epic_run in the plan scratch.
struct RunLayout {
  int64_t n_int;
  int splits;
  size_t u_off, p_off, gh_off;   // gh_off: gain history when the caller passes none
  size_t band_off;               // band solve: raw solutions [F][Na], model [Na][8], barrier counter
};

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

static int solve_ps(const HostArray& h) {
  const int RB = h.na * epic::efmt_bytes(h.efmt);
  return RB % 16 == 0 ? 16 : RB % 4 == 0 ? 4 : 1;
}

// The persistent batched kernel's body for an array (0: the array is imaged
// by its own launch in the batched sequence: complex float E-fields at 64 x 64
// and above, the one-wave class engines, the DFT-GEMM form).
static int body_of(epic_plan_t plan, const ArrayPlan& ap) {
  ImageArgs ia = engine_probe(ap);
  ia.n_slots = ap.n_slots;
  return epic::batch_body(ia, ap.h.nx, uses_dft(plan, ap));
}

static bool own_launch(epic_plan_t plan, const ArrayPlan& ap) { return body_of(plan, ap) == 0; }

// The fused run (one launch for the solve and the imaging) applies when every
// array's solve runs at kSolveMainThreads threads (no band; one tapped pixel,
// not the one-wave solve of tiny arrays, or several pixels with at most
// kSolveMainThreads antennas) and is imaged by a body of the persistent kernel, and pays when the separate solve launch
// would leave CUs idle: fewer solve tasks (channels of all arrays) than CUs.
// With more, the solve fills the chip by itself and the fused run only adds
// the cost of finer imaging items (HERA shape, 512 channels: 23.0 against
// 22.8 ms; eight uneven arrays of 256 channels: 61.3 against 61.1 ms).
static bool fused_eligible(epic_plan_t plan) {
  if (!plan->overlap || plan->arrays.size() > size_t(epic::kMaxBatch)) return false;
  int n_chan = 0;
  for (const ArrayPlan& ap : plan->arrays) n_chan += ap.h.F;
  if (n_chan >= plan->n_cu) return false;
  for (const ArrayPlan& ap : plan->arrays) {
    if (ap.band_mode != EPIC_BAND_NONE || own_launch(plan, ap)) return false;
    if (ap.n_pix > 1) {
      if (!epic::solve_multi_fusable(ap.h.na, ap.h.efmt)) return false;
      continue;
    }
    epic::SolveArgs probe{};
    probe.Na = ap.h.na;
    probe.n_pix = 1;
    probe.t_cal = ap.t_cal;
    if (epic::solve_by_wave(probe)) return false;
  }
  return true;
}

// Work items {array, channel, class group, split}, most expensive first;
// none for the arrays with their own launch.
static int build_items(epic_plan_t plan, const std::vector<RunLayout>& lay, int64_t n_samples) {
  std::vector<int> key{int(n_samples & 0x7fffffff), int(n_samples >> 31)};
  for (size_t i = 0; i < lay.size(); ++i) key.push_back(lay[i].splits);
  for (size_t i = 0; i < lay.size(); ++i) key.push_back(own_launch(plan, plan->arrays[i]) ? 1 : 0);
  if (plan->items_built && key == plan->items_key) return EPIC_OK;
  struct It {
    int4 w;
    double cost;
  };
  std::vector<It> items;
  for (size_t i = 0; i < lay.size(); ++i) {
    if (own_launch(plan, plan->arrays[i])) continue;
    const HostArray& h = plan->arrays[i].h;
    const int N = h.nx, cg = units_for(plan->arrays[i]);
    const double per_frame = double(N) * N * std::log2(double(N) * N) / cg + 32.0 * h.na;
    for (int s = 0; s < lay[i].splits; ++s) {
      const int64_t tb = n_samples * s / lay[i].splits, te = n_samples * (s + 1) / lay[i].splits;
      for (int f = 0; f < h.F; ++f)
        for (int c = 0; c < cg; ++c) items.push_back({make_int4(int(i), f, c, s), per_frame * double(te - tb)});
    }
  }
  std::stable_sort(items.begin(), items.end(), [](const It& a, const It& b) { return a.cost > b.cost; });
  std::vector<int4> w(items.size());
  for (size_t k = 0; k < items.size(); ++k) w[k] = items[k].w;
  // A launch of an earlier call may still be reading the list, on any stream
  // (the caller's, or the plan's graph stream): drain the device before the
  // list is rewritten, and retire every graph that captured the old one.
  if (plan->d_items) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before the work list upload");
  }
  plan->generation++;
  if (w.size() > plan->items_cap) {
    hipFree(plan->d_items);
    plan->d_items = nullptr;
    plan->items_cap = 0;
    if (hipMalloc(&plan->d_items, w.size() * sizeof(int4)) != hipSuccess)
      return fail(EPIC_ERR_ALLOC, "work list allocation failed");
    plan->items_cap = w.size();
  }
  if (!w.empty()) {
    hipError_t e = hipMemcpy(plan->d_items, w.data(), w.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "work list upload");
  }
  plan->n_items = int(w.size());
  plan->items_key = key;
  plan->items_built = true;
  return EPIC_OK;
}

// The calibration solve of one array in the per-array form: the cooperative
// band solve when its channels share gains, else one workgroup per channel.
static hipError_t solve_array(epic_plan_t plan, const ArrayPlan& ap, const epic::SolveArgs& sa, char* band_scr,
                              hipStream_t s) {
  if (ap.band_mode == EPIC_BAND_NONE) return epic::launch_solve(sa, s);
  const HostArray& h = ap.h;
  epic::BandArgs b{};
  b.s = sa;
  b.b0 = ap.band_b0;
  b.b1 = ap.band_b1;
  b.mode = ap.band_mode;
  b.deg_amp = ap.band_deg_amp;
  b.deg_phase = ap.band_deg_phase;
  b.x = ap.d_band_x;
  b.raw = reinterpret_cast<double2*>(band_scr);
  b.coef = reinterpret_cast<double*>(band_scr + align256(size_t(h.F) * h.na * sizeof(double2)));
  b.bar = reinterpret_cast<uint32_t*>(band_scr + align256(size_t(h.F) * h.na * sizeof(double2)) +
                                      align256(size_t(h.na) * epic::kBandCoef * sizeof(double)));
  return epic::launch_solve_band(b, plan->n_cu, s);
}

static epic::SolveArgs solve_args(const ArrayPlan& ap, const RunLayout& lay, char* scr, const void* efield,
                                  int64_t n_samples, double* gains, double* gain_hist, uint32_t* status) {
  const HostArray& h = ap.h;
  epic::SolveArgs sa{static_cast<const uint8_t*>(efield), n_samples, h.F, h.na, h.efmt, ap.t_cal, int(lay.n_int),
                     ap.d_A, ap.d_D, ap.d_hold, double(h.na_eff), ap.gamma, reinterpret_cast<double2*>(gains),
                     reinterpret_cast<float2*>(scr + lay.u_off),
                     gain_hist ? reinterpret_cast<double2*>(gain_hist)
                               : reinterpret_cast<double2*>(scr + lay.gh_off),
                     status};
  sa.n_pix = ap.n_pix;
  return sa;
}

// Scratch of one array's run, appended at `need`: u history, partial images
// (`partials` floats per split), gain history, band scratch.
static int layout_array(const ArrayPlan& ap, int64_t n_samples, int splits, size_t partials, RunLayout& lay,
                        size_t& need, bool& any_band) {
  lay.n_int = (n_samples + ap.t_cal - 1) / ap.t_cal;
  if (lay.n_int > std::numeric_limits<int>::max()) return fail(EPIC_ERR_ARG, "too many calibration intervals");
  lay.splits = splits;
  lay.u_off = need;
  need += align256(size_t(lay.n_int) * ap.h.F * ap.h.na * sizeof(float2));
  lay.p_off = need;
  need += align256(size_t(splits) * partials * sizeof(float));
  lay.gh_off = need;
  need += align256(size_t(lay.n_int + 1) * ap.h.F * ap.h.na * sizeof(double2));
  lay.band_off = need;
  if (ap.band_mode != EPIC_BAND_NONE) {
    if (ap.n_pix != 1) return fail(EPIC_ERR_UNSUPPORTED, "gains shared over a band take one tapped pixel");
    any_band = true;
    need += align256(size_t(ap.h.F) * ap.h.na * sizeof(double2)) +
            align256(size_t(ap.h.na) * epic::kBandCoef * sizeof(double)) + align256(256 * sizeof(uint32_t));
  }
  return EPIC_OK;
}

// The reduction of every array's partial images (batched and fused runs).
static int enqueue_reduce_batch(epic_plan_t plan, const std::vector<RunLayout>& lay, char* scr, int64_t n_samples,
                                float* const* image, hipStream_t s, bool timed, const int* error) {
  const int na_arr = int(plan->arrays.size());
  epic::BatchReduceArgs b{};
  b.n_arrays = na_arr;
  b.off[0] = 0;
  for (int i = 0; i < na_arr; ++i) {
    const HostArray& h = plan->arrays[i].h;
    b.partial[i] = reinterpret_cast<const float*>(scr + lay[i].p_off);
    b.image[i] = image[i];
    b.splits[i] = lay[i].splits;
    b.per_split[i] = int64_t(h.F) * h.nx * h.ny;
    b.scale[i] = 1.0 / (double(n_samples) * double(h.na_eff) * double(h.na_eff));
    b.off[i + 1] = b.off[i] + b.per_split[i];
  }
  b.error = error;
  Timed tm(plan, EPIC_TIMER_REDUCE, s, timed);
  hipError_t e = epic::launch_reduce_batch(b, s);
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "batched reduction launch");
}

// The fused run: one launch for the calibration solve and the imaging of
// every array (the solve publishes u interval by interval, the imaging items
// wait for the intervals they need), then the reduction.  Timed as imaging.
static int enqueue_fused(epic_plan_t plan, const std::vector<RunLayout>& lay, char* scr,
                         const std::vector<epic::SolveArgs>& sa, const void* const* efield, int64_t n_samples,
                         float* const* image, hipStream_t s, bool timed) {
  const int na_arr = int(plan->arrays.size());
  epic::BatchImageArgs b{};
  epic::FusedArgs fa{};
  b.n_arrays = na_arr;
  fa.chan_off[0] = 0;
  for (int i = 0; i < na_arr; ++i) {
    ArrayPlan& ap = plan->arrays[i];
    b.arr[i] = image_args(plan, ap, efield[i], n_samples, reinterpret_cast<const float2*>(scr + lay[i].u_off),
                          ap.t_cal, reinterpret_cast<float*>(scr + lay[i].p_off), lay[i].splits);
    b.code[i] = body_of(plan, ap);
    const epic::SolveArgs& a = sa[i];
    const int code = ap.n_pix > 1 ? epic::kFusedMultiCode + solve_ps(ap.h)
                                  : 100 * epic::solve_main_j(ap.h.na) + solve_ps(ap.h);
    fa.sx[i] = epic::FusedSolveExtra{a.A, a.D, a.hold, a.gains, a.g_hist, a.status, a.na_eff, a.gamma, a.n_int,
                                     code, ap.n_pix};
    fa.chan_off[i + 1] = fa.chan_off[i] + ap.h.F;
  }
  fa.n_solve = fa.chan_off[na_arr];
  fa.ticket = plan->d_fused;
  fa.error = plan->d_fused + 1;
  fa.progress = plan->d_fused + 64;
  fa.max_polls = plan->fused_polls;
  b.items = plan->d_items;
  b.n_items = plan->n_items;
  b.counter = plan->d_counter;
  {
    Timed tm(plan, EPIC_TIMER_IMAGE, s, timed);
    hipError_t e = epic::launch_run_fused(b, fa, plan->n_cu, s);
    if (e != hipSuccess) return hip_fail(e, "fused solve and imaging launch");
  }
  return enqueue_reduce_batch(plan, lay, scr, n_samples, image, s, timed, fa.error);
}

// Enqueue the whole run on `s`; batched selects the one-launch-per-stage form,
// fused the one launch for the solve and the imaging.
static int enqueue_run(epic_plan_t plan, const std::vector<RunLayout>& lay, char* scr, const void* const* efield,
                       int64_t n_samples, double* const* gains, float* const* image, double* const* gain_hist,
                       uint32_t* const* ant_status, hipStream_t s, bool batched, bool timed, bool fused = false) {
  const int na_arr = int(plan->arrays.size());
  std::vector<epic::SolveArgs> sa(na_arr);
  for (int i = 0; i < na_arr; ++i)
    sa[i] = solve_args(plan->arrays[i], lay[i], scr, efield[i], n_samples, gains[i],
                       gain_hist ? gain_hist[i] : nullptr, ant_status ? ant_status[i] : nullptr);
  // FP32 u of every interval from the gain history the solve wrote
  auto hist_to_u = [&](int i) -> hipError_t {
    const HostArray& h = plan->arrays[i].h;
    return epic::launch_hist_to_u(sa[i].g_hist, plan->arrays[i].d_hold, lay[i].n_int, h.F, h.na, sa[i].u_hist, s);
  };
  if (fused) return enqueue_fused(plan, lay, scr, sa, efield, n_samples, image, s, timed);
  if (!batched) {
    for (int i = 0; i < na_arr; ++i) {
      ArrayPlan& ap = plan->arrays[i];
      {
        Timed tm(plan, EPIC_TIMER_SOLVE, s, timed);
        hipError_t e = solve_array(plan, ap, sa[i], scr + lay[i].band_off, s);
        if (e == hipSuccess) e = hist_to_u(i);
        if (e != hipSuccess) return hip_fail(e, "calibration solve launch");
      }
      int rc = image_pass(plan, ap, efield[i], n_samples, reinterpret_cast<float2*>(scr + lay[i].u_off), ap.t_cal,
                          image[i], s, reinterpret_cast<float*>(scr + lay[i].p_off), lay[i].splits, timed);
      if (rc) return rc;
    }
    return EPIC_OK;
  }
  // calibration: one launch when every array shares the solve variant
  {
    Timed tm(plan, EPIC_TIMER_SOLVE, s, timed);
    bool same = true;
    const int j0 = epic::solve_main_j(plan->arrays[0].h.na), ps0 = solve_ps(plan->arrays[0].h);
    for (int i = 1; i < na_arr; ++i)
      same = same && epic::solve_main_j(plan->arrays[i].h.na) == j0 && solve_ps(plan->arrays[i].h) == ps0;
    for (int i = 0; i < na_arr; ++i) same = same && !epic::solve_by_wave(sa[i]) && sa[i].n_pix == 1;
    if (same) {
      epic::BatchSolveArgs b{};
      b.n_arrays = na_arr;
      b.chan_off[0] = 0;
      for (int i = 0; i < na_arr; ++i) {
        b.arr[i] = sa[i];
        b.chan_off[i + 1] = b.chan_off[i] + plan->arrays[i].h.F;
      }
      hipError_t e = epic::launch_solve_batch(b, j0, ps0, s);
      if (e != hipSuccess) return hip_fail(e, "batched calibration solve launch");
    } else {
      for (int i = 0; i < na_arr; ++i) {
        hipError_t e = epic::launch_solve(sa[i], s);
        if (e != hipSuccess) return hip_fail(e, "calibration solve launch");
      }
    }
    for (int i = 0; i < na_arr; ++i) {
      hipError_t e = hist_to_u(i);
      if (e != hipSuccess) return hip_fail(e, "gain history conversion launch");
    }
  }
  // imaging: one persistent launch over the work items of every array a body
  // of the batched kernel covers; the others by their own launches
  {
    Timed tm(plan, EPIC_TIMER_IMAGE, s, timed);
    for (int i = 0; i < na_arr; ++i) {
      ArrayPlan& ap = plan->arrays[i];
      if (!own_launch(plan, ap)) continue;
      const ImageArgs ia = image_args(plan, ap, efield[i], n_samples,
                                      reinterpret_cast<const float2*>(scr + lay[i].u_off), ap.t_cal,
                                      reinterpret_cast<float*>(scr + lay[i].p_off), lay[i].splits);
      hipError_t e = uses_dft(plan, ap) ? epic::launch_image_dft(ap.h.nx, ia, s) : epic::launch_image(ap.h.nx, ia, s);
      if (e != hipSuccess) return hip_fail(e, "imaging launch");
    }
  }
  if (plan->n_items > 0) {
    epic::BatchImageArgs b{};
    b.n_arrays = na_arr;
    for (int i = 0; i < na_arr; ++i) {
      ArrayPlan& ap = plan->arrays[i];
      b.arr[i] = image_args(plan, ap, efield[i], n_samples, reinterpret_cast<const float2*>(scr + lay[i].u_off),
                            ap.t_cal, reinterpret_cast<float*>(scr + lay[i].p_off), lay[i].splits);
      b.code[i] = body_of(plan, ap);
    }
    b.items = plan->d_items;
    b.n_items = plan->n_items;
    b.counter = plan->d_counter;
    Timed tm(plan, EPIC_TIMER_IMAGE, s, timed);
    hipError_t e = epic::launch_image_batch(b, plan->n_cu, s);
    if (e != hipSuccess) return hip_fail(e, "batched imaging launch");
  }
  return enqueue_reduce_batch(plan, lay, scr, n_samples, image, s, timed, nullptr);
}

// Argument checks of a run over every array of the plan and its scratch
// layout (splits[i] > 0 overrides the time splits of array i).
static int prepare_run(epic_plan_t plan, const void* const* efield, int64_t n_samples, double* const* gains,
                       float* const* image, double* const* gain_hist, uint32_t* const* ant_status,
                       std::vector<RunLayout>& lay, size_t& need, bool& all_batchable, bool& any_band,
                       const std::vector<int>* splits = nullptr, bool fused = false) {
  if (!plan) return fail(EPIC_ERR_ARG, "plan is NULL");
  if (!efield || !gains || !image) return fail(EPIC_ERR_ARG, "efield, gains and image arrays must not be NULL");
  if (n_samples < 1) return fail(EPIC_ERR_ARG, "n_samples must be >= 1");
  const int na_arr = int(plan->arrays.size());
  lay.assign(na_arr, RunLayout{});
  need = 0;
  all_batchable = na_arr <= epic::kMaxBatch;
  any_band = false;
  for (int i = 0; i < na_arr; ++i) {
    int rc = check_plan(plan, i);
    if (rc) return rc;
    ArrayPlan& ap = plan->arrays[i];
    if (!ap.has_model) return fail(EPIC_ERR_STATE, "epical_set_model has not been called for array %d", i);
    if ((rc = check_grid_supported(ap))) return rc;
    if (!epic::solve_supported(ap.h.na, ap.h.efmt, ap.n_pix))
      return fail(EPIC_ERR_UNSUPPORTED, "calibration solve supports Na <= 2048 and Na * bytes per sample <= 16 KiB");
    if (!efield[i] || !gains[i] || !image[i]) return fail(EPIC_ERR_ARG, "NULL buffer for array %d", i);
    if ((rc = check_aligned({{efield[i], "efield"}, {gains[i], "gains"}, {image[i], "image"},
                             {gain_hist ? gain_hist[i] : nullptr, "gain_hist"},
                             {ant_status ? ant_status[i] : nullptr, "ant_status"}})))
      return rc;
    const SplitUse use = fused ? SplitUse::fused : SplitUse::image;
    const int sp = splits && (*splits)[i] > 0 ? (*splits)[i] : pick_splits(plan, ap, n_samples, ap.tune_splits, use);
    rc = layout_array(ap, n_samples, sp, size_t(ap.h.F) * ap.h.nx * ap.h.ny, lay[i], need, any_band);
    if (rc) return rc;
  }
  return EPIC_OK;
}

int epic_run(epic_plan_t plan, const void* const* efield, int64_t n_samples, double* const* gains,
             float* const* image, double* const* gain_hist, uint32_t* const* ant_status, epic_stream_t stream) {
  std::vector<RunLayout> lay;
  size_t need = 0;
  bool all_batchable = false, any_band = false;
  const bool fused_plan = plan && plan->arrays.size() <= size_t(epic::kMaxBatch) && fused_eligible(plan);
  int rc = prepare_run(plan, efield, n_samples, gains, image, gain_hist, ant_status, lay, need, all_batchable,
                       any_band, nullptr, fused_plan);
  if (rc) return rc;
  const int na_arr = int(plan->arrays.size());
  if (any_band && plan->batch == 1)
    return fail(EPIC_ERR_UNSUPPORTED, "gains shared over a band run in the per-array form (EPIC_OPT_BATCH 0 or 2)");
  const bool fused = !any_band && all_batchable && fused_eligible(plan);
  const bool batched = !any_band && all_batchable && (plan->batch == 1 || (plan->batch == 0 && na_arr > 1));
  if (plan->graph && !batched && !fused)
    return fail(EPIC_ERR_UNSUPPORTED, "graph replay needs the batched form (EPIC_OPT_BATCH and supported engines)");
  void* scr = nullptr;
  rc = plan_scratch(plan, need, &scr);
  if (rc) return rc;
  if (batched || fused) {
    if (!plan->d_counter) {
      if (hipMalloc(&plan->d_counter, 256) != hipSuccess) return fail(EPIC_ERR_ALLOC, "counter allocation failed");
      plan->generation++;
    }
    if ((rc = build_items(plan, lay, n_samples))) return rc;
  }
  if (fused) {
    int n_chan = 0;
    for (const ArrayPlan& ap : plan->arrays) n_chan += ap.h.F;
    if (64 + n_chan > plan->fused_cap) {
      if (plan->d_fused) {
        hipError_t e = hipDeviceSynchronize();   // a launch of an earlier call may still use the old buffer
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before the progress buffer is replaced");
        hipFree(plan->d_fused);
        plan->d_fused = nullptr;
        plan->fused_cap = 0;
      }
      if (hipMalloc(&plan->d_fused, size_t(64 + n_chan) * sizeof(int)) != hipSuccess)
        return fail(EPIC_ERR_ALLOC, "progress buffer allocation failed");
      plan->fused_cap = 64 + n_chan;
      plan->generation++;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!plan->graph)
    return enqueue_run(plan, lay, static_cast<char*>(scr), efield, n_samples, gains, image, gain_hist, ant_status, s,
                       batched, true, fused);

  // hipGraph: capture once per (buffers, n_samples, plan memory generation), replay afterwards
  if (!plan->gstream) {
    hipError_t e = hipStreamCreateWithFlags(&plan->gstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "graph stream setup");
  }
  GraphKey key;
  key.n_samples = n_samples;
  key.generation = plan->generation;
  for (int i = 0; i < na_arr; ++i) {
    key.ptrs.push_back(efield[i]);
    key.ptrs.push_back(gains[i]);
    key.ptrs.push_back(image[i]);
    key.ptrs.push_back(gain_hist ? gain_hist[i] : nullptr);
    key.ptrs.push_back(ant_status ? ant_status[i] : nullptr);
  }
  if (!(plan->graph_x && key == plan->graph_key)) {
    if (plan->graph_x) hipGraphExecDestroy(plan->graph_x);
    if (plan->graph_g) hipGraphDestroy(plan->graph_g);
    plan->graph_x = nullptr;
    plan->graph_g = nullptr;
    hipError_t e = hipStreamBeginCapture(plan->gstream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    rc = enqueue_run(plan, lay, static_cast<char*>(scr), efield, n_samples, gains, image, gain_hist, ant_status,
                     plan->gstream, true, false, fused);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(plan->gstream, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hipGraphDestroy(g);
      return hip_fail(e, "hipGraphInstantiate");
    }
    plan->graph_g = g;
    plan->graph_x = x;
    plan->graph_key = key;
  }
  hipError_t e = hipEventRecord(plan->ev_in, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(plan->gstream, plan->ev_in, 0);
  if (e != hipSuccess) return hip_fail(e, "graph stream ordering");
  {
    Timed tm(plan, EPIC_TIMER_GRAPH, plan->gstream, true);
    e = hipGraphLaunch(plan->graph_x, plan->gstream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  e = hipEventRecord(plan->ev_out, plan->gstream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, plan->ev_out, 0);
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "graph stream ordering");
}

int epic_run_noalloc(epic_plan_t plan, const void* const* efield, int64_t n_samples, double* const* gains,
                     float* const* image, double* const* gain_hist, uint32_t* const* ant_status,
                     epic_stream_t stream) {
  std::vector<RunLayout> lay;
  size_t need = 0;
  bool all_batchable = false, any_band = false;
  int rc = prepare_run(plan, efield, n_samples, gains, image, gain_hist, ant_status, lay, need, all_batchable,
                       any_band);
  if (rc) return rc;
  // fewer time splits (smaller partial images) until the run fits the static
  // scratch: halve the splits of the array whose partials take the most room
  std::vector<int> sp(lay.size());
  for (size_t i = 0; i < lay.size(); ++i) sp[i] = lay[i].splits;
  while (need > kStaticScratchBytes) {
    int best = -1;
    size_t best_bytes = 0;
    for (size_t i = 0; i < lay.size(); ++i) {
      const HostArray& h = plan->arrays[i].h;
      const size_t b = size_t(sp[i]) * h.F * h.nx * h.ny * sizeof(float);
      if (sp[i] > 1 && b > best_bytes) {
        best = int(i);
        best_bytes = b;
      }
    }
    if (best < 0)
      return fail(EPIC_ERR_ARG, "the run needs %zu bytes of scratch; the static scratch of epic_run_noalloc holds "
                  "%zu (pass gain_hist, or fewer samples or channels per call)", need, kStaticScratchBytes);
    sp[best] = (sp[best] + 1) / 2;
    if ((rc = prepare_run(plan, efield, n_samples, gains, image, gain_hist, ant_status, lay, need, all_batchable,
                          any_band, &sp)))
      return rc;
  }
  hipError_t e = hipSuccess;
  char* scr = static_cast<char*>(static_scratch_ptr(plan->device, &e));
  if (!scr) return hip_fail(e, "static scratch address (hipGetSymbolAddress at plan creation)");
  // per-array launches only (no work list, graph or timing events); every
  // buffer in the scratch is written before it is read, the band solve's
  // barrier flags by a fill kernel
  return enqueue_run(plan, lay, scr, efield, n_samples, gains, image, gain_hist, ant_status,
                     static_cast<hipStream_t>(stream), false, false);
}

int epic_run_snapshots(epic_plan_t plan, int32_t array, const void* efield, int64_t n_samples, int64_t t_acc,
                       double* gains, float* images, double* gain_hist, uint32_t* ant_status, epic_stream_t stream) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if (!ap.has_model) return fail(EPIC_ERR_STATE, "epical_set_model has not been called for array %d", array);
  if ((rc = check_grid_supported(ap))) return rc;
  if (ap.h.nx > 64) return fail(EPIC_ERR_UNSUPPORTED, "snapshot images support grids up to 64 x 64 (got %d)", ap.h.nx);
  if (!epic::solve_supported(ap.h.na, ap.h.efmt, ap.n_pix))
    return fail(EPIC_ERR_UNSUPPORTED, "calibration solve supports Na <= 2048 and Na * bytes per sample <= 16 KiB");
  if (n_samples < 1) return fail(EPIC_ERR_ARG, "n_samples must be >= 1");
  if (t_acc < 1) return fail(EPIC_ERR_ARG, "t_acc must be >= 1");
  if (!efield || !gains || !images) return fail(EPIC_ERR_ARG, "efield, gains and images must not be NULL");
  if ((rc = check_aligned({{efield, "efield"}, {gains, "gains"}, {images, "images"}, {gain_hist, "gain_hist"},
                           {ant_status, "ant_status"}})))
    return rc;
  const int64_t n_win = (n_samples + t_acc - 1) / t_acc;
  const int splits = pick_splits(plan, ap, n_samples, ap.tune_splits);
  RunLayout lay{};
  size_t need = 0;
  bool any_band = false;
  if ((rc = layout_array(ap, n_samples, splits, 0, lay, need, any_band))) return rc;
  void* scr = nullptr;
  if ((rc = plan_scratch(plan, need, &scr))) return rc;
  char* sc = static_cast<char*>(scr);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const HostArray& h = ap.h;
  const epic::SolveArgs sa = solve_args(ap, lay, sc, efield, n_samples, gains, gain_hist, ant_status);
  {
    Timed tm(plan, EPIC_TIMER_SOLVE, s, true);
    hipError_t e = solve_array(plan, ap, sa, sc + lay.band_off, s);
    if (e == hipSuccess) e = epic::launch_hist_to_u(sa.g_hist, ap.d_hold, lay.n_int, h.F, h.na, sa.u_hist, s);
    if (e != hipSuccess) return hip_fail(e, "calibration solve launch");
  }
  ImageArgs ia{static_cast<const uint8_t*>(efield), n_samples, h.F, h.na, h.efmt, sa.u_hist, ap.t_cal, ap.d_slots,
               ap.n_slots, splits, nullptr, ap.d_slots_h, ap.n_slots_h0, ap.n_slots_h1};
  ia.t_acc = t_acc;
  ia.snap = images;
  ia.snap_scale = 1.0 / (double(h.na_eff) * double(h.na_eff));
  // every split holds at least one window per frame slot (per workgroup when
  // its waves share long windows); the splits fill the chip as in epic_run
  const bool group = t_acc >= epic::kSnapGroupWindow && epic::pair_engine(ia, h.nx);
  ia.splits = int(std::min<int64_t>(splits, std::max<int64_t>(1, n_win / (group ? 1 : slots_for(h.nx)))));
  Timed tm(plan, EPIC_TIMER_IMAGE, s, true);
  hipError_t e = epic::launch_image_snap(h.nx, ia, s);
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "snapshot imaging launch");
}

int epic_image(epic_plan_t plan, int32_t array, const void* efield, int64_t n_samples, const double* gains,
               float* image, epic_stream_t stream) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if ((rc = check_grid_supported(ap))) return rc;
  if (n_samples < 1) return fail(EPIC_ERR_ARG, "n_samples must be >= 1");
  if (!efield || !gains || !image) return fail(EPIC_ERR_ARG, "efield, gains and image must not be NULL");
  if ((rc = check_aligned({{efield, "efield"}, {gains, "gains"}, {image, "image"}}))) return rc;
  if (ap.h.na_eff < 1) return fail(EPIC_ERR_ARG, "all antennas are flagged");
  const HostArray& h = ap.h;
  const int splits = pick_splits(plan, ap, n_samples, ap.tune_splits, SplitUse::image);
  const size_t ub = ((size_t(h.F) * h.na * sizeof(float2) + 255) / 256) * 256;
  void* scr = nullptr;
  rc = plan_scratch(plan, ub + size_t(splits) * h.F * h.nx * h.ny * sizeof(float), &scr);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float2* u = static_cast<float2*>(scr);
  hipError_t e = epic::launch_recip(reinterpret_cast<const double2*>(gains), ap.d_flag, h.F, h.na, u, s);
  if (e != hipSuccess) return hip_fail(e, "reciprocal launch");
  return image_pass(plan, ap, efield, n_samples, u, std::numeric_limits<int64_t>::max(), image, s,
                    reinterpret_cast<float*>(static_cast<char*>(scr) + ub), splits);
}

int epic_image_adjoint(epic_plan_t plan, int32_t array, const void* efield, int64_t n_samples, const double* gains,
                       const float* dL_dI, double* dL_dg, epic_stream_t stream) {
  int rc = check_plan(plan, array);
  if (rc) return rc;
  ArrayPlan& ap = plan->arrays[array];
  if ((rc = check_grid_supported(ap, true))) return rc;
  if (n_samples < 1) return fail(EPIC_ERR_ARG, "n_samples must be >= 1");
  if (!efield || !gains || !dL_dI || !dL_dg) return fail(EPIC_ERR_ARG, "efield, gains, dL_dI and dL_dg must not be NULL");
  if ((rc = check_aligned({{efield, "efield"}, {gains, "gains"}, {dL_dI, "dL_dI"}, {dL_dg, "dL_dg"}}))) return rc;
  if (ap.h.na_eff < 1) return fail(EPIC_ERR_ARG, "all antennas are flagged");
  const HostArray& h = ap.h;
  const int splits = pick_splits(plan, ap, n_samples, ap.tune_splits);
  const size_t ub = ((size_t(h.F) * h.na * sizeof(float2) + 255) / 256) * 256;
  void* scr = nullptr;
  rc = plan_scratch(plan, ub + size_t(splits) * h.F * h.na * sizeof(double2), &scr);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float2* u = static_cast<float2*>(scr);
  double2* partial = reinterpret_cast<double2*>(static_cast<char*>(scr) + ub);
  hipError_t e = epic::launch_recip(reinterpret_cast<const double2*>(gains), ap.d_flag, h.F, h.na, u, s);
  if (e != hipSuccess) return hip_fail(e, "reciprocal launch");
  epic::AdjointArgs a{static_cast<const uint8_t*>(efield), n_samples, h.F, h.na, h.efmt, u, dL_dI, ap.d_slots,
                      ap.n_slots, ap.d_cell_ixy, ap.d_cell_w, h.k2, splits, partial,
                      ap.d_slots_h, ap.n_slots_h0, ap.n_slots_h1};
  {
    Timed tm(plan, EPIC_TIMER_ADJOINT, s);
    e = epic::launch_adjoint(h.nx, a, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  }
  const double scale = 1.0 / (double(n_samples) * double(h.na_eff) * double(h.na_eff));
  e = epic::launch_adjoint_reduce(partial, splits, h.F, h.na, reinterpret_cast<const double2*>(gains), scale,
                                  reinterpret_cast<double2*>(dL_dg), s);
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "adjoint reduction launch");
}

// Time the candidate imaging launches of array i and keep the fastest
// (transform, time splits, residue-class engine and its gridding batch).
static int autotune_array(epic_plan_t plan, int i, const void* efield, int64_t n_samples, hipStream_t s) {
  ArrayPlan& ap = plan->arrays[i];
  int rc = check_grid_supported(ap);
  if (rc) return rc;
  if (!efield) return fail(EPIC_ERR_ARG, "NULL efield for array %d", i);
  if ((rc = check_aligned({{efield, "efield"}}))) return rc;
  const HostArray& h = ap.h;
  // candidates: the FFT and the three DFT-GEMM precisions
  std::vector<int> trs{1};
  if (epic::dft_supported(h.nx, h.na, dft_nslots(ap)))
    for (int t : {2, 3, 4}) trs.push_back(t);
  const int base = pick_splits(plan, ap, n_samples, 0);
  std::vector<int> sps;
  for (int c : {base / 2, base, 2 * base, 4 * base}) {
    const int v = int(std::max<int64_t>(1, std::min<int64_t>(c, n_samples)));
    if (std::find(sps.begin(), sps.end(), v) == sps.end()) sps.push_back(v);
  }
  const int max_sp = *std::max_element(sps.begin(), sps.end());
  const size_t ub = align256(size_t(h.F) * h.na * sizeof(float2));
  const size_t ib = align256(size_t(h.F) * h.nx * h.ny * sizeof(float));
  void* scr = nullptr;
  if ((rc = plan_scratch(plan, ub + ib + size_t(max_sp) * h.F * h.nx * h.ny * sizeof(float), &scr))) return rc;
  char* base_p = static_cast<char*>(scr);
  std::vector<float2> ones(size_t(h.F) * h.na, make_float2(1.f, 0.f));
  hipError_t e = hipMemcpy(base_p, ones.data(), ones.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "autotune setup");
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess) return fail(EPIC_ERR_HIP, "autotune event");
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return fail(EPIC_ERR_HIP, "autotune event");
  }
  int best_tr = 1, best_sp = base, best_gb = 0;
  double best_us = 1e300;
  const int keep_tr = ap.tune_transform, keep_sp = ap.tune_splits, keep_gb = ap.tune_batch;
  for (int tr : trs)
    for (int sp : sps) {
      ap.tune_transform = tr;
      // the residue-class engine: the default, and the dense engine with each
      // gridding batch where it applies (0 and 2 are one candidate where the
      // dense engine is the default)
      std::vector<int> gbs{0};
      if (!uses_dft(plan, ap)) {
        ap.tune_batch = 0;
        const bool pair_default = epic::cls_pair_engine(engine_probe(ap), h.nx);
        ap.tune_batch = 2;
        if (epic::cls_dense_engine(engine_probe(ap), h.nx)) {
          if (pair_default) gbs.push_back(2);
          gbs.push_back(4);
        }
      }
      ap.tune_batch = 0;
      for (int gb : gbs) {
        ap.tune_batch = gb;
        ap.tune_splits = sp;
        auto once = [&]() {
          return image_pass(plan, ap, efield, n_samples, reinterpret_cast<const float2*>(base_p),
                            std::numeric_limits<int64_t>::max(), reinterpret_cast<float*>(base_p + ub), s,
                            reinterpret_cast<float*>(base_p + ub + ib), sp, false);
        };
        if ((rc = once())) break;
        hipEventRecord(a, s);
        for (int r = 0; r < 2 && !rc; ++r) rc = once();
        hipEventRecord(b, s);
        if (rc) break;
        e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) {
          rc = hip_fail(e, "autotune timing");
          break;
        }
        const double us = 1e3 * ms / 2.0;
        if (us < best_us) {
          best_us = us;
          best_tr = tr;
          best_sp = sp;
          best_gb = gb;
        }
      }
      if (rc) break;
    }
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (rc) {
    ap.tune_transform = keep_tr;
    ap.tune_splits = keep_sp;
    ap.tune_batch = keep_gb;
    return rc;
  }
  ap.tune_transform = best_tr;
  ap.tune_splits = best_sp;
  ap.tune_batch = best_gb;
  ap.tune_us = best_us;
  return EPIC_OK;
}

int epic_plan_autotune(epic_plan_t plan, const void* const* efield, int64_t n_samples, epic_stream_t stream) {
  if (!plan) return fail(EPIC_ERR_ARG, "plan is NULL");
  if (!efield) return fail(EPIC_ERR_ARG, "efield array is NULL");
  if (n_samples < 1) return fail(EPIC_ERR_ARG, "n_samples must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < int(plan->arrays.size()); ++i) {
    int rc = check_plan(plan, i);
    if (rc) return rc;
    if ((rc = autotune_array(plan, i, efield[i], n_samples, s))) return rc;
  }
  plan->generation++;
  hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? EPIC_OK : hip_fail(e, "autotune synchronise");
}

// Tuning cache: one JSON object, one entry per line,
//   "<arch>|N=<n>|Na=<na>|K=<k>|fmt=<fmt>|F=<f>|T=<t>": {"transform": t, "splits": s, "batch": b, "us": u}
// keyed by everything the imaging launch's speed depends on.
static std::string tune_key(const HostArray& h, int64_t n_samples, const char* arch) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s|N=%d|Na=%d|K=%d|fmt=%d|F=%d|T=%lld", arch, h.nx, h.na, h.kernel, h.efmt, h.F,
           (long long)n_samples);
  return buf;
}

struct TuneEntry {
  int transform, splits, batch;
  double us;
};

static void read_tune_cache(const char* path, std::vector<std::pair<std::string, TuneEntry>>& out) {
  out.clear();
  FILE* fp = fopen(path, "r");
  if (!fp) return;
  char line[1024];
  while (fgets(line, sizeof line, fp)) {
    const char* q0 = strchr(line, '"');
    const char* q1 = q0 ? strchr(q0 + 1, '"') : nullptr;
    if (!q0 || !q1) continue;
    TuneEntry t{};
    const char* body = strchr(q1, '{');
    if (!body || sscanf(body, "{\"transform\": %d, \"splits\": %d, \"batch\": %d, \"us\": %lf", &t.transform,
                        &t.splits, &t.batch, &t.us) != 4)
      continue;   // not an entry of this format: ignored (retuned)
    if (t.transform < 1 || t.transform > 4 || t.splits < 1 || (t.batch != 0 && t.batch != 4)) continue;
    out.push_back({std::string(q0 + 1, q1), t});
  }
  fclose(fp);
}

static int write_tune_cache(const char* path, const std::vector<std::pair<std::string, TuneEntry>>& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fp = fopen(tmp.c_str(), "w");
  if (!fp) return fail(EPIC_ERR_ARG, "cannot write the tuning cache %s", tmp.c_str());
  fprintf(fp, "{\n");
  for (size_t k = 0; k < entries.size(); ++k) {
    const TuneEntry& t = entries[k].second;
    fprintf(fp, "  \"%s\": {\"transform\": %d, \"splits\": %d, \"batch\": %d, \"us\": %.3f}%s\n",
            entries[k].first.c_str(), t.transform, t.splits, t.batch, t.us, k + 1 < entries.size() ? "," : "");
  }
  fprintf(fp, "}\n");
  const bool ok = fclose(fp) == 0 && rename(tmp.c_str(), path) == 0;
  return ok ? EPIC_OK : fail(EPIC_ERR_ARG, "cannot write the tuning cache %s", path);
}

int epic_plan_autotune_cached(epic_plan_t plan, const void* const* efield, int64_t n_samples, const char* cache_path,
                              epic_stream_t stream) {
  if (!plan) return fail(EPIC_ERR_ARG, "plan is NULL");
  if (!cache_path) return epic_plan_autotune(plan, efield, n_samples, stream);
  if (!efield) return fail(EPIC_ERR_ARG, "efield array is NULL");
  if (n_samples < 1) return fail(EPIC_ERR_ARG, "n_samples must be >= 1");
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, plan->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  std::vector<std::pair<std::string, TuneEntry>> cache;
  read_tune_cache(cache_path, cache);
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool added = false;
  for (int i = 0; i < int(plan->arrays.size()); ++i) {
    int rc = check_plan(plan, i);
    if (rc) return rc;
    ArrayPlan& ap = plan->arrays[i];
    const std::string key = tune_key(ap.h, n_samples, arch.c_str());
    auto it = std::find_if(cache.begin(), cache.end(), [&](const auto& kv) { return kv.first == key; });
    if (it != cache.end()) {
      ap.tune_transform = it->second.transform;
      ap.tune_splits = it->second.splits;
      ap.tune_batch = it->second.batch;
      ap.tune_us = it->second.us;
      continue;
    }
    if ((rc = autotune_array(plan, i, efield[i], n_samples, s))) return rc;
    cache.push_back({key, TuneEntry{ap.tune_transform, ap.tune_splits, ap.tune_batch, ap.tune_us}});
    added = true;
  }
  plan->generation++;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "autotune synchronise");
  return added ? write_tune_cache(cache_path, cache) : EPIC_OK;
}

int epic_plan_get_tuning(epic_plan_t plan, int32_t* tuning) {
  if (!plan || !tuning) return fail(EPIC_ERR_ARG, "plan and tuning must not be NULL");
  for (size_t i = 0; i < plan->arrays.size(); ++i) {
    tuning[4 * i] = plan->arrays[i].tune_transform;
    tuning[4 * i + 1] = plan->arrays[i].tune_splits;
    tuning[4 * i + 2] = plan->arrays[i].tune_batch;
    tuning[4 * i + 3] = int32_t(std::min(plan->arrays[i].tune_us, 2e9));
  }
  return EPIC_OK;
}

int epic_plan_set_tuning(epic_plan_t plan, const int32_t* tuning) {
  if (!plan || !tuning) return fail(EPIC_ERR_ARG, "plan and tuning must not be NULL");
  for (size_t i = 0; i < plan->arrays.size(); ++i)
    if (tuning[4 * i] < 0 || tuning[4 * i] > 4 || tuning[4 * i + 1] < 0 ||
        (tuning[4 * i + 2] != 0 && tuning[4 * i + 2] != 2 && tuning[4 * i + 2] != 4))
      return fail(EPIC_ERR_ARG, "bad tuning entry for array %zu", i);
  for (size_t i = 0; i < plan->arrays.size(); ++i) {
    plan->arrays[i].tune_transform = tuning[4 * i];
    plan->arrays[i].tune_splits = tuning[4 * i + 1];
    plan->arrays[i].tune_batch = tuning[4 * i + 2];
  }
  plan->generation++;
  return EPIC_OK;
}

}  // extern "C"
