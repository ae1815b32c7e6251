// Host-side memory and undefined-behaviour check of the library's host code.
//
// Built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
// side only (device code is compiled as usual), linked against the library's
// objects, and run as a plain executable:
//
//   epic_asan_check host   the host-only helpers (grid cells, calibrator
//                          tables, band coordinate), argument checks and
//                          the plan-creation error path; needs no GPU
//   epic_asan_check gpu    plans of several arrays through every host path
//                          around the kernels: models of one and several
//                          pixels, a band model (cooperative solve), a
//                          caller-supplied denominator, options, the tuning
//                          cache, epic_run (per-array, batched, graph),
//                          epic_run_noalloc, snapshots, the fixed-gain image
//                          and its adjoint, table read-back, device unpack,
//                          then plan destruction and process exit
//
// Results are not compared with anything here (the parity tests do that);
// every call must return EPIC_OK or the documented error, and the sanitizers
// must stay silent through teardown.  Exit status 0 on success.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include <sanitizer/lsan_interface.h>

#include "epic.h"

namespace {

int g_fail = 0;

void expect(int got, int want, const char* what) {
  if (got != want) {
    std::fprintf(stderr, "FAIL %s: status %d, expected %d (%s)\n", what, got, want, epic_last_error());
    ++g_fail;
  } else {
    std::printf("ok   %s\n", what);
  }
  std::fflush(stdout);
}

#define HIPCHK(x)                                                               \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      std::fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_),   \
                   __FILE__, __LINE__);                                         \
      std::exit(2);                                                             \
    }                                                                           \
  } while (0)

// xorshift64*: deterministic inputs without the library's own code
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 1) {}
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 0x2545F4914F6CDD1Dull;
  }
  double uniform() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct ArrayData {
  std::vector<double> xy, freq;
  std::vector<uint8_t> flag;
  epic_array_desc desc{};
};

ArrayData make_array(int na, int nchan, int n, int kernel, int efmt, uint64_t seed, bool flag_one) {
  ArrayData a;
  Rng r(seed);
  const double dx = 2.0;
  a.xy.resize(size_t(na) * 2);
  for (int i = 0; i < na; ++i) {
    a.xy[2 * i] = (r.uniform() - 0.5) * 0.8 * n * dx;
    a.xy[2 * i + 1] = (r.uniform() - 0.5) * 0.8 * n * dx;
  }
  a.freq.resize(nchan);
  for (int f = 0; f < nchan; ++f) a.freq[f] = 50e6 + 1e6 * f;
  a.flag.assign(na, 0);
  if (flag_one) a.flag[na / 3] = 1;
  a.desc.n_ant = na;
  a.desc.n_chan = nchan;
  a.desc.nx = a.desc.ny = n;
  a.desc.kernel = kernel;
  a.desc.efmt = efmt;
  a.desc.dx = a.desc.dy = dx;
  a.desc.x0 = -0.5 * n * dx;
  a.desc.y0 = -0.5 * n * dx;
  a.desc.ant_xy = a.xy.data();
  a.desc.freq_hz = a.freq.data();
  a.desc.ant_flag = a.flag.data();
  return a;
}

std::vector<double> make_sources(int n_src, uint64_t seed) {
  Rng r(seed);
  std::vector<double> s(size_t(n_src) * 3);
  s[0] = 0.0, s[1] = 0.0, s[2] = 100.0;  // calibrator at the phase centre
  for (int i = 1; i < n_src; ++i) {
    s[3 * i] = (r.uniform() - 0.5) * 0.6;
    s[3 * i + 1] = (r.uniform() - 0.5) * 0.6;
    s[3 * i + 2] = 1.0 + 4.0 * r.uniform();
  }
  return s;
}

size_t sample_bytes(int efmt) { return efmt == EPIC_CF32 ? 8 : efmt == EPIC_CI8 ? 2 : 1; }

std::vector<uint8_t> make_efield(const epic_array_desc& d, int64_t T, uint64_t seed) {
  Rng r(seed);
  const size_t n = size_t(T) * d.n_chan * d.n_ant;
  std::vector<uint8_t> e(n * sample_bytes(d.efmt));
  if (d.efmt == EPIC_CF32) {
    float* p = reinterpret_cast<float*>(e.data());
    for (size_t i = 0; i < 2 * n; ++i) p[i] = float(r.uniform() * 4.0 - 2.0);
  } else {
    for (auto& b : e) b = uint8_t(r.next() >> 56);
  }
  return e;
}

void host_checks() {
  ArrayData a = make_array(40, 3, 32, 2, EPIC_CI8, 1, true);
  std::vector<double> src = make_sources(12, 2);
  epic_model_desc m{src.data(), 12, 0.0, 0.0, 0.5, 10};

  std::printf("abi %d\n", epic_abi_version());
  std::vector<int32_t> ixy(size_t(a.desc.n_ant) * 4 * 2);
  std::vector<double> w(size_t(a.desc.n_ant) * 4);
  expect(epic_host_grid_cells(&a.desc, ixy.data(), w.data()), EPIC_OK, "epic_host_grid_cells");

  const size_t fa = size_t(a.desc.n_chan) * a.desc.n_ant;
  std::vector<int32_t> k0(size_t(a.desc.n_chan) * 2);
  std::vector<double> A(fa * 2), D(fa * 2);
  expect(epic_host_calibrator(&a.desc, &m, k0.data(), A.data(), D.data()), EPIC_OK, "epic_host_calibrator");

  const double pix[4] = {0.0, 0.0, 0.1, -0.05};
  std::vector<int32_t> k0p(size_t(2) * a.desc.n_chan * 2);
  std::vector<double> Ap(2 * fa * 2), Dp(2 * fa * 2);
  expect(epic_host_calibrator_pixels(&a.desc, &m, pix, 2, k0p.data(), Ap.data(), Dp.data()), EPIC_OK,
         "epic_host_calibrator_pixels");

  std::vector<double> x(a.desc.n_chan);
  expect(epic_host_band_coordinate(&a.desc, 0, a.desc.n_chan, x.data()), EPIC_OK, "epic_host_band_coordinate");

  // argument errors must come back as errors, not as memory faults
  epic_array_desc bad = a.desc;
  bad.nx = bad.ny = 48;
  expect(epic_host_grid_cells(&bad, ixy.data(), w.data()), EPIC_ERR_ARG, "grid 48 rejected");
  bad = a.desc;
  bad.n_ant = 0;
  expect(epic_host_grid_cells(&bad, ixy.data(), w.data()), EPIC_ERR_ARG, "zero antennas rejected");
  expect(epic_host_grid_cells(nullptr, ixy.data(), w.data()), EPIC_ERR_ARG, "null descriptor rejected");
  epic_model_desc bm = m;
  bm.gamma = 1.0;
  expect(epic_host_calibrator(&a.desc, &bm, k0.data(), A.data(), D.data()), EPIC_ERR_ARG, "gamma 1 rejected");
  expect(epic_host_band_coordinate(&a.desc, 2, 1, x.data()), EPIC_ERR_ARG, "empty band rejected");

  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev == 0) {
    epic_plan_t p = nullptr;
    const int rc = epic_plan_create(&a.desc, 1, &p);
    if (rc == EPIC_OK) {
      std::fprintf(stderr, "FAIL plan created without a device\n");
      ++g_fail;
      epic_plan_destroy(p);
    } else {
      std::printf("ok   plan creation without a device fails cleanly (%d: %s)\n", rc, epic_last_error());
    }
  }
}

struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t n) { HIPCHK(hipMalloc(&p, n ? n : 256)); }
  ~DevBuf() { (void)hipFree(p); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

void gpu_checks(const std::string& cache) {
  // three arrays: a paired 64 x 64 array (band model), a 128 x 128 class
  // array, a 32 x 32 cf32 array
  const int64_t T = 120;
  std::vector<ArrayData> arr;
  arr.push_back(make_array(200, 6, 64, 2, EPIC_CI4, 11, true));
  arr.push_back(make_array(300, 4, 128, 2, EPIC_CI8, 12, false));
  arr.push_back(make_array(40, 4, 32, 1, EPIC_CF32, 13, false));
  const int n_arr = int(arr.size());
  std::vector<epic_array_desc> descs;
  for (auto& a : arr) descs.push_back(a.desc);
  std::vector<double> src = make_sources(20, 3);

  hipStream_t s;
  HIPCHK(hipStreamCreate(&s));

  std::vector<std::unique_ptr<DevBuf>> e_dev, g_dev, img_dev, hist_dev, st_dev;
  std::vector<std::vector<double>> g0(n_arr);
  for (int i = 0; i < n_arr; ++i) {
    const auto& d = arr[i].desc;
    auto e = make_efield(d, T, 100 + i);
    e_dev.emplace_back(new DevBuf(e.size()));
    HIPCHK(hipMemcpy(e_dev.back()->p, e.data(), e.size(), hipMemcpyHostToDevice));
    const size_t fa = size_t(d.n_chan) * d.n_ant;
    g0[i].assign(fa * 2, 0.0);
    for (size_t k = 0; k < fa; ++k) g0[i][2 * k] = 1.0;
    g_dev.emplace_back(new DevBuf(fa * 16));
    img_dev.emplace_back(new DevBuf(size_t(d.n_chan) * d.nx * d.ny * 4));
    hist_dev.emplace_back(new DevBuf((size_t(T) / 10 + 2) * fa * 16));
    st_dev.emplace_back(new DevBuf(fa * 4));
  }
  auto reset_gains = [&]() {
    for (int i = 0; i < n_arr; ++i)
      HIPCHK(hipMemcpy(g_dev[i]->p, g0[i].data(), g0[i].size() * 8, hipMemcpyHostToDevice));
  };
  std::vector<const void*> ep;
  std::vector<double*> gp, hp;
  std::vector<float*> ip;
  std::vector<uint32_t*> sp;
  for (int i = 0; i < n_arr; ++i) {
    ep.push_back(e_dev[i]->p);
    gp.push_back(static_cast<double*>(g_dev[i]->p));
    ip.push_back(static_cast<float*>(img_dev[i]->p));
    hp.push_back(static_cast<double*>(hist_dev[i]->p));
    sp.push_back(static_cast<uint32_t*>(st_dev[i]->p));
  }

  for (int round = 0; round < 2; ++round) {   // two plans in turn: teardown, then a fresh plan
    epic_plan_t plan = nullptr;
    expect(epic_plan_create(descs.data(), n_arr, &plan), EPIC_OK, "epic_plan_create");
    if (!plan) break;
    for (int i = 0; i < n_arr; ++i) {
      epic_model_desc m{src.data(), 20, 0.0, 0.0, 0.5, 10};
      expect(epical_set_model(plan, i, &m), EPIC_OK, "epical_set_model");
    }
    expect(epic_plan_set_option(plan, EPIC_OPT_TIMING, 1), EPIC_OK, "timing on");

    // caller-supplied denominator for array 1: the plan's own, read through the host helper
    {
      const auto& d = arr[1].desc;
      epic_model_desc m{src.data(), 20, 0.0, 0.0, 0.5, 10};
      const size_t fa = size_t(d.n_chan) * d.n_ant;
      std::vector<int32_t> k0(size_t(d.n_chan) * 2);
      std::vector<double> A(fa * 2), D(fa * 2);
      expect(epic_host_calibrator(&d, &m, k0.data(), A.data(), D.data()), EPIC_OK, "host calibrator");
      expect(epical_set_denominator(plan, 1, D.data()), EPIC_OK, "epical_set_denominator");
    }

    // batched and per-array runs, graph replays
    for (int batch : {2, 1}) {
      expect(epic_plan_set_option(plan, EPIC_OPT_BATCH, batch), EPIC_OK, "batch option");
      expect(epic_plan_set_option(plan, EPIC_OPT_GRAPH, batch == 1), EPIC_OK, "graph option");
      for (int rep = 0; rep < 2; ++rep) {
        reset_gains();
        expect(epic_run(plan, ep.data(), T, gp.data(), ip.data(), hp.data(), sp.data(), s), EPIC_OK, "epic_run");
      }
      HIPCHK(hipStreamSynchronize(s));
    }
    expect(epic_plan_set_option(plan, EPIC_OPT_GRAPH, 0), EPIC_OK, "graph off");
    double ms[EPIC_TIMER_COUNT];
    int64_t launches[EPIC_TIMER_COUNT];
    expect(epic_plan_get_timing(plan, ms, launches, EPIC_TIMER_COUNT), EPIC_OK, "epic_plan_get_timing");

    // the tuning cache: written by the first plan, read by the second
    expect(epic_plan_autotune_cached(plan, ep.data(), T, cache.c_str(), s), EPIC_OK, "epic_plan_autotune_cached");
    std::vector<int32_t> tun(size_t(4) * n_arr);
    expect(epic_plan_get_tuning(plan, tun.data()), EPIC_OK, "epic_plan_get_tuning");
    expect(epic_plan_set_tuning(plan, tun.data()), EPIC_OK, "epic_plan_set_tuning");

    reset_gains();
    expect(epic_run_noalloc(plan, ep.data(), T, gp.data(), ip.data(), hp.data(), sp.data(), s), EPIC_OK,
           "epic_run_noalloc");
    HIPCHK(hipStreamSynchronize(s));

    // stage-free calls on array 0 (64 x 64)
    {
      const auto& d = arr[0].desc;
      const size_t fa = size_t(d.n_chan) * d.n_ant;
      const int64_t t_acc = 40, n_win = (T + t_acc - 1) / t_acc;
      DevBuf snaps(size_t(n_win) * d.n_chan * d.nx * d.ny * 4), grad(fa * 16), dldi(size_t(d.n_chan) * d.nx * d.ny * 4);
      HIPCHK(hipMemset(dldi.p, 0, size_t(d.n_chan) * d.nx * d.ny * 4));
      reset_gains();
      expect(epic_run_snapshots(plan, 0, ep[0], T, t_acc, gp[0], static_cast<float*>(snaps.p), nullptr, nullptr, s),
             EPIC_OK, "epic_run_snapshots");
      reset_gains();
      expect(epic_image(plan, 0, ep[0], T, gp[0], ip[0], s), EPIC_OK, "epic_image");
      expect(epic_image_adjoint(plan, 0, ep[0], T, gp[0], static_cast<const float*>(dldi.p),
                                static_cast<double*>(grad.p), s), EPIC_OK, "epic_image_adjoint");
      std::vector<int32_t> ixy(size_t(d.n_ant) * 4 * 2);
      std::vector<float> w(size_t(d.n_ant) * 4);
      expect(epic_plan_get_cells(plan, 0, ixy.data(), w.data()), EPIC_OK, "epic_plan_get_cells");
      DevBuf un(size_t(1000) * 4);
      expect(epic_debug_unpack(plan, 0, ep[0], 1000, static_cast<int16_t*>(un.p), s), EPIC_OK,
             "epic_debug_unpack");
      expect(epic_run_snapshots(plan, 0, ep[0], T, 0, gp[0], static_cast<float*>(snaps.p), nullptr, nullptr, s),
             EPIC_ERR_ARG, "t_acc 0 rejected");
      expect(epic_run(plan, ep.data(), -1, gp.data(), ip.data(), nullptr, nullptr, s), EPIC_ERR_ARG,
             "negative n_samples rejected");
      HIPCHK(hipStreamSynchronize(s));
    }

    // several tapped pixels, then a band model (cooperative solve) on array 0
    {
      epic_model_desc m{src.data(), 20, 0.0, 0.0, 0.5, 10};
      const double pix[6] = {0.0, 0.0, 0.1, 0.05, -0.08, 0.02};
      expect(epical_set_model_pixels(plan, 0, &m, pix, 3), EPIC_OK, "epical_set_model_pixels");
      expect(epic_plan_set_option(plan, EPIC_OPT_BATCH, 2), EPIC_OK, "per-array form");
      reset_gains();
      expect(epic_run(plan, ep.data(), T, gp.data(), ip.data(), nullptr, sp.data(), s), EPIC_OK,
             "epic_run, three pixels");
      expect(epical_set_model(plan, 0, &m), EPIC_OK, "back to one pixel");
      for (int mode : {EPIC_BAND_MEAN, EPIC_BAND_POLY}) {
        expect(epical_set_band(plan, 0, 1, 5, mode, 1, 1), EPIC_OK, "epical_set_band");
        reset_gains();
        expect(epic_run(plan, ep.data(), T, gp.data(), ip.data(), hp.data(), sp.data(), s), EPIC_OK,
               "epic_run, band model");
        HIPCHK(hipStreamSynchronize(s));
      }
      reset_gains();
      expect(epic_run_noalloc(plan, ep.data(), T, gp.data(), ip.data(), hp.data(), sp.data(), s), EPIC_OK,
             "epic_run_noalloc, band model");
      HIPCHK(hipStreamSynchronize(s));
    }
    std::vector<double> g(g0[0].size());
    HIPCHK(hipMemcpy(g.data(), gp[0], g.size() * 8, hipMemcpyDeviceToHost));
    for (double v : g)
      if (!std::isfinite(v)) {
        std::fprintf(stderr, "FAIL non-finite gain after the band run\n");
        ++g_fail;
        break;
      }
    expect(epic_plan_destroy(plan), EPIC_OK, "epic_plan_destroy");
  }
  HIPCHK(hipStreamDestroy(s));
}

}  // namespace

int main(int argc, char** argv) {
  const std::string mode = argc > 1 ? argv[1] : "host";
  host_checks();
  if (mode == "gpu") {
    const std::string cache = argc > 2 ? argv[2] : "epic_asan_tune.json";
    std::remove(cache.c_str());
    gpu_checks(cache);
  }
  // Leaks are checked here, after every plan is destroyed, and the process
  // then ends without running the static destructors of the HIP and HSA
  // runtimes: with the ROCm AddressSanitizer runtime those destructors free
  // runtime memory after the runtime has been marked unloaded, which stops
  // the process in the sanitizer's own device-allocator check (a stack
  // entirely inside libamdhip64 / libhsa-runtime64, not this library's code).
  const int leaks = __lsan_do_recoverable_leak_check();
  std::printf("%s: %d failure(s), leak check %s\n", mode.c_str(), g_fail, leaks ? "FAILED" : "clean");
  std::fflush(stdout);
  std::fflush(stderr);
  std::_Exit(g_fail || leaks ? 1 : 0);
}
